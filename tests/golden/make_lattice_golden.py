"""Write lattice_m4.txt and lattice_wc2.txt: the converged h-rho solution on a
simple cubic lattice for the M4 kernel (h_fact 1.2) and the Wendland C2
kernel (h_fact 1.3).

On a lattice of spacing dx (mass m, rho0 = m/dx^3) every particle sees the same
shells: r3(k) lattice vectors of squared length k dx^2.  So
    rho(h)/rho0 = dx^3 sum_k r3(k) W(sqrt(k) dx, h)
and the h-rho relation rho(h) = m (h_fact/h)^3 is one scalar equation, solved
here by bracketing (brentq).  Omega = 1 + h/(3 rho) d rho/dh is taken by a
central difference of the same shell sum.  Only the oracle's kernel function W
is used (itself pinned by its normalisation and continuity tests); r3(k) are
counted by brute force.  Run: python tests/golden/make_lattice_golden.py
"""
import itertools
import os
import sys

import numpy as np
from scipy.optimize import brentq

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402


def shell_counts(kmax):
    r3 = {}
    n = int(np.ceil(np.sqrt(kmax))) + 1
    for i, j, k in itertools.product(range(-n, n + 1), repeat=3):
        s = i * i + j * j + k * k
        if s <= kmax:
            r3[s] = r3.get(s, 0) + 1
    return r3


def lattice_rho(h, r3, kernel):
    return sum(c * oracle.w(np.sqrt(k), h, kernel) for k, c in r3.items()
               if k < (2.0 * h) ** 2)


def write(fname, label, kernel, hfact):
    r3 = shell_counts(16)
    h = brentq(lambda hh: lattice_rho(hh, r3, kernel) - (hfact / hh) ** 3, 1.0, 1.5,
               xtol=1e-15, rtol=1e-15)
    rho = lattice_rho(h, r3, kernel)
    eps = 1e-5
    drho = (lattice_rho(h + eps, r3, kernel) - lattice_rho(h - eps, r3, kernel)) / (2 * eps)
    omega = 1.0 + h * drho / (3.0 * rho)
    nn = sum(c for k, c in r3.items() if k < (2.0 * h) ** 2)
    with open(os.path.join(HERE, fname), "w") as f:
        f.write("# simple cubic lattice, spacing dx = 1, m = 1, %s kernel, h_fact = %g\n"
                % (label, hfact))
        f.write("# written by make_lattice_golden.py (shell sums + brentq; Omega by a\n")
        f.write("# central difference of the shell sum, accurate to ~1e-10)\n")
        f.write("h_over_dx %.15f\n" % h)
        f.write("rho_over_rho0 %.15f\n" % rho)
        f.write("omega %.15f\n" % omega)
        f.write("nneigh_incl_self %d\n" % nn)
        f.write("rho_over_rho0_at_h%g %.15f\n" % (hfact, lattice_rho(hfact, r3, kernel)))


def main():
    write("lattice_m4.txt", "M4", 0, 1.2)
    write("lattice_wc2.txt", "Wendland C2", 1, 1.3)


if __name__ == "__main__":
    main()
