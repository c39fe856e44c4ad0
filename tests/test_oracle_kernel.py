"""Pins of the oracle's kernels against closed forms (no GPU).

The paper pairs the M4 cubic spline with h_fact = 1.2 and a mean neighbour
number of 57.9 (appendix "Kernel choice", kernel table), and runs its examples
with the Wendland C2 kernel, kernel radius 2h and h_fact = 1.3 (Sec. 3)."""
import os

import numpy as np
import pytest
from scipy.integrate import quad

pytestmark = pytest.mark.filterwarnings("ignore")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_normalisation(orc):
    # int_0^{2h} 4 pi r^2 W(r, h) dr = 1 for any h
    for h in (0.3, 1.0, 2.7):
        parts = [quad(lambda r: 4 * np.pi * r * r * orc.w(r, h), a, b, epsabs=1e-15,
                      epsrel=1e-14)[0] for a, b in ((0, h), (h, 2 * h))]
        assert abs(sum(parts) - 1.0) < 1e-13


def test_textbook_values(orc):
    # f(0) = 1 (so W(0,h) = 1/(pi h^3)), f(1) = 1/4, f(2) = 0; f'(1) = -3/4
    assert orc.m4_f(0.0) == 1.0
    assert orc.m4_f(1.0) == 0.25
    assert orc.m4_f(2.0) == 0.0 and orc.m4_f(2.5) == 0.0
    assert orc.m4_df(1.0) == -0.75 and orc.m4_df(0.0) == 0.0
    assert abs(orc.w(0.0, 2.0) - 1.0 / (np.pi * 8.0)) < 1e-18


def test_c2_continuity(orc):
    e = 1e-9
    for q in (1.0, 2.0):
        for fn in (orc.m4_f, orc.m4_df, orc.m4_d2f):
            assert abs(fn(q - e) - fn(q + e)) < 1e-8


def test_derivatives_match_differences(orc):
    for q in np.linspace(0.05, 1.95, 39) + 0.013:
        e = 1e-6
        fd = (orc.m4_f(q + e) - orc.m4_f(q - e)) / (2 * e)
        assert abs(fd - orc.m4_df(q)) < 1e-8
        fd2 = (orc.m4_df(q + e) - orc.m4_df(q - e)) / (2 * e)
        assert abs(fd2 - orc.m4_d2f(q)) < 1e-7


def test_dwdh_matches_difference(orc):
    for r in (0.0, 0.3, 0.9, 1.3, 1.9):
        h = 1.1
        e = 1e-6
        fd = (orc.w(r, h + e) - orc.w(r, h - e)) / (2 * e)
        assert abs(fd - orc.dwdh(r, h)) < 1e-8


def test_paper_neighbour_number():
    # the paper's kernel table: M4 at h_fact 1.2 has N_neigh 57.9, which is the
    # number of particles of a uniform medium inside the 2h sphere
    rows = [l.split() for l in open(os.path.join(GOLDEN, "kernel_table.txt"))
            if l.strip() and not l.startswith("#")]
    m4 = [r for r in rows if r[0] == "M4_cubic"][0]
    nn, hfact = float(m4[1]), float(m4[2])
    assert abs(4.0 * np.pi / 3.0 * (2 * hfact) ** 3 - nn) < 0.05


# ------------------------------------------------------------- Wendland C2
def test_wc2_normalisation(orc):
    for h in (0.3, 1.0, 2.7):
        v = quad(lambda r: 4 * np.pi * r * r * orc.w(r, h, 1), 0, 2 * h, epsabs=1e-15,
                 epsrel=1e-14)[0]
        assert abs(v - 1.0) < 1e-13


def test_wc2_textbook_values(orc):
    # Wendland's phi_{3,1}(s) = (1 - s)^4 (4 s + 1) on s = q/2, normalised in 3D
    # by 21/(16 pi): W(0, h) = 21/(16 pi h^3); f(1) = 21/16 * 3/16 = 63/256
    assert orc.wc2_f(0.0) == 21.0 / 16.0
    assert orc.wc2_f(1.0) == 63.0 / 256.0
    assert orc.wc2_f(2.0) == 0.0 and orc.wc2_f(2.5) == 0.0
    assert orc.wc2_df(0.0) == 0.0  # smooth at the origin
    assert abs(orc.w(0.0, 2.0, 1) - 21.0 / (16.0 * np.pi * 8.0)) < 1e-18
    # the selector returns the same functions
    for q in (0.0, 0.7, 1.3, 1.99):
        assert orc.kf(q, 1) == orc.wc2_f(q) and orc.kdf(q, 1) == orc.wc2_df(q)
        assert orc.kd2f(q, 1) == orc.wc2_d2f(q) and orc.kf(q, 0) == orc.m4_f(q)


def test_wc2_smooth_at_support_edge(orc):
    # C2: f, f', f'' all reach 0 continuously at q = 2
    e = 1e-9
    for fn in (orc.wc2_f, orc.wc2_df, orc.wc2_d2f):
        assert abs(fn(2.0 - e)) < 1e-8 and fn(2.0 + e) == 0.0


def test_wc2_derivatives_match_differences(orc):
    for q in np.linspace(0.05, 1.95, 39) + 0.013:
        e = 1e-6
        fd = (orc.wc2_f(q + e) - orc.wc2_f(q - e)) / (2 * e)
        assert abs(fd - orc.wc2_df(q)) < 1e-8
        fd2 = (orc.wc2_df(q + e) - orc.wc2_df(q - e)) / (2 * e)
        assert abs(fd2 - orc.wc2_d2f(q)) < 1e-7


def test_wc2_dwdh_matches_difference(orc):
    for r in (0.0, 0.3, 0.9, 1.3, 1.9, 2.15):
        h = 1.1
        e = 1e-6
        fd = (orc.w(r, h + e, 1) - orc.w(r, h - e, 1)) / (2 * e)
        assert abs(fd - orc.dwdh(r, h, 1)) < 1e-8


def test_wc2_neighbour_number_reading():
    # Sec. 3 fixes h_fact = 1.3 with kernel radius 2h, so a uniform medium has
    # (4 pi/3) (2.6)^3 = 73.6 neighbours.  The kernel table prints 92 beside
    # h_fact 1.3; 92 is the count for h_fact 1.4 ((4 pi/3) 2.8^3 = 91.95), so
    # the table's two columns disagree and the text's h_fact is the one taken.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "kernel_table.txt"))
            if l.strip() and not l.startswith("#")]
    c2 = [r for r in rows if r[0] == "Wendland_C2"][0]
    nn, hfact = float(c2[1]), float(c2[2])
    assert hfact == 1.3
    assert abs(4.0 * np.pi / 3.0 * (2 * hfact) ** 3 - 73.6) < 0.05
    assert abs(4.0 * np.pi / 3.0 * (2 * 1.4) ** 3 - nn) < 0.1
