"""Hand-worked pins of the oracle's artificial viscosity, du/dt and v_sig (no GPU).

The force pins elsewhere (momentum, energy, dissipation) hold for any
viscosity that is antisymmetric and acts on approaching pairs, so a wrong
factor in q, a swapped sound speed or a sign slip inside v_sig would keep
them.  These cases fix the numbers themselves, worked out by hand below from
the grad-h force with a per-particle viscosity (the reading of the force and
AV that the oracle takes; the paper runs Phantom's compressible SPH and
states no formula):

  a_a     = -sum_b m_b [A_a F_ab(h_a) + B_b F_ab(h_b)] rhat_ab,
  du_a/dt =  sum_b m_b A_a (v_ab . rhat_ab) F_ab(h_a),
  A_a = (P_a + q^a)/(Omega_a rho_a^2),  B_b = (P_b + q^b)/(Omega_b rho_b^2),
  q^a = -1/2 rho_a vsig_a (v_ab . rhat)  only if v_ab . rhat < 0,
  vsig_a = alpha c_a + beta |v_ab . rhat|,   F(h) = f'(r/h)/(pi h^4),
  reported vsig_a = max(alpha c_a, max over approaching pairs of vsig_a).

Set-up (M4 kernel, alpha = 1, beta = 2, adiabatic gamma = 5/3, m0 = 1):

  particle  x   level (m)   h     rho  Omega  u      P = (2/3) rho u   c = sqrt(10 u / 9)
  a         0   0 (1)       1     2    4/5    9/10   6/5               1
  b         1   1 (1/2)     4/5   1    5/4    18/5   12/5              2

r = 1, so q_a = 1 and q_b = 5/4; M4 gives f'(1) = -3/4 and
f'(5/4) = -3/4 (3/4)^2 = -27/64, hence
  pi F(h_a) = -3/4,   pi F(h_b) = (-27/64) / (4/5)^4 = -16875/16384.
Seen from a, rhat_ab = -x; seen from b, rhat_ba = +x.

Approaching (v_a = +1/4, v_b = -1/4 along x): v_ab . rhat = -1/2.
  vsig_a = 1 + 2 (1/2) = 2,     vsig_b = 2 + 1 = 3,
  q^a = -1/2 * 2 * 2 * (-1/2) = 1,   q^b = -1/2 * 1 * 3 * (-1/2) = 3/4,
  A_a = (6/5 + 1)/(4/5 * 4) = 11/16,   B_b = (12/5 + 3/4)/(5/4) = 63/25.
  pi ax_a = m_b (A_a pi F_a + B_b pi F_b) = 1/2 (-33/64 - 63/25 * 16875/16384)
          = -50973/32768
  pi du_a/dt = m_b A_a (-1/2) pi F_a = 1/2 * 11/16 * (-1/2) * (-3/4) = 33/256
  pi ax_b = -m_a (B_b pi F_b + A_a pi F_a) = 50973/16384
  pi du_b/dt = m_a B_b (-1/2) pi F_b = 42525/32768
  vsig: a 2, b 3.
Receding (velocities reversed): v . rhat = +1/2, no q, vsig = alpha c.
  A_a = (6/5)/(16/5) = 3/8,   B_b = (12/5)/(5/4) = 48/25,
  pi ax_a = 1/2 (-9/32 - 48/25 * 16875/16384) = -2313/2048,
  pi du_a/dt = 1/2 * 3/8 * 1/2 * (-3/4) = -9/128,
  pi ax_b = 2313/1024,  pi du_b/dt = 48/25 * 1/2 * (-16875/16384) = -2025/2048,
  vsig: a 1, b 2.
Three particles: b as above approaching a from x = 1, and a copy c of b at
x = -1 moving with v_c = -1/4, so that c recedes from a (b and c are 2 apart,
beyond 2 max(h_b, h_c) = 8/5, and do not interact).  By the mirror image of
the receding pair, c adds +2313/2048 to pi ax_a and -9/128 to pi du_a/dt:
  pi ax_a = -50973/32768 + 37008/32768 = -13965/32768,
  pi du_a/dt = 33/256 - 18/256 = 15/256,   vsig_a = 2.
Gates are 1e-12 relative: the only rounding is in the EOS (u = 9/10 is not a
binary fraction) and the square roots."""
import math

import numpy as np

PI = math.pi


def _run(orc, x, v, level, h, rho, om, u):
    n = len(x)
    z = np.zeros(n)
    return orc.forces(np.array(x, float), z, z, np.array(v, float), z, z, np.array(u, float),
                      np.array(level, np.int8), np.array(h, float), np.array(rho, float),
                      np.array(om, float), m0=1.0, eos=2, gamma=5.0 / 3.0, alpha=1.0, beta=2.0,
                      kernel=0)


A = dict(level=0, h=1.0, rho=2.0, om=0.8, u=0.9)
B = dict(level=1, h=0.8, rho=1.0, om=1.25, u=3.6)


def _pair(orc, va, vb):
    return _run(orc, [0.0, 1.0], [va, vb], [A["level"], B["level"]], [A["h"], B["h"]],
                [A["rho"], B["rho"]], [A["om"], B["om"]], [A["u"], B["u"]])


def _close(got, want):
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)


def test_av_approaching_pair(orc):
    f = _pair(orc, 0.25, -0.25)
    _close(f["ax"][0], -50973 / 32768 / PI)
    _close(f["dudt"][0], 33 / 256 / PI)
    _close(f["ax"][1], 50973 / 16384 / PI)
    _close(f["dudt"][1], 42525 / 32768 / PI)
    _close(f["vsig"][0], 2.0)
    _close(f["vsig"][1], 3.0)
    assert np.all(f["ay"] == 0.0) and np.all(f["az"] == 0.0)


def test_av_receding_pair(orc):
    f = _pair(orc, -0.25, 0.25)
    _close(f["ax"][0], -2313 / 2048 / PI)
    _close(f["dudt"][0], -9 / 128 / PI)
    _close(f["ax"][1], 2313 / 1024 / PI)
    _close(f["dudt"][1], -2025 / 2048 / PI)
    _close(f["vsig"][0], 1.0)
    _close(f["vsig"][1], 2.0)


def test_av_one_approaching_one_receding(orc):
    f = _run(orc, [0.0, 1.0, -1.0], [0.25, -0.25, -0.25], [0, 1, 1], [1.0, 0.8, 0.8],
             [2.0, 1.0, 1.0], [0.8, 1.25, 1.25], [0.9, 3.6, 3.6])
    _close(f["ax"][0], -13965 / 32768 / PI)
    _close(f["dudt"][0], 15 / 256 / PI)
    _close(f["vsig"][0], 2.0)
    # b sees only a (approaching), c sees only a (receding): the two-particle values
    _close(f["ax"][1], 50973 / 16384 / PI)
    _close(f["vsig"][1], 3.0)
    _close(f["ax"][2], -2313 / 1024 / PI)
    _close(f["dudt"][2], -2025 / 2048 / PI)
    _close(f["vsig"][2], 2.0)
