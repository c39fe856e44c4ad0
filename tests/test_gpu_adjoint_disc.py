"""Adjoint parity on disc geometry: the 1M-particle planet disc (its spread
of h, multi-chunk candidate walks and the locally isothermal EOS), by
sampled balls in both forms.  Cotangents sit on one ball's targets only;
the GPU's gradients over all 1M particles are compared with the dense FP64
gradient oracle solved on the ball's dependency set (tests/_gpu.py,
ball_vjp_check).  Gates as for the other adjoint parity tests: 1e-6 (FP64
form) and 1e-3 (FP32 form) of the gradient's max-norm.  The 8M-particle
circumbinary disc's balls (levels 0, 1 and 2) are in test_gpu_large.py."""
import numpy as np
import pytest

import workloads as W
from _gpu import ball_vjp_check

pytestmark = pytest.mark.gpu

GTOL = {"fp64": 1e-6, "fp32": 1e-3}


@pytest.fixture(scope="module")
def planet_disc():
    return W.planet_disc()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ball", [0, 1])
def test_planet_disc_1M_vjp_sampled(planet_disc, prec, ball):
    st, p = planet_disc
    rng = np.random.default_rng(2409114703 + ball)
    centre = int(rng.integers(st["x"].shape[0]))
    ball_vjp_check(("planet", ball), st, p, prec, centre, seed=ball, gtol=GTOL[prec])
