"""The numpy model of the surrogate kernels' algorithm (tests/surrogate_model.py)
against the autograd oracle: forward-mode jets, the head's directional loss
derivatives, the origin's Taylor terms and the reverse pass must reproduce the
oracle's loss and gradient to rounding."""
import numpy as np

import oracle
from oracle import surrogate as OS
from tests import surrogate_model as SM


def test_jet_algorithm_matches_autograd_oracle():
    st, Ch = oracle.linear_homogenized(2, 8, oracle.phase_by_centroid(2, 8, 0.25), oracle.two_phase_lame(10.0))
    desc = OS.make_desc(Ch, w_scale=0.1)
    th = OS.random_params(31, scale=1.5)
    rng = np.random.default_rng(32)
    F = (np.eye(2)[None] + rng.uniform(-0.3, 0.3, (12, 2, 2))).reshape(12, 4)
    P0, A0 = OS.eval_PA(th, desc, F)
    Pt = P0 * (1 + 0.5 * rng.normal(size=P0.shape))
    At = A0 * (1 + 0.5 * rng.normal(size=A0.shape))
    L, g = SM.loss_grad(th, desc, F, Pt, At)
    Lr, gr = OS.loss_and_grad(th, desc, F, Pt, At)
    assert abs(L - Lr) <= 1e-12 * abs(Lr)
    for name, a, b in SM.BLOCKS:
        assert np.linalg.norm(g[a:b] - gr[a:b]) <= 1e-11 * np.linalg.norm(gr[a:b]), name


def test_bf16_rounding_model():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 1e-30])
    r = SM.bf16(x)
    # 7 stored mantissa bits: 1 + 2^-8 is a tie and goes to the even neighbour 1
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert abs(r[3] + 3.140625) < 1e-12
    assert np.all(np.abs(r - x) <= 2 ** -8 * np.abs(x))
