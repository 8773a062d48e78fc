"""Pins of the surrogate oracle (oracle/surrogate.py) against what the
mathematics fixes, independent of the oracle's own formulas."""
import numpy as np
import torch

import oracle
from oracle import surrogate as S


def _A0():
    lame = oracle.two_phase_lame(10.0)
    ph = oracle.phase_by_centroid(2, 8, 0.25)
    st, Ch = oracle.linear_homogenized(2, 8, ph, lame)
    assert st == 0
    return Ch


def _F(n, seed, amp=0.15):
    rng = np.random.default_rng(seed)
    F = np.eye(2)[None] + rng.uniform(-amp, amp, (n, 2, 2))
    return F.reshape(n, 4)


def test_identity_gives_zero_stress_and_small_strain_tangent():
    # the network part vanishes to second order at F = I: P(I) = 0, A(I) = A0
    # (A0: the RVE oracle's linear homogenized tangent, which has the minor and
    # major symmetries the quadratic energy reproduces)
    A0 = _A0()
    desc = S.make_desc(A0)
    th = S.random_params(1, scale=2.0)
    P, A = S.eval_PA(th, desc, np.eye(2).reshape(1, 4))
    assert np.abs(P).max() < 1e-14
    np.testing.assert_allclose(A[0].reshape(4, 4), A0, rtol=1e-12, atol=1e-12 * np.abs(A0).max())


def test_zero_network_is_st_venant_kirchhoff():
    # w4 = 0: W = 1/2 E:C0:E, so S = C0:E and P = F S with C0 the tangent A0
    # read as C0_IJKL = A0[(I,J),(K,L)] at F = I (closed form, no autograd)
    A0 = _A0()
    desc = S.make_desc(A0)
    th = S.random_params(2)
    th[S.OFF_W4:] = 0.0
    F = _F(6, 3)
    P, _ = S.eval_PA(th, desc, F)
    C0 = A0.reshape(2, 2, 2, 2)
    # minor-symmetrize as the baseline does
    C0 = 0.25 * (C0 + C0.transpose(1, 0, 2, 3) + C0.transpose(0, 1, 3, 2) + C0.transpose(1, 0, 3, 2))
    C0 = 0.5 * (C0 + C0.transpose(2, 3, 0, 1))
    for b in range(len(F)):
        Fb = F[b].reshape(2, 2)
        E = 0.5 * (Fb.T @ Fb - np.eye(2))
        Sb = np.einsum("IJKL,KL->IJ", C0, E)
        np.testing.assert_allclose(P[b].reshape(2, 2), Fb @ Sb, rtol=1e-12, atol=1e-14)


def test_stress_is_energy_derivative_and_tangent_is_stress_derivative():
    desc = S.make_desc(_A0())
    th = S.random_params(4, scale=2.0)
    F = _F(3, 5)
    P, A = S.eval_PA(th, desc, F)
    h = 1e-6

    def W(Fv):
        with torch.enable_grad():
            return S.energy(S.to_t(th), desc, S.to_t(Fv).reshape(-1, 2, 2)).detach().numpy()
    for c in range(4):
        Fp, Fm = F.copy(), F.copy()
        Fp[:, c] += h
        Fm[:, c] -= h
        np.testing.assert_allclose((W(Fp) - W(Fm)) / (2 * h), P[:, c], rtol=1e-6, atol=1e-9)
        Pp, _ = S.eval_PA(th, desc, Fp)
        Pm, _ = S.eval_PA(th, desc, Fm)
        np.testing.assert_allclose((Pp - Pm) / (2 * h), A.reshape(-1, 4, 4)[:, :, c], rtol=1e-6, atol=1e-8)


def test_frame_invariance_and_major_symmetry():
    desc = S.make_desc(_A0())
    th = S.random_params(6, scale=2.0)
    F = _F(4, 7)
    P, A = S.eval_PA(th, desc, F)
    a = 0.7
    Q = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
    FQ = np.stack([(Q @ f.reshape(2, 2)).reshape(4) for f in F])
    PQ, AQ = S.eval_PA(th, desc, FQ)
    for b in range(len(F)):
        np.testing.assert_allclose(PQ[b].reshape(2, 2), Q @ P[b].reshape(2, 2), rtol=1e-11, atol=1e-13)
        A4 = A[b].reshape(2, 2, 2, 2)
        AQ4 = np.einsum("ia,kb,aJbL->iJkL", Q, Q, A4)
        np.testing.assert_allclose(AQ[b].reshape(2, 2, 2, 2), AQ4, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(A[b].reshape(4, 4), A[b].reshape(4, 4).T, rtol=1e-11, atol=1e-13)


def test_loss_gradient_matches_finite_differences():
    desc = S.make_desc(_A0())
    th = S.random_params(8, scale=1.5)
    F = _F(5, 9)
    rng = np.random.default_rng(10)
    Pt = rng.normal(size=(5, 4)) * 0.1
    At = rng.normal(size=(5, 16))
    L, g = S.loss_and_grad(th, desc, F, Pt, At)
    h = 1e-5
    for i in [S.OFF_W1 + 4, S.OFF_B1 + 7, S.OFF_W2 + 1000, S.OFF_B2 + 3, S.OFF_W3 + 5000, S.OFF_B3 + 100,
              S.OFF_W4 + 17]:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        Lp, _ = S.loss_and_grad(tp, desc, F, Pt, At)
        Lm, _ = S.loss_and_grad(tm, desc, F, Pt, At)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(11)
    th0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(5)]
    p = torch.nn.Parameter(torch.tensor(th0.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = th0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(grads, 1):
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = S.adam_step(th, m, v, g, t, 3e-3)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)
