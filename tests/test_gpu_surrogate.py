"""Surrogate kernels (through the C ABI) against the FP64 autograd oracle, and a
short training run judged by the batched RVE solver.

Tolerances.  The 128 x 128 layers multiply bf16 operands with FP32
accumulation.  In the split form (hi*hi + hi*lo + lo*hi) each product keeps
about 16 mantissa bits (relative error ~2^-16), in the plain form 8 bits (unit
roundoff 2^-9 ~ 2e-3); the remaining arithmetic is FP32 (network) and FP64
(head).  The Taylor-free energy subtracts the origin's derivatives, so errors
are measured against the size of the raw network derivatives that enter P and
A: for P, s_W/s * (|g(x)| + |g(0)| + |H(0)| |x|) * 2 |F|; for A,
s_W/s^2 * (|H(x)| + |H(0)|) * 4 |F|^2 plus the S-term of P's bound.  Split
form: 2e-4 of that bound; plain bf16: 3e-2.
"""
import numpy as np
import pytest

import oracle
from oracle import surrogate as OS
from tests import surrogate_model as SM

pytestmark = pytest.mark.gpu


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _A0():
    st, Ch = oracle.linear_homogenized(2, 8, oracle.phase_by_centroid(2, 8, 0.25), oracle.two_phase_lame(10.0))
    assert st == 0
    return Ch


def _F(n, seed, amp=0.2):
    rng = np.random.default_rng(seed)
    F = np.eye(2)[None] + rng.uniform(-amp, amp, (n, 2, 2))
    return F.reshape(n, 4)


def _bounds(theta, desc, F):
    x = OS.scaled_inputs(desc, F)
    g, H = OS.network_derivs(theta, x)
    g0, H0 = OS.network_derivs(theta, np.zeros((1, 3)))
    smin = min(desc["c_scale"])
    nF = np.linalg.norm(F, axis=1)
    bP = desc["w_scale"] / smin * (np.linalg.norm(g, axis=1) + np.linalg.norm(g0) +
                                   np.linalg.norm(H0) * np.linalg.norm(x, axis=1)) * 2 * nF
    bA = desc["w_scale"] / smin ** 2 * (np.linalg.norm(H, axis=(1, 2)) + np.linalg.norm(H0)) * 4 * nF ** 2 + bP
    return bP, bA


@pytest.mark.parametrize("precision,rtol", [(1, 2e-4), (0, 3e-2)])
def test_eval_matches_oracle(precision, rtol):
    torch = torch_cuda()
    from paper_1908_08292_amd import surrogate as S
    A0 = _A0()
    desc = OS.make_desc(A0, w_scale=0.1)
    th = OS.random_params(21, scale=1.5).astype(np.float32).astype(np.float64)
    n = 37  # three tiles, ragged
    F = _F(n, 22)
    F[0] = [1.0, 0.0, 0.0, 1.0]
    Pr, Ar = OS.eval_PA(th, desc, F)
    sg = S.Surrogate(A0, w_scale=0.1)
    sg.set_params(th)
    Fd = torch.tensor(F, device="cuda")
    P = torch.full((n, 4), np.nan, dtype=torch.float64, device="cuda")
    A = torch.full((n, 16), np.nan, dtype=torch.float64, device="cuda")
    ind = torch.zeros(n, dtype=torch.float32, device="cuda")
    sg.eval(Fd, P, A, ind, precision=precision)
    torch.cuda.synchronize()
    P, A, ind = P.cpu().numpy(), A.cpu().numpy(), ind.cpu().numpy()
    bP, bA = _bounds(th, desc, F)
    eP = np.abs(P - Pr).max(1)
    eA = np.abs(A - Ar).max(1)
    print(f"precision {precision}: max eP/bP {np.max(eP / bP):.3e}, max eA/bA {np.max(eA / bA):.3e}")
    assert np.all(eP <= rtol * bP + 1e-14), np.max(eP / bP)
    assert np.all(eA <= rtol * bA + 1e-12), np.max(eA / bA)
    # F = I: the network part vanishes exactly (same arithmetic at x = 0)
    assert np.abs(P[0]).max() < 1e-12
    np.testing.assert_allclose(A[0], Ar[0], rtol=1e-10, atol=1e-12)
    assert np.all(np.isinf(ind))  # not calibrated
    sg.destroy()


@pytest.mark.parametrize("precision", [0, 1])
def test_loss_gradient_matches_oracle(precision):
    torch = torch_cuda()
    from paper_1908_08292_amd import surrogate as S
    A0 = _A0()
    desc = OS.make_desc(A0, w_scale=0.1)
    th = OS.random_params(31, scale=1.5).astype(np.float32).astype(np.float64)
    n = 50  # four training tiles of 15, ragged
    # |x| of order 1: the gradient of the Taylor-free energy is a difference
    # between the network at x and at the origin, so at small |x| the bf16
    # rounding is amplified by about 1/|x|^2; the code path is the same at any x
    F = _F(n, 32, amp=0.45)
    assert np.all(np.linalg.det(F.reshape(-1, 2, 2)) > 0.2)
    # targets O(50%) away from the prediction, so the loss residual is far above
    # the bf16 rounding of the forward pass (about 1% of |P| here)
    P0, A0p = OS.eval_PA(th, desc, F)
    rng = np.random.default_rng(33)
    Pt = P0 * (1.0 + 0.5 * rng.normal(size=P0.shape))
    At = A0p * (1.0 + 0.5 * rng.normal(size=A0p.shape))
    L_ref, g_ref = OS.loss_and_grad(th, desc, F, Pt, At, wP=1.0, wA=0.1, rhoP=1e-3, rhoA=1e-3)
    sg = S.Surrogate(A0, w_scale=0.1)
    sg.set_params(th)
    L, g = sg.loss_grad(torch.tensor(F, device="cuda"), torch.tensor(Pt, device="cuda"),
                        torch.tensor(At, device="cuda"), S.train_opts(precision=precision))
    g = g.cpu().numpy().astype(np.float64)
    print(f"loss gpu {L:.6e} oracle {L_ref:.6e}")
    assert abs(L - L_ref) <= 3e-2 * L_ref
    errs = {}
    for name, a, b in [("W1", OS.OFF_W1, OS.OFF_B1), ("b1", OS.OFF_B1, OS.OFF_W2), ("W2", OS.OFF_W2, OS.OFF_B2),
                       ("b2", OS.OFF_B2, OS.OFF_W3), ("W3", OS.OFF_W3, OS.OFF_B3), ("b3", OS.OFF_B3, OS.OFF_W4),
                       ("w4", OS.OFF_W4, OS.NPARAM)]:
        e = np.linalg.norm(g[a:b] - g_ref[a:b]) / np.linalg.norm(g_ref[a:b])
        errs[name] = e
    print("gradient rel err per block:", {k: f"{v:.2e}" for k, v in errs.items()})
    for name, e in errs.items():
        assert e <= 2e-2, (name, e)
    cos = g @ g_ref / np.linalg.norm(g) / np.linalg.norm(g_ref)
    assert cos > 0.999, cos
    # the same algorithm modelled in numpy, tile by tile, with bf16 rounding at
    # the kernel's rounding points.  Plain bf16: what remains is FP32
    # accumulation order (and the rare bf16 rounding it flips), measured
    # <= 1e-4.  Split forward: the model's forward is exact, the kernel's keeps
    # ~2^-16 per product, amplified by the origin's cancellation (~2e-3).
    Lm, gm = SM.loss_grad(th, desc, F, Pt, At, round_bf16=True, round_fwd=(precision == 0))
    errm = {name: np.linalg.norm(g[a:b] - gm[a:b]) / np.linalg.norm(gm[a:b]) for name, a, b in SM.BLOCKS}
    print("gradient rel err vs bf16 model:", {k: f"{v:.2e}" for k, v in errm.items()})
    for name, e in errm.items():
        assert e <= (5e-4 if precision == 0 else 6e-3), (name, e)
    sg.destroy()


def test_adam_step_matches_oracle():
    torch = torch_cuda()
    from paper_1908_08292_amd import surrogate as S
    A0 = _A0()
    th = OS.random_params(41).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(42)
    sg = S.Surrogate(A0)
    sg.set_params(th)
    opts = S.train_opts(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8)
    ref, m, v = th.copy(), np.zeros_like(th), np.zeros_like(th)
    for t in (1, 2):
        g = rng.normal(size=OS.NPARAM).astype(np.float32).astype(np.float64)
        sg.adam_step(torch.tensor(g, dtype=torch.float32, device="cuda"), opts)
        ref, m, v = OS.adam_step(ref, m, v, g, t, 1e-3)
        got = sg.get_params().astype(np.float64)
        np.testing.assert_allclose(got, ref, rtol=2e-6, atol=2e-8)
    sg.destroy()


def test_select_compacts_indices():
    torch = torch_cuda()
    from paper_1908_08292_amd import surrogate as S
    n = 1000
    rng = np.random.default_rng(5)
    v = rng.uniform(0, 2e-3, n).astype(np.float32)
    v[::97] = np.inf
    v[3] = np.nan
    ind = torch.tensor(v, device="cuda")
    idx, cnt = S.select(ind, 1e-3)
    k = int(cnt.item())
    got = np.sort(idx[:k].cpu().numpy())
    want = np.nonzero(~(v <= 1e-3))[0]
    np.testing.assert_array_equal(got, want)


def test_training_reduces_stress_error_against_rve_judge():
    """Triples from the batched RVE solver (16 x 16 RVE, inclusion r = 0.25,
    ratio 10, H in [-0.2, 0.2]); a short run of the library's own training must
    bring the held-out stress error well below the baseline energy's."""
    torch = torch_cuda()
    from paper_1908_08292_amd import api, surrogate as S, workloads
    n_train, n_test = 6000, 600
    F = workloads.draw_F(np.random.default_rng(77), n_train + n_test, 2, 0.2).reshape(-1, 4)
    batch, meshes = api.build_batch(2, np.full(len(F), 16), np.full(len(F), 0.25), np.full(len(F), 10.0))
    sol = api.Solver(batch)
    sol.set_F(F)
    sol.solve()
    torch.cuda.synchronize()
    res = sol.results()
    ok = res["status"] == 0
    assert ok.mean() > 0.99
    Fd = torch.tensor(F[ok], device="cuda")
    Pd = torch.tensor(res["P"][ok].reshape(-1, 4), device="cuda")
    Ad = torch.tensor(res["A"][ok].reshape(-1, 16), device="cuda")
    # small-strain tangent from the same solver
    b1, _ = api.build_batch(2, np.array([16]), np.array([0.25]), np.array([10.0]))
    s1 = api.Solver(b1)
    s1.set_F(np.eye(2).reshape(1, 4))
    s1.solve()
    A0 = s1.results()["A"][0].reshape(16)
    ntr = int(ok[:n_train].sum())
    sg = S.Surrogate(A0, w_scale=0.1, seed=3)
    th0 = sg.get_params()
    th_base = th0.copy()
    th_base[OS.OFF_W4:] = 0.0  # the quadratic baseline energy alone
    sg.set_params(th_base)
    Ps = torch.empty_like(Pd)
    sg.eval(Fd[ntr:], Ps[ntr:])
    torch.cuda.synchronize()
    sg.set_params(th0)

    def err(Pa, Pb):
        return np.linalg.norm(Pa - Pb, axis=1) / np.linalg.norm(Pb, axis=1)
    e_base = err(Ps[ntr:].cpu().numpy(), Pd[ntr:].cpu().numpy())
    import time
    t0 = time.perf_counter()
    loss = sg.train(Fd[:ntr], Pd[:ntr], Ad[:ntr], S.train_opts(steps=800, batch=1920, lr=3e-3, lr_final=1e-4))
    print(f"800 training steps of 1920 points: {time.perf_counter() - t0:.2f} s")
    sg.eval(Fd[ntr:], Ps[ntr:])
    torch.cuda.synchronize()
    e_net = err(Ps[ntr:].cpu().numpy(), Pd[ntr:].cpu().numpy())
    print(f"loss {loss[0]:.3e} -> {loss[-1]:.3e}; held-out err_P baseline median {np.median(e_base):.2e} "
          f"max {e_base.max():.2e}; trained median {np.median(e_net):.2e} p99 {np.quantile(e_net, 0.99):.2e} "
          f"max {e_net.max():.2e}")
    assert np.all(np.isfinite(loss)) and loss[-1] < 0.1 * loss[0]
    assert np.median(e_net) < 0.25 * np.median(e_base)
    sg.destroy()


def test_subset_solve_matches_full_solve():
    torch = torch_cuda()
    from paper_1908_08292_amd import api, workloads
    B = 300
    F = workloads.draw_F(np.random.default_rng(9), B, 2, 0.15).reshape(-1, 4)
    batch, meshes = api.build_batch(2, np.full(B, 8), np.full(B, 0.25), np.full(B, 10.0))
    full = api.Solver(batch)
    full.set_F(F)
    full.solve()
    sub = api.Solver(batch)
    sub.set_F(F)
    sub.P.fill_(np.nan)
    sub.status.fill_(-7)
    pick = np.array([5, 17, 299, 0, 123, -1, 400, 42], np.int32)  # two entries out of range: skipped
    idx = torch.tensor(pick, device="cuda")
    cnt = torch.tensor([len(pick)], dtype=torch.int32, device="cuda")
    batch.solve_subset(idx, cnt, sub.F, sub.P, sub.A, sub.w, sub.status, sub.iters)
    torch.cuda.synchronize()
    rf, rs = full.results(), sub.results()
    valid = pick[(pick >= 0) & (pick < B)]
    np.testing.assert_array_equal(rs["P"][valid], rf["P"][valid])
    np.testing.assert_array_equal(rs["A"][valid], rf["A"][valid])
    np.testing.assert_array_equal(rs["status"][valid], rf["status"][valid])
    rest = np.setdiff1d(np.arange(B), valid)
    assert np.all(np.isnan(rs["P"][rest])) and np.all(rs["status"][rest] == -7)


@pytest.fixture(scope="module")
def fitted():
    torch_cuda()
    from paper_1908_08292_amd import api
    info = {}
    sg = api.fit_surrogate(n=16, radius=0.25, ratio=10.0, timings=info)
    print("fit:", info)
    yield sg, info
    sg.destroy()


def test_surrogate_audit_against_rve_judge(fitted):
    """Fresh judged sample (4000 points, 2% of the training size) from the same
    generator: every point the indicator accepts at 1e-3 is within 1e-3 of the
    RVE solve in P, and most points are accepted."""
    torch = torch_cuda()
    from paper_1908_08292_amd import api, workloads
    sg, _ = fitted
    n = 4000
    F = workloads.draw_F(np.random.default_rng(2024), n, 2, 0.2).reshape(-1, 4)
    batch, _ = api.build_batch(2, np.full(n, 16), np.full(n, 0.25), np.full(n, 10.0))
    sol = api.Solver(batch, keep_state=False)
    sol.set_F(F)
    sol.solve()
    Fd = sol.F.view(-1, 4)
    Ps = torch.empty(n, 4, dtype=torch.float64, device="cuda")
    As = torch.empty(n, 16, dtype=torch.float64, device="cuda")
    ind = torch.empty(n, dtype=torch.float32, device="cuda")
    sg.eval(Fd, Ps, As, ind)
    torch.cuda.synchronize()
    Pj = sol.P.view(-1, 4).cpu().numpy()
    Aj = sol.A.view(-1, 16).cpu().numpy()
    ok = sol.status.cpu().numpy() == 0
    e = np.linalg.norm(Ps.cpu().numpy() - Pj, axis=1) / np.linalg.norm(Pj, axis=1)
    eA = np.linalg.norm(As.cpu().numpy() - Aj, axis=1) / np.linalg.norm(Aj, axis=1)
    acc = (ind.cpu().numpy() <= 1e-3) & ok
    print(f"accepted {acc.mean():.3f}; err_P accepted max {e[acc].max():.2e} p99 {np.quantile(e[acc], .99):.2e}; "
          f"all points median {np.median(e[ok]):.2e}; err_A accepted median {np.median(eA[acc]):.2e}")
    assert acc.mean() > 0.5
    assert e[acc].max() <= 1e-3


def test_surrogate_gain_on_two_scale_problem(fitted):
    """Plate with a hole (16 x 16 macro grid, r = 0.2, uniaxial stretch to 1.15 in
    20 steps, first 4 steps), nested two-level Newton on 16 x 16 RVEs, with and
    without the surrogate: the surrogate run must reach the same macro solution
    (relative displacement difference below 1e-3) with a fraction of the RVE
    solves and in less time.  With the surrogate the macro Newton stops at 1e-4
    of the step's first residual (its stresses carry FP32 rounding); the plain
    run converges to 1e-10."""
    torch = torch_cuda()
    import time
    from paper_1908_08292_amd import fehmm, rve
    sg, _ = fitted
    lame = rve.two_phase_lame(10.0)
    res = {}
    for use in (False, True):
        mesh = rve.Mesh(2, 16, lame, radius=0.25)
        drv = fehmm.Driver(mesh, nx=16, ny=16, hole_r=0.2, bc=fehmm.BC_UNIAXIAL, stretch=1.15, nsteps=20)
        if use:
            drv.set_surrogate(sg, threshold=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solves = evals = 0
        for k in range(1, 5):
            st = drv.step(k)
            assert st["status"] == 0, (use, k, st)
            n_eval = (st["macro_iters"] + 1) * drv.nqp
            solves += st["fallback_points"] if use else n_eval
            evals += n_eval
        dt = time.perf_counter() - t0
        res[use] = dict(u=drv.u(), t=dt, solves=solves, evals=evals)
        drv.destroy()
    du = np.linalg.norm(res[True]["u"] - res[False]["u"]) / np.linalg.norm(res[False]["u"])
    frac = res[True]["solves"] / res[True]["evals"]
    print(f"RVE solves {res[False]['solves']} -> {res[True]['solves']} ({frac:.3f} of evaluations); "
          f"time {res[False]['t']:.3f} s -> {res[True]['t']:.3f} s; rel |du| {du:.2e}")
    assert du < 1e-3
    assert frac < 0.5
    assert res[True]["t"] < res[False]["t"]
