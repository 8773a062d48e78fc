"""P1 micro elements (the paper's linear simplices; every grid cell split into d!
Kuhn simplices) on the GPU against the FP64 oracle with the same elements:
P rel <= 1e-8, A rel <= 1e-6, equal statuses and Newton counts (FP64), in 2D
and 3D, with FP32 factors, and combined with the other laws and with KUBC."""
import numpy as np
import pytest

import oracle
from paper_1908_08292_amd import api, rve, workloads

pytestmark = pytest.mark.gpu
P_TOL, A_TOL = 1e-8, 1e-6


def _run(d, wl, prec="fp64", law=rve.LAW_NEOHOOKE, bc=rve.BC_PERIODIC):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    batch, meshes = api.build_batch(d, wl.n, wl.radius, wl.ratio, law=law, bc=bc, elem=rve.ELEM_P1)
    s = api.Solver(batch)
    s.set_F(wl.F)
    s.solve(opts=rve.default_opts(precision=rve.PREC_FP64 if prec == "fp64" else rve.PREC_FP32_IR))
    torch.cuda.synchronize()
    return s.results()


def _compare(d, wl, out, exact_iters=True, olaw=oracle.LAW_NEOHOOKE, obc=oracle.BC_PERIODIC):
    worst = [0.0, 0.0]
    with oracle.element_kind(oracle.ELEM_P1), oracle.law(olaw), oracle.bc(obc):
        for b in range(len(wl.F)):
            n = int(wl.n[b])
            lame = oracle.two_phase_lame(float(wl.ratio[b]))
            ref = oracle.rve_solve(d, n, oracle.phase_by_centroid(d, n, float(wl.radius[b])), lame, wl.F[b])
            assert out["status"][b] == ref["status"] == 0, (b, out["status"][b], ref["status"])
            if exact_iters:
                assert out["iters"][b] == ref["iters"], (b, out["iters"][b], ref["iters"])
            else:
                assert abs(int(out["iters"][b]) - ref["iters"]) <= 1
            fl = 1e-12 * lame[:, 1].max()
            eP = np.linalg.norm(out["P"][b] - ref["P"]) / max(np.linalg.norm(ref["P"]), fl)
            eA = np.linalg.norm(out["A"][b] - ref["A"]) / max(np.linalg.norm(ref["A"]), fl)
            worst = [max(worst[0], eP), max(worst[1], eA)]
            assert eP <= P_TOL and eA <= A_TOL, (b, eP, eA)
    print(f"  worst P {worst[0]:.2e} A {worst[1]:.2e}", flush=True)


@pytest.mark.parametrize("d,n", [(2, 2), (2, 3), (2, 4), (2, 8), (2, 16), (2, 32), (3, 2), (3, 3), (3, 4), (3, 6)])
def test_p1_parity(d, n):
    B = 5 if n < 16 else 3
    wl = workloads.rve2d(B, n=n, seed=1600 + n) if d == 2 else workloads.rve3d(B, sizes=(n,), seed=1700 + n)
    print(f"case p1 {d}d n={n} B={B}", flush=True)
    _compare(d, wl, _run(d, wl))


@pytest.mark.parametrize("d,n", [(2, 16), (2, 32), (3, 6)])
def test_p1_fp32_factors(d, n):
    wl = workloads.rve2d(3, n=n, seed=1800 + n) if d == 2 else workloads.rve3d(2, sizes=(n,), seed=1800 + n)
    print(f"case p1 {d}d n={n} fp32ir", flush=True)
    _compare(d, wl, _run(d, wl, "fp32ir"), exact_iters=False)


def test_p1_with_linear_law_and_kubc():
    wl = workloads.rve2d(4, n=8, seed=1900)
    print("case p1 2d n=8: fully linear law; kubc", flush=True)
    _compare(2, wl, _run(2, wl, law=rve.LAW_LINEAR), olaw=oracle.LAW_LINEAR)
    _compare(2, wl, _run(2, wl, bc=rve.BC_LINEAR), obc=oracle.BC_LINEAR)
