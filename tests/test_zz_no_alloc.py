"""rve_solve_batch_static (workspace in the library's static device array, no
allocation) against rve_solve_batch on the same inputs, through the C ABI: two
calls in a row, the second with a smaller batch of smaller RVEs.  Both run the
same kernels, so the outputs are bitwise identical."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1908_08292_amd import api, rve, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(wl, static, w0=None, d=2, opts=None):
    batch, meshes = api.build_batch(d, wl.n, wl.radius, wl.ratio)
    s = api.Solver(batch)
    s.set_F(wl.F)
    if w0 is not None:
        s.w.copy_(w0)
    # outputs start as garbage so that stale contents cannot pass
    s.P.fill_(7.0)
    s.A.fill_(7.0)
    s.status.fill_(9)
    s.iters.fill_(-1)
    batch.solve(s.F, s.P, s.A, s.w, s.status, s.iters, opts=opts, static=static)
    torch.cuda.synchronize()
    out = s.results()
    out["w"] = s.w.cpu().numpy()
    batch.destroy()
    for m in set(meshes):
        m.destroy()
    return out


def _same(a, b):
    for k in ("P", "A", "status", "iters", "w"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_static_matches_allocating_entry_point_twice():
    print("[no_alloc] call 1: 1200 RVEs of 32x32 (more RVEs than static slots)", flush=True)
    big = workloads.rve2d(1200, n=32, seed=2024)
    ref1 = _run(big, static=False)
    got1 = _run(big, static=True)
    assert np.all(ref1["status"] == 0)
    _same(got1, ref1)
    print("[no_alloc] call 2: 50 RVEs of 8x8 with a warm start", flush=True)
    small = workloads.rve2d(50, n=8, seed=2025)
    w0 = torch.zeros(50 * 2 * 64, dtype=torch.float64, device="cuda")
    ref2 = _run(small, static=False, w0=w0)
    got2 = _run(small, static=True, w0=w0)
    assert np.all(ref2["status"] == 0)
    _same(got2, ref2)


def test_static_matches_allocating_entry_point_3d_fp32():
    """The same on global-front plans (3D 6^3 and 8^3) with FP32 factors."""
    print("[no_alloc] 3D: 8 RVEs of 6^3 / 8^3, FP32 factors", flush=True)
    wl = workloads.rve3d(8, sizes=(6, 8), seed=2026)
    o = rve.default_opts(precision=rve.PREC_FP32_IR)
    ref = _run(wl, static=False, d=3, opts=o)
    got = _run(wl, static=True, d=3, opts=o)
    assert np.all(ref["status"] == 0)
    _same(got, ref)


def test_static_rejects_a_slot_larger_than_the_array():
    print("[no_alloc] rejection: one 3D 20^3 RVE", flush=True)
    lame = rve.two_phase_lame(10.0)
    mesh = rve.Mesh(3, 20, lame, radius=0.3)
    batch = rve.Batch([mesh])
    F = torch.eye(3, dtype=torch.float64, device="cuda").reshape(-1).contiguous()
    P = torch.zeros(9, dtype=torch.float64, device="cuda")
    with pytest.raises(rve.RveError) as ei:
        batch.solve(F, P, static=True)
    assert ei.value.code == rve.RVE_EINVAL
    assert "static scratch" in rve.last_error()
    batch.destroy()
    mesh.destroy()
