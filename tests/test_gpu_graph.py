"""A batch solve captured in a HIP graph: the persistent launch and its queue
reset become two kernel nodes (no memset node), and every replay must equal the
eager launch bitwise, with the program's own eager work between replays."""
import numpy as np
import pytest

from paper_1908_08292_amd import api, rve, workloads

pytestmark = pytest.mark.gpu


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def uneven(d):
    if d == 3:
        return workloads.rve3d(8, sizes=(4, 6, 8), seed=1700)
    # 32 x 32 FP64 fronts: the eight-wave solver
    wl = workloads.rve2d(48, seed=1701)
    wl.n[:] = np.resize(np.array([8, 16, 32], np.int32), 48)
    return wl


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32ir"])
def test_uneven_batch_graph_replays_match_eager(d, prec):
    torch = torch_cuda()
    wl = uneven(d)
    print(f"case graph replay, {d}d uneven n={list(wl.n)}, {prec}", flush=True)
    batch, meshes = api.build_batch(d, wl.n, wl.radius, wl.ratio)
    s = api.Solver(batch, keep_state=False)
    s.set_F(wl.F)
    o = rve.default_opts(precision=rve.PREC_FP32_IR if prec == "fp32ir" else rve.PREC_FP64)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s.solve(opts=o, stream=st.cuda_stream)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (s.P, s.A, s.status, s.iters)]
    assert int((ref[2] != 0).sum()) == 0
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        s.solve(opts=o, stream=st.cuda_stream)
    for k in range(3):
        # eager work of the program between replays: outputs overwritten
        s.P.fill_(float("nan"))
        s.A.fill_(0.0)
        s.status.fill_(-1)
        s.iters.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip((s.P, s.A, s.status, s.iters), ref):
            assert torch.equal(got, want), k
    del g
    torch.cuda.synchronize()
