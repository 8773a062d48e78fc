"""Macro driver (fehmm_macro_step) on the GPU against the oracle's macro driver."""
import numpy as np
import pytest

import oracle
from paper_1908_08292_amd import fehmm, rve
from tests.test_oracle_macro import single_scale_fe

pytestmark = pytest.mark.gpu


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def match_u(xy_a, u_a, xy_b, u_b):
    order = [int(np.argmin(np.abs(xy_b - p).sum(axis=1))) for p in xy_a]
    return u_b.reshape(-1, 2)[order].reshape(-1)


def run_pair(nx, ny, n, r, nsteps, stretch, bc, scheme, hole_r=0.0, steps=None, micro_opts=None):
    lame = rve.two_phase_lame(10.0)
    mesh = rve.Mesh(2, n, lame, radius=r)
    drv = fehmm.Driver(mesh, nx, ny, hole_r=hole_r, bc=bc, stretch=stretch, nsteps=nsteps, scheme=scheme,
                       micro_opts=micro_opts)
    orc = oracle.Macro(nx, ny, n, oracle.phase_by_centroid(2, n, r), oracle.two_phase_lame(10.0), hole_r=hole_r,
                       bc=bc, stretch=stretch, nsteps=nsteps, scheme=scheme)
    out = []
    for k in (steps or range(1, nsteps + 1)):
        g = drv.step(k)
        o = orc.step(k)
        print(f"  step {k}: gpu macro iters {g['macro_iters']} hist {g['res_hist'][-1]:.2e}, "
              f"oracle {o['macro_iters']}", flush=True)
        assert g["status"] == 0 and o["status"] == 0
        assert g["macro_iters"] == o["macro_iters"]
        ug = drv.u()
        uo = match_u(drv.nodes(), ug, orc.nodes(), orc.u())
        err = np.abs(ug - uo).max() / max(np.abs(uo).max(), 1e-300)
        assert err < 1e-8, (k, err)
        out.append((g, o, err))
    return drv, orc, out


@pytest.mark.parametrize("scheme", [fehmm.NESTED, fehmm.ALTERNATING])
def test_macro_parity_small(scheme):
    need_gpu()
    print(f"case macro 3x3, RVE 4x4, scheme {scheme}", flush=True)
    run_pair(3, 3, 4, 0.3, 3, 1.1, fehmm.BC_CLAMPED_PULL, scheme)


@pytest.mark.parametrize("scheme", [fehmm.NESTED, fehmm.ALTERNATING])
def test_macro_parity_fp32_micro_solves(scheme):
    """The driver with FP32 micro assembly and factors (FP64 refinement): the
    micro outputs meet the FP64 bar, so the macro Newton takes the oracle's
    iterations and reaches its displacements."""
    need_gpu()
    print(f"case macro 4x4, RVE 8x8, FP32 micro solves, scheme {scheme}", flush=True)
    run_pair(4, 4, 8, 0.25, 3, 1.1, fehmm.BC_CLAMPED_PULL, scheme,
             micro_opts=rve.default_opts(precision=rve.PREC_FP32_IR))


def test_macro_parity_uniaxial_with_hole():
    need_gpu()
    print("case macro 6x6 with hole, RVE 4x4, uniaxial", flush=True)
    drv, orc, out = run_pair(6, 6, 4, 0.3, 2, 1.08, fehmm.BC_UNIAXIAL, fehmm.NESTED, hole_r=0.2)
    assert drv.nqp == orc.nqp


@pytest.mark.parametrize("nx,ny", [(70, 2), (90, 1), (120, 1)])
def test_macro_parity_wide_band(nx, ny):
    """The band solvers past the windowed one: an nx-element-wide plate has band
    width 2 (nx + 2) + 1; 70 wide (bw 145) is just past the LDS window (tile rows
    (bw + 15) / 16 + 1 <= 10), so the panel solver runs with three panel rows per
    lane, 90 wide (bw 185) with four, and 120 wide (bw 245) takes the unblocked
    solver.  (The 64 x 64 plate, bw 133, and every smaller plate run the windowed
    solver.)"""
    need_gpu()
    print(f"case macro {nx}x{ny}, RVE 4x4, wide band", flush=True)
    run_pair(nx, ny, 4, 0.3, 2, 1.05, fehmm.BC_UNIAXIAL, fehmm.NESTED)


def test_macro_parity_window_edge():
    """The widest band of the windowed solver: 64 elements wide, bw = 2 (65 + 1)
    + 1 = 133, ten tile rows; a short plate so the window reaches its last panels
    while still full."""
    need_gpu()
    print("case macro 64x3, RVE 4x4", flush=True)
    run_pair(64, 3, 4, 0.3, 2, 1.05, fehmm.BC_UNIAXIAL, fehmm.NESTED)


def test_config0_full():
    """Macro 4 x 4 Q1 on the unit square, RVE 8 x 8 (r = 0.25, ratio 10), left edge
    clamped, right edge stretched to 1.1 in 10 steps, both Newton levels 1e-10."""
    need_gpu()
    print("case config 0 (10 steps)", flush=True)
    drv, orc, out = run_pair(4, 4, 8, 0.25, 10, 1.1, fehmm.BC_CLAMPED_PULL, fehmm.NESTED)
    for g, o, err in out:
        h = g["res_hist"]
        assert h[-1] <= 1e-10


def test_homogeneous_rve_equals_single_scale():
    need_gpu()
    lame = rve.two_phase_lame(10.0)
    mesh = rve.Mesh(2, 3, lame, phase=np.zeros(9, np.uint8))
    drv = fehmm.Driver(mesh, 3, 3, bc=fehmm.BC_CLAMPED_PULL, stretch=1.1, nsteps=2, rtol_macro=1e-12)
    for k in (1, 2):
        assert drv.step(k)["status"] == 0
    xy_ref, u_ref = single_scale_fe(3, 3, *lame[0], 1.1, 2, 0)
    u = drv.u()
    u_ref = match_u(drv.nodes(), u, xy_ref, u_ref)
    assert np.abs(u - u_ref).max() < 1e-10 * np.abs(u_ref).max()


def test_checkpoint_resume_bitwise():
    need_gpu()
    lame = rve.two_phase_lame(10.0)
    mesh = rve.Mesh(2, 4, lame, radius=0.3)
    kw = dict(bc=fehmm.BC_CLAMPED_PULL, stretch=1.1, nsteps=4)
    a = fehmm.Driver(mesh, 3, 3, **kw)
    for k in range(1, 5):
        a.step(k)
    b = fehmm.Driver(mesh, 3, 3, **kw)
    for k in (1, 2):
        b.step(k)
    u, w = b.get_state()
    b.destroy()
    c = fehmm.Driver(mesh, 3, 3, **kw)
    c.set_state(u, w)
    for k in (3, 4):
        c.step(k)
    assert np.array_equal(a.u(), c.u())


@pytest.mark.parametrize("nx", [20, 60, 100, 130])
def test_uniaxial_homogeneous_exact(nx):
    """Homogeneous RVE, uniaxial stretch a = 1.02 in 4 load steps (the first
    Newton iterate of a step has the increment only on the right edge, one
    element wide): the discrete solution is the
    homogeneous deformation u = ((a - 1) x, (b - 1) y) with P22 = 0, i.e.
    b^2 = (mu + lam/2) / (mu + lam a^2 / 2) for P = mu F - (mu - lam/2 (J^2 - 1)) F^-T.
    The grid sizes give band widths 43, 123, 203 and 263, which exercise every
    variant of the macro band solver (panel registers per lane 2, 3, 4, and the
    unblocked kernel beyond width 240)."""
    need_gpu()
    print(f"case uniaxial homogeneous {nx} x {nx}", flush=True)
    lame = rve.two_phase_lame(10.0)
    lam, mu = lame[0]
    mesh = rve.Mesh(2, 3, lame, phase=np.zeros(9, np.uint8))
    a = 1.02
    drv = fehmm.Driver(mesh, nx, nx, bc=fehmm.BC_UNIAXIAL, stretch=a, nsteps=4, rtol_macro=1e-12)
    for k in range(1, 5):
        st = drv.step(k)
        assert st["status"] == 0 and st["macro_iters"] <= 8, (k, st)
    b = np.sqrt((mu + lam / 2) / (mu + lam * a * a / 2))
    xy = drv.nodes()
    u = drv.u().reshape(-1, 2)
    ue = np.stack([(a - 1) * xy[:, 0], (b - 1) * xy[:, 1]], 1)
    assert np.abs(u - ue).max() <= 1e-9, np.abs(u - ue).max()


@pytest.mark.parametrize("scheme", [fehmm.NESTED, fehmm.ALTERNATING])
def test_graph_step_matches_eager(scheme):
    """A load step replayed as one captured graph gives bitwise the same
    displacements, iteration counts and residual history as the eager path."""
    need_gpu()
    print(f"case graph vs eager, scheme {scheme}", flush=True)
    lame = rve.two_phase_lame(10.0)
    mesh = rve.Mesh(2, 4, lame, radius=0.3)
    kw = dict(hole_r=0.2, bc=fehmm.BC_UNIAXIAL, stretch=1.08, nsteps=3, scheme=scheme)
    a = fehmm.Driver(mesh, 6, 6, **kw)
    b = fehmm.Driver(mesh, 6, 6, **kw)
    b.set_graph(True)
    for k in (1, 2, 3):
        sa, sb = a.step(k), b.step(k)
        assert sa["status"] == sb["status"] == 0
        assert sa["macro_iters"] == sb["macro_iters"] and sa["micro_iters"] == sb["micro_iters"]
        assert np.array_equal(sa["res_hist"], sb["res_hist"])
        assert np.array_equal(a.u(), b.u()), k


@pytest.mark.parametrize("scheme", [fehmm.NESTED, fehmm.ALTERNATING])
def test_p1_macro_parity(scheme):
    """P1 macro triangles (Sec. 3.1 macro spaces; each cell split along its
    (0,0)-(1,1) diagonal, one point per triangle) against the oracle's driver."""
    need_gpu()
    print(f"case P1 macro 4x4, RVE 8x8, scheme {scheme}", flush=True)
    lame = rve.two_phase_lame(10.0)
    n, r = 8, 0.25
    mesh = rve.Mesh(2, n, lame, radius=r)
    drv = fehmm.Driver(mesh, 4, 4, bc=fehmm.BC_CLAMPED_PULL, stretch=1.1, nsteps=3, scheme=scheme,
                       elem=fehmm.ELEM_P1)
    orc = oracle.Macro(4, 4, n, oracle.phase_by_centroid(2, n, r), oracle.two_phase_lame(10.0), bc=0, stretch=1.1,
                       nsteps=3, scheme=scheme, elem=1)
    assert drv.nqp == orc.nqp == 32
    for k in (1, 2, 3):
        g, o = drv.step(k), orc.step(k)
        assert g["status"] == 0 and o["status"] == 0 and g["macro_iters"] == o["macro_iters"]
        uo = match_u(drv.nodes(), drv.u(), orc.nodes(), orc.u())
        assert np.abs(drv.u() - uo).max() <= 1e-8 * np.abs(uo).max()
    drv.destroy()
    orc.close()
