"""Pins of the oracle's macro FE-HMM driver."""
import numpy as np
import pytest

import oracle
from tests import fe_ref

LAME = oracle.two_phase_lame(10.0)


def _cell_points(elem, hx, hy):
    """Integration points of one cell: (gradients [4 nodes, 2], weight) each.
    Q1: 2x2 Gauss; P1: the triangles (0,1,2) and (0,2,3) of the counter-clockwise
    cell nodes, gradients from the inverted edge matrix of the vertex coordinates."""
    X = np.array([[0.0, 0.0], [hx, 0.0], [hx, hy], [0.0, hy]])
    pts = []
    if elem == 0:
        g = 1 / np.sqrt(3)
        sx, sy = np.array([-1, 1, 1, -1]), np.array([-1, -1, 1, 1])
        for xi, eta in [(-g, -g), (g, -g), (g, g), (-g, g)]:
            dN = np.zeros((4, 2))
            dN[:, 0] = 0.25 * sx * (1 + sy * eta) * 2 / hx
            dN[:, 1] = 0.25 * sy * (1 + sx * xi) * 2 / hy
            pts.append((dN, hx * hy / 4))
    else:
        for tri in ((0, 1, 2), (0, 2, 3)):
            E = np.array([X[tri[1]] - X[tri[0]], X[tri[2]] - X[tri[0]]]).T
            Gi = np.linalg.inv(E)
            G = np.vstack([-Gi.sum(axis=0), Gi])
            dN = np.zeros((4, 2))
            for k, a in enumerate(tri):
                dN[a] = G[k]
            pts.append((dN, abs(np.linalg.det(E)) / 2))
    return pts


def single_scale_fe(nx, ny, lam, mu, stretch, nsteps, bc, through_solve=False, hist=None, elem=0):
    """Independent dense single-scale Q1 neo-Hookean FE with the same BCs.
    through_solve: the step's prescribed increment enters the first Newton
    iteration as an inhomogeneous Dirichlet condition of the linear system
    (otherwise it is written into u before the first iteration); hist, a list,
    receives each step's residual history normalized to its first residual."""
    hx, hy = 1.0 / nx, 1.0 / ny
    nn = (nx + 1) * (ny + 1)
    xy = np.array([[i * hx, j * hy] for j in range(ny + 1) for i in range(nx + 1)])
    conn = np.array([[j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i]
                     for j in range(ny) for i in range(nx)])
    pts = _cell_points(elem, hx, hy)
    fixed = np.zeros(2 * nn, bool)
    for v, (x, y) in enumerate(xy):
        if x == 0:
            fixed[2 * v] = True
            if bc == 0 or y == 0:
                fixed[2 * v + 1] = True
        if abs(x - 1) < 1e-12:
            fixed[2 * v] = True
    u = np.zeros(2 * nn)
    right = np.zeros(2 * nn, bool)
    right[0::2] = np.abs(xy[:, 0] - 1) < 1e-12
    for k in range(1, nsteps + 1):
        target = np.where(right, (stretch - 1) * k / nsteps, 0.0)
        dud = np.where(fixed, target - u, 0.0)
        if not through_solve:
            u[fixed] = target[fixed]
            dud[:] = 0.0
        r0 = None
        h = []
        for it in range(30):
            R = np.zeros(2 * nn); K = np.zeros((2 * nn, 2 * nn))
            for e in conn:
                dofs = np.ravel([[2 * a, 2 * a + 1] for a in e])
                for dN, wdet in pts:
                    F = np.eye(2) + np.einsum("ai,aJ->iJ", u[dofs].reshape(4, 2), dN)
                    P = fe_ref.P_closed(F, lam, mu)
                    A = fe_ref.A_closed(F, lam, mu).reshape(2, 2, 2, 2)
                    R[dofs] += np.einsum("iJ,aJ->ai", P, dN).ravel() * wdet
                    K[np.ix_(dofs, dofs)] += np.einsum("aJ,iJkL,bL->aibk", dN, A, dN).reshape(8, 8) * wdet
            free = ~fixed
            if it == 0:
                R[free] += K[np.ix_(free, fixed)] @ dud[fixed]
            rn = np.linalg.norm(R[free])
            r0 = rn if r0 is None else r0
            h.append(rn / r0)
            if rn <= 1e-12 * r0:
                break
            u[free] -= np.linalg.solve(K[np.ix_(free, free)], R[free])
            if it == 0:
                u[fixed] += dud[fixed]
        if hist is not None:
            hist.append(np.array(h))
    return xy, u


@pytest.mark.parametrize("bc", [0, 1])
def test_homogeneous_rve_fe_hmm_equals_single_scale_fe(bc):
    """e_mod = 0 for periodic coupling (Sec. 4): with a one-phase RVE the FE-HMM
    macro solution is the single-scale FE solution of the same law."""
    nx = ny = 3
    n = 2
    ph = np.zeros(n * n, np.uint8)
    m = oracle.Macro(nx, ny, n, ph, LAME, bc=bc, stretch=1.1, nsteps=2, rtol_macro=1e-12)
    for k in (1, 2):
        st = m.step(k)
        assert st["status"] == 0
    xy_ref, u_ref = single_scale_fe(nx, ny, *LAME[0], 1.1, 2, bc)
    xy = m.nodes()
    u = m.u()
    order = [int(np.argmin(np.abs(xy_ref - p).sum(axis=1))) for p in xy]
    u_ref = u_ref.reshape(-1, 2)[order].reshape(-1)
    assert np.abs(u - u_ref).max() < 1e-10 * np.abs(u_ref).max()


@pytest.mark.parametrize("bc", [0, 1])
def test_load_increment_enters_through_the_solve(bc):
    """With a one-phase RVE the FE-HMM macro Newton is the single-scale FE
    Newton iteration by iteration.  The independent single-scale code applies
    each step's prescribed increment as an inhomogeneous Dirichlet condition of
    the first linear solve (K_ff du_f = -(R_f + K_fd du_d)); the oracle's
    residual histories, normalized to that load-equivalent first residual,
    and its solution must follow it."""
    nx = ny = 3
    ph = np.zeros(4, np.uint8)
    m = oracle.Macro(nx, ny, 2, ph, LAME, bc=bc, stretch=1.1, nsteps=2, rtol_macro=1e-12)
    hist = []
    xy_ref, u_ref = single_scale_fe(nx, ny, *LAME[0], 1.1, 2, bc, through_solve=True, hist=hist)
    for k in (1, 2):
        st = m.step(k)
        assert st["status"] == 0
        h_ref = hist[k - 1]
        assert st["macro_iters"] == len(h_ref) - 1
        # early iterates agree tightly; the last ones sit at round-off
        big = h_ref > 1e-8
        assert np.allclose(st["res_hist"][big], h_ref[big], rtol=1e-6)
    xy = m.nodes()
    order = [int(np.argmin(np.abs(xy_ref - p).sum(axis=1))) for p in xy]
    u_ref = u_ref.reshape(-1, 2)[order].reshape(-1)
    assert np.abs(m.u() - u_ref).max() < 1e-10 * np.abs(u_ref).max()
    # the other way of applying the increment takes a different path
    hist_w = []
    single_scale_fe(nx, ny, *LAME[0], 1.1, 2, bc, through_solve=False, hist=hist_w)
    assert len(hist_w[0]) != len(hist[0]) or not np.allclose(hist_w[0], hist[0], rtol=1e-3)


def test_uniaxial_stretch_gives_uniform_macro_state():
    """Roller BCs (bc 1) with free top/bottom: the homogeneous macro state is an
    equilibrium, so every quadrature point sees the same Fbar, Pbar."""
    n = 4
    ph = oracle.phase_by_centroid(2, n, 0.3)
    m = oracle.Macro(2, 2, n, ph, LAME, bc=1, stretch=1.08, nsteps=1)
    st = m.step(1)
    assert st["status"] == 0
    F, P, A = m.qp()
    assert np.abs(F - F[0]).max() < 1e-10
    assert F[0, 0, 0] == pytest.approx(1.08, abs=1e-12)
    # traction-free top/bottom: P_21 = P_22 = 0 on average state; P_12 = 0 by symmetry
    assert np.abs(P[0, 1, :]).max() < 1e-10 * abs(P[0, 0, 0])


def test_nested_newton_is_quadratic_and_alternating_agrees():
    """Algorithm 1 (nested) converges quadratically in the macro residual; the
    alternating Algorithm 2 reaches the same macro solution (Sec. 5)."""
    n = 4
    ph = oracle.phase_by_centroid(2, n, 0.25)
    kw = dict(bc=0, stretch=1.1, nsteps=2, rtol_macro=1e-10)
    mn = oracle.Macro(3, 3, n, ph, LAME, scheme=0, **kw)
    ma = oracle.Macro(3, 3, n, ph, LAME, scheme=1, **kw)
    for k in (1, 2):
        sn = mn.step(k)
        sa = ma.step(k)
        assert sn["status"] == 0 and sa["status"] == 0
        h = sn["res_hist"]
        assert h[-1] <= 1e-10
        assert h[-2] < 1e-3 and h[-1] <= 10 * h[-2] ** 2
    assert np.abs(mn.u() - ma.u()).max() < 1e-7 * np.abs(mn.u()).max()


def test_holed_plate_mesh_counts():
    """The 64 x 64 plate with a centred hole of radius 0.2 (elements removed by
    centroid, strict '<'): 3572 kept elements, 14288 quadrature points, 3752
    nodes (7504 dofs), counted here by brute force over the grid, and equal to
    the counts derived for this workload beforehand."""
    nx = ny = 64
    h = 1.0 / nx
    keep = np.zeros((ny, nx), bool)
    for j in range(ny):
        for i in range(nx):
            keep[j, i] = np.hypot((i + 0.5) * h - 0.5, (j + 0.5) * h - 0.5) >= 0.2
    used = np.zeros((ny + 1, nx + 1), bool)
    for j, i in zip(*np.nonzero(keep)):
        used[j:j + 2, i:i + 2] = True
    assert keep.sum() == 3572 and used.sum() == 3752
    ph = oracle.phase_by_centroid(2, 2, 0.25)
    m = oracle.Macro(nx, ny, 2, ph, LAME, hole_r=0.2, bc=1, stretch=1.15, nsteps=20)
    assert m.nqp == 4 * 3572 == 14288
    assert m.ndof == 2 * 3752 == 7504
    xy = m.nodes()
    # exactly the grid nodes of kept elements, none inside the hole's removed core
    got = {(int(round(x / h)), int(round(y / h))) for x, y in xy}
    want = {(i, j) for j, i in zip(*np.nonzero(used))}
    assert got == want
    m.close()


@pytest.mark.parametrize("bc", [0, 1])
def test_p1_macro_triangles_equal_single_scale_fe(bc):
    """P1 macro triangles (each grid cell split along its (0,0)-(1,1) diagonal,
    one point per triangle, Sec. 3.1 macro spaces): with a one-phase RVE the
    FE-HMM solution is the single-scale P1 FE solution, residual history by
    residual history, and the literal transfer equals B^T Abar B."""
    nx = ny = 3
    m = oracle.Macro(nx, ny, 2, np.zeros(4, np.uint8), LAME, bc=bc, stretch=1.1, nsteps=2, rtol_macro=1e-12,
                     elem=1)
    assert m.nqp == 2 * nx * ny
    hist = []
    xy_ref, u_ref = single_scale_fe(nx, ny, *LAME[0], 1.1, 2, bc, through_solve=True, hist=hist, elem=1)
    for k in (1, 2):
        st = m.step(k)
        assert st["status"] == 0 and st["macro_iters"] == len(hist[k - 1]) - 1
    xy = m.nodes()
    order = [int(np.argmin(np.abs(xy_ref - p).sum(axis=1))) for p in xy]
    u_ref = u_ref.reshape(-1, 2)[order].reshape(-1)
    assert np.abs(m.u() - u_ref).max() < 1e-10 * np.abs(u_ref).max()
    # with the clamped edge the field is not affine and the P1 and Q1 solutions
    # differ; under uniaxial stretch both spaces hold the uniform solution
    _, u_q1 = single_scale_fe(nx, ny, *LAME[0], 1.1, 2, bc, through_solve=True)
    diff = np.abs(u_q1.reshape(-1, 2)[order].reshape(-1) - u_ref).max()
    if bc == 0:
        assert diff > 1e-8 * np.abs(u_ref).max()
    else:
        assert diff < 1e-12 * np.abs(u_ref).max()
    m.close()


def test_p1_macro_literal_transfer_and_uniform_state():
    n = 4
    ph = oracle.phase_by_centroid(2, n, 0.3)
    m = oracle.Macro(3, 3, n, ph, LAME, bc=0, stretch=1.1, nsteps=2, elem=1)
    for k in (1, 2):
        assert m.step(k)["status"] == 0
    for e in range(m.nelem()):
        kl, kc = m.element_stiffness(e, True), m.element_stiffness(e, False)
        assert np.abs(kl - kc).max() <= 1e-11 * np.abs(kc).max()
    m.close()
    u = oracle.Macro(2, 2, n, ph, LAME, bc=1, stretch=1.08, nsteps=1, elem=1)
    assert u.step(1)["status"] == 0
    F, _, _ = u.qp()
    assert np.abs(F - F[0]).max() < 1e-10 and F[0, 0, 0] == pytest.approx(1.08, abs=1e-12)
    u.close()
