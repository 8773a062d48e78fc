"""Pins of the oracle's constitutive variants: geometrically nonlinear linear
elasticity (St. Venant-Kirchhoff) and the fully linear case, the two laws the
paper sets beside the neo-Hookean law in its micro-convergence comparisons
(Sec. 6).  None of the expected values re-calls the oracle's formulas: they come
from finite differences of its own energy, from properties the laws must have
(reference state, homogeneity in the strain, objectivity, linearity), from the
separate small-strain cell-problem path, and from an independent numpy
first-Piola residual solved by scipy on tiny meshes."""
import numpy as np
import pytest
from scipy.optimize import root

import oracle
from tests import fe_ref

LAME = oracle.two_phase_lame(10.0)
SVK, LIN = oracle.LAW_SVK, oracle.LAW_LINEAR


def rand_F(rng, d, amp=0.25):
    while True:
        F = np.eye(d) + rng.uniform(-amp, amp, (d, d))
        if np.linalg.det(F) > 0.4:
            return F


def sqrt_spd(C):
    ev, V = np.linalg.eigh(C)
    return V @ np.diag(np.sqrt(ev)) @ V.T


def rot(d, rng):
    if d == 2:
        t = rng.uniform(0, 2 * np.pi)
        return np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def lin_tensor(d, lam, mu):
    I = np.eye(d)
    return lam * np.einsum("IJ,KL->IJKL", I, I) + mu * (np.einsum("IK,JL->IJKL", I, I) + np.einsum("IL,JK->IJKL", I, I))


# ---------------------------------------------------------------- material level
@pytest.mark.parametrize("which", [SVK, LIN])
@pytest.mark.parametrize("d", [2, 3])
def test_reference_state_is_linear_elasticity(which, d):
    lam, mu = 1.3, 0.7
    st, S, Cm, psi = oracle.law_sc(which, d, lam, mu, np.eye(d))
    assert st == 0 and abs(psi) < 1e-15 and np.abs(S).max() < 1e-15
    assert np.abs(Cm - lin_tensor(d, lam, mu)).max() < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_svk_stress_and_tangent_are_derivatives_of_psi(d):
    """S = 2 dpsi/dC and C = 4 d^2psi/dCdC by central differences (through F = U)."""
    rng = np.random.default_rng(11)
    lam, mu = 0.8, 0.45
    for _ in range(5):
        F = rand_F(rng, d)
        Cc = F.T @ F
        st, S, Cm, _ = oracle.law_sc(SVK, d, lam, mu, F)
        assert st == 0
        h = 1e-6
        for I in range(d):
            for J in range(I, d):
                E = np.zeros((d, d)); E[I, J] = E[J, I] = 1.0
                dpsi = (oracle.law_sc(SVK, d, lam, mu, sqrt_spd(Cc + h * E))[3] -
                        oracle.law_sc(SVK, d, lam, mu, sqrt_spd(Cc - h * E))[3]) / (2 * h)
                assert dpsi == pytest.approx(0.5 * np.sum(S * E), rel=1e-7, abs=1e-9)
                Sp = oracle.law_sc(SVK, d, lam, mu, sqrt_spd(Cc + 1e-4 * E))[1]
                Sm = oracle.law_sc(SVK, d, lam, mu, sqrt_spd(Cc - 1e-4 * E))[1]
                pred = 0.5 * np.einsum("IJKL,KL->IJ", Cm, E)
                assert np.abs((Sp - Sm) / 2e-4 - pred).max() < 1e-7 * max(1.0, np.abs(pred).max())


@pytest.mark.parametrize("d", [2, 3])
def test_svk_energy_is_quadratic_in_green_strain_and_objective(d):
    """psi(E) homogeneous of degree 2 in E = (C - 1)/2 (C = 1 + 2 s E along a ray),
    S of degree 1; frame invariance psi(QF) = psi(F), S(QF) = S(F)."""
    rng = np.random.default_rng(12)
    lam, mu = 1.1, 0.5
    for _ in range(5):
        F = rand_F(rng, d, 0.2)
        E = 0.5 * (F.T @ F - np.eye(d))
        _, S1, _, p1 = oracle.law_sc(SVK, d, lam, mu, sqrt_spd(np.eye(d) + 2 * E))
        _, S2, _, p2 = oracle.law_sc(SVK, d, lam, mu, sqrt_spd(np.eye(d) + 4 * E))
        assert p2 == pytest.approx(4 * p1, rel=1e-12)
        assert np.abs(S2 - 2 * S1).max() < 1e-12 * np.abs(S1).max()
        Q = rot(d, rng)
        _, Sq, _, pq = oracle.law_sc(SVK, d, lam, mu, Q @ F)
        _, S0, _, p0 = oracle.law_sc(SVK, d, lam, mu, F)
        assert pq == pytest.approx(p0, rel=1e-12) and np.abs(Sq - S0).max() < 1e-12


def test_svk_plane_strain_is_3d_law_with_unit_stretch():
    rng = np.random.default_rng(13)
    for _ in range(5):
        F2 = rand_F(rng, 2)
        F3 = np.eye(3); F3[:2, :2] = F2
        _, S2, C2, p2 = oracle.law_sc(SVK, 2, 1.1, 0.4, F2)
        _, S3, C3, p3 = oracle.law_sc(SVK, 3, 1.1, 0.4, F3)
        assert np.abs(S2 - S3[:2, :2]).max() < 1e-14 and np.abs(C2 - C3[:2, :2, :2, :2]).max() < 1e-14
        assert p2 == pytest.approx(p3, rel=1e-14, abs=1e-16)


@pytest.mark.parametrize("d", [2, 3])
def test_linear_law_is_linear_in_the_symmetric_gradient(d):
    """sigma depends on sym(H) only (H = F - 1) and linearly; sigma = dpsi/deps."""
    rng = np.random.default_rng(14)
    lam, mu = 0.9, 0.6
    for _ in range(5):
        H = rng.uniform(-0.1, 0.1, (d, d))
        W = rng.uniform(-0.1, 0.1, (d, d)); W = W - W.T
        _, s1, Cm, p1 = oracle.law_sc(LIN, d, lam, mu, np.eye(d) + H)
        _, s2, _, _ = oracle.law_sc(LIN, d, lam, mu, np.eye(d) + 2 * H)
        _, s3, _, _ = oracle.law_sc(LIN, d, lam, mu, np.eye(d) + H + W)
        assert np.abs(s2 - 2 * s1).max() < 1e-14 and np.abs(s3 - s1).max() < 1e-14
        eps = 0.5 * (H + H.T)
        for I in range(d):
            for J in range(I, d):
                D = np.zeros((d, d)); D[I, J] = D[J, I] = 1.0
                dp = (oracle.law_sc(LIN, d, lam, mu, np.eye(d) + eps + 1e-6 * D)[3] -
                      oracle.law_sc(LIN, d, lam, mu, np.eye(d) + eps - 1e-6 * D)[3]) / 2e-6
                assert dp == pytest.approx(np.sum(s1 * D), rel=1e-7, abs=1e-12)


# ---------------------------------------------------------------- RVE level
def _numpy_svk_P(F, lam, mu):
    """First Piola stress of the St. Venant-Kirchhoff law, written here in numpy."""
    d = F.shape[-1]
    E = 0.5 * (np.swapaxes(F, -1, -2) @ F - np.eye(d))
    trE = np.trace(E, axis1=-2, axis2=-1)
    S = lam[..., None, None] * trE[..., None, None] * np.eye(d) + 2 * mu[..., None, None] * E
    return F @ S


def _numpy_residual(m, Fbar, w, lam_e, mu_e, which):
    F = m.grads(Fbar, w)
    lam = np.broadcast_to(lam_e[:, None], F.shape[:2])
    mu = np.broadcast_to(mu_e[:, None], F.shape[:2])
    if which == SVK:
        P = _numpy_svk_P(F, lam, mu)
    else:
        eps = 0.5 * (F + np.swapaxes(F, -1, -2)) - np.eye(m.d)
        P = lam[..., None, None] * np.trace(eps, axis1=-2, axis2=-1)[..., None, None] * np.eye(m.d) + \
            2 * mu[..., None, None] * eps
    fe = np.einsum("epiJ,paJ->eai", P, m.dN) * m.wJ
    R = np.zeros((m.nn, m.d))
    np.add.at(R, m.elems, fe)
    return R.reshape(-1), P.sum(axis=(0, 1)) * m.wJ


@pytest.mark.parametrize("which", [SVK, LIN])
@pytest.mark.parametrize("d,n", [(2, 2), (2, 3), (3, 2)])
def test_brute_force_tiny_meshes(which, d, n):
    """R(w) = 0 of an independent numpy residual solved by scipy: same <P>; A by
    central differences of that brute-force <P>."""
    rng = np.random.default_rng(20 + n + 10 * d + which)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    lam_e, mu_e = LAME[ph, 0], LAME[ph, 1]
    m = fe_ref.PeriodicMesh(d, n)

    def bf(Fbar):
        def fun(x):
            return _numpy_residual(m, Fbar, np.concatenate([np.zeros(d), x]), lam_e, mu_e, which)[0][d:]
        sol = root(fun, np.zeros(d * (n ** d - 1)), method="hybr", tol=1e-14)
        return _numpy_residual(m, Fbar, np.concatenate([np.zeros(d), sol.x]), lam_e, mu_e, which)[1]

    Fbar = rand_F(rng, d, 0.15)
    with oracle.law(which):
        r = oracle.rve_solve(d, n, ph, LAME, Fbar)
    assert r["status"] == 0
    P_bf = bf(Fbar)
    assert np.linalg.norm(r["P"] - P_bf) <= 1e-9 * np.linalg.norm(P_bf)
    h = 1e-5
    A_fd = np.zeros((d * d, d * d))
    for q in range(d * d):
        dF = np.zeros(d * d); dF[q] = h
        A_fd[:, q] = (bf(Fbar + dF.reshape(d, d)) - bf(Fbar - dF.reshape(d, d))).reshape(-1) / (2 * h)
    assert np.linalg.norm(r["A"] - A_fd) <= 1e-6 * np.linalg.norm(A_fd)


@pytest.mark.parametrize("d,n", [(2, 6), (3, 3)])
def test_svk_homogeneous_rve_objectivity_and_tangent(d, n):
    rng = np.random.default_rng(30 + d)
    one = np.zeros(n ** d, np.uint8)
    with oracle.law(SVK):
        F = rand_F(rng, d, 0.15)
        r = oracle.rve_solve(d, n, one, LAME, F)
        assert r["status"] == 0 and r["iters"] == 0
        lam, mu = LAME[0]
        assert np.abs(r["P"] - _numpy_svk_P(F, np.array(lam), np.array(mu))).max() < 1e-13
        ph = oracle.phase_by_centroid(d, n, 0.3)
        a = oracle.rve_solve(d, n, ph, LAME, F)
        Q = rot(d, rng)
        b = oracle.rve_solve(d, n, ph, LAME, Q @ F)
        assert np.linalg.norm(b["P"] - Q @ a["P"]) <= 1e-10 * np.linalg.norm(a["P"])
        A4 = a["A"].reshape(d, d, d, d)
        Aq = np.einsum("ia,kb,aJbL->iJkL", Q, Q, A4).reshape(d * d, d * d)
        assert np.linalg.norm(b["A"] - Aq) <= 1e-10 * np.linalg.norm(Aq)
        # A = dP/dF by central differences, and major symmetry
        h = 1e-5
        A_fd = np.zeros((d * d, d * d))
        for q in range(d * d):
            dF = np.zeros(d * d); dF[q] = h
            pp = oracle.rve_solve(d, n, ph, LAME, F + dF.reshape(d, d), rtol=1e-13)["P"]
            pm = oracle.rve_solve(d, n, ph, LAME, F - dF.reshape(d, d), rtol=1e-13)["P"]
            A_fd[:, q] = (pp - pm).reshape(-1) / (2 * h)
        assert np.linalg.norm(a["A"] - A_fd) <= 1e-6 * np.linalg.norm(A_fd)
        assert np.abs(a["A"] - a["A"].T).max() <= 1e-12 * np.abs(a["A"]).max()


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_linear_rve_is_the_linear_cell_problem(d, n):
    """Fully linear case: the tangent is the small-strain homogenized tensor of the
    separate linear cell-problem path at any Fbar; <sigma> = C^h : H exactly; one
    Newton update."""
    rng = np.random.default_rng(40 + d)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    st, Ch = oracle.linear_homogenized(d, n, ph, LAME)
    assert st == 0
    with oracle.law(LIN):
        for _ in range(3):
            F = rand_F(rng, d, 0.15)
            r = oracle.rve_solve(d, n, ph, LAME, F)
            assert r["status"] == 0 and r["iters"] == 1
            assert np.linalg.norm(r["A"] - Ch) <= 1e-12 * np.linalg.norm(Ch)
            P_lin = (Ch @ (F - np.eye(d)).reshape(-1)).reshape(d, d)
            assert np.linalg.norm(r["P"] - P_lin) <= 1e-11 * np.linalg.norm(P_lin)
            assert np.abs(r["P"] - r["P"].T).max() <= 1e-12 * np.abs(r["P"]).max()


def test_law_switch_is_restored():
    assert oracle.get_law() == oracle.LAW_NEOHOOKE
    with oracle.law(SVK):
        assert oracle.get_law() == SVK
    assert oracle.get_law() == oracle.LAW_NEOHOOKE
