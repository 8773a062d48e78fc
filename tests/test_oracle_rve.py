"""Pins of the oracle's RVE solve against what the method and the mathematics fix.

Each test names the property it relies on; none of them re-calls the oracle's
own formulas to produce an expected value.
"""
import numpy as np
import pytest
from scipy.optimize import fsolve

import oracle
from tests import fe_ref

LAME = oracle.two_phase_lame(10.0)


def solve(d, n, phase, F, lame=LAME, **kw):
    r = oracle.rve_solve(d, n, phase, lame, F, **kw)
    assert r["status"] == 0, r
    return r


def rand_F(rng, d, amp):
    return np.eye(d) + rng.uniform(-amp, amp, (d, d))


def rot(d, rng):
    if d == 2:
        t = rng.uniform(0, 2 * np.pi)
        return np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    return Q * np.sign(np.linalg.det(Q))


def relerr(a, b, floor=1e-12):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), floor)


# ---------------------------------------------------------------- homogeneous RVE
@pytest.mark.parametrize("d,n", [(2, 4), (2, 8), (3, 3)])
def test_homogeneous_rve_reproduces_constitutive_law(d, n):
    """One phase: R(0) = 0 because constant P integrates to zero against the
    periodic grad N; FE-HMM then reduces to the constitutive law (e_mod = 0 for
    periodic coupling, Sec. 4)."""
    rng = np.random.default_rng(10 + d)
    lam, mu = LAME[0]
    ph = np.zeros(n ** d, np.uint8)
    for _ in range(3):
        F = rand_F(rng, d, 0.2)
        r = solve(d, n, ph, F)
        assert r["iters"] == 0
        assert relerr(r["P"], fe_ref.P_closed(F, lam, mu)) < 1e-13
        assert relerr(r["A"], fe_ref.A_closed(F, lam, mu)) < 1e-12


# ---------------------------------------------------------------- invariances
@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_objectivity(d, n):
    """psi depends on C only (eq. NH-free-energy): P(QF) = Q P(F) and
    A(QF)_iJkL = Q_ia Q_kb A(F)_aJbL for a rigid rotation Q."""
    rng = np.random.default_rng(20 + d)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = rand_F(rng, d, 0.15)
    Q = rot(d, rng)
    r1 = solve(d, n, ph, F)
    r2 = solve(d, n, ph, Q @ F)
    assert relerr(r2["P"], Q @ r1["P"]) < 1e-10
    A1 = r1["A"].reshape((d,) * 4)
    A2 = r2["A"].reshape((d,) * 4)
    assert relerr(A2, np.einsum("ia,kb,aJbL->iJkL", Q, Q, A1)) < 1e-9


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_hill_mandel_and_equilibrium(d, n):
    """At equilibrium (checked with an independent residual code): <F^eps> = Fbar
    and <P^eps : F^eps> = Pbar : Fbar (eqs. Hill-Mandel, Average-of-P-and-F), and
    Pbar Fbar^T is symmetric (balance of angular momentum on average)."""
    rng = np.random.default_rng(30 + d)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = rand_F(rng, d, 0.15)
    r = solve(d, n, ph, F, w=np.zeros(d * n ** d))
    w = r["w"]
    m = fe_ref.PeriodicMesh(d, n)
    lam_e, mu_e = LAME[ph, 0], LAME[ph, 1]
    R = m.residual(F, w, lam_e, mu_e)
    assert np.abs(R[d:]).max() < 1e-11
    Fe = m.grads(F, w)
    Pe = fe_ref.P_closed(Fe, lam_e[:, None], mu_e[:, None])
    assert np.abs(Fe.sum(axis=(0, 1)) * m.wJ - F).max() < 1e-14
    PF = np.sum(Pe * Fe) * m.wJ
    assert PF == pytest.approx(np.sum(r["P"] * F), rel=1e-11)
    assert relerr(Pe.sum(axis=(0, 1)) * m.wJ, r["P"]) < 1e-13
    S = r["P"] @ F.T
    assert np.abs(S - S.T).max() < 1e-11 * np.abs(S).max()


# ---------------------------------------------------------------- derivatives
@pytest.mark.parametrize("d,n", [(2, 8), (3, 3)])
def test_tangent_is_derivative_of_average_stress(d, n):
    """Abar = dPbar/dFbar (total derivative through w*) by central differences,
    and major symmetry of Abar (hyperelastic, eq. hyperelasticity-PF)."""
    rng = np.random.default_rng(40 + d)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = rand_F(rng, d, 0.15)
    r = solve(d, n, ph, F, rtol=1e-14)
    A = r["A"]
    h = 1e-5
    Afd = np.zeros_like(A)
    for c in range(d * d):
        E = np.zeros(d * d); E[c] = h
        Pp = solve(d, n, ph, F + E.reshape(d, d), rtol=1e-14)["P"].reshape(-1)
        Pm = solve(d, n, ph, F - E.reshape(d, d), rtol=1e-14)["P"].reshape(-1)
        Afd[:, c] = (Pp - Pm) / (2 * h)
    assert relerr(A, Afd) < 1e-7
    assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()


def test_average_stress_is_derivative_of_homogenized_energy():
    """Pbar = dWbar/dFbar with Wbar(Fbar) = Pi(w*(Fbar)) (minimum of the cell
    energy; the independent energy code evaluates Pi)."""
    d, n = 2, 8
    rng = np.random.default_rng(50)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = rand_F(rng, d, 0.15)
    m = fe_ref.PeriodicMesh(d, n)
    lam_e, mu_e = LAME[ph, 0], LAME[ph, 1]

    def W(Fq):
        r = solve(d, n, ph, Fq, w=np.zeros(d * n * n), rtol=1e-14)
        return m.energy(Fq, r["w"], lam_e, mu_e)

    P = solve(d, n, ph, F)["P"]
    h = 1e-5
    for c in range(4):
        E = np.zeros(4); E[c] = h
        dW = (W(F + E.reshape(2, 2)) - W(F - E.reshape(2, 2))) / (2 * h)
        assert dW == pytest.approx(P.reshape(-1)[c], rel=1e-7, abs=1e-9)


# ---------------------------------------------------------------- small strain / bounds
@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_small_strain_limit_is_linear_fe_hmm(d, n):
    """At Fbar = I, S = 0 and the tangent is linear elasticity, so Abar(I) equals
    the linear FE-HMM homogenized tensor C^{0,h} (separate small-strain code), and
    Pbar(I + eps H) / eps -> C^{0,h} : sym H."""
    ph = oracle.phase_by_centroid(d, n, 0.3)
    st, Ch = oracle.linear_homogenized(d, n, ph, LAME)
    assert st == 0
    r = solve(d, n, ph, np.eye(d))
    assert r["iters"] == 0
    assert relerr(r["A"], Ch) < 1e-12
    H = np.random.default_rng(60).uniform(-1, 1, (d, d))
    lin = (Ch @ (0.5 * (H + H.T)).reshape(-1)).reshape(d, d)
    errs = []
    for eps in [1e-3, 1e-4]:
        P = solve(d, n, ph, np.eye(d) + eps * H, rtol=1e-13)["P"]
        errs.append(relerr(P / eps, lin))
    assert errs[1] < 1e-3 and errs[1] < 0.2 * errs[0]   # O(eps)


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_voigt_reuss_bounds(d, n):
    """Reuss <= C^h <= Voigt in the energy sense for symmetric strains (textbook
    Hill bounds), checked on the nonlinear code's Abar(I)."""
    ph = oracle.phase_by_centroid(d, n, 0.3)
    A = solve(d, n, ph, np.eye(d))["A"]
    f = ph.mean()
    I = np.eye(d)

    def Clin(lam, mu):
        return (lam * np.einsum("ij,kl->ijkl", I, I) +
                mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I))).reshape(d * d, d * d)

    C0, C1 = Clin(*LAME[0]), Clin(*LAME[1])
    Voigt = (1 - f) * C0 + f * C1
    # Reuss via compliance on the symmetric subspace
    Psym = 0.5 * (np.eye(d * d) + np.einsum("ijkl->ijlk", np.eye(d * d).reshape((d,) * 4)).reshape(d * d, d * d))
    Reuss = np.linalg.pinv((1 - f) * np.linalg.pinv(C0 @ Psym) + f * np.linalg.pinv(C1 @ Psym))
    rng = np.random.default_rng(70)
    for _ in range(20):
        e = rng.normal(size=(d, d)); e = (0.5 * (e + e.T)).reshape(-1)
        assert e @ Reuss @ e <= e @ A @ e * (1 + 1e-12)
        assert e @ A @ e <= e @ Voigt @ e * (1 + 1e-12)


def test_nonlinear_energy_bound():
    """w = 0 is admissible, so Wbar(Fbar) = min Pi <= <psi(Fbar)>."""
    d, n = 2, 8
    ph = oracle.phase_by_centroid(d, n, 0.3)
    m = fe_ref.PeriodicMesh(d, n)
    lam_e, mu_e = LAME[ph, 0], LAME[ph, 1]
    rng = np.random.default_rng(80)
    for _ in range(3):
        F = rand_F(rng, d, 0.2)
        r = solve(d, n, ph, F, w=np.zeros(d * n * n))
        assert m.energy(F, r["w"], lam_e, mu_e) <= m.energy(F, np.zeros(d * n * n), lam_e, mu_e)


# ---------------------------------------------------------------- exact special case
def laminate_P(d, F, f1, lam1, mu1, lam0, mu0):
    """Rank-one laminate with interfaces normal to e1: F_a = F + a_a (x) e1,
    f1 a1 + f0 a0 = 0 and traction continuity P(F1) e1 = P(F0) e1."""
    def Fs(a1):
        a0 = -f1 * a1 / (1 - f1)
        F1 = F.copy(); F1[:, 0] += a1
        F0 = F.copy(); F0[:, 0] += a0
        return F1, F0

    def g(a1):
        F1, F0 = Fs(a1)
        return fe_ref.P_closed(F1, lam1, mu1)[:, 0] - fe_ref.P_closed(F0, lam0, mu0)[:, 0]

    a1 = fsolve(g, np.zeros(d), xtol=1e-15)
    F1, F0 = Fs(a1)
    assert np.abs(g(a1)).max() < 1e-13
    return f1 * fe_ref.P_closed(F1, lam1, mu1) + (1 - f1) * fe_ref.P_closed(F0, lam0, mu0)


@pytest.mark.parametrize("d,n,k", [(2, 8, 3), (3, 4, 1)])
def test_laminate_closed_form(d, n, k):
    """Stripes of phase 1 over element columns i < k: the piecewise-affine
    laminate field lies in the Q1/hex8 space, so Pbar is exact; Abar matches
    central differences of the closed-form laminate Pbar."""
    rng = np.random.default_rng(90 + d)
    idx = np.arange(n ** d) % n
    ph = (idx < k).astype(np.uint8)
    F = rand_F(rng, d, 0.15)
    f1 = k / n
    args = (f1, *LAME[1], *LAME[0])
    r = solve(d, n, ph, F, rtol=1e-14)
    assert relerr(r["P"], laminate_P(d, F, *args)) < 1e-12
    h = 1e-5
    Afd = np.zeros((d * d, d * d))
    for c in range(d * d):
        E = np.zeros(d * d); E[c] = h
        Afd[:, c] = (laminate_P(d, F + E.reshape(d, d), *args) -
                     laminate_P(d, F - E.reshape(d, d), *args)).reshape(-1) / (2 * h)
    assert relerr(r["A"], Afd) < 1e-7


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("d,n", [(2, 2), (2, 3), (3, 2)])
def test_brute_force_tiny_meshes(d, n):
    """Solve R(w) = 0 with scipy's hybrid Powell method on the independent numpy
    residual; Pbar must agree, and Abar must match differences of the brute-force
    Pbar."""
    rng = np.random.default_rng(100 + 10 * d + n)
    ph = rng.integers(0, 2, n ** d).astype(np.uint8)
    F = rand_F(rng, d, 0.15)
    Pb, wb, res = fe_ref.brute_force_P(d, n, ph, LAME, F)
    assert res < 1e-12
    r = solve(d, n, ph, F, rtol=1e-14)
    assert relerr(r["P"], Pb) < 1e-10
    h = 1e-5
    Afd = np.zeros((d * d, d * d))
    for c in range(d * d):
        E = np.zeros(d * d); E[c] = h
        Afd[:, c] = (fe_ref.brute_force_P(d, n, ph, LAME, F + E.reshape(d, d))[0] -
                     fe_ref.brute_force_P(d, n, ph, LAME, F - E.reshape(d, d))[0]).reshape(-1) / (2 * h)
    assert relerr(r["A"], Afd) < 1e-6


# ---------------------------------------------------------------- Newton
def test_newton_converges_quadratically():
    d, n = 2, 16
    ph = oracle.phase_by_centroid(d, n, 0.25)
    F = np.array([[1.15, 0.1], [-0.05, 0.9]])
    r = solve(d, n, ph, F, rtol=1e-14)
    h = r["res_hist"]
    assert len(h) >= 3
    # once in the asymptotic regime the residual roughly squares (tail ratio)
    k = len(h) - 2
    assert h[k] / h[0] < 1e-4
    assert h[k] <= 10.0 * h[k - 1] ** 2 / h[0]


def test_warm_start_from_converged_state_needs_no_iteration():
    d, n = 2, 8
    ph = oracle.phase_by_centroid(d, n, 0.25)
    F = np.array([[1.1, 0.05], [0.0, 0.97]])
    r1 = solve(d, n, ph, F, w=np.zeros(d * n * n), rtol=1e-14)
    r2 = oracle.rve_solve(d, n, ph, LAME, F, w=r1["w"], rtol=1e-10, atol=1e-13)
    assert r2["status"] == 0 and r2["iters"] == 0
    assert relerr(r2["P"], r1["P"]) < 1e-13


def test_failure_statuses():
    d, n = 2, 4
    ph = oracle.phase_by_centroid(d, n, 0.25)
    r = oracle.rve_solve(d, n, ph, LAME, np.array([[1.0, 0.0], [0.0, -1.0]]))
    assert r["status"] == oracle.DETF and np.isnan(r["P"]).all() and np.isnan(r["A"]).all()
    r = oracle.rve_solve(d, n, ph, LAME, np.array([[np.nan, 0.0], [0.0, 1.0]]))
    assert r["status"] == oracle.NONFINITE
    r = oracle.rve_solve(d, n, ph, LAME, np.array([[1.2, 0.1], [0.0, 0.9]]), max_iter=1)
    assert r["status"] == oracle.NOCONV and np.isnan(r["P"]).all()


def test_batch_equals_single():
    d, n, B = 2, 8, 6
    rng = np.random.default_rng(5)
    F = np.stack([rand_F(rng, d, 0.15) for _ in range(B)])
    phases = np.stack([oracle.phase_by_centroid(d, n, r) for r in rng.uniform(0.15, 0.35, B)])
    out = oracle.rve_solve_batch(d, n, phases, LAME, F, nthreads=2)
    for b in range(B):
        r = solve(d, n, phases[b], F[b])
        assert np.array_equal(out["P"][b], r["P"]) and np.array_equal(out["A"][b], r["A"])
        assert out["iters"][b] == r["iters"]


def test_infeasible_warm_start_restarts_from_zero():
    """A stored fluctuation that folds an element under the new Fbar is
    discarded: the solve equals the cold start (the fluctuation field the
    two-scale schemes carry between iterations is only a starting guess)."""
    d, n = 2, 6
    lame = oracle.two_phase_lame(10.0)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = np.array([[1.1, 0.05], [-0.03, 0.95]])
    w_bad = np.zeros(d * n ** d)
    w_bad[2 * 7] = 0.5  # node (1, 1) pushed past its right neighbours
    assert oracle.element(d, n, ph, lame, 1 + n * 1, F, w_bad)[0] == oracle.DETF
    cold = oracle.rve_solve(d, n, ph, lame, F)
    warm = oracle.rve_solve(d, n, ph, lame, F, w=w_bad)
    assert cold["status"] == warm["status"] == oracle.OK
    assert warm["iters"] == cold["iters"]
    np.testing.assert_array_equal(warm["P"], cold["P"])
