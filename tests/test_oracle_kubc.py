"""Pins of the oracle's linear-displacement (KUBC) micro coupling: u = Fbar X on
the RVE boundary, one of the energetically consistent couplings of Sec. 3.2 and
the one of the paper's 3D example.  Expected values come from an independent
numpy residual on the true (n+1)^d node grid with the boundary nodes held at
w = 0 (no periodic numbering), solved by scipy on tiny meshes, and from what the
textbook coupling hierarchy fixes: the KUBC admissible fluctuations are a subset
of the periodic ones, so the KUBC energy and tangent bound the periodic ones from
above, and the Voigt average bounds them all."""
import itertools

import numpy as np
import pytest
from scipy.optimize import root

import oracle
from tests import fe_ref

LAME = oracle.two_phase_lame(10.0)
KUBC, PBC = oracle.BC_LINEAR, oracle.BC_PERIODIC


class OpenMesh:
    """n^d Q1/hex8 elements on (n+1)^d nodes, x-fastest, no periodic identification."""

    def __init__(self, d, n):
        self.d, self.n, self.N = d, n, n + 1
        corners = list(itertools.product((0, 1), repeat=d))
        elems = []
        for c in itertools.product(range(n), repeat=d):
            idx = c[::-1]
            elems.append([sum((idx[k] + o[k]) * self.N ** k for k in range(d)) for o in corners])
        self.elems = np.array(elems)
        self.nn = self.N ** d
        per = fe_ref.PeriodicMesh(d, n)   # same local corner order and Gauss rule
        self.dN, self.wJ = per.dN, per.wJ
        coords = np.array(list(itertools.product(range(self.N), repeat=d)))[:, ::-1]
        self.free = ~np.any((coords == 0) | (coords == n), axis=1)

    def fields(self, Fbar, x, lam_e, mu_e):
        w = np.zeros((self.nn, self.d))
        w[self.free] = x.reshape(-1, self.d)
        W = w[self.elems]
        F = Fbar[None, None] + np.einsum("eai,paJ->epiJ", W, self.dN)
        P = fe_ref.P_closed(F, lam_e[:, None], mu_e[:, None])
        fe = np.einsum("epiJ,paJ->eai", P, self.dN) * self.wJ
        R = np.zeros((self.nn, self.d))
        np.add.at(R, self.elems, fe)
        return R[self.free].reshape(-1), P.sum(axis=(0, 1)) * self.wJ


def brute_force_kubc(d, n, phase, Fbar):
    m = OpenMesh(d, n)
    lam_e, mu_e = LAME[phase, 0], LAME[phase, 1]
    nfree = int(m.free.sum()) * d
    sol = root(lambda x: m.fields(Fbar, x, lam_e, mu_e)[0], np.zeros(nfree), method="hybr", tol=1e-14)
    R, P = m.fields(Fbar, sol.x, lam_e, mu_e)
    assert np.linalg.norm(R) < 1e-11
    return P


def rand_F(rng, d, amp=0.15):
    while True:
        F = np.eye(d) + rng.uniform(-amp, amp, (d, d))
        if np.linalg.det(F) > 0.5:
            return F


@pytest.mark.parametrize("d,n", [(2, 3), (2, 4), (3, 3)])
def test_kubc_against_brute_force_on_the_open_grid(d, n):
    rng = np.random.default_rng(50 + 10 * d + n)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = rand_F(rng, d)
    with oracle.bc(KUBC):
        r = oracle.rve_solve(d, n, ph, LAME, F)
    assert r["status"] == 0
    P_bf = brute_force_kubc(d, n, ph, F)
    assert np.linalg.norm(r["P"] - P_bf) <= 1e-10 * np.linalg.norm(P_bf)
    h = 1e-5
    A_fd = np.zeros((d * d, d * d))
    for q in range(d * d):
        dF = np.zeros(d * d); dF[q] = h
        A_fd[:, q] = (brute_force_kubc(d, n, ph, F + dF.reshape(d, d)) -
                      brute_force_kubc(d, n, ph, F - dF.reshape(d, d))).reshape(-1) / (2 * h)
    assert np.linalg.norm(r["A"] - A_fd) <= 1e-6 * np.linalg.norm(A_fd)


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_kubc_homogeneous_rve_is_exact(d, n):
    F = rand_F(np.random.default_rng(60 + d), d)
    with oracle.bc(KUBC):
        r = oracle.rve_solve(d, n, np.zeros(n ** d, np.uint8), LAME, F)
    assert r["status"] == 0 and r["iters"] == 0
    lam, mu = LAME[0]
    assert np.abs(r["P"] - fe_ref.P_closed(F, lam, mu)).max() < 1e-13
    assert np.abs(r["A"] - fe_ref.A_closed(F, lam, mu)).max() < 1e-12


def _sym_strain_basis(d):
    out = []
    for I in range(d):
        for J in range(I, d):
            E = np.zeros((d, d)); E[I, J] = E[J, I] = 1.0
            out.append(E.reshape(-1))
    return np.array(out)


@pytest.mark.parametrize("d,n", [(2, 8), (2, 12), (3, 4)])
def test_coupling_hierarchy_at_small_strain(d, n):
    """Voigt >= KUBC >= periodic in the energy sense on symmetric strains (the
    admissible fluctuations shrink from periodic to KUBC to none)."""
    ph = oracle.phase_by_centroid(d, n, 0.3)
    I = np.eye(d)
    with oracle.bc(KUBC):
        Ak = oracle.rve_solve(d, n, ph, LAME, I)["A"]
    Ap = oracle.rve_solve(d, n, ph, LAME, I)["A"]
    lam_e, mu_e = LAME[ph, 0], LAME[ph, 1]
    Cv = np.mean([fe_ref.A_closed(I, l, m) for l, m in zip(lam_e, mu_e)], axis=0)
    B = _sym_strain_basis(d)
    for hi, lo in ((Cv, Ak), (Ak, Ap)):
        M = B @ (hi - lo) @ B.T
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 1e-10 * np.abs(B @ lo @ B.T).max()


@pytest.mark.parametrize("d,n", [(2, 8), (3, 4)])
def test_kubc_energy_and_averages(d, n):
    """Nonlinear: W_PBC(F) <= W_KUBC(F) <= <psi(F)>; Hill-Mandel and <F> = Fbar
    with the KUBC fluctuation; A = dP/dF by central differences."""
    rng = np.random.default_rng(70 + d)
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = rand_F(rng, d)
    m = fe_ref.PeriodicMesh(d, n)
    lam_e, mu_e = LAME[ph, 0], LAME[ph, 1]
    wp = oracle.rve_solve(d, n, ph, LAME, F, w=np.zeros(d * n ** d))["w"]
    with oracle.bc(KUBC):
        rk = oracle.rve_solve(d, n, ph, LAME, F, w=np.zeros(d * n ** d))
        assert rk["status"] == 0
        wk = rk["w"]
        # boundary (grid index 0) fluctuations vanish
        coords = np.array(list(itertools.product(range(n), repeat=d)))[:, ::-1]
        bnd = np.any(coords == 0, axis=1)
        assert np.abs(wk.reshape(-1, d)[bnd]).max() == 0.0
        Wp = m.energy(F, wp, lam_e, mu_e)
        Wk = m.energy(F, wk, lam_e, mu_e)
        W0 = m.energy(F, np.zeros_like(wk), lam_e, mu_e)
        assert Wp < Wk < W0
        Fq = m.grads(F, wk)
        Pq = fe_ref.P_closed(Fq, lam_e[:, None], mu_e[:, None])
        assert np.abs(Fq.mean(axis=(0, 1)) - F).max() < 1e-13
        hm = np.sum(Pq * Fq, axis=(2, 3)).sum() * m.wJ
        assert hm == pytest.approx(np.sum(rk["P"] * F), rel=1e-10)
        h = 1e-5
        A_fd = np.zeros((d * d, d * d))
        for q in range(d * d):
            dF = np.zeros(d * d); dF[q] = h
            pp = oracle.rve_solve(d, n, ph, LAME, F + dF.reshape(d, d), rtol=1e-13)["P"]
            pm = oracle.rve_solve(d, n, ph, LAME, F - dF.reshape(d, d), rtol=1e-13)["P"]
            A_fd[:, q] = (pp - pm).reshape(-1) / (2 * h)
        assert np.linalg.norm(rk["A"] - A_fd) <= 1e-6 * np.linalg.norm(A_fd)


def test_bc_switch_is_restored():
    assert oracle.get_bc() == PBC
    with oracle.bc(KUBC):
        assert oracle.get_bc() == KUBC
        assert oracle.n_free_nodes(2, 5) == 16
    assert oracle.get_bc() == PBC
