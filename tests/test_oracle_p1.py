"""Pins of the oracle's P1 micro elements (the paper's linear simplices, Sec. 3.1):
each grid cell split into d! simplices along its (0..0)-(1..1) diagonal.  The
expected values come from an independent numpy P1 mesh that builds every
simplex from vertex coordinates and inverts its edge matrix for the gradients
(no barycentric closed form), solved by scipy on tiny meshes; from the patch
test (affine fields are exact, so a one-phase RVE is the constitutive law); and
from the rank-one laminate, whose piecewise-affine field P1 represents exactly."""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import root

import oracle
from tests import fe_ref
from tests.test_oracle_rve import laminate_P

LAME = oracle.two_phase_lame(10.0)
P1 = oracle.ELEM_P1


class PeriodicSimplexMesh:
    def __init__(self, d, n):
        self.d, self.n, self.nn = d, n, n ** d
        h = 1.0 / n
        simp, grads, vols, cell = [], [], [], []
        for c in itertools.product(range(n), repeat=d):
            idx = c[::-1]
            for perm in itertools.permutations(range(d)):
                verts = [np.zeros(d, int)]
                for k in perm:
                    v = verts[-1].copy(); v[k] += 1
                    verts.append(v)
                X = np.array([(np.array(idx) + v) * h for v in verts])
                E = (X[1:] - X[0]).T
                Ginv = np.linalg.inv(E)            # rows: grad of barycentric coords 1..d
                G = np.vstack([-Ginv.sum(axis=0), Ginv])
                nodes = [sum(((idx[k] + v[k]) % n) * n ** k for k in range(d)) for v in verts]
                simp.append(nodes); grads.append(G); vols.append(abs(np.linalg.det(E)) / math.factorial(d))
                cell.append(sum(idx[k] * n ** k for k in range(d)))
        self.simp, self.G, self.vol, self.cell = np.array(simp), np.array(grads), np.array(vols), np.array(cell)

    def fields(self, Fbar, w, lam_c, mu_c):
        W = w.reshape(self.nn, self.d)[self.simp]                 # [ns, d+1, d]
        F = Fbar[None] + np.einsum("sai,saJ->siJ", W, self.G)
        lam, mu = lam_c[self.cell], mu_c[self.cell]
        P = np.array([fe_ref.P_closed(F[s], lam[s], mu[s]) for s in range(len(F))])
        fe = np.einsum("siJ,saJ->sai", P, self.G) * self.vol[:, None, None]
        R = np.zeros((self.nn, self.d))
        np.add.at(R, self.simp, fe)
        return R.reshape(-1), (P * self.vol[:, None, None]).sum(axis=0)


def brute_force_p1(d, n, phase, F):
    m = PeriodicSimplexMesh(d, n)
    lam_c, mu_c = LAME[phase, 0], LAME[phase, 1]

    def fun(x):
        return m.fields(F, np.concatenate([np.zeros(d), x]), lam_c, mu_c)[0][d:]

    sol = root(fun, np.zeros(d * (n ** d - 1)), method="hybr", tol=1e-14)
    R, P = m.fields(F, np.concatenate([np.zeros(d), sol.x]), lam_c, mu_c)
    assert np.linalg.norm(R[d:]) < 1e-11
    return P


def rand_F(rng, d, amp=0.15):
    while True:
        F = np.eye(d) + rng.uniform(-amp, amp, (d, d))
        if np.linalg.det(F) > 0.5:
            return F


@pytest.mark.parametrize("d,n", [(2, 2), (2, 3), (2, 4), (3, 2)])
def test_p1_against_brute_force(d, n):
    rng = np.random.default_rng(110 + 10 * d + n)
    ph = rng.integers(0, 2, n ** d).astype(np.uint8)
    F = rand_F(rng, d)
    with oracle.element_kind(P1):
        r = oracle.rve_solve(d, n, ph, LAME, F, rtol=1e-14)
    assert r["status"] == 0
    P_bf = brute_force_p1(d, n, ph, F)
    assert np.linalg.norm(r["P"] - P_bf) <= 1e-10 * np.linalg.norm(P_bf)
    h = 1e-5
    A_fd = np.zeros((d * d, d * d))
    for q in range(d * d):
        dF = np.zeros(d * d); dF[q] = h
        A_fd[:, q] = (brute_force_p1(d, n, ph, F + dF.reshape(d, d)) -
                      brute_force_p1(d, n, ph, F - dF.reshape(d, d))).reshape(-1) / (2 * h)
    assert np.linalg.norm(r["A"] - A_fd) <= 1e-6 * np.linalg.norm(A_fd)


@pytest.mark.parametrize("d,n", [(2, 6), (3, 3)])
def test_p1_patch_test(d, n):
    F = rand_F(np.random.default_rng(120 + d), d)
    with oracle.element_kind(P1):
        r = oracle.rve_solve(d, n, np.zeros(n ** d, np.uint8), LAME, F)
    assert r["status"] == 0 and r["iters"] == 0
    lam, mu = LAME[0]
    assert np.abs(r["P"] - fe_ref.P_closed(F, lam, mu)).max() < 1e-13
    assert np.abs(r["A"] - fe_ref.A_closed(F, lam, mu)).max() < 1e-12


@pytest.mark.parametrize("d,n,k", [(2, 8, 3), (3, 4, 1)])
def test_p1_laminate_closed_form(d, n, k):
    rng = np.random.default_rng(130 + d)
    ph = ((np.arange(n ** d) % n) < k).astype(np.uint8)
    F = rand_F(rng, d)
    with oracle.element_kind(P1):
        r = oracle.rve_solve(d, n, ph, LAME, F, rtol=1e-14)
    assert r["status"] == 0
    Pl = laminate_P(d, F, k / n, *LAME[1], *LAME[0])
    assert np.linalg.norm(r["P"] - Pl) <= 1e-12 * np.linalg.norm(Pl)


def test_p1_differs_from_q1_and_switch_is_restored():
    d, n = 2, 8
    ph = oracle.phase_by_centroid(d, n, 0.3)
    F = np.array([[1.05, 0.04], [-0.02, 0.97]])
    q1 = oracle.rve_solve(d, n, ph, LAME, F)["P"]
    with oracle.element_kind(P1):
        p1 = oracle.rve_solve(d, n, ph, LAME, F)["P"]
    assert np.linalg.norm(p1 - q1) > 1e-6 * np.linalg.norm(q1)
    assert oracle.get_element() == oracle.ELEM_Q1
