"""Pins of the oracle's single micro update of the alternating two-level Newton
(Algorithm 2, Sec. 5.2): one Newton update of the stored fluctuation, then the
stress and stiffness transfer at the UPDATED micro state.

The expected values come from the independent first-Piola numpy code
(``tests/fe_ref.py``): the average stress <P> and the condensed tangent
<A> - Y^T K^-1 Y assembled from the hand-derived closed form of A = dP/dF, with
no call into the oracle's S/C/B-matrix arithmetic.
"""
import numpy as np
import pytest

import oracle
from tests import fe_ref

LAME = oracle.two_phase_lame(10.0)


def _fields(d, n, r):
    ph = oracle.phase_by_centroid(d, n, r)
    return ph, LAME[ph, 0], LAME[ph, 1]


def condensed_tangent(m, Fbar, w, lam_e, mu_e):
    """<A> - Y_f^T K_ff^-1 Y_f at an arbitrary (not necessarily converged)
    fluctuation w, node 0 pinned: the transfer of the unit macro-gradient states
    (eqs. k-mac-element-5..7) written with A = dP/dF."""
    d = m.d
    F = m.grads(Fbar, w)                                           # [ne, ngp, d, d]
    A = np.array([[fe_ref.A_closed(F[e, p], lam_e[e], mu_e[e]).reshape(d, d, d, d) for p in range(F.shape[1])]
                  for e in range(F.shape[0])])
    Aavg = A.sum(axis=(0, 1)).reshape(d * d, d * d) * m.wJ
    nn = m.nn
    Y = np.zeros((nn, d, d, d))
    K = np.zeros((nn, d, nn, d))
    ye = np.einsum("paJ,epiJkL->eaikL", m.dN, A) * m.wJ             # [ne, nen, d, d, d]
    ke = np.einsum("paJ,epiJkL,pbL->eaibk", m.dN, A, m.dN) * m.wJ  # [ne, nen, d, nen, d]
    for e, nodes in enumerate(m.elems):
        for a, na in enumerate(nodes):
            Y[na] += ye[e, a]
            for b, nb in enumerate(nodes):
                K[na, :, nb, :] += ke[e, a, :, b, :]
    Yf = Y.reshape(nn * d, d * d)[d:]
    Kf = K.reshape(nn * d, nn * d)[d:, d:]
    return Aavg - Yf.T @ np.linalg.solve(Kf, Yf)


@pytest.mark.parametrize("d,n,amp,seed", [(2, 4, 0.15, 1), (2, 6, 0.2, 2), (3, 3, 0.1, 3)])
def test_one_step_transfers_at_updated_state(d, n, amp, seed):
    """P and A returned by the single micro update are the averages and the
    condensed tangent at the state AFTER the update (D_{K,1}), not at the
    stored state it started from (D_{K,0})."""
    rng = np.random.default_rng(seed)
    Fbar = np.eye(d) + rng.uniform(-amp, amp, (d, d))
    ph, lam_e, mu_e = _fields(d, n, 0.3)
    m = fe_ref.PeriodicMesh(d, n)
    w0 = np.zeros(d * n ** d)
    r = oracle.rve_one_step(d, n, ph, LAME, Fbar, w0)
    assert r["status"] == 0
    w1 = r["w"]
    assert np.linalg.norm(w1) > 1e-3  # the update moved the state
    assert np.abs(w1[:d]).max() == 0.0  # node 0 stays pinned
    # stress at the updated state
    P1 = m.average_P(Fbar, w1, lam_e, mu_e)
    P0 = m.average_P(Fbar, w0, lam_e, mu_e)
    assert np.linalg.norm(r["P"] - P1) <= 1e-12 * np.linalg.norm(P1)
    assert np.linalg.norm(P1 - P0) > 1e3 * 1e-12 * np.linalg.norm(P1)
    # tangent at the updated state
    A1 = condensed_tangent(m, Fbar, w1, lam_e, mu_e)
    A0 = condensed_tangent(m, Fbar, w0, lam_e, mu_e)
    assert np.linalg.norm(r["A"] - A1) <= 1e-11 * np.linalg.norm(A1)
    assert np.linalg.norm(A1 - A0) > 1e3 * 1e-11 * np.linalg.norm(A1)
    # the reported norm is the free residual before the update
    R0 = m.residual(Fbar, w0, lam_e, mu_e)[d:]
    assert r["rnorm"] == pytest.approx(np.linalg.norm(R0), rel=1e-12)


def test_one_step_is_a_newton_update():
    """Repeated single updates are Newton's method: the free residual (computed
    by the independent code) contracts quadratically, ||R_{k+1}|| <= C ||R_k||^2,
    and the converged state's outputs are the full solve's."""
    d, n = 2, 8
    Fbar = np.array([[1.12, 0.07], [-0.05, 0.93]])
    ph, lam_e, mu_e = _fields(d, n, 0.25)
    m = fe_ref.PeriodicMesh(d, n)
    w = np.zeros(d * n * n)
    res = [np.linalg.norm(m.residual(Fbar, w, lam_e, mu_e)[d:])]
    for _ in range(4):
        r = oracle.rve_one_step(d, n, ph, LAME, Fbar, w)
        assert r["status"] == 0
        assert r["rnorm"] == pytest.approx(res[-1], rel=1e-9, abs=1e-15)
        w = r["w"]
        res.append(np.linalg.norm(m.residual(Fbar, w, lam_e, mu_e)[d:]))
    assert res[1] < 0.2 * res[0]
    for k in (2, 3):
        assert res[k] <= 10.0 * res[k - 1] ** 2 / res[0]
    assert res[4] < 1e-13
    full = oracle.rve_solve(d, n, ph, LAME, Fbar)
    assert np.linalg.norm(r["P"] - full["P"]) <= 1e-12 * np.linalg.norm(full["P"])
    assert np.linalg.norm(r["A"] - full["A"]) <= 1e-10 * np.linalg.norm(full["A"])


def test_one_step_at_equilibrium_keeps_the_state():
    """Below the absolute floor the update is skipped: the state is unchanged and
    the outputs are the converged ones."""
    d, n = 2, 6
    Fbar = np.array([[1.05, 0.02], [0.01, 0.97]])
    ph, lam_e, mu_e = _fields(d, n, 0.25)
    full = oracle.rve_solve(d, n, ph, LAME, Fbar, w=np.zeros(d * n * n), rtol=0.0)
    assert full["status"] == 0
    r = oracle.rve_one_step(d, n, ph, LAME, Fbar, full["w"])
    assert r["status"] == 0
    assert r["rnorm"] <= oracle.default_atol(LAME, n, d)
    assert np.array_equal(r["w"], full["w"])
    assert np.linalg.norm(r["P"] - full["P"]) <= 1e-14 * np.linalg.norm(full["P"])
