"""Pins of the oracle's element routines (Sec. 3.3) and its sparse solver."""
import numpy as np
import pytest

import oracle
from tests import fe_ref


def setup(d, n, seed=0, amp=0.05):
    rng = np.random.default_rng(seed)
    lame = oracle.two_phase_lame(10.0)
    phase = rng.integers(0, 2, n ** d).astype(np.uint8)
    Fbar = np.eye(d) + rng.uniform(-0.1, 0.1, (d, d))
    w = rng.uniform(-amp, amp, d * n ** d) / n
    return lame, phase, Fbar, w


@pytest.mark.parametrize("d", [2, 3])
def test_fe_is_gradient_of_element_energy(d):
    n = 3
    lame, phase, Fbar, w = setup(d, n)
    nen = 2 ** d
    for e in [0, 4, n ** d - 1]:
        st, fe, ke, en = oracle.element(d, n, phase, lame, e, Fbar, w)
        assert st == 0
        # nodes of element e: perturb the global dofs of that element's nodes
        c = [(e // n ** k) % n for k in range(d)]
        offs = [(0, 0), (1, 0), (1, 1), (0, 1)]
        if d == 3:
            offs = [o + (0,) for o in offs] + [o + (1,) for o in offs]
        nodes = [sum(((c[k] + o[k]) % n) * n ** k for k in range(d)) for o in offs]
        h = 1e-6
        for a in range(nen):
            for i in range(d):
                wp = w.copy(); wp[nodes[a] * d + i] += h
                wm = w.copy(); wm[nodes[a] * d + i] -= h
                ep = oracle.element(d, n, phase, lame, e, Fbar, wp)[3]
                em = oracle.element(d, n, phase, lame, e, Fbar, wm)[3]
                assert (ep - em) / (2 * h) == pytest.approx(fe[a * d + i], rel=1e-6, abs=1e-9)
                fp = oracle.element(d, n, phase, lame, e, Fbar, wp)[1]
                fm = oracle.element(d, n, phase, lame, e, Fbar, wm)[1]
                col = (fp - fm) / (2 * h)
                assert np.abs(col - ke[:, a * d + i]).max() < 1e-6 * max(1, np.abs(ke).max())
        assert np.abs(ke - ke.T).max() < 1e-12 * np.abs(ke).max()
        # rigid translation is a zero-energy mode of the tangent
        for i in range(d):
            t = np.zeros(nen * d); t[i::d] = 1.0
            assert np.abs(ke @ t).max() < 1e-12 * np.abs(ke).max()


@pytest.mark.parametrize("d", [2, 3])
def test_global_residual_matches_independent_first_piola_code(d):
    n = 3
    lame, phase, Fbar, w = setup(d, n, seed=5)
    st, R, en = oracle.residual(d, n, phase, lame, Fbar, w)
    m = fe_ref.PeriodicMesh(d, n)
    lam_e, mu_e = lame[phase, 0], lame[phase, 1]
    R2 = m.residual(Fbar, w, lam_e, mu_e)
    assert np.abs(R - R2).max() < 1e-13 * max(1, np.abs(R2).max())
    assert en == pytest.approx(m.energy(Fbar, w, lam_e, mu_e), rel=1e-13)


@pytest.mark.parametrize("d,n", [(2, 4), (3, 2)])
def test_sparse_ldlt_newton_step_matches_dense_solve(d, n):
    """The oracle's skyline LDL^T step equals numpy's dense solve, and the
    assembled tangent is the derivative of the independent residual."""
    lame, phase, Fbar, w = setup(d, n, seed=7)
    st, Rf, K, dw = oracle.debug_system(d, n, phase, lame, Fbar, w)
    assert st == 0
    assert np.abs(K - K.T).max() < 1e-13 * np.abs(K).max()
    ref = np.linalg.solve(K, -Rf)
    assert np.abs(dw - ref).max() < 1e-10 * np.abs(ref).max()
    m = fe_ref.PeriodicMesh(d, n)
    lam_e, mu_e = lame[phase, 0], lame[phase, 1]
    h = 1e-6
    for j in range(0, K.shape[0], max(1, K.shape[0] // 7)):
        wp = w.copy(); wp[d + j] += h
        wm = w.copy(); wm[d + j] -= h
        col = (m.residual(Fbar, wp, lam_e, mu_e) - m.residual(Fbar, wm, lam_e, mu_e))[d:] / (2 * h)
        assert np.abs(col - K[:, j]).max() < 1e-6 * np.abs(K).max()


def test_sparse_ldlt_matches_scipy_superlu():
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    d, n = 2, 8
    lame, phase, Fbar, w = setup(d, n, seed=9)
    st, Rf, K, dw = oracle.debug_system(d, n, phase, lame, Fbar, w)
    ref = spla.spsolve(sp.csc_matrix(K), -Rf)
    assert np.abs(dw - ref).max() < 1e-10 * np.abs(ref).max()
