"""The algebra behind the condensation from the last Newton factorization (CPU).

The macro tangent is <A> - Y^T K^-1 Y with K the free-dof tangent and Y the
coupling columns (Sec. 3.3).  With any approximation X of X* = K^-1 Y, the
stationary form <A> - Y^T X - X^T (Y - K X) equals the exact tangent plus
(X - X*)^T K (X - X*): the error is second order in X's.  Assembled from
element blocks with X zero on the pinned dofs, Y^T X + X^T Y - X^T K X is the
sum over elements of X_e^T y_e + y_e^T X_e - X_e^T k_e X_e.  Both identities are
checked on random element data; the GPU kernels' use of them is checked against
the oracle in test_gpu_parity.py.
"""
import numpy as np


def assembled(rng, n_nodes=30, n_el=40, nen=4, d=2, nc=4, pinned=(0,)):
    ndof = n_nodes * d
    conn = np.stack([rng.choice(n_nodes, nen, replace=False) for _ in range(n_el)])
    ke, ye = [], []
    K = np.zeros((ndof, ndof))
    Y = np.zeros((ndof, nc))
    for e in range(n_el):
        dofs = (conn[e][:, None] * d + np.arange(d)).ravel()
        B = rng.standard_normal((nen * d, nen * d))
        k = B @ B.T + 0.1 * np.eye(nen * d)
        y = rng.standard_normal((nen * d, nc))
        K[np.ix_(dofs, dofs)] += k
        Y[dofs] += y
        ke.append((dofs, k))
        ye.append(y)
    free = np.setdiff1d(np.arange(ndof), (np.asarray(pinned)[:, None] * d + np.arange(d)).ravel())
    return K, Y, free, ke, ye


def test_stationary_form_error_is_second_order():
    rng = np.random.default_rng(7)
    K, Y, free, _, _ = assembled(rng)
    Kf, Yf = K[np.ix_(free, free)], Y[free]
    Xs = np.linalg.solve(Kf, Yf)
    exact = -Yf.T @ Xs
    D = rng.standard_normal(Xs.shape)
    err_stat, err_plain = [], []
    for eps in (1e-2, 1e-4, 1e-6):
        E = eps * D
        X = Xs + E
        stat = -(Yf.T @ X + X.T @ (Yf - Kf @ X))
        np.testing.assert_allclose(stat - exact, E.T @ Kf @ E, rtol=1e-6, atol=1e-12 * np.abs(exact).max())
        err_stat.append(np.abs(stat - exact).max())
        err_plain.append(np.abs(-Yf.T @ X - exact).max())
    # a hundredfold smaller error in X: 1e4 times smaller in the stationary
    # form, only 1e2 times in the plain one
    for i in range(2):
        assert 0.5e4 < err_stat[i] / err_stat[i + 1] < 2e4
        assert 0.5e2 < err_plain[i] / err_plain[i + 1] < 2e2


def test_element_assembly_of_the_correction():
    rng = np.random.default_rng(11)
    K, Y, free, ke, ye = assembled(rng)
    X = np.zeros_like(Y)
    X[free] = rng.standard_normal((len(free), Y.shape[1]))  # zero on the pinned dofs
    Kf, Yf, Xf = K[np.ix_(free, free)], Y[free], X[free]
    node = Yf.T @ Xf + Xf.T @ Yf - Xf.T @ Kf @ Xf
    elem = np.zeros_like(node)
    for (dofs, k), y in zip(ke, ye):
        xe = X[dofs]
        elem += xe.T @ y + y.T @ xe - xe.T @ k @ xe
    np.testing.assert_allclose(elem, node, rtol=1e-12, atol=1e-12 * np.abs(node).max())
