"""Independent numpy reference pieces used to pin the oracle (tests only).

Written separately from ``oracle/`` in the first-Piola form rather than the
oracle's S/C/B-matrix form:

* neo-Hookean energy of the paper's Sec. 6 (plane strain in 2D: tr C gains the
  out-of-plane 1), with P = dpsi/dF and A = d^2 psi / dF dF derived by hand:
      P = mu (F - F^-T) + lambda/2 (J^2 - 1) F^-T
      A_iJkL = mu d_ik d_JL + (mu - lambda/2 (J^2-1)) Fi_Jk Fi_Li + lambda J^2 Fi_Ji Fi_Lk
  where Fi = F^-1;
* a vectorised periodic Q1/hex8 mesh with the energy Pi(w) = sum psi w|J| and
  its gradient R(w) = sum P : grad N w|J|, used for brute-force solves on tiny
  meshes and for Hill-Mandel checks.
"""
import itertools

import numpy as np


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def psi(F, lam, mu):
    d = F.shape[-1]
    J = np.linalg.det(F)
    trC = np.sum(F * F, axis=(-2, -1)) + (1.0 if d == 2 else 0.0)
    return lam / 4 * (J ** 2 - 1) - (lam / 2 + mu) * np.log(J) + mu / 2 * (trC - 3)


def P_closed(F, lam, mu):
    J = np.linalg.det(F)
    FiT = np.swapaxes(np.linalg.inv(F), -1, -2)
    lam = np.broadcast_to(lam, J.shape)[..., None, None]
    mu = np.broadcast_to(mu, J.shape)[..., None, None]
    return mu * (F - FiT) + (lam / 2 * (J ** 2 - 1)[..., None, None]) * FiT


def A_closed(F, lam, mu):
    d = F.shape[-1]
    J = np.linalg.det(F)
    Fi = np.linalg.inv(F)
    I = np.eye(d)
    A = mu * np.einsum("ik,JL->iJkL", I, I)
    A = A + (mu - lam / 2 * (J ** 2 - 1)) * np.einsum("Jk,Li->iJkL", Fi, Fi)
    A = A + lam * J ** 2 * np.einsum("Ji,Lk->iJkL", Fi, Fi)
    return A.reshape(d * d, d * d)


class PeriodicMesh:
    """n^d periodic grid on the unit cell; nodes/elements x-fastest."""

    def __init__(self, d, n):
        self.d, self.n = d, n
        self.nn = n ** d
        corners = list(itertools.product((0, 1), repeat=d))  # any fixed local order works here
        elems = []
        for c in itertools.product(range(n), repeat=d):
            idx = c[::-1]  # itertools varies the last entry fastest; make x fastest
            nodes = []
            for o in corners:
                nodes.append(sum(((idx[k] + o[k]) % n) * n ** k for k in range(d)))
            elems.append(nodes)
        self.elems = np.array(elems)  # [ne, 2^d]
        h = 1.0 / n
        g = 1 / np.sqrt(3)
        gps = list(itertools.product((-g, g), repeat=d))
        dN = np.zeros((len(gps), len(corners), d))
        for p, xi in enumerate(gps):
            for a, o in enumerate(corners):
                s = [1 if oo else -1 for oo in o]
                for k in range(d):
                    v = 1.0
                    for m in range(d):
                        v *= 0.5 * s[m] if m == k else 0.5 * (1 + s[m] * xi[m])
                    dN[p, a, k] = v * 2 / h
        self.dN = dN
        self.wJ = (h / 2) ** d

    def grads(self, Fbar, w):
        """F at every (element, gp): [ne, ngp, d, d]."""
        W = w.reshape(self.nn, self.d)[self.elems]  # [ne, nen, d]
        G = np.einsum("eai,paJ->epiJ", W, self.dN)
        return Fbar[None, None] + G

    def energy(self, Fbar, w, lam_e, mu_e):
        F = self.grads(Fbar, w)
        return float(np.sum(psi(F, lam_e[:, None], mu_e[:, None])) * self.wJ)

    def residual(self, Fbar, w, lam_e, mu_e):
        F = self.grads(Fbar, w)
        P = P_closed(F, lam_e[:, None], mu_e[:, None])
        fe = np.einsum("epiJ,paJ->eai", P, self.dN) * self.wJ
        R = np.zeros((self.nn, self.d))
        np.add.at(R, self.elems, fe)
        return R.reshape(-1)

    def average_P(self, Fbar, w, lam_e, mu_e):
        F = self.grads(Fbar, w)
        P = P_closed(F, lam_e[:, None], mu_e[:, None])
        return P.sum(axis=(0, 1)) * self.wJ


def brute_force_P(d, n, phase, lame_tab, Fbar, tol=1e-13):
    """Solve R(w) = 0 on a tiny mesh with scipy (node 0 pinned) and return <P>, w."""
    from scipy.optimize import root

    m = PeriodicMesh(d, n)
    lam_e = lame_tab[phase, 0]
    mu_e = lame_tab[phase, 1]

    def fun(x):
        w = np.concatenate([np.zeros(d), x])
        return m.residual(Fbar, w, lam_e, mu_e)[d:]

    x0 = np.zeros(d * (n ** d - 1))
    sol = root(fun, x0, method="hybr", tol=tol, options={"xtol": tol, "maxfev": 20000})
    w = np.concatenate([np.zeros(d), sol.x])
    return m.average_P(Fbar, w, lam_e, mu_e), w, float(np.linalg.norm(fun(sol.x)))
