"""Numpy model of the surrogate kernels' algorithm (test helper).

The HIP kernels differentiate the network forward-mode (a jet of value, three
first and six second input derivatives per neuron), assemble P and A from the
energy derivatives in c = (C11, C22, C12), take the loss derivative with
respect to the 9 network outputs by directional derivatives, and run the
reverse pass through the jets.  This module restates that algorithm in fp64
numpy so that

* a CPU test can pin it to the autograd oracle (same loss and gradient to
  rounding), independently of the GPU, and
* a GPU test can compare the kernels with this model run with bf16 rounding at
  exactly the kernel's rounding points (MFMA operands: W2, W3, the layer-1/2
  activation jets and the layer-2/3 pre-activation adjoints), which isolates
  implementation mistakes from the bf16 noise that the Taylor-free energy
  amplifies.
"""
import numpy as np

from oracle import surrogate as OS

PA = [0, 1, 2, 0, 0, 1]
PB = [0, 1, 2, 1, 2, 2]


def bf16(a):
    """Round to bfloat16 (nearest even) through float32."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _silu4(z):
    g = 1 / (1 + np.exp(-z))
    gp = g * (1 - g)
    gpp = gp * (1 - 2 * g)
    gppp = gp * (1 - 6 * g + 6 * g * g)
    return z * g, g + z * gp, 2 * gp + z * gpp, 3 * gpp + z * gppp


def jet_fwd(z):
    s0, s1, s2, _ = _silu4(z[0])
    h = np.zeros_like(z)
    h[0] = s0
    for k in range(3):
        h[1 + k] = s1 * z[1 + k]
    for m in range(6):
        h[4 + m] = s2 * z[1 + PA[m]] * z[1 + PB[m]] + s1 * z[4 + m]
    return h


def jet_bwd(z, dh):
    _, s1, s2, s3 = _silu4(z[0])
    dz = np.zeros_like(z)
    d0 = s1 * dh[0]
    dzt = [s1 * dh[1 + k] for k in range(3)]
    for k in range(3):
        d0 = d0 + s2 * z[1 + k] * dh[1 + k]
    for m in range(6):
        g = dh[4 + m]
        a, b = PA[m], PB[m]
        d0 = d0 + (s3 * z[1 + a] * z[1 + b] + s2 * z[4 + m]) * g
        dzt[a] = dzt[a] + s2 * z[1 + b] * g
        dzt[b] = dzt[b] + s2 * z[1 + a] * g
        dz[4 + m] = s1 * g
    dz[0] = d0
    for k in range(3):
        dz[1 + k] = dzt[k]
    return dz


def assemble(F, G, Hc):
    S = np.array([2 * G[0], G[2], G[2], 2 * G[1]])
    vI, fI = [0, 2, 2, 1], [2.0, 1.0, 1.0, 2.0]
    P = np.array([F[i * 2] * S[J] + F[i * 2 + 1] * S[2 + J] for i in range(2) for J in range(2)])
    A = np.zeros(16)
    for i in range(2):
        for J in range(2):
            for k in range(2):
                for L in range(2):
                    s = S[J * 2 + L] if i == k else 0.0
                    for Mi in range(2):
                        for Ni in range(2):
                            mj, nl = Mi * 2 + J, Ni * 2 + L
                            s += F[i * 2 + Mi] * F[k * 2 + Ni] * fI[mj] * fI[nl] * Hc[vI[mj] * 3 + vI[nl]]
                    A[(i * 2 + J) * 4 + k * 2 + L] = s
    return P, A


def loss_grad(theta, desc, F, Pt, At, wP=1.0, wA=0.1, rhoP=1e-3, rhoA=1e-3, round_bf16=False, round_fwd=None,
              tile=15):
    """Mean loss and gradient as the kernels compute them: tiles of `tile`
    points, each with its own copy of the origin (whose adjoint cancels the
    tile's first-order terms, so where the rounding happens matters).
    round_bf16 rounds the reverse pass's MFMA operands; round_fwd (default:
    round_bf16) those of the forward pass (off for the split hi/lo products)."""
    F = np.asarray(F, np.float64).reshape(-1, 4)
    n = len(F)
    step = tile if tile else n
    L, g = 0.0, np.zeros(OS.NPARAM)
    for a in range(0, n, step):
        b = min(n, a + step)
        La, ga = _tile(theta, desc, F[a:b], Pt[a:b], At[a:b], wP, wA, rhoP, rhoA, round_bf16, round_fwd)
        L += La
        g += ga
    return L / n, g / n


def _tile(theta, desc, F, Pt, At, wP, wA, rhoP, rhoA, round_bf16, round_fwd):
    rb = bf16 if round_bf16 else (lambda a: a)
    r = bf16 if (round_bf16 if round_fwd is None else round_fwd) else (lambda a: a)
    p = OS.unpack(np.asarray(theta, np.float64))
    W1, b1, W2, b2, W3, b3, w4 = [np.asarray(p[k]) for k in ["W1", "b1", "W2", "b2", "W3", "b3", "w4"]]
    M = np.asarray(desc["M"]).reshape(9)
    s, sw = desc["c_scale"], desc["w_scale"]
    F = np.asarray(F, np.float64).reshape(-1, 4)
    X = OS.scaled_inputs(desc, F)
    n = len(X)
    Xa = np.vstack([X, np.zeros((1, 3))])
    Z1 = np.zeros((10, 128, n + 1))
    Z1[0] = W1 @ Xa.T + b1[:, None]
    for k in range(3):
        Z1[1 + k] = W1[:, k][:, None]
    H1 = jet_fwd(Z1)
    Z2 = np.einsum("rn,qnp->qrp", r(W2), r(H1))
    Z2[0] += b2[:, None]
    H2 = jet_fwd(Z2)
    Z3 = np.einsum("rn,qnp->qrp", r(W3), r(H2))
    Z3[0] += b3[:, None]
    H3 = jet_fwd(Z3)
    Y = np.einsum("r,qrp->qp", w4, H3)[1:]
    y0 = Y[:, n]
    dY = np.zeros((9, n + 1))
    L = 0.0
    dd = [0.5, 0.5, 1.0]
    H0 = np.zeros(9)
    for m in range(6):
        H0[PA[m] * 3 + PB[m]] = H0[PB[m] * 3 + PA[m]] = y0[3 + m]
    for i in range(n):
        Fi, x, y = F[i], X[i], Y[:, i]
        C = [Fi[0] ** 2 + Fi[2] ** 2, Fi[1] ** 2 + Fi[3] ** 2, Fi[0] * Fi[1] + Fi[2] * Fi[3]]
        e = [0.5 * (C[0] - 1), 0.5 * (C[1] - 1), C[2]]
        G = [dd[k] * sum(M[k * 3 + b] * e[b] for b in range(3))
             + sw / s[k] * (y[k] - y0[k] - sum(H0[k * 3 + b] * x[b] for b in range(3))) for k in range(3)]
        Hc = np.array([dd[k // 3] * M[k] * dd[k % 3] for k in range(9)])
        for m in range(6):
            a, b = PA[m], PB[m]
            v = sw / (s[a] * s[b]) * (y[3 + m] - y0[3 + m])
            Hc[a * 3 + b] += v
            if a != b:
                Hc[b * 3 + a] += v
        P, A = assemble(Fi, G, Hc)
        kP = wP / (rhoP ** 2 + np.sum(Pt[i] ** 2))
        kA = wA / (rhoA ** 2 + np.sum(At[i] ** 2))
        L += kP * np.sum((P - Pt[i]) ** 2) + kA * np.sum((A - At[i]) ** 2)
        dy = np.zeros(9)
        for m in range(9):
            dG, dH = np.zeros(3), np.zeros(9)
            if m < 3:
                dG[m] = sw / s[m]
            else:
                a, b = PA[m - 3], PB[m - 3]
                dH[a * 3 + b] = dH[b * 3 + a] = sw / (s[a] * s[b])
            dP, dA = assemble(Fi, dG, dH)
            dy[m] = 2 * kP * np.sum((P - Pt[i]) * dP) + 2 * kA * np.sum((A - At[i]) * dA)
        dY[:, i] = dy
        for k in range(3):
            dY[k, n] -= dy[k]
        for mm in range(6):
            a, b = PA[mm], PB[mm]
            via = dy[a] * x[a] if a == b else dy[a] * x[b] + dy[b] * x[a]
            dY[3 + mm, n] -= dy[3 + mm] + via
    g = np.zeros(OS.NPARAM)
    dH3 = np.zeros((10, 128, n + 1))
    dH3[1:] = w4[None, :, None] * dY[:, None, :]
    g[OS.OFF_W4:] = np.einsum("qrp,qp->r", H3[1:], dY)
    dZ3 = jet_bwd(Z3, dH3)
    g[OS.OFF_B3:OS.OFF_W4] = dZ3[0].sum(1)
    g[OS.OFF_W3:OS.OFF_B3] = np.einsum("qrp,qnp->rn", rb(dZ3), rb(H2)).reshape(-1)
    dZ2 = jet_bwd(Z2, np.einsum("rn,qrp->qnp", rb(W3), rb(dZ3)))
    g[OS.OFF_B2:OS.OFF_W3] = dZ2[0].sum(1)
    g[OS.OFF_W2:OS.OFF_B2] = np.einsum("qrp,qnp->rn", rb(dZ2), rb(H1)).reshape(-1)
    dZ1 = jet_bwd(Z1, np.einsum("rn,qrp->qnp", rb(W2), rb(dZ2)))
    gW1 = np.einsum("rp,pk->rk", dZ1[0], Xa) + np.stack([dZ1[1 + k].sum(1) for k in range(3)], 1)
    g[OS.OFF_W1:OS.OFF_B1] = gW1.reshape(-1)
    g[OS.OFF_B1:OS.OFF_W2] = dZ1[0].sum(1)
    return L, g


BLOCKS = [("W1", OS.OFF_W1, OS.OFF_B1), ("b1", OS.OFF_B1, OS.OFF_W2), ("W2", OS.OFF_W2, OS.OFF_B2),
          ("b2", OS.OFF_B2, OS.OFF_W3), ("W3", OS.OFF_W3, OS.OFF_B3), ("b3", OS.OFF_B3, OS.OFF_W4),
          ("w4", OS.OFF_W4, OS.NPARAM)]
