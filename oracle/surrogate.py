"""FP64 CPU oracle of the learned homogenized-energy surrogate (TEST INFRASTRUCTURE ONLY).

Plain PyTorch CPU code in float64.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may use it; the product library shares no code
with it.

What it computes (2D plane strain):

* The homogenized response of the micro problem is hyperelastic: the macro
  stress is the derivative of the volume-averaged strain energy with respect
  to the macro deformation gradient, and the macro tangent is its second
  derivative (Hill-Mandel condition, paper Sec. 2.3, Eqs. for P-bar and
  A-bar).  Frame invariance makes that energy a function of the right
  Cauchy-Green tensor C = F^T F only, so the surrogate is an energy W(C).
* W(C) = W0(C) + s_W * T(x), with
    - W0 = 1/2 e^T M e, e = (E11, E22, 2 E12), E = (C - I)/2: the quadratic
      (St. Venant-Kirchhoff type) energy whose tangent at F = I equals the
      homogenized small-strain tangent A0 (M is read off A0 by averaging the
      entries that minor symmetry makes equal);
    - x = ((C11 - 1)/s0, (C22 - 1)/s1, C12/s2) the scaled inputs;
    - N(x) the MLP 3 -> 128 -> 128 -> 128 -> 1 with SiLU activations;
    - T(x) = N(x) - N(0) - grad N(0).x - 1/2 x^T hess N(0) x, so the network
      adds nothing to the energy, stress or tangent at F = I.
* P = dW/dF and A = dP/dF are taken by automatic differentiation in F itself
  (no Voigt bookkeeping), A[(i*2+J), (k*2+L)] = dP_iJ / dF_kL.
* Training loss over n points (F_i, P*_i, A*_i):
    L = 1/n sum_i [ wP |P_i - P*_i|^2 / (|P*_i|^2 + rhoP^2)
                  + wA |A_i - A*_i|^2 / (|A*_i|^2 + rhoA^2) ]   (Frobenius norms)
* Adam (Kingma & Ba 2015) with bias correction.

Parameter vector layout (float, 33664 entries): W1[128][3], b1[128],
W2[128][128], b2[128], W3[128][128], b3[128], w4[128]; W_l[out][in].

Parity pins (tests/test_oracle_surrogate.py): P(I) = 0 and A(I) = A0 for a
tangent from the RVE oracle's linear homogenization; with w4 = 0 the closed
St. Venant-Kirchhoff form P = F (C0 : E); frame invariance; major symmetry
of A; the loss gradient against central finite differences; Adam against
torch.optim.Adam.
"""
import numpy as np
import torch

WIDTH = 128
OFF_W1, OFF_B1 = 0, 384
OFF_W2, OFF_B2 = 512, 512 + 16384
OFF_W3, OFF_B3 = OFF_B2 + 128, OFF_B2 + 128 + 16384
OFF_W4 = OFF_B3 + 128
NPARAM = OFF_W4 + 128

_PAIRS = {0: [(0, 0)], 1: [(1, 1)], 2: [(0, 1), (1, 0)]}


def unpack(theta):
    t = theta
    return dict(W1=t[OFF_W1:OFF_B1].reshape(WIDTH, 3), b1=t[OFF_B1:OFF_W2],
                W2=t[OFF_W2:OFF_B2].reshape(WIDTH, WIDTH), b2=t[OFF_B2:OFF_W3],
                W3=t[OFF_W3:OFF_B3].reshape(WIDTH, WIDTH), b3=t[OFF_B3:OFF_W4], w4=t[OFF_W4:NPARAM])


def baseline_M(A0):
    """3x3 matrix M of W0 from the d^2 x d^2 tangent A0 at F = I: entry (a, b)
    averages A0[(I*2+J), (K*2+L)] over the index pairs of Voigt slots a and b
    (slot 2 is the shear pair 12/21); then symmetrized."""
    A0 = np.asarray(A0, np.float64).reshape(4, 4)
    M = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            vals = [A0[I * 2 + J, K * 2 + L] for (I, J) in _PAIRS[a] for (K, L) in _PAIRS[b]]
            M[a, b] = np.mean(vals)
    return 0.5 * (M + M.T)


def silu(z):
    return z * torch.sigmoid(z)


def mlp(p, x):
    """N(x) for x [n,3] -> [n]."""
    h = silu(x @ p["W1"].T + p["b1"])
    h = silu(h @ p["W2"].T + p["b2"])
    h = silu(h @ p["W3"].T + p["b3"])
    return h @ p["w4"]


def taylor_free(p, x):
    """T(x) = N(x) - N(0) - g0.x - 1/2 x^T H0 x with g0, H0 the gradient and
    Hessian of N at the origin (kept in the graph so parameter gradients flow
    through them)."""
    z = torch.zeros(1, 3, dtype=x.dtype, requires_grad=True)
    n0 = mlp(p, z).sum()
    g0 = torch.autograd.grad(n0, z, create_graph=True)[0][0]
    H0 = torch.stack([torch.autograd.grad(g0[k], z, create_graph=True)[0][0] for k in range(3)])
    return mlp(p, x) - n0 - x @ g0 - 0.5 * ((x @ H0) * x).sum(1)


def energy(theta, desc, F):
    """W(F) per point; F [n,2,2] (requires_grad allowed)."""
    p = unpack(theta)
    C = F.transpose(1, 2) @ F
    M = torch.as_tensor(desc["M"], dtype=F.dtype)
    e = torch.stack([0.5 * (C[:, 0, 0] - 1), 0.5 * (C[:, 1, 1] - 1), C[:, 0, 1]], 1)
    W0 = 0.5 * ((e @ M) * e).sum(1)
    s = desc["c_scale"]
    x = torch.stack([(C[:, 0, 0] - 1) / s[0], (C[:, 1, 1] - 1) / s[1], C[:, 0, 1] / s[2]], 1)
    return W0 + desc["w_scale"] * taylor_free(p, x)


def stress_tangent(theta, desc, F, create_graph=False):
    """P [n,4] = dW/dF and A [n,4,4] = dP/dF by automatic differentiation."""
    F = F.detach().clone().requires_grad_(True) if not F.requires_grad else F
    W = energy(theta, desc, F).sum()
    P = torch.autograd.grad(W, F, create_graph=True)[0].reshape(-1, 4)
    rows = [torch.autograd.grad(P[:, c].sum(), F, create_graph=create_graph, retain_graph=True)[0].reshape(-1, 4)
            for c in range(4)]
    A = torch.stack(rows, 1)
    if not create_graph:
        P, A = P.detach(), A.detach()
    return P, A


def make_desc(A0, c_scale=(0.5, 0.5, 0.5), w_scale=0.1):
    return dict(M=baseline_M(A0), c_scale=[float(v) for v in c_scale], w_scale=float(w_scale))


def loss(theta, desc, F, Pt, At, wP=1.0, wA=0.1, rhoP=1e-3, rhoA=1e-3):
    P, A = stress_tangent(theta, desc, F, create_graph=True)
    Pt = torch.as_tensor(Pt, dtype=torch.float64).reshape(-1, 4)
    At = torch.as_tensor(At, dtype=torch.float64).reshape(-1, 4, 4)
    nP = (Pt ** 2).sum(1) + rhoP ** 2
    nA = (At ** 2).sum((1, 2)) + rhoA ** 2
    li = wP * ((P - Pt) ** 2).sum(1) / nP + wA * ((A - At) ** 2).sum((1, 2)) / nA
    return li.mean()


def to_t(a):
    return torch.as_tensor(np.asarray(a, np.float64))


def eval_PA(theta, desc, F):
    """numpy in / out: theta [NPARAM], F [n,4] -> P [n,4], A [n,16]."""
    P, A = stress_tangent(to_t(theta), desc, to_t(F).reshape(-1, 2, 2))
    return P.numpy(), A.reshape(-1, 16).numpy()


def loss_and_grad(theta, desc, F, Pt, At, **w):
    th = to_t(theta).clone().requires_grad_(True)
    L = loss(th, desc, to_t(F).reshape(-1, 2, 2), Pt, At, **w)
    g = torch.autograd.grad(L, th)[0]
    return float(L.detach()), g.numpy()


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step index t >= 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def random_params(seed, scale=1.0):
    """Glorot-uniform weights, small random biases (test inputs)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(NPARAM)

    def glorot(fi, fo):
        a = np.sqrt(6.0 / (fi + fo)) * scale
        return rng.uniform(-a, a, size=fo * fi)
    th[OFF_W1:OFF_B1] = glorot(3, WIDTH)
    th[OFF_B1:OFF_W2] = rng.uniform(-0.1, 0.1, WIDTH)
    th[OFF_W2:OFF_B2] = glorot(WIDTH, WIDTH)
    th[OFF_B2:OFF_W3] = rng.uniform(-0.1, 0.1, WIDTH)
    th[OFF_W3:OFF_B3] = glorot(WIDTH, WIDTH)
    th[OFF_B3:OFF_W4] = rng.uniform(-0.1, 0.1, WIDTH)
    th[OFF_W4:NPARAM] = glorot(WIDTH, 1)
    return th


def network_derivs(theta, x):
    """Gradient [n,3] and Hessian [n,3,3] of the raw network N at the scaled
    inputs x [n,3] (used to scale comparison tolerances)."""
    p = unpack(to_t(theta))
    xt = to_t(x).clone().requires_grad_(True)
    g = torch.autograd.grad(mlp(p, xt).sum(), xt, create_graph=True)[0]
    H = torch.stack([torch.autograd.grad(g[:, k].sum(), xt, retain_graph=True)[0] for k in range(3)], 1)
    return g.detach().numpy(), H.detach().numpy()


def scaled_inputs(desc, F):
    F = np.asarray(F, np.float64).reshape(-1, 2, 2)
    C = np.einsum("nki,nkj->nij", F, F)
    s = desc["c_scale"]
    return np.stack([(C[:, 0, 0] - 1) / s[0], (C[:, 1, 1] - 1) / s[1], C[:, 0, 1] / s[2]], 1)
