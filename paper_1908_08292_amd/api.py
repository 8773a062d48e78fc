"""Convenience layer over the binding: builds meshes/batches for a workload and
runs rve_solve_batch on torch device tensors (allocation and marshalling only)."""
import numpy as np

from . import rve


def build_batch(d, n_list, radius_list, ratio_list, nu=0.3, E=1.0, center=None, law=rve.LAW_NEOHOOKE,
                bc=rve.BC_PERIODIC, elem=rve.ELEM_Q1):
    """One mesh per distinct (n, radius, ratio); returns (Batch, meshes)."""
    cache = {}
    meshes = []
    for n, r, q in zip(n_list, radius_list, ratio_list):
        key = (int(n), float(r), float(q))
        if key not in cache:
            cache[key] = rve.Mesh(d, int(n), rve.two_phase_lame(float(q), E=E, nu=nu), radius=float(r),
                                  center=center, law=law, bc=bc, elem=elem)
        meshes.append(cache[key])
    return rve.Batch(meshes), meshes


class Solver:
    """Device buffers for one batch; solve() runs the whole hot path on the GPU."""

    def __init__(self, batch, want_A=True, keep_state=True, device="cuda"):
        import torch
        self.batch = batch
        B, d = batch.B, batch.d
        self.F = torch.zeros(B * d * d, dtype=torch.float64, device=device)
        self.P = torch.zeros(B * d * d, dtype=torch.float64, device=device)
        self.A = torch.zeros(B * d ** 4, dtype=torch.float64, device=device) if want_A else None
        self.w = torch.zeros(int(batch.state_offsets[-1]), dtype=torch.float64, device=device) if keep_state else None
        self.status = torch.zeros(B, dtype=torch.int32, device=device)
        self.iters = torch.zeros(B, dtype=torch.int32, device=device)

    def set_F(self, F):
        import torch
        self.F.copy_(torch.as_tensor(np.ascontiguousarray(F, np.float64).reshape(-1)))

    def solve(self, opts=None, stream=None):
        return self.batch.solve(self.F, self.P, self.A, self.w, self.status, self.iters, opts=opts, stream=stream)

    def results(self):
        B, d = self.batch.B, self.batch.d
        out = dict(P=self.P.cpu().numpy().reshape(B, d, d), status=self.status.cpu().numpy(),
                   iters=self.iters.cpu().numpy())
        if self.A is not None:
            out["A"] = self.A.cpu().numpy().reshape(B, d * d, d * d)
        return out


def small_strain_tangent(n, radius, ratio):
    """Homogenized tangent at F = I of one 2D RVE, from the GPU solver ([4,4])."""
    b, _ = build_batch(2, np.array([n]), np.array([radius]), np.array([ratio]))
    s = Solver(b, keep_state=False)
    s.set_F(np.eye(2).reshape(1, 4))
    s.solve()
    out = s.results()
    if out["status"][0] != 0:
        raise RuntimeError("RVE solve at F = I failed")
    return out["A"][0]


def fit_surrogate(n=16, radius=0.25, ratio=10.0, n_train=200000, n_calib=20000, h=0.2, seed=1004,
                  train_opts=None, precision=1, w_scale=0.1, timings=None):
    """A trained and calibrated surrogate of one 2D RVE (surrogate.h), from
    (F, P, A) triples that the batched RVE solver generates: F = I + H with H_ij
    iid U[-h, h] (det F >= 0.5), n_train for Adam and n_calib more, judged by the
    same solver, for the error indicator.  Returns the Surrogate."""
    import time

    import torch

    from . import surrogate, workloads
    t0 = time.perf_counter()
    F = workloads.draw_F(np.random.default_rng(seed), n_train + n_calib, 2, h).reshape(-1, 4)
    batch, _ = build_batch(2, np.full(len(F), n), np.full(len(F), radius), np.full(len(F), ratio))
    sol = Solver(batch, keep_state=False)
    sol.set_F(F)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # training tangents from the direct Schur form at the converged state (exact
    # to rounding; the default reuse of the last Newton factorization is exact
    # to second order in the last Newton step, about 1e-11 here)
    sol.solve(opts=rve.default_opts(flags=rve.FLAG_DIRECT_TANGENT))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ok = sol.status == 0
    ok_tr, ok_cal = ok.clone(), ok.clone()
    ok_tr[n_train:] = False
    ok_cal[:n_train] = False
    Fv, Pv, Av = sol.F.view(-1, 4), sol.P.view(-1, 4), sol.A.view(-1, 16)
    sg = surrogate.Surrogate(small_strain_tangent(n, radius, ratio), w_scale=w_scale, seed=seed)
    opts = train_opts if train_opts is not None else surrogate.train_opts()
    loss = sg.train(Fv[ok_tr].contiguous(), Pv[ok_tr].contiguous(), Av[ok_tr].contiguous(), opts)
    t3 = time.perf_counter()
    sg.calibrate(Fv[ok_cal].contiguous(), Pv[ok_cal].contiguous(), precision=precision)
    t4 = time.perf_counter()
    if timings is not None:
        timings.update(setup_s=t1 - t0, data_s=t2 - t1, data_solves=len(F), failed_solves=int((~ok).sum().item()),
                       train_s=t3 - t2, train_steps=int(opts.steps), train_batch=int(opts.batch),
                       final_loss=float(np.mean(loss[-min(50, len(loss)):])) if len(loss) else None,
                       calibrate_s=t4 - t3)
    return sg


def square_inclusion_phase(n, half=0.25):
    """Phase ids of an n x n cell with the centred square inclusion
    |x - 1/2| < half, |y - 1/2| < half (by element centroid); resolved exactly
    when half * n is an integer."""
    c = (np.arange(n) + 0.5) / n - 0.5
    inside = (np.abs(c)[None, :] < half) & (np.abs(c)[:, None] < half)
    return inside.reshape(-1).astype(np.uint8)


def micro_convergence(law, ns=(4, 8, 16, 32, 64), F=None, ratio=10.0, half=0.25):
    """Pbar and Abar of one 2D RVE with a square inclusion resolved exactly at
    every n of ns (the micro-convergence setting of Sec. 6 with a synthetic
    microstructure), solved on the GPU; returns dict n -> (P, A) and the orders
    p_n = log2(|X_n - X_2n| / |X_2n - X_4n|) of successive differences."""
    import torch
    F = np.array([[1.08, 0.05], [-0.03, 0.94]]) if F is None else np.asarray(F, np.float64)
    lame = rve.two_phase_lame(ratio)
    out = {}
    for n in ns:
        mesh = rve.Mesh(2, int(n), lame, phase=square_inclusion_phase(int(n), half), law=law)
        batch = rve.Batch([mesh])
        s = Solver(batch, keep_state=False)
        s.set_F(F.reshape(1, 4))
        s.solve()
        torch.cuda.synchronize()
        r = s.results()
        if r["status"][0] != 0:
            raise RuntimeError(f"micro convergence: RVE n={n} failed with status {r['status'][0]}")
        out[int(n)] = (r["P"][0].copy(), r["A"][0].copy())
        batch.destroy()
        mesh.destroy()
    orders = {}
    for key, idx in (("P", 0), ("A", 1)):
        diffs = [np.linalg.norm(out[a][idx] - out[b][idx]) for a, b in zip(ns[:-1], ns[1:])]
        orders[key] = [float(np.log2(diffs[k] / diffs[k + 1])) for k in range(len(diffs) - 1)]
        orders[key + "_diffs"] = [float(x) for x in diffs]
    return out, orders
