"""Convenience layer over the binding: builds meshes/batches for a workload and
runs rve_solve_batch on torch device tensors (allocation and marshalling only)."""
import numpy as np

from . import rve


def build_batch(d, n_list, radius_list, ratio_list, nu=0.3, E=1.0, center=None):
    """One mesh per distinct (n, radius, ratio); returns (Batch, meshes)."""
    cache = {}
    meshes = []
    for n, r, q in zip(n_list, radius_list, ratio_list):
        key = (int(n), float(r), float(q))
        if key not in cache:
            cache[key] = rve.Mesh(d, int(n), rve.two_phase_lame(float(q), E=E, nu=nu), radius=float(r),
                                  center=center)
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
