#!/usr/bin/env python3
"""Benchmark: converged RVE solves/s of the batched periodic-RVE hot path on one
MI355X, with roofline and CPU-oracle baseline.

Default workload: 4096 RVEs of 32 x 32 bilinear quads (2D plane strain,
neo-Hookean matrix E = 1, nu = 0.3, centred circular inclusion of radius
U[0.15, 0.35] with stiffness ratio 10), F = I + H with H_ij ~ U[-0.15, 0.15],
FP64, Newton to rtol 1e-10, outputs P and A.  One step = one rve_solve_batch
call over the whole batch from a zero initial fluctuation (inputs resident in
HBM; every RVE solved to convergence inside the timed region).

Prints one JSON line.  Options:
  --steps K --warmup W     timed / untimed steps
  --gpus N                 only N = 1 is supported (one GPU)
  --workload NAME          rve2d_32 (default), rve2d_16, rve2d_8, rve3d_mixed
  --no-cpu-baseline        skip the oracle timing
  --calib-copy MiB         after the timed steps, run one plain device copy of
                           this size (for HBM counter calibration under rocprofv3)
  --macro                  also time the two-scale driver (macro steps/s): 4 x 4
                           macro grid / RVE 8 x 8 over 10 load steps, and the
                           64 x 64 plate with a hole (14288 RVEs of 16 x 16) over
                           its first --macro-steps of 20 load steps, nested and
                           alternating two-level Newton
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector = FP64 matrix (dense)
PEAK_HBM_GBS = 8000.0


def make_workload(name):
    from paper_1908_08292_amd import workloads
    if name == "rve2d_32":
        return workloads.rve2d(4096, n=32), dict(workload="rve2d_32x32_B4096", B=4096, d=2, n=32)
    if name == "rve2d_16":
        return workloads.rve2d(14288, n=16, seed=1003), dict(workload="rve2d_16x16_B14288", B=14288, d=2, n=16)
    if name == "rve2d_8":
        return workloads.rve2d(64, n=8, seed=1000), dict(workload="rve2d_8x8_B64", B=64, d=2, n=8)
    if name == "rve3d_mixed":
        return workloads.rve3d(1024), dict(workload="rve3d_8-12-16_B1024", B=1024, d=3, n="8/12/16")
    raise SystemExit(f"unknown workload {name}")


def algorithmic_flops(rve, d, n_arr, iters):
    """LDL^T factorizations (iters + 1 per RVE, one at the converged state) and
    triangular solves (2 nnz(L) flops per sweep per right-hand side: forward and
    backward per Newton step, forward with d^2 columns for the condensation),
    counted from the symbolic plan of each RVE's mesh size."""
    total = 0.0
    cache = {}
    for n, it in zip(n_arr, iters):
        n = int(n)
        if n not in cache:
            cache[n] = rve.plan_info(d, n)
        pi = cache[n]
        total += (it + 1) * pi["factor_flops"] + it * 4.0 * pi["nnz_L"] + 2.0 * d * d * pi["nnz_L"]
    return total


KERNEL_SOURCES = ["rve_solve.hip", "plan.cpp", "plan.h", "solver_dev.h", "mesh_common.h"]


def kernel_source_hash():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1908_08292_amd", "csrc")
    blob = b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES)
    return hashlib.sha256(blob).hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this workload, scaled by the copy-kernel calibration; None when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"rve_solve_kernel_{workload}.hbm.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(wl, meta, budget_rves):
    import oracle
    d = meta["d"]
    B = min(budget_rves, len(wl.F))
    nthreads = len(os.sched_getaffinity(0))
    t_total = 0.0
    ndone = 0
    for n in sorted(set(int(x) for x in wl.n[:B])):
        idx = np.nonzero(wl.n[:B] == n)[0]
        phases = np.stack([oracle.phase_by_centroid(d, n, wl.radius[b]) for b in idx])
        lame = oracle.two_phase_lame(10.0)
        if len(set(wl.ratio[idx])) != 1:
            # per-RVE material: solve one by one (still OpenMP-free per RVE)
            t0 = time.perf_counter()
            for k, b in enumerate(idx):
                oracle.rve_solve(d, n, phases[k], oracle.two_phase_lame(wl.ratio[b]), wl.F[b])
            t_total += time.perf_counter() - t0
        else:
            lame = oracle.two_phase_lame(float(wl.ratio[idx[0]]))
            t0 = time.perf_counter()
            out = oracle.rve_solve_batch(d, n, phases, lame, wl.F[idx], nthreads=nthreads)
            t_total += time.perf_counter() - t0
            assert np.all(out["status"] == 0)
        ndone += len(idx)
    return dict(value=ndone / t_total, unit="RVE solves/s", cores=nthreads, kind="oracle",
                sample=f"first {ndone} of {len(wl.F)} RVEs of the same workload ({t_total:.1f} s, "
                       f"OpenMP over RVEs, {nthreads} threads)")


def macro_bench(nsteps3):
    """Macro steps/s of the GPU two-scale driver (host wall clock per load step)."""
    from paper_1908_08292_amd import fehmm, rve
    res = {}
    lame = rve.two_phase_lame(10.0)
    cases = [("plate4x4_rve8x8", dict(nx=4, ny=4, hole_r=0.0, bc=fehmm.BC_CLAMPED_PULL, stretch=1.1, nsteps=10),
              8, 10),
             ("plate64x64_hole_rve16x16", dict(nx=64, ny=64, hole_r=0.2, bc=fehmm.BC_UNIAXIAL, stretch=1.15,
                                                nsteps=20), 16, nsteps3)]
    for name, kw, n, nrun in cases:
        for scheme, sname in ((fehmm.NESTED, "nested"), (fehmm.ALTERNATING, "alternating")):
            mesh = rve.Mesh(2, n, lame, radius=0.25)
            drv = fehmm.Driver(mesh, scheme=scheme, **kw)
            t0 = time.perf_counter()
            its, mic, ok = [], 0, True
            for k in range(1, nrun + 1):
                st = drv.step(k)
                its.append(st["macro_iters"])
                mic += st["micro_iters"]
                ok = ok and st["status"] == 0
                print(f"[bench] {name} {sname} step {k}: {st['macro_iters']} macro iters", file=sys.stderr,
                      flush=True)
            dt = time.perf_counter() - t0
            res[f"{name}_{sname}"] = dict(macro_steps_per_s=nrun / dt, steps=nrun, rves=drv.nqp,
                                          macro_iters=its, micro_iters=int(mic), converged=bool(ok),
                                          seconds=dt)
            drv.destroy()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rve2d_32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--calib-copy", type=int, default=0)
    ap.add_argument("--macro", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32ir"], default="fp64")
    ap.add_argument("--macro-steps", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the RVE batch would be sharded by macro elements "
              "across GPUs; see DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_08292_amd import api, rve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl, meta = make_workload(args.workload)
    d = meta["d"]
    batch, meshes = api.build_batch(d, wl.n, wl.radius, wl.ratio)
    s = api.Solver(batch, want_A=True, keep_state=False)
    s.set_F(wl.F)
    opts = rve.default_opts(precision=rve.PREC_FP32_IR if args.precision == "fp32ir" else rve.PREC_FP64)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    print(f"[bench] {meta['workload']}: warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        s.solve(opts=opts, stream=sp)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(args.steps):
        s.solve(opts=opts, stream=sp)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    print(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    res = s.results()
    nbad = int((res["status"] != 0).sum())
    if args.calib_copy > 0:
        nel = args.calib_copy * (1 << 20) // 8
        x = torch.ones(nel, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
    B = meta["B"]
    value = B / (ms * 1e-3)
    flops = algorithmic_flops(rve, d, wl.n, res["iters"])
    achieved = flops / (ms * 1e-3) / 1e12
    out = {
        "metric": "converged RVE solves/s (P+A, rel err <=1e-8 vs FP64 oracle)",
        "value": value,
        "unit": "RVE solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 factors + f64 refinement",
        "data": "synthetic",
        "config": {"workload": meta["workload"], "rves": B, "dim": d, "elements_per_edge": meta["n"],
                   "precision": args.precision, "newton_rtol": 1e-10,
                   "mean_newton_iters": float(res["iters"].mean()), "failed_rves": nbad},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": measured_traffic(meta["workload"]),
                     "kernel": f"rve_solve_kernel<{d}>", "flops_per_launch": flops,
                     "flops_counted": "LDL^T factorizations + triangular solves from the symbolic plan"},
    }
    if args.macro:
        out["macro"] = macro_bench(args.macro_steps)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, meta, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
