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
  --no-macro               skip the two-scale driver block (macro steps/s): 4 x 4
                           macro grid / RVE 8 x 8 over 10 load steps, and the
                           64 x 64 plate with a hole (14288 RVEs of 16 x 16) over
                           all 20 load steps, nested and alternating two-level
                           Newton (and, on the plate, nested with FP32 micro
                           assembly and factors), with the oracle's macro driver
                           beside it (all steps of the 4 x 4 plate, step 1 of the
                           64 x 64 plate)
  --no-assembly            skip the assembly phase timed alone (HBM roofline)
  --no-peaks               skip the measured FP64 / FP32 MFMA and HBM copy rates
  --no-cpu-3d              skip the oracle subsample of the uneven 3D batch
                           (16 RVEs of 8^3 and of 12^3)
  --cpu-3d-full            also time 16 RVEs of 16^3 on the host (minutes) and
                           extrapolate the oracle to the whole 3D batch
  --precision fp64|fp32ir|both   the timed RVE path(s); `value` is the FP64 path
                           when it is timed, the FP32-factor path otherwise
  --no-surrogate           skip the surrogate block: MLP energy W(C) trained by the
                           library on 2e5 solver-generated triples (16 x 16 RVE,
                           H in [-0.2, 0.2]), its evals/s on 14288 points, a 2 %
                           random audit of the plate problem's accepted points
                           against RVE solves, and macro steps/s of the 64 x 64
                           plate with a hole over its first --macro-steps load
                           steps, nested, plain FP64 (macro rtol 1e-10 and 1e-4)
                           vs surrogate with fallback at indicator 1e-3
  --no-3d                  skip the uneven 3D block (with a 2D workload): 1024 RVEs
                           of 8^3 / 12^3 / 16^3, one timed launch per precision
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X published FP64 (vector and matrix)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 MFMA
PEAK_FP32_TFLOPS = 157.3
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
    """LDL^T factorizations and triangular solves (2 nnz(L) flops per sweep per
    right-hand side), counted from the symbolic plan of each RVE's mesh size.
    The condensation reuses the last Newton factorization (2D, and 3D plans with
    fronts in global memory): iters factorizations, the last one with the d^2
    condensation columns forward-substituted beside the residual, then their
    backward sweep (a missed convergence prediction adds a factorization that is
    not counted).  3D plans with fronts in LDS: iters + 1 factorizations (one at
    the converged state, with the d^2 columns forward-substituted)."""
    total = 0.0
    cache = {}
    for n, it in zip(n_arr, iters):
        n = int(n)
        if n not in cache:
            sch = rve.plan_schedule(d, n)
            lds = bool(sch["wave"].any()) or len(sch["steps"]) > 0
            cache[n] = (rve.plan_info(d, n), d == 2 or not lds)
        pi, reuse = cache[n]
        if reuse:
            total += it * pi["factor_flops"] + it * 4.0 * pi["nnz_L"] + 4.0 * d * d * pi["nnz_L"]
        else:
            total += (it + 1) * pi["factor_flops"] + it * 4.0 * pi["nnz_L"] + 2.0 * d * d * pi["nnz_L"]
    return total


KERNEL_SOURCES = ["rve_solve.hip", "rve_solve512.hip", "plan.cpp", "plan.h", "solver_dev.h", "mesh_common.h"]


def kernel_source_hash():
    import hashlib
    csrc = os.path.join(ROOT, "paper_1908_08292_amd", "csrc")
    blob = b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES)
    return hashlib.sha256(blob).hexdigest()[:16]


def measured_traffic(workload, precision="fp64", kernel="rve_solve_kernel"):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary of this workload, scaled by the copy-kernel calibration; None when
    the kernel sources changed since the counters were taken."""
    tag = "" if precision == "fp64" else "_" + precision
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}{tag}.hbm.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(wl, meta, budget_rves, gpu_results=None):
    """Oracle throughput on the first RVEs of the (single-material) 2D workload:
    one untimed warm-up on 32 RVEs, then three timed runs of the sample, median
    reported (OpenMP over RVEs on every host thread).  When GPU results of the
    same RVEs are given, also the largest relative errors against them."""
    import oracle
    d = meta["d"]
    B = min(budget_rves, len(wl.F))
    nthreads = len(os.sched_getaffinity(0))
    n = int(wl.n[0])
    assert np.all(wl.n[:B] == n) and len(set(wl.ratio[:B])) == 1
    phases = np.stack([oracle.phase_by_centroid(d, n, wl.radius[b]) for b in range(B)])
    lame = oracle.two_phase_lame(float(wl.ratio[0]))
    oracle.rve_solve_batch(d, n, phases[:32], lame, wl.F[:32], nthreads=nthreads)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        out = oracle.rve_solve_batch(d, n, phases, lame, wl.F[:B], nthreads=nthreads)
        times.append(time.perf_counter() - t0)
    assert np.all(out["status"] == 0)
    t_med = float(np.median(times))
    worst = {}
    mu_max = lame[:, 1].max()
    Po, Ao = out["P"].reshape(B, -1), out["A"].reshape(B, -1)
    for name, res in (gpu_results or {}).items():
        Pg = res["P"].reshape(len(wl.F), -1)[:B]
        Ag = res["A"].reshape(len(wl.F), -1)[:B]
        eP = np.linalg.norm(Pg - Po, axis=1) / np.maximum(np.linalg.norm(Po, axis=1), 1e-12 * mu_max)
        eA = np.linalg.norm(Ag - Ao, axis=1) / np.maximum(np.linalg.norm(Ao, axis=1), 1e-12 * mu_max)
        worst[name] = {"max_rel_err_P": float(eP.max()), "max_rel_err_A": float(eA.max())}
    res = dict(value=B / t_med, unit="RVE solves/s", cores=nthreads, kind="oracle",
               sample=f"first {B} of {len(wl.F)} RVEs of the same workload: median of 3 runs "
                      f"({', '.join(f'{t:.2f}' for t in times)} s) after a 32-RVE warm-up, OpenMP over RVEs, "
                      f"{nthreads} threads", cpu_model=cpu_model())
    if worst:
        res["gpu_vs_oracle_on_sample"] = worst
    return res


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline_3d(per_size, full16=False):
    """Oracle on a subsample of the uneven 3D workload: per mesh size the first
    per_size RVEs of that size, solved concurrently on the host threads (one
    RVE per thread; ctypes releases the GIL).  16^3 (about 4 minutes per RVE and
    core) is timed only with full16; the batch estimate then extrapolates the
    per-size rates to the 1024-RVE mix."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1908_08292_amd import workloads
    wl = workloads.rve3d(1024)
    nthreads = len(os.sched_getaffinity(0))
    out = {"workload": "rve3d_8-12-16_B1024", "cores": nthreads, "kind": "oracle", "per_size": {}}
    sizes = (8, 12, 16) if full16 else (8, 12)

    def one(b):
        n = int(wl.n[b])
        r = oracle.rve_solve(3, n, oracle.phase_by_centroid(3, n, float(wl.radius[b])),
                             oracle.two_phase_lame(float(wl.ratio[b])), wl.F[b])
        return r["status"]

    for n in sizes:
        idx = [int(i) for i in np.nonzero(wl.n == n)[0][:per_size]]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=nthreads) as ex:
            st = list(ex.map(one, idx))
        dt = time.perf_counter() - t0
        out["per_size"][f"{n}^3"] = dict(rves=len(idx), seconds=dt, solves_per_s=len(idx) / dt,
                                         threads=min(nthreads, len(idx)), failed=int(sum(x != 0 for x in st)))
        print(f"[bench] oracle 3d {n}^3: {len(idx)} RVEs in {dt:.1f} s", file=sys.stderr, flush=True)
    if full16:
        counts = {n: int((wl.n == n).sum()) for n in (8, 12, 16)}
        est = sum(counts[n] / out["per_size"][f"{n}^3"]["solves_per_s"] for n in (8, 12, 16))
        out["batch_estimate"] = dict(seconds=est, solves_per_s=1024 / est, extrapolated=True,
                                     note="per-size rates of the subsample applied to the 1024-RVE mix")
    else:
        out["note"] = "16^3 not timed in the default run (about 230 s per RVE and core); bench.py --cpu-3d-full"
    return out


def time_solves(s, opts, stream, steps, warmup):
    import torch
    sp = stream.cuda_stream
    for _ in range(warmup):
        s.solve(opts=opts, stream=sp)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        s.solve(opts=opts, stream=sp)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def surrogate_bench(macro_steps):
    """The surrogate of the 64 x 64 plate problem's 16 x 16 RVE: training, evaluation, audit, macro steps."""
    import torch

    from paper_1908_08292_amd import api, fehmm, rve, surrogate
    out = {}
    fit = {}
    sg = api.fit_surrogate(n=16, radius=0.25, ratio=10.0, n_train=200000, n_calib=20000, h=0.2, timings=fit)
    out["train"] = fit
    print(f"[bench] surrogate trained: {fit}", file=sys.stderr, flush=True)
    # macro steps/s, plain FP64 vs surrogate with fallback (nested)
    lame = rve.two_phase_lame(10.0)
    runs = {}
    # plain FP64 at the default macro tolerance (1e-10) and at the surrogate's (1e-4)
    for use in (False, "plain_rtol", True):
        mesh = rve.Mesh(2, 16, lame, radius=0.25)
        drv = fehmm.Driver(mesh, nx=64, ny=64, hole_r=0.2, bc=fehmm.BC_UNIAXIAL, stretch=1.15, nsteps=20,
                           rtol_macro=1e-4 if use == "plain_rtol" else 1e-10)
        if use is True:
            drv.set_surrogate(sg, threshold=1e-3, precision=surrogate.BF16X3, macro_rtol=1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its, fb, ev, ok = [], 0, 0, True
        for k in range(1, macro_steps + 1):
            st = drv.step(k)
            its.append(st["macro_iters"])
            ev += (st["macro_iters"] + 1) * drv.nqp
            fb += st["fallback_points"] if use is True else (st["macro_iters"] + 1) * drv.nqp
            ok = ok and st["status"] == 0
        dt = time.perf_counter() - t0
        runs[use] = dict(macro_steps_per_s=macro_steps / dt, seconds=dt, macro_iters=its, rve_solves=int(fb),
                         qp_evaluations=int(ev), converged=bool(ok), u=drv.u(),
                         macro_rtol=1e-10 if use is False else 1e-4)
        if use is True:
            F_last = torch.tensor(drv.qp()[0], device="cuda").reshape(-1, 4).contiguous()
        drv.destroy()
        print(f"[bench] plate 64x64 {use}: {runs[use]['seconds']:.2f} s", file=sys.stderr, flush=True)
    ref = runs[False]["u"]
    du = float(np.linalg.norm(runs[True]["u"] - ref) / np.linalg.norm(ref))
    du_plain = float(np.linalg.norm(runs["plain_rtol"]["u"] - ref) / np.linalg.norm(ref))
    for r in runs.values():
        r.pop("u")
    runs["plain_rtol"]["rel_displacement_diff"] = du_plain
    out["macro_plate64_hole_rve16"] = dict(
        plain_fp64=runs[False], plain_fp64_at_surrogate_rtol=runs["plain_rtol"], surrogate=runs[True],
        speedup=runs[True]["macro_steps_per_s"] / runs[False]["macro_steps_per_s"],
        speedup_at_equal_rtol=runs[True]["macro_steps_per_s"] / runs["plain_rtol"]["macro_steps_per_s"],
        rel_displacement_diff=du, steps=macro_steps, rves=int(F_last.shape[0]),
        note="rel_displacement_diff against the plain run at macro rtol 1e-10")
    # evals/s on the last state's 14288 points, and the audit of a 2% random sample
    nq = F_last.shape[0]
    P = torch.empty(nq, 4, dtype=torch.float64, device="cuda")
    A = torch.empty(nq, 16, dtype=torch.float64, device="cuda")
    ind = torch.empty(nq, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(3):
        sg.eval(F_last, P, A, ind, precision=surrogate.BF16X3, stream=stream.cuda_stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    reps = 50
    ev0.record(stream)
    for _ in range(reps):
        sg.eval(F_last, P, A, ind, precision=surrogate.BF16X3, stream=stream.cuda_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) / reps * 1e3
    rng = np.random.default_rng(1004)
    pick = np.sort(rng.choice(nq, size=max(1, int(np.ceil(0.02 * nq))), replace=False))
    Fa = F_last.cpu().numpy()[pick]
    batch, _ = api.build_batch(2, np.full(len(pick), 16), np.full(len(pick), 0.25), np.full(len(pick), 10.0))
    judge = api.Solver(batch, keep_state=False)
    judge.set_F(Fa)
    judge.solve()
    jr = judge.results()
    Pj = jr["P"].reshape(-1, 4)
    Ps = P.cpu().numpy()[pick]
    acc = (ind.cpu().numpy()[pick] <= 1e-3) & (jr["status"] == 0)
    e = np.linalg.norm(Ps - Pj, axis=1) / np.linalg.norm(Pj, axis=1)
    flops = 2 * 2.0 * 128 * 128 * 10  # two 128x128 layers on 10-component jets (algorithmic, per point)
    out["eval"] = dict(points=int(nq), us_per_launch=us, evals_per_s=nq / (us * 1e-6), precision="bf16x3",
                       roofline={"bound": "mfma", "achieved": flops * nq / (us * 1e-6) / 1e12,
                                 "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                                 "frac": flops * nq / (us * 1e-6) / 1e12 / PEAK_BF16_TFLOPS,
                                 "flops_counted": "2 x 2*128*128*10 per point (jet GEMMs; the split "
                                                  "form executes 3x that on the MFMA)"})
    out["audit"] = dict(sample=f"{len(pick)} random points (2%) of the last load step's {nq}",
                        accepted_fraction=float(acc.mean()),
                        max_rel_err_P_accepted=float(e[acc].max()) if acc.any() else None,
                        p99_rel_err_P_accepted=float(np.quantile(e[acc], 0.99)) if acc.any() else None,
                        threshold=1e-3)
    sg.destroy()
    return out


MACRO_CASES = [
    # name, driver keywords, RVE elements per edge, load steps run
    ("plate4x4_rve8x8", dict(nx=4, ny=4, hole_r=0.0, bc=0, stretch=1.1, nsteps=10), 8, 10),
    ("plate64x64_hole_rve16x16", dict(nx=64, ny=64, hole_r=0.2, bc=1, stretch=1.15, nsteps=20), 16, 20),
]


def macro_bench(oracle_baseline=True):
    """Macro steps/s of the GPU two-scale driver (host wall clock per load step),
    nested and alternating two-level Newton, on the 4 x 4 plate (RVE 8 x 8, 10
    steps) and the 64 x 64 plate with a hole (14288 RVEs of 16 x 16, all 20
    steps); beside it the oracle's macro driver on the host: all 10 steps of the
    4 x 4 plate (both schemes) and load step 1 of the 64 x 64 plate (nested)."""
    from paper_1908_08292_amd import fehmm, rve
    res = {}
    lame = rve.two_phase_lame(10.0)
    u_end = {}
    for name, kw, n, nrun in MACRO_CASES:
        runs = [(fehmm.NESTED, "nested", rve.PREC_FP64), (fehmm.ALTERNATING, "alternating", rve.PREC_FP64)]
        if nrun == 20:
            runs.append((fehmm.NESTED, "nested_fp32_micro", rve.PREC_FP32_IR))
        for scheme, sname, prec in runs:
            mesh = rve.Mesh(2, n, lame, radius=0.25)
            drv = fehmm.Driver(mesh, scheme=scheme, max_macro_iter=40, micro_opts=rve.default_opts(precision=prec),
                               **kw)
            t0 = time.perf_counter()
            its, mic, ok = [], 0, True
            for k in range(1, nrun + 1):
                st = drv.step(k)
                its.append(st["macro_iters"])
                mic += st["micro_iters"]
                ok = ok and st["status"] == 0
            dt = time.perf_counter() - t0
            print(f"[bench] {name} {sname}: {nrun} steps in {dt:.2f} s, macro iters {its}", file=sys.stderr,
                  flush=True)
            res[f"{name}_{sname}"] = dict(macro_steps_per_s=nrun / dt, steps=nrun, rves=drv.nqp,
                                          macro_iters=its, total_macro_iters=int(sum(its)),
                                          micro_updates=int(mic), converged=bool(ok), seconds=dt,
                                          u_max=float(st["u_max"]))
            u_end[sname] = drv.u()
            if sname == "nested_fp32_micro":
                u64 = u_end["nested"]
                res[f"{name}_{sname}"].update(
                    micro_precision="f32 assembly and factors + f64 refinement",
                    speedup_vs_fp64_micro=res[f"{name}_nested"]["seconds"] / dt,
                    rel_displacement_diff_vs_fp64_micro=float(np.abs(u_end[sname] - u64).max() /
                                                              max(np.abs(u64).max(), 1e-300)))
            drv.destroy()
    for name in ("plate4x4_rve8x8", "plate64x64_hole_rve16x16"):
        a, b = res[f"{name}_nested"], res[f"{name}_alternating"]
        res[f"{name}_alternating_vs_nested"] = dict(
            time_ratio=b["seconds"] / a["seconds"], macro_iter_ratio=b["total_macro_iters"] / a["total_macro_iters"],
            micro_update_ratio=b["micro_updates"] / max(a["micro_updates"], 1))
    if oracle_baseline:
        res["cpu_baseline"] = macro_oracle_baseline()
    return res


def macro_oracle_baseline():
    import oracle
    nthreads = len(os.sched_getaffinity(0))
    out = {"kind": "oracle", "cores": nthreads}
    lame = oracle.two_phase_lame(10.0)
    for name, kw, n, nrun in MACRO_CASES:
        ph = oracle.phase_by_centroid(2, n, 0.25)
        schemes = (0, 1) if nrun == 10 else (0,)
        for scheme in schemes:
            m = oracle.Macro(kw["nx"], kw["ny"], n, ph, lame, hole_r=kw["hole_r"], bc=kw["bc"],
                             stretch=kw["stretch"], nsteps=kw["nsteps"], scheme=scheme, max_macro_iter=40)
            steps = nrun if nrun == 10 else 1
            t0 = time.perf_counter()
            its = [m.step(k)["macro_iters"] for k in range(1, steps + 1)]
            dt = time.perf_counter() - t0
            m.close()
            sname = "nested" if scheme == 0 else "alternating"
            out[f"{name}_{sname}"] = dict(macro_steps_per_s=steps / dt, steps_timed=steps, seconds=dt,
                                         macro_iters=its)
            print(f"[bench] oracle {name} {sname}: {steps} steps in {dt:.1f} s", file=sys.stderr, flush=True)
    return out


def assembly_block(s, wl, meta, reps=20):
    """The assembly phase alone (element pass + residual gather of every RVE,
    rve_assemble_batch) on the timed batch at w = 0, against HBM: algorithmic
    bytes per assembly = w + phase + R + the symmetric node-block tangent
    (nodes x d^2 x (3^d + 1) / 2 doubles), and the bytes this kernel moves
    (w, phase, element residuals written and read back, element tangents, R)."""
    import torch
    d, n, B = meta["d"], int(wl.n[0]), meta["B"]
    nn = ne = n ** d
    nen = 2 ** d
    nd = nen * d
    alg = 8 * nn * d * 2 + ne + 8 * nn * d * d * (3 ** d + 1) / 2
    moved = 8 * nn * d * 2 + ne + 8 * ne * nd * 2 + 8 * ne * nd * nd + 8 * nn * d
    stream = torch.cuda.current_stream()
    for _ in range(3):
        s.batch.assemble(s.F, None, s.status, stream=stream.cuda_stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        s.batch.assemble(s.F, None, s.status, stream=stream.cuda_stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    ach = alg * B / (ms * 1e-3) / 1e9
    ach_moved = moved * B / (ms * 1e-3) / 1e9
    return {"kernel": f"rve_assembly_kernel<{d}>", "ms_per_launch": ms, "rves": B,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": ach / PEAK_HBM_GBS, "bytes_per_assembly": alg,
                         "traffic": measured_traffic(meta["workload"], "fp64", "rve_assembly_kernel"),
                         "bytes_counted": "w + phase + R + symmetric node-block K (algorithmic)"},
            "moved_bytes_per_assembly": moved, "achieved_gbs_on_moved_bytes": ach_moved}


def rve3d_block(precs, steps=1, warmup=1):
    """The uneven 3D batch (1024 RVEs of 8^3 / 12^3 / 16^3, cost-ordered queue) in
    each precision: one timed launch after one warm-up, with its roofline."""
    import torch
    from paper_1908_08292_amd import api, rve
    wl, meta = make_workload("rve3d_mixed")
    batch, meshes = api.build_batch(3, wl.n, wl.radius, wl.ratio)
    s = api.Solver(batch, want_A=True, keep_state=False)
    s.set_F(wl.F)
    stream = torch.cuda.current_stream()
    out = {"workload": meta["workload"], "rves": meta["B"]}
    for p in precs:
        opts = rve.default_opts(precision=rve.PREC_FP32_IR if p == "fp32ir" else rve.PREC_FP64)
        print(f"[bench] {meta['workload']} {p}: warmup {warmup}, steps {steps}", file=sys.stderr, flush=True)
        ms = time_solves(s, opts, stream, steps, warmup)
        res = s.results()
        flops = algorithmic_flops(rve, 3, wl.n, res["iters"])
        achieved = flops / (ms * 1e-3) / 1e12
        peak = PEAK_FP64_TFLOPS if p == "fp64" else PEAK_FP32_TFLOPS
        out[p] = {"value": meta["B"] / (ms * 1e-3), "unit": "RVE solves/s", "ms_per_step": ms,
                  "failed_rves": int((res["status"] != 0).sum()),
                  "mean_newton_iters": float(res["iters"].mean()),
                  "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                               "frac": achieved / peak, "traffic": measured_traffic(meta["workload"], p)}}
        print(f"[bench] {p}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    if "fp64" in out and "fp32ir" in out:
        out["fp32ir"]["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32ir"]["ms_per_step"]
    del s
    batch.destroy()
    for m in meshes:
        m.destroy()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rve2d_32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=768)
    ap.add_argument("--calib-copy", type=int, default=0)
    ap.add_argument("--no-macro", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32ir", "both"], default="both")
    ap.add_argument("--macro-steps", type=int, default=4)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-3d", action="store_true")
    ap.add_argument("--no-cpu-3d", action="store_true")
    ap.add_argument("--cpu-3d-full", action="store_true")
    ap.add_argument("--no-peaks", action="store_true")
    ap.add_argument("--no-assembly", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (the RVE batch would be sharded by macro elements "
              "across GPUs); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1908_08292_amd import api, rve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl, meta = make_workload(args.workload)
    d = meta["d"]
    batch, meshes = api.build_batch(d, wl.n, wl.radius, wl.ratio)
    s = api.Solver(batch, want_A=True, keep_state=False)
    s.set_F(wl.F)
    stream = torch.cuda.current_stream()
    precs = ["fp64", "fp32ir"] if args.precision == "both" else [args.precision]
    timed = {}
    for p in precs:
        opts = rve.default_opts(precision=rve.PREC_FP32_IR if p == "fp32ir" else rve.PREC_FP64)
        print(f"[bench] {meta['workload']} {p}: warmup {args.warmup}, steps {args.steps}", file=sys.stderr,
              flush=True)
        ms = time_solves(s, opts, stream, args.steps, args.warmup)
        res = s.results()
        timed[p] = dict(ms=ms, res=res, nbad=int((res["status"] != 0).sum()))
        print(f"[bench] {p}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    head = "fp64" if "fp64" in timed else precs[0]
    ms, res = timed[head]["ms"], timed[head]["res"]
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
    peak = PEAK_FP64_TFLOPS if head == "fp64" else PEAK_FP32_TFLOPS  # the factors' arithmetic type
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
        "dtype": "f64" if head == "fp64" else "f32 tangents and factors + f64 refinement",
        "data": "synthetic",
        "config": {"workload": meta["workload"], "rves": B, "dim": d, "elements_per_edge": meta["n"],
                   "precision": head, "newton_rtol": 1e-10,
                   "mean_newton_iters": float(res["iters"].mean()), "failed_rves": timed[head]["nbad"]},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(meta["workload"], head),
                     "kernel": f"rve_solve_kernel<{d}>", "flops_per_launch": flops,
                     "flops_counted": "LDL^T factorizations + triangular solves from the symbolic plan: one "
                                      "factorization per Newton step (the condensation reuses the last one), "
                                      "none at the converged state"},
    }
    if "fp32ir" in timed and head != "fp32ir":
        t = timed["fp32ir"]
        out["mixed_precision"] = dict(value=B / (t["ms"] * 1e-3), unit="RVE solves/s", ms_per_step=t["ms"],
                                      speedup_vs_fp64=ms / t["ms"], failed_rves=t["nbad"],
                                      traffic=measured_traffic(meta["workload"], "fp32ir"),
                                      mean_newton_iters=float(t["res"]["iters"].mean()),
                                      dtype="f32 element tangents and factors (LDL^T, solves) + f64 residuals "
                                            "(matrix-free K x), refinement, norms, averages and condensation")
    if not args.no_assembly and d == 2:
        out["assembly"] = assembly_block(s, wl, meta)
        print(f"[bench] assembly: {out['assembly']['ms_per_launch']:.3f} ms", file=sys.stderr, flush=True)
    if not args.no_peaks:
        out["measured_peaks"] = dict(rve.probe_peaks(stream.cuda_stream),
                                     probe="rve_probe_peaks: v_mfma_*_16x16x4 with 8 independent accumulators "
                                           "per wave; 1 GiB device copy (read + write bytes)")
        print(f"[bench] peaks: {out['measured_peaks']}", file=sys.stderr, flush=True)
    if not args.no_3d and d == 2:
        out["rve3d_uneven"] = rve3d_block(precs)
    if not args.no_macro and d == 2:
        out["macro"] = macro_bench(oracle_baseline=not args.no_cpu_baseline)
    if not args.no_surrogate and d == 2:
        out["surrogate"] = surrogate_bench(args.macro_steps)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, meta, args.cpu_sample,
                                           gpu_results={p: t["res"] for p, t in timed.items()})
        if not args.no_cpu_3d and not args.no_3d and d == 2:
            out["rve3d_uneven"]["cpu_baseline"] = cpu_baseline_3d(16, full16=args.cpu_3d_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
