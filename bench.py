"""Benchmark: solved DOF/s of the non-negative diffusion QP at KKT tol 1e-8.

One step = one full solve of the 128^3-cell anisotropic Kuhn-tet problem
(2,048,383 free DOF, 30,340,171 nonzeros; D = R diag(1, 1e-2, 1e-4) R^T,
f = 1 on the central cube of side 1/4, c = 0 on the boundary) from the
paper's start value c = 1e-8, FP64, until ||pg||_2 <= 1e-8 ||f||_2.  K and f
are assembled on the device before the timed region.

Prints one JSON line.  `roofline` is for the dominant kernel (the CG matrix
pass): algorithmic bytes of its launches (perfect-cache model) over their
average duration, both measured with HIP events on the solve stream inside
the timed region.  `cpu_baseline` times the CPU oracle on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# The paper's own numbers, as context only (vs_baseline stays null): the
# single-core CPU times, in seconds, of its cube-with-hole case A3 (2,175,330
# vertices of unstructured tets, the size class of the 128^3 cube; bounds
# [0, 1]; TAO/KSP relative tolerance 1e-6), Tables Tab:S5_cube_times_mustang
# (AMD Opteron 6176, 2.3 GHz) and Tab:S5_cube_times_wolf (Intel Xeon E5-2670,
# 2.6 GHz), one core each.
PAPER_A3_SECONDS = {
    "mustang_1_core": {"galerkin": 121.0, "tron1": 225.0, "tron2": 414.0, "tron3": 599.0,
                       "blmvm": 1167.0},
    "wolf_1_core": {"galerkin": 48.0, "tron1": 98.4, "tron2": 129.0, "tron3": 247.0,
                    "blmvm": 609.0},
}


def paper_context() -> dict:
    return {"case": "A3: cube with a hole, 2,175,330 vertices (unstructured tets), bounds [0, 1]",
            "tolerance": "TAO/KSP relative 1e-6", "seconds": PAPER_A3_SECONDS,
            "note": "single-core CPU times from the paper, context only: other meshes, "
                    "tolerance and hardware"}
EXTRAS = ("mixed", "small", "transient", "batch", "serve")
CSRC = os.path.join(ROOT, "paper_1506_08435_amd", "csrc")
# sources that decide what a kernel reads and writes: its code, the slice
# walkers, the constants and the host code that chooses layouts and launches
KERNEL_SOURCES = {
    "single": ("kernels.hip", "rows.hpp", "nnqp_internal.hpp", "solver.hip", "api.hip"),
    "batch": ("batch.hip", "rows.hpp", "nnqp_internal.hpp", "api.hip"),
}


def kernel_hash(group: str = "single") -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[group]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_file(kernel: str, workload: str, precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.txt")


def read_traffic(kernel: str, workload: str, precision: str, group: str = "single"):
    """HBM bytes per working launch of `kernel` on `workload` in `precision`
    (fp64 / mixed) from the committed rocprofv3 counter summary
    profiles/traffic_<kernel>_<workload>_<precision>.txt, or None when no such
    summary exists or it was taken on other kernel sources."""
    path = traffic_file(kernel, workload, precision)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_hash(group):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline_of(dom: dict, kernel: str, traffic_bytes, extra=None) -> dict:
    """Roofline object of the dominant kernel from its HIP-event timing:
    achieved = algorithmic bytes per launch (the layout the kernel reads) /
    average launch time; csr_model = the same launches under the paper's CSR
    byte model (4-byte column indices, unfused vector operands); traffic =
    counter-measured HBM bytes per launch (null if not measured for this
    kernel, workload, precision and source)."""
    cnt = max(dom["count"], 1)
    avg_s = dom["ms"] / cnt * 1e-3
    bpl = dom["bytes"] / cnt
    bcsr = dom.get("bytes_csr", dom["bytes"]) / cnt
    ach = bpl / avg_s / 1e9 if dom["count"] else 0.0
    ach_csr = bcsr / avg_s / 1e9 if dom["count"] else 0.0
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic_bytes,
           "kernel": kernel, "launches": dom["count"], "avg_us": round(avg_s * 1e6, 2),
           "algorithmic_bytes_per_launch": round(bpl),
           "csr_model": {"bytes_per_launch": round(bcsr), "achieved": round(ach_csr, 1),
                         "frac": round(ach_csr / PEAK_HBM_GBS, 4)}}
    if traffic_bytes and dom["count"]:
        out["traffic_GBps"] = round(traffic_bytes / avg_s / 1e9, 1)
        out["traffic_frac"] = round(traffic_bytes / avg_s / 1e9 / PEAK_HBM_GBS, 4)
        out["traffic_over_algorithmic"] = round(traffic_bytes / bpl, 3)
    if extra:
        out.update(extra)
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_side: int, threads: int, single_n: int = 32):
    """The oracle on the host: all threads on the n_side^3 cube, and one
    thread on a smaller cube (the paper's single-core comparison axis)."""
    import numpy as np  # noqa: F401
    import oracle
    from paper_1506_08435_amd import workloads as W
    if threads > 0:
        oracle.set_num_threads(threads)
    # a full-size run takes minutes: the oracle reports its own progress
    oracle.set_progress(30.0 if n_side >= 96 else 0.0)
    p = W.cube3d(n_side)
    S = oracle.assemble(p)
    r = oracle.solve(S, tol=1e-8)
    nthr = oracle.num_threads()
    out = {"value": S.n / r.seconds, "unit": "DOF/s", "cores": nthr, "kind": "oracle",
           "sample": (f"oracle GPCG + face solve, tol 1e-8, on the same workload at {n_side}^3 cells "
                      f"({S.n} free DOF)" + (" instead of 128^3" if n_side != 128 else "")
                      + f": {r.seconds:.2f} s"),
           "seconds": r.seconds, "cpu_model": cpu_model(),
           "affinity_cores": len(os.sched_getaffinity(0))}
    if single_n > 0:
        oracle.set_num_threads(1)
        S1 = oracle.assemble(W.cube3d(single_n))
        r1 = oracle.solve(S1, tol=1e-8)
        oracle.set_num_threads(nthr)
        out["single_thread"] = {"value": S1.n / r1.seconds, "unit": "DOF/s", "cores": 1,
                                "sample": f"{single_n}^3 cells ({S1.n} free DOF): {r1.seconds:.2f} s"}
    return out


def recorded_cpu_baseline(n_side: int = 128):
    """The oracle's full-size run on the same host type, as recorded in
    profiles/oracle_cube3d_<n>.txt by `bench.py --workload cpu --cpu-n <n>`
    (minutes of CPU time, so it is not repeated inside every bench run), or
    None when no record exists."""
    path = os.path.join(ROOT, "profiles", f"oracle_cube3d_{n_side}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    try:
        return {"value": float(vals["dof_per_s"]), "unit": "DOF/s", "cores": int(vals["threads"]),
                "kind": "oracle", "recorded": True, "seconds": float(vals["seconds"]),
                "sample": f"oracle GPCG + face solve, tol 1e-8, the full {n_side}^3 workload "
                          f"({vals['free_dof']} free DOF), recorded in profiles/oracle_cube3d_{n_side}.txt"}
    except (KeyError, ValueError):
        return None


def run_cpu(args):
    """Only the CPU oracle on the cube workload (no GPU work)."""
    out = cpu_baseline(args.cpu_n, int(os.environ.get("OMP_NUM_THREADS", "0") or 0), single_n=0)
    return {"metric": "oracle solved DOF/s on the host cores", "workload": f"cube3d_{args.cpu_n}",
            "n_gpus": 0, "cpu_baseline": out}


def triad_gbs(torch) -> float:
    """Achievable HBM bandwidth: a = b + s c on 3 x 512 MiB float64 vectors,
    median of 10 launches timed with events (bytes: 2 reads + 1 write)."""
    n = 64 << 20
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.ones(n, dtype=torch.float64, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ts = []
    for _ in range(12):
        ev[0].record()
        torch.add(b, c, alpha=0.5, out=a)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    del a, b, c
    ts = sorted(ts[2:])
    return 24.0 * n / (ts[len(ts) // 2] * 1e-3) / 1e9


def run_small(args):
    """The 64x64 2D workload (3,969 free DOF): launch-bound, so latency per
    solve (median of many) and DOF/s, FP64 and mixed."""
    import torch
    from paper_1506_08435_amd import nnqp, workloads as W
    p = W.config_small()
    ctx = nnqp.Context(0)
    K, F, _ = ctx.assemble(p)
    out = {}
    for prec_name in ("fp64", "mixed"):
        prec = nnqp.NN_MIXED if prec_name == "mixed" else nnqp.NN_FP64
        opts = nnqp.default_opts(tol=1e-8, inner_rtol=args.inner_rtol, precision=prec,
                                 subspace=args.subspace,
                                 engine=args.engine if prec == nnqp.NN_FP64 else min(args.engine, 1))
        c = torch.empty(K.n, dtype=torch.float64, device=ctx.device)
        for _ in range(3):
            ctx.solve_nonneg(K, F, opts=opts, c=c)
        lat = []
        for _ in range(args.small_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, st = ctx.solve_nonneg(K, F, opts=opts, c=c)
            lat.append(time.perf_counter() - t0)
        lat.sort()
        med = lat[len(lat) // 2]
        out[prec_name] = {"value": round(K.n / med, 1), "unit": "DOF/s",
                          "median_latency_ms": round(med * 1e3, 3),
                          "p99_latency_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))] * 1e3, 3),
                          "kkt_rel": st["kkt_rel"], "outer_its": st["outer_its"], "cg_its": st["cg_its"]}
    line = {"metric": "solve latency and DOF/s, small 2D problem (launch-bound)",
            "workload": f"square2d_64: 64^2 cells x 2 triangles, {K.n} free DOF, {K.nnz} nnz, "
                        f"D = R(pi/6) diag(1, 1e-3) R^T, f = 1 on [3/8,5/8]^2, KKT tol 1e-8, "
                        f"{args.small_reps} solves",
            "n_gpus": 1, **out}
    return line


def run_hole(args):
    """The structured cube-with-hole stand-in (Sec. 5.1): 9k cells per side,
    c = 0 outside, c = 1 on the hole, f = 0, dispersion tensor of v = (1,1,1),
    bounds [0, 1] (the DMP variant).  Times K bounded solves (DOF/s), then the
    Galerkin baseline on the same system with its DMP statistics (Table
    Tab:S5_cube_dmp) and the time ratio (Tables Tab:S5_cube_times_*)."""
    import torch
    from paper_1506_08435_amd import nnqp, workloads as W
    p = W.cube_hole(args.hole_k)
    ctx = nnqp.Context(0)
    K, F, _ = ctx.assemble(p)
    n = K.n
    prec = nnqp.NN_MIXED if args.precision == "mixed" else nnqp.NN_FP64
    opts = nnqp.default_opts(tol=1e-8, inner_rtol=args.inner_rtol, precision=prec,
                             lower=0.0, upper=1.0, precond_degree=args.precond_degree,
                             subspace=args.subspace)
    c = torch.empty(n, dtype=torch.float64, device=ctx.device)
    act = torch.empty(n, dtype=torch.uint8, device=ctx.device)
    for _ in range(args.warmup):
        ctx.solve_nonneg(K, F, opts=opts, c=c, active=act)
    ctx.set_profiling(not args.no_kernel_timing, ("cg_spmv",), every=args.time_every)
    ctx.kernel_times(reset=True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, st = ctx.solve_nonneg(K, F, opts=opts, c=c, active=act)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.kernel_times(reset=True)
    ctx.set_profiling(False)
    dom = kt["cg_spmv"]
    avg_ms = dom["ms"] / max(dom["count"], 1)
    bpl = dom["bytes"] / max(dom["count"], 1)
    achieved = bpl / (avg_ms * 1e-3) / 1e9 if dom["count"] else 0.0
    at_lo = int((act[:n] == 1).sum().item())
    at_hi = int((act[:n] == 2).sum().item())
    gopts = nnqp.default_opts(tol=1e-8, max_cg=200000)
    ctx.solve_galerkin(K, F, opts=gopts)
    gal = [ctx.solve_galerkin(K, F, opts=gopts) for _ in range(args.galerkin_reps)]
    g_med = sorted(g[1]["seconds"] for g in gal)[len(gal) // 2]
    gc, gst = gal[-1]
    over = int((gc > 1.0).sum().item())
    nn_med = sorted(x["seconds"] for x in stats)[len(stats) // 2]
    gal_block = {"median_device_ms": round(g_med * 1e3, 3)}
    blmvm = None if args.no_blmvm or prec != nnqp.NN_FP64 else \
        run_blmvm(ctx, K, F, n, stats, gal_block, args, bounds=(0.0, 1.0))
    line = {
        "metric": "solved DOF/s at KKT tol 1e-8, bounds [0, 1]",
        "value": round(n * args.steps / wall, 1), "unit": "DOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "dtype": "f64" if prec == nnqp.NN_FP64 else "f32 values+CG vectors / f64 residual",
        "data": "synthetic",
        "config": {"workload": f"cube_hole_k{args.hole_k}: [0,1]^3 minus [4/9,5/9]^3, "
                               f"{9 * args.hole_k}^3 cells x 6 P1 tets (hole removed), {n} free DOF, "
                               f"{K.nnz} nnz, c = 0 outside / 1 on the hole (lifted), f = 0, "
                               f"D = dispersion(v = (1,1,1), alpha_L = 1, alpha_T = 1e-3), "
                               f"bounds [0, 1], from c0 = 1e-8 to KKT tol 1e-8",
                   "inner_rtol": args.inner_rtol, "precond_degree": args.precond_degree},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": "k_cg_spmv", "launches": dom["count"],
                     "avg_us": round(avg_ms * 1e3, 2), "algorithmic_bytes_per_launch": round(bpl)},
        "solve": {"median_device_ms": round(nn_med * 1e3, 3), "outer_its": stats[-1]["outer_its"],
                  "cg_its": stats[-1]["cg_its"], "kkt_rel": stats[-1]["kkt_rel"],
                  "min_c": stats[-1]["min_c"], "nodes_at_0": at_lo, "nodes_at_1": at_hi},
        "galerkin": {"median_device_ms": round(g_med * 1e3, 3), "cg_its": gst["cg_its"],
                     "residual_rel": gst["kkt_rel"], "min_c": gst["min_c"], "max_c": gst["max_c"],
                     "negative_nodes": gst["n_negative"], "nodes_above_1": over,
                     "pct_violating": round(100.0 * (gst["n_negative"] + over) / max(n, 1), 2),
                     "bounded_over_galerkin_time": round(nn_med / g_med, 3)},
    }
    if blmvm is not None:
        line["blmvm"] = blmvm
        line["tron_levels"] = run_tron_levels(ctx, K, F, args, bounds=(0.0, 1.0))
    line["paper_context"] = paper_context()
    print(json.dumps(line), flush=True)


def run_transient(args):
    """50 backward-Euler steps of the 256x256x64 heterogeneous workload (warm
    started, K~ = M/dt + K formed once); value = free DOF x steps / second."""
    import torch
    from paper_1506_08435_amd import nnqp, workloads as W
    p = W.config_transient3d(*args.tdims)
    ctx = nnqp.Context(0)
    K, F, _ = ctx.assemble(p, with_mass=True)
    n = K.n
    out, finals = {}, {}
    for prec_name in ("fp64", "mixed"):
        prec = nnqp.NN_MIXED if prec_name == "mixed" else nnqp.NN_FP64
        opts = nnqp.default_opts(tol=1e-8, inner_rtol=args.inner_rtol, precision=prec,
                                 precond_degree=args.precond_degree, subspace=args.subspace,
                                 cg_chunk=args.cg_chunk)
        c = torch.zeros(n, dtype=torch.float64, device=ctx.device)
        ctx.step_transient(K, args.dt, F, c, opts=opts)          # warm-up (forms K~)
        c.zero_()
        ctx.set_profiling(not args.no_kernel_timing, None if args.profile_all else ("cg_spmv",),
                    every=args.time_every)
        ctx.kernel_times(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_step = []
        for _ in range(args.tsteps):
            _, _, st = ctx.step_transient(K, args.dt, F, c, opts=opts)
            per_step.append(st)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = ctx.kernel_times(reset=True)
        ctx.set_profiling(False)
        dom = kt["cg_spmv"]
        wl = "transient3d_" + "x".join(map(str, args.tdims))
        out[prec_name] = {
            "value": round(n * args.tsteps / wall, 1), "unit": "DOF*steps/s",
            "ms_per_step": round(wall / args.tsteps * 1e3, 3),
            "max_kkt_rel": max(s["kkt_rel"] for s in per_step),
            "outer_its_total": sum(s["outer_its"] for s in per_step),
            "cg_its_total": sum(s["cg_its"] for s in per_step),
            "final_max_c": float(c.max()), "final_active": int(per_step[-1]["n_active"]),
            "roofline": roofline_of(dom, "k_cg_spmv", read_traffic("k_cg_spmv", wl, prec_name),
                                    {"timed_one_launch_in": args.time_every})}
        finals[prec_name] = c.clone()
    line = {"metric": "solved DOF*steps/s, backward Euler, KKT tol 1e-8 per step",
            "workload": f"transient3d_{'x'.join(map(str, args.tdims))}: {n} free DOF, {K.nnz} nnz, "
                        f"D = exp(G) R diag(1,.1,1e-3) R^T (Gaussian random field, seed 1506), "
                        f"dt = {args.dt}, {args.tsteps} steps from c0 = 0, warm-started",
            "precond": "Jacobi" if args.precond_degree <= 1 else
                       f"Chebyshev-Jacobi degree {args.precond_degree}",
            "n_gpus": 1, **out}
    # the mixed-precision end state against the float64 one (both at KKT 1e-8)
    a, b = finals["mixed"], finals["fp64"]
    line["mixed_vs_fp64_rel_diff"] = float((a - b).abs().max() / b.abs().max())
    line["active_nodes_fp64_mixed"] = [out["fp64"]["final_active"], out["mixed"]["final_active"]]
    line["active_note"] = ("the two end states differ in which degenerate nodes (c = 0 with "
                           "g = 0 up to the 1e-8 tolerance) sit exactly at zero")
    return line


def run_batch(args):
    """The 512-member batch of 2D problems (grid sides U{32..256}, random
    theta, anisotropy and source square; seed 8435) solved by one batched call
    per step, FP64 and mixed; value = free DOF of all members / second."""
    import torch
    from paper_1506_08435_amd import nnqp, workloads as W
    probs = [W.batch_problem(i) for i in range(args.nbatch)]
    ctx = nnqp.Context(0)
    Ks, Fs = [], []
    for p in probs:
        K, F, _ = ctx.assemble(p)
        Ks.append(K)
        Fs.append(F)
    ndof = sum(K.n for K in Ks)
    nnz = sum(K.nnz for K in Ks)
    out = {}
    for prec_name in ("fp64", "mixed"):
        prec = nnqp.NN_MIXED if prec_name == "mixed" else nnqp.NN_FP64
        opts = nnqp.default_opts(tol=1e-8, inner_rtol=args.inner_rtol, precision=prec,
                                 verbose=int(args.verbose))
        cs = [torch.empty(max(K.n, 1), dtype=torch.float64, device=ctx.device) for K in Ks]
        bsteps = args.batch_steps
        for _ in range(max(args.warmup, 1)):
            ctx.solve_batch(Ks, Fs, opts=opts, cs=cs)      # also tunes the launch shape
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(bsteps):
            _, _, stats, _ = ctx.solve_batch(Ks, Fs, opts=opts, cs=cs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # Kernel timing needs events between launches, which the captured CG
        # graphs do not carry: one more solve with profiling on (CG launches
        # enqueued one by one, each bracketed by events) gives the roofline.
        kt = {k: {"count": 0, "ms": 0.0, "bytes": 0.0} for k in nnqp.KCLASS_NAMES}
        if not args.no_kernel_timing:
            ctx.set_profiling(True)
            ctx.kernel_times(reset=True)
            ctx.solve_batch(Ks, Fs, opts=opts, cs=cs)
            kt = ctx.kernel_times(reset=True)
            ctx.set_profiling(False)
        dom = kt["cg_spmv"]
        out[prec_name] = {
            "value": round(ndof * bsteps / wall, 1), "unit": "DOF/s",
            "ms_per_step": round(wall / bsteps * 1e3, 3),
            "max_kkt_rel": max(s["kkt_rel"] for s in stats),
            "max_outer_its": max(s["outer_its"] for s in stats),
            "sum_cg_its": sum(s["cg_its"] for s in stats),
            "roofline": roofline_of(
                dom, "kb_rows (batched row pass: gradient, Cauchy trial, CG matrix pass or search "
                     "trial of each member)",
                read_traffic("kb_rows", f"batch2d_{args.nbatch}", prec_name, group="batch"),
                {"measured_in": "one extra profiled solve, steps launched one by one"}),
            "kernel_classes": {k: {"count": v["count"],
                                   "avg_us": round(v["ms"] / max(v["count"], 1) * 1e3, 2)}
                               for k, v in kt.items()}}
    line = {"metric": "solved DOF/s at KKT tol 1e-8 (batch of independent QPs)",
            "workload": f"batch2d_{args.nbatch}: {args.nbatch} 2D problems, grid side U{{32..256}}, "
                        f"theta U[0,pi), ratio 10^-U(1,4), f = 1 on a random square; {ndof} free DOF, "
                        f"{nnz} nnz in total; one nn_solve_batch call per step",
            "n_gpus": 1, "steps": args.batch_steps, "warmup": max(args.warmup, 1), **out}
    if not args.no_cpu_baseline:
        import oracle
        S_list = [oracle.assemble(probs[k]) for k in range(args.cpu_members)]
        t0 = time.perf_counter()
        for S in S_list:
            oracle.solve(S, tol=1e-8)
        sec = time.perf_counter() - t0
        nd = sum(S.n for S in S_list)
        line["cpu_baseline"] = {"value": round(nd / sec, 1), "unit": "DOF/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"oracle GPCG, tol 1e-8, on members 0..{args.cpu_members - 1} "
                                          f"of the batch ({nd} DOF): {sec:.2f} s"}
    return line


def run_serve(args, rates=None):
    """Continuous-batching server on a Poisson stream of transient requests
    (2D/3D 50/50, free DOF log-uniform in [1e3, 1e6], 10 backward-Euler steps
    each, dt = 1e-3, KKT tol 1e-8 per step), FP64 and mixed precision on the
    same stream; p50/p99 latency (arrival to last step) and DOF*steps/s, and
    the mixed end state of every request against its FP64 end state."""
    import numpy as np
    from paper_1506_08435_amd import nnqp, workloads as W
    from paper_1506_08435_amd.serve import Request, Server
    rates = args.rates if rates is None else rates
    problems = [W.serve_problem(k, seed=args.serve_seed) for k in range(args.nreq)]
    dofs = [p.n_free for p in problems]
    out = {}
    budget = int(args.hbm_budget_gib * (1 << 30)) if args.hbm_budget_gib > 0 else None
    for rate in rates:
        arrivals = W.serve_arrivals(args.nreq, rate, seed=args.serve_seed)
        reqs = [Request(k, problems[k], args.serve_steps, float(arrivals[k])) for k in range(args.nreq)]
        finals = {}
        for prec_name in ("fp64", "mixed"):
            prec = nnqp.NN_MIXED if prec_name == "mixed" else nnqp.NN_FP64
            srv = Server(precision=prec, hbm_budget=budget, tol=1e-8, inner_rtol=args.serve_inner_rtol,
                         lane_bounds=tuple(args.serve_lanes), solo_lanes=args.serve_solo_lanes,
                         keep_states=True, subspace=args.subspace)
            rep = srv.run(reqs)
            sm = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.summary().items()}
            sm["max_kkt_rel"] = max(s["kkt_rel"] for r in rep.results for s in r.step_stats)
            out[f"rate{rate:g}_{prec_name}"] = sm
            finals[prec_name] = {r.rid: r.c for r in rep.results if r.status == 0}
        diffs = []
        for rid, c64 in finals["fp64"].items():
            cm = finals["mixed"].get(rid)
            if cm is not None and c64 is not None:
                diffs.append(float((cm - c64).abs().max() / max(float(c64.abs().max()), 1e-300)))
        if diffs:
            out[f"rate{rate:g}_mixed_vs_fp64"] = {
                "requests": len(diffs), "max_rel_diff": max(diffs),
                "p99_rel_diff": float(np.percentile(diffs, 99)),
                "note": "per request: ||c_mixed - c_fp64||_inf / ||c_fp64||_inf of the end "
                        "states, both at KKT tol 1e-8 per step"}
    line = {"metric": "served transient requests: p50/p99 latency and solved DOF*steps/s",
            "workload": f"serve: {args.nreq} requests per rate, Poisson arrivals at {list(rates)} per s, "
                        f"2D/3D 50/50, free DOF log-uniform in [1e3, 1e6] (here {min(dofs)}..{max(dofs)}, "
                        f"total {sum(dofs)}), {args.serve_steps} backward-Euler steps each, dt = 1e-3, "
                        f"seed {args.serve_seed}; size lanes split at {list(args.serve_lanes)} free DOF, "
                        f"the top {args.serve_solo_lanes} stepped by the single-problem solver",
            "n_gpus": 1, **out}
    if not args.no_cpu_baseline:
        import oracle
        sample = [p for p in problems if p.n_free <= 60000][:args.cpu_members]
        t0 = time.perf_counter()
        ds = 0
        for pr in sample:
            S = oracle.assemble(pr, with_mass=True)
            c = np.zeros(S.n)
            for _ in range(args.serve_steps):
                c = oracle.transient_step(S, 1e-3, c, tol=1e-8).c
            ds += S.n * args.serve_steps
        sec = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(ds / sec, 1), "unit": "DOF*steps/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"oracle assembly + {args.serve_steps} steps of the first "
                                          f"{len(sample)} requests with at most 60000 DOF, one after "
                                          f"another: {sec:.2f} s"}
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="cells per side of the cube workload")
    ap.add_argument("--inner-rtol", type=float, default=0.5,
                    help="relative tolerance of each inner CG solve (does not change the minimiser)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--subspace", type=int, choices=[0, 1], default=0,
                    help="TRON's subspace loop (1) or a Cauchy step every iteration (0, the "
                         "library default); the minimiser is the same")
    ap.add_argument("--cg-chunk", type=int, default=16,
                    help="CG iterations between convergence reads (0: adaptive first chunk)")
    ap.add_argument("--engine", type=int, choices=[0, 1, 2], default=0,
                    help="single-problem solves: 0 = by size (one workgroup up to 4,096 rows), "
                         "1 = multi-block passes, 2 = one workgroup")
    ap.add_argument("--precond-degree", type=int, default=1,
                    help="inner CG preconditioner: 1 = Jacobi, k > 1 = Chebyshev of degree k")
    ap.add_argument("--cpu-n", type=int, default=64, help="cube side of the CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--time-every", type=int, default=16,
                    help="inside timed regions, time one CG launch in this many (the passes of a "
                         "solve have one size; 1: every launch)")
    ap.add_argument("--profile-all", action="store_true",
                    help="time every kernel class inside the timed region (default: the CG matrix pass only)")
    ap.add_argument("--verbose", action="store_true", help="per-outer-iteration trace on stderr")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run three 512 MiB device-to-device copies first (reference for HBM counters)")
    ap.add_argument("--workload", choices=["cube", "small", "transient", "batch", "serve", "hole", "cpu"],
                    default="cube")
    ap.add_argument("--hole-k", type=int, default=14,
                    help="cube-with-hole workload: 9k cells per side (k = 14: about 2M DOF)")
    ap.add_argument("--small-reps", type=int, default=50, help="solves timed by the small workload")
    ap.add_argument("--no-galerkin", action="store_true",
                    help="skip the unconstrained Galerkin baseline solve (cube workload)")
    ap.add_argument("--galerkin-reps", type=int, default=3)
    ap.add_argument("--no-blmvm", action="store_true",
                    help="skip the BLMVM comparison solves (cube and hole workloads)")
    ap.add_argument("--blmvm-reps", type=int, default=3)
    ap.add_argument("--no-triad", action="store_true",
                    help="skip the achievable-bandwidth (triad) reference")
    ap.add_argument("--nreq", type=int, default=32, help="requests of the serve workload")
    ap.add_argument("--rates", type=float, nargs="+", default=[50.0, 500.0, 2000.0],
                    help="arrival rates (requests/s) of the serve workload")
    ap.add_argument("--serve-steps", type=int, default=10)
    ap.add_argument("--serve-seed", type=int, default=2015)
    ap.add_argument("--serve-inner-rtol", type=float, default=0.1,
                    help="inner CG tolerance of the served solves (TRON1)")
    ap.add_argument("--serve-lanes", type=float, nargs="*", default=[30000, 300000],
                    help="free-DOF bounds between the server's size lanes (none: one lane)")
    ap.add_argument("--serve-solo-lanes", type=int, default=2,
                    help="top lanes that step requests with the single-problem solver")
    ap.add_argument("--hbm-budget-gib", type=float, default=0.0,
                    help="server HBM budget (0: 3/4 of the free device memory)")
    ap.add_argument("--nbatch", type=int, default=512, help="members of the batch workload")
    ap.add_argument("--cpu-members", type=int, default=16,
                    help="batch members the CPU-baseline sample solves")
    ap.add_argument("--extras", nargs="*", default=list(EXTRAS),
                    choices=list(EXTRAS),
                    help="sections the cube workload's line carries besides the FP64 cube "
                         "(default: all)")
    ap.add_argument("--no-extras", action="store_true", help="the same as --extras with no name")
    ap.add_argument("--extra-rates", type=float, nargs="+", default=[500.0],
                    help="arrival rates of the serve section of the default line")
    ap.add_argument("--batch-steps", type=int, default=2, help="timed calls of the batch workload")
    ap.add_argument("--tdims", type=int, nargs=3, default=[256, 256, 64])
    ap.add_argument("--tsteps", type=int, default=50)
    ap.add_argument("--dt", type=float, default=1e-3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        # three 512 MiB device-to-device copies: the reference that scales the
        # HBM counters (FETCH_SIZE, WRITE_SIZE) of a profiled run to bytes
        import torch
        a = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    single = {"transient": run_transient, "batch": run_batch, "serve": run_serve,
              "small": run_small, "hole": run_hole, "cpu": run_cpu}
    if args.workload in single:
        line = single[args.workload](args)
        if line is not None:
            print(json.dumps(line), flush=True)
        return

    import torch
    from paper_1506_08435_amd import nnqp, workloads as W

    p = W.cube3d(args.n)
    ctx = nnqp.Context(0)
    K, F, _ = ctx.assemble(p)
    n = K.n
    prec = nnqp.NN_MIXED if args.precision == "mixed" else nnqp.NN_FP64
    opts = nnqp.default_opts(tol=1e-8, inner_rtol=args.inner_rtol, verbose=int(args.verbose),
                             precision=prec, precond_degree=args.precond_degree,
                             subspace=args.subspace, cg_chunk=args.cg_chunk)
    c = torch.empty(n, dtype=torch.float64, device=ctx.device)
    for _ in range(args.warmup):
        ctx.solve_nonneg(K, F, opts=opts, c=c)
    # only the dominant kernel is bracketed by events unless asked otherwise:
    # fewer events, less perturbation of the timed solves
    ctx.set_profiling(not args.no_kernel_timing, None if args.profile_all else ("cg_spmv",),
                    every=args.time_every)
    ctx.kernel_times(reset=True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, st = ctx.solve_nonneg(K, F, opts=opts, c=c)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = ctx.kernel_times(reset=True)
    ctx.set_profiling(False)
    wall = t1 - t0
    ms_per_step = wall / args.steps * 1e3
    value = n * args.steps / wall

    dom = kt["cg_spmv"]
    wl = f"cube3d_{args.n}"
    roofline = roofline_of(dom, "k_cg_spmv (CG matrix pass with fused direction update)",
                           read_traffic("k_cg_spmv", wl, args.precision),
                           {"timed_one_launch_in": args.time_every})
    if not args.no_triad:
        tri = triad_gbs(torch)
        roofline["achievable_triad_GBps"] = round(tri, 1)
        roofline["frac_of_achievable"] = round(roofline["achieved"] / tri, 4)
    galerkin = None
    if not args.no_galerkin and prec == nnqp.NN_FP64:
        galerkin = run_galerkin(ctx, K, F, n, stats, args)
    blmvm = None
    if not args.no_blmvm and prec == nnqp.NN_FP64:
        blmvm = run_blmvm(ctx, K, F, n, stats, galerkin, args)

    out = {
        "metric": "solved DOF/s at KKT tol 1e-8",
        "value": round(value, 1),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == nnqp.NN_FP64 else "f32 values+CG vectors / f64 residual",
        "data": "synthetic",
        "config": {"workload": f"cube3d_{args.n}: {args.n}^3 cells x 6 P1 tets, {n} free DOF, "
                               f"{K.nnz} nnz, D = R diag(1,1e-2,1e-4) R^T, f = 1 on central cube, "
                               + ("FP64 plain solve" if prec == nnqp.NN_FP64 else "mixed-precision solve")
                               + " from c0 = 1e-8 to KKT tol 1e-8",
                   "inner_rtol": args.inner_rtol, "solver": "TRON-style active-set Newton-CG",
                   "precond": "Jacobi" if args.precond_degree <= 1 else
                              f"Chebyshev-Jacobi degree {args.precond_degree}"},
        "roofline": roofline,
        "solve": {"median_device_ms": round(1e3 * sorted(x["seconds"] for x in stats)[len(stats) // 2], 3),
                  "outer_its": stats[-1]["outer_its"], "cg_its": stats[-1]["cg_its"],
                  "spmvs": stats[-1]["spmvs"], "kkt_rel": stats[-1]["kkt_rel"],
                  "device_s": round(stats[-1]["seconds"], 4),
                  "algorithmic_GBps_whole_solve": round(stats[-1]["bytes_moved"] / stats[-1]["seconds"] / 1e9, 1),
                  "kernel_classes": {k: {"count": v["count"],
                                         "avg_us": round(v["ms"] / max(v["count"], 1) * 1e3, 2)}
                                     for k, v in kt.items() if v["count"]}},
    }
    if galerkin is not None:
        out["galerkin"] = galerkin
    if blmvm is not None:
        out["blmvm"] = blmvm
    if not args.no_blmvm and prec == nnqp.NN_FP64:
        out["tron_levels"] = run_tron_levels(ctx, K, F, args)
    extras = [] if args.no_extras else args.extras
    if "mixed" in extras and prec == nnqp.NN_FP64:
        out["mixed"] = run_cube_mixed(ctx, K, F, c, args)
    K.free()
    del ctx
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, int(os.environ.get("OMP_NUM_THREADS", "0") or 0))
        full = recorded_cpu_baseline(args.n)
        if full is not None:
            out["cpu_baseline"]["full_size_recorded"] = full
    out["paper_context"] = paper_context()
    # the other workloads of the metric, each in its own section: the small
    # 2D solve (latency), the heterogeneous transient run, the 512-member
    # batch and the served stream (p50/p99), FP64 and mixed precision
    sub_args = argparse.Namespace(**vars(args))
    sub_args.no_cpu_baseline = True
    for key, fn in (("small", run_small), ("transient", run_transient),
                    ("batch", run_batch), ("serve", run_serve)):
        if key not in extras:
            continue
        t0 = time.perf_counter()
        sec = fn(sub_args, rates=args.extra_rates) if fn is run_serve else fn(sub_args)
        sec["section_wall_s"] = round(time.perf_counter() - t0, 1)
        out[key] = sec
        print(f"bench: {key} section done in {sec['section_wall_s']} s", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


def run_cube_mixed(ctx, K, F, c, args):
    """The same system in mixed precision (float32 values and CG vectors,
    float64 residual): DOF/s over `steps` solves, its CG-pass roofline and
    the end state against the float64 one."""
    import torch
    from paper_1506_08435_amd import nnqp
    c64 = c.clone()
    opts = nnqp.default_opts(tol=1e-8, inner_rtol=args.inner_rtol, precision=nnqp.NN_MIXED,
                             subspace=args.subspace, cg_chunk=args.cg_chunk)
    cm = torch.empty_like(c)
    ctx.solve_nonneg(K, F, opts=opts, c=cm)              # warm-up (forms the float32 copies)
    ctx.set_profiling(not args.no_kernel_timing, ("cg_spmv",), every=args.time_every)
    ctx.kernel_times(reset=True)
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, st = ctx.solve_nonneg(K, F, opts=opts, c=cm)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.kernel_times(reset=True)
    ctx.set_profiling(False)
    return {"value": round(K.n * args.steps / wall, 1), "unit": "DOF/s",
            "ms_per_step": round(wall / args.steps * 1e3, 3),
            "dtype": "f32 values+CG vectors / f64 residual",
            "outer_its": stats[-1]["outer_its"], "cg_its": stats[-1]["cg_its"],
            "kkt_rel": stats[-1]["kkt_rel"],
            "rel_diff_vs_fp64": float((cm - c64).abs().max() / c64.abs().max()),
            "roofline": roofline_of(kt["cg_spmv"], "k_cg_spmv (float32 values and vectors)",
                                    read_traffic("k_cg_spmv", f"cube3d_{args.n}", "mixed"),
                                    {"timed_one_launch_in": args.time_every})}


def run_galerkin(ctx, K, F, n, stats, args):
    """The unconstrained Galerkin baseline on the same system (Jacobi-PCG to
    ||K c - f|| <= 1e-8 ||f||): its time, the DMP statistics of its solution
    (Table Tab:S5_cube_dmp) and the time ratio of the non-negative solve to
    it (Tables Tab:S5_cube_times_mustang/wolf compare the same two)."""
    from paper_1506_08435_amd import nnqp
    opts = nnqp.default_opts(tol=1e-8, max_cg=200000)
    ctx.solve_galerkin(K, F, opts=opts)               # warm-up
    runs = [ctx.solve_galerkin(K, F, opts=opts)[1] for _ in range(args.galerkin_reps)]
    g_med = sorted(r["seconds"] for r in runs)[len(runs) // 2]
    nn_med = sorted(x["seconds"] for x in stats)[len(stats) // 2]
    r = runs[-1]
    return {"median_device_ms": round(g_med * 1e3, 3), "cg_its": r["cg_its"],
            "residual_rel": r["kkt_rel"], "min_c": r["min_c"], "max_c": r["max_c"],
            "negative_nodes": r["n_negative"],
            "pct_negative": round(100.0 * r["n_negative"] / max(n, 1), 2),
            "algorithmic_GBps": round(r["bytes_moved"] / r["seconds"] / 1e9, 1),
            "nonneg_over_galerkin_time": round(nn_med / g_med, 3),
            "nonneg_min_c": stats[-1]["min_c"]}


def run_tron_levels(ctx, K, F, args, bounds=(0.0, float("inf"))):
    """TRON with the paper's three inner CG tolerances (TRON1/2/3: 1e-1, 1e-2,
    1e-3, Sec. 5.1), median device time of a few solves each: the TRON columns
    of Tables Tab:S5_cube_times_mustang/wolf."""
    from paper_1506_08435_amd import nnqp
    out = {}
    for name, rtol in (("tron1", 1e-1), ("tron2", 1e-2), ("tron3", 1e-3)):
        opts = nnqp.default_opts(tol=1e-8, inner_rtol=rtol, lower=bounds[0], upper=bounds[1])
        ctx.solve_nonneg(K, F, opts=opts)
        runs = [ctx.solve_nonneg(K, F, opts=opts)[2] for _ in range(args.blmvm_reps)]
        r = runs[-1]
        out[name] = {"median_device_ms": round(sorted(x["seconds"] for x in runs)[len(runs) // 2] * 1e3, 3),
                     "outer_its": r["outer_its"], "cg_its": r["cg_its"]}
    return out


def run_blmvm(ctx, K, F, n, stats, galerkin, args, bounds=(0.0, float("inf"))):
    """The paper's second bound-constrained solver on the same system, to the
    same tolerance: median time of a few solves, iterations, and its time
    relative to TRON and to the Galerkin solve (the columns of Tables
    Tab:S5_cube_times_mustang/wolf)."""
    from paper_1506_08435_amd import nnqp
    opts = nnqp.default_opts(tol=1e-8, method=nnqp.NN_BLMVM, lower=bounds[0], upper=bounds[1])
    ctx.solve_nonneg(K, F, opts=opts)                 # warm-up
    runs = [ctx.solve_nonneg(K, F, opts=opts)[2] for _ in range(args.blmvm_reps)]
    med = sorted(r["seconds"] for r in runs)[len(runs) // 2]
    nn_med = sorted(x["seconds"] for x in stats)[len(stats) // 2]
    r = runs[-1]
    out = {"median_device_ms": round(med * 1e3, 3), "iterations": r["outer_its"],
           "line_search_trials": r["search_trials"], "memory_resets": r["refinements"],
           "kkt_rel": r["kkt_rel"], "dof_per_s": round(n / med, 1),
           "algorithmic_GBps": round(r["bytes_moved"] / r["seconds"] / 1e9, 1),
           "blmvm_over_tron_time": round(med / nn_med, 3)}
    if galerkin is not None:
        out["blmvm_over_galerkin_time"] = round(med * 1e3 / galerkin["median_device_ms"], 3)
    return out


if __name__ == "__main__":
    main()
