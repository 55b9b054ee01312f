#!/usr/bin/env python3
"""Benchmark of the randomized-preconditioned SC-4DVAR hot path on one MI355X.

Workload (N=1): burgers-4096 -- periodic Burgers, n = 4096, 500 RK4 steps,
observations every 16th point every 25 steps (m = 5120), Gaussian prior,
FP64 throughout.  One timed step is the whole hot path for one assimilation:
3 Gauss-Newton iterations from the background, each = FWD + gradient (ADJ) +
a 64-column Nystrom sketch of the data-misfit Hessian (64 TLM + 64 ADJ sweeps)
+ PCG to relative residual 1e-6 with the limited-memory preconditioner + update.
Inputs are synthesised on the device before timing (x_b = x_true + Gamma^{1/2} xi,
y = O M(x_true) + sigma_o eta from seeded draws).

value = Hessian-vector products per second over the timed steps (sketch columns
plus PCG products, counted by the library), ms_per_step = one assimilation
(3 GN iterations).  The roofline object describes the dominant sweep kernel,
timed with HIP events on the library's stream inside the timed region; the
cpu_baseline object times the FP64 numpy oracle on one GN iteration.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6      # MI355X FP64 vector peak
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E peak
PEAK_FP32_VALU_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sketch", default="nystrom", choices=["nystrom", "randsvd"])
    ap.add_argument("--sketch-dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--gn-iters", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning-cache", default=None, help="JSON tiling cache (default: the package's tuning.json)")
    ap.add_argument("--tune-budget", type=float, default=20.0, help="seconds per tuned shape when not cached")
    ap.add_argument("--no-bve", action="store_true", help="skip the bve-256 section")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch-64 section")
    ap.add_argument("--no-serve", action="store_true", help="skip the serve-mix section")
    ap.add_argument("--no-wall", action="store_true", help="skip the burgers-wall-399 section")
    ap.add_argument("--only", choices=["bve", "batch", "serve", "wall"],
                    help="run this section alone and print its record (for profiling; no headline line)")
    ap.add_argument("--gn-only", action="store_true",
                    help="burgers-4096: only the timed GN steps and the isolated block products (no reuse, "
                         "adaptive or SingleView runs), so that a profile holds the k = ell sweeps alone")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB with a plain elementwise kernel "
                         "(reference dispatch for the HBM byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "burgers_sweep_k64_traffic.json")
# the sources that define the periodic sweep kernels (hashed together, in this order)
SWEEP_SOURCES = [os.path.join(ROOT, "paper_2401_15758_amd", "csrc", f)
                 for f in ("burgers_sweep.hip", "sweep_common.hpp")]
FFT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "bve256_k100_traffic.json")
# the sources that define the 2-D column pass (hashed together, in this order)
FFT_SOURCES = [os.path.join(ROOT, "paper_2401_15758_amd", "csrc", f) for f in ("fft2d.hip", "fft_line.hpp")]


def measured_traffic(kname, tiling, cfg, sources=None, path=None):
    """HBM bytes per launch of a kernel, from the counter runs recorded next to
    the profiles (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain
    copy).  None unless the record is for this kernel source, kernel
    instantiation, tiling and workload."""
    import hashlib
    sources = SWEEP_SOURCES if sources is None else sources
    path = (TRAFFIC_FILE if sources is SWEEP_SOURCES else FFT_TRAFFIC_FILE) if path is None else path
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in sources:
            with open(src, "rb") as f:
                h.update(f.read())
        sha = h.hexdigest()
    except (OSError, ValueError):
        return None
    keys = ("ppt", "kc", "threads", "tile", "steps", "xch")
    for r in rec.get("records", []):
        if (r.get("source_sha256") == sha and r.get("kernel") == kname and r.get("workload") == cfg["name"]
                and all(r.get("tiling", {}).get(k) == tiling.get(k) for k in keys)):
            return r["bytes_per_launch"]
    return None


def bve_section(rp4d, inputs, torch, np, gn=True):
    """bve-256: the 2-D workload.  One FP64 block Hessian product with k = 100,
    timed per kernel class (the column passes of the spectral solves and the
    fused row passes of the RK stages), one k = 1 product (the PCG's) and one
    Gauss-Newton iteration (100-column Nystrom sketch, PCG to 1e-6) from the
    background."""
    cfg = dict(inputs.CFG_BVE)
    ell = cfg["ell"]
    ctx = rp4d.Context(0)
    p = rp4d.Problem(ctx, cfg)
    d = inputs.draws(cfg, seed=0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    xb, y = p.synthesize(dev(d["x_true"]), dev(d["xi"]), dev(d["eta"].reshape(-1)))
    p.set_data(xb, y.reshape(-1))
    tr = p.traj()
    p.fwd(xb, tr, want_J=False)
    V = torch.empty((cfg["n"], ell), dtype=torch.float64, device="cuda")
    ctx.philox_normal(11, V.numel(), V)
    HV = torch.empty_like(V)
    p.hessian_block(tr, V, HV)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    p.hessian_block(tr, V, HV)
    torch.cuda.synchronize()
    hb = time.perf_counter() - t0
    g, sten = ctx.kernel_stats(rp4d.K_SPECTRAL), ctx.kernel_stats(rp4d.K_STENCIL)
    ctx.set_timing(False)
    # single-vector product (the PCG's), median of 5
    v1 = V[:, :1].contiguous()
    hv1 = torch.empty_like(v1)
    p.hessian_block(tr, v1, hv1)
    t1s = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.hessian_block(tr, v1, hv1)
        torch.cuda.synchronize()
        t1s.append(time.perf_counter() - t0)
    hk1 = float(np.median(t1s))
    # column passes of the k = 100 product's spectral solves (one launch per RK
    # stage: the column DFTs, the diagonal and the inverse column DFTs of k/2
    # complex pairs in place): algorithmic traffic the k fields' spectra in and
    # out, 2 k n 8 bytes per launch
    solve_s = g["total_ms"] * 1e-3 / max(1, g["launches"])
    fft_tf = g["alg_flops"] / (g["total_ms"] * 1e-3) / 1e12
    solve_gbs = 2.0 * ell * cfg["n"] * 8 / solve_s / 1e9
    row_tf = sten["alg_flops"] / (sten["total_ms"] * 1e-3) / 1e12 if sten["total_ms"] > 0 else 0.0
    gn_rec = {}
    if gn:
        st = p.gn_state()
        p.reset_counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = p.gn_step(st, sketch=rp4d.NYSTROM, ell=ell, seed=1000, sketch_dtype=rp4d.F64, rtol=1e-6)
        torch.cuda.synchronize()
        gn_s = time.perf_counter() - t0
        gn_rec = {"gn_step_s": gn_s, "pcg_iters": info["pcg_iters"], "hv_per_s": p.counters()["hv_columns"] / gn_s}
        # the configured precision of this workload: FP32 sketch sweeps and the
        # BF16 Gram of the eigendecomposition, FP64 PCG and Hessian products
        ctx.set_gram_precision(rp4d.BF16)
        st2 = p.gn_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info2 = p.gn_step(st2, sketch=rp4d.NYSTROM, ell=ell, seed=1000, sketch_dtype=rp4d.F32, rtol=1e-6,
                          exact_lmp=True)
        torch.cuda.synchronize()
        gn2 = time.perf_counter() - t0
        ctx.set_gram_precision(rp4d.F64)
        gn_rec["configured_precision"] = {"sketch_sweeps": "f32", "gram": "bf16", "pcg": "f64",
                                          "gn_step_s": gn2, "pcg_iters": info2["pcg_iters"],
                                          "pcg_relres": info2["pcg_relres"],
                                          "x_reldiff_vs_f64": float(torch.linalg.norm(st2.get()[1] - st.get()[1])
                                                                    / torch.linalg.norm(st.get()[1]))}
    return {"workload": cfg["name"], "n": cfg["n"], "nsteps": cfg["nsteps"], "k": ell, **gn_rec,
            "hessian_block_k100_ms": 1e3 * hb, "hessian_block_hv_per_s": ell / hb,
            "hessian_k1_ms": 1e3 * hk1, "hessian_k1_hv_per_s": 1.0 / hk1,
            "roofline": {"bound": "hbm",
                         "kernel": "fft_cols<double, 16>: column pass of the stage solves (FP64, k=100)",
                         "achieved": solve_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": solve_gbs / PEAK_HBM_GBS,
                         "traffic": measured_traffic("fft_cols<double, 16>", {}, cfg, FFT_SOURCES),
                         "fft_equivalent_tflops": fft_tf,
                         "avg_launch_us": 1e6 * solve_s, "launches": g["launches"]},
            "row_pass": {"kernel": "bve_tlm_rows / bve_adj_rows (FP64, k=100)", "total_ms": sten["total_ms"],
                         "launches": sten["launches"],
                         "avg_launch_us": 1e3 * sten["total_ms"] / max(1, sten["launches"]),
                         "tflops_stencil_plus_fft_equivalent": row_tf},
            "row_pass_ms": sten["total_ms"], "column_pass_ms": g["total_ms"]}


def wall_section(rp4d, inputs, torch, np, max_gn=8):
    """burgers-wall-399: the paper's Burgers setup (Dirichlet walls, RK3-TVD,
    8000 steps, 15 x 20 observations, prior (0.5 I - 500 Lap*)^{-2}) assimilated
    from the background until |g_v|_inf falls below 1e-6 of its first value
    (at most max_gn GN iterations), PCG to 1e-9, sketches of l = l1 = 15 and
    l2 = 31 redrawn every iteration: Prec_Gamma, SketchPrec with each sketch and
    SketchSolv with each sketch.  Counts in the style of the paper's Burgers
    table (its own counts are not reproducible: observation locations unknown)."""
    cfg = dict(inputs.CFG_WALL)
    ell = cfg["ell"]
    ctx = rp4d.Context(0)
    p = rp4d.Problem(ctx, cfg)
    d = inputs.draws(cfg, seed=0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    xb, y = p.synthesize(dev(d["x_true"]), dev(d["xi"]), dev(d["eta"].reshape(-1)))
    p.set_data(xb, y.reshape(-1))
    tr = p.traj()
    methods = [("Prec_Gamma", rp4d.NOPREC, rp4d.SOLVE_PCG), ("SketchPrec RandSVD", rp4d.RANDSVD, rp4d.SOLVE_PCG),
               ("SketchPrec Nystrom", rp4d.NYSTROM, rp4d.SOLVE_PCG),
               ("SketchPrec SingleView", rp4d.SINGLEVIEW, rp4d.SOLVE_PCG),
               ("SketchSolv RandSVD", rp4d.RANDSVD, rp4d.SOLVE_SKETCH),
               ("SketchSolv Nystrom", rp4d.NYSTROM, rp4d.SOLVE_SKETCH),
               ("SketchSolv SingleView", rp4d.SINGLEVIEW, rp4d.SOLVE_SKETCH)]
    rows = []
    for name, sk, solve in methods:
        st = p.gn_state()
        p.reset_counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g0, gn, pcg, ok = None, 0, 0, False
        for it in range(max_gn):
            info = p.gn_step(st, sketch=sk, ell=ell, ell2=2 * ell + 1, seed=5000 + it, rtol=1e-9, maxit=400,
                             solve=solve, raise_noconv=False)
            g0 = info["gnorm_inf"] if g0 is None else g0
            gn += 1
            pcg += info["pcg_iters"]
            v, x = st.get()
            p.fwd(x, tr, want_J=False)
            g = p.gradient(tr, v)
            if float(g.abs().max()) < 1e-6 * g0:
                ok = True
                break
        torch.cuda.synchronize()
        c = p.counters()
        rows.append({"method": name, "gn_iters": gn, "converged": ok, "pcg_iters": pcg,
                     "offline_tlm": c["tlm_offline"], "offline_adj": c["adj_offline"],
                     "online_tlm": c["tlm_online"], "online_adj": c["adj_online"], "fwd": c["fwd"],
                     "seconds": time.perf_counter() - t0})
    return {"workload": cfg["name"], "n": cfg["n"], "nsteps": cfg["nsteps"], "m": p.m, "l": ell, "l2": 2 * ell + 1,
            "stop": "|g_v|_inf < 1e-6 |g_v(0)|_inf (checked with one FWD + gradient after each step)",
            "methods": rows}


def batch_section(rp4d, inputs, torch, np):
    """batch-64: 64 uneven Burgers problems (n in [256, 4096], N in [50, 500]),
    one batched Gauss-Newton iteration each (32-column Nystrom sketch, FP64 PCG
    to 1e-6), with FP64 and with FP32 sketch sweeps, each with the lock-step
    PCG eager and graph-replayed, against the same 64 iterations run one
    problem at a time through the single-problem FP64 path."""
    cfgs = inputs.batch_configs(64, seed=0)
    ctx = rp4d.Context(0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    probs, states = [], []
    for i, cfg in enumerate(cfgs):
        p = rp4d.Problem(ctx, cfg)
        p.set_id(i)
        d = inputs.draws(cfg, seed=cfg["seed"] % (2 ** 31))
        xb, y = p.synthesize(dev(d["x_true"]), dev(d["xi"]), dev(d["eta"].reshape(-1)))
        p.set_data(xb, y.reshape(-1))
        probs.append(p)
        states.append(p.gn_state())
    b = rp4d.Batch(ctx, probs)
    from paper_2401_15758_amd import autotune
    # the batched sweep tilings found by the batched search (tuning.json), per precision
    tuned = {name: autotune.apply_cached_batch(b, 32, dt) for name, dt in (("f64", rp4d.F64), ("f32", rp4d.F32))}
    # and the single-vector sweeps' own tiling (gradient and PCG products, FP64)
    tuned["k1_f64"] = autotune.apply_cached_batch(b, 1, rp4d.F64)
    res = {"workload": "batch-64", "problems": len(cfgs), "k": 32,
           "tiling": {name: (ent["sweep"] if ent else "library default") for name, ent in tuned.items()}}
    # the lock-step PCG eager and with its iteration body replayed as a HIP
    # graph (captured again whenever a problem converges)
    for name, skd, graphs in (("f64", rp4d.F64, False), ("f64_graph", rp4d.F64, True),
                              ("f32", rp4d.F32, False), ("f32_graph", rp4d.F32, True)):
        ctx.set_graphs(graphs)
        times = []
        for rep in range(3):
            for s in states:
                s.reset()
            for p in probs:
                p.reset_counters()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = b.gn_step(states, sketch=rp4d.NYSTROM, ell=32, seed=1, sketch_dtype=skd, rtol=1e-6)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        hv = sum(p.counters()["hv_columns"] for p in probs)
        t = min(times[1:])
        res[f"sketch_{name}"] = {"gn_step_ms": 1e3 * t, "hv_per_s": hv / t,
                                 "pcg_iters_max": max(i["pcg_iters"] for i in infos),
                                 "pcg_iters_total": sum(i["pcg_iters"] for i in infos)}
    ctx.set_graphs(False)
    for s in states:
        s.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, s in zip(probs, states):
        p.gn_step(s, sketch=rp4d.NYSTROM, ell=32, seed=1, sketch_dtype=rp4d.F64, rtol=1e-6)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    res["sequential_f64_gn_ms"] = 1e3 * seq
    res["speedup_vs_sequential"] = seq / (res["sketch_f64"]["gn_step_ms"] * 1e-3)
    return res


def serve_section(nreq=100):
    """serve-mix at reduced 2-D sizes: a Poisson stream of `nreq` solves (70 %
    Burgers, n 512-8192, 100-500 steps; 30 % vorticity at 64^2-128^2, 100-200
    steps; 3 GN iterations to 1e-6 each).  The served path's capacity is
    measured with every request queued at once (FP32 sketch sweeps); the same
    stream then arrives at 0.7 x that rate and runs through the served path with
    FP32 sketch sweeps (the mixed-precision form) and with FP64 ones, and
    through the plain FP64 one-at-a-time path.  The configured 2-D sizes
    (128^2-512^2, 100-300 steps) take minutes per request in the plain path:
    that run is `python -m paper_2401_15758_amd.serve`."""
    from paper_2401_15758_amd import rp4d, serve
    kw = dict(bve_nx=(64, 128), bve_N=(100, 200))
    cap = serve.summary(serve.serve(serve.make_trace(nreq, 0.0, seed=7, **kw), sketch_dtype=rp4d.F32))
    rate = 0.7 * cap["solves_per_s"]
    trace = serve.make_trace(nreq, rate, seed=7, **kw)
    mixed = serve.serve(serve.clone_trace(trace), sketch_dtype=rp4d.F32)
    f64 = serve.serve(serve.clone_trace(trace), sketch_dtype=rp4d.F64)
    seq = serve.serve_sequential(serve.clone_trace(trace))
    sm, sf, ss = serve.summary(mixed), serve.summary(f64), serve.summary(seq)
    sm["vs_sequential"], sf["vs_sequential"] = serve.compare(mixed, seq), serve.compare(f64, seq)
    return {"workload": "serve-mix (2-D at 64^2-128^2)", "requests": nreq,
            "capacity_solves_per_s": cap["solves_per_s"], "arrival_rate": rate,
            "served_mixed": sm, "served_fp64": sf, "sequential_fp64": ss,
            "throughput_ratio": sm["solves_per_s"] / ss["solves_per_s"],
            "p99_ratio": ss["p99_latency_s"] / sm["p99_latency_s"],
            "throughput_ratio_fp64": sf["solves_per_s"] / ss["solves_per_s"],
            "p99_ratio_fp64": ss["p99_latency_s"] / sf["p99_latency_s"]}


def cpu_baseline(cfg, ell, rtol, runs=3):
    """The oracle as it stands: one GN iteration of the same workload with BLAS
    threads on every core of the process's affinity, and four Hessian columns on
    one thread; each the median of `runs` timings."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import gn as ogn
    from oracle.problem import burgers_problem
    from paper_2401_15758_amd import inputs
    cores = len(os.sched_getaffinity(0))
    rates, secs = [], []
    with threadpool_limits(limits=cores):
        orc = burgers_problem(cfg, inputs.draws(cfg, seed=0))
        Om = inputs.omega(cfg["n"], ell, seed=1000)
        for _ in range(runs):
            t0 = time.perf_counter()
            _, _, _, info = ogn.gn_step(orc, np.zeros(cfg["n"]), method="nystrom", Omega=Om, rtol=rtol)
            dt = time.perf_counter() - t0
            secs.append(dt)
            rates.append((ell + info["pcg"]["iters"]) / dt)
    rates1, secs1 = [], []
    with threadpool_limits(limits=1):
        tr = orc.fwd(orc.xb)
        for _ in range(runs):
            t0 = time.perf_counter()
            orc.hessian(tr, Om[:, :4])
            dt1 = time.perf_counter() - t0
            secs1.append(dt1)
            rates1.append(4 / dt1)
    return {"value": float(np.median(rates)), "unit": "Hv/s", "cores": cores, "kind": "oracle",
            "runs": [float(r) for r in rates],
            "sample": f"one GN iteration of burgers-4096 ({ell}-column Nystrom sketch + "
                      f"{info['pcg']['iters']} PCG products to rtol {rtol:g}), FP64 numpy, median of {runs} "
                      f"runs of {min(secs):.1f}-{max(secs):.1f} s",
            "one_thread": {"value": float(np.median(rates1)), "unit": "Hv/s", "cores": 1,
                           "runs": [float(r) for r in rates1],
                           "sample": f"4 Hessian columns of burgers-4096, median of {runs} runs of "
                                     f"{min(secs1):.1f}-{max(secs1):.1f} s"}}


def calib_copy(torch, mib, rec):
    """One elementwise copy that reads and writes `mib` MiB: the reference
    dispatch for the HBM byte counters of a profiled run."""
    if mib <= 0:
        return
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    rec["calib_copy_mib"] = mib


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build measures one GPU only (requested --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the sharded multi-GPU path is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2401_15758_amd import autotune, inputs, rp4d

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only:
        sec = {"bve": lambda: bve_section(rp4d, inputs, torch, np, gn=args.gn_iters > 0),
               "batch": lambda: batch_section(rp4d, inputs, torch, np),
               "serve": serve_section, "wall": lambda: wall_section(rp4d, inputs, torch, np)}[args.only]
        rec = {args.only: sec()}
        calib_copy(torch, args.calib_copy_mib, rec)
        print(json.dumps(rec), flush=True)
        return
    cfg = dict(inputs.CFG_LARGE)
    ell, rtol = cfg["ell"], 1e-6
    sk = rp4d.NYSTROM if args.sketch == "nystrom" else rp4d.RANDSVD
    skd = rp4d.F64 if args.sketch_dtype == "f64" else rp4d.F32
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")

    ctx = rp4d.Context(0)
    prob = rp4d.Problem(ctx, cfg)
    d = inputs.draws(cfg, seed=0)
    xb, y = prob.synthesize(dev(d["x_true"]), dev(d["xi"]), dev(d["eta"].reshape(-1)))
    prob.set_data(xb, y.reshape(-1))
    state = prob.gn_state()

    # sweep tilings for the sketch block (k = ell) and the single-vector products
    # of the gradient and PCG: tuned on the device unless cached
    cache_path = args.tuning_cache or autotune.CACHE_PATH
    traj0 = prob.traj()
    prob.fwd(xb, traj0, want_J=False)
    tilings = {}
    for k, dt in ((ell, skd), (1, rp4d.F64)):
        tilings[f"k{k}-{'f64' if dt == rp4d.F64 else 'f32'}"] = autotune.tune_or_load(
            prob, traj0, cfg["nsteps"], k, dt, budget_s=args.tune_budget, cache_path=cache_path,
            x0=xb if k == 1 else None)
    del traj0

    def step():
        state.reset()
        infos = []
        for it in range(args.gn_iters):
            infos.append(prob.gn_step(state, sketch=sk, ell=ell, seed=1000 + it, sketch_dtype=skd, rtol=rtol))
        return infos

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prob.reset_counters()
    # one HIP event pair per sweep (not per launch): timing must not slow the steps
    ctx.set_timing(rp4d.TIMING_SPAN)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, step_ms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        infos.extend(step())
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - ts))
    t1 = time.perf_counter()
    elapsed = t1 - t0
    cnt = prob.counters()
    kst = {name: ctx.kernel_stats(kind) for name, kind in
           (("tlm", rp4d.K_TLM), ("adj", rp4d.K_ADJ), ("tlm1", rp4d.K_TLM1), ("adj1", rp4d.K_ADJ1),
            ("fwd", rp4d.K_FWD), ("bhalf", rp4d.K_BHALF), ("eig", rp4d.K_EIG))}
    ctx.set_timing(False)

    hv_per_s = cnt["hv_columns"] / elapsed
    # the k = 64 ADJ sweep: the kernel with the largest share of the step in the
    # profile.  Its span holds its launches only, while the TLM sweep's span also
    # holds its waits for the rows of the FWD it follows on the other stream.
    dom = "adj"
    ks = kst[dom]
    achieved = ks["alg_flops"] / (ks["total_ms"] * 1e-3) / 1e12 if ks["total_ms"] > 0 else 0.0
    peak = PEAK_FP64_VALU_TFLOPS if skd == rp4d.F64 else PEAK_FP32_VALU_TFLOPS
    tl = tilings[f"k{ell}-{'f64' if skd == rp4d.F64 else 'f32'}"][dom]
    kname = (f"burgers_{dom}{'_wave' if tl.get('xch') == rp4d.XCH_WAVE else ''}_kernel"
             f"<{'double' if skd == rp4d.F64 else 'float'}, {tl['ppt']}, {tl['kc']}>")
    roofline = {"bound": "alu", "kernel": kname + f" (k={ell} block sweep)", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(kname, tl, cfg),
                "avg_launch_us": 1e3 * ks["total_ms"] / max(1, ks["launches"]),
                "launches": ks["launches"],
                "timing": "HIP events on the library stream, one pair around each sweep's launches"}

    reuse_ms, reuse_infos, adaptive = None, [], None
    if not args.gn_only:
        # the same assimilation with the sketch-reuse test (kappa_re < 10 keeps the
        # resident preconditioner, Sec. 3.2): fewer products per GN step
        state.reset()
        torch.cuda.synchronize()
        tr0 = time.perf_counter()
        reuse_infos = [prob.gn_step(state, sketch=sk, ell=ell, seed=1000 + it, sketch_dtype=skd, rtol=rtol,
                                    reuse_eps=10.0) for it in range(args.gn_iters)]
        torch.cuda.synchronize()
        reuse_ms = 1e3 * (time.perf_counter() - tr0) / args.gn_iters

        # SketchPrecA: adaptive RandSVD (Alg. 4; 32 columns, 16 more while kappa_sk >
        # 1.01, at most 128) with the kappa_re < 10 reuse test, as in the paper's
        # adaptive runs; one warm-up assimilation, then one timed
        def adaptive_run():
            state.reset()
            return [prob.gn_step(state, sketch=rp4d.RANDSVD_ADAPTIVE, ell=32, ell_hat=16, ell_max=128, eps_sk=1.01,
                                 seed=2000 + it, rtol=rtol, reuse_eps=10.0) for it in range(args.gn_iters)]
        adaptive_run()
        torch.cuda.synchronize()
        prob.reset_counters()
        ta0 = time.perf_counter()
        ad_infos = adaptive_run()
        torch.cuda.synchronize()
        ad_ms = 1e3 * (time.perf_counter() - ta0) / args.gn_iters
        ad_cnt = prob.counters()
        adaptive = {"method": "adaptive RandSVD (Alg. 4) + reuse test", "ell0": 32, "ell_hat": 16, "ell_max": 128,
                    "eps_sk": 1.01, "reuse_eps": 10.0, "gn_step_ms": ad_ms,
                    "sketch_ell": [i["sketch_ell"] for i in ad_infos], "kappa_sk": [i["kappa_sk"] for i in ad_infos],
                    "reused": [i["reused"] for i in ad_infos], "pcg_iters": [i["pcg_iters"] for i in ad_infos],
                    "offline_tlm": ad_cnt["tlm_offline"], "online_tlm": ad_cnt["tlm_online"]}

    # isolated block Hessian product, k = 64, FP64 (sketch shape)
    traj = prob.traj()
    prob.fwd(xb, traj, want_J=False)
    V = torch.empty((cfg["n"], ell), dtype=torch.float64, device="cuda")
    ctx.philox_normal(7, V.numel(), V)
    HV = torch.empty_like(V)
    for _ in range(2):
        prob.hessian_block(traj, V, HV)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        prob.hessian_block(traj, V, HV)
    e1.record()
    torch.cuda.synchronize()
    block_ms = e0.elapsed_time(e1) / reps

    # single-vector product (the PCG's), FP64
    v1 = V[:, :1].contiguous()
    hv1 = torch.empty_like(v1)
    prob.hessian_block(traj, v1, hv1)
    torch.cuda.synchronize()
    reps1 = 20
    e0.record()
    for _ in range(reps1):
        prob.hessian_block(traj, v1, hv1)
    e1.record()
    torch.cuda.synchronize()
    hv1_ms = e0.elapsed_time(e1) / reps1

    singleview = None
    if not args.gn_only:
        # SketchPrec with SingleView (Alg. 3): l1 = ell TLM columns and l2 = 2 l1 + 1
        # ADJ columns (the paper's pairing), the ADJ block on a second stream beside
        # the TLM block or both on one stream; RandSVD / Nystrom builds of the same
        # l for comparison.  The l2-column sweeps have tilings of their own (tuned
        # on the device unless cached).
        l2 = 2 * ell + 1
        autotune.tune_or_load(prob, traj, cfg["nsteps"], l2, rp4d.F64, budget_s=args.tune_budget, cache_path=cache_path)

        def build_ms(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            tb = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return 1e3 * (time.perf_counter() - tb) / reps

        sv_two = build_ms(lambda: prob.build_precond_singleview(traj, ell, l2, seed=5))
        sv_one = build_ms(lambda: prob.build_precond_singleview(traj, ell, l2, seed=5, serial=True))
        rs_build = build_ms(lambda: prob.build_precond(traj, rp4d.RANDSVD, ell, seed=5))
        ny_build = build_ms(lambda: prob.build_precond(traj, rp4d.NYSTROM, ell, seed=5))

        def sv_run():
            state.reset()
            return [prob.gn_step(state, sketch=rp4d.SINGLEVIEW, ell=ell, ell2=l2, seed=3000 + it, rtol=rtol)
                    for it in range(args.gn_iters)]
        sv_run()
        torch.cuda.synchronize()
        tv0 = time.perf_counter()
        sv_infos = sv_run()
        torch.cuda.synchronize()
        singleview = {"method": "SingleView (Alg. 3)", "l1": ell, "l2": l2,
                      "build_ms_two_streams": sv_two, "build_ms_one_stream": sv_one,
                      "randsvd_build_ms": rs_build, "nystrom_build_ms": ny_build,
                      "gn_step_ms": 1e3 * (time.perf_counter() - tv0) / args.gn_iters,
                      "pcg_iters": [i["pcg_iters"] for i in sv_infos]}

    # achievable HBM bandwidth: a plain 1 GiB device copy (reads and writes 1 GiB)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    hbm_gbs = 2 * src.numel() * 8 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    del src, dst

    out = {
        "metric": "Hessian-vec products/s; time per GN step to 1e-6 residual; p50/p99 latency",
        "value": hv_per_s,
        "unit": "Hv/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if skd == rp4d.F64 else "f64 (sketch sweeps f32)",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": cfg["n"], "nsteps": cfg["nsteps"], "dt": cfg["dt"],
                   "obs_stride": cfg["obs_stride"], "obs_every": cfg["obs_every"], "k": ell,
                   "sketch": args.sketch, "gn_iters": args.gn_iters, "pcg_rtol": rtol},
        "gn_step_ms": 1e3 * elapsed / (args.steps * args.gn_iters),
        "pcg_iters_per_gn": [i["pcg_iters"] for i in infos[: args.gn_iters]],
        "step_ms_median": float(np.median(step_ms)), "step_ms_p10": float(np.percentile(step_ms, 10)),
        "step_ms_p90": float(np.percentile(step_ms, 90)),
        "gn_step_ms_with_reuse": reuse_ms,
        "reuse_decisions": [i["reused"] for i in reuse_infos],
        "pcg_iters_with_reuse": [i["pcg_iters"] for i in reuse_infos],
        "adaptive": adaptive,
        "singleview": singleview,
        "hessian_block_ms": block_ms,
        "hessian_block_hv_per_s": ell / (block_ms * 1e-3),
        "hessian_k1_ms": hv1_ms, "hessian_k1_hv_per_s": 1.0 / (hv1_ms * 1e-3),
        "hbm_copy_gbs_measured": hbm_gbs,
        "roofline": roofline,
        "kernels": {k: {"launches": v["launches"], "total_ms": v["total_ms"],
                        "tflops": (v["alg_flops"] / (v["total_ms"] * 1e-3) / 1e12) if v["total_ms"] > 0 else 0.0}
                    for k, v in kst.items()},
        "counters": cnt,
        "tiling": tilings,
    }
    def note(msg):
        print(f"bench: {msg}", file=sys.stderr, flush=True)

    note("burgers-4096 done")
    if not args.no_wall:
        note("burgers-wall-399 section")
        out["wall"] = wall_section(rp4d, inputs, torch, np)
    if not args.no_bve:
        note("bve-256 section")
        out["bve"] = bve_section(rp4d, inputs, torch, np)
    if not args.no_batch:
        note("batch-64 section")
        out["batch"] = batch_section(rp4d, inputs, torch, np)
    if not args.no_serve:
        note("serve-mix section")
        out["serve"] = serve_section()
    if not args.no_cpu_baseline:
        note("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(cfg, ell, rtol)
    calib_copy(torch, args.calib_copy_mib, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
