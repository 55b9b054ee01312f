"""Serving loop for SC-4DVAR solves on one GPU (Sec. 3.2: reuse or recompute the
sketch across Gauss-Newton iterations).

A request is one assimilation: synthesise its data on the device, then run
`gn_steps` Gauss-Newton iterations (PCG to `rtol` each) from the background.
Requests arrive as a Poisson stream and are served with:

* admission by an HBM footprint estimate (trajectory, 2-D stage storage,
  resident preconditioner, sketch and PCG workspaces) against a budget; a
  request waits in FIFO order until its footprint fits;
* continuous batching: admitted 1-D (Burgers) requests join the running batch
  at GN-step boundaries -- every batched GN step advances all of them by one
  iteration in fused launches -- and leave it when done; 2-D (vorticity)
  requests run on a second stream from a second host thread, so their work
  overlaps the batch on the device;
* residency: each request's trajectory and preconditioner stay in its GN state
  across its iterations, and the reuse test kappa_re < reuse_eps decides
  whether to keep the preconditioner or sketch again;
* cancellation: a request whose `cancel_at` has passed (or that has done
  `cancel_after` GN steps) is dropped from the queue, or leaves service at its
  next GN-step boundary (its memory and budget released, its state at that
  point kept in `x`); the others are unaffected.

Every random draw of a request is keyed by the request id and its iteration
number, and all reductions are per problem, so a request's result does not
depend on which other requests share the GPU with it.

The baseline is the plain path: FP64, one request at a time in arrival order,
single-problem calls, a new sketch every iteration.
"""
import math
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs


# ---------------------------------------------------------------------------
# workload
# ---------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    cfg: dict
    arrival: float          # seconds after the start of the run
    seed: int
    admitted: float = math.nan
    done: float = math.nan
    gn_done: int = 0
    pcg_iters: list = field(default_factory=list)
    reused: int = 0
    J: list = field(default_factory=list)
    relres: list = field(default_factory=list)   # final PCG relative residual of each GN step
    x: np.ndarray = None    # final state (host copy)
    hbm_peak: int = 0       # peak device bytes the served run's contexts held (library count)
    cancel_at: float = math.inf   # cancellation time (seconds after the start of the run)
    cancel_after: int = None      # or: cancelled once this many GN steps are done
    cancelled: bool = False

    def cancel_due(self, now):
        return self.cancel_at <= now or (self.cancel_after is not None and self.gn_done >= self.cancel_after)

    @property
    def model(self):
        return self.cfg.get("model", "burgers")

    @property
    def latency(self):
        return self.done - self.arrival


# grid sides of the 2-D model's FFTs: 16 B, B in {2,3,4,5,6,8,10,12,16,20,24,32}
BVE_SIDES = (32, 48, 64, 80, 96, 128, 160, 192, 256, 320, 384, 512)


def bve_side(x, lim):
    """The supported side within [lim[0], lim[1]] nearest to x in log scale."""
    cands = [s for s in BVE_SIDES if lim[0] <= s <= lim[1]] or [min(BVE_SIDES, key=lambda s: abs(s - x))]
    return min(cands, key=lambda s: abs(math.log(s / x)))


def make_trace(nreq, rate, seed=0, frac_burgers=0.7, burgers_n=(512, 8192), burgers_N=(100, 500),
               bve_nx=(128, 512), bve_N=(100, 300)):
    """Poisson arrivals at `rate` per second of a mix of solves: Burgers with n
    log-uniform in `burgers_n` and N uniform in `burgers_N` (observations every 4th
    point every 10 steps, sketch 32); vorticity with nx log-uniform in `bve_nx`,
    rounded to the nearest side the FFTs take, and N uniform in `bve_N` (every
    16th cell every 20 steps, sketch 100)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(nreq):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        if rng.uniform() < frac_burgers:
            n = int(round(math.exp(rng.uniform(math.log(burgers_n[0]), math.log(burgers_n[1])))))
            N = int(rng.integers(burgers_N[0], burgers_N[1] + 1))
            cfg = inputs.burgers_config(n, N, 4, 10, dt_cfg=1e-3, ell=32, name=f"req{rid}-burgers-{n}")
        else:
            nx = bve_side(math.exp(rng.uniform(math.log(bve_nx[0]), math.log(bve_nx[1]))), bve_nx)
            N = int(rng.integers(bve_N[0], bve_N[1] + 1))
            cfg = inputs.bve_config(nx, nsteps=N, obs_stride=16, obs_every=20, ell=100, name=f"req{rid}-bve-{nx}")
        out.append(Request(rid=rid, cfg=cfg, arrival=t, seed=int(rng.integers(0, 2 ** 31))))
    return out


def footprint_bytes(cfg):
    """Upper estimate of the device memory one request holds while in service
    (problem, trajectory, GN state with its preconditioner, sketch and sweep
    workspaces), with 15 % and 32 MiB of headroom for the allocator's
    granularity and the small per-problem buffers."""
    ell = cfg["ell"]
    n = cfg["n"]
    N = cfg["nsteps"]
    m = inputs.n_obs(cfg) * inputs.n_t(cfg)
    w = 8
    if cfg.get("model") == "bve":
        nx = cfg["nx"]
        traj = w * n * (N + 1) + 7 * w * n * N + 2 * w * m
        basis = 1.5 * (4 * w * nx * nx + 2 * w * n)
        sweeps = 8 * w * n * ell + 3 * w * n * ell + 12 * w * n    # block fields, prior scratch, FWD
        sketch = 6 * w * n * ell + 2 * w * m * ell + 8 * w * ell * ell
        state = w * n * ell + 12 * w * n
        return int(1.15 * (traj + basis + sweeps + sketch + state) + (32 << 20))
    traj = w * n * (N + 1) + 2 * w * m
    sweeps = 4 * w * n * (ell + 8) + w * m * ell
    sketch = 6 * w * n * ell + 2 * w * m * ell + 8 * w * ell * ell
    state = w * n * ell + 12 * w * n + w * n * 80      # resident basis, vectors, spectral prior
    return int(1.15 * (traj + sweeps + sketch + state) + (32 << 20))


# ---------------------------------------------------------------------------
# request execution (device work through the C ABI)
# ---------------------------------------------------------------------------
def _setup(rp4d, torch, ctx, req, pid=None):
    """Problem + data synthesised on the device + GN state, on ctx's stream."""
    cfg = req.cfg
    p = rp4d.Problem(ctx, cfg)
    p.set_id(req.rid * 8 if pid is None else pid)
    d = inputs.draws(cfg, seed=req.seed)
    with torch.cuda.stream(ctx.stream):
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda", non_blocking=False)
        xb, y = p.synthesize(dev(d["x_true"]), dev(d["xi"]), dev(d["eta"].reshape(-1)))
        p.set_data(xb, y.reshape(-1))
    st = p.gn_state()
    return p, st


def _finish(torch, ctx, req, st, t0, verbose=False):
    with torch.cuda.stream(ctx.stream):
        _, x = st.get()
        req.x = x.cpu().numpy()
    req.done = time.perf_counter() - t0
    if verbose:
        print(f"serve: request {req.rid} ({req.cfg['name']}, {req.cfg['nsteps']} steps) done at {req.done:.1f} s, "
              f"PCG iterations {req.pcg_iters}", file=sys.stderr, flush=True)


def _step_seed(req, it):
    return (req.seed * 1000003 + 7919 * (it + 1)) % (2 ** 63)


class _Budget:
    def __init__(self, limit):
        self.limit, self.used = limit, 0
        self.lock = threading.Lock()

    def try_take(self, b):
        with self.lock:
            if self.used + b <= self.limit or self.used == 0:
                self.used += b
                return True
            return False

    def give(self, b):
        with self.lock:
            self.used -= b


def serve(trace, budget_bytes=64 << 30, gn_steps=3, rtol=1e-6, reuse_eps=10.0, sketch_dtype=None, bve_lanes=2,
          verbose=False):
    """Run `trace` through the served path; returns the requests with their
    timings and final states.  Arrival times are honoured from the start."""
    import torch

    from . import rp4d
    if sketch_dtype is None:
        sketch_dtype = rp4d.F64
    t0 = time.perf_counter()
    budget = _Budget(budget_bytes)
    # each lane's context carries the served budget as its hard cap in the
    # library: the reservations above keep the lanes' sum within it, and an
    # estimate that fell short would surface as ENOMEM, not as an overcommit
    lane_ctx = []
    peak = [0]

    def lane_context():
        c = rp4d.Context(0, stream=torch.cuda.Stream(), hbm_budget=budget_bytes)
        lane_ctx.append(c)
        return c

    def note_usage():
        peak[0] = max(peak[0], sum(c.hbm()["used"] for c in list(lane_ctx)))
    pend_b = [r for r in trace if r.model == "burgers"]
    pend_v = [r for r in trace if r.model != "burgers"]
    vlock = threading.Lock()
    errors = []

    def now():
        return time.perf_counter() - t0

    def burgers_lane():
        ctx = lane_context()
        active = []   # (req, problem, state, footprint)
        queue = list(pend_b)
        batch, members = None, ()
        while queue or active:
            # drop queued requests whose cancellation time has passed
            for r in [q for q in queue if q.cancel_due(now())]:
                queue.remove(r)
                r.cancelled, r.done = True, now()
            # admit arrived requests in FIFO order while their footprint fits
            while queue and queue[0].arrival <= now():
                fp = footprint_bytes(queue[0].cfg)
                if not budget.try_take(fp):
                    break
                r = queue.pop(0)
                r.admitted = now()
                p, st = _setup(rp4d, torch, ctx, r)
                active.append((r, p, st, fp))
            if not active:
                time.sleep(0.0005)
                continue
            for r, p, st, fp in active:
                p.set_id(r.rid * 8 + r.gn_done)     # per-request, per-iteration draws
            ids = tuple(a[0].rid for a in active)
            if ids != members:                       # membership changed: new batch descriptor set
                if batch is not None:
                    batch.close()
                batch, members = rp4d.Batch(ctx, [a[1] for a in active]), ids
            infos = batch.gn_step([a[2] for a in active], ell=32, seed=12345, sketch_dtype=sketch_dtype, rtol=rtol,
                                  reuse_eps=reuse_eps)
            note_usage()
            keep = []
            for (r, p, st, fp), inf in zip(active, infos):
                r.gn_done += 1
                r.pcg_iters.append(inf["pcg_iters"])
                r.J.append(inf["J"])
                r.relres.append(inf["pcg_relres"])
                r.reused += inf["reused"]
                if r.gn_done < gn_steps and r.cancel_due(now()):
                    r.cancelled = True
                if r.gn_done >= gn_steps or r.cancelled:
                    _finish(torch, ctx, r, st, t0, verbose)
                    st.close()
                    budget.give(fp)
                else:
                    keep.append((r, p, st, fp))
            if len(keep) != len(active) and batch is not None:
                batch.close()
                batch, members = None, ()
            for (r, p, st, fp) in active:
                if r.gn_done >= gn_steps or r.cancelled:
                    p.close()
            active = keep
        if batch is not None:
            batch.close()

    def bve_lane():
        ctx = lane_context()
        while True:
            with vlock:
                if not pend_v:
                    return
                r = pend_v[0]
                if r.cancel_due(now()):          # cancelled while queued
                    pend_v.pop(0)
                    r.cancelled, r.done = True, now()
                    continue
                take = r.arrival <= now() and budget.try_take(footprint_bytes(r.cfg))
                if take:
                    pend_v.pop(0)
            if not take:
                time.sleep(0.0005)
                continue
            fp = footprint_bytes(r.cfg)
            r.admitted = now()
            p, st = _setup(rp4d, torch, ctx, r)
            for it in range(gn_steps):
                if it > 0 and r.cancel_due(now()):
                    r.cancelled = True
                    break
                inf = p.gn_step(st, ell=r.cfg["ell"], seed=_step_seed(r, it), sketch_dtype=sketch_dtype, rtol=rtol,
                                reuse_eps=reuse_eps)
                r.gn_done += 1
                r.pcg_iters.append(inf["pcg_iters"])
                r.J.append(inf["J"])
                r.relres.append(inf["pcg_relres"])
                r.reused += inf["reused"]
                note_usage()
                if verbose:
                    print(f"serve: request {r.rid} GN step {it + 1} at {now():.1f} s, {inf['pcg_iters']} PCG iterations",
                          file=sys.stderr, flush=True)
            _finish(torch, ctx, r, st, t0, verbose)
            st.close()
            p.close()
            budget.give(fp)

    def guard(fn):
        def run():
            try:
                fn()
            except BaseException as e:      # re-raised by the caller
                errors.append(e)
        return run

    threads = [threading.Thread(target=guard(burgers_lane))]
    threads += [threading.Thread(target=guard(bve_lane)) for _ in range(max(1, bve_lanes) if pend_v else 0)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]
    for r in trace:
        r.hbm_peak = peak[0]
    return trace


def serve_sequential(trace, gn_steps=3, rtol=1e-6, verbose=False):
    """The plain path: FP64, one request at a time in arrival order, a new
    sketch every iteration, single-problem calls."""
    import torch

    from . import rp4d
    t0 = time.perf_counter()
    ctx = rp4d.Context(0, stream=torch.cuda.Stream())
    for r in sorted(trace, key=lambda q: q.arrival):
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(0.0005)
        r.admitted = time.perf_counter() - t0
        p, st = _setup(rp4d, torch, ctx, r)
        for it in range(gn_steps):
            inf = p.gn_step(st, ell=r.cfg["ell"], seed=_step_seed(r, it), sketch_dtype=rp4d.F64, rtol=rtol)
            r.gn_done += 1
            r.pcg_iters.append(inf["pcg_iters"])
            r.J.append(inf["J"])
            r.relres.append(inf["pcg_relres"])
            if verbose:
                print(f"serve: request {r.rid} GN step {it + 1} at {time.perf_counter() - t0:.1f} s, "
                      f"{inf['pcg_iters']} PCG iterations (sequential)", file=sys.stderr, flush=True)
        _finish(torch, ctx, r, st, t0, verbose)
        st.close()
        p.close()
    return trace


def summary(trace):
    cancelled = sum(1 for r in trace if r.cancelled)
    trace = [r for r in trace if not r.cancelled]
    lat = np.array([r.latency for r in trace])
    span = max(r.done for r in trace) - min(r.arrival for r in trace)
    last_res = [r.relres[-1] for r in trace if r.relres]
    return {"requests": len(trace), "cancelled": cancelled, "solves_per_s": len(trace) / span, "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "makespan_s": span,
            "pcg_iters_total": int(sum(sum(r.pcg_iters) for r in trace)),
            "reuses": int(sum(r.reused for r in trace)),
            "final_relres_max": float(max(last_res)) if last_res else None,
            "hbm_peak_bytes": int(max(r.hbm_peak for r in trace))}


def compare(a, b):
    """Per-request agreement of two runs of the same trace: the final cost J
    after the last GN step (relative difference) and the final PCG residuals."""
    by = {r.rid: r for r in b}
    dj = [abs(r.J[-1] - by[r.rid].J[-1]) / abs(by[r.rid].J[-1]) for r in a]
    return {"J_final_reldiff_max": float(max(dj)), "J_final_reldiff_median": float(np.median(dj)),
            "relres_final_max": [float(max(r.relres[-1] for r in a)), float(max(r.relres[-1] for r in b))]}


def clone_trace(trace):
    return [Request(rid=r.rid, cfg=dict(r.cfg), arrival=r.arrival, seed=r.seed, cancel_at=r.cancel_at,
                    cancel_after=r.cancel_after) for r in trace]


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serve a Poisson stream of SC-4DVAR solves")
    ap.add_argument("--requests", type=int, default=24)
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals per second (0: 0.7 x measured capacity)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--bve-nx", type=int, nargs=2, default=(128, 512))
    ap.add_argument("--bve-steps", type=int, nargs=2, default=(100, 300))
    ap.add_argument("--budget-gib", type=float, default=64.0)
    ap.add_argument("--sketch", choices=["f32", "f64", "both"], default="both",
                    help="sketch sweeps of the served path: FP32 (the mixed-precision form), FP64, or both")
    ap.add_argument("--bve-lanes", type=int, default=2, help="2-D requests served concurrently (own stream each)")
    ap.add_argument("--no-sequential", action="store_true", help="skip the one-request-at-a-time comparison")
    args = ap.parse_args()
    from . import rp4d
    kw = dict(bve_nx=tuple(args.bve_nx), bve_N=tuple(args.bve_steps))
    budget = int(args.budget_gib * 2 ** 30)
    rate = args.rate
    out = {"requests": args.requests, "bve_nx": list(args.bve_nx), "bve_steps": list(args.bve_steps)}

    def note(msg):
        print(f"serve: {msg}", file=sys.stderr, flush=True)
    if rate <= 0:
        cap = serve(make_trace(args.requests, 0.0, seed=args.seed, **kw), budget_bytes=budget, bve_lanes=args.bve_lanes,
                    verbose=True)
        out["capacity_solves_per_s"] = summary(cap)["solves_per_s"]
        rate = 0.7 * out["capacity_solves_per_s"]
        note(f"capacity {out['capacity_solves_per_s']:.3f} solves/s")
    trace = make_trace(args.requests, rate, seed=args.seed, **kw)
    out["rate"] = rate
    runs = {}
    chosen = {"f32": ("served_mixed",), "f64": ("served_fp64",), "both": ("served_mixed", "served_fp64")}[args.sketch]
    for name, dt in (("served_mixed", rp4d.F32), ("served_fp64", rp4d.F64)):
        if name in chosen:
            runs[name] = serve(clone_trace(trace), budget_bytes=budget, sketch_dtype=dt, bve_lanes=args.bve_lanes,
                               verbose=True)
            out[name] = summary(runs[name])
            note(f"{name} done")
    out["bve_lanes"] = args.bve_lanes
    if not args.no_sequential:
        seq = serve_sequential(clone_trace(trace), verbose=True)
        out["sequential_fp64"] = summary(seq)
        for name, run in runs.items():
            out[name]["vs_sequential"] = compare(run, seq)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
