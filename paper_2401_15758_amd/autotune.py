"""Autotuner for the block-sweep tiling of the rp4d library.

The TLM/ADJ sweeps are parameterised by points per thread (ppt), vectors per
workgroup (kc), threads per workgroup, tile length (grid points owned per
workgroup) and steps per launch (which fixes the halo, 4*steps+4 points per
side).  For a problem shape (n, nsteps, k, dtype) the tuner enumerates valid
tilings, times rp4d_tlm and rp4d_adj with each on the device (HIP events on the
library stream), and keeps the fastest.  Results are cached as JSON keyed by
the shape so later runs apply them without searching.
"""
import json
import math
import os
import time

import torch

from . import rp4d

CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
PPTS = (1, 2, 4)
KCS = (1, 2, 4, 8)
LDS_LIMIT = 160 * 1024


def key(n, nsteps, k, dtype):
    return f"n{n}-N{nsteps}-k{k}-{'f64' if dtype == rp4d.F64 else 'f32'}"


def candidates(n, k, dtype=rp4d.F64, min_groups_tiles=32):
    """Valid tilings for an n-point problem with k vectors."""
    es = 8 if dtype == rp4d.F64 else 4
    out = []
    for kc in KCS:
        if kc > max(1, k) and kc != 1:
            continue
        groups = -(-k // kc)
        for ntiles in (1, 2, 4, 8, 16, 32, 64, 128):
            tile = -(-n // ntiles)
            if tile < 16:
                continue
            if groups * ntiles < min(min_groups_tiles, groups * 128):
                continue
            for steps in (2, 4, 8, 12, 16, 25, 32, 50):
                halo = 4 * steps + 4
                region = tile + 2 * halo
                if region > 3 * tile + 64:          # halo-dominated: wasteful
                    continue
                for ppt in PPTS:
                    if kc == 8 and ppt > 2:
                        continue
                    threads = -(-region // ppt)
                    threads = -(-threads // 64) * 64
                    if threads > (512 if ppt * kc >= 8 else 1024) or threads < 64:
                        continue
                    if 2 * 2 * threads * (1 + kc) * es > LDS_LIMIT:
                        continue
                    out.append(dict(ppt=ppt, kc=kc, threads=threads, tile=tile, steps=steps, xch=rp4d.XCH_LDS))
    out.extend(wave_candidates(n, WAVE_PK))
    return out


# (ppt, kc) pairs with a wave-region kernel instance
WAVE_PK = ((1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2), (8, 1))
WAVE_STEPS = (2, 3, 4, 6, 8, 10, 12, 13, 14, 15, 16, 20, 25, 32, 50)


def wave_candidates(n, pk):
    """Wave-region tilings: each 64-lane wave covers 64 * ppt points, the owned
    tile the rest after two halos of 4 * steps + 4; tiles are balanced over n."""
    out = []
    for ppt, kc in pk:
        for steps in WAVE_STEPS:
            tmax = 64 * ppt - 2 * (4 * steps + 4)
            if tmax < 4 and tmax < n:   # single-vector sweeps favour many small regions
                continue
            tmax = min(tmax, n)
            ntiles = -(-n // tmax)
            tile = -(-n // ntiles)
            for threads in (64, 256):
                out.append(dict(ppt=ppt, kc=kc, threads=threads, tile=tile, steps=steps, xch=rp4d.XCH_WAVE))
    return out


def _time(fn, reps):
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


FIELDS = ("ppt", "kc", "threads", "tile", "steps", "xch")


def tune(prob, traj, k, dtype=rp4d.F64, reps=2, budget_s=30.0, verbose=False):
    """Search tilings for the TLM and the ADJ sweep of (prob, k, dtype) separately
    (timing rp4d_tlm / rp4d_adj); applies the best of each and returns
    {"tlm": {...tiling, ms}, "adj": {...}}."""
    tdtype = torch.float64 if dtype == rp4d.F64 else torch.float32
    V = torch.empty((prob.n, k), dtype=torch.float64, device=prob.dev)
    prob.ctx.philox_normal(11, V.numel(), V)
    V = V.to(tdtype)
    W = torch.empty((prob.n_t, prob.n_obs, k), dtype=torch.float64, device=prob.dev)
    prob.ctx.philox_normal(12, W.numel(), W)
    W = W.to(tdtype)
    Z = torch.empty_like(W)
    U = torch.empty_like(V)
    ops = {rp4d.MODE_TLM: lambda: prob.tlm(traj, V, Z), rp4d.MODE_ADJ: lambda: prob.adj(traj, W, U)}
    cands = candidates(prob.n, k, dtype)
    cands.sort(key=lambda c: (-c["steps"], -c["tile"]))
    out = {}
    for mode, name in ((rp4d.MODE_TLM, "tlm"), (rp4d.MODE_ADJ, "adj")):
        prob.set_sweep_tiling(dtype, k, mode=mode)          # heuristic baseline
        best = dict(prob.get_sweep_tiling(dtype, k, mode=mode))
        best_ms = _time(ops[mode], reps)
        t_end = time.perf_counter() + budget_s / 2
        timed = 0
        for c in cands:
            if time.perf_counter() > t_end:
                break
            prob.set_sweep_tiling(dtype, k, mode=mode, **c)
            try:
                ms = _time(ops[mode], reps)
            except rp4d.Rp4dError:
                continue
            timed += 1
            if verbose:
                print(f"  {name} {c} {ms:.3f} ms", flush=True)
            if ms < best_ms:
                best, best_ms = dict(c), ms
        prob.set_sweep_tiling(dtype, k, mode=mode, **best)
        out[name] = dict(best, ms=best_ms, timed=timed, total=len(cands))
    return out


def fwd_candidates(n):
    """Valid tilings of the single nonlinear forward sweep."""
    out = []
    for ntiles in (1, 2, 4, 8, 16, 32, 64, 128):
        tile = -(-n // ntiles)
        if tile < 16:
            continue
        for steps in (4, 8, 12, 16, 25, 32, 50):
            region = tile + 2 * (4 * steps + 4)
            if region > 3 * tile + 64:
                continue
            for ppt in (1, 2, 4, 8):
                threads = -(-region // ppt)
                threads = -(-threads // 64) * 64
                if 64 <= threads <= 1024:
                    out.append(dict(ppt=ppt, kc=1, threads=threads, tile=tile, steps=steps, xch=rp4d.XCH_LDS))
    out.extend(wave_candidates(n, ((1, 1), (2, 1), (4, 1), (8, 1))))
    return out


def tune_fwd(prob, traj, x0, reps=2, budget_s=10.0, verbose=False):
    """Search the forward sweep's tiling (timing rp4d_fwd from x0 into traj);
    applies the best and returns it with its time."""
    op = lambda: prob.fwd(x0, traj, want_J=False)
    prob.set_sweep_tiling(mode=rp4d.MODE_FWD)               # heuristic baseline
    best = dict(prob.get_sweep_tiling(mode=rp4d.MODE_FWD))
    best_ms = _time(op, reps)
    cands = fwd_candidates(prob.n)
    cands.sort(key=lambda c: (-c["steps"], -c["tile"]))
    t_end = time.perf_counter() + budget_s
    timed = 0
    for c in cands:
        if time.perf_counter() > t_end:
            break
        prob.set_sweep_tiling(mode=rp4d.MODE_FWD, **c)
        try:
            ms = _time(op, reps)
        except rp4d.Rp4dError:
            continue
        timed += 1
        if verbose:
            print(f"  fwd {c} {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = dict(c), ms
    prob.set_sweep_tiling(mode=rp4d.MODE_FWD, **{f: best[f] for f in FIELDS})
    return dict(best, ms=best_ms, timed=timed, total=len(cands))


def load_cache(path=CACHE_PATH):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(cache, path=CACHE_PATH):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_cached(prob, nsteps, k, dtype=rp4d.F64, cache=None):
    """Apply a cached tiling for this shape if there is one; returns it or None."""
    cache = load_cache() if cache is None else cache
    ent = cache.get(key(prob.n, nsteps, k, dtype))
    if not ent or "tlm" not in ent or "adj" not in ent:
        return None
    for mode, name in ((rp4d.MODE_TLM, "tlm"), (rp4d.MODE_ADJ, "adj")):
        prob.set_sweep_tiling(dtype, k, mode=mode, **{f: ent[name].get(f, 0) for f in FIELDS})
    if "fwd" in ent:
        prob.set_sweep_tiling(mode=rp4d.MODE_FWD, **{f: ent["fwd"].get(f, 0) for f in FIELDS})
    return ent


def tune_or_load(prob, traj, nsteps, k, dtype=rp4d.F64, budget_s=30.0, cache_path=CACHE_PATH, save=True, x0=None):
    """Apply the cached tilings of this shape or search them.  With k = 1 and an
    initial state x0 the forward sweep's tiling is searched too (kept in the
    same entry)."""
    cache = load_cache(cache_path)
    ent = apply_cached(prob, nsteps, k, dtype, cache)
    if ent is not None and (x0 is None or k != 1 or "fwd" in ent):
        return ent
    best = dict(ent) if ent is not None else tune(prob, traj, k, dtype, budget_s=budget_s)
    if x0 is not None and k == 1:
        best["fwd"] = tune_fwd(prob, traj, x0, budget_s=budget_s / 2)
    cache[key(prob.n, nsteps, k, dtype)] = best
    if save:
        try:
            save_cache(cache, cache_path)
        except OSError:
            pass
    return best



# ---------------------------------------------------------------------------
# Batched sweeps (rp4d_batch_set_tiling): one tiling per (mode, dtype) for the
# whole batch; the tile follows from the region and the halo.
# (ppt, kc) pairs with a batched wave-region instance, and with a batched
# workgroup-region instance
BATCH_WAVE_PK = ((1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2))
BATCH_LDS_PK = ((1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (2, 4), (4, 1), (4, 2))
BATCH_STEPS = (4, 6, 8, 10, 12, 16, 20)


def batch_candidates(dtype=rp4d.F64):
    """Every batched sweep tiling the batch search tries: wave regions with 64,
    128 or 256 threads per workgroup and workgroup regions of 256 or 512
    threads, for every steps-per-launch value whose halo leaves owned points."""
    es = 8 if dtype == rp4d.F64 else 4
    out = []
    for ppt, kc in BATCH_WAVE_PK:
        for steps in BATCH_STEPS:
            if 64 * ppt - 2 * (4 * steps + 4) < 1:
                continue
            for threads in (64, 128, 256):
                out.append(dict(xch=rp4d.XCH_WAVE, ppt=ppt, kc=kc, threads=threads, steps=steps))
    for ppt, kc in BATCH_LDS_PK:
        for threads in (256, 512):
            if threads > (512 if ppt * kc >= 8 else 1024) or 2 * 2 * threads * (1 + kc) * es > LDS_LIMIT:
                continue
            for steps in BATCH_STEPS:
                if threads * ppt - 2 * (4 * steps + 4) < 1:
                    continue
                out.append(dict(xch=rp4d.XCH_LDS, ppt=ppt, kc=kc, threads=threads, steps=steps))
    return out


def batch_key(problems, k, dtype):
    """Cache key of a batch shape: the multiset of (n, nsteps) and k, dtype."""
    import hashlib
    dims = sorted((p.n, int(p.cfg["nsteps"])) for p in problems)
    h = hashlib.sha1(repr(dims).encode()).hexdigest()[:12]
    return f"batch{len(dims)}-{h}-k{k}-{'f64' if dtype == rp4d.F64 else 'f32'}"


def tune_batch(batch, trajs, k, dtype=rp4d.F64, reps=2, budget_s=60.0, verbose=False):
    """Search the batched sweep tiling (one for the TLM and the ADJ sweep of
    rp4d_batch_hessian_block) by timing the batched block Hessian of k vectors
    over the whole batch with each candidate; applies and returns the best
    {"sweep": {...tiling, ms}}.  k = 1 searches the single-vector sweeps' own
    entry (the gradient and PCG products; one vector per group), any other k
    the entry of every sweep.  Candidates are tried cheapest-looking first
    (more steps per launch, larger regions) until the budget is spent."""
    tdtype = torch.float64 if dtype == rp4d.F64 else torch.float32
    Vs = []
    for i, p in enumerate(batch.problems):
        V = torch.empty((p.n, k), dtype=torch.float64, device=p.dev)
        batch.ctx.philox_normal(100 + i, V.numel(), V)
        Vs.append(V.to(tdtype))
    HVs = [torch.empty_like(v) for v in Vs]
    op = lambda: batch.hessian_block(trajs, Vs, HVs)
    kk = 1 if k == 1 else 0
    for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
        batch.set_tiling(mode, dtype, k=kk)                    # library default
    best, best_ms = None, _time(op, reps)
    cands = [c for c in batch_candidates(dtype) if kk == 0 or c["kc"] == 1]
    cands.sort(key=lambda c: (-c["steps"] * c["ppt"], -c["kc"], c["threads"]))
    t_end = time.perf_counter() + budget_s
    for c in cands:
        if time.perf_counter() > t_end:
            break
        for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
            batch.set_tiling(mode, dtype, k=kk, **c)
        try:
            ms = _time(op, reps)
        except rp4d.Rp4dError:                                 # e.g. a staged group beyond the ring
            continue
        if verbose:
            print(f"batch {c} {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = dict(c), ms
    for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
        if best is None:
            batch.set_tiling(mode, dtype, k=kk)
        else:
            batch.set_tiling(mode, dtype, k=kk, **best)
    return {"sweep": dict(best or {}, ms=best_ms, default=best is None)}


def apply_cached_batch(batch, k, dtype=rp4d.F64, cache=None):
    cache = load_cache() if cache is None else cache
    ent = cache.get(batch_key(batch.problems, k, dtype))
    if not ent or "sweep" not in ent:
        return None
    t = {f: ent["sweep"].get(f, 0) for f in ("xch", "ppt", "kc", "threads", "steps")}
    for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
        batch.set_tiling(mode, dtype, k=1 if k == 1 else 0, **t)
    return ent


def tune_batch_or_load(batch, trajs, k, dtype=rp4d.F64, budget_s=60.0, cache_path=CACHE_PATH, save=True,
                       verbose=False):
    cache = load_cache(cache_path)
    ent = apply_cached_batch(batch, k, dtype, cache)
    if ent is not None:
        return ent
    best = tune_batch(batch, trajs, k, dtype, budget_s=budget_s, verbose=verbose)
    cache[batch_key(batch.problems, k, dtype)] = best
    if save:
        try:
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best
