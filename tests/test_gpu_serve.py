"""GPU tests of the serving loop: each request's result is bitwise the same
served in a mix (continuous batching, concurrent 2-D lanes, sketch reuse) and
alone; admission never holds more than the budget; the footprint estimate
bounds the device memory a request actually holds."""
import numpy as np
import pytest

from gpu_util import need_gpu
from paper_2401_15758_amd import inputs, serve

pytestmark = pytest.mark.gpu

SMALL_MIX = dict(burgers_n=(256, 700), burgers_N=(40, 80), bve_nx=(32, 48), bve_N=(20, 40))


@pytest.mark.parametrize("sketch", ["f64", "f32"])
def test_alone_and_in_mix_bitwise(sketch):
    """Served in a mix and alone, every request ends bitwise the same, with FP64
    sketch sweeps and with FP32 ones (the mixed-precision served form); every
    GN step's PCG meets the tolerance."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    dt = rp4d.F64 if sketch == "f64" else rp4d.F32
    trace = serve.make_trace(8, rate=40.0, seed=11, frac_burgers=0.65, **SMALL_MIX)
    assert {r.model for r in trace} == {"burgers", "bve"}
    mixed = serve.serve(serve.clone_trace(trace), sketch_dtype=dt)
    for r in mixed:
        assert r.gn_done == 3 and len(r.J) == 3 and r.J[-1] < r.J[0]
        assert len(r.relres) == 3 and max(r.relres) <= 1e-6, r.cfg["name"]
        alone = serve.serve([serve.Request(rid=r.rid, cfg=dict(r.cfg), arrival=0.0, seed=r.seed)], sketch_dtype=dt)[0]
        assert np.array_equal(alone.x, r.x), r.cfg["name"]
        assert alone.pcg_iters == r.pcg_iters and alone.reused == r.reused


def test_served_and_sequential_reach_the_same_cost():
    """The served mixed-precision path and the plain FP64 one-at-a-time path
    solve each GN step to the same PCG tolerance, so after three GN steps each
    request's cost J agrees to well within the tolerance's effect."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    trace = serve.make_trace(8, rate=0.0, seed=13, frac_burgers=0.65, **SMALL_MIX)
    served = serve.serve(serve.clone_trace(trace), sketch_dtype=rp4d.F32)
    seq = serve.serve_sequential(serve.clone_trace(trace))
    cmp = serve.compare(served, seq)
    assert max(cmp["relres_final_max"]) <= 1e-6
    assert cmp["J_final_reldiff_max"] <= 1e-6


def test_cancellation_leaves_other_requests_unchanged():
    """One request cancelled while queued and one after its first GN step: the
    first is never admitted, the second ends with its state after one step
    (bitwise that of the same request served alone for one step), and every
    other request ends bitwise as in the run without cancellations."""
    need_gpu()
    import math
    trace = serve.make_trace(6, rate=0.0, seed=14, frac_burgers=0.65, **SMALL_MIX)
    base = {r.rid: r for r in serve.serve(serve.clone_trace(trace))}
    tr = serve.clone_trace(trace)
    burg = [r for r in tr if r.model == "burgers"]
    bve = [r for r in tr if r.model == "bve"]
    queued, mid = burg[0], (bve or burg[1:])[0]
    queued.cancel_at = 0.0
    mid.cancel_after = 1
    done = {r.rid: r for r in serve.serve(tr)}
    assert done[queued.rid].cancelled and done[queued.rid].gn_done == 0 and done[queued.rid].x is None
    m = done[mid.rid]
    assert m.cancelled and m.gn_done == 1
    one = serve.serve([serve.Request(rid=mid.rid, cfg=dict(mid.cfg), arrival=0.0, seed=mid.seed)], gn_steps=1)[0]
    assert np.array_equal(one.x, m.x)
    for rid, r in done.items():
        if rid in (queued.rid, mid.rid):
            continue
        assert not r.cancelled and r.gn_done == 3
        assert np.array_equal(r.x, base[rid].x), r.cfg["name"]
    s = serve.summary(list(done.values()))
    assert s["cancelled"] == 2 and s["requests"] == len(trace) - 2 and math.isfinite(s["p99_latency_s"])


def test_admission_respects_budget():
    need_gpu()
    trace = serve.make_trace(10, rate=0.0, seed=12, frac_burgers=0.8, **SMALL_MIX)
    fps = {r.rid: serve.footprint_bytes(r.cfg) for r in trace}
    budget = int(2.5 * max(fps.values()))
    done = serve.serve(serve.clone_trace(trace), budget_bytes=budget)
    events = sorted({r.admitted for r in done} | {r.done for r in done})
    for t in events:
        held = sum(fps[r.rid] for r in done if r.admitted <= t < r.done)
        assert held <= budget
    assert all(r.gn_done == 3 for r in done)


@pytest.mark.parametrize("which", ["burgers", "bve"])
def test_footprint_estimate_bounds_device_memory(which):
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    cfg = (inputs.burgers_config(2048, 200, 4, 10, ell=32) if which == "burgers"
           else inputs.bve_config(64, nsteps=60, obs_stride=16, obs_every=20, ell=100))
    req = serve.Request(rid=0, cfg=cfg, arrival=0.0, seed=5)
    torch.cuda.synchronize()
    free0, res0 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    ctx = rp4d.Context(0)
    p, st = serve._setup(rp4d, torch, ctx, req)
    p.gn_step(st, ell=cfg["ell"], seed=1, rtol=1e-6)
    torch.cuda.synchronize()
    free1, res1 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    held = (free0 - free1) - (res1 - res0)        # library allocations only
    est = serve.footprint_bytes(cfg)
    assert 0 < held <= est, (held, est)
    assert est <= 3 * held + (64 << 20)           # not uselessly loose
    st.close()
    p.close()
