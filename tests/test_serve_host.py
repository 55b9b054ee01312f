"""Host logic of the serving loop (no GPU): the Poisson trace, the workload mix,
the footprint estimate and the admission budget."""
import numpy as np
import pytest

from paper_2401_15758_amd import inputs
from paper_2401_15758_amd import serve


def test_trace_is_poisson_with_the_stated_mix():
    tr = serve.make_trace(4000, rate=2.0, seed=3)
    gaps = np.diff([0.0] + [r.arrival for r in tr])
    assert np.all(gaps >= 0)
    assert np.mean(gaps) == pytest.approx(0.5, rel=0.05)          # exponential, mean 1/rate
    assert np.std(gaps) == pytest.approx(0.5, rel=0.08)
    frac = np.mean([r.model == "burgers" for r in tr])
    assert frac == pytest.approx(0.7, abs=0.03)
    for r in tr[:200]:
        c = r.cfg
        if r.model == "burgers":
            assert 512 <= c["n"] <= 8192 and 100 <= c["nsteps"] <= 500 and c["ell"] == 32
            assert 4 * c["nu"] * c["dt"] * c["n"] ** 2 <= 2.785 + 1e-12     # RK4-stable step
        else:
            assert c["nx"] % 16 == 0 and 128 <= c["nx"] <= 512 and 100 <= c["nsteps"] <= 300 and c["ell"] == 100


def test_trace_at_rate_zero_arrives_at_once_and_is_seeded():
    a = serve.make_trace(10, 0.0, seed=1)
    b = serve.make_trace(10, 0.0, seed=1)
    assert all(r.arrival == 0.0 for r in a)
    assert [(r.cfg["name"], r.seed) for r in a] == [(r.cfg["name"], r.seed) for r in b]


def test_footprint_covers_trajectory_and_grows_with_size():
    b1 = inputs.burgers_config(1024, 200, 4, 10, ell=32)
    b2 = inputs.burgers_config(4096, 200, 4, 10, ell=32)
    assert serve.footprint_bytes(b2) > serve.footprint_bytes(b1) >= 8 * 1024 * 201
    v = inputs.bve_config(256, nsteps=200, obs_stride=16, obs_every=20, ell=100)
    # states + 7 stage fields per step dominate: > 8 n (N+1) + 56 n N
    assert serve.footprint_bytes(v) > 8 * 65536 * 201 + 56 * 65536 * 200


def test_budget_admits_until_full_then_one_oversize_alone():
    bud = serve._Budget(100)
    assert bud.try_take(60) and not bud.try_take(50) and bud.try_take(40)
    bud.give(60)
    bud.give(40)
    assert bud.try_take(500)          # an oversize request runs alone rather than never
    assert not bud.try_take(1)
