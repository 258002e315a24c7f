"""Serving policy on the CPU with a fake-clock executor: first-come-first-served
admission, HBM-footprint budget, slot limit, completion, latency statistics."""
import math

import numpy as np
import pytest

from paper_0901_1053_amd import inputs, serve
from paper_0901_1053_amd.autotune import size_class


def _cases(n, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nt = int(rng.choice([16, 24, 32]))
        nz = int(rng.choice([32, 64, 96]))
        out.append(inputs.scaled_wake_case(nt, nz, seed=seed + i, sigma_dz=2.0))
    return out


def test_poisson_arrivals_are_seeded_and_have_the_rate():
    a = serve.poisson_arrivals(50.0, 4000, 7)
    b = serve.poisson_arrivals(50.0, 4000, 7)
    assert np.array_equal(a, b)
    assert np.all(np.diff(a) > 0)
    assert abs(np.mean(np.diff(a)) - 1 / 50.0) < 0.1 / 50.0


def test_all_served_fifo_and_latency_bounds():
    reqs = serve.make_requests(_cases(40), rate=200.0, seed=1)
    ex = serve.MockExecutor(rate_cells_per_s=2e8)
    st = serve.Server(ex, budget_bytes=10 ** 12, max_slots=8, block_steps=16).run(reqs)
    assert st.completed == 40
    assert st.max_active <= 8
    order = [e[2] for e in ex.log if e[0] == "admit"]
    assert order == sorted(order)                       # first come, first served
    for r in reqs:
        assert r.admitted >= r.arrival - 1e-12
        assert r.done > r.admitted
        assert r.wake is not None and r.wake.shape == (r.case.nw,)
    lat = [r.latency for r in reqs]
    assert st.p50_s == pytest.approx(np.percentile(lat, 50))
    assert st.p99_s == pytest.approx(np.percentile(lat, 99))
    assert st.solves_per_s == pytest.approx(40 / max(r.done for r in reqs))


def test_memory_budget_limits_admission():
    cases = _cases(12)
    ex = serve.MockExecutor(rate_cells_per_s=1e8)
    fp = max(ex.footprint(c) for c in cases)
    reqs = serve.make_requests(cases, rate=1e4, seed=2)     # everything arrives at once
    st = serve.Server(ex, budget_bytes=2 * fp, max_slots=64, block_steps=8).run(reqs)
    assert st.completed == 12
    assert st.peak_bytes <= 2 * fp
    foot = {r.rid: r.footprint for r in reqs}
    used = 0
    for e in ex.log:
        if e[0] == "admit":
            used += foot[e[2]]
        elif e[0] == "finish":
            used -= foot[e[2]]
        assert used <= 2 * fp
    assert st.max_active < len(cases)                 # the budget held requests back


def test_steps_stop_at_each_completion():
    """Each request gets exactly its own step count (completion is detected at
    the step it happens, not at the end of a block)."""
    cases = _cases(6)
    reqs = serve.make_requests(cases, rate=1e4, seed=3)
    ex = serve.MockExecutor()
    taken = {}
    orig = ex.step

    def step(k):
        for slot, r in ex.active.items():
            taken[r.rid] = taken.get(r.rid, 0) + k
        orig(k)
    ex.step = step
    serve.Server(ex, max_slots=4, block_steps=1000).run(reqs)
    for r in reqs:
        assert taken[r.rid] == r.case.steps


def test_request_larger_than_budget_is_rejected():
    reqs = serve.make_requests(_cases(2), rate=10.0, seed=4)
    with pytest.raises(ValueError):
        serve.Server(serve.MockExecutor(), budget_bytes=1000).run(reqs)


def test_idle_server_waits_for_arrivals():
    reqs = serve.make_requests(_cases(3), rate=0.5, seed=6)
    ex = serve.MockExecutor(rate_cells_per_s=1e12)
    st = serve.Server(ex).run(reqs)
    for r in reqs:
        assert r.admitted >= r.arrival
        assert r.latency < 0.1                       # an idle server starts at once
    assert st.completed == 3 and not math.isnan(st.p99_s)


def test_size_classes():
    assert size_class(64, 64, 256, "fp32") == "fp32:64x64x256"
    assert size_class(96, 96, 768, "fp32") == "fp32:128x128x1024"
    assert size_class(65, 64, 256, "fp64") == "fp64:128x64x256"


def test_fifo_completions_by_hand():
    assert serve.fifo_completions([0.0, 0.5, 4.0], [1.0, 2.0, 1.0]) == [1.0, 3.0, 5.0]
    assert serve.fifo_completions([], []) == []


def test_one_at_a_time_model_equals_served_stream():
    """The FIFO model over solve-alone times reproduces what the server does
    with one slot, at a low and a high rate."""
    cases = _cases(10, seed=8)
    ex = serve.MockExecutor(rate_cells_per_s=3e8)
    times, wakes = serve.solve_alone(ex, cases)
    assert len(wakes) == len(cases) and all(w.shape == (c.nw,) for w, c in zip(wakes, cases))
    for rate in (0.5, 500.0):
        reqs = serve.make_requests(cases, rate, seed=9)
        st = serve.Server(serve.MockExecutor(rate_cells_per_s=3e8), max_slots=1, block_steps=10 ** 9).run(reqs)
        model = serve.one_at_a_time_stats([r.arrival for r in reqs], times)
        assert model.completed == st.completed
        assert model.latencies == pytest.approx(st.latencies, rel=1e-9, abs=1e-9)
        assert model.p99_s == pytest.approx(st.p99_s, rel=1e-9)


def test_cell_limit_bounds_work_in_flight():
    """With a cell limit, the cells of the admitted requests never exceed it
    (except a single request larger than the limit, admitted alone), every
    request is served, and order stays first come first served."""
    cases = _cases(16, seed=12)
    cap = int(np.median([c.cells for c in cases]) * 2)
    ex = serve.MockExecutor(rate_cells_per_s=2e8)
    reqs = serve.make_requests(cases, rate=1e4, seed=13)
    st = serve.Server(ex, max_slots=64, block_steps=32, max_cells=cap).run(reqs)
    assert st.completed == len(cases)
    cells = {r.rid: r.case.cells for r in reqs}
    inflight = {}
    for e in ex.log:
        if e[0] == "admit":
            inflight[e[2]] = cells[e[2]]
            assert sum(inflight.values()) <= cap or len(inflight) == 1
        elif e[0] == "finish":
            inflight.pop(e[2])
    order = [e[2] for e in ex.log if e[0] == "admit"]
    assert order == sorted(order)
    assert st.max_active < len(cases)


def test_tuner_keys_and_kernels(tmp_path):
    """The tuner times the fused single step or the two-step kernel; its cache
    keeps shapes apart by kernel and by batch context."""
    from paper_0901_1053_amd.autotune import Tuner
    with pytest.raises(ValueError):
        Tuner(cache_path=None, kernel="split")
    a = Tuner(cache_path=None)
    b = Tuner(cache_path=None, kernel="fused2")
    c = Tuner(cache_path=None, kernel="fused2", batch=8)
    keys = {t._key(96, 96, 768, "fp32") for t in (a, b, c)}
    assert len(keys) == 3
    assert all(k.startswith("fp32:128x128x1024/") for k in keys)
