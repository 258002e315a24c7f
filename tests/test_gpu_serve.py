"""Serving on the GPU: a Poisson stream of wake requests served by continuous
batching; every result equals the same request solved alone (bitwise, FP32),
FP32 wakes stay within 1e-5 (delta norm) of FP64 solo solves, and the
autotuner's cached shape is used."""
import numpy as np
import pytest

from paper_0901_1053_amd import inputs, serve, tete
from paper_0901_1053_amd.autotune import Tuner
from tests import parity as P

pytestmark = pytest.mark.gpu


def _cases(n, seed=11):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nt = int(rng.choice([16, 24, 32]))
        nz = int(rng.choice([48, 64, 96, 128]))
        out.append(inputs.scaled_wake_case(nt, nz, seed=seed + i, sigma_dz=float(rng.uniform(2.0, 4.0))))
    return out


def _solo(case, precision):
    G = P.gpu_grid(case, precision)
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.step(case.steps)
    return G.wake()


def test_served_equals_alone_and_fp64(tmp_path):
    cases = _cases(10)
    # the two-step kernel's shapes, which FP32 batch members then run with
    tuner = Tuner(cache_path=str(tmp_path / "tune.json"), xchunks=(0, 32), orders=(1, 2), steps=2, warmup=1,
                  kernel="fused2", batch=2)
    for c in cases[:2]:
        tuner.tune(c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.cdt, "fp32")
    assert (tmp_path / "tune.json").exists()
    reqs = serve.make_requests(cases, rate=400.0, seed=12)
    ex = serve.GpuExecutor("fp32", batch=True, graph_steps=8, tuner=tuner)
    st = serve.Server(ex, max_slots=4, block_steps=32).run(reqs)
    ex.close()
    assert st.completed == len(cases)
    assert st.max_active >= 2                        # requests overlapped on the device
    for r in reqs:
        assert np.array_equal(r.wake, _solo(r.case, "fp32")), r.rid
    for r in reqs[:4]:
        w64 = _solo(r.case, "fp64")
        assert P.delta_norm(r.wake, w64) <= 1e-5


def test_one_at_a_time_baseline_fp64():
    cases = _cases(3, seed=21)
    reqs = serve.make_requests(cases, rate=100.0, seed=22)
    ex = serve.GpuExecutor("fp64", batch=False)
    st = serve.Server(ex, max_slots=1, block_steps=10 ** 6).run(reqs)
    ex.close()
    assert st.completed == 3 and st.max_active == 1
    for r in reqs:
        assert np.array_equal(r.wake, _solo(r.case, "fp64"))


def test_arrival_during_a_long_solve_is_admitted_before_it_completes():
    """A request that arrives while a long solve is on the device is admitted
    at the next block boundary (the executor keeps one block in flight), so it
    runs beside the long solve and finishes first; its wake is the one it
    gets alone."""
    big = inputs.scaled_wake_case(192, 1024, seed=3)
    small = inputs.scaled_wake_case(24, 64, seed=4, sigma_dz=2.0)
    reqs = [serve.Request(0, big, 0.0), serve.Request(1, small, 0.2)]
    ex = serve.GpuExecutor("fp32", batch=True, graph_steps=8)
    st = serve.Server(ex, max_slots=4, block_steps=64).run(reqs)
    ex.close()
    b, s = reqs
    print("big admitted %.3f done %.3f; small arrival %.3f admitted %.3f done %.3f"
          % (b.admitted, b.done, s.arrival, s.admitted, s.done), flush=True)
    assert st.completed == 2 and st.max_active == 2
    assert b.admitted <= s.arrival < b.done            # the long solve is running when it arrives
    assert s.arrival <= s.admitted < b.done             # admitted before the long solve completes
    assert s.done < b.done
    assert np.array_equal(s.wake, _solo(small, "fp32"))
    assert np.array_equal(b.wake, _solo(big, "fp32"))
