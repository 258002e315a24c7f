"""The two-step (temporally blocked) fused kernel: two steps per launch must give
exactly the fields and wake of two single fused steps, for every launch shape
(tile and chunk boundaries everywhere, the bunch line on and off tile edges),
with diagnostics that force single steps in between, and within the FP32
tolerance of the FP64 oracle."""
import numpy as np
import pytest

from paper_0901_1053_amd import inputs, tete
from tests import parity as P

pytestmark = pytest.mark.gpu

SHAPES = [(13, 11, 37), (40, 29, 130), (7, 70, 200), (2, 2, 2), (3, 25, 61), (9, 20, 1000)]


def _grid(shape, seed, kernel, xchunk=0, order=0, precision="fp32", **kw):
    nx, ny, nz = shape
    G = tete.Grid(nx, ny, nz, 2.0e-3, 1.7e-3, 1.0e-3, 0.9e-3, precision=precision, **kw)
    G.set_pec_cells(inputs.random_cells(nx, ny, nz, seed, frac=0.1))
    G.set_tuning(kernel, 0, xchunk, 0, order)
    assert G.get_tuning()["kernel"] == kernel
    G.set_fields(inputs.random_fields(G.shape, seed))
    return G


def _fields(shape, seed, kernel, steps, xchunk=0, order=0):
    G = _grid(shape, seed, kernel, xchunk, order)
    G.step(steps)
    return G.get_fields()


def _same(a, b):
    for k in tete.KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("shape", SHAPES)
def test_two_steps_equal_single_steps(shape):
    for steps in (2, 25):
        _same(_fields(shape, 31, "fused2", steps), _fields(shape, 31, "fused", steps))


@pytest.mark.parametrize("xchunk,order", [(1, 2), (2, 1), (3, 3), (5, 4), (7, 0), (1000, 2), (0, 4), (0, 1), (4, 5), (0, 6)])
def test_launch_shape_invariance(xchunk, order):
    shape = (40, 29, 1000)
    base = _fields(shape, 32, "fused", 12)
    _same(_fields(shape, 32, "fused2", 12, xchunk, order), base)


def _wake_run(case, kernel, steps, jmin, nw, precision="fp32", xchunk=0, diag=0, probes=None):
    G = P.gpu_grid(case, precision, max_series=steps + 16)
    if kernel != "auto":
        G.set_tuning(kernel, 0, xchunk, 0, 0)
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, jmin, nw)
    if diag:
        G.set_diagnostics(diag)
    if probes is not None:
        G.set_probes(probes)
    G.step(steps)
    return G


@pytest.mark.parametrize("nt,nz,xchunk", [(24, 150, 0), (32, 200, 3), (16, 130, 1), (40, 96, 7)])
def test_wake_identical_to_single_steps(nt, nz, xchunk):
    """Injection and the paired wake update: bitwise the single-step wake
    (nt = 32 puts the bunch row on a tile edge, nt = 24 inside a tile)."""
    case = inputs.scaled_wake_case(nt, nz, seed=nt + nz, sigma_dz=3.0)
    M = case.M
    jmin, nw = -M - 3, 2 * M + 40
    steps = case.nz + M + jmin + nw
    for s in (steps, steps + 1):
        a = _wake_run(case, "fused2", s, jmin, nw, xchunk=xchunk)
        b = _wake_run(case, "fused", s, jmin, nw)
        assert np.array_equal(a.wake(), b.wake())
        _same(a.get_fields(), b.get_fields())


def test_wake_within_tolerance_of_oracle():
    case = inputs.scaled_wake_case(24, 150, seed=9, sigma_dz=3.0)
    M = case.M
    jmin, nw = -M - 3, 2 * M + 40
    steps = case.nz + M + jmin + nw
    ref = P.oracle_wake(case, steps, jmin=jmin, nw=nw)
    W = _wake_run(case, "fused2", steps, jmin, nw).wake()
    assert P.delta_norm(W, ref["W"]) <= 1e-5


def test_diagnostics_force_single_steps():
    """An energy sample every 3 steps (odd, so pairs must break) and, in a
    second run, probes every step: the series equal those of single steps."""
    case = inputs.scaled_wake_case(24, 100, seed=4, sigma_dz=3.0)
    jmin, nw = -case.M, 2 * case.M + 20
    steps = 40
    a = _wake_run(case, "fused2", steps, jmin, nw, diag=3)
    b = _wake_run(case, "fused", steps, jmin, nw, diag=3)
    assert np.array_equal(a.energy_series(), b.energy_series())
    assert np.array_equal(a.wake(), b.wake())
    idx = np.array([5, 1000, 20000], dtype=np.int64)
    a = _wake_run(case, "fused2", steps, jmin, nw, probes=idx)
    b = _wake_run(case, "fused", steps, jmin, nw, probes=idx)
    assert np.array_equal(a.probes(3), b.probes(3))
    _same(a.get_fields(), b.get_fields())


def test_timing_counts_steps():
    G = _grid((20, 20, 300), 3, "fused2")
    G.set_timing(16)
    G.step(7)                      # three two-step launches and one single step
    ms, _, n = G.timing()
    assert n == 7 and ms > 0


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_materials_kernel_choice(precision):
    """Per-entry arrays with many tuples: FP32 pairs steps in the two-step
    kernel's arrays instance; FP64 falls back to the single step's materials
    instance and refuses a forced two-step kernel."""
    G = tete.Grid(8, 8, 40, 2.0e-3, 1.7e-3, 1.0e-3, 0.9e-3, precision=precision, materials=True)
    G.set_tuning("fused2")
    assert G.get_tuning()["kernel"] == "fused2"
    rng = np.random.default_rng(0)
    G.set_materials({k: rng.uniform(0.5, 1.0, G.shape) for k in tete.KEYS})
    assert G.get_tuning()["kernel"] == ("fused2" if precision == "fp32" else "fused")
    G.set_tuning("split")
    assert G.get_tuning()["kernel"] == "split"
    if precision == "fp32":
        G.set_tuning("fused2")
        assert G.get_tuning()["kernel"] == "fused2"
    else:
        with pytest.raises(tete.TeteError):
            G.set_tuning("fused2")


@pytest.mark.parametrize("shape", [(13, 11, 37), (40, 29, 130), (2, 2, 2), (9, 20, 1000)])
def test_fp64_two_steps_equal_single_steps(shape):
    """FP64 two-step kernel (two rows per wave): bitwise the single steps."""
    def run(kernel, steps):
        G = _grid(shape, 41, kernel, precision="fp64")
        G.step(steps)
        return G.get_fields()
    for steps in (2, 25):
        _same(run("fused2", steps), run("fused", steps))


@pytest.mark.parametrize("nt,nz,xchunk", [(24, 150, 0), (32, 200, 3)])
def test_fp64_wake_identical_and_oracle(nt, nz, xchunk):
    case = inputs.scaled_wake_case(nt, nz, seed=nt + nz + 1, sigma_dz=3.0)
    M = case.M
    jmin, nw = -M - 3, 2 * M + 40
    steps = case.nz + M + jmin + nw
    a = _wake_run(case, "fused2", steps, jmin, nw, precision="fp64", xchunk=xchunk)
    b = _wake_run(case, "fused", steps, jmin, nw, precision="fp64")
    assert np.array_equal(a.wake(), b.wake())
    _same(a.get_fields(), b.get_fields())
    ref = P.oracle_wake(case, steps, jmin=jmin, nw=nw)
    assert P.delta_norm(a.wake(), ref["W"]) <= 1e-12


@pytest.mark.parametrize("rows,depth", [(32, 0), (24, 0), (24, 1), (24, 3), (16, 2)])
@pytest.mark.parametrize("xchunk", [0, 3])
def test_fp32_other_shapes(rows, depth, xchunk):
    """The other FP32 shapes of the two-step kernel (rows of 32 lanes: 32 rows,
    24 rows with one, two or three planes loaded ahead; 16 rows of 64 lanes with
    two) give the single-step results bitwise, fields and wake."""
    print("fp32 shape", rows, depth, xchunk, flush=True)
    shape = (20, 70, 300)
    G = _grid(shape, 51, "fused2")
    G.set_tuning("fused2", rows, xchunk, depth, 0)
    G.step(13)
    _same(G.get_fields(), _fields(shape, 51, "fused", 13))
    case = inputs.scaled_wake_case(32, 200, seed=77, sigma_dz=3.0)
    M = case.M
    jmin, nw = -M - 3, 2 * M + 40
    steps = case.nz + M + jmin + nw
    a = P.gpu_grid(case, "fp32")
    a.set_tuning("fused2", rows, xchunk, depth, 0)
    a.set_bunch(case.Q, case.sigma, case.i0, case.j0, M, jmin, nw)
    a.step(steps)
    b = _wake_run(case, "fused", steps, jmin, nw)
    assert np.array_equal(a.wake(), b.wake())
    _same(a.get_fields(), b.get_fields())
