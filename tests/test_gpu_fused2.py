"""The two-step (temporally blocked) fused kernel: two steps per launch must give
exactly the fields and wake of two single fused steps, for every launch shape
(tile and chunk boundaries everywhere, the bunch line on and off tile edges),
with probes (their values between a pair's two steps evaluated from the pair's
input) and energy samples taken inside the paired launches, and within the FP32
tolerance of the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
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


def test_diagnostics_and_single_steps():
    """An energy sample every 3 steps (odd: the paired launches take the
    samples between their two steps) and, in a second run, probes every step
    (the steps stay paired; a pair's first-step values come from its input):
    fields, wake and probes equal those of single steps bitwise, the energy
    series to the rounding of its FP64 sums (the paired launch adds the same
    terms in another order)."""
    case = inputs.scaled_wake_case(24, 100, seed=4, sigma_dz=3.0)
    jmin, nw = -case.M, 2 * case.M + 20
    steps = 40
    a = _wake_run(case, "fused2", steps, jmin, nw, diag=3)
    b = _wake_run(case, "fused", steps, jmin, nw, diag=3)
    ea, eb = a.energy_series(), b.energy_series()
    assert len(ea) == len(eb) == 14
    assert np.max(np.abs(ea - eb)) <= 1e-13 * np.max(np.abs(eb))
    assert np.array_equal(a.wake(), b.wake())
    _same(a.get_fields(), b.get_fields())
    idx = np.array([5, 1000, 20000], dtype=np.int64)
    a = _wake_run(case, "fused2", steps, jmin, nw, probes=idx)
    b = _wake_run(case, "fused", steps, jmin, nw, probes=idx)
    assert np.array_equal(a.probes(3), b.probes(3))
    _same(a.get_fields(), b.get_fields())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("materials", [False, True])
def test_probes_in_paired_launches(precision, materials):
    """Probes on the bunch line (its current enters their step), on a PEC
    edge, on the last k (no e_z edge) and inside, over an odd number of steps:
    the series of the paired run equals that of single steps bitwise, and so
    do the fields.  With materials (0.9 x vacuum with PEC zeros, a few
    distinct tuples: the two-step kernel's class instance)."""
    print("probes in pairs", precision, materials, flush=True)
    case = inputs.scaled_wake_case(24, 100, seed=5, sigma_dz=3.0)
    g = P.oracle_geom(case)
    cells = case.cell_mask()
    sp, sz = (case.ny + 1) * (case.nz + 1), case.nz + 1
    line = case.i0 * sp + case.j0 * sz
    m = O.vacuum_materials(g, cells)
    pec = [int(i) for i in np.flatnonzero(m["ez"] == 0) if (i % sz) < case.nz]
    idx = np.array([line + 10, line + 50, line + 90, line + case.nz, pec[len(pec) // 2], 3 * sp + 5 * sz + 40],
                   dtype=np.int64)
    steps = 41
    runs = []
    for kernel in ("auto", "fused"):
        G = P.gpu_grid(case, precision, cells=not materials, materials=materials, max_series=steps + 16)
        if materials:
            G.set_materials({k: 0.9 * v for k, v in m.items()})
        G.set_tuning(kernel)
        G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, -case.M, 2 * case.M + 20)
        G.set_probes(idx)
        G.step(steps)
        runs.append(G)
    pa, pb = runs[0].probes(len(idx)), runs[1].probes(len(idx))
    assert pa.shape == (steps, len(idx))
    assert np.abs(pb[:, :3]).max() > 0
    assert np.array_equal(pa, pb)
    _same(runs[0].get_fields(), runs[1].get_fields())


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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("diag", [1, 2, 3, 5])
def test_energy_samples_in_paired_launches(precision, diag):
    """Energy samples taken inside the two-step launches (of y^n from the
    first stage's input, of y^{n+1} from the second's): every sample against
    the oracle's energy within 1e-12 (FP64) / 1e-5 (FP32) of the largest, and
    against the energy kernel between single steps to its FP64 rounding; the
    fields bitwise those of single steps.  Random fields, obstacles and a
    bunch on a ragged grid, every x-chunk boundary and an odd step count."""
    print("energy in pairs", precision, diag, flush=True)
    nx, ny, nz = 23, 17, 71
    g = O.Geom(nx, ny, nz, 2.0e-3, 1.7e-3, 1.0e-3, 1.0e-3)         # c dt = dz: the bunch moves at c
    cells = inputs.random_cells(nx, ny, nz, 91, frac=0.08)
    m = O.vacuum_materials(g, cells)
    f0 = inputs.random_fields((nx + 1, ny + 1, nz + 1), 92)
    steps = 23
    res = []
    for kernel, xchunk in (("fused2", 0), ("fused2", 5), ("fused", 0)):
        G = tete.Grid(nx, ny, nz, g.dx, g.dy, g.dz, g.cdt, precision=precision, max_series=64)
        G.set_pec_cells(cells)
        G.set_tuning(kernel, 0, xchunk, 0, 0)
        G.set_fields(f0)
        G.set_bunch(1e-9, 2e-3, 11, 8, 10, -12, 40)
        G.set_diagnostics(diag)
        G.step(steps)
        res.append((G.energy_series(), G.get_fields()))
        G.close()
    ref = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, ref)
    b = O.Bunch(Q=1e-9, sigma=2e-3, i0=11, j0=8, M=10, jmin=-12, nw=40)
    e_ref = np.array(O.run(g, m, ref, steps, bunch=b, want_energy=True)["energy"])[::diag]
    tol = 1e-12 if precision == "fp64" else 1e-5
    scale = np.max(np.abs(e_ref))
    for e, f in res:
        assert len(e) == len(e_ref)
        assert np.max(np.abs(e - e_ref)) <= tol * scale
        assert np.max(np.abs(e - res[2][0])) <= 1e-13 * scale
        _same(f, res[2][1])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("diag", [1, 3])
def test_energy_samples_in_paired_launches_with_classes(precision, diag):
    """Materials by class (0.9 and 0.75 of vacuum in the two halves along x,
    PEC zeros: three classes recognised in the per-entry arrays) with energy
    samples, which the paired launches take with each entry's class
    coefficients (FP64: single exchange buffers).  Every sample against
    the oracle within 1e-12 (FP64) / 1e-5 (FP32) of the largest, against the
    energy kernel between single steps to its FP64 rounding; the fields
    bitwise those of single steps."""
    print("energy in pairs, classes", precision, diag, flush=True)
    nx, ny, nz = 23, 17, 71
    g = O.Geom(nx, ny, nz, 2.0e-3, 1.7e-3, 1.0e-3, 1.0e-3)
    cells = inputs.random_cells(nx, ny, nz, 93, frac=0.08)
    m = O.vacuum_materials(g, cells)
    f = np.where(np.arange(nx + 1) < nx // 2, 0.9, 0.75)[:, None, None]
    m = {k: v * f for k, v in m.items()}
    f0 = inputs.random_fields((nx + 1, ny + 1, nz + 1), 94)
    steps = 23
    res = []
    for kernel, xchunk in (("fused2", 0), ("fused2", 5), ("fused", 0)):
        G = tete.Grid(nx, ny, nz, g.dx, g.dy, g.dz, g.cdt, precision=precision, materials=True, max_series=64)
        G.set_materials(m)
        G.set_tuning(kernel, 0, xchunk, 0, 0)
        assert G.get_tuning()["kernel"] == kernel
        G.set_fields(f0)
        G.set_bunch(1e-9, 2e-3, 11, 8, 10, -12, 40)
        G.set_diagnostics(diag)
        G.step(steps)
        res.append((G.energy_series(), G.get_fields()))
        G.close()
    ref = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, ref)
    b = O.Bunch(Q=1e-9, sigma=2e-3, i0=11, j0=8, M=10, jmin=-12, nw=40)
    e_ref = np.array(O.run(g, m, ref, steps, bunch=b, want_energy=True)["energy"])[::diag]
    tol = 1e-12 if precision == "fp64" else 1e-5
    scale = np.max(np.abs(e_ref))
    for e, fl in res:
        assert len(e) == len(e_ref)
        assert np.max(np.abs(e - e_ref)) <= tol * scale
        assert np.max(np.abs(e - res[2][0])) <= 1e-13 * scale
        _same(fl, res[2][1])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("diag", [1, 3])
def test_energy_samples_with_witness_lines(precision, diag):
    """Witness lines and an energy sample every `diag` steps: the paired
    launches keep the lines' e_z^{n+1/2} and take the samples together; the
    witness wakes, the wake and the fields equal those of single steps
    bitwise, the energy series to the rounding of its FP64 sums."""
    print("energy in pairs, witness", precision, diag, flush=True)
    case = inputs.scaled_wake_case(24, 100, seed=6, sigma_dz=3.0)
    jmin, nw = -case.M, 2 * case.M + 20
    steps = 41
    runs = []
    for kernel in ("auto", "fused"):
        G = P.gpu_grid(case, precision, max_series=steps + 16)
        G.set_tuning(kernel)
        G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, jmin, nw)
        G.set_witness(case.i0 + 3, case.j0 - 2)
        G.set_diagnostics(diag)
        G.step(steps)
        runs.append(G)
    a, b = runs
    ea, eb = a.energy_series(), b.energy_series()
    assert len(ea) == len(eb) == (steps + diag - 1) // diag
    assert np.max(np.abs(ea - eb)) <= 1e-13 * np.max(np.abs(eb))
    assert np.array_equal(a.wake(), b.wake())
    wa, wb = a.witness_wake(), b.witness_wake()
    for x, y in zip(wa, wb):
        assert np.array_equal(x, y)
    assert np.abs(wb[0]).max() > 0
    _same(a.get_fields(), b.get_fields())
