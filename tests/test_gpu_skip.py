"""Static-tile skip (TETE_F_SKIP_STATIC): a grid that leaves out the two-step
kernel's tiles lying wholly in PEC gives the same fields, wake and witness
wakes as a grid that steps every tile, over odd step counts, new fields and
geometry mid-run, changed tilings and both precisions; the table's count of
static tiles matches one derived on the CPU from the oracle's PEC edges."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_1053_amd import inputs, tete

pytestmark = pytest.mark.gpu

DZ = 1.0e-3


JC = 14   # the pipe's axis and the bunch: node (nx // 2, JC)


def _pipe_cells(nx, ny, nz, r_cells, seed=0):
    """Metal block with a round pipe along z (radius r_cells about node
    (nx // 2, JC)) and a few random metal cells: the tiles away from the
    pipe are wholly metal, the pipe's are not."""
    i = np.arange(nx)[:, None] + 0.5 - nx // 2
    j = np.arange(ny)[None, :] + 0.5 - JC
    metal = (i * i + j * j) > r_cells * r_cells
    cells = np.repeat(metal[:, :, None], nz, axis=2)
    extra = inputs.random_cells(nx, ny, nz, seed, frac=0.03)
    return (cells | extra.astype(bool)).astype(np.uint8)


def _grid(shape, precision, skip, cells, fields_seed, xchunk=0, rows=0, order=0):
    nx, ny, nz = shape
    G = tete.Grid(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ, precision=precision, skip_static=skip)
    if xchunk or rows or order:
        G.set_tuning("fused2", rows, xchunk, 0, order)
    G.set_pec_cells(cells)
    G.set_fields(inputs.random_fields(G.shape, fields_seed))
    G.set_bunch(1e-9, 2e-3, nx // 2, JC, 10, -14, 40)
    return G


def _same(a, b):
    fa, fb = a.get_fields(), b.get_fields()
    for k in tete.KEYS:
        assert np.array_equal(fa[k], fb[k]), k
    assert np.array_equal(a.wake(), b.wake())


SHAPE = (40, 61, 150)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("xchunk,rows,order", [(0, 0, 0), (8, 0, 0), (5, 16, 2), (11, 32, 1), (7, 0, 4),
                                               (3, 0, 6)])
def test_skip_matches_full(precision, xchunk, rows, order):
    """15 steps (seven two-step launches and one single step) with a bunch:
    the same fields and wake as the grid without the skip, over tilings and
    tile orders."""
    if rows == 32 and precision == "fp64":
        pytest.skip("32-row tiles are FP32 only")
    print("skip", precision, xchunk, rows, order, flush=True)
    cells = _pipe_cells(*SHAPE, 6, seed=81)
    A = _grid(SHAPE, precision, True, cells, 82, xchunk, rows, order)
    B = _grid(SHAPE, precision, False, cells, 82, xchunk, rows, order)
    A.step(15)
    B.step(15)
    assert A.get_tuning()["kernel"] in ("fused2", "auto")
    skipped, total = A.static_tiles()
    assert 0 < skipped < total
    _same(A, B)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_skip_history(precision):
    """Other geometry, fields and steps first, then new geometry and fields,
    a change of x-chunk mid-run and new fields again: the same as a grid
    without the skip given the same calls."""
    print("skip history", precision, flush=True)
    c1 = _pipe_cells(*SHAPE, 4, seed=83)
    c2 = _pipe_cells(*SHAPE, 7, seed=84)
    grids = []
    for skip in (True, False):
        G = _grid(SHAPE, precision, skip, c1, 85, xchunk=6)
        G.step(6)
        G.set_pec_cells(c2)
        G.set_fields(inputs.random_fields(G.shape, 86))
        G.step(5)
        G.set_tuning("fused2", 0, 13)
        G.step(6)
        G.set_fields(inputs.random_fields(G.shape, 87))
        G.step(4)
        grids.append(G)
    _same(*grids)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_skip_with_witness(precision):
    """Witness lines with the skip, first in the pipe, then moved into the
    metal block, where they lie in static tiles that store no witness values
    (the lines must not keep the earlier lines' values): fields and witness
    wakes match the grid without the skip."""
    print("skip witness", precision, flush=True)
    cells = _pipe_cells(*SHAPE, 6, seed=88)
    A = _grid(SHAPE, precision, True, cells, 89, xchunk=5)
    B = _grid(SHAPE, precision, False, cells, 89, xchunk=5)
    for iw, steps in ((SHAPE[0] // 2 + 2, 12), (SHAPE[0] // 2 + 16, 10)):
        for G in (A, B):
            G.set_witness(iw, JC)
            G.step(steps)
        _same(A, B)
        for a, b in zip(A.witness_wake(), B.witness_wake()):
            assert np.array_equal(a, b), iw
    assert A.static_tiles()[0] > 0
    assert np.abs(B.witness_wake()[0]).max() == 0.0   # the second lines lie in the metal


def _expected_static(shape, cells, precision, rows, xchunk):
    """Tiles whose loaded window (rows and lanes with halos, planes
    max(0, xs-4) .. min(xe+3, nx)) holds only entries whose three e edges
    are PEC or absent, from the oracle's materials (kappa 0 on such edges)."""
    nx, ny, nz = shape
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    m = O.vacuum_materials(g, cells)
    s = (m["ex"] == 0) & (m["ey"] == 0) & (m["ez"] == 0)
    r = rows or 16
    lw = 32 if precision == "fp64" or r == 32 else 64
    TY, KT = r - 6, lw - 4
    nyt, nzt, nxc = -(-(ny + 1) // TY), -(-(nz + 1) // KT), -(-(nx + 1) // xchunk)
    count = 0
    for cx in range(nxc):
        xs, xe = cx * xchunk, min(cx * xchunk + xchunk, nx + 1)
        pl = s[max(0, xs - 4):min(xe + 3, nx) + 1].all(axis=0)
        for ty in range(nyt):
            j0, j1 = max(0, ty * TY - 3), min(ny, ty * TY - 3 + r - 1)
            for tz in range(nzt):
                k0, k1 = max(0, tz * KT - 2), min(nz, tz * KT - 2 + lw - 1)
                count += bool(pl[j0:j1 + 1, k0:k1 + 1].all())
    return count, nxc * nyt * nzt


@pytest.mark.parametrize("precision,rows,xchunk", [("fp32", 0, 7), ("fp32", 32, 4), ("fp64", 0, 9)])
def test_static_tile_count(precision, rows, xchunk):
    print("static count", precision, rows, xchunk, flush=True)
    cells = _pipe_cells(*SHAPE, 6, seed=90)
    G = _grid(SHAPE, precision, True, cells, 91, xchunk, rows)
    got = G.static_tiles()
    assert got == _expected_static(SHAPE, cells, precision, rows, xchunk)
    # all metal: every tile; vacuum: none
    G.set_pec_cells(np.ones(SHAPE, np.uint8))
    n = G.static_tiles()
    assert n[0] == n[1] > 0
    G.set_pec_cells(np.zeros(SHAPE, np.uint8))
    assert G.static_tiles()[0] == 0


def test_skip_flag_rules():
    """The flag is refused with Yee's scheme and the implicit scheme;
    static_tiles needs the flag."""
    for kw in ({"yee": True}, {"implicit": True}):
        with pytest.raises(tete.TeteError):
            tete.Grid(8, 8, 8, 2 * DZ, 2 * DZ, DZ, DZ, skip_static=True, **kw)
    G = tete.Grid(8, 8, 8, 2 * DZ, 2 * DZ, DZ, DZ)
    with pytest.raises(tete.TeteError):
        G.static_tiles()


def test_skip_large_case_samples():
    """The large tapered collimator (512 x 512 x 2048, FP32) for 8 steps with
    and without the skip, compared on the device (max |difference| over every
    component must be 0)."""
    import torch
    print("skip large", flush=True)
    case = inputs.large_case()
    res = []
    for skip in (True, False):
        G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision="fp32",
                      skip_static=skip)
        G.set_pec_cells(case.cell_mask())
        G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
        G.step(8)
        if skip:
            sk, tot = G.static_tiles()
            print("static tiles", sk, tot, flush=True)
            assert sk > tot // 2
        res.append((G.get_fields(dtype="fp32", numpy=False), G.wake()))
        del G
        torch.cuda.synchronize()
    (fa, wa), (fb, wb) = res
    for k in tete.KEYS:
        assert torch.equal(fa[k], fb[k]), k
    assert np.array_equal(wa, wb)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_skip_all_static(precision):
    """Every cell metal: once both sets agree no workgroup is launched, and
    the fields (random h, zero e) stay those of the grid without the skip."""
    print("skip all static", precision, flush=True)
    cells = np.ones(SHAPE, np.uint8)
    A = _grid(SHAPE, precision, True, cells, 92, xchunk=9)
    B = _grid(SHAPE, precision, False, cells, 92, xchunk=9)
    A.step(10)
    B.step(10)
    n = A.static_tiles()
    assert n[0] == n[1] > 0
    _same(A, B)


def test_skip_large_full_run():
    """The large tapered collimator run until the bunch has left the grid
    (2243 steps, FP32, wake window around the bunch) with and without the
    skip: the same wake and field energy, bitwise."""
    from tests import parity as P
    case = inputs.large_case()
    M = case.M
    jmin, jmax = -M - 8, M + 8
    nw = jmax - jmin + 1
    steps = case.nz + M + jmax + 1
    out = []
    for skip in (True, False):
        print("skip large full run", skip, steps, flush=True)
        G = P.gpu_grid(case, "fp32", skip_static=skip)
        G.set_bunch(case.Q, case.sigma, case.i0, case.j0, M, jmin, nw)
        G.step(steps)
        out.append((G.wake(), G.energy()[0]))
        G.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
    assert np.any(out[0][0] != 0.0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_skip_grid_in_batch(precision):
    """A skip grid stepped alone, then in a batch (which steps every tile),
    then alone again matches a grid without the skip given the same calls."""
    print("skip batch", precision, flush=True)
    cells = _pipe_cells(*SHAPE, 6, seed=93)
    grids = []
    for skip in (True, False):
        G = _grid(SHAPE, precision, skip, cells, 94, xchunk=6)
        G.step(6)
        B = tete.Batch(precision)
        B.set(0, G)
        B.step(7)
        B.close()
        G.step(8)
        grids.append(G)
    assert grids[0].steps_done() == 21
    _same(*grids)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_skip_matches_oracle(precision):
    """The skip grid against the oracle directly: 15 steps with a bunch on
    the mostly-metal grid, fields within 1e-12 (FP64) / 2e-5 (FP32) and the
    wake within the paper's delta norm 1e-12 / 1e-5."""
    from tests import parity as P
    print("skip oracle", precision, flush=True)
    nx, ny, nz = SHAPE
    cells = _pipe_cells(*SHAPE, 6, seed=95)
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    m = O.vacuum_materials(g, cells)
    f = inputs.random_fields(g.shape, 96)
    O.apply_pec(g, m, f)
    b = O.Bunch(Q=1e-9, sigma=2e-3, i0=nx // 2, j0=JC, M=10, jmin=-14, nw=40)
    r = O.run(g, m, f, 15, bunch=b)
    W = r["acc"] / (b.Q * P.EPS0)
    G = _grid(SHAPE, precision, True, cells, 96)
    G.step(15)
    assert G.static_tiles()[0] > 0
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert P.field_rel_err(G.get_fields(), f) <= tol
    assert P.delta_norm(G.wake(), W) <= (1e-12 if precision == "fp64" else 1e-5)


def _skip_materials(precision, skip, cells, seed):
    nx, ny, nz = SHAPE
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    rng = np.random.default_rng(seed)
    m = O.vacuum_materials(g, cells)
    for k in O.KEYS:
        m[k] = np.where(m[k] > 0, m[k] * rng.uniform(0.5, 1.0, size=m[k].shape), 0.0)
    G = tete.Grid(nx, ny, nz, g.dx, g.dy, g.dz, g.cdt, precision=precision, materials=True, skip_static=skip)
    G.set_materials(m)
    G.set_fields(inputs.random_fields(G.shape, seed + 1))
    G.set_bunch(1e-9, 2e-3, nx // 2, JC, 10, -14, 40)
    return G, g, m


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_skip_materials(precision):
    """Per-entry materials (the fused single step): tiles whose kappa is zero
    on every e edge they load are left out.  15 steps with a bunch give the
    fields and wake of the grid without the skip, and fields within 1e-12
    (FP64) / 2e-5 (FP32) of the oracle; new materials mid-run as well."""
    print("skip materials", precision, flush=True)
    cells = _pipe_cells(*SHAPE, 6, seed=97)
    A, g, m = _skip_materials(precision, True, cells, 98)
    B, _, _ = _skip_materials(precision, False, cells, 98)
    assert A.get_tuning()["kernel"] == "fused"
    A.step(15)
    B.step(15)
    sk, tot = A.static_tiles()
    assert 0 < sk < tot
    _same(A, B)
    f = inputs.random_fields(g.shape, 99)
    O.apply_pec(g, m, f)
    r = O.run(g, m, f, 15, bunch=O.Bunch(Q=1e-9, sigma=2e-3, i0=SHAPE[0] // 2, j0=JC, M=10, jmin=-14, nw=40))
    C, _, _ = _skip_materials(precision, True, cells, 98)
    C.set_fields(inputs.random_fields(C.shape, 99))
    C.step(15)
    from tests import parity as P
    assert P.field_rel_err(C.get_fields(), f) <= (1e-12 if precision == "fp64" else 2e-5)
    # new materials (another geometry) mid-run
    c2 = _pipe_cells(*SHAPE, 4, seed=100)
    for G in (A, B):
        G2, _, m2 = _skip_materials(precision, False, c2, 101)
        G.set_materials(m2)
        G.step(6)
    _same(A, B)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("rows,depth", [(0, 0), (12, 1), (16, 3)])
def test_skip_single_steps(precision, rows, depth):
    """The fused single step over the active tiles: with the single-step
    kernel chosen, then with probes and an energy sample every 3 steps (the
    samples at odd steps leave single steps between the pairs): fields, wake
    and probe series equal those of the grid without the skip, the energy
    series to the rounding of its FP64 sums (the grid without the skip takes
    its samples inside the paired launches, the skip grid with the energy
    kernel)."""
    print("skip single", precision, rows, depth, flush=True)
    cells = _pipe_cells(*SHAPE, 6, seed=102)
    nx, ny, nz = SHAPE
    probes = [(nx // 2) * (ny + 1) * (nz + 1) + JC * (nz + 1) + k for k in (5, 40, 90)]
    grids = []
    for skip in (True, False):
        G = tete.Grid(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ, precision=precision, skip_static=skip, max_series=64)
        G.set_tuning("fused", rows, 7, depth)
        G.set_pec_cells(cells)
        G.set_fields(inputs.random_fields(G.shape, 103))
        G.set_bunch(1e-9, 2e-3, nx // 2, JC, 10, -14, 40)
        G.step(9)
        G.set_tuning("auto")
        G.set_probes(probes)
        G.set_diagnostics(3)
        G.step(8)
        grids.append(G)
    assert grids[0].static_tiles()[0] > 0
    _same(*grids)
    assert np.array_equal(grids[0].probes(3), grids[1].probes(3))
    ea, eb = grids[0].energy_series(), grids[1].energy_series()
    assert len(ea) == len(eb) > 0
    assert np.max(np.abs(ea - eb)) <= 1e-13 * np.max(np.abs(eb))
