"""Materials by class (tete_set_material_classes): the two-step kernel's class
instance against the oracle and, bitwise, against single materials steps over
the same per-entry values.

The oracle takes per-entry arrays: the test expands the classes by the rule
of the C-ABI (an entry takes its class's kappa and mu; kappa is 0 on the PEC
edges of the staircase geometry and the walls, which are exactly the edges
where the oracle's vacuum kappa is 0; components outside their range are 0)."""
import numpy as np
import pytest

from paper_0901_1053_amd import inputs, tete
from tests import parity as P

pytestmark = pytest.mark.gpu
KEYS = tete.KEYS


def _setup(orc, shape, seed, ncls=5, scale=(0.5, 1.0)):
    nx, ny, nz = shape
    dz = 1e-3
    g = orc.Geom(nx, ny, nz, 2 * dz, 2 * dz, dz, dz)
    cells = inputs.random_cells(nx, ny, nz, seed, frac=0.08)
    cells[nx // 2, ny // 2, :] = 0
    vac = orc.vacuum_materials(g, cells)
    rng = np.random.default_rng(seed)
    vx = [g.dx / (g.dy * g.dz), g.dy / (g.dz * g.dx), g.dz / (g.dx * g.dy)]
    table = np.array([[vx[0], vx[1], vx[2], vx[0], vx[1], vx[2]]] * ncls) * rng.uniform(*scale, size=(ncls, 6))
    cls = rng.integers(0, ncls, size=g.shape).astype(np.uint8)
    mat = {k: np.where(vac[k] > 0, table[cls, c], 0.0) for c, k in enumerate(KEYS)}
    return g, cells, cls, table, mat


def _grid(g, cells, precision, cls=None, table=None, mat=None, **kw):
    G = tete.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.cdt, precision=precision, materials=True, **kw)
    G.set_pec_cells(cells)
    if cls is not None:
        G.set_material_classes(cls, table)
    else:
        G.set_materials(mat)
    return G


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(13, 11, 37), (30, 47, 120), (3, 25, 61)])
def test_classes_match_oracle(orc, precision, shape):
    """Random fields, 5 classes on a ragged grid with obstacles, 24 steps (12
    two-step launches): fields within 1e-12 (FP64) / 2e-5 (FP32) of the
    oracle with the expanded materials, and the energy within 1e-12 / 1e-5."""
    print("classes vs oracle", precision, shape, flush=True)
    g, cells, cls, table, mat = _setup(orc, shape, 41)
    f0 = inputs.random_fields(g.shape, 42)
    orc.apply_pec(g, mat, f0)
    G = _grid(g, cells, precision, cls, table)
    assert G.get_tuning()["kernel"] == "fused2"
    G.set_fields(f0)
    G.step(24)
    ref = {k: v.copy() for k, v in f0.items()}
    orc.run(g, mat, ref, 24)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert P.field_rel_err(G.get_fields(), ref) <= tol
    e, _ = G.energy()
    e_ref = orc.energy(g, mat, ref)
    assert abs(e - e_ref) <= (1e-12 if precision == "fp64" else 1e-5) * abs(e_ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_classes_two_step_equals_single_materials_steps(orc, precision):
    """Paired steps of the class instance give bitwise the fields and wake of
    single materials steps over the same per-entry values (an odd step count,
    a bunch through the classes, chunk and tile boundaries)."""
    g, cells, cls, table, mat = _setup(orc, (33, 38, 150), 43)
    out = []
    for use_cls in (True, False):
        G = _grid(g, cells, precision, cls if use_cls else None, table, None if use_cls else mat)
        if not use_cls:
            G.set_tuning("fused")      # the arrays hold few tuples: force the materials step
        G.set_fields(inputs.random_fields(g.shape, 44))
        G.set_bunch(1e-9, 3e-3, g.nx // 2, g.ny // 2, 18, -20, 120)
        assert G.get_tuning()["kernel"] == ("fused2" if use_cls else "fused")
        G.step(31)
        out.append((G.get_fields(), G.wake()))
        G.close()
    for k in KEYS:
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
    assert np.array_equal(out[0][1], out[1][1])
    assert np.any(out[0][1] != 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_classes_wake_against_oracle(orc, precision):
    """A bunch through random classes: the wake within the delta norm 1e-12
    (FP64) / 1e-5 (FP32) of the oracle."""
    case = inputs.scaled_wake_case(24, 120, seed=45, sigma_dz=2.5)
    g = orc.Geom(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt)
    cells = case.cell_mask()
    vac = orc.vacuum_materials(g, cells)
    rng = np.random.default_rng(46)
    table = np.array([[vac[k].max() for k in KEYS]] * 4) * rng.uniform(0.6, 1.0, size=(4, 6))
    cls = rng.integers(0, 4, size=g.shape).astype(np.uint8)
    cls[case.i0, case.j0, :] = 0
    mat = {k: np.where(vac[k] > 0, table[cls, c], 0.0) for c, k in enumerate(KEYS)}
    steps = case.steps
    b = orc.Bunch(Q=case.Q, sigma=case.sigma, i0=case.i0, j0=case.j0, M=case.M, jmin=case.jmin, nw=case.nw)
    f = orc.zeros(g)
    W_ref = orc.run(g, mat, f, steps, bunch=b)["acc"] / (case.Q * P.EPS0)
    G = _grid(g, cells, precision, cls, table)
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.step(steps)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert P.delta_norm(G.wake(), W_ref) <= tol


def test_classes_with_diagnostics_and_skip(orc):
    """Energy samples every 3 steps (single steps in between) and the
    static-tile skip leave the fields and energy series bitwise those of the
    same classes without either."""
    g, cells, cls, table, mat = _setup(orc, (20, 70, 300), 47)
    cells[:, :45, :] = 1                     # a block of metal: static tiles
    vac = orc.vacuum_materials(g, cells)
    mat = {k: np.where(vac[k] > 0, table[cls, c], 0.0) for c, k in enumerate(KEYS)}
    f0 = inputs.random_fields(g.shape, 48)
    res = []
    for skip, diag in ((False, 0), (True, 0), (False, 3)):
        G = _grid(g, cells, "fp32", cls, table, max_series=64, skip_static=skip)
        G.set_fields(f0)
        if diag:
            G.set_diagnostics(diag)
        G.step(17)
        res.append(G.get_fields())
        if skip:
            assert G.static_tiles()[0] > 0
        G.close()
    for r in res[1:]:
        for k in KEYS:
            assert np.array_equal(r[k], res[0][k]), k
    ref = {k: v.copy() for k, v in f0.items()}
    orc.apply_pec(g, mat, ref)
    orc.run(g, mat, ref, 17)
    assert P.field_rel_err(res[0], ref) <= 2e-5


def test_class_rules(orc):
    """Class bytes beyond the table, negative or non-finite table values and
    unstable tables are refused and change nothing; grids without the
    materials flag refuse classes; new geometry drops them."""
    g, cells, cls, table, mat = _setup(orc, (9, 8, 17), 49, ncls=3)
    G = _grid(g, cells, "fp64", cls, table)
    G.set_fields(inputs.random_fields(g.shape, 50))
    G.step(4)
    before = G.get_fields()
    bad_cls = cls.copy()
    bad_cls[2, 3, 4] = 3
    for c, t, status in ((bad_cls, table, "TETE_ERR_ARG"), (cls, -table, "TETE_ERR_ARG"),
                         (cls, np.where(table > 0, np.nan, table), "TETE_ERR_ARG"),
                         (cls, 1.5 * table, "TETE_ERR_UNSTABLE")):
        with pytest.raises(tete.TeteError) as e:
            G.set_material_classes(c, t)
        assert e.value.status == status
    after = G.get_fields()
    for k in KEYS:
        assert np.array_equal(before[k], after[k])
    H = tete.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.cdt)
    with pytest.raises(tete.TeteError) as e:
        H.set_material_classes(cls, table)
    assert e.value.status == "TETE_ERR_STATE"
    G.set_pec_cells(cells)
    assert G.get_tuning()["kernel"] == "fused2"
