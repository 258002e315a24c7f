"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle on
the same seeded inputs.  FP64 must agree to 1e-12 relative; the FP32 field path
to 1e-5 relative on the wake (the paper's delta norm, Sec. 5) and the energy."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_1053_amd import inputs
from tests import parity as P
from tests.test_oracle_dispersion import _fit, omega27

pytestmark = pytest.mark.gpu


def _probe_points(g, seed, count=3):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < count:
        p = (int(rng.integers(1, g.nx)), int(rng.integers(1, g.ny)), int(rng.integers(0, g.nz)))
        if p not in pts:
            pts.append(p)
    return [int(np.ravel_multi_index(p, g.shape)) for p in pts]


def test_cavity_fp64_matches_oracle():
    """Vacuum PEC cavity 24x24x48 (dz = 1 mm, dx = dy = 2 mm, c dt = dz), 500 steps,
    three seeded analytic modes: per-step energy, e_z probe traces and the final
    fields agree with the oracle; the energy is conserved; the traces oscillate
    at the frequencies of (27)."""
    case = inputs.cavity_case()
    modes = inputs.seeded_modes(case.seed)
    f0 = inputs.cavity_fields(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, modes)
    g = P.oracle_geom(case)
    m = O.vacuum_materials(g)
    fo = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, fo)
    probes = _probe_points(g, case.seed)
    ref = O.run(g, m, fo, case.steps, want_energy=True, probes=probes)

    G = P.gpu_grid(case, "fp64", cells=False, max_series=case.steps)
    G.set_fields(f0)
    G.set_diagnostics(1)
    G.set_probes(probes)
    G.step(case.steps)
    en = G.energy_series()
    pr = G.probes(len(probes))
    fg = G.get_fields()
    assert len(en) == case.steps and pr.shape == (case.steps, len(probes))
    assert np.max(np.abs(en - ref["energy"])) <= 1e-12 * np.max(np.abs(ref["energy"]))
    assert np.max(np.abs(pr - ref["probes"])) <= 1e-12 * np.max(np.abs(ref["probes"]))
    assert P.field_rel_err(fg, fo) <= 1e-12
    assert np.max(np.abs(en - en[0])) <= 1e-13 * abs(en[0])
    Oms = [omega27(md.m, md.n, md.p, case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt) for md in modes]
    for p in range(len(probes)):
        assert _fit(pr[:, p], Oms) < 1e-9


@pytest.mark.parametrize("shape,seed,precision", [
    ((13, 11, 37), 1, "fp64"), ((5, 70, 9), 2, "fp64"), ((2, 2, 2), 3, "fp64"),
    ((64, 3, 130), 4, "fp64"), ((13, 11, 37), 5, "fp32"), ((33, 17, 65), 6, "fp32")])
def test_random_fields_with_obstacles(shape, seed, precision):
    """Ragged sizes (odd counts, tails that are not multiples of any tile),
    random obstacles and random fields, including out-of-range and PEC entries
    that the library must zero."""
    nx, ny, nz = shape
    g = O.Geom(nx, ny, nz, 2.0e-3, 1.7e-3, 1.0e-3, 0.9e-3)
    cells = inputs.random_cells(nx, ny, nz, seed, frac=0.1)
    m = O.vacuum_materials(g, cells)
    f0 = inputs.random_fields(g.shape, seed)
    fo = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, fo)
    steps = 40
    O.run(g, m, fo, steps)
    from paper_0901_1053_amd import tete
    G = tete.Grid(nx, ny, nz, g.dx, g.dy, g.dz, g.cdt, precision=precision)
    G.set_pec_cells(cells)
    G.set_fields(f0)
    G.step(steps)
    fg = G.get_fields()
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert P.field_rel_err(fg, fo) <= tol
    # entries outside the component ranges stay zero
    masks = P.range_masks(g.shape)
    for k in P.KEYS:
        assert np.all(fg[k][~masks[k]] == 0.0), k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_general_materials(precision):
    """Per-entry diagonal M_eps^-1, M_mu^-1 (random, with PEC zeros).  The factors
    stay at or below vacuum so the local wave speed never exceeds c and the
    step stays inside the stability bound (25)."""
    nx, ny, nz = 9, 10, 21
    g = O.Geom(nx, ny, nz, 2.0e-3, 2.0e-3, 1.0e-3, 0.8e-3)
    rng = np.random.default_rng(11)
    m = O.vacuum_materials(g, inputs.random_cells(nx, ny, nz, 12, frac=0.1))
    for k in O.KEYS:
        m[k] = np.where(m[k] > 0, m[k] * rng.uniform(0.5, 1.0, size=m[k].shape), 0.0)
    f0 = inputs.random_fields(g.shape, 13)
    fo = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, fo)
    e_init = O.energy(g, m, fo)
    O.run(g, m, fo, 30)
    from paper_0901_1053_amd import tete
    G = tete.Grid(nx, ny, nz, g.dx, g.dy, g.dz, g.cdt, precision=precision, materials=True)
    G.set_materials(m)
    G.set_fields(f0)
    G.step(30)
    tol = 1e-12 if precision == "fp64" else 2e-5
    assert P.field_rel_err(G.get_fields(), fo) <= tol
    e_gpu, _ = G.energy()
    e_ref = O.energy(g, m, fo)
    assert abs(e_ref - e_init) <= 1e-13 * abs(e_init)
    assert abs(e_gpu - e_ref) <= (1e-12 if precision == "fp64" else 1e-5) * abs(e_ref)


def _small_wake_case():
    case = inputs.scaled_wake_case(16, 96, seed=7, sigma_dz=3.0)
    return case


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_wake_matches_oracle(precision):
    """Tapered-jaw collimator 16x16x96, sigma = 3 dz: the wake W(s) over a window
    reaching ahead of the bunch head, and the final field energy."""
    case = _small_wake_case()
    M = case.M
    jmin, nw = -M - 4, case.nw + (case.jmin + M + 4)
    steps = case.nz + M + jmin + nw
    ref = P.oracle_wake(case, steps, jmin=jmin, nw=nw)
    got = P.gpu_wake(case, steps, precision, jmin=jmin, nw=nw)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert P.delta_norm(got["W"], ref["W"]) <= tol
    assert abs(got["energy_final"] - ref["energy_final"]) <= tol * ref["energy_final"]
    j = jmin + np.arange(nw)
    assert np.all(got["W"][j < -M] == 0.0)          # causality, bitwise
    if precision == "fp64":
        res_e, res_h = got["grid"].charges()
        assert res_e <= 1e-13 * case.Q and res_h <= 1e-13 * case.Q


def test_charges_each_step_fp64():
    """Modified Gauss law (35) and (34) hold after every step of a wake run."""
    case = _small_wake_case()
    G = P.gpu_grid(case, "fp64")
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    for _ in range(60):
        G.step(1)
        e, h = G.charges()
        assert e <= 1e-13 * case.Q and h <= 1e-13 * case.Q


def test_energy_series_and_energy_law_with_bunch_fp64():
    """Per-step energy recorded during stepping matches the oracle's."""
    case = _small_wake_case()
    steps = 150
    ref = P.oracle_wake(case, steps, want_energy=True)
    G = P.gpu_grid(case, "fp64", max_series=steps)
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.set_diagnostics(1)
    G.step(steps)
    en = G.energy_series()
    assert len(en) == steps
    assert np.max(np.abs(en - ref["energy"])) <= 1e-12 * np.max(np.abs(ref["energy"]))
