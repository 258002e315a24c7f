"""Pins of the sufficient stability test for general materials (Sec. 4.4).

The scheme is stable when Q^e = [[I - a^2 R_0, a L], [a L^T, I - a^2 R_1]] is
positive definite.  ``tests/gershgorin.py`` states the library's test: Q^e
splits into three blocks that share no variable, and each is positive
semi-definite when its Gershgorin row sums are at most 1.  Here both claims
are checked against the dense Q^e assembled from the geometric curl
(tests/dense_scheme.py), and the vacuum case against the bound (25)."""
import numpy as np
import pytest

from tests import gershgorin as GB
from tests.dense_scheme import DenseScheme


def _geom(orc, nx, ny, nz, dx, dy, dz, cdt):
    return orc.Geom(nx, ny, nz, dx, dy, dz, cdt)


def _random_materials(orc, g, seed, lo, hi, pec_frac=0.1):
    from paper_0901_1053_amd import inputs
    rng = np.random.default_rng(seed)
    m = orc.vacuum_materials(g, inputs.random_cells(g.nx, g.ny, g.nz, seed, frac=pec_frac))
    for k in m:
        m[k] = np.where(m[k] > 0, m[k] * rng.uniform(lo, hi, size=m[k].shape), 0.0)
    return m


@pytest.mark.parametrize("dxr,cdtr", [(2.0, 1.0), (2.0, 0.8), (1.2, 1.0), (3.0, 0.5), (0.9, 0.6)])
def test_vacuum_bound_is_25(orc, dxr, cdtr):
    """Empty PEC box: the largest row sum is max(cdt^2 (dx^-2 + dy^-2), cdt / dz),
    the two lines of the bound (25)."""
    dz = 1e-3
    g = _geom(orc, 6, 5, 7, dxr * dz, dxr * dz, dz, cdtr * dz)
    m = orc.vacuum_materials(g)
    want = max(g.cdt ** 2 * (g.dx ** -2 + g.dy ** -2), g.cdt / g.dz)
    assert abs(GB.bound(m, g.cdt) - want) <= 1e-12 * want


def test_three_blocks_share_no_variable(orc):
    """Q^e couples e_z only with e_z, h_z only with h_z, and (h_x, h_y, e_x,
    e_y) only among themselves (random materials, interior PEC)."""
    g = _geom(orc, 4, 3, 5, 2e-3, 1.7e-3, 1e-3, 0.9e-3)
    D = DenseScheme(g, _random_materials(orc, g, 3, 0.5, 1.3))
    grp = np.array([{"ez": 0, "hz": 1}.get("%s%s" % (kind, ax), 2) for (kind, ax, _) in D.lab])
    off = np.abs(D.Qe) * (grp[:, None] != grp[None, :])
    assert np.max(off) == 0.0
    assert np.max(np.abs(D.Qe - D.Qe.T)) <= 1e-12 * np.max(np.abs(D.Qe))


@pytest.mark.parametrize("seed", range(12))
def test_gershgorin_bounds_dense_spectrum(orc, seed):
    """For random materials (vacuum x U[0.3, 1.6], random PEC cells) and steps
    on both sides of the limit: lambda_min(Q^e) >= 1 - (largest row sum), so a
    set passing the test (sum <= 1) has Q^e >= 0."""
    rng = np.random.default_rng(100 + seed)
    nx, ny, nz = (int(v) for v in rng.integers(2, 5, size=3))
    dz = 1e-3
    dx, dy = dz * rng.uniform(1.2, 2.5), dz * rng.uniform(1.2, 2.5)
    cdt = dz * rng.uniform(0.6, 1.4)
    g = _geom(orc, nx, ny, nz, dx, dy, dz, cdt)
    m = _random_materials(orc, g, seed, 0.3, 1.6)
    b = GB.bound(m, cdt)
    lam = np.linalg.eigvalsh(DenseScheme(g, m).Qe)
    assert lam[0] >= 1.0 - b - 1e-12, (lam[0], b)
    if b <= 1.0:
        assert lam[0] >= -1e-12


def test_bound_is_tight_for_vacuum(orc):
    """The test is not vacuous: in vacuum just above the transverse limit of
    (25) Q^e has a negative eigenvalue, and the row sum exceeds 1 there;
    just below, both are on the stable side."""
    dz = 1e-3
    for nx in (6, 10):
        dx = 1.1 * dz
        lim = (2.0 / dx ** 2) ** -0.5
        for f, stable in ((0.98, True), (1.25, False)):
            g = _geom(orc, nx, nx, 3, dx, dx, dz, f * lim)
            m = orc.vacuum_materials(g)
            b = GB.bound(m, g.cdt)
            lam = np.linalg.eigvalsh(DenseScheme(g, m).Qe)[0]
            assert (b <= 1.0) == stable
            assert (lam >= 0.0) == stable, (nx, f, lam)


def test_passing_materials_stay_bounded(orc):
    """Random materials that pass the test: 600 oracle steps from random fields
    keep the discrete energy to round-off and the fields bounded."""
    from paper_0901_1053_amd import inputs
    g = _geom(orc, 7, 6, 9, 2e-3, 2e-3, 1e-3, 1e-3)
    m = _random_materials(orc, g, 17, 0.6, 1.0)
    assert GB.bound(m, g.cdt) <= 1.0
    f = inputs.random_fields(g.shape, 5)
    orc.apply_pec(g, m, f)
    e0 = orc.energy(g, m, f)
    peak0 = max(np.max(np.abs(v)) for v in f.values())
    orc.run(g, m, f, 600)
    assert abs(orc.energy(g, m, f) - e0) <= 1e-12 * e0
    assert max(np.max(np.abs(v)) for v in f.values()) <= 100 * peak0
