"""Closed-form pins of the oracle: the explicit dispersion relation (27),
the magic time step dtau = dz (no dispersion along z), the stability limit
(25) and the cavity eigenfrequencies."""
import math

import numpy as np
import pytest

from paper_0901_1053_amd import inputs


def rhs27(Kx, Ky, Kz, dx, dy, dz, dt):
    """Right side of (27): sin^2 Om / dtau^2 = this."""
    T = np.sin(Kx) ** 2 / dx ** 2 + np.sin(Ky) ** 2 / dy ** 2
    return np.sin(Kz) ** 2 / dz ** 2 + T * (1.0 - (dt * dt / (dz * dz)) * np.sin(Kz) ** 2)


def omega27(m, n, p, nx, ny, nz, dx, dy, dz, dt):
    """Half phase advance per step Om = omega dtau / 2 from (27)."""
    K = (m * math.pi / (2 * nx), n * math.pi / (2 * ny), p * math.pi / (2 * nz))
    return math.asin(dt * math.sqrt(rhs27(*K, dx, dy, dz, dt)))


def one_step_matrix(orc, g, m):
    """Matrix of one oracle step on the in-range, non-PEC degrees of freedom."""
    f0 = orc.zeros(g)
    probe = {k: np.ones(g.shape) for k in orc.KEYS}
    orc.apply_pec(g, m, probe)
    # in-range mask: entries the oracle updates / reads (non-periodic ranges)
    nx, ny, nz = g.nx, g.ny, g.nz
    rng_mask = {k: np.zeros(g.shape, bool) for k in orc.KEYS}
    rng_mask["ex"][:nx, :, :] = True
    rng_mask["ey"][:, :ny, :] = True
    rng_mask["ez"][:, :, :nz] = True
    rng_mask["hx"][:, :ny, :nz] = True
    rng_mask["hy"][:nx, :, :nz] = True
    rng_mask["hz"][:nx, :ny, :] = True
    dofs = [(k, idx) for k in orc.KEYS for idx in zip(*np.nonzero(rng_mask[k] & (probe[k] != 0)))]
    n = len(dofs)
    Mx = np.zeros((n, n))
    for c, (k, idx) in enumerate(dofs):
        f = {kk: v.copy() for kk, v in f0.items()}
        f[k][idx] = 1.0
        orc.step(g, m, f)
        Mx[:, c] = [f[kk][ii] for (kk, ii) in dofs]
    return Mx


def test_one_step_eigenvalues_follow_27(orc):
    nx, ny, nz = 3, 4, 5
    dx, dy, dz, dt = 1.3, 1.1, 1.0, 0.6
    g = orc.Geom(nx, ny, nz, dx, dy, dz, dt)
    m = orc.vacuum_materials(g)
    lam = np.linalg.eigvals(one_step_matrix(orc, g, m))
    assert np.max(np.abs(lam)) <= 1 + 1e-12
    modes = [(a, b, c) for a in range(nx + 1) for b in range(ny + 1) for c in range(nz + 1)]
    K = np.array([(a * math.pi / (2 * nx), b * math.pi / (2 * ny), c * math.pi / (2 * nz)) for a, b, c in modes])
    r = rhs27(K[:, 0], K[:, 1], K[:, 2], dx, dy, dz, dt)
    osc = lam[np.abs(lam - 1) > 1e-7]
    assert len(osc) >= 40
    worst = 0.0
    for l in osc:
        assert abs(abs(l) - 1) < 1e-12
        Om = abs(np.angle(l)) / 2
        lhs = math.sin(Om) ** 2 / dt ** 2
        worst = max(worst, np.min(np.abs(r - lhs)) * dt * dt)
    assert worst < 1e-11
    # every mode with a non-trivial TM_mn0 / general pattern shows up
    for (a, b, c) in [(1, 1, 0), (2, 3, 1), (1, 2, 4)]:
        Om = omega27(a, b, c, nx, ny, nz, dx, dy, dz, dt)
        assert np.min(np.abs(np.abs(np.angle(osc)) - 2 * Om)) < 1e-10


def test_magic_step_plane_wave_moves_one_cell_per_step(orc):
    """Transversely uniform wave (periodic x, y): with dtau = dz an arbitrary
    pulse is transported exactly one cell per step; below it disperses."""
    nz, shift = 80, 30
    rng = np.random.default_rng(4)
    F = np.zeros(nz + 2)
    F[10:26] = rng.standard_normal(16)
    for dt, exact in ((1.0, True), (0.8, False)):
        g = orc.Geom(2, 2, nz, 2.0, 2.0, 1.0, dt, periodic_xy=True)
        m = orc.vacuum_materials(g)
        f = orc.zeros(g)
        k = np.arange(nz + 1)
        f["ex"][:2, :2, :] = F[k][None, None, :] * g.dx
        f["hy"][:2, :2, :nz] = F[k[:nz] + 1][None, None, :] * g.dy
        orc.apply_pec(g, m, f)
        orc.run(g, m, f, shift)
        want = np.zeros(nz + 1)
        want[shift:] = F[: nz + 1 - shift]
        err = np.max(np.abs(f["ex"][:2, :2, :] / g.dx - want[None, None, :]))
        if exact:
            assert err < 1e-13
        else:
            assert err > 1e-2


def _fit(trace, Oms):
    n = np.arange(len(trace))
    cols = [np.ones_like(trace)]
    for Om in Oms:
        cols += [np.cos(2 * Om * n), np.sin(2 * Om * n)]
    A = np.stack(cols, 1)
    coef, *_ = np.linalg.lstsq(A, trace, rcond=None)
    return np.max(np.abs(A @ coef - trace)) / np.max(np.abs(trace))


@pytest.mark.parametrize("kind", ["TM", "TE"])
def test_cavity_mode_oscillates_at_27_frequency(orc, kind):
    """An analytic cavity mode sampled on the grid stays in its discrete
    (m,n,p) pattern space; every probe trace is c0 + c1 cos(2 Om n) + c2 sin(2 Om n)
    with Om from (27).  The continuum frequency or Yee's relation (9) do not fit."""
    nx, ny, nz, dz = 12, 12, 24, 1.0
    dx = dy = 2.0
    dt = dz
    md = inputs.CavityMode(2, 1, 3, kind, 0.7)
    g = orc.Geom(nx, ny, nz, dx, dy, dz, dt)
    m = orc.vacuum_materials(g)
    f = inputs.cavity_fields(nx, ny, nz, dx, dy, dz, dt, [md])
    orc.apply_pec(g, m, f)
    probes = [np.ravel_multi_index(p, g.shape) for p in ((3, 4, 5), (7, 2, 11), (5, 9, 20))]
    tr = orc.run(g, m, f, 400, probes=probes)["probes"]
    Om = omega27(2, 1, 3, nx, ny, nz, dx, dy, dz, dt)
    kx, ky, kz = 2 * math.pi / (nx * dx), math.pi / (ny * dy), 3 * math.pi / (nz * dz)
    Om_cont = 0.5 * dt * math.sqrt(kx * kx + ky * ky + kz * kz)
    Om_yee = math.asin(dt * math.sqrt(math.sin(kx * dx / 2) ** 2 / dx ** 2 + math.sin(ky * dy / 2) ** 2 / dy ** 2
                                      + math.sin(kz * dz / 2) ** 2 / dz ** 2))
    for p in range(3):
        assert _fit(tr[:, p], [Om]) < 1e-11
        assert _fit(tr[:, p], [Om_cont]) > 1e-4
        assert _fit(tr[:, p], [Om_yee]) > 1e-4


def test_eigenfrequency_converges_second_order(orc):
    """omega~ from (27) -> omega = c|k| as O(h^2) under refinement (box and mode
    fixed, dx = dy = 2 dz, dtau = dz), and the oracle follows (27) at each level."""
    errs = []
    for lev in (1, 2, 4):
        nx, ny, nz = 4 * lev, 4 * lev, 8 * lev
        dz = 1.0 / lev
        dx = dy = 2 * dz
        Om = omega27(1, 1, 2, nx, ny, nz, dx, dy, dz, dz)
        w = 2 * Om / dz
        k = math.sqrt((math.pi / (nx * dx)) ** 2 + (math.pi / (ny * dy)) ** 2 + (2 * math.pi / (nz * dz)) ** 2)
        errs.append(abs(w - k) / k)
        g = orc.Geom(nx, ny, nz, dx, dy, dz, dz)
        m = orc.vacuum_materials(g)
        f = inputs.cavity_fields(nx, ny, nz, dx, dy, dz, dz, [inputs.CavityMode(1, 1, 2, "TM", 1.0)])
        orc.apply_pec(g, m, f)
        tr = orc.run(g, m, f, 200, probes=[np.ravel_multi_index((nx // 2 - 1, ny // 2 - 1, 1), g.shape)])["probes"]
        assert _fit(tr[:, 0], [Om]) < 1e-10
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5


def test_stability_limit_is_sharp(orc):
    """Spectral radius <= 1 just below the discrete limit implied by (27)
    (dtau^2 max_K T(K) = 1 with dz not binding), > 1 just above it; the
    limit tends to (25) as the grid is refined."""
    nx, ny, nz = 4, 3, 4
    dx, dy, dz = 1.0, 1.2, 10.0
    T = (math.sin((nx - 1) * math.pi / (2 * nx)) / dx) ** 2 + (math.sin((ny - 1) * math.pi / (2 * ny)) / dy) ** 2
    dt_lim = 1 / math.sqrt(T)
    assert dt_lim > (dx ** -2 + dy ** -2) ** -0.5
    for fac, stable in ((0.999, True), (1.001, False)):
        g = orc.Geom(nx, ny, nz, dx, dy, dz, fac * dt_lim)
        m = orc.vacuum_materials(g)
        rho = np.max(np.abs(np.linalg.eigvals(one_step_matrix(orc, g, m))))
        if stable:
            assert rho <= 1 + 1e-9
        else:
            assert rho > 1 + 1e-4
    big = [(1 / math.sqrt((math.sin((N - 1) * math.pi / (2 * N)) / dx) ** 2
                          + (math.sin((N - 1) * math.pi / (2 * N)) / dy) ** 2)) for N in (10, 100, 1000)]
    b25 = (dx ** -2 + dy ** -2) ** -0.5
    assert big[0] > big[1] > big[2] > b25 and abs(big[2] / b25 - 1) < 1e-5
