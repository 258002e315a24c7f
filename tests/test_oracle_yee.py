"""Pins of the oracle's Yee baseline (scheme (7) of Sec. 3): its dispersion
relation (9) and the z-form (10), the stability limit (8), the leapfrog
invariant, the discrete Gauss law with and without current, and exact
transport at dtau = dz for fields uniform across the beam (one cell per step)."""
import math

import numpy as np
import pytest

from paper_0901_1053_amd import inputs


def rhs9(Kx, Ky, Kz, dx, dy, dz):
    """Right side of (9): sin^2 Om / dtau^2 = this."""
    return np.sin(Kx) ** 2 / dx ** 2 + np.sin(Ky) ** 2 / dy ** 2 + np.sin(Kz) ** 2 / dz ** 2


def yee_step_matrix(orc, g, m):
    """Matrix of one Yee step of the oracle on the in-range, non-PEC degrees of
    freedom of a PEC box (or of a box periodic in x and y)."""
    probe = {k: np.ones(g.shape) for k in orc.KEYS}
    orc.apply_pec(g, m, probe)
    nx, ny, nz = g.nx, g.ny, g.nz
    rng_mask = {k: np.zeros(g.shape, bool) for k in orc.KEYS}
    if g.periodic_xy:
        for k in orc.KEYS:
            rng_mask[k][:nx, :ny, :] = True
        for k in ("ez", "hx", "hy"):
            rng_mask[k][:, :, nz] = False
    else:
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
        f = orc.zeros(g)
        f[k][idx] = 1.0
        orc.step_yee(g, m, f)
        Mx[:, c] = [f[kk][ii] for (kk, ii) in dofs]
    return Mx


def limit8(dx, dy, dz):
    return (dx ** -2 + dy ** -2 + dz ** -2) ** -0.5


def test_yee_eigenvalues_follow_9(orc):
    nx, ny, nz = 3, 4, 5
    dx, dy, dz = 1.3, 1.1, 1.0
    dt = 0.6
    assert dt < limit8(dx, dy, dz)
    g = orc.Geom(nx, ny, nz, dx, dy, dz, dt)
    m = orc.vacuum_materials(g)
    lam = np.linalg.eigvals(yee_step_matrix(orc, g, m))
    assert np.max(np.abs(lam)) <= 1 + 1e-12
    modes = [(a, b, c) for a in range(nx + 1) for b in range(ny + 1) for c in range(nz + 1)]
    K = np.array([(a * math.pi / (2 * nx), b * math.pi / (2 * ny), c * math.pi / (2 * nz)) for a, b, c in modes])
    r = rhs9(K[:, 0], K[:, 1], K[:, 2], dx, dy, dz)
    osc = lam[np.abs(lam - 1) > 1e-7]
    assert len(osc) >= 40
    worst = 0.0
    for l in osc:
        assert abs(abs(l) - 1) < 1e-12
        Om = abs(np.angle(l)) / 2
        worst = max(worst, np.min(np.abs(r - math.sin(Om) ** 2 / dt ** 2)) * dt * dt)
    assert worst < 1e-11
    # particular modes of the box
    for (a, b, c) in [(2, 3, 1), (1, 2, 4), (1, 1, 3)]:
        Om = math.asin(dt * math.sqrt(rhs9(a * math.pi / (2 * nx), b * math.pi / (2 * ny), c * math.pi / (2 * nz),
                                           dx, dy, dz)))
        assert np.min(np.abs(np.abs(np.angle(osc)) - 2 * Om)) < 1e-10


def test_yee_z_plane_waves_follow_10(orc):
    """Transversely uniform waves (periodic x, y, PEC ends in z): every standing
    wave k = p pi / L_z has the frequency of (10), below c k for dtau < dz."""
    nz, dz, dt = 12, 1.0, 0.7
    g = orc.Geom(2, 2, nz, 2.0, 2.0, dz, dt, periodic_xy=True)
    m = orc.vacuum_materials(g)
    lam = np.linalg.eigvals(yee_step_matrix(orc, g, m))
    assert np.max(np.abs(lam)) <= 1 + 1e-12
    ang = np.abs(np.angle(lam))
    for p in range(1, nz):
        k = p * math.pi / (nz * dz)
        w = 2 * math.asin(dt * math.sin(k * dz / 2) / dz) / dt      # solves (10) for omega
        assert abs(math.sin(k * dz / 2) / (dz / 2) - math.sin(dt * w / 2) / (dt / 2)) < 1e-14
        assert np.min(np.abs(ang - w * dt)) < 1e-10
        assert w < k                                                 # the wave lags: dispersion


def test_yee_stability_limit_is_sharp(orc):
    """Spectral radius <= 1 just below the finite-grid limit implied by (9),
    > 1 just above it; the limit tends to (8) under refinement."""
    nx, ny, nz = 3, 3, 4
    dx, dy, dz = 1.0, 1.2, 0.9

    def lim(Nx, Ny, Nz):
        s = sum((math.sin((N - 1) * math.pi / (2 * N)) / d) ** 2 for N, d in ((Nx, dx), (Ny, dy), (Nz, dz)))
        return 1 / math.sqrt(s)
    dt_lim = lim(nx, ny, nz)
    assert dt_lim > limit8(dx, dy, dz)
    for fac, stable in ((0.999, True), (1.001, False)):
        g = orc.Geom(nx, ny, nz, dx, dy, dz, fac * dt_lim)
        m = orc.vacuum_materials(g)
        rho = np.max(np.abs(np.linalg.eigvals(yee_step_matrix(orc, g, m))))
        if stable:
            assert rho <= 1 + 1e-9
        else:
            assert rho > 1 + 1e-4
    big = [lim(N, N, N) for N in (10, 100, 1000)]
    b8 = limit8(dx, dy, dz)
    assert big[0] > big[1] > big[2] > b8 and abs(big[2] / b8 - 1) < 1e-5


def _random_case(orc, seed, frac=0.1):
    nx, ny, nz = 9, 8, 14
    dx, dy, dz = 2.0e-3, 1.7e-3, 1.0e-3
    g = orc.Geom(nx, ny, nz, dx, dy, dz, 0.97 * limit8(dx, dy, dz))
    m = orc.vacuum_materials(g, inputs.random_cells(nx, ny, nz, seed, frac=frac))
    f = inputs.random_fields(g.shape, seed)
    orc.apply_pec(g, m, f)
    return g, m, f


def test_yee_leapfrog_invariant_conserved(orc):
    g, m, f = _random_case(orc, 3)
    vals = []
    for _ in range(60):
        fo = {k: v.copy() for k, v in f.items()}
        orc.step_yee(g, m, f)
        vals.append(orc.yee_invariant(g, m, fo, f))
    vals = np.array(vals)
    assert np.max(np.abs(vals - vals[0])) <= 1e-12 * abs(vals[0])
    # a plain sum of squares is not conserved by the scheme
    sq = [sum(np.sum(f[k] ** 2) for k in orc.KEYS)]
    orc.step_yee(g, m, f)
    sq.append(sum(np.sum(f[k] ** 2) for k in orc.KEYS))
    assert abs(sq[1] - sq[0]) > 1e-6 * sq[0]


def _free_nodes(g, m):
    """Nodes whose six edges all exist and are not PEC (the law holds there)."""
    ok = np.zeros(g.shape, bool)
    ok[1:g.nx, 1:g.ny, 1:g.nz] = True
    ok[1:, :, :] &= m["ex"][:-1, :, :] > 0
    ok[:-1, :, :] &= m["ex"][:-1, :, :] > 0
    ok[:, 1:, :] &= m["ey"][:, :-1, :] > 0
    ok[:, :-1, :] &= m["ey"][:, :-1, :] > 0
    ok[:, :, 1:] &= m["ez"][:, :, :-1] > 0
    ok[:, :, :-1] &= m["ez"][:, :, :-1] > 0
    return ok


def test_yee_gauss_law(orc):
    """Without current the node charges never change; with a current on some
    e_z edges they change by -dtau times its divergence (physical sign), at
    every node whose six edges are free."""
    g, m, f = _random_case(orc, 5)
    ok = _free_nodes(g, m)
    assert ok.sum() > 200
    q0 = orc.yee_charge(g, m, f)
    for _ in range(30):
        orc.step_yee(g, m, f)
    q1 = orc.yee_charge(g, m, f)
    scale = np.max(np.abs(q0))
    assert np.max(np.abs(q1 - q0)[ok]) <= 1e-12 * scale
    assert np.max(np.abs(q1 - q0)[~ok]) > 1e-6 * scale      # the PEC edges' flux is not counted
    rng = np.random.default_rng(6)
    jz = np.zeros(g.shape)
    live = m["ez"] > 0
    pick = np.argwhere(live)[rng.choice(int(live.sum()), 12, replace=False)]
    for p in pick:
        jz[tuple(p)] = rng.standard_normal()
    orc.step_yee(g, m, f, jz=jz)
    q2 = orc.yee_charge(g, m, f)
    want = np.zeros(g.shape)
    want[:, :, :] -= g.cdt * jz                       # flux leaves node k along +z ...
    want[:, :, 1:] += g.cdt * jz[:, :, :-1]           # ... and enters node k+1
    assert np.max(np.abs(q2 - q1 - want)[ok]) <= 1e-12 * scale
    assert np.count_nonzero(want[ok]) >= 4            # the current reaches free nodes


def test_yee_transversely_uniform_pulse(orc):
    """Fields uniform in x and y (periodic): the transverse curl terms vanish and
    Yee's scheme is the 1-D leapfrog, which at dtau = dz moves any pulse exactly
    one cell per step; at dtau < dz (as (8) forces in 3-D) it disperses."""
    nz, shift = 80, 30
    rng = np.random.default_rng(4)
    F = np.zeros(nz + 2)
    F[10:26] = rng.standard_normal(16)
    for dt, exact in ((1.0, True), (0.8, False)):
        g = orc.Geom(2, 2, nz, 2.0, 2.0, 1.0, dt, periodic_xy=True)
        m = orc.vacuum_materials(g)
        f = orc.zeros(g)
        k = np.arange(nz + 1)
        # state (e^{-1/2}, h^0) of a right-moving wave u(z - tau): e_x at
        # (z = k, tau = -1/2) and h_y at (z = k + 1/2, tau = 0) both sample
        # u(k + 1/2), here F[k]
        f["ex"][:2, :2, :] = F[k][None, None, :] * g.dx
        f["hy"][:2, :2, :nz] = F[k[:nz]][None, None, :] * g.dy
        orc.apply_pec(g, m, f)
        for _ in range(shift):
            orc.step_yee(g, m, f)
        want = np.zeros(nz + 1)
        want[shift:] = F[: nz + 1 - shift]
        err = np.max(np.abs(f["ex"][:2, :2, :] / g.dx - want[None, None, :]))
        if exact:
            assert err < 1e-13
        else:
            assert err > 1e-2
