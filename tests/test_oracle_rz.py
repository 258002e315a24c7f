"""Pins of the r-z oracle of the rotationally symmetric scheme (24) (Sec. 4.3):
facet areas that tile the cross-section, pillbox eigenfrequencies of the
Bessel closed forms converging at second order for m = 0, 1, 2 (TM and TE),
the discrete energy conserved to round-off, the stable step independent of m
(Sec. 4.4) against Yee's falling as 1/m, exact transport of a coaxial TEM pulse
at dtau = dz, the discrete Gauss law of a moving ring charge, the energy
balance and causality of the wake lines, and the Panofsky-Wenzel transverse
wake against a direct integral of the Lorentz force."""
import math

import numpy as np
import pytest
from scipy.special import jn_zeros, jnp_zeros

from oracle import rz_oracle


@pytest.fixture(scope="module")
def rz():
    return rz_oracle


def step_matrix(Z, g, m, yee=False):
    """Matrix of one step on the in-range, non-PEC degrees of freedom."""
    probe = {k: np.ones(g.shape) for k in Z.KEYS}
    Z.apply_pec(g, m, probe)
    R = Z.ranges(g)
    dofs = [(k, idx) for k in Z.KEYS for idx in zip(*np.nonzero(R[k] & (probe[k] != 0)))]
    A = np.zeros((len(dofs), len(dofs)))
    stepf = Z.step_yee if yee else Z.step
    for c, (k, idx) in enumerate(dofs):
        f = Z.zeros(g)
        f[k][idx] = 1.0
        stepf(g, m, f)
        A[:, c] = [f[kk][ii] for kk, ii in dofs]
    return A


def rho(Z, g, yee=False, cells=None):
    return float(np.max(np.abs(np.linalg.eigvals(step_matrix(Z, g, Z.materials(g, cells), yee)))))


def freqs(Z, g):
    lam = np.linalg.eigvals(step_matrix(Z, g, Z.materials(g)))
    return np.abs(np.angle(lam)) / g.cdt


def test_rz_facets_tile_the_cross_section(rz):
    """Per radian, the dual facets of the e_z edges (the disk of radius dr/2 on
    the axis, annuli elsewhere) tile the disk up to r_{nr-1/2}, and the facets
    of h_z tile the whole disk; the phi facets are the r-z cells."""
    for mode in (0, 1):
        nr, nz, dr, dz = 7, 3, 0.3, 0.2
        g = rz.RZGeom(nr, nz, dr, dz, 0.1, mode)
        g_open = rz.RZGeom(nr + 1, nz, dr, dz, 0.1, mode)       # one more ring: row nr is free here
        m = rz.materials(g_open)
        az = [dz / m["ez"][j, 1] for j in range(nr) if m["ez"][j, 1] > 0]
        hz = [dz / m["hz"][j, 1] for j in range(nr)]
        if mode == 0:
            assert math.isclose(sum(az), 0.5 * ((nr - 0.5) * dr) ** 2, rel_tol=1e-14)
        else:                       # no e_z on the axis for m >= 1
            assert len(az) == nr - 1
            assert math.isclose(sum(az), 0.5 * ((nr - 0.5) * dr) ** 2 - 0.5 * (0.5 * dr) ** 2, rel_tol=1e-14)
        assert math.isclose(sum(hz), 0.5 * (nr * dr) ** 2, rel_tol=1e-14)
        m = rz.materials(g)
        for j in range(1, nr):
            assert math.isclose(j * dr / m["ephi"][j, 1], dr * dz, rel_tol=1e-14)
            assert math.isclose((j + 0.5) * dr / m["hphi"][j, 1], dr * dz, rel_tol=1e-14)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_rz_tm_modes_converge_second_order(rz, mode):
    """TM_{m10} of a PEC pillbox: omega = x_{m1} / R (x the first zero of J_m);
    the discrete frequency converges at O(h^2) with dtau proportional to h."""
    R = 1.0
    wa = jn_zeros(mode, 1)[0] / R
    errs = []
    for nr in (8, 16, 32):
        dr = R / nr
        g = rz.RZGeom(nr, 1, dr, 0.5, 0.5 * dr, mode)
        errs.append(np.min(np.abs(freqs(rz, g) - wa)) / wa)
    assert errs[-1] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


@pytest.mark.parametrize("kind,mode,p", [("TE", 1, 1), ("TM", 0, 1), ("TE", 0, 1), ("TM", 1, 1)])
def test_rz_modes_with_z_variation(rz, kind, mode, p):
    """TE_{m1p} (x'_{m1}, zero of J_m') and TM_{m1p} of a pillbox of length L:
    omega^2 = (x / R)^2 + (p pi / L)^2, reached at second order."""
    R = L = 1.0
    x = jnp_zeros(mode, 1)[0] if kind == "TE" else jn_zeros(mode, 1)[0]
    wa = math.hypot(x / R, p * math.pi / L)
    errs = []
    for n in (6, 12):
        g = rz.RZGeom(n, n, R / n, L / n, 0.5 * R / n, mode)
        errs.append(np.min(np.abs(freqs(rz, g) - wa)) / wa)
    assert errs[1] < 5e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


def _random_state(Z, g, seed, frac=0.1):
    rng = np.random.default_rng(seed)
    cells = rng.random((g.nr, g.nz)) < frac
    m = Z.materials(g, cells)
    f = {k: rng.standard_normal(g.shape) for k in Z.KEYS}
    Z.apply_pec(g, m, f)
    return m, f


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_rz_energy_conserved(rz, mode):
    """With j = 0 the discrete energy 1/2 <Q y, y> is constant to round-off, with
    staircase obstacles; the plain sum of squares is not."""
    g = rz.RZGeom(10, 14, 1.0, 0.8, 0.75, mode)
    m, f = _random_state(rz, g, 11 + mode)
    E = []
    for _ in range(50):
        E.append(rz.energy(g, m, f))
        rz.step(g, m, f)
    E = np.array(E)
    assert E[0] > 0
    assert np.max(np.abs(E - E[0])) <= 1e-13 * E[0]
    sq0 = sum(np.sum(f[k] ** 2) for k in rz.KEYS)
    rz.step(g, m, f)
    assert abs(sum(np.sum(f[k] ** 2) for k in rz.KEYS) - sq0) > 1e-6 * sq0


# largest eigenvalue of the radial operator next to the axis (m = 0), in 1/dr^2:
# the tridiagonal with e_z dual facets dr^2/8 on the axis and j dr^2 elsewhere
M0_LIMIT = 2.0 / math.sqrt(4.841942263591951)        # = 0.90891 dr


def test_rz_axis_limit_constant():
    """The m = 0 radial limit from the tridiagonal operator, independent of its
    length (computed here from the facet areas, not from the oracle)."""
    from scipy.linalg import eigh_tridiagonal
    for nr in (4, 64, 1000):
        kz = np.array([8.0] + [1.0 / j for j in range(1, nr)])
        mu = np.arange(nr) + 0.5
        d = kz * (np.concatenate([[0.0], mu[:-1]]) + mu)
        o = np.sqrt(kz[:-1] * kz[1:]) * mu[:-1]
        lmax = eigh_tridiagonal(d, o, eigvals_only=True)[-1]
        assert abs(2 / math.sqrt(lmax) - M0_LIMIT) < 3e-4


def test_rz_stability_independent_of_m(rz):
    """Sec. 4.4: the stable step of (24) does not depend on m.  Just below
    min(dz, dr) every m >= 1 is stable (m = 0: below min(dz, 0.9089 dr), the
    on-axis cell), and just above the axis limit m = 0 is not.  Yee's scheme on
    the same grid needs dtau of order dr / m: unstable at min(dz, dr) for m >= 2,
    with its limit between 0.9 dr / m and 1.2 dr / m for m = 4, 8."""
    for dr, dz in ((1.0, 1.3), (1.3, 1.0)):
        for mode in (1, 2, 5, 8):
            g = rz.RZGeom(8, 6, dr, dz, 0.999 * min(dr, dz), mode)
            assert rho(rz, g) <= 1 + 1e-9, (dr, dz, mode)
        g = rz.RZGeom(8, 6, dr, dz, 0.999 * min(dz, M0_LIMIT * dr), 0)
        assert rho(rz, g) <= 1 + 1e-9
    g = rz.RZGeom(8, 6, 1.0, 1.3, 1.01 * M0_LIMIT, 0)
    assert rho(rz, g) > 1 + 1e-6
    for mode in (2, 4):
        assert rho(rz, rz.RZGeom(8, 6, 1.0, 1.3, 0.999, mode), yee=True) > 1 + 1e-6
    for mode in (4, 8):
        assert rho(rz, rz.RZGeom(8, 6, 1.0, 1.3, 0.9 / mode, mode), yee=True) <= 1 + 1e-9
        assert rho(rz, rz.RZGeom(8, 6, 1.0, 1.3, 1.2 / mode, mode), yee=True) > 1 + 1e-6


def test_rz_stable_with_obstacles(rz):
    """Staircase obstacles only remove degrees of freedom: still stable at the
    same step, for m = 0 and m = 3."""
    cells = np.random.default_rng(9).random((8, 6)) < 0.2
    for mode, dt in ((0, 0.999 * M0_LIMIT), (3, 0.999)):
        g = rz.RZGeom(8, 6, 1.0, 1.3, dt, mode)
        assert rho(rz, g, cells=cells) <= 1 + 1e-9


def test_rz_coax_tem_moves_one_cell_per_step(rz):
    """A coaxial TEM pulse (E_r ~ 1/r, inner conductor of radius 3 dr): at
    dtau = dz it moves exactly one cell per step with e_z and h_z staying zero;
    below dz it disperses.  e_r and h_phi stand where e_y and h_x stand in the
    3-D scheme, so the forward wave has h_phi = -e_r r / dr."""
    nr, nz, jin, shift = 10, 80, 3, 30
    rng = np.random.default_rng(4)
    F = np.zeros(nz + 2)
    F[10:26] = rng.standard_normal(16)
    cells = np.zeros((nr, nz), bool)
    cells[:jin, :] = True
    for dt, exact in ((1.0, True), (0.8, False)):
        g = rz.RZGeom(nr, nz, 1.2, 1.0, dt, 0)
        m = rz.materials(g, cells)
        f = rz.zeros(g)
        rh = (np.arange(nr + 1)[:, None] + 0.5) * g.dr
        k = np.arange(nz + 1)[None, :]
        f["er"][:] = F[k] * g.dr / rh
        f["hphi"][:, :nz] = -F[k[:, :nz] + 1] * np.ones((nr + 1, 1))
        f["hphi"][:jin, :] = 0.0
        rz.apply_pec(g, m, f)
        for _ in range(shift):
            rz.step(g, m, f)
        want = np.zeros(nz + 1)
        want[shift:] = F[: nz + 1 - shift]
        err = np.max(np.abs(f["er"][jin:nr, :] * rh[jin:nr] / g.dr - want[None, :]))
        if exact:
            assert err < 1e-13
            assert np.max(np.abs(f["ez"])) < 1e-13 and np.max(np.abs(f["hz"])) == 0.0
        else:
            assert err > 1e-2


def _free_nodes(Z, g, m):
    """Nodes whose edges (e_r on both sides, e_z on both sides, e_phi for m >= 1)
    all exist and are free: the law holds there."""
    ok = np.ones(g.shape, bool)
    ok[:, 0] = ok[:, -1] = False
    ok[-1, :] = False
    if g.m > 0:
        ok &= m["ephi"] > 0
    ok[:, 1:] &= m["ez"][:, :-1] > 0
    ok[:, :-1] &= m["ez"][:, :-1] > 0
    ok &= m["er"] > 0
    ok[1:, :] &= m["er"][:-1, :] > 0
    return ok


@pytest.mark.parametrize("mode,j0,dr", [(0, 0, 1.25), (1, 3, 1.0), (2, 4, 1.0)])
def test_rz_gauss_law_ring_bunch(rz, mode, j0, dr):
    """While a ring charge (the axis for m = 0) moves through an iris, the node
    charge changes by dtau (j(k-1) - j(k)) at every node with free edges, to
    round-off; from zero fields it therefore equals the charge that has passed."""
    g = rz.RZGeom(10, 40, dr, 1.0, 1.0, mode)
    cells = np.zeros((10, 40), bool)
    cells[6:, 18:24] = True
    m = rz.materials(g, cells)
    ok = _free_nodes(rz, g, m)
    assert ok.sum() > 250
    f = rz.zeros(g)
    b = rz.RZBunch(1.0, 2.0, j0, 6, 2, -8, 30)
    lam = rz.bunch_cells(1.0, 2.0, 1.0, 6)
    wm = (1 / (2 * math.pi)) if mode == 0 else (1 / math.pi)
    rz.run(g, m, f, 1, n0=0, bunch=b)
    qprev = None
    moved = 0.0
    for n in range(1, 34):
        f0 = {k: v.copy() for k, v in f.items()}
        rz.run(g, m, f, 1, n0=n, bunch=b)
        q = rz.charge(g, m, f0, f)
        if qprev is not None:
            jz = np.zeros(g.shape)
            for k in range(g.nz):
                mm = k - n + 6
                if -6 <= mm <= 6:
                    jz[j0, k] = wm * lam[mm + 6]
            want = -jz
            want[:, 1:] += jz[:, :-1]
            moved = max(moved, np.max(np.abs(want[ok])))
            assert np.max(np.abs(q - qprev - want)[ok]) <= 1e-14
        qprev = q
    assert moved > 1e-3


def _wake_case(Z, mode, nz=30):
    dr = 1.25 if mode == 0 else 1.0                 # the axis cell needs dtau < 0.909 dr
    g = Z.RZGeom(8, nz, dr, 1.0, 1.0, mode)
    cells = np.zeros((8, nz), bool)
    cells[4:, :] = True
    cells[4:, 10:18] = False
    m = Z.materials(g, cells)
    j0 = 0 if mode == 0 else 2
    return g, m, Z.zeros(g), Z.RZBunch(1.0, 1.5, j0, 5, j0, -8, 40)


@pytest.mark.parametrize("mode", [0, 1])
def test_rz_wake_energy_identity(rz, mode):
    """After the bunch has left, the field energy equals w_m sum_m lam_m acc(-m dz)
    on the bunch's own line (energy law with j^n dtau = w_m lam), with the
    weight of the harmonic w_0 = 1/(2 pi), w_m = 1/pi."""
    g, m, f, b = _wake_case(rz, mode)
    N = g.nz + 2 * b.M + 2
    r = rz.run(g, m, f, N, bunch=b)
    WN = rz.energy(g, m, f)
    wm = (1 / (2 * math.pi)) if mode == 0 else (1 / math.pi)
    tot = sum(r["lam"][mm + b.M] * r["acc"][0, -mm - b.jmin] for mm in range(-b.M, b.M + 1))
    assert WN > 0
    assert abs(WN - wm * tot) <= 1e-13 * WN


def test_rz_wake_causality(rz):
    """At dtau = dz nothing outruns the bunch: both wake lines are zero ahead
    of its head, bitwise, and so is the grid ahead of the head."""
    g, m, f, b = _wake_case(rz, 1)
    r = rz.run(g, m, f, g.nz + 3 * b.M, bunch=b)
    j = np.arange(b.jmin, b.jmin + b.nw)
    assert np.all(r["acc"][:, j < -b.M] == 0.0)
    assert np.any(r["acc"][:, j == -b.M] != 0.0)
    g2, m2, f2, b2 = _wake_case(rz, 1, nz=40)
    rz.run(g2, m2, f2, 12, bunch=b2)
    for key in rz.KEYS:
        assert np.all(f2[key][:, 14:] == 0.0), key


def _direct_and_pw(Z, lev):
    """Transverse wake of m = 1 at r_{jw+1/2} two ways: Panofsky-Wenzel from the
    two wake lines, and the direct integral of E_r - B_phi (B_phi = -h_phi / r,
    the sign the coaxial pulse fixes) along the witness path, e_r averaged to
    time n + 1/2 and h_phi^{n+1/2} averaged to z_k."""
    nr, nz = 8 * lev, 60 * lev
    dr = dz = 1.0 / lev
    g = Z.RZGeom(nr, nz, dr, dz, dz, 1)
    cells = np.zeros((nr, nz), bool)
    cells[4 * lev:, :] = True
    cells[4 * lev:, 20 * lev:35 * lev] = False
    m = Z.materials(g, cells)
    M, jw, nw = 5 * lev, lev, 20 * lev
    b = Z.RZBunch(1.0, 1.0, 2 * lev, M, jw, -M, nw)
    f = Z.zeros(g)
    acc = np.zeros((2, nw))
    direct = np.zeros(nw)
    rh = (jw + 0.5) * dr
    for n in range(nz + 2 * M + nw):
        er_o = f["er"][jw, :].copy()
        Z.run(g, m, f, 1, n0=n, bunch=b, acc=acc)
        er = 0.5 * (er_o + f["er"][jw, :]) / dr
        hp = f["hphi"][jw, :] / rh
        hk = np.zeros(nz + 1)
        hk[1:nz] = 0.5 * (hp[: nz - 1] + hp[1:nz])
        Fr = er + hk
        for k in range(1, nz):
            jj = n + 1 - k - M
            if -M <= jj < -M + nw:
                direct[jj + M] += Fr[k] * dz
    pw = Z.transverse_wake(acc, 1.0, dr, dz)
    s = np.arange(-M, -M + nw) * dz
    sel = (s > 2) & (s < 15)
    return np.max(np.abs(pw[sel] - direct[sel])) / np.max(np.abs(direct[sel]))


def test_rz_transverse_wake_matches_lorentz_force(rz):
    """The Panofsky-Wenzel transverse wake and the direct integral of the
    Lorentz force agree ever better under refinement."""
    e = [_direct_and_pw(rz, lev) for lev in (1, 2, 4)]
    assert e[0] > e[1] > e[2]
    assert e[1] < 0.1 and e[2] < 0.04
