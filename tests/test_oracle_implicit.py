"""Pins of the oracle of the implicit TE/TM scheme (16) (Sec. 4.1): the
dispersion relation of Sec. 4.5 for the implicit scheme (and its transverse
form tan^2 Omega = ...), stability for any transverse mesh at dtau <= dz (where
the explicit scheme's bound (25) fails) and instability beyond dz, the energy
law (19) with and without current, the discrete Gauss law, and exact transport
of a transversely uniform pulse at dtau = dz."""
import math

import numpy as np
import pytest

from oracle import implicit_oracle as IM
from paper_0901_1053_amd import inputs


@pytest.fixture(scope="module")
def imp():
    return IM


def step_matrix(im, g, m, explicit=False):
    """One-step matrix on the in-range, non-PEC degrees of freedom."""
    O = im.O
    probe = {k: np.ones(g.shape) for k in O.KEYS}
    O.apply_pec(g, m, probe)
    ix = im._Index(g)
    R = {c: im._in_range(g, c, ix.i, ix.j, ix.k).reshape(g.shape) for c in range(6)}
    dofs = [(k, idx) for c, k in enumerate(O.KEYS) for idx in zip(*np.nonzero(R[c] & (probe[k] != 0)))]
    S = None if explicit else im.Implicit(g, m)
    A = np.zeros((len(dofs), len(dofs)))
    for col, (k, idx) in enumerate(dofs):
        f = O.zeros(g)
        f[k][idx] = 1.0
        if explicit:
            O.step(g, m, f)
        else:
            S.step(f)
        A[:, col] = [f[kk][ii] for kk, ii in dofs]
    return A


def omega_implicit(Kx, Ky, Kz, dx, dy, dz, dt):
    """Omega of the implicit relation sin^2 W / dt^2 = sin^2 Kz / dz^2 + St cos^2 W,
    St = sin^2 Kx / dx^2 + sin^2 Ky / dy^2, solved for sin^2 W."""
    st = math.sin(Kx) ** 2 / dx ** 2 + math.sin(Ky) ** 2 / dy ** 2
    s2 = (math.sin(Kz) ** 2 / dz ** 2 + st) / (1 / dt ** 2 + st)
    return math.asin(math.sqrt(s2))


def test_implicit_eigenvalues_follow_the_dispersion_relation(imp):
    """PEC box with a fine transverse mesh at dtau = dz: every oscillating
    eigenvalue of the one-step matrix is exp(+-2i Omega) of a box mode
    (Kx, Ky, Kz) = (a pi / 2nx, b pi / 2ny, c pi / 2nz) under the implicit
    relation; the explicit relation (27) does not fit; the transverse modes
    (c = 0) satisfy tan^2 Omega = dtau^2 St."""
    O = imp.O
    nx, ny, nz = 3, 4, 5
    dx, dy, dz, dt = 0.7, 0.6, 1.0, 1.0
    g = O.Geom(nx, ny, nz, dx, dy, dz, dt)
    lam = np.linalg.eigvals(step_matrix(imp, g, O.vacuum_materials(g)))
    assert np.max(np.abs(lam)) <= 1 + 1e-12
    osc = lam[np.abs(lam - 1) > 1e-7]
    assert len(osc) >= 100
    modes = [(a, b, c) for a in range(nx + 1) for b in range(ny + 1) for c in range(nz + 1)]
    K = [(a * math.pi / (2 * nx), b * math.pi / (2 * ny), c * math.pi / (2 * nz)) for a, b, c in modes]
    pred = np.array([2 * omega_implicit(*k, dx, dy, dz, dt) for k in K])
    ang = np.abs(np.angle(osc))
    assert max(np.min(np.abs(pred - a)) for a in ang) < 1e-10
    assert np.all(np.abs(np.abs(osc) - 1) < 1e-12)
    # particular modes present, including transverse ones with the tan^2 form
    for a, b, c in [(1, 2, 0), (2, 3, 0), (1, 1, 3), (2, 2, 4)]:
        Kx, Ky, Kz = a * math.pi / (2 * nx), b * math.pi / (2 * ny), c * math.pi / (2 * nz)
        W = omega_implicit(Kx, Ky, Kz, dx, dy, dz, dt)
        if c == 0:
            st = math.sin(Kx) ** 2 / dx ** 2 + math.sin(Ky) ** 2 / dy ** 2
            assert abs(math.tan(W) ** 2 - dt ** 2 * st) < 1e-12 * (1 + dt ** 2 * st)
        assert np.min(np.abs(ang - 2 * W)) < 1e-10
    # the explicit relation (27) gives another frequency for mode (1, 1, 3)
    Kx, Ky, Kz = math.pi / (2 * nx), math.pi / (2 * ny), 3 * math.pi / (2 * nz)
    st = math.sin(Kx) ** 2 / dx ** 2 + math.sin(Ky) ** 2 / dy ** 2
    s2 = dt ** 2 * (math.sin(Kz) ** 2 / dz ** 2 + st * (1 - dt ** 2 / dz ** 2 * math.sin(Kz) ** 2))
    assert s2 < 1
    assert np.min(np.abs(ang - 2 * math.asin(math.sqrt(s2)))) > 1e-6


def test_implicit_stable_for_any_transverse_mesh(imp):
    """dx = dy = dz/4: the explicit scheme (bound (25): dtau <= 0.18 dz) blows up
    at dtau = 0.9 dz, the implicit one stays on the unit circle up to dtau = dz
    and becomes unstable beyond it (the longitudinal bound)."""
    O = imp.O
    g = O.Geom(4, 4, 5, 0.25, 0.25, 1.0, 0.9)
    m = O.vacuum_materials(g)
    assert np.max(np.abs(np.linalg.eigvals(step_matrix(imp, g, m, explicit=True)))) > 1 + 1e-3
    for dt, stable in ((0.9, True), (1.0, True), (1.2, False)):
        g = O.Geom(4, 4, 5, 0.25, 0.25, 1.0, dt)
        rho = np.max(np.abs(np.linalg.eigvals(step_matrix(imp, g, O.vacuum_materials(g)))))
        if stable:
            assert rho <= 1 + 1e-10, dt
        else:
            assert rho > 1 + 1e-3, dt


def _random_case(im, seed, frac=0.1, dt=1.0e-3):
    O = im.O
    nx, ny, nz = 7, 6, 10
    g = O.Geom(nx, ny, nz, 0.8e-3, 0.7e-3, 1.0e-3, dt)          # beyond (25) for the explicit scheme
    m = O.vacuum_materials(g, inputs.random_cells(nx, ny, nz, seed, frac=frac))
    f = inputs.random_fields(g.shape, seed)
    O.apply_pec(g, m, f)
    return g, m, f


def test_implicit_energy_law(imp):
    """(19) for (16): without current the energy is constant to round-off; with
    a current on some e_z edges it changes by -dtau/2 sum (e_z^{n+1/2} + e_z^{n-1/2}) j_z^n."""
    g, m, f = _random_case(imp, 3)
    S = imp.Implicit(g, m)
    E = []
    for _ in range(40):
        E.append(imp.energy(g, m, f))
        S.step(f)
    E = np.array(E)
    assert E[0] > 0
    assert np.max(np.abs(E - E[0])) <= 1e-13 * E[0]
    rng = np.random.default_rng(8)
    for _ in range(5):
        jz = np.where(m["ez"] > 0, rng.standard_normal(g.shape), 0.0)
        ez0 = f["ez"].copy()
        W0 = imp.energy(g, m, f)
        S.step(f, jz=jz)
        W1 = imp.energy(g, m, f)
        want = -0.5 * g.cdt * float(np.sum((f["ez"] + ez0) * jz))
        assert abs((W1 - W0) - want) <= 1e-12 * W0


def _free_nodes(g, m):
    ok = np.zeros(g.shape, bool)
    ok[1:g.nx, 1:g.ny, 1:g.nz] = True
    ok[1:, :, :] &= m["ex"][:-1, :, :] > 0
    ok[:-1, :, :] &= m["ex"][:-1, :, :] > 0
    ok[:, 1:, :] &= m["ey"][:, :-1, :] > 0
    ok[:, :-1, :] &= m["ey"][:, :-1, :] > 0
    ok[:, :, 1:] &= m["ez"][:, :, :-1] > 0
    ok[:, :, :-1] &= m["ez"][:, :, :-1] > 0
    return ok


def test_implicit_gauss_law(imp):
    """The time-averaged node charge of (16) is constant without current and
    changes by dtau (j(k-1) - j(k)) with it, at every node with six free edges
    (no alpha^2 correction: the transverse operators are time-centred)."""
    g, m, f = _random_case(imp, 5)
    S = imp.Implicit(g, m)
    ok = _free_nodes(g, m)
    assert ok.sum() > 100
    fo = {k: v.copy() for k, v in f.items()}
    S.step(f)
    q0 = imp.charge(g, m, fo, f)
    for _ in range(20):
        fo = {k: v.copy() for k, v in f.items()}
        S.step(f)
    q1 = imp.charge(g, m, fo, f)
    scale = np.max(np.abs(q0))
    assert np.max(np.abs(q1 - q0)[ok]) <= 1e-12 * scale
    assert np.max(np.abs(q1 - q0)[~ok]) > 1e-6 * scale
    rng = np.random.default_rng(6)
    jz = np.zeros(g.shape)
    live = np.argwhere(m["ez"] > 0)
    for p in live[rng.choice(len(live), 12, replace=False)]:
        jz[tuple(p)] = rng.standard_normal()
    fo = {k: v.copy() for k, v in f.items()}
    S.step(f, jz=jz)
    q2 = imp.charge(g, m, fo, f)
    want = -g.cdt * jz
    want[:, :, 1:] += g.cdt * jz[:, :, :-1]
    assert np.max(np.abs(q2 - q1 - want)[ok]) <= 1e-12 * scale
    assert np.count_nonzero(want[ok]) >= 4


def test_implicit_transversely_uniform_pulse(imp):
    """Periodic x, y and fields uniform across: at dtau = dz any pulse moves
    exactly one cell per step; below dz it disperses."""
    O = imp.O
    nz, shift = 60, 20
    rng = np.random.default_rng(4)
    F = np.zeros(nz + 2)
    F[8:22] = rng.standard_normal(14)
    for dt, exact in ((1.0, True), (0.8, False)):
        g = O.Geom(2, 2, nz, 0.5, 0.5, 1.0, dt, periodic_xy=True)
        m = O.vacuum_materials(g)
        S = imp.Implicit(g, m)
        f = O.zeros(g)
        k = np.arange(nz + 1)
        f["ex"][:2, :2, :] = F[k][None, None, :] * g.dx
        f["hy"][:2, :2, :nz] = F[k[:nz] + 1][None, None, :] * g.dy
        O.apply_pec(g, m, f)
        for _ in range(shift):
            S.step(f)
        want = np.zeros(nz + 1)
        want[shift:] = F[: nz + 1 - shift]
        err = np.max(np.abs(f["ex"][:2, :2, :] / g.dx - want[None, None, :]))
        if exact:
            assert err < 1e-13
        else:
            assert err > 1e-2
