"""Pins of the open-pipe oracle (the bunch's own field in a uniform entrance
pipe and the wake quadrature that ends before the exit wall's reflections).

The checks come from outside the oracle's own construction:
  - the cross-section's potential against the discrete sine series of a
    rectangle (the 5-point operator's exact eigen-expansion);
  - the scheme itself: the field must be carried one cell per step with e_z
    and h_z zero, and the energy W^{n,e} (Sec. 4.4) must stay constant;
  - the conserved charges (35) of Sec. 4.5: the field's node charges must be
    the bunch's cell charges, and zero elsewhere;
  - the wake of a uniform pipe must vanish, and the wake of a collimator must
    not depend on the length of the pipes beyond what causality allows.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import pipe_oracle as PIPE

DZ = 1e-3


@pytest.fixture
def po():
    O.lib()
    return PIPE


def _pipe_grid(nx, ny, nz, dx=2 * DZ, dy=2 * DZ, cut=True, collimator=None):
    g = O.Geom(nx, ny, nz, dx, dy, DZ, DZ)
    cells = np.zeros((nx, ny, nz), dtype=np.uint8)
    if cut:                                   # an asymmetric cross-section
        cells[:2, :, :] = 1
        cells[:, :3, :] = 1
        cells[nx - 3:, ny - 2:, :] = 1
    if collimator is not None:                # jaws |y - yc| >= h over planes k0 .. k1-1
        k0, k1, h = collimator
        yc = ny // 2
        for j in range(ny):
            if abs(j + 0.5 - yc) >= h:
                cells[:, j, k0:k1] = 1
    return g, cells, O.vacuum_materials(g, cells)


def test_potential_matches_discrete_sine_series(po):
    """Rectangle (dx != dy): phi equals the eigen-expansion of the 5-point
    operator, sum_ab (2/nx)(2/ny) s_a(i0) s_b(j0) s_a(i) s_b(j) / lambda_ab,
    lambda_ab = (dy/dx)(2 - 2 cos(a pi/nx)) + (dx/dy)(2 - 2 cos(b pi/ny))."""
    nx, ny = 9, 13
    g, cells, m = _pipe_grid(nx, ny, 4, dx=1.7 * DZ, dy=2.9 * DZ, cut=False)
    i0, j0 = 4, 5
    phi = po.potential(g, po.pec_nodes(m), i0, j0)
    a = np.arange(1, nx)[:, None]
    b = np.arange(1, ny)[None, :]
    lam = (g.dy / g.dx) * (2 - 2 * np.cos(a * np.pi / nx)) + (g.dx / g.dy) * (2 - 2 * np.cos(b * np.pi / ny))
    ref = np.zeros((nx + 1, ny + 1))
    for i in range(nx + 1):
        for j in range(ny + 1):
            si = np.sin(a * np.pi * i / nx) * np.sin(a * np.pi * i0 / nx)
            sj = np.sin(b * np.pi * j / ny) * np.sin(b * np.pi * j0 / ny)
            ref[i, j] = (4.0 / (nx * ny)) * np.sum(si * sj / lam)
    assert np.abs(phi - ref).max() <= 1e-13 * np.abs(ref).max()


def _run(po, g, m, i0, j0, M, n0, steps, sigma=2.5 * DZ, jmin=None, nw=40, kend=0, energy=False):
    b = O.Bunch(Q=1e-9, sigma=sigma, i0=i0, j0=j0, M=M, jmin=-M if jmin is None else jmin, nw=nw, kend=kend)
    out = po.run(g, m, b, n0, steps, want_energy=energy)
    return b, out


@pytest.mark.parametrize("i0,j0,ratio", [(5, 7, 1.0), (6, 9, 0.6)])
def test_self_field_moves_one_cell_per_step(po, i0, j0, ratio):
    """A uniform pipe (asymmetric, off-centre bunch, dx != dy): after 30 steps
    the fields ahead of the entrance wall's causal front equal the field built
    for the later step, e_z and h_z stay 0 to rounding, and W^{n,e} is
    constant."""
    g, cells, m = _pipe_grid(12, 16, 90, dx=2 * DZ, dy=2 * DZ * ratio)
    M, n0, K = 15, 40, 30
    b, out = _run(po, g, m, i0, j0, M, n0, K, energy=True)
    f = out["field"]
    lam = O.bunch_cells(b.Q, b.sigma, DZ, M)
    ref = po.self_field(g, m, out["phi"], lam, M, n0 + K)
    scale = max(np.abs(ref[k]).max() for k in O.KEYS)
    front = K + 2                             # the wall's influence after K steps
    for k in O.KEYS:
        assert np.abs(f[k][:, :, front:] - ref[k][:, :, front:]).max() <= 1e-13 * scale, k
    # behind the front only the cut checkerboard tail acts, at its own level
    F = po.profile(lam, M, g.cdt, np.arange(-2 * M - 1, 1))
    tail = abs(F[0]) / np.abs(F).max()
    assert 0 < tail < 1e-7
    assert np.abs(f["ez"]).max() <= 0.1 * tail * scale
    assert np.abs(f["ez"][:, :, front:]).max() <= 1e-14 * scale
    assert np.abs(f["hz"]).max() <= 1e-14 * scale
    e = out["energy"]
    assert np.ptp(e) <= 1e-13 * e[0]


def test_self_field_node_charges_are_the_bunch(po):
    """The conserved charges (35) of the first step: q_e at the bunch line's
    nodes k equals the charge of bunch cell k - n0 - 1 + M, and every other
    interior node and every cell (q_h) holds none."""
    g, cells, m = _pipe_grid(10, 14, 70)
    i0, j0, M, n0 = 5, 7, 10, 30
    b = O.Bunch(Q=1e-9, sigma=2.0 * DZ, i0=i0, j0=j0, M=M, jmin=-M, nw=10)
    phi = po.potential(g, po.pec_nodes(m), i0, j0)
    lam = O.bunch_cells(b.Q, b.sigma, DZ, M)
    fo = po.self_field(g, m, phi, lam, M, n0)
    fn = {k: v.copy() for k, v in fo.items()}
    O.run(g, m, fn, 1, n0=n0, bunch=b)
    qe, qh = O.charges(g, m, fo, fn)
    want = np.zeros_like(qe)
    for k in range(g.nz + 1):
        c = k - n0 - 1 + M
        if -M <= c <= M:
            want[i0, j0, k] = lam[c + M]
    inner = np.zeros(qe.shape, dtype=bool)
    inner[1:-1, 1:-1, 3:-1] = True            # nodes with six edges (and clear of the wall's cut)
    inner &= m["ez"] > 0
    err = np.abs(qe - want)[inner].max()
    assert err <= 1e-12 * b.Q
    assert np.abs(qh).max() <= 1e-12 * b.Q * max(1.0 / g.dx, 1.0 / DZ)
    assert np.abs(want).max() > 0.1 * b.Q


def test_uniform_pipe_wake_vanishes(po):
    """Open pipes: the wake of a uniform pipe is 0 to rounding for the samples
    the entrance cut cannot reach; the closed box's wake on the same grid is
    not (the bunch leaves the z = 0 wall)."""
    g, cells, m = _pipe_grid(12, 16, 150)
    i0, j0, M, n0 = 6, 8, 15, 60
    jmax = n0 - M - 2
    b, out = _run(po, g, m, i0, j0, M, n0, 80, jmin=-M, nw=jmax + M + 1)
    W = out["acc"] / b.Q
    bc = O.Bunch(Q=b.Q, sigma=b.sigma, i0=i0, j0=j0, M=M, jmin=-M, nw=jmax + M + 1)
    fc = O.zeros(g)
    Wc = O.run(g, m, fc, n0 + 80, bunch=bc)["acc"] / b.Q
    assert np.abs(Wc).max() > 1e3 * np.abs(W).max()
    assert np.abs(W).max() <= 1e-12 * np.abs(Wc).max()


def _collimator_wake(po, pre, post, kend_rel, n0_rel=-2, M=10, jmax=30):
    """Wake of a short collimator (planes k0 .. k0+12) with `pre` pipe planes
    before it and `post` planes after it; n0 sits n0_rel planes from the
    collimator's first plane, kend kend_rel planes after its last (or 0)."""
    k0 = pre
    nz = pre + 12 + post
    g, cells, m = _pipe_grid(10, 14, nz, cut=False, collimator=(k0, k0 + 12, 4))
    n0 = k0 + n0_rel
    kend = k0 + 12 + kend_rel if kend_rel is not None else 0
    steps = (kend if kend else nz) + M + jmax
    b, out = _run(po, g, m, 5, 7, M, n0, steps - n0, sigma=2.0 * DZ, jmin=-M, nw=jmax + M + 1, kend=kend)
    return out["acc"] / b.Q


def test_exit_truncation_is_causal(po):
    """A longer outgoing pipe changes nothing when the quadrature ends early
    enough (bitwise: the same operations on the same values); with the
    quadrature over all edges it does (the exit wall's reflection)."""
    M, jmax = 10, 30
    post = (M + jmax + 2 + 1) // 2 + 4        # kend = collimator end + 4 = nz - (M + jmax + 3)//2
    Wa = _collimator_wake(po, 50, post, 4, M=M, jmax=jmax)
    Wb = _collimator_wake(po, 50, post + 9, 4, M=M, jmax=jmax)
    assert np.array_equal(Wa, Wb)
    assert np.abs(Wa).max() > 0
    Wc = _collimator_wake(po, 50, post, None, M=M, jmax=jmax)
    Wd = _collimator_wake(po, 50, post + 9, None, M=M, jmax=jmax)
    assert np.abs(Wc - Wd).max() > 1e-6 * np.abs(Wc).max()


def test_entrance_length_does_not_matter(po):
    """A longer ingoing pipe (the bunch starting the same distance before the
    collimator) gives the same wake to rounding for the samples that neither
    the entrance cut nor the entrance wall's reflection can reach."""
    M, jmax = 10, 30
    post = (M + jmax + 2 + 1) // 2 + 4
    pre = jmax + 2 * M + 6                    # n0 - M - 1 > jmax and 2 kst - M - 1 > jmax
    Wa = _collimator_wake(po, pre, post, 4, M=M, jmax=jmax)
    Wb = _collimator_wake(po, pre + 13, post, 4, M=M, jmax=jmax)
    assert np.abs(Wa - Wb).max() <= 1e-13 * np.abs(Wa).max()
    assert np.abs(Wa).max() > 0


def test_uniformity_and_node_checks(po):
    """The oracle refuses a start inside a non-uniform pipe and a bunch on
    PEC."""
    g, cells, m = _pipe_grid(10, 14, 60, cut=False, collimator=(20, 30, 4))
    b = O.Bunch(Q=1e-9, sigma=2e-3, i0=5, j0=7, M=5, jmin=-5, nw=10)
    assert po.uniform_entrance(g, m, 20)
    assert not po.uniform_entrance(g, m, 21)
    with pytest.raises(ValueError):
        po.run(g, m, b, 20, 1)
    g2, cells2, m2 = _pipe_grid(10, 14, 60)
    with pytest.raises(ValueError):
        po.potential(g2, po.pec_nodes(m2), 1, 7)


# ---- the rotationally symmetric scheme (24)
from oracle import rz_oracle as Z   # noqa: E402


def _rz_pipe(mode, nr=20, nz=90, radius=15, collimator=None):
    dr = 1.2 * DZ if mode == 0 else DZ          # m = 0 is stable for dtau <= 0.9089 dr
    g = Z.RZGeom(nr, nz, dr, DZ, DZ, mode)
    cells = np.zeros((nr, nz), bool)
    cells[radius:, :] = True
    if collimator is not None:
        k0, k1, r_in = collimator
        cells[r_in:, k0:k1] = True
    return g, Z.materials(g, cells)


@pytest.mark.parametrize("mode,j0", [(0, 0), (1, 4), (2, 6)])
def test_rz_self_field_moves_one_cell_per_step(po, mode, j0):
    """r-z pipe of radius 15 dr, a ring bunch at mode m: after 30 steps the
    fields ahead of the entrance wall's front equal the state built for the
    later step, e_z and h_z stay 0 to rounding, the energy of (24) is
    constant."""
    g, m = _rz_pipe(mode)
    M, n0, K = 15, 40, 30
    b = Z.RZBunch(1e-9, 2.5 * DZ, j0, M, 5, -M, 20)
    out = po.rz_run(g, m, b, n0, K, want_energy=True)
    f = out["field"]
    lam = Z.bunch_cells(b.Q, b.sigma, DZ, M)
    ref = po.rz_self_field(g, m, out["phi"], lam, M, n0 + K)
    sc = max(np.abs(ref[k]).max() for k in Z.KEYS)
    front = K + 2
    for k in Z.KEYS:
        assert np.abs(f[k][:, front:] - ref[k][:, front:]).max() <= 1e-13 * sc, k
    assert np.abs(f["ez"][:, front:]).max() <= 1e-14 * sc
    assert np.abs(f["hz"]).max() <= 1e-14 * sc
    e = np.array(out["energy"])
    assert np.ptp(e) <= 1e-13 * e[0]


@pytest.mark.parametrize("mode,j0", [(0, 0), (1, 4)])
def test_rz_self_field_node_charges_are_the_ring(po, mode, j0):
    """The r-z node charges of the first step: the ring's weighted cell
    charge on its node line, nothing at the other free nodes."""
    g, m = _rz_pipe(mode)
    M, n0 = 10, 30
    b = Z.RZBunch(1e-9, 2.0 * DZ, j0, M, 5, -M, 10)
    phi = po.rz_potential(g, m, j0)
    lam = Z.bunch_cells(b.Q, b.sigma, DZ, M)
    fo = po.rz_self_field(g, m, phi, lam, M, n0)
    fn = {k: v.copy() for k, v in fo.items()}
    Z.run(g, m, fn, 1, n0=n0, bunch=b)
    q = Z.charge(g, m, fo, fn)
    want = np.zeros_like(q)
    for k in range(g.nz + 1):
        c = k - n0 - 1 + M
        if -M <= c <= M:
            want[j0, k] = Z.mode_weight(mode) * lam[c + M]
    inner = np.zeros(q.shape, bool)
    inner[:14, 3:-1] = True                      # nodes with free edges, clear of the wall's cut
    inner &= m["ez"] > 0
    assert np.abs(q - want)[inner].max() <= 1e-12 * b.Q
    assert np.abs(want).max() > 0.1 * Z.mode_weight(mode) * b.Q


def test_rz_uniform_pipe_wake_vanishes(po):
    """Mode 1, uniform pipe: both wake lines are 1e-12 of the closed box's
    for the samples the entrance cut cannot reach."""
    g, m = _rz_pipe(1, nz=150)
    M, n0 = 15, 60
    nw = (n0 - M - 2) + M + 1
    b = Z.RZBunch(1e-9, 2.5 * DZ, 4, M, 5, -M, nw)
    W = po.rz_run(g, m, b, n0, 80)["acc"]
    Wc = Z.run(g, m, Z.zeros(g), n0 + 80, bunch=Z.RZBunch(1e-9, 2.5 * DZ, 4, M, 5, -M, nw))["acc"]
    assert np.abs(Wc).max() > 1e3 * np.abs(W).max()
    assert np.abs(W).max() <= 1e-12 * np.abs(Wc).max()


def test_rz_exit_truncation_is_causal(po):
    """An iris between open pipes: a longer outgoing pipe leaves the wake
    bitwise unchanged when the quadrature ends early enough."""
    M, jmax = 10, 24
    out = []
    k0 = 45
    kend = k0 + 14                               # 4 planes past the iris
    for post in (4 + (M + jmax + 3) // 2, 13 + (M + jmax + 3) // 2):
        g, m = _rz_pipe(1, nz=k0 + 10 + post, collimator=(k0, k0 + 10, 8))
        assert g.nz - kend >= (M + jmax + 3) // 2
        b = Z.RZBunch(1e-9, 2.0 * DZ, 4, M, 5, -M, jmax + M + 1, kend=kend)
        steps = kend + M + jmax - (k0 - 2)
        out.append(po.rz_run(g, m, b, k0 - 2, steps)["acc"])
    assert np.array_equal(out[0], out[1])
    assert np.abs(out[0]).max() > 0
