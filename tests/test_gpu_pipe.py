"""Open entrance and exit pipes on the GPU (tete_set_open_pipes): the bunch's
field in the uniform entrance pipe (the cross-section's potential by
conjugate gradients on the device) and the wake quadrature that ends before
the exit wall's reflections, against the open-pipe oracle.

Tolerances: the device solves for the potential iteratively to a residual of
1e-16 and the oracle factorises the same matrix, so the two potentials (and
every field built from them) differ by about 1e-14 of their size; the fields
and wakes then keep the scheme's bars, 1e-12 in FP64 and 1e-5 (wake) / 2e-5
(fields) in FP32 relative to the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import pipe_oracle as PO
from oracle import witness_oracle as WO
from paper_0901_1053_amd import tete

pytestmark = pytest.mark.gpu

EPS0 = 8.8541878128e-12
DZ = 1e-3
Q = 1e-9


def _cells(nx, ny, nz, cut=True, collimator=None):
    cells = np.zeros((nx, ny, nz), dtype=np.uint8)
    if cut:
        cells[:2, :, :] = 1
        cells[:, :3, :] = 1
        cells[nx - 3:, ny - 2:, :] = 1
    if collimator is not None:
        k0, k1, h = collimator
        yc = ny // 2
        for j in range(ny):
            if abs(j + 0.5 - yc) >= h:
                cells[:, j, k0:k1] = 1
    return cells


def _grid(g, cells, precision, **kw):
    G = tete.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.cdt, precision=precision, **kw)
    G.set_pec_cells(cells)
    return G


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape,src,ratio", [((12, 16, 60), (5, 7), 1.0), ((23, 17, 41), (9, 10), 0.7),
                                             ((64, 48, 20), (30, 21), 1.3)])
def test_initial_field_matches_oracle(precision, shape, src, ratio):
    """The state written by tete_set_open_pipes against the oracle's field:
    every entry within 1e-12 (FP64) / 1e-6 (FP32, its rounding) of the
    largest; the step counter at n0; e_z and h_z zero."""
    nx, ny, nz = shape
    print("open-pipe field", shape, src, ratio, precision, flush=True)
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ * ratio, DZ, DZ)
    cells = _cells(nx, ny, nz)
    m = O.vacuum_materials(g, cells)
    M, n0 = 6, nz // 2
    phi = PO.potential(g, PO.pec_nodes(m), *src)
    lam = O.bunch_cells(Q, 1.5 * DZ, DZ, M)
    ref = PO.self_field(g, m, phi, lam, M, n0)
    G = _grid(g, cells, precision)
    G.set_bunch(Q, 1.5 * DZ, src[0], src[1], M, -M, 20)
    it = G.set_open_pipes(n0)
    assert 0 < it < 20 * (nx + ny) + 1000
    assert G.steps_done() == n0
    f = G.get_fields()
    scale = max(np.abs(ref[k]).max() for k in tete.KEYS)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for k in tete.KEYS:
        assert np.abs(f[k] - ref[k]).max() <= tol * scale, k
    assert not np.any(f["ez"]) and not np.any(f["hz"])


def _collimator(pre, post, kend_rel, M=8, jmax=26, nx=12, ny=16):
    k0 = pre
    nz = pre + 14 + post
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    cells = _cells(nx, ny, nz, cut=False, collimator=(k0, k0 + 14, 5))
    n0 = k0 - 2
    kend = k0 + 14 + kend_rel
    return g, cells, M, jmax, n0, kend


def _oracle_wake(g, cells, M, jmax, n0, kend, src=(6, 8), wit=None):
    m = O.vacuum_materials(g, cells)
    b = O.Bunch(Q=Q, sigma=2.0 * DZ, i0=src[0], j0=src[1], M=M, jmin=-M, nw=jmax + M + 1, kend=kend)
    steps = kend + M + jmax - n0
    if wit is None:
        return PO.run(g, m, b, n0, steps)["acc"] / (Q * EPS0), None
    phi = PO.potential(g, PO.pec_nodes(m), *src)
    lam = O.bunch_cells(Q, b.sigma, DZ, M)
    f = PO.self_field(g, m, phi, lam, M, n0)
    r = WO.run(g, m, f, steps, b, WO.witness_lines(*wit), n0=n0)
    return r["src_acc"] / (Q * EPS0), r["acc"] / (Q * EPS0)


def _gpu_wake(g, cells, M, jmax, n0, kend, precision, src=(6, 8), wit=None, kernel="auto", chunks=(None,), **kw):
    G = _grid(g, cells, precision, **kw)
    if kernel != "auto":
        G.set_tuning(kernel=kernel)
    G.set_bunch(Q, 2.0 * DZ, src[0], src[1], M, -M, jmax + M + 1)
    if wit is not None:
        G.set_witness(*wit)
    G.set_open_pipes(n0, kend)
    steps = kend + M + jmax - n0
    if chunks == (None,):
        G.step(steps)
    else:
        done = 0
        for c in chunks:
            G.step(c)
            done += c
        G.step(steps - done)
    return G


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kernel", ["auto", "fused", "split"])
def test_collimator_wake_matches_oracle(precision, kernel):
    """A collimator between open pipes: W(s) within the delta norm 1e-12
    (FP64) / 1e-5 (FP32) of the oracle, for the two-step kernel, the fused
    single step and the reference kernels."""
    g, cells, M, jmax, n0, kend = _collimator(30, 22, 4)
    print("open-pipe wake", precision, kernel, g.nz, n0, kend, flush=True)
    W, _ = _oracle_wake(g, cells, M, jmax, n0, kend)
    G = _gpu_wake(g, cells, M, jmax, n0, kend, precision, kernel=kernel, chunks=(1, 6, 3))
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.abs(W).max() > 0
    assert _rel(G.wake(), W) <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_witness_lines_end_with_the_quadrature(precision):
    """Witness lines of an open-pipe run take the same quadrature end: the five
    W_par lines within 1e-12 / 1e-5 of the witness oracle run from the pipe
    field."""
    g, cells, M, jmax, n0, kend = _collimator(30, 22, 4)
    Wsrc, Wl = _oracle_wake(g, cells, M, jmax, n0, kend, wit=(6, 9))
    G = _gpu_wake(g, cells, M, jmax, n0, kend, precision, wit=(6, 9))
    gW, _, _ = G.witness_wake()
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert _rel(G.wake(), Wsrc) <= tol
    for l in range(5):
        assert _rel(gW[l], Wl[l]) <= tol, l


def test_skip_static_and_batch_are_bitwise_the_plain_run():
    """The static-tile skip and a batch member step an open-pipe run to
    bitwise the fields and wake of the plain grid (FP32, two-step kernel)."""
    nx, ny, k0, M, jmax = 12, 40, 30, 8, 26
    nz = k0 + 14 + 22
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    cells = np.zeros((nx, ny, nz), dtype=np.uint8)
    cells[:, :20, :] = 1                                 # a block of metal beside the pipe: static tiles
    cells[:, 34:, k0:k0 + 14] = 1                        # a one-sided collimator
    src, n0, kend = (6, 27), k0 - 2, k0 + 18
    steps = kend + M + jmax - n0
    A = _gpu_wake(g, cells, M, jmax, n0, kend, "fp32", src=src)
    S = _gpu_wake(g, cells, M, jmax, n0, kend, "fp32", src=src, skip_static=True)
    assert S.static_tiles()[0] > 0
    B1 = _grid(g, cells, "fp32")
    B1.set_bunch(Q, 2.0 * DZ, src[0], src[1], M, -M, jmax + M + 1)
    B1.set_open_pipes(n0, kend)
    B = tete.Batch("fp32")
    B.set_launch(graph_steps=4)
    B.set(0, B1)
    B.step(steps)
    assert B1.steps_done() == n0 + steps
    fa = A.get_fields()
    assert np.abs(A.wake()).max() > 0
    for H in (S, B1):
        assert np.array_equal(H.wake(), A.wake())
        fh = H.get_fields()
        for k in tete.KEYS:
            assert np.array_equal(fh[k], fa[k]), k
    B.set(0, None)
    B.close()


def test_uniform_pipe_wake_vanishes():
    """FP64, uniform pipe: the open-pipe wake is 1e-12 of the closed box's
    (which the bunch enters through the z = 0 wall) for the samples the
    entrance cut cannot reach."""
    nx, ny, nz = 14, 18, 160
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    cells = _cells(nx, ny, nz)
    M, n0 = 12, 60
    nw = (n0 - M - 2) + M + 1
    G = _grid(g, cells, "fp64")
    G.set_bunch(Q, 2.5 * DZ, 7, 9, M, -M, nw)
    G.set_open_pipes(n0)
    G.step(90)
    C = _grid(g, cells, "fp64")
    C.set_bunch(Q, 2.5 * DZ, 7, 9, M, -M, nw)
    C.step(n0 + 90)
    Wc = C.wake()
    assert np.abs(G.wake()).max() <= 1e-12 * np.abs(Wc).max()


def test_open_pipe_rules():
    """Refusals leave the state alone; set_fields and set_bunch end the run."""
    nx, ny, nz = 12, 16, 60
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    cells = _cells(nx, ny, nz, cut=False, collimator=(25, 35, 5))
    G = _grid(g, cells, "fp64")
    with pytest.raises(tete.TeteError) as e:              # no bunch
        G.set_open_pipes(10)
    assert e.value.status == "TETE_ERR_STATE"
    G.set_bunch(Q, 2 * DZ, 6, 8, 6, -6, 20)
    f0 = {k: np.random.default_rng(3).standard_normal(g.shape) for k in tete.KEYS}
    G.set_fields(f0)
    before = G.get_fields()
    for n0, kend, status in ((25, 0, "TETE_ERR_ARG"),     # the collimator starts at plane 25
                             (-1, 0, "TETE_ERR_ARG"), (nz, 0, "TETE_ERR_ARG"), (10, nz + 1, "TETE_ERR_ARG"),
                             (10, -1, "TETE_ERR_ARG")):
        with pytest.raises(tete.TeteError) as e:
            G.set_open_pipes(n0, kend)
        assert e.value.status == status, (n0, kend)
        after = G.get_fields()
        for k in tete.KEYS:
            assert np.array_equal(before[k], after[k]), (n0, kend, k)
    assert G.steps_done() == 0
    G.set_pec_cells(_cells(nx, ny, nz, cut=True))          # node (1, 8) now touches PEC cells
    G.set_bunch(Q, 2 * DZ, 1, 8, 6, -6, 20)
    with pytest.raises(tete.TeteError) as e:
        G.set_open_pipes(10)
    assert e.value.status == "TETE_ERR_ARG"
    for kw in ({"materials": True}, {"yee": True}, {"implicit": True}):
        cdt = DZ if not kw.get("yee") else 0.5 * DZ
        H = tete.Grid(nx, ny, nz, g.dx, g.dy, g.dz, cdt, precision="fp64", **kw)
        if not kw.get("yee"):
            H.set_bunch(Q, 2 * DZ, 6, 8, 6, -6, 20)
            with pytest.raises(tete.TeteError) as e:
                H.set_open_pipes(10)
            assert e.value.status == "TETE_ERR_STATE", kw
        H.close()
    # set_bunch ends the open-pipe run: the quadrature takes every edge again
    g2, cells2, M, jmax, n0, kend = _collimator(30, 22, 4)
    A = _gpu_wake(g2, cells2, M, jmax, n0, kend, "fp64")
    A.set_bunch(Q, 2.0 * DZ, 6, 8, M, -M, jmax + M + 1)
    A.set_fields({k: np.zeros(g2.shape) for k in tete.KEYS})
    A.step(g2.nz + M + jmax)
    C = _grid(g2, cells2, "fp64")
    C.set_bunch(Q, 2.0 * DZ, 6, 8, M, -M, jmax + M + 1)
    C.step(g2.nz + M + jmax)
    assert np.array_equal(A.wake(), C.wake())


def test_large_cross_section_potential():
    """A 512 x 512 cross-section (round pipe of 200 cells radius, off-centre
    bunch): the device's conjugate gradients converge, and e_x, e_y on the
    bunch's planes match the oracle's direct solve within 1e-12 of the
    largest (FP64)."""
    nx = ny = 512
    nz = 12
    g = O.Geom(nx, ny, nz, 2 * DZ, 2 * DZ, DZ, DZ)
    i = np.arange(nx)[:, None] + 0.5 - nx / 2
    j = np.arange(ny)[None, :] + 0.5 - ny / 2
    pec = (i * i + j * j) > 200.0 ** 2
    cells = np.repeat(pec[:, :, None], nz, axis=2).astype(np.uint8)
    m = O.vacuum_materials(g, cells)
    src = (nx // 2 + 37, ny // 2 - 21)
    M, n0 = 3, 8
    phi = PO.potential(g, PO.pec_nodes(m), *src)
    lam = O.bunch_cells(Q, 1.5 * DZ, DZ, M)
    ref = PO.self_field(g, m, phi, lam, M, n0)
    G = _grid(g, cells, "fp64")
    G.set_bunch(Q, 1.5 * DZ, src[0], src[1], M, -M, 10)
    it = G.set_open_pipes(n0)
    print("512 x 512 cross-section: %d conjugate-gradient iterations" % it, flush=True)
    assert 0 < it < 20 * (nx + ny) + 1000
    f = G.get_fields()
    for k in ("ex", "ey", "hx", "hy"):
        sc = np.abs(ref[k]).max()
        assert sc > 0
        assert np.abs(f[k] - ref[k]).max() <= 1e-12 * sc, k
