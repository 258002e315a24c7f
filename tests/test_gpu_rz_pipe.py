"""Open entrance and exit pipes on the r-z grid (tete_rz_set_open_pipes)
against the r-z open-pipe oracle: the ring bunch's field in the uniform pipe
(the device's tridiagonal solve against the oracle's sparse solve of the same
radial problem), wakes of an iris between open pipes on both lines and the
transverse wake, the uniform pipe's vanishing wake, and the refusals.
Tolerances as in 3-D: 1e-12 (FP64) and 1e-6 (FP32 state) / 1e-5 (FP32 wakes,
the delta norm) relative to the FP64 oracle."""
import numpy as np
import pytest

from oracle import pipe_oracle as PO
from oracle import rz_oracle as Z
from paper_0901_1053_amd import tete

pytestmark = pytest.mark.gpu

EPS0 = 8.8541878128e-12
DZ = 1e-3
Q = 1e-9


def _geom(mode, nr, nz, radius, iris=None):
    dr = 1.2 * DZ if mode == 0 else DZ              # m = 0 is stable for dtau <= 0.9089 dr
    g = Z.RZGeom(nr, nz, dr, DZ, DZ, mode)
    cells = np.zeros((nr, nz), bool)
    cells[radius:, :] = True
    if iris is not None:
        k0, k1, r_in = iris
        cells[r_in:, k0:k1] = True
    return g, cells, Z.materials(g, cells)


def _grid(g, cells, precision):
    G = tete.RZGrid(g.nr, g.nz, g.dr, g.dz, g.cdt, g.m, precision)
    G.set_pec_cells(cells.astype(np.uint8))
    return G


def _delta(a, b):
    return float(np.max(np.abs(a - b)) / (np.max(b) - np.min(b)))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode,j0", [(0, 0), (1, 4), (2, 7)])
def test_rz_pipe_field_matches_oracle(precision, mode, j0):
    """The state of the ring's field in the pipe against the oracle's, every
    entry within 1e-12 (FP64) / 1e-6 (FP32) of the largest."""
    print("rz open-pipe field", precision, mode, flush=True)
    g, cells, m = _geom(mode, 24, 70, 18)
    M, n0 = 8, 30
    lam = Z.bunch_cells(Q, 2.0 * DZ, DZ, M)
    ref = PO.rz_self_field(g, m, PO.rz_potential(g, m, j0), lam, M, n0)
    G = _grid(g, cells, precision)
    G.set_bunch(Q, 2.0 * DZ, j0, M, 5, -M, 20)
    G.set_open_pipes(n0)
    assert G.steps_done() == n0
    f = G.get_fields()
    sc = max(np.abs(ref[k]).max() for k in Z.KEYS)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for k in Z.KEYS:
        assert np.abs(f[k] - ref[k]).max() <= tol * sc, k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mode,j0", [(0, 0), (1, 3)])
@pytest.mark.parametrize("kernel", ["auto", "fused"])
def test_rz_iris_between_open_pipes(precision, mode, j0, kernel):
    """An iris between open pipes: both wake lines within the delta norm 1e-12
    / 1e-5 of the oracle, for paired and single steps."""
    M, jmax = 10, 24
    k0 = 45
    kend = k0 + 14
    g, cells, m = _geom(mode, 20, kend + (M + jmax + 3) // 2, 15, iris=(k0, k0 + 10, 7))
    n0 = k0 - 2
    steps = kend + M + jmax - n0
    b = Z.RZBunch(Q, 2.0 * DZ, j0, M, 5, -M, jmax + M + 1, kend=kend)
    W = PO.rz_run(g, m, b, n0, steps)["acc"] / (Q * EPS0)
    G = _grid(g, cells, precision)
    G.set_tuning(kernel=kernel)
    G.set_bunch(Q, 2.0 * DZ, j0, M, 5, -M, jmax + M + 1)
    G.set_open_pipes(n0, kend)
    G.step(3)
    G.step(steps - 3)
    Wg, _ = G.wake()
    tol = 1e-12 if precision == "fp64" else 1e-5
    for line in range(2):
        assert np.abs(W[line]).max() > 0
        assert _delta(Wg[line], W[line]) <= tol, line


def test_rz_uniform_pipe_wake_vanishes():
    """Mode 1, uniform pipe: the open-pipe wake is 1e-12 of the closed box's
    for the samples the entrance cut cannot reach."""
    g, cells, m = _geom(1, 20, 150, 15)
    M, n0 = 15, 60
    nw = n0 - 1
    G = _grid(g, cells, "fp64")
    G.set_bunch(Q, 2.5 * DZ, 4, M, 5, -M, nw)
    G.set_open_pipes(n0)
    G.step(80)
    C = _grid(g, cells, "fp64")
    C.set_bunch(Q, 2.5 * DZ, 4, M, 5, -M, nw)
    C.step(n0 + 80)
    assert np.abs(G.wake()[0]).max() <= 1e-12 * np.abs(C.wake()[0]).max()


def test_rz_open_pipe_rules():
    """No bunch, ranges, a non-uniform entrance: refused, state unchanged; a
    new bunch ends the open-pipe run."""
    g, cells, m = _geom(1, 16, 60, 12, iris=(20, 30, 6))
    G = _grid(g, cells, "fp64")
    with pytest.raises(tete.TeteError) as e:
        G.set_open_pipes(5)
    assert e.value.status == "TETE_ERR_STATE"
    G.set_bunch(Q, 2 * DZ, 3, 6, 4, -6, 20)
    for n0, kend in ((20, 0), (-1, 0), (60, 0), (5, 61), (5, -1)):
        with pytest.raises(tete.TeteError) as e:
            G.set_open_pipes(n0, kend)
        assert e.value.status == "TETE_ERR_ARG", (n0, kend)
    assert G.steps_done() == 0
    G.set_open_pipes(10, 40)
    assert G.steps_done() == 10
    G.set_bunch(Q, 2 * DZ, 3, 6, 4, -6, 20)          # ends the run: quadrature over every edge again
    G.set_fields({k: np.zeros(g.shape) for k in Z.KEYS})
    G.step(60 + 6 + 13)
    C = _grid(g, cells, "fp64")
    C.set_bunch(Q, 2 * DZ, 3, 6, 4, -6, 20)
    C.step(60 + 6 + 13)
    assert np.array_equal(G.wake()[0], C.wake()[0])
