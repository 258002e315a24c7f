"""The open-pipe oracle against closed boxes (CPU).

Open pipes stand for infinite entrance and exit pipes (Sec. 5; the oracle's
reading is in ``oracle/pipe_oracle``).  A closed box with a long entrance pipe
approaches the same physics as the pipe grows: the field the bunch makes when
it leaves the z = 0 wall falls behind it (catch-up), so the difference of two
closed-box runs that share the entrance pipe, one with and one without a
step-out into a wider pipe, tends to the step's own wake.  The closed boxes use
none of the open-pipe machinery (potential, self-field, profile, quadrature
end), so this pins it from outside: the loss factor k = sum_j W(s_j) lam_j of
the open-pipe run equals the closed-box limit, and the closed-box difference
approaches it as the entrance pipe grows (3-D, scheme (23); r-z, scheme (24)
at m = 0)."""
import numpy as np

from oracle import oracle as O
from oracle import pipe_oracle as PO
from oracle import rz_oracle as Z

DZ = 1e-3
SIG = 1.5 * DZ
M = 9                       # ceil(6 sigma / dz)
JMIN, JMAX = -M, 2 * M
NW = JMAX - JMIN + 1


def _loss(W, lam):
    return float(np.sum(W[:2 * M + 1] * lam))


def _aperture(n, half):
    i = np.arange(n)[:, None] + 0.5 - n / 2
    return (np.abs(i) > half) | (np.abs(i.T) > half)


def test_3d_step_out_open_pipes_equal_closed_box_limit(po=PO):
    """Square pipe of 12 x 12 cells entered through a 6 x 6 aperture pipe; the
    exit pipe runs 200 planes past the step."""
    n, L = 12, 200
    ap = _aperture(n, 3)
    lam = O.bunch_cells(1.0, SIG, DZ, M)

    def geom(nz):
        return O.Geom(n, n, nz, 2 * DZ, 2 * DZ, DZ, DZ)

    def cells(nz, kst):
        c = np.zeros((n, n, nz), np.uint8)
        c[:, :, :kst] = ap[:, :, None]
        return c

    def bunch(kend):
        return O.Bunch(Q=1.0, sigma=SIG, i0=n // 2, j0=n // 2, M=M, jmin=JMIN, nw=NW, kend=kend)

    k0 = 2 * M + 12
    kend = k0 + L
    nz = kend + (M + JMAX + 3) // 2 + 4
    g = geom(nz)
    k_open = _loss(po.run(g, O.vacuum_materials(g, cells(nz, k0)), bunch(kend), k0 - 1,
                          kend + M + JMAX - k0 + 2)["acc"], lam)
    errs = []
    for E in (100, 200):
        kend2 = E + L
        nz2 = kend2 + (M + JMAX + 3) // 2 + 4
        g2 = geom(nz2)
        W = []
        for kst in (E, nz2):             # with the step-out at E, and the aperture pipe throughout
            W.append(O.run(g2, O.vacuum_materials(g2, cells(nz2, kst)), O.zeros(g2), kend2 + M + JMAX + 1,
                           bunch=bunch(kend2))["acc"])
        errs.append(abs(_loss(W[0] - W[1], lam) - k_open) / abs(k_open))
    assert k_open > 0
    assert errs[1] < errs[0] / 5
    assert errs[1] < 2e-4


def test_rz_step_out_open_pipes_equal_closed_box_limit(po=PO):
    """Round pipe of radius 12 dr entered through a pipe of radius 5 dr
    (dr = 1.2 dz, m = 0); the exit pipe runs 300 planes past the step."""
    nb, na, L = 12, 5, 300
    dr = 1.2 * DZ
    lam = Z.bunch_cells(1.0, SIG, DZ, M)

    def run_closed(E, step):
        kend = E + L
        nz = kend + (M + JMAX + 3) // 2 + 4
        g = Z.RZGeom(nb, nz, dr, DZ, DZ, 0)
        c = np.zeros((nb, nz), bool)
        c[na:, :E if step else nz] = True
        b = Z.RZBunch(1.0, SIG, 0, M, 0, JMIN, NW, kend=kend)
        return Z.run(g, Z.materials(g, c), Z.zeros(g), kend + M + JMAX + 1, bunch=b)["acc"][0]

    k0 = 2 * M + 12
    kend = k0 + L
    nz = kend + (M + JMAX + 3) // 2 + 4
    g = Z.RZGeom(nb, nz, dr, DZ, DZ, 0)
    c = np.zeros((nb, nz), bool)
    c[na:, :k0] = True
    b = Z.RZBunch(1.0, SIG, 0, M, 0, JMIN, NW, kend=kend)
    k_open = _loss(po.rz_run(g, Z.materials(g, c), b, k0 - 1, kend + M + JMAX - k0 + 2)["acc"][0], lam)
    errs = [abs(_loss(run_closed(E, True) - run_closed(E, False), lam) - k_open) / abs(k_open) for E in (120, 240)]
    assert k_open > 0
    assert errs[1] < errs[0] / 5
    assert errs[1] < 1e-5
