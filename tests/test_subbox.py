"""CPU check of the sampled-parity method: the oracle on a sub-box reproduces
the oracle on the full grid at the sampled points, bitwise."""
import numpy as np

from oracle import oracle as O
from paper_0901_1053_amd import inputs
from tests import parity as P
from tests.subbox import oracle_point


def test_subbox_reproduces_full_grid():
    nx, ny, nz, steps = 40, 36, 30, 3
    g = O.Geom(nx, ny, nz, 2.0, 2.0, 1.0, 1.0)
    cells = inputs.random_cells(nx, ny, nz, 5, frac=0.05)
    m = O.vacuum_materials(g, cells)
    f0 = inputs.random_fields(g.shape, 6)
    f = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, f)
    O.run(g, m, f, steps)
    masks = P.range_masks(g.shape)
    fz = {k: v.copy() for k, v in f0.items()}
    O.apply_pec(g, m, fz)       # the full grid's initial state as the library stores it
    for p in inputs.sample_points(g.shape, 7, count=24):
        vals, _ = oracle_point(p, g.shape, g.dx, g.dy, g.dz, g.cdt,
                               lambda lo, hi: {k: fz[k][lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] for k in O.KEYS},
                               lambda lo, hi: cells[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]], steps)
        for k in O.KEYS:
            if masks[k][p]:
                assert vals[k] == f[k][p], (p, k)
