"""Oracle evaluation of single output points of a large run.

After s steps of the explicit scheme an entry depends only on initial data
within 4 s cells transversely and s cells along z (each half step reaches two
cells transversely through its recomputed intermediate sub-update and one
cell along z).  The oracle therefore reproduces any sampled entry of a large
grid from a sub-box around it with a margin beyond that radius; the sub-box's
own walls lie outside the domain of dependence."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

KEYS = O.KEYS


def subbox_bounds(p, shape, steps):
    rt, rz = 4 * steps + 3, steps + 3
    nx, ny, nz = shape[0] - 1, shape[1] - 1, shape[2] - 1
    lo = (max(0, p[0] - rt), max(0, p[1] - rt), max(0, p[2] - rz))
    hi = (min(nx, p[0] + rt), min(ny, p[1] + rt), min(nz, p[2] + rz))
    return lo, hi


def oracle_point(p, shape, dx, dy, dz, cdt, fields_slice, cells_slice, steps):
    """fields_slice(lo, hi) -> dict of float64 node arrays [lo..hi] inclusive;
    cells_slice(lo, hi) -> uint8 cells [lo..hi) or None.  Returns the six
    component values at p after `steps` steps (None where out of range)."""
    lo, hi = subbox_bounds(p, shape, steps)
    g = O.Geom(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], dx, dy, dz, cdt)
    m = O.vacuum_materials(g, cells_slice(lo, hi))
    f = fields_slice(lo, hi)
    f = {k: np.ascontiguousarray(f[k], dtype=np.float64) for k in KEYS}
    O.apply_pec(g, m, f)
    O.run(g, m, f, steps)
    q = (p[0] - lo[0], p[1] - lo[1], p[2] - lo[2])
    return {k: f[k][q] for k in KEYS}, f
