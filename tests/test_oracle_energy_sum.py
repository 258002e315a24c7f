"""The oracle's energy sum is accurate to a few units of its last place.

W^{n,e} (Sec. 4.4) is evaluated as one sum over every grid entry; on the
full-size workloads that is ~1e8 terms, and a plain running sum would lose
~1e-12 of the total, the size of the parity tolerance.  The oracle sums with
compensation; here its value is held against the exactly rounded sum
(math.fsum) of the same terms, written out per entry from the expansion in
the oracle's header (squares, the alpha^2 transverse-difference terms and the
alpha coupling term), on a grid with a bunch-driven field and random fields."""
import math

import numpy as np

from paper_0901_1053_amd import inputs


def _sh(x, di, dj, dk):
    y = np.zeros_like(x)
    X, Y, Z = x.shape
    src = tuple(slice(max(0, d), n + min(0, d)) for d, n in zip((di, dj, dk), (X, Y, Z)))
    dst = tuple(slice(max(0, -d), n - max(0, d)) for d, n in zip((di, dj, dk), (X, Y, Z)))
    y[dst] = x[src]
    return y


def _exact_energy(g, m, f):
    nx, ny, nz = g.nx, g.ny, g.nz
    rng = {k: np.zeros(g.shape, bool) for k in f}
    rng["ex"][:nx] = True
    rng["ey"][:, :ny] = True
    rng["ez"][:, :, :nz] = True
    rng["hx"][:, :ny, :nz] = True
    rng["hy"][:nx, :, :nz] = True
    rng["hz"][:nx, :ny] = True
    a = 0.5 * g.cdt
    t = []
    for c in ("ex", "ey", "ez", "hx", "hy", "hz"):
        sel = rng[c] & (m[c] > 0)
        t.append(0.5 * f[c][sel] ** 2 / m[c][sel])
    d = _sh(f["ez"], 0, 1, 0) - f["ez"]
    t.append((-0.5 * a * a * m["hx"] * d * d)[rng["hx"]])
    d = _sh(f["ez"], 1, 0, 0) - f["ez"]
    t.append((-0.5 * a * a * m["hy"] * d * d)[rng["hy"]])
    sel = rng["ex"] & (m["ex"] > 0)
    d = _sh(f["hz"], 0, -1, 0) - f["hz"]
    t.append((-0.5 * a * a * m["ex"] * d * d)[sel])
    sel = rng["ey"] & (m["ey"] > 0)
    d = _sh(f["hz"], -1, 0, 0) - f["hz"]
    t.append((-0.5 * a * a * m["ey"] * d * d)[sel])
    t.append((a * f["hx"] * (_sh(f["ey"], 0, 0, 1) - f["ey"]))[rng["hx"]])
    t.append((-a * f["hy"] * (_sh(f["ex"], 0, 0, 1) - f["ex"]))[rng["hy"]])
    return math.fsum(np.concatenate([x.ravel() for x in t]))


def test_energy_sum_is_exactly_rounded_to_a_few_ulp(orc):
    case = inputs.scaled_wake_case(48, 160, seed=8, sigma_dz=2.5)
    g = orc.Geom(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt)
    m = orc.vacuum_materials(g, case.cell_mask())
    f = orc.zeros(g)
    b = orc.Bunch(Q=case.Q, sigma=case.sigma, i0=case.i0, j0=case.j0, M=case.M, jmin=case.jmin, nw=case.nw)
    orc.run(g, m, f, case.nz + case.M, bunch=b)
    for fields in (f, inputs.random_fields(g.shape, 9)):
        orc.apply_pec(g, m, fields)
        w = orc.energy(g, m, fields)
        ex = _exact_energy(g, m, fields)
        assert abs(w - ex) <= 8 * np.finfo(float).eps * abs(ex), (w, ex)
