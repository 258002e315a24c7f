"""FP64 CPU oracle of the implicit TE/TM scheme (16) of Sec. 4.1.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product package;
it shares no code with the HIP path.

The scheme advances y^n = (u^{n-1/2}, v^n), u = (h_x, h_y, e_z), v = (e_x, e_y,
h_z), by the two half steps of (16): the transverse operators T_0, T_1 are taken
at the mean of the old and new level, the longitudinal coupling L explicitly,

    (I - alpha T_0) u^{n+1/2} = (I + alpha T_0) u^{n-1/2} + dtau (L v^n + j_u^n),
    (I - alpha T_1) v^{n+1}   = (I + alpha T_1) v^n       + dtau (-L^T u^{n+1/2} + j_v^{n+1/2}),

alpha = dtau / 2.  Here the operators act on FIT voltages with the material
matrices inside (the form of the semi-discrete system (15) in the grid's own
variables, as the explicit oracle uses for (23)):

    T_0 u = ( -mu_x P_y e_z,  mu_y P_x e_z,  kappa_z (P_y^T h_x - P_x^T h_y) )
    L v   = (  mu_x P_z e_y, -mu_y P_z e_x,  0 )
    T_1 v = ( -kappa_x P_y^T h_z,  kappa_y P_x^T h_z,  mu_z (P_y e_x - P_x e_y) )
    -L^T u = ( kappa_x P_z^T h_y, -kappa_y P_z^T h_x, 0 )
    j_u = (0, 0, -kappa_z j_z),  j_v = 0 (the bunch current is along z),

with (P f)(i) = f(i+1) - f(i), P^T g(i) = g(i-1) - g(i), values outside a
component's range zero (periodic x, y wrap), and the current with its physical
sign as in the explicit oracle.  Each half step is one sparse linear system,
solved with a sparse LU factorisation (a library primitive); no elimination
or iteration of the method's own is used here.

Materials, ranges and the staircase rule are those of the explicit oracle
(``oracle.vacuum_materials``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O

KEYS = O.KEYS
EX, EY, EZ, HX, HY, HZ = range(6)


def _in_range(g: O.Geom, c: int, i, j, k):
    """Vectorised range test of component c (the explicit oracle's rule)."""
    imax, jmax = (g.nx - 1, g.ny - 1) if g.periodic_xy else (g.nx, g.ny)
    ok = (i >= 0) & (j >= 0) & (k >= 0) & (i <= imax) & (j <= jmax) & (k <= g.nz)
    per = g.periodic_xy
    if c == EX:
        return ok & (per | (i < g.nx))
    if c == EY:
        return ok & (per | (j < g.ny))
    if c == EZ:
        return ok & (k < g.nz)
    if c == HX:
        return ok & (per | (j < g.ny)) & (k < g.nz)
    if c == HY:
        return ok & (per | (i < g.nx)) & (k < g.nz)
    return ok & (per | ((i < g.nx) & (j < g.ny)))


class _Index:
    def __init__(self, g: O.Geom):
        self.g = g
        self.np = int(np.prod(g.shape))
        i, j, k = np.meshgrid(np.arange(g.nx + 1), np.arange(g.ny + 1), np.arange(g.nz + 1), indexing="ij")
        self.i, self.j, self.k = i.ravel(), j.ravel(), k.ravel()

    def flat(self, i, j, k):
        g = self.g
        if g.periodic_xy:
            i = np.mod(i, g.nx)
            j = np.mod(j, g.ny)
        return k + (g.nz + 1) * (j + (g.ny + 1) * i)


class Implicit:
    """Scheme (16) on a grid with given materials; the two half-step matrices
    are built and factorised once."""

    def __init__(self, g: O.Geom, m: dict):
        self.g, self.m = g, m
        self.a = 0.5 * g.cdt
        self.ix = _Index(g)
        n = self.ix.np
        self.n = n
        # operators on the stacked vectors u = (hx, hy, ez), v = (ex, ey, hz)
        self.T0 = self._op([(HX, EZ, "py", -1.0, "mu"), (HY, EZ, "px", +1.0, "mu"),
                            (EZ, HX, "pyt", +1.0, "ka"), (EZ, HY, "pxt", -1.0, "ka")], (HX, HY, EZ), (HX, HY, EZ))
        self.L = self._op([(HX, EY, "pz", +1.0, "mu"), (HY, EX, "pz", -1.0, "mu")], (HX, HY, EZ), (EX, EY, HZ))
        self.T1 = self._op([(EX, HZ, "pyt", -1.0, "ka"), (EY, HZ, "pxt", +1.0, "ka"),
                            (HZ, EX, "py", +1.0, "mu"), (HZ, EY, "px", -1.0, "mu")], (EX, EY, HZ), (EX, EY, HZ))
        self.mLT = self._op([(EX, HY, "pzt", +1.0, "ka"), (EY, HX, "pzt", -1.0, "ka")], (EX, EY, HZ), (HX, HY, EZ))
        I = sp.identity(3 * n, format="csc")
        self.lu0 = spla.splu((I - self.a * self.T0).tocsc())
        self.lu1 = spla.splu((I - self.a * self.T1).tocsc())
        self.P0 = (I + self.a * self.T0).tocsr()
        self.P1 = (I + self.a * self.T1).tocsr()

    def _op(self, terms, rows, cols):
        """Sparse operator: each term (c_out, c_in, diff, sign, coef) adds
        sign * coef[c_out] * (difference of c_in) to the c_out rows; rows and
        cols give the component order of the stacked output and input."""
        g, ix, n = self.g, self.ix, self.n
        R, C, V = [], [], []
        shift = {"px": (1, 0, 0), "py": (0, 1, 0), "pz": (0, 0, 1),
                 "pxt": (-1, 0, 0), "pyt": (0, -1, 0), "pzt": (0, 0, -1)}
        for c_out, c_in, d, sign, _ in terms:
            coef = self.m[KEYS[c_out]].ravel()
            out_ok = _in_range(g, c_out, ix.i, ix.j, ix.k) & (coef != 0.0)
            di, dj, dk = shift[d]
            ro = rows.index(c_out) * n + np.nonzero(out_ok)[0]
            i0, j0, k0 = ix.i[out_ok], ix.j[out_ok], ix.k[out_ok]
            cf = sign * coef[out_ok]
            # forward difference f(x+1) - f(x); transposed difference g(x-1) - g(x)
            for (si, sj, sk), w in (((di, dj, dk), +1.0), ((0, 0, 0), -1.0)):
                ii, jj, kk = i0 + si, j0 + sj, k0 + sk
                ok = _in_range(g, c_in, np.mod(ii, g.nx) if g.periodic_xy else ii,
                               np.mod(jj, g.ny) if g.periodic_xy else jj, kk)
                col = cols.index(c_in) * n + ix.flat(ii[ok], jj[ok], kk[ok])
                R.append(ro[ok])
                C.append(col)
                V.append(w * cf[ok])
        R, C, V = np.concatenate(R), np.concatenate(C), np.concatenate(V)
        return sp.csr_matrix((V, (R, C)), shape=(3 * n, 3 * n))

    def _stack(self, f, comps):
        return np.concatenate([f[KEYS[c]].ravel() for c in comps])

    def _unstack(self, x, f, comps):
        for q, c in enumerate(comps):
            f[KEYS[c]][...] = x[q * self.n:(q + 1) * self.n].reshape(self.g.shape)

    def step(self, f: dict, jz=None) -> None:
        """One step of (16) in place; jz (or None) is j_z^n per e_z edge as
        current through its dual facet."""
        dt = self.g.cdt
        u = self._stack(f, (HX, HY, EZ))
        v = self._stack(f, (EX, EY, HZ))
        rhs = self.P0 @ u + dt * (self.L @ v)
        if jz is not None:
            rhs[2 * self.n:] -= dt * self.m["ez"].ravel() * jz.ravel()
        u1 = self.lu0.solve(rhs)
        v1 = self.lu1.solve(self.P1 @ v + dt * (self.mLT @ u1))
        self._unstack(u1, f, (HX, HY, EZ))
        self._unstack(v1, f, (EX, EY, HZ))


def energy(g: O.Geom, m: dict, f: dict) -> float:
    """Discrete energy 1/2 <Q y, y> of (16) with Q = B - alpha A (Sec. 4.1): the
    transverse operators drop out of Q, leaving
        1/2 [sum h^2/mu + sum_{kappa>0} e^2/kappa] + alpha [sum_hx h_x P_z e_y - sum_hy h_y P_z e_x]."""
    a = 0.5 * g.cdt
    ix = _Index(g)
    s = 0.0
    for c in range(6):
        key = KEYS[c]
        ok = _in_range(g, c, ix.i, ix.j, ix.k)
        coef = m[key].ravel()
        sel = ok & (coef > 0)
        s += 0.5 * float(np.sum(f[key].ravel()[sel] ** 2 / coef[sel]))

    def at(c, i, j, k):
        ok = _in_range(g, c, np.mod(i, g.nx) if g.periodic_xy else i, np.mod(j, g.ny) if g.periodic_xy else j, k)
        out = np.zeros(i.shape)
        out[ok] = f[KEYS[c]].ravel()[ix.flat(i[ok], j[ok], k[ok])]
        return out
    i, j, k = ix.i, ix.j, ix.k
    okx = _in_range(g, HX, i, j, k)
    oky = _in_range(g, HY, i, j, k)
    lc = np.sum((f["hx"].ravel() * (at(EY, i, j, k + 1) - at(EY, i, j, k)))[okx])
    lc -= np.sum((f["hy"].ravel() * (at(EX, i, j, k + 1) - at(EX, i, j, k)))[oky])
    return s + a * float(lc)


def charge(g: O.Geom, m: dict, fo: dict, fn: dict) -> np.ndarray:
    """Node charges of (16): q^{n+1/2} = -[P_x^T dbar_x + P_y^T dbar_y + P_z^T d_z^{n+1/2}]
    with d = e / kappa (0 on PEC edges), dbar = (d^n + d^{n+1}) / 2; fo = y^n and
    fn = y^{n+1}.  Between steps it changes by dtau (j(k-1) - j(k)) at nodes
    whose six edges are free."""
    ix = _Index(g)
    i, j, k = ix.i, ix.j, ix.k

    def d(f, c):
        coef = m[KEYS[c]].ravel()
        ok = _in_range(g, c, i, j, k) & (coef > 0)
        out = np.zeros(ix.np)
        out[ok] = f[KEYS[c]].ravel()[ok] / coef[ok]
        return out
    dx = 0.5 * (d(fo, EX) + d(fn, EX))
    dy = 0.5 * (d(fo, EY) + d(fn, EY))
    dz = d(fn, EZ)

    def back(arr, c, si, sj, sk):          # arr at (i+si, j+sj, k+sk), zero outside the component's range
        ii, jj, kk = i + si, j + sj, k + sk
        ok = _in_range(g, c, np.mod(ii, g.nx) if g.periodic_xy else ii, np.mod(jj, g.ny) if g.periodic_xy else jj, kk)
        out = np.zeros(ix.np)
        out[ok] = arr[ix.flat(ii[ok], jj[ok], kk[ok])]
        return out
    q = -((back(dx, EX, -1, 0, 0) - dx) + (back(dy, EY, 0, -1, 0) - dy) + (back(dz, EZ, 0, 0, -1) - dz))
    return q.reshape(g.shape)
