"""FP64 CPU oracle of open (infinite) entrance and exit pipes for the 3-D
explicit TE/TM scheme (23).

TEST INFRASTRUCTURE ONLY: imported by the tests and the smoke check, never by
the product package; it shares no code with the HIP path.

The paper's 3-D example is a structure between infinite ingoing and outgoing
pipes (Sec. 5); the paper gives no method for them.  The reading used here
emulates both on a finite grid, exactly up to rounding for the samples it
names, by the scheme's own transport and by causality.

Entrance: the bunch's own field in a uniform pipe.  Let the grid be uniform
in z over the planes the field occupies, the bunch move at v = c on the node
line (i0, j0) with dtau = dz, and p = k - n.  The state y^n = (u^{n-1/2}, v^n)

    e_x = -(P_x phi) F(p),              e_y = -(P_y phi) F(p),
    h_x = (dx/dy) (P_y phi) F(p + 1),   h_y = -(dy/dx) (P_x phi) F(p + 1),
    e_z = h_z = 0

is carried by the scheme one cell per step, with the bunch current of
``oracle.run``, if

  - phi is the potential of the pipe's cross-section: (L phi)(i, j) = 1 at
    the bunch node and 0 at every other node whose e_z edge is not PEC, with
    phi = 0 on the nodes whose e_z edge is PEC, where
    (L phi)(i, j) = (dy/dx) (2 phi - phi(i+1, j) - phi(i-1, j))
                  + (dx/dy) (2 phi - phi(i, j+1) - phi(i, j-1));
  - (F(p) + F(p + 1)) / 2 = lambda_{p+M} / dtau, the current of edge k in
    step n (the charge of bunch cell p + M crosses edge k in step n), and
    F(p) = 0 for p > 0 (no field ahead of the head).

Why, in terms of the ten sub-updates of Sec. 4.2: with e_z = h_z = 0 the h_x,
h_y and e_x, e_y sub-updates (S1, S2, S4, S5 and S6, S7, S9, S10) reduce
along z, per transverse edge, to the one-dimensional leapfrog at Courant number
one (alpha mu_x dy/dx = alpha kappa_y dx/dy = 1/2 at dtau = dz in the vacuum
of Sec. 2), which moves any profile exactly one cell per step with h^{n+1/2}
tied to e^n as above; S8 leaves h_z = 0 because the transverse e is a
gradient; S3 leaves e_z = 0 because the transverse divergence
P_y^T h_x - P_x^T h_y at step n equals (F(p) + F(p+1))/2 (L phi), the current.

A run starts at step n0 with this field in place: the bunch centre then sits
on edge n0 - M, wholly inside the grid, and nothing appears at the entrance
wall.  The recurrence leaves behind the bunch a checkerboard F(p) = +-A, A the
alternating sum of the truncated bunch's cell charges (over dtau), a free wave
that carries no charge and moves with the bunch; the PEC wall at z = 0 cuts it
from step n0 on, and the cut follows the bunch at c, n0 - M cells behind its
centre: samples j < n0 - M - 1 never meet it.  A is about the charge of the
last bunch cell (1e-8 of the peak for a cut at six sigma).

Exit: the wake quadrature ends at edge kend.  Fields reach the exit wall
z = nz dz no earlier than step nz (nothing runs ahead of the bunch head), so a
reflected field reaches edge k no earlier than step 2 nz - k, while sample j
meets edge k in step k + M + j: every edge k < nz - (M + j + 2)/2 is met first.

Together: W(s_j) of the open-pipe run equals, up to rounding, the wake of the
same structure between infinitely long uniform pipes, integrated from the
grid's first plane to plane kend, for samples j < n0 - M - 1 and j <= 2 (nz -
kend) - M - 2, if the structure begins at a plane kst with 2 kst - M - 1 > j
(the entrance wall's reflection of the structure's field starts no earlier
than step 2 kst) and the entrance pipe covers the initial field (kst > n0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import oracle as O


def pec_nodes(m: dict) -> np.ndarray:
    """(nx+1, ny+1) bool: nodes of the entrance cross-section whose e_z edge
    (plane k = 0, spanning the first cell plane) is PEC."""
    return m["ez"][:, :, 0] == 0.0


def uniform_entrance(g: O.Geom, m: dict, kst: int) -> bool:
    """True if cell planes 0 .. kst-1 form a uniform vacuum pipe: every kappa
    there is 0 (PEC) or its vacuum value, every mu its vacuum value, and each
    component repeats its first plane inside the pipe (e_x, e_y from plane 1,
    the others from plane 0; plane 0 of e_x, e_y lies on the wall)."""
    vac = (g.dx / (g.dy * g.dz), g.dy / (g.dz * g.dx), g.dz / (g.dx * g.dy))
    for c, key in enumerate(("ex", "ey", "ez")):
        a = m[key][:, :, :kst]
        if not np.all((a == 0.0) | (a == vac[c])):
            return False
    for c, key in enumerate(("hx", "hy", "hz")):
        lo = 1 if key == "hz" else 0
        hi = m[key].shape[0] - (1 if key == "hy" or key == "hz" else 0)
        hj = m[key].shape[1] - (1 if key == "hx" or key == "hz" else 0)
        a = m[key][:hi, :hj, lo:kst]
        if not np.all(a == vac[c]):
            return False
    for key, lo in (("ex", 1), ("ey", 1), ("ez", 0), ("hx", 0), ("hy", 0), ("hz", 1)):
        a = m[key][:, :, lo:kst]
        if not np.array_equal(a, np.repeat(a[:, :, :1], a.shape[2], axis=2)):
            return False
    return True


def potential(g: O.Geom, pec: np.ndarray, i0: int, j0: int) -> np.ndarray:
    """phi of the cross-section: L phi = delta_(i0, j0) on the free nodes,
    phi = 0 on the PEC nodes, by a sparse direct solve (the library routine is
    the step; the matrix is L written out node by node)."""
    nx, ny = g.nx, g.ny
    free = ~pec
    if not free[i0, j0]:
        raise ValueError("the bunch node lies on PEC")
    ids = -np.ones((nx + 1, ny + 1), dtype=np.int64)
    nfree = int(free.sum())
    ids[free] = np.arange(nfree)
    wx, wy = g.dy / g.dx, g.dx / g.dy
    rows, cols, vals = [], [], []
    for i in range(nx + 1):
        for j in range(ny + 1):
            if not free[i, j]:
                continue
            r = ids[i, j]
            rows.append(r)
            cols.append(r)
            vals.append(2.0 * wx + 2.0 * wy)
            for di, dj, w in ((1, 0, wx), (-1, 0, wx), (0, 1, wy), (0, -1, wy)):
                a, b = i + di, j + dj
                if 0 <= a <= nx and 0 <= b <= ny and free[a, b]:
                    rows.append(r)
                    cols.append(ids[a, b])
                    vals.append(-w)
    A = sp.csc_matrix((vals, (rows, cols)), shape=(nfree, nfree))
    rhs = np.zeros(nfree)
    rhs[ids[i0, j0]] = 1.0
    phi = np.zeros((nx + 1, ny + 1))
    phi[free] = spl.spsolve(A, rhs)
    return phi


def profile(lam: np.ndarray, M: int, dtau: float, p: np.ndarray) -> np.ndarray:
    """F(p) for integer p: zero for p > 0, then (F(p) + F(p+1))/2 =
    lam[p + 2M] / dtau downwards from the head (bunch cell p + M, array index
    p + 2M), and the alternating continuation F(p) = -F(p+1) below p = -2M."""
    F = {1: 0.0}
    for q in range(0, -2 * M - 2, -1):
        cur = lam[q + 2 * M] / dtau if q >= -2 * M else 0.0
        F[q] = 2.0 * cur - F[q + 1]
    low = -2 * M - 1
    out = np.zeros(len(p))
    for t, q in enumerate(np.asarray(p, dtype=np.int64)):
        if q > 0:
            out[t] = 0.0
        elif q >= low:
            out[t] = F[int(q)]
        else:
            out[t] = F[low] * (1.0 if (low - q) % 2 == 0 else -1.0)
    return out


def self_field(g: O.Geom, m: dict, phi: np.ndarray, lam: np.ndarray, M: int, n0: int) -> dict:
    """The state y^{n0} above, PEC edges zeroed."""
    f = O.zeros(g)
    k = np.arange(g.nz + 1)
    Fe = profile(lam, M, g.cdt, k - n0)          # e at plane k, time n0
    Fh = profile(lam, M, g.cdt, k + 1 - n0)      # h at plane k + 1/2, time n0 - 1/2
    Ex = -(phi[1:, :] - phi[:-1, :])             # (i + 1/2, j)
    Ey = -(phi[:, 1:] - phi[:, :-1])             # (i, j + 1/2)
    f["ex"][:-1, :, :] = Ex[:, :, None] * Fe[None, None, :]
    f["ey"][:, :-1, :] = Ey[:, :, None] * Fe[None, None, :]
    f["hx"][:, :-1, :-1] = (-(g.dx / g.dy) * Ey)[:, :, None] * Fh[None, None, :-1]
    f["hy"][:-1, :, :-1] = ((g.dy / g.dx) * Ex)[:, :, None] * Fh[None, None, :-1]
    O.apply_pec(g, m, f)
    return f


def exit_limit(nz: int, M: int, jmax: int) -> int:
    """Largest kend for which every sample j <= jmax is met before any
    reflection from the exit wall."""
    return nz - (M + jmax + 2 + 1) // 2


def run(g: O.Geom, m: dict, bunch: O.Bunch, n0: int, nsteps: int, want_energy: bool = False) -> dict:
    """Open-pipe wake run: the self-field at step n0, then nsteps steps of
    ``oracle.run`` with the quadrature ending at bunch.kend.  Returns
    oracle.run's dict plus the field and phi."""
    if not uniform_entrance(g, m, n0 + 1):
        raise ValueError("cell planes 0 .. n0 are not a uniform vacuum pipe")
    phi = potential(g, pec_nodes(m), bunch.i0, bunch.j0)
    lam = O.bunch_cells(bunch.Q, bunch.sigma, g.dz, bunch.M)
    f = self_field(g, m, phi, lam, bunch.M, n0)
    out = O.run(g, m, f, nsteps, n0=n0, bunch=bunch, want_energy=want_energy)
    out["field"] = f
    out["phi"] = phi
    return out


# ---------------------------------------------------------------------------
# The rotationally symmetric scheme (24) at azimuthal mode m (Sec. 4.3), on the
# r-z grid of ``oracle/rz_oracle``.  The same construction: with e_z = h_z = 0
# the pairs (e_r, h_phi) and (e_phi, h_r) see the one-dimensional leapfrog at
# Courant number one along z (alpha^2 mu_phi kappa_r = alpha^2 kappa_phi mu_r =
# 1/4 at dtau = dz), S8 keeps h_z = 0 when P_r e_phi = m e_r, which the radial
# gradient form e_r = -P_r Phi, e_phi = -m Phi gives, and S3 keeps e_z = 0 when
# P_r^* h_phi - m h_r at step n equals the ring current.  With h tied to e as
# in 3-D (h = -2 alpha mu e for the pair (e_r, h_phi), +2 alpha mu_r e for
# (e_phi, h_r)), the last condition is the radial problem
#   (L_m Phi)(j) = [r_{j-1/2} (Phi_j - Phi_{j-1}) - r_{j+1/2} (Phi_{j+1} - Phi_j)] / dr
#                  + m^2 (dr / r_j) Phi_j = w_m delta_{j, j0}
# on the nodes whose e_z edge has kappa_z > 0 (r_{-1/2} = 0; on the axis for
# m = 0 the disk facet gives the row (Phi_0 - Phi_1) / 2), Phi = 0 on the
# others (the wall, the axis for m >= 1, PEC nodes), w_m the harmonic weight
# of the ring charge.  Then, with F the profile of the 3-D case:
#   e_phi = -m Phi_j F(p),  e_r = -(Phi_{j+1} - Phi_j) F(p),
#   h_phi = (r_{j+1/2} / dr)(Phi_{j+1} - Phi_j) F(p+1),  h_r = -(dr / r_j) m Phi_j F(p+1).
# ---------------------------------------------------------------------------
def rz_uniform_entrance(m: dict, kst: int) -> bool:
    """True if the r-z materials repeat along z over cell planes 0 .. kst-1
    (e_phi, e_r from plane 1, e_z and the h from plane 0)."""
    for key, lo in (("ephi", 1), ("er", 1), ("ez", 0), ("hphi", 0), ("hr", 0), ("hz", 1)):
        a = m[key][:, lo:kst]
        if not np.array_equal(a, np.repeat(a[:, :1], a.shape[1], axis=1)):
            return False
    return True


def rz_potential(g, m: dict, j0: int) -> np.ndarray:
    """Phi of the radial problem above by a sparse direct solve of L_m written
    out row by row."""
    import scipy.sparse as sp
    from oracle import rz_oracle as Z
    nr = g.nr
    free = m["ez"][:, 0] > 0.0
    if not free[j0]:
        raise ValueError("the ring lies on a node without e_z")
    ids = -np.ones(nr + 1, dtype=np.int64)
    ids[free] = np.arange(int(free.sum()))
    rows, cols, vals = [], [], []
    for j in range(nr + 1):
        if not free[j]:
            continue
        rm = (j - 0.5) * g.dr if j > 0 else 0.0
        rp = (j + 0.5) * g.dr
        diag = (rm + rp) / g.dr + (g.m * g.m * g.dr / (j * g.dr) if j > 0 else 0.0)
        rows.append(ids[j]); cols.append(ids[j]); vals.append(diag)
        for jj, w in ((j - 1, rm / g.dr), (j + 1, rp / g.dr)):
            if 0 <= jj <= nr and free[jj] and w != 0.0:
                rows.append(ids[j]); cols.append(ids[jj]); vals.append(-w)
    n = int(free.sum())
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    rhs = np.zeros(n)
    rhs[ids[j0]] = Z.mode_weight(g.m)
    phi = np.zeros(nr + 1)
    phi[free] = spl.spsolve(A, rhs)
    return phi


def rz_self_field(g, m: dict, phi: np.ndarray, lam: np.ndarray, M: int, n0: int) -> dict:
    """The r-z state y^{n0} above, with e on PEC edges and entries outside
    their range zeroed."""
    from oracle import rz_oracle as Z
    f = Z.zeros(g)
    k = np.arange(g.nz + 1)
    Fe = profile(lam, M, g.cdt, k - n0)
    Fh = profile(lam, M, g.cdt, k + 1 - n0)
    j = np.arange(g.nr + 1, dtype=float)
    Ep = -g.m * phi                                   # e_phi shape at node j
    Er = np.zeros(g.nr + 1)
    Er[:-1] = -(phi[1:] - phi[:-1])                   # e_r shape at j + 1/2
    f["ephi"] = Ep[:, None] * Fe[None, :]
    f["er"] = Er[:, None] * Fe[None, :]
    f["hphi"] = (((j + 0.5) * g.dr / g.dr) * (-Er))[:, None] * Fh[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        hr = np.where(j > 0, (g.dr / (j * g.dr)) * Ep, 0.0)
    f["hr"] = hr[:, None] * Fh[None, :]
    Z.apply_pec(g, m, f)
    return f


def rz_run(g, m: dict, bunch, n0: int, nsteps: int, want_energy: bool = False) -> dict:
    """Open-pipe r-z wake run: the self-field at step n0, then nsteps steps of
    ``rz_oracle.run`` with the quadrature ending at bunch.kend."""
    from oracle import rz_oracle as Z
    if not rz_uniform_entrance(m, n0 + 1):
        raise ValueError("cell planes 0 .. n0 are not a uniform pipe")
    phi = rz_potential(g, m, bunch.j0)
    lam = Z.bunch_cells(bunch.Q, bunch.sigma, g.dz, bunch.M)
    f = rz_self_field(g, m, phi, lam, bunch.M, n0)
    out = Z.run(g, m, f, nsteps, n0=n0, bunch=bunch, want_energy=want_energy)
    out["field"] = f
    out["phi"] = phi
    return out
