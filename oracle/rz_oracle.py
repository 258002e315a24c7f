"""FP64 CPU oracle of the explicit TE/TM scheme for rotationally symmetric
structures, scheme (24) of Sec. 4.3, at azimuthal mode m.

TEST INFRASTRUCTURE ONLY: imported by the tests and never by the product
package; it shares no code with the HIP path.

Grid (a reading: the paper refers the r-z FIT grid to another work and does
not print it).  Nodes (r_j, z_k) = (j dr, k dz), j = 0..nr, k = 0..nz; the
azimuthal direction is carried by the harmonic m, so every FIT quantity is
taken per radian.  Components and positions (the layout of the 3-D grid with
x -> phi, y -> r, z -> z, as (24) follows (23) with those roles):

    e_phi (r_j,     z_k)        e_r (r_{j+1/2}, z_k)        e_z (r_j,     z_{k+1/2})
    h_phi (r_{j+1/2}, z_{k+1/2}) h_r (r_j,       z_{k+1/2})  h_z (r_{j+1/2}, z_k)

Edge voltages e^ = E * (edge length per radian), dual voltages h^ = H * (dual
edge length per radian); M_eps^-1 = kappa = edge length / dual-facet area,
M_mu^-1 = mu = dual-edge length / facet area, per radian (c = eps0 = mu0 = 1):

    kappa_phi = r_j / (dr dz)            (0 on the axis: the edge has no length)
    kappa_r   = dr / (r_{j+1/2} dz)
    kappa_z   = dz / (r_j dr),  on the axis dz / (dr^2 / 8) for m = 0 (the dual
                facet is the disk sector of radius dr/2) and 0 for m >= 1
    mu_phi    = r_{j+1/2} / (dr dz)
    mu_r      = dr / (r_j dz)            (the axis has no h_r: facet of no area)
    mu_z      = dz / (r_{j+1/2} dr)

Walls: PEC at r = nr dr and at z = 0, nz dz (kappa = 0 on tangential edges);
staircase obstacles from a cell mask (nr, nz) as in 3-D (an edge is PEC if any
adjacent cell is; cells beyond r = 0 are the axis, not a wall).

Step (24) as printed, with two readings: the current enters with its physical
sign (-j, as in 3-D), and the implicit factors of the e_z and h_z updates are
(1 + a^2 m^2 kappa_z mu_r)^-1 and (1 + a^2 m^2 mu_z kappa_r)^-1, the products of
the coefficients that share the position of e_z (with h_r) and of h_z (with
e_r); the text prints the two pairs of subscripts the other way round.
Differences: (P_r f)(j) = f(j+1) - f(j), (P_r^* g)(j) = g(j-1) - g(j), the same
in z; values outside a component's index range are zero.

Stability (Sec. 4.4): the paper bounds dtau by min(dz, dr) for every m.  On this
grid that holds for m >= 1 (the axis carries no e_z there); for m = 0 the
on-axis e_z cell, whose dual facet is the disk of radius dr/2, raises the
largest eigenvalue of the radial operator to 4.8419 / dr^2, so the radial limit
is 0.9089 dr.

Wake: a ring bunch of mode m (Sec. 5 for the charge model, the harmonic weight of
a point charge for the ring) and two e_z lines at radius indices jw and jw + 1;
the longitudinal wake is the 3-D quadrature on each line and the transverse one
follows from their difference by the Panofsky-Wenzel relation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

KEYS = ("ephi", "er", "ez", "hphi", "hr", "hz")


@dataclass
class RZGeom:
    nr: int
    nz: int
    dr: float
    dz: float
    cdt: float
    m: int = 0

    @property
    def shape(self):
        return (self.nr + 1, self.nz + 1)


def ranges(g: RZGeom) -> dict:
    """Index-range masks of the six components."""
    nr, nz = g.nr, g.nz
    R = {k: np.zeros(g.shape, bool) for k in KEYS}
    R["ephi"][:, :] = True
    R["er"][:nr, :] = True
    R["ez"][:, :nz] = True
    R["hphi"][:nr, :nz] = True
    R["hr"][1:, :nz] = True
    R["hz"][:nr, :] = True
    return R


def materials(g: RZGeom, cell_pec=None) -> dict:
    """kappa and mu per radian (vacuum), PEC edges with kappa = 0."""
    nr, nz, dr, dz = g.nr, g.nz, g.dr, g.dz
    j = np.arange(nr + 1, dtype=float)[:, None] * np.ones((1, nz + 1))
    r = j * dr
    rh = (j + 0.5) * dr
    R = ranges(g)
    m = {k: np.zeros(g.shape) for k in KEYS}
    m["ephi"] = np.where(j > 0, r / (dr * dz), 0.0)
    m["er"] = dr / (rh * dz)
    with np.errstate(divide="ignore"):
        m["ez"] = np.where(j > 0, dz / (r * dr), (dz / (dr * dr / 8.0)) if g.m == 0 else 0.0)
        m["hr"] = np.where(j > 0, dr / np.where(j > 0, r, 1.0) / dz, 0.0)
    m["hphi"] = rh / (dr * dz)
    m["hz"] = dz / (rh * dr)
    # cells (j+1/2, k+1/2): PEC beyond the outer radius and the z ends, or by mask
    cell = np.zeros((nr + 2, nz + 2), bool)     # padded: index (j+1, k+1); j = -1 is the axis side
    cell[nr + 1, :] = True
    cell[:, 0] = True
    cell[:, nz + 1] = True
    if cell_pec is not None:
        cell[1:nr + 1, 1:nz + 1] = np.asarray(cell_pec, bool)
    cell[0, :] = cell[1, :]                     # mirror across the axis (not a wall)

    def c(jj, kk):                              # cell (jj, kk) with jj, kk >= -1
        return cell[jj + 1, kk + 1]
    jj, kk = np.meshgrid(np.arange(nr + 1), np.arange(nz + 1), indexing="ij")
    # e_phi at a node touches the four cells around it; e_r (r-edge) the two
    # cells above and below in z; e_z (z-edge) the two cells inside and outside in r
    pec_phi = c(jj - 1, kk - 1) | c(jj, kk - 1) | c(jj - 1, kk) | c(jj, kk)
    pec_r = c(jj, kk - 1) | c(jj, kk)
    pec_z = c(jj - 1, kk) | c(jj, kk)
    m["ephi"] = np.where(pec_phi, 0.0, m["ephi"])
    m["er"] = np.where(pec_r, 0.0, m["er"])
    m["ez"] = np.where(pec_z, 0.0, m["ez"])
    for k in KEYS:
        m[k] = np.where(R[k], m[k], 0.0)
    return m


def zeros(g: RZGeom) -> dict:
    return {k: np.zeros(g.shape) for k in KEYS}


def apply_pec(g: RZGeom, m: dict, f: dict) -> None:
    """Zero e on PEC edges and every entry outside its index range."""
    R = ranges(g)
    for k in KEYS:
        f[k][~R[k]] = 0.0
    for k in ("ephi", "er", "ez"):
        f[k][m[k] == 0.0] = 0.0


def _sh(a, dj, dk):
    """a(j + dj, k + dk), zero outside the array."""
    out = np.zeros_like(a)
    nr1, nz1 = a.shape
    js, je = max(0, -dj), min(nr1, nr1 - dj)
    ks, ke = max(0, -dk), min(nz1, nz1 - dk)
    out[js:je, ks:ke] = a[js + dj:je + dj, ks + dk:ke + dk]
    return out


def pr(f):   return _sh(f, 1, 0) - f        # P_r f
def prs(g_): return _sh(g_, -1, 0) - g_     # P_r^* g
def pz(f):   return _sh(f, 0, 1) - f        # P_z f
def pzs(g_): return _sh(g_, 0, -1) - g_     # P_z^* g


def step(g: RZGeom, m: dict, f: dict, jz=None) -> None:
    """One step of (24) in place: y^n = (u^{n-1/2}, v^n) -> y^{n+1}, with
    u = (h_phi, h_r, e_z), v = (e_phi, e_r, h_z) and alpha = dtau / 2.  jz
    (or None) is the current through the dual facet of each e_z edge."""
    a = 0.5 * g.cdt
    M = g.m
    R = ranges(g)
    Jz = np.zeros(g.shape) if jz is None else jz

    def upd_hphi():
        f["hphi"] += np.where(R["hphi"], a * m["hphi"] * (pz(f["er"]) - pr(f["ez"])), 0.0)

    def upd_hr():
        f["hr"] += np.where(R["hr"], a * m["hr"] * (-pz(f["ephi"]) + M * f["ez"]), 0.0)

    def upd_ephi():
        f["ephi"] += np.where(R["ephi"], a * m["ephi"] * (pzs(f["hr"]) - prs(f["hz"])), 0.0)

    def upd_er():
        f["er"] += np.where(R["er"], a * m["er"] * (-pzs(f["hphi"]) + M * f["hz"]), 0.0)

    upd_hphi()                                                            # S1
    upd_hr()                                                              # S2
    fac = 1.0 / (1.0 + a * a * M * M * m["ez"] * m["hr"])                 # S3
    f["ez"] += np.where(R["ez"], fac * 2 * a * m["ez"] * (prs(f["hphi"]) - M * f["hr"] - Jz), 0.0)
    upd_hphi()                                                            # S4
    upd_hr()                                                              # S5
    upd_ephi()                                                            # S6
    upd_er()                                                              # S7
    fac = 1.0 / (1.0 + a * a * M * M * m["hz"] * m["er"])                 # S8
    f["hz"] += np.where(R["hz"], fac * 2 * a * m["hz"] * (pr(f["ephi"]) - M * f["er"]), 0.0)
    upd_ephi()                                                            # S9
    upd_er()                                                              # S10


def step_yee(g: RZGeom, m: dict, f: dict, jz=None) -> None:
    """Yee's scheme (7) on the same r-z grid at mode m, the comparison of
    Sec. 4.4: every e component from h^n with factor dtau, then every h
    component from e^{n+1/2}.  State (e^{n-1/2}, h^n)."""
    dt = g.cdt
    M = g.m
    R = ranges(g)
    Jz = np.zeros(g.shape) if jz is None else jz
    f["ephi"] += np.where(R["ephi"], dt * m["ephi"] * (pzs(f["hr"]) - prs(f["hz"])), 0.0)
    f["er"] += np.where(R["er"], dt * m["er"] * (-pzs(f["hphi"]) + M * f["hz"]), 0.0)
    f["ez"] += np.where(R["ez"], dt * m["ez"] * (prs(f["hphi"]) - M * f["hr"] - Jz), 0.0)
    f["hphi"] += np.where(R["hphi"], dt * m["hphi"] * (pz(f["er"]) - pr(f["ez"])), 0.0)
    f["hr"] += np.where(R["hr"], dt * m["hr"] * (-pz(f["ephi"]) + M * f["ez"]), 0.0)
    f["hz"] += np.where(R["hz"], dt * m["hz"] * (pr(f["ephi"]) - M * f["er"]), 0.0)


def _inv(x):
    return np.where(x > 0, 1.0 / np.where(x > 0, x, 1.0), 0.0)


def energy(g: RZGeom, m: dict, f: dict) -> float:
    """Discrete energy 1/2 <Q y, y> of (24) with y^n = (u^{n-1/2}, v^n) (Sec. 4.4).
    Q = B^{e,r} - alpha A: the 3-D form of Q^e with only the radial part of the
    splitting operator R, since the azimuthal coupling (the m^2 terms) stays in
    the implicit factors.  Sums over non-PEC edges."""
    a = 0.5 * g.cdt
    R = ranges(g)
    s = 0.0
    for k in KEYS:
        s += 0.5 * np.sum(np.where(R[k], f[k] ** 2 * _inv(m[k]), 0.0))
    r0 = np.sum(np.where(R["hphi"], m["hphi"] * pr(f["ez"]) ** 2, 0.0))
    r1 = np.sum(np.where(m["ephi"] > 0, m["ephi"] * prs(f["hz"]) ** 2, 0.0))
    lc = (np.sum(np.where(R["hphi"], f["hphi"] * pz(f["er"]), 0.0))
          - np.sum(np.where(R["hr"], f["hr"] * pz(f["ephi"]), 0.0)))
    return float(s - 0.5 * a * a * (r0 + r1) + a * lc)


def charge(g: RZGeom, m: dict, fo: dict, fn: dict) -> np.ndarray:
    """Node charges q^{n+1/2} of the scheme (Sec. 4.3; the 3-D conserved charge
    with the azimuthal divergence m d_phi):
        q = -[m dbar_phi + P_r^T dbar_r + P_z^T dtil_z],
    dbar = (e^n + e^{n+1}) / (2 kappa) for phi and r, and
    dtil_z = e_z^{n+1/2} / kappa_z - alpha^2 P_r^T mu_phi P_r e_z^{n+1/2}.
    fo = y^n, fn = y^{n+1} (the step that took fo to fn).  Between steps it
    changes by dtau (j(k-1) - j(k)) at every node whose edges are all free."""
    a = 0.5 * g.cdt
    R = ranges(g)
    dphi = 0.5 * (fo["ephi"] + fn["ephi"]) * _inv(m["ephi"])
    dr_ = 0.5 * (fo["er"] + fn["er"]) * _inv(m["er"])
    ez = fn["ez"]
    rz = prs(np.where(R["hphi"], m["hphi"] * pr(ez), 0.0))
    dz_ = np.where(m["ez"] > 0, ez * _inv(m["ez"]) - a * a * rz, 0.0)
    return -(g.m * dphi + prs(dr_) + pzs(dz_))


def bunch_cells(Q: float, sigma: float, dz: float, M: int) -> np.ndarray:
    """Charge of a Gaussian bunch (RMS sigma, charge Q) in cells of length dz
    centred m dz ahead of its centre, |m| <= M, via erfc (tails accurate)."""
    from math import erfc, sqrt
    out = np.zeros(2 * M + 1)
    for mm in range(-M, M + 1):
        lo, hi = (mm - 0.5) * dz / sigma, (mm + 0.5) * dz / sigma
        if lo >= 0:
            v = 0.5 * (erfc(lo / sqrt(2)) - erfc(hi / sqrt(2)))
        elif hi <= 0:
            v = 0.5 * (erfc(-hi / sqrt(2)) - erfc(-lo / sqrt(2)))
        else:
            v = 1.0 - 0.5 * erfc(-lo / sqrt(2)) - 0.5 * erfc(hi / sqrt(2))
        out[mm + M] = Q * v
    return out


def mode_weight(mode: int) -> float:
    """Per-radian weight of a point charge's azimuthal harmonic: the delta in
    phi is (1 + 2 sum_m cos m phi) / (2 pi), so 1/(2 pi) for m = 0 and 1/pi above."""
    return 1.0 / (2.0 * np.pi) if mode == 0 else 1.0 / np.pi


@dataclass
class RZBunch:
    """Ring bunch at radius index j0 (the axis for m = 0), moving along +z at
    v = c with dtau = dz; the wake is sampled on the two e_z lines at radius
    indices jw and jw + 1 for s_j = j dz, j = jmin .. jmin + nw - 1."""
    Q: float
    sigma: float
    j0: int
    M: int
    jw: int
    jmin: int
    nw: int
    kend: int = 0          # wake quadrature over edges k < kend (0: all edges)


def run(g: RZGeom, m: dict, f: dict, nsteps: int, n0: int = 0, bunch: RZBunch | None = None,
        acc=None, want_energy: bool = False):
    """nsteps steps of (24) in place.  With a bunch: the charge of cell
    k - n + M crosses the dual facet of e_z edge (j0, k) in step n (current
    = charge / dtau, times the mode weight), and each wake line L in (jw, jw+1)
    accumulates acc[L - jw, j - jmin] += -1/2 (e_z^{n-1/2} + e_z^{n+1/2})(L, k)
    with n = k + M + j, the quadrature of the 3-D wake, over edges k < kend
    (all edges for kend 0).  W_par^m(s_j) = acc / Q."""
    out = {"energy": [], "acc": acc}
    if bunch is not None:
        lam = bunch_cells(bunch.Q, bunch.sigma, g.dz, bunch.M)
        if out["acc"] is None:
            out["acc"] = np.zeros((2, bunch.nw))
        out["lam"] = lam
        lines = (bunch.jw, bunch.jw + 1)
    wm = mode_weight(g.m)
    for s in range(nsteps):
        n = n0 + s
        if want_energy:
            out["energy"].append(energy(g, m, f))
        jz = None
        if bunch is not None:
            jz = np.zeros(g.shape)
            for k in range(g.nz):
                mm = k - n + bunch.M
                if -bunch.M <= mm <= bunch.M:
                    jz[bunch.j0, k] = wm * lam[mm + bunch.M] / g.cdt
            ezo = f["ez"][list(lines), :].copy()
        step(g, m, f, jz)
        if bunch is not None:
            kend = bunch.kend if 0 < bunch.kend < g.nz else g.nz
            for k in range(kend):
                jj = n - k - bunch.M
                if bunch.jmin <= jj < bunch.jmin + bunch.nw:
                    for li, L in enumerate(lines):
                        out["acc"][li, jj - bunch.jmin] += -0.5 * (ezo[li, k] + f["ez"][L, k])
    return out


def transverse_wake(acc: np.ndarray, Q: float, dr: float, ds: float) -> np.ndarray:
    """Radial wake W_r(r_{jw+1/2}, theta = 0, s) from the two wake lines by the
    Panofsky-Wenzel relation d/ds W_perp = grad_perp W_par (v = c, W_par = -1/Q
    int E_z dz, W_perp = 1/Q int (E + c z x B)_perp dz), with the radial
    derivative a difference of the lines and the s-integral the trapezoidal
    rule from the first sample (ahead of the bunch head, where the wake is zero):
        W_r(s_j) = sum_{i<j} ds (D_i + D_{i+1}) / 2,  D = (acc[1] - acc[0]) / (Q dr)."""
    D = (acc[1] - acc[0]) / (Q * dr)
    out = np.zeros_like(D)
    out[1:] = np.cumsum(0.5 * (D[1:] + D[:-1])) * ds
    return out
