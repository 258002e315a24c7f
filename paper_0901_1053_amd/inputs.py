"""Seeded synthetic inputs for the explicit TE/TM wake solver.

This module is shared by the tests (which feed the same inputs to the CPU oracle
and to the HIP library) and by the benchmark.  It holds none of the scheme's
arithmetic: only geometry masks, analytic (continuum) cavity fields sampled at
the FIT positions, random fields, and the workload parameters.

Units: c = eps0 = mu0 = 1, lengths in metres, charge in coulombs.  Field arrays
are float64 of shape (nx+1, ny+1, nz+1), z fastest, holding FIT voltages
(E times the edge length for e^, H times the dual-edge length for h^).

Grid positions (node (i,j,k) at (i dx, j dy, k dz)):
  e_x (i+1/2, j, k)   e_y (i, j+1/2, k)   e_z (i, j, k+1/2)
  h_x (i, j+1/2, k+1/2)  h_y (i+1/2, j, k+1/2)  h_z (i+1/2, j+1/2, k)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KEYS = ("ex", "ey", "ez", "hx", "hy", "hz")
MM = 1e-3


def random_fields(shape, seed: int, scale: float = 1.0) -> dict:
    """Independent N(0, scale^2) values in every entry of every component."""
    rng = np.random.default_rng(seed)
    return {k: scale * rng.standard_normal(shape) for k in KEYS}


def random_cells(nx: int, ny: int, nz: int, seed: int, frac: float = 0.08) -> np.ndarray:
    """Random staircase obstacles: each cell PEC with probability frac."""
    rng = np.random.default_rng(seed)
    return (rng.random((nx, ny, nz)) < frac).astype(np.uint8)


# ---------------------------------------------------------------------------
# Rectangular PEC cavity eigenmodes (continuum), sampled at FIT positions.
# Box [0,a]x[0,b]x[0,d]; k = (m pi/a, n pi/b, p pi/d), omega = |k| (c = 1).
# E = A_x cos(kx x) sin(ky y) sin(kz z) x^ + A_y sin cos sin y^ + A_z sin sin cos z^
# with A . k = 0, times cos(omega t); H = -(curl E_s) sin(omega t) / omega.
# ---------------------------------------------------------------------------

@dataclass
class CavityMode:
    m: int
    n: int
    p: int
    kind: str          # "TM" (A_z != 0) or "TE" (A_z = 0)
    amp: float         # seeded amplitude in [-1, 1]


def mode_amplitudes(md: CavityMode, a: float, b: float, d: float):
    kx, ky, kz = md.m * math.pi / a, md.n * math.pi / b, md.p * math.pi / d
    if md.kind == "TM":
        A = np.array([-kx * kz, -ky * kz, kx * kx + ky * ky])
    else:
        A = np.array([ky, -kx, 0.0])
    A = md.amp * A / np.abs(A).max()
    return (kx, ky, kz), A


def cavity_fields(nx, ny, nz, dx, dy, dz, cdt, modes) -> dict:
    """Sum of analytic cavity modes: e^ at tau = 0, h^ at tau = -cdt/2."""
    a, b, d = nx * dx, ny * dy, nz * dz
    i = np.arange(nx + 1)[:, None, None]
    j = np.arange(ny + 1)[None, :, None]
    k = np.arange(nz + 1)[None, None, :]
    f = {key: np.zeros((nx + 1, ny + 1, nz + 1)) for key in KEYS}
    for md in modes:
        (kx, ky, kz), A = mode_amplitudes(md, a, b, d)
        w = math.sqrt(kx * kx + ky * ky + kz * kz)
        th = math.sin(-w * cdt / 2.0) / w           # H time factor -sin(w t)/w at t = -cdt/2
        S, Co = np.sin, np.cos
        xi, xh = i * dx, (i + 0.5) * dx
        yj, yh = j * dy, (j + 0.5) * dy
        zk, zh = k * dz, (k + 0.5) * dz
        f["ex"] += A[0] * Co(kx * xh) * S(ky * yj) * S(kz * zk) * dx
        f["ey"] += A[1] * S(kx * xi) * Co(ky * yh) * S(kz * zk) * dy
        f["ez"] += A[2] * S(kx * xi) * S(ky * yj) * Co(kz * zh) * dz
        cx = A[2] * ky - A[1] * kz
        cy = A[0] * kz - A[2] * kx
        cz = A[1] * kx - A[0] * ky
        f["hx"] += -th * cx * S(kx * xi) * Co(ky * yh) * Co(kz * zh) * dx
        f["hy"] += -th * cy * Co(kx * xh) * S(ky * yj) * Co(kz * zh) * dy
        f["hz"] += -th * cz * Co(kx * xh) * Co(ky * yh) * S(kz * zk) * dz
    # entries outside each component's index range hold no grid object
    f["ex"][nx, :, :] = 0.0
    f["ey"][:, ny, :] = 0.0
    f["ez"][:, :, nz] = 0.0
    f["hx"][:, ny, :] = 0.0
    f["hx"][:, :, nz] = 0.0
    f["hy"][nx, :, :] = 0.0
    f["hy"][:, :, nz] = 0.0
    f["hz"][nx, :, :] = 0.0
    f["hz"][:, ny, :] = 0.0
    return f


def seeded_modes(seed: int, count: int = 3, maxidx: int = 3):
    """count distinct (m,n,p), 1 <= m,n <= maxidx, 0 <= p <= maxidx, TM or TE."""
    rng = np.random.default_rng(seed)
    out, seen = [], set()
    while len(out) < count:
        m, n, p = (int(v) for v in rng.integers(1, maxidx + 1, size=3))
        p = int(rng.integers(0, maxidx + 1))
        if (m, n, p) in seen:
            continue
        seen.add((m, n, p))
        kind = "TM" if (p == 0 or rng.random() < 0.5) else "TE"
        out.append(CavityMode(m, n, p, kind, float(rng.uniform(-1.0, 1.0))))
    return out


# ---------------------------------------------------------------------------
# Staircase geometries (cell masks, 1 = PEC).  A cell is PEC if its centre
# lies in the conductor.  Mask shape (nx, ny, nz).
# ---------------------------------------------------------------------------

def _centres(nx, ny, nz, dx, dy, dz):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    z = (np.arange(nz) + 0.5) * dz
    return x, y, z


def step_collimator_cells(nx, ny, nz, dx, dy, dz, half_gap, z0, z1) -> np.ndarray:
    """Flat jaws |y - y_c| >= half_gap across the full x width for z0 <= z <= z1."""
    x, y, z = _centres(nx, ny, nz, dx, dy, dz)
    yc = ny * dy / 2.0
    jaw_y = np.abs(y - yc) >= half_gap
    in_z = (z >= z0) & (z <= z1)
    return (jaw_y[None, :, None] & in_z[None, None, :]).repeat(nx, axis=0).astype(np.uint8)


def round_taper_cells(nx, ny, nz, dx, dy, dz, r_min, r_max, taper_deg, zc) -> np.ndarray:
    """Round aperture in a square pipe: PEC where r > a(z),
    a(z) = min(r_max, r_min + |z - zc| tan(taper))."""
    x, y, z = _centres(nx, ny, nz, dx, dy, dz)
    r2 = (x[:, None] - nx * dx / 2.0) ** 2 + (y[None, :] - ny * dy / 2.0) ** 2
    a = np.minimum(r_max, r_min + np.abs(z - zc) * math.tan(math.radians(taper_deg)))
    return (r2[:, :, None] > (a * a)[None, None, :]).astype(np.uint8)


def tapered_jaws_cells(nx, ny, nz, dx, dy, dz, gap, theta_deg, zc, flat, g_max) -> np.ndarray:
    """Flat jaws |y - y_c| >= g(z), g(z) = min(g_max, gap + max(0, |z-zc| - flat) tan(theta))."""
    x, y, z = _centres(nx, ny, nz, dx, dy, dz)
    g = np.minimum(g_max, gap + np.maximum(0.0, np.abs(z - zc) - flat) * math.tan(math.radians(theta_deg)))
    yc = ny * dy / 2.0
    mask = np.abs(y - yc)[:, None] >= g[None, :]
    return np.broadcast_to(mask[None, :, :], (nx, ny, nz)).astype(np.uint8)


# ---------------------------------------------------------------------------
# Workloads.  The cell counts, bunch and step counts are those of the five
# workloads; the transverse step is 2 dz so that c dt = dz satisfies the
# stability bound (25) (cubic cells at c dt = dz violate it).
# ---------------------------------------------------------------------------

def trunc_cells(sigma: float, dz: float, nsig: float = 6.0) -> int:
    """Bunch truncation half-width M = ceil(nsig sigma / dz) cells."""
    return int(math.ceil(nsig * sigma / dz - 1e-9))


@dataclass
class WakeCase:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    cdt: float
    steps: int
    Q: float = 1e-9
    sigma: float = 1e-3
    jmin: int = 0
    nw: int = 0
    geometry: dict = field(default_factory=dict)
    seed: int = 20260901

    @property
    def M(self) -> int:
        return trunc_cells(self.sigma, self.dz)

    @property
    def i0(self) -> int:
        return self.nx // 2

    @property
    def j0(self) -> int:
        return self.ny // 2

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def cell_mask(self) -> np.ndarray | None:
        g = dict(self.geometry)
        kind = g.pop("kind", None)
        if kind is None:
            return None
        fn = {"step": step_collimator_cells, "round_taper": round_taper_cells,
              "jaws": tapered_jaws_cells}[kind]
        return fn(self.nx, self.ny, self.nz, self.dx, self.dy, self.dz, **g)


def wake_window(sigma: float, dz: float, s_lo: float = -5.0, s_hi: float = 50.0):
    """(jmin, nw) of wake samples s_j = j dz for s in [s_lo sigma, s_hi sigma]."""
    jmin = int(math.floor(s_lo * sigma / dz + 1e-9))
    jmax = int(math.floor(s_hi * sigma / dz + 1e-9))
    return jmin, jmax - jmin + 1


def cavity_case():
    """Vacuum PEC cavity 24 x 24 x 48 cells, dz = 1 mm, 500 steps, 3 seeded modes."""
    dz = 1.0 * MM
    return WakeCase("cavity_24x24x48", 24, 24, 48, 2 * dz, 2 * dz, dz, dz, 500, Q=0.0, sigma=0.0)


def single_wake_case():
    """Square 20 x 20 mm pipe with a step collimator (half gap 5 mm, 20 mm long),
    128 x 128 x 1024 cells, 1 nC, sigma 1 mm, 3072 steps, s in [-5, 50] sigma."""
    dx = 20.0 * MM / 128
    dz = dx / 2
    sigma = 1.0 * MM
    jmin, nw = wake_window(sigma, dz)
    return WakeCase("step_collimator_128x128x1024", 128, 128, 1024, dx, dx, dz, dz, 3072,
                    Q=1e-9, sigma=sigma, jmin=jmin, nw=nw,
                    geometry=dict(kind="step", half_gap=5.0 * MM, z0=30.0 * MM, z1=50.0 * MM))


def large_case():
    """Tapered round-in-square collimator (10 deg, aperture 2 -> 10 mm diameter),
    512 x 512 x 2048 cells (0.54 G cells), sigma 0.3 mm, 4096 steps."""
    dx = 20.0 * MM / 512
    dz = dx / 2
    sigma = 0.3 * MM
    jmin, nw = wake_window(sigma, dz)
    nz = 2048
    return WakeCase("round_taper_512x512x2048", 512, 512, nz, dx, dx, dz, dz, 4096,
                    Q=1e-9, sigma=sigma, jmin=jmin, nw=nw,
                    geometry=dict(kind="round_taper", r_min=1.0 * MM, r_max=5.0 * MM,
                                  taper_deg=10.0, zc=nz * dz / 2))


def scaled_wake_case(nt: int, nz: int, seed: int, sigma_dz: float | None = None):
    """A tapered-jaw collimator instance with nt x nt x nz cells, dx = 20 mm / nt,
    dz = dx / 2, geometry and sigma drawn from the seeded ranges of the batched
    workload (gap 1-10 mm, taper 5-45 deg, sigma 0.5-2 mm)."""
    rng = np.random.default_rng(seed)
    dx = 20.0 * MM / nt
    dz = dx / 2
    gap = float(rng.uniform(1.0, 10.0)) * MM
    theta = float(rng.uniform(5.0, 45.0))
    sigma = float(rng.uniform(0.5, 2.0)) * MM if sigma_dz is None else sigma_dz * dz
    jmin, nw = wake_window(sigma, dz)
    lz = nz * dz
    M = trunc_cells(sigma, dz)
    steps = M + nz + (jmin + nw - 1)
    return WakeCase("jaws_%dx%dx%d" % (nt, nt, nz), nt, nt, nz, dx, dx, dz, dz, steps,
                    Q=1e-9, sigma=sigma, jmin=jmin, nw=nw, seed=seed,
                    geometry=dict(kind="jaws", gap=gap, theta_deg=theta, zc=lz / 2,
                                  flat=lz / 8, g_max=10.0 * MM))


def batched_cases(count: int = 64, seed: int = 20260901, nts=(64, 96, 128, 160, 192),
                  nzs=(256, 512, 768, 1024)):
    """Uneven instances of the batched workload (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        nt = int(rng.choice(nts))
        nz = int(rng.choice(nzs))
        out.append(scaled_wake_case(nt, nz, seed + 1 + r))
    return out


def random_fields_torch(shape, seed: int, device, dtype):
    """Seeded N(0,1) fields generated on the device (for full-size runs)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return {k: torch.randn(shape, generator=gen, device=device, dtype=dtype) for k in KEYS}


def sample_points(shape, seed: int, count: int = 16):
    """Seeded node indices for sampled parity checks: random interior points
    plus points on the walls and corners of the box."""
    nx, ny, nz = shape[0] - 1, shape[1] - 1, shape[2] - 1
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (nx, ny, nz), (nx // 2, ny // 2, 0), (nx // 2, ny // 2, nz - 1), (1, ny - 1, nz // 2),
           (nx - 1, 1, 1)]
    while len(pts) < count:
        pts.append((int(rng.integers(0, nx + 1)), int(rng.integers(0, ny + 1)), int(rng.integers(0, nz + 1))))
    return pts


def serve_cases(count: int = 200, seed: int = 20260905, nts=(64, 128, 192, 256), nzs=(256, 512, 1024, 2048)):
    """Requests of the serving workload: geometry and sigma as in the batched
    workload, grids from 64^2 x 256 to 256^2 x 2048 (seeded)."""
    return batched_cases(count, seed, nts=nts, nzs=nzs)


# ---------------------------------------------------------------------------
# Rotationally symmetric (r-z) inputs.  Arrays of shape (nr+1, nz+1), z
# fastest, components e_phi, e_r, e_z, h_phi, h_r, h_z (FIT voltages per
# radian); cell masks (nr, nz) for cells (j+1/2, k+1/2).
# ---------------------------------------------------------------------------
RZ_KEYS = ("ephi", "er", "ez", "hphi", "hr", "hz")


def rz_random_fields(shape, seed: int, scale: float = 1.0) -> dict:
    """Independent N(0, scale^2) values in every entry of every r-z component."""
    rng = np.random.default_rng(seed)
    return {k: scale * rng.standard_normal(shape) for k in RZ_KEYS}


def rz_random_cells(nr: int, nz: int, seed: int, frac: float = 0.08) -> np.ndarray:
    """Random staircase obstacles in the r-z plane."""
    rng = np.random.default_rng(seed)
    return (rng.random((nr, nz)) < frac).astype(np.uint8)


def disk_loaded_cells(nr, nz, dr, dz, a_iris, period, t_iris, z0, ncell) -> np.ndarray:
    """Disk-loaded waveguide (the outer wall is the grid's r = nr dr): irises of
    aperture radius a_iris and thickness t_iris at the start of each of ncell
    periods from z0, and a beam pipe of radius a_iris before and after the
    structure.  A cell (j+1/2, k+1/2) is PEC if its centre is metal."""
    rc = (np.arange(nr) + 0.5) * dr
    zc = (np.arange(nz) + 0.5) * dz
    zend = z0 + ncell * period + t_iris
    inside = (zc >= z0) & (zc < zend)
    ph = np.mod(zc - z0, period)
    iris = inside & (ph < t_iris)
    metal_z = ~inside | iris                      # pipe or iris: metal outside a_iris
    return (metal_z[None, :] & (rc[:, None] > a_iris)).astype(np.uint8)


@dataclass
class RZCase:
    """One rotationally symmetric wake solve: grid, harmonic, ring bunch and
    wake lines (sizes in metres, charge in coulombs)."""
    name: str
    nr: int
    nz: int
    dr: float
    dz: float
    mode: int
    sigma: float
    r0: float            # ring radius (0 = the axis, m = 0)
    a_iris: float
    period: float
    t_iris: float
    z0: float
    ncell: int
    charge: float = 1e-9
    s_lo: float = -5.0
    s_hi: float = 50.0

    @property
    def cdt(self) -> float:
        return self.dz

    @property
    def M(self) -> int:
        return trunc_cells(self.sigma, self.dz)

    @property
    def j0(self) -> int:
        return int(round(self.r0 / self.dr))

    @property
    def jw(self) -> int:
        return max(self.j0, 1 if self.mode > 0 else 0)

    def window(self):
        return wake_window(self.sigma, self.dz, self.s_lo, self.s_hi)

    def cells(self) -> np.ndarray:
        return disk_loaded_cells(self.nr, self.nz, self.dr, self.dz, self.a_iris, self.period, self.t_iris,
                                 self.z0, self.ncell)

    def steps(self) -> int:
        """Steps until the last wake sample is complete."""
        jmin, nw = self.window()
        return self.nz - 1 + self.M + jmin + nw


def tds_case(mode: int = 1) -> RZCase:
    """Transverse-deflecting-structure-like workload (the paper's first example,
    whose geometry is not given): a 15-period disk-loaded structure of 30 mm
    outer radius, iris aperture 11 mm, period 33.3 mm, irises 6 mm thick, with
    20 mm pipes on both sides; sigma = 300 um at dr = dz = 30 um (sigma / dz = 10,
    the paper's fine mesh); dipole ring at r0 = 1 mm."""
    dz = 30e-6
    L = 0.02 + 15 * 0.0333 + 0.006 + 0.02
    return RZCase("tds_rz", nr=1000, nz=int(round(L / dz)), dr=dz, dz=dz, mode=mode, sigma=300e-6,
                  r0=1e-3 if mode > 0 else 0.0, a_iris=11e-3, period=0.0333, t_iris=6e-3, z0=0.02, ncell=15)


def small_rz_case(mode: int = 1) -> RZCase:
    """A scaled version for parity tests: 3 periods, 24 x 260 cells."""
    dz = 1e-3
    dr = dz if mode > 0 else 1.25 * dz           # m = 0: the axis cell needs dtau < 0.909 dr
    return RZCase("small_rz", nr=24, nz=260, dr=dr, dz=dz, mode=mode, sigma=3e-3,
                  r0=3 * dr if mode > 0 else 0.0, a_iris=9 * dr, period=0.06, t_iris=0.01, z0=0.04, ncell=3)
