"""Sufficient stability test for general diagonal materials (test side).

Sec. 4.4: the explicit scheme is stable when Q^e is positive definite.  In
the scaled variables a = h / sqrt(mu), b = e / sqrt(kappa) the energy form
2 W^{n,e} = |u|^2 + |v|^2 - alpha^2 (<R_0 u,u> + <R_1 v,v>) + 2 alpha <L v,u>
(the oracle's energy, expanded in FIT variables) splits into three blocks that
share no variable: e_z alone, h_z alone, and (h_x, h_y, e_x, e_y) coupled by
the z-differences of L.  Each block is positive semi-definite when every
Gershgorin row sum of its subtracted and off-diagonal parts is at most 1.
This module forms those row sums with numpy from the material arrays, for
the tests to hold the library's verdict and the dense Q^e against.
"""
from __future__ import annotations

import numpy as np

KEYS = ("ex", "ey", "ez", "hx", "hy", "hz")


def _masked(m: dict, shape):
    """Copies of the material arrays, zero outside each component's range."""
    X, Y, Z = shape
    nx, ny, nz = X - 1, Y - 1, Z - 1
    out = {k: np.array(m[k], dtype=float) for k in KEYS}
    out["ex"][nx, :, :] = 0
    out["ey"][:, ny, :] = 0
    out["ez"][:, :, nz] = 0
    out["hx"][:, ny, :] = 0
    out["hx"][:, :, nz] = 0
    out["hy"][nx, :, :] = 0
    out["hy"][:, :, nz] = 0
    out["hz"][nx, :, :] = 0
    out["hz"][:, ny, :] = 0
    return out


def _sh(a, di, dj, dk):
    """b[i, j, k] = a[i + di, j + dj, k + dk], zero outside the array."""
    b = np.zeros_like(a)
    X, Y, Z = a.shape
    src = [slice(max(0, d), n + min(0, d)) for d, n in zip((di, dj, dk), (X, Y, Z))]
    dst = [slice(max(0, -d), n - max(0, d)) for d, n in zip((di, dj, dk), (X, Y, Z))]
    b[tuple(dst)] = a[tuple(src)]
    return b


def row_sums(m: dict, cdt: float) -> dict:
    """Gershgorin row sums per component (arrays of the grid's shape)."""
    a = 0.5 * cdt
    shape = m["ex"].shape
    q = _masked(m, shape)
    kx, ky, kz, mx, my, mz = (q[k] for k in KEYS)
    r = {}
    ez = (mx * (kz + np.sqrt(kz * _sh(kz, 0, 1, 0))) + _sh(mx, 0, -1, 0) * (kz + np.sqrt(kz * _sh(kz, 0, -1, 0)))
          + my * (kz + np.sqrt(kz * _sh(kz, 1, 0, 0))) + _sh(my, -1, 0, 0) * (kz + np.sqrt(kz * _sh(kz, -1, 0, 0))))
    r["ez"] = np.where(kz > 0, a * a * ez, 0.0)
    hz = (kx * (mz + np.sqrt(mz * _sh(mz, 0, -1, 0))) + _sh(kx, 0, 1, 0) * (mz + np.sqrt(mz * _sh(mz, 0, 1, 0)))
          + ky * (mz + np.sqrt(mz * _sh(mz, -1, 0, 0))) + _sh(ky, 1, 0, 0) * (mz + np.sqrt(mz * _sh(mz, 1, 0, 0))))
    r["hz"] = np.where(mz > 0, a * a * hz, 0.0)
    r["hx"] = a * np.sqrt(mx) * (np.sqrt(ky) + np.sqrt(_sh(ky, 0, 0, 1)))
    r["hy"] = a * np.sqrt(my) * (np.sqrt(kx) + np.sqrt(_sh(kx, 0, 0, 1)))
    r["ey"] = a * np.sqrt(ky) * (np.sqrt(mx) + np.sqrt(_sh(mx, 0, 0, -1)))
    r["ex"] = a * np.sqrt(kx) * (np.sqrt(my) + np.sqrt(_sh(my, 0, 0, -1)))
    return r


def bound(m: dict, cdt: float) -> float:
    """Largest row sum: Q^e >= 0 if it is at most 1."""
    return max(float(np.max(v)) for v in row_sums(m, cdt).values())
