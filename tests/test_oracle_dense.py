"""Pins of the oracle against the dense matrix form of scheme (23).

The oracle's ten sub-updates (Sec. 4.2) must equal one solve of
B^e (y^{n+1} - y^n)/dtau + A y^n = f^n built from the paper's operator
definitions; its energy must equal 1/2 <Q^e y, y> (Sec. 4.4).  General
(random, positive) diagonal materials and interior staircase PEC are used so
that a dropped or mis-indexed material factor fails.
"""
import numpy as np
import pytest

from tests.dense_scheme import DenseScheme


def _setup(orc, seed, nx=2, ny=3, nz=4, dx=2.0, dy=1.5, dz=1.0, cdt=0.9, pec_frac=0.15,
           random_materials=True):
    g = orc.Geom(nx, ny, nz, dx, dy, dz, cdt)
    rng = np.random.default_rng(seed)
    cells = (rng.random((nx, ny, nz)) < pec_frac).astype(np.uint8)
    m = orc.vacuum_materials(g, cells)
    if random_materials:
        for k in orc.KEYS:
            m[k] = np.where(m[k] > 0, m[k] * rng.uniform(0.5, 1.5, size=m[k].shape), 0.0)
    f = {k: rng.standard_normal(g.shape) for k in orc.KEYS}
    orc.apply_pec(g, m, f)
    return g, m, f, rng


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ten_updates_equal_dense_scheme(orc, seed):
    g, m, f, rng = _setup(orc, seed)
    D = DenseScheme(g, m)
    y = D.to_y(f)
    for _ in range(3):
        jx = rng.standard_normal(g.shape)
        jy = rng.standard_normal(g.shape)
        jz = rng.standard_normal(g.shape)
        y_ref = D.step(y, D.source(jx, jy, jz))
        orc.step(g, m, f, jx, jy, jz)
        y = D.to_y(f)
        assert np.max(np.abs(y - y_ref)) <= 1e-12 * max(1.0, np.max(np.abs(y_ref)))


def test_operator_structure(orc):
    """A is skew, the v-u block of the scaled system is -L^T, Q^e is symmetric,
    and L_T U_T = I - alpha T - alpha^2 R (the R-sign reading)."""
    g, m, f, _ = _setup(orc, 5)
    D = DenseScheme(g, m)
    a = D.alpha
    assert np.allclose(D.A, -D.A.T, atol=1e-14)
    assert np.allclose(D.minusLT, -D.L.T, atol=1e-14)
    assert np.allclose(D.Qe, D.Qe.T, atol=1e-13)
    for T, LT, UT, R in ((D.T0, D.LT0, D.UT0, D.R0), (D.T1, D.LT1, D.UT1, D.R1)):
        n = T.shape[0]
        assert np.allclose(LT @ UT, np.eye(n) - a * T - a * a * R, atol=1e-13)
    # Q^e = [[I - a^2 R0, a L], [a L^T, I - a^2 R1]]
    nu = D.nu
    Q = np.zeros_like(D.Qe)
    Q[:nu, :nu] = np.eye(nu) - a * a * D.R0
    Q[:nu, nu:] = a * D.L
    Q[nu:, :nu] = a * D.L.T
    Q[nu:, nu:] = np.eye(D.nv) - a * a * D.R1
    assert np.allclose(D.Qe, Q, atol=1e-13)
    # T_i block structure of (15): only the (h, e_z) / (e, h_z) blocks are non-zero
    assert np.all(D.T0[D.u_hx, D.u_hx] == 0) and np.all(D.T0[D.u_hx, D.u_hy] == 0)
    assert np.allclose(D.T0[D.u_ez, D.u_hx], D.X0.T) and np.allclose(D.T0[D.u_ez, D.u_hy], -D.Y0.T)
    assert np.allclose(D.T1[D.v_hz, D.v_ex], D.X1.T) and np.allclose(D.T1[D.v_hz, D.v_ey], -D.Y1.T)


def test_curl_incidence_is_divergence_free(orc):
    """The geometric curl satisfies S C = 0 (div curl = 0) on the primary grid."""
    g, m, f, _ = _setup(orc, 3)
    D = DenseScheme(g, m)
    fid = {t: n for n, t in enumerate(D.facets)}
    nx, ny, nz = g.nx, g.ny, g.nz
    S = np.zeros((nx * ny * nz, len(D.facets)))
    r = 0
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                S[r, fid[("x", (i + 1, j, k))]] += 1
                S[r, fid[("x", (i, j, k))]] -= 1
                S[r, fid[("y", (i, j + 1, k))]] += 1
                S[r, fid[("y", (i, j, k))]] -= 1
                S[r, fid[("z", (i, j, k + 1))]] += 1
                S[r, fid[("z", (i, j, k))]] -= 1
                r += 1
    assert np.all(S @ D.C_full == 0)


@pytest.mark.parametrize("seed", [0, 4])
def test_energy_is_half_yQy(orc, seed):
    g, m, f, _ = _setup(orc, seed)
    D = DenseScheme(g, m)
    for _ in range(2):
        y = D.to_y(f)
        assert abs(orc.energy(g, m, f) - D.energy(y)) <= 1e-12 * abs(D.energy(y))
        orc.step(g, m, f)


def test_energy_law_with_source(orc):
    """(19): W^{n+1} - W^n = (dtau/2) <f^n, y^{n+1} + y^n> for arbitrary currents."""
    g, m, f, rng = _setup(orc, 7)
    D = DenseScheme(g, m)
    for _ in range(3):
        jx, jy, jz = (rng.standard_normal(g.shape) for _ in range(3))
        y0 = D.to_y(f)
        w0 = orc.energy(g, m, f)
        orc.step(g, m, f, jx, jy, jz)
        y1 = D.to_y(f)
        w1 = orc.energy(g, m, f)
        rhs = 0.5 * g.cdt * D.source(jx, jy, jz) @ (y0 + y1)
        assert abs((w1 - w0) - rhs) <= 1e-12 * max(abs(w0), abs(w1))


def test_stability_condition_25_positive_definite(orc):
    """Q^e > 0 in vacuum with staircase PEC when (25) holds; indefinite well beyond it."""
    dx, dy, dz = 2.0, 1.5, 1.0
    bound = min(dz, (dx ** -2 + dy ** -2) ** -0.5)
    for cdt, positive in ((bound, True), (0.8 * bound, True), (1.6 * bound, False)):
        g, m, f, _ = _setup(orc, 9, nx=4, ny=4, nz=3, dx=dx, dy=dy, dz=dz, cdt=cdt,
                            random_materials=False, pec_frac=0.1)
        D = DenseScheme(g, m)
        lmin = np.linalg.eigvalsh(0.5 * (D.Qe + D.Qe.T)).min()
        assert (lmin > 0) == positive, (cdt, lmin)
