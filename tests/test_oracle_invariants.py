"""Invariant pins of the oracle: energy (Sec. 4.4), charge (Sec. 4.5, (34)/(35)),
bunch injection (Fig. 1) and the wake potential quadrature (Sec. 5)."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from paper_0901_1053_amd import inputs


def _box(orc, nx, ny, nz, dz=1.0, ratio=2.0, cells=None, cdt=None):
    g = orc.Geom(nx, ny, nz, ratio * dz, ratio * dz, dz, dz if cdt is None else cdt)
    return g, orc.vacuum_materials(g, cells)


@pytest.mark.parametrize("with_obstacles", [False, True])
def test_energy_conserved_without_current(orc, with_obstacles):
    g, m = _box(orc, 8, 8, 12, cells=inputs.random_cells(8, 8, 12, 3) if with_obstacles else None)
    f = inputs.random_fields(g.shape, 11)
    orc.apply_pec(g, m, f)
    r = orc.run(g, m, f, 500, want_energy=True)
    e = r["energy"]
    assert np.max(np.abs(e - e[0])) <= 1e-13 * abs(e[0])


def test_literal_cubic_cells_blow_up(orc):
    """Cubic cells with c dt = dz violate (25); random data grows without bound."""
    g = orc.Geom(24, 24, 48, 1.0, 1.0, 1.0, 1.0)
    m = orc.vacuum_materials(g)
    f = inputs.random_fields(g.shape, 1)
    orc.apply_pec(g, m, f)
    a0 = max(np.abs(v).max() for v in f.values())
    orc.run(g, m, f, 60)
    a1 = max(np.abs(v).max() for v in f.values())
    assert a1 > 1e10 * a0


def _bunch_run(orc, nx=10, ny=10, nz=40, sigma_dz=2.5, jaws=True, extra=0, win=None):
    dz = 1.0
    cells = None
    if jaws:
        cells = inputs.step_collimator_cells(nx, ny, nz, 2 * dz, 2 * dz, dz, half_gap=3.0 * 2 * dz,
                                             z0=15 * dz, z1=25 * dz)
    g, m = _box(orc, nx, ny, nz, dz=dz, cells=cells)
    sigma = sigma_dz * dz
    M = inputs.trunc_cells(sigma, dz)
    jmin, nw = (-M - 6, 2 * M + 20) if win is None else win
    b = orc.Bunch(Q=1.0, sigma=sigma, i0=nx // 2, j0=ny // 2, M=M, jmin=jmin, nw=nw)
    f = orc.zeros(g)
    return g, m, f, b


def test_bunch_cells_match_normal_distribution(orc):
    """lam_m = Q [Phi((m+1/2)dz/s) - Phi((m-1/2)dz/s)], checked against scipy."""
    for sigma, dz in ((1.0, 0.078125), (0.3, 0.01953125), (2.0, 0.5)):
        M = inputs.trunc_cells(sigma, dz)
        lam = orc.bunch_cells(2.5, sigma, dz, M)
        mm = np.arange(-M, M + 1)
        ref = 2.5 * (norm.cdf((mm + 0.5) * dz / sigma) - norm.cdf((mm - 0.5) * dz / sigma))
        assert np.max(np.abs(lam - ref)) <= 1e-15 * 2.5 * 4
        assert np.allclose(lam, lam[::-1], rtol=0, atol=1e-16 * 2.5 * 4)
        assert abs(lam.sum() - 2.5 * (1 - 2 * norm.cdf(-(M + 0.5) * dz / sigma))) < 1e-14


def test_gauss_law_moving_bunch(orc):
    """(35): q_e^{n+1/2} equals the bunch charge of each interior node's dual cell
    (all six edges non-PEC) at tau_{n+1/2}; (34): q_h^n = 0 in every cell.
    The expected node charge is computed from the bunch position alone
    (centre at (n - M + 1) dz at tau_{n+1/2}) with scipy's normal CDF."""
    g, m, f, b = _bunch_run(orc)
    sigma = b.sigma
    lam = orc.bunch_cells(b.Q, sigma, g.dz, b.M)
    interior = np.ones(g.shape, bool)
    kx, ky, kz = m["ex"], m["ey"], m["ez"]
    for i in range(g.nx + 1):
        for j in range(g.ny + 1):
            for k in range(g.nz + 1):
                ok = (0 < i < g.nx and 0 < j < g.ny and 0 < k < g.nz and kx[i, j, k] > 0 and kx[i - 1, j, k] > 0
                      and ky[i, j, k] > 0 and ky[i, j - 1, k] > 0 and kz[i, j, k] > 0 and kz[i, j, k - 1] > 0)
                interior[i, j, k] = ok
    worst_e = worst_h = 0.0
    acc = None
    for n in range(70):
        fo = {k: v.copy() for k, v in f.items()}
        r = orc.run(g, m, f, 1, n0=n, bunch=b, acc=acc)
        acc = r["acc"]
        qe, qh = orc.charges(g, m, fo, f)
        expect = np.zeros(g.shape)
        zc = (n - b.M + 1) * g.dz                     # bunch centre at tau_{n+1/2}
        kk = np.arange(g.nz + 1)
        lo = ((kk - 0.5) * g.dz - zc) / sigma
        hi = ((kk + 0.5) * g.dz - zc) / sigma
        node_q = b.Q * (norm.cdf(hi) - norm.cdf(lo))
        node_q[np.abs(kk * g.dz - zc) > (b.M + 0.5) * g.dz] = 0.0   # truncated Gaussian
        expect[b.i0, b.j0, :] = node_q
        worst_e = max(worst_e, np.max(np.abs(qe - expect)[interior]))
        worst_h = max(worst_h, np.max(np.abs(qh)))
        if n == 30:
            assert np.max(np.abs(qe - expect)[interior]) < 1e-13
    assert worst_e < 1e-13 * b.Q
    assert worst_h < 1e-13 * b.Q


def test_naive_gauss_is_not_the_invariant(orc):
    """The plain S~ d (no time average, no alpha^2 term) is only first order (28):
    its residual is O(1) relative to the bunch charge while the modified q_e is exact."""
    g, m, f, b = _bunch_run(orc, jaws=False)
    for n in range(30):
        orc.run(g, m, f, 1, n0=n, bunch=b)
    d = {k: np.where(m[k] > 0, f[k] / np.where(m[k] > 0, m[k], 1.0), 0.0) for k in ("ex", "ey", "ez")}
    i, j = b.i0, b.j0
    div = np.zeros(g.nz + 1)
    for k in range(1, g.nz):
        div[k] = (d["ex"][i, j, k] - d["ex"][i - 1, j, k] + d["ey"][i, j, k] - d["ey"][i, j - 1, k]
                  + d["ez"][i, j, k] - d["ez"][i, j, k - 1])
    zc = (29 - b.M + 1) * g.dz
    kk = np.arange(g.nz + 1)
    node_q = norm.cdf(((kk + 0.5) * g.dz - zc) / b.sigma) - norm.cdf(((kk - 0.5) * g.dz - zc) / b.sigma)
    assert np.max(np.abs(div - node_q)[1:-1]) > 1e-3


def test_wake_energy_identity(orc):
    """Energy balance of the wake quadrature: after the bunch has left, the field
    energy W^N equals sum_m lam_m acc(s = -m dz) (charge ahead by m cells is the
    witness at s = -m dz), from the energy law (19) with j_z^n dtau = lam."""
    g, m, f, b = _bunch_run(orc, nz=30)
    N = g.nz + 2 * b.M + 2
    r = orc.run(g, m, f, N, bunch=b)
    WN = orc.energy(g, m, f)
    lam = r["lam"]
    acc = r["acc"]
    tot = 0.0
    for mm in range(-b.M, b.M + 1):
        tot += lam[mm + b.M] * acc[-mm - b.jmin]
    assert WN > 0
    assert abs(WN - tot) <= 1e-13 * WN


def test_wake_causality(orc):
    """With dtau = dz nothing travels faster than one cell per step in z: the wake
    ahead of the bunch head (s < -M dz) is exactly zero, bitwise."""
    g, m, f, b = _bunch_run(orc, nz=30)
    r = orc.run(g, m, f, g.nz + 3 * b.M, bunch=b)
    acc = r["acc"]
    j = np.arange(b.jmin, b.jmin + b.nw)
    assert np.all(acc[j < -b.M] == 0.0)
    assert np.any(acc[j == -b.M] != 0.0)
    # and the whole grid is zero ahead of the head after n steps
    g2, m2, f2, b2 = _bunch_run(orc, nz=40)
    orc.run(g2, m2, f2, 12, bunch=b2)
    for key in orc.KEYS:
        assert np.all(f2[key][:, :, 14:] == 0.0), key


def test_loss_factor_positive_and_scales_with_charge(orc):
    """W_par is linear in the source: doubling Q leaves W(s) = acc/Q unchanged
    to rounding, and the loss factor k = sum lam W / Q^2 is positive."""
    out = []
    for Q in (1.0, 2.0):
        g, m, f, b = _bunch_run(orc, nz=30)
        b.Q = Q
        r = orc.run(g, m, f, g.nz + 2 * b.M + 2, bunch=b)
        out.append((r["acc"] / Q, r["lam"], b))
    (w1, lam1, b1), (w2, lam2, _) = out
    assert np.max(np.abs(w1 - w2)) <= 1e-13 * np.max(np.abs(w1))
    kloss = sum(lam1[mm + b1.M] * w1[-mm - b1.jmin] for mm in range(-b1.M, b1.M + 1)) / 1.0
    assert kloss > 0


def test_staircase_pec_edges_are_cell_edges(orc):
    """Staircase reading: the PEC edges are exactly the edges of the PEC cells
    (12 cube edges each) plus the edges tangential to the box walls."""
    nx, ny, nz = 5, 4, 6
    rng = np.random.default_rng(2)
    cells = (rng.random((nx, ny, nz)) < 0.2).astype(np.uint8)
    g = orc.Geom(nx, ny, nz, 1.0, 1.0, 1.0, 0.5)
    m = orc.vacuum_materials(g, cells)
    want = {c: np.zeros(g.shape, bool) for c in ("ex", "ey", "ez")}
    for (i, j, k) in zip(*np.nonzero(cells)):
        for a in (0, 1):
            for b in (0, 1):
                want["ex"][i, j + a, k + b] = True
                want["ey"][i + a, j, k + b] = True
                want["ez"][i + a, j + b, k] = True
    want["ex"][:, [0, ny], :] = True
    want["ex"][:, :, [0, nz]] = True
    want["ey"][[0, nx], :, :] = True
    want["ey"][:, :, [0, nz]] = True
    want["ez"][[0, nx], :, :] = True
    want["ez"][:, [0, ny], :] = True
    sl = {"ex": np.s_[:nx, :, :], "ey": np.s_[:, :ny, :], "ez": np.s_[:, :, :nz]}
    for c in ("ex", "ey", "ez"):
        got = (m[c] == 0.0)[sl[c]]
        assert np.array_equal(got, want[c][sl[c]]), c
