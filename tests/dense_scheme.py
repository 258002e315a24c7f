"""Dense-matrix form of the explicit TE/TM scheme (23) on tiny grids.

An independent route to the same discrete time step as the oracle's ten
sub-updates.  The curl matrix C is assembled geometrically (each primary facet's
boundary circulation, right-hand rule) rather than from the difference stencils;
the scheme is then built from the matrix definitions of Sec. 4.1-4.2:

  scaled system (5):  d/dtau h = -C0 e,  d/dtau e = C0^T h + (current),
                      C0 = M_mu^{1/2} C M_eps^{1/2}  (c = 1)
  grouping (15):      u = (h_x, h_y, e_z), v = (e_x, e_y, h_z),
                      du/dtau = T0 u + L v,  dv/dtau = T1 v - L^T u
  factors (Sec. 4.2): T_i = [[0,0,-X],[0,0,Y],[X^T,-Y^T,0]],
                      L_Ti = [[I,0,0],[0,I,0],[-a X^T, a Y^T, I]],
                      U_Ti = [[I,0,a X],[0,I,-a Y],[0,0,I]]
  scheme (23):        B^e (y^{n+1}-y^n)/dtau + A y^n = f^n,
                      B^e = [[L_T0 U_T0, 0], [2 a L^T, L_T1 U_T1]],
                      A = [[-T0, -L], [L^T, -T1]],  a = dtau/2.

PEC edges (kappa = 0) carry no degree of freedom and are dropped.
"""
from __future__ import annotations

import numpy as np

AXES = "xyz"
CYC = {"x": ("y", "z"), "y": ("z", "x"), "z": ("x", "y")}
UNIT = {"x": (1, 0, 0), "y": (0, 1, 0), "z": (0, 0, 1)}


def _add(p, d, s=1):
    return (p[0] + s * d[0], p[1] + s * d[1], p[2] + s * d[2])


class DenseScheme:
    def __init__(self, g, mat):
        self.g = g
        nx, ny, nz = g.nx, g.ny, g.nz
        self.alpha = 0.5 * g.cdt

        def node_ok(p):
            return 0 <= p[0] <= nx and 0 <= p[1] <= ny and 0 <= p[2] <= nz

        # primary edges e_b(q): q -> q + b
        edges = []
        for b in AXES:
            for i in range(nx + 1):
                for j in range(ny + 1):
                    for k in range(nz + 1):
                        q = (i, j, k)
                        if node_ok(q) and node_ok(_add(q, UNIT[b])):
                            edges.append((b, q))
        # primary facets with normal a at base node p spanning +b, +c
        facets = []
        for a in AXES:
            b, c = CYC[a]
            for i in range(nx + 1):
                for j in range(ny + 1):
                    for k in range(nz + 1):
                        p = (i, j, k)
                        corners = [p, _add(p, UNIT[b]), _add(p, UNIT[c]), _add(_add(p, UNIT[b]), UNIT[c])]
                        if all(node_ok(t) for t in corners):
                            facets.append((a, p))
        eid = {e: n for n, e in enumerate(edges)}
        Cf = np.zeros((len(facets), len(edges)))
        for r, (a, p) in enumerate(facets):
            b, c = CYC[a]
            # counter-clockwise about +a: p -> p+b -> p+b+c -> p+c -> p
            Cf[r, eid[(b, p)]] += 1.0
            Cf[r, eid[(c, _add(p, UNIT[b]))]] += 1.0
            Cf[r, eid[(b, _add(p, UNIT[c]))]] -= 1.0
            Cf[r, eid[(c, p)]] -= 1.0
        self.C_full = Cf
        self.edges, self.facets = edges, facets

        ekey = {"x": "ex", "y": "ey", "z": "ez"}
        hkey = {"x": "hx", "y": "hy", "z": "hz"}
        kap = np.array([mat[ekey[b]][q] for (b, q) in edges])
        mu = np.array([mat[hkey[a]][p] for (a, p) in facets])
        act = kap > 0.0
        self.act_edges = [e for e, on in zip(edges, act) if on]
        self.kap = kap[act]
        self.mu = mu
        C0 = np.sqrt(mu)[:, None] * Cf[:, act] * np.sqrt(self.kap)[None, :]
        nh, ne = C0.shape
        # full operator on (h, e)
        K = np.zeros((nh + ne, nh + ne))
        K[:nh, nh:] = -C0
        K[nh:, :nh] = C0.T
        # u / v ordering
        lab = [("h", a, p) for (a, p) in facets] + [("e", b, q) for (b, q) in self.act_edges]
        sel = lambda kind, ax: [n for n, t in enumerate(lab) if t[0] == kind and t[1] == ax]
        self.I = {"hx": sel("h", "x"), "hy": sel("h", "y"), "ez": sel("e", "z"),
                  "ex": sel("e", "x"), "ey": sel("e", "y"), "hz": sel("h", "z")}
        uo = self.I["hx"] + self.I["hy"] + self.I["ez"]
        vo = self.I["ex"] + self.I["ey"] + self.I["hz"]
        self.order = uo + vo
        self.nu, self.nv = len(uo), len(vo)
        self.lab = [lab[n] for n in self.order]
        Kp = K[np.ix_(self.order, self.order)]
        self.K = Kp
        nu = self.nu
        self.T0 = Kp[:nu, :nu]
        self.L = Kp[:nu, nu:]
        self.T1 = Kp[nu:, nu:]
        self.minusLT = Kp[nu:, :nu]
        # block index sets inside u and v
        n1, n2 = len(self.I["hx"]), len(self.I["hy"])
        self.u_hx, self.u_hy, self.u_ez = (slice(0, n1), slice(n1, n1 + n2), slice(n1 + n2, nu))
        m1, m2 = len(self.I["ex"]), len(self.I["ey"])
        self.v_ex, self.v_ey, self.v_hz = (slice(0, m1), slice(m1, m1 + m2), slice(m1 + m2, self.nv))
        self._build()

    def _factors(self, T, s1, s2, s3):
        a = self.alpha
        X = -T[s1, s3]
        Y = T[s2, s3]
        n = T.shape[0]
        LT = np.eye(n)
        UT = np.eye(n)
        LT[s3, s1] = -a * X.T
        LT[s3, s2] = a * Y.T
        UT[s1, s3] = a * X
        UT[s2, s3] = -a * Y
        R = np.zeros((n, n))
        R[s3, s3] = X.T @ X + Y.T @ Y
        return X, Y, LT, UT, R

    def _build(self):
        a = self.alpha
        nu, nv = self.nu, self.nv
        self.X0, self.Y0, self.LT0, self.UT0, self.R0 = self._factors(self.T0, self.u_hx, self.u_hy, self.u_ez)
        self.X1, self.Y1, self.LT1, self.UT1, self.R1 = self._factors(self.T1, self.v_ex, self.v_ey, self.v_hz)
        Be = np.zeros((nu + nv, nu + nv))
        Be[:nu, :nu] = self.LT0 @ self.UT0
        Be[nu:, :nu] = 2 * a * self.L.T
        Be[nu:, nu:] = self.LT1 @ self.UT1
        A = np.zeros_like(Be)
        A[:nu, :nu] = -self.T0
        A[:nu, nu:] = -self.L
        A[nu:, :nu] = self.L.T
        A[nu:, nu:] = -self.T1
        self.Be, self.A = Be, A
        self.Qe = Be - a * A

    # -- conversions between FIT arrays and the scaled state y = (u, v) --------
    def to_y(self, f):
        y = np.zeros(self.nu + self.nv)
        lab = self.lab
        hkey = {"x": "hx", "y": "hy", "z": "hz"}
        ekey = {"x": "ex", "y": "ey", "z": "ez"}
        fidx = {t: n for n, t in enumerate(self.facets)}
        eidx = {t: n for n, t in enumerate(self.act_edges)}
        for r, (kind, ax, p) in enumerate(lab):
            if kind == "h":
                y[r] = f[hkey[ax]][p] / np.sqrt(self.mu[fidx[(ax, p)]])
            else:
                y[r] = f[ekey[ax]][p] / np.sqrt(self.kap[eidx[(ax, p)]])
        return y

    def source(self, jx=None, jy=None, jz=None):
        """f^n of (23): e-rows carry -kappa^{1/2} j (physical sign)."""
        out = np.zeros(self.nu + self.nv)
        eidx = {t: n for n, t in enumerate(self.act_edges)}
        J = {"x": jx, "y": jy, "z": jz}
        for r, (kind, ax, p) in enumerate(self.lab):
            if kind == "e" and J[ax] is not None:
                out[r] = -np.sqrt(self.kap[eidx[(ax, p)]]) * J[ax][p]
        return out

    def step(self, y, fsrc=None):
        rhs = -self.A @ y
        if fsrc is not None:
            rhs = rhs + fsrc
        return y + self.g.cdt * np.linalg.solve(self.Be, rhs)

    def energy(self, y):
        return 0.5 * y @ self.Qe @ y
