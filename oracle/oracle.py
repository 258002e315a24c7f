"""ctypes wrapper of the FP64 CPU oracle (``tete_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP path; the two meet only through seeded inputs.

Field dictionaries use the keys ``ex ey ez hx hy hz`` with float64 arrays of
shape (nx+1, ny+1, nz+1) (z fastest, C order), holding FIT edge voltages e^ and
dual-edge voltages h^ in units c = eps0 = mu0 = 1.  Materials use the same keys
for the diagonals of M_eps^-1 (kappa, on e) and M_mu^-1 (mu, on h).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tete_oracle.c")
LIB = os.path.join(HERE, "libtete_oracle.so")
KEYS = ("ex", "ey", "ez", "hx", "hy", "hz")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, no FMA contraction; OpenMP shares
    the planes of each sub-update among threads, which leaves every result
    bitwise that of one thread)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Geom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("periodic_xy", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("cdt", C.c_double)]


class _Bunch(C.Structure):
    _fields_ = [("active", C.c_int), ("i0", C.c_int), ("j0", C.c_int), ("M", C.c_int),
                ("lam", C.POINTER(C.c_double)), ("jmin", C.c_int), ("nw", C.c_int), ("kend", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        P6 = C.POINTER(C.c_double) * 6
        L.orc_vacuum_materials.argtypes = [C.POINTER(_Geom), C.c_void_p, P6]
        L.orc_apply_pec.argtypes = [C.POINTER(_Geom), P6, P6]
        L.orc_step.argtypes = [C.POINTER(_Geom), P6, P6, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_energy.argtypes = [C.POINTER(_Geom), P6, P6]
        L.orc_step_yee.argtypes = [C.POINTER(_Geom), P6, P6, C.c_void_p]
        L.orc_yee_invariant.argtypes = [C.POINTER(_Geom), P6, P6, P6]
        L.orc_yee_invariant.restype = C.c_double
        L.orc_yee_charge.argtypes = [C.POINTER(_Geom), P6, P6, C.c_void_p]
        L.orc_energy.restype = C.c_double
        L.orc_charges.argtypes = [C.POINTER(_Geom), P6, P6, P6, C.c_void_p, C.c_void_p]
        L.orc_bunch_cells.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_void_p]
        L.orc_run.argtypes = [C.POINTER(_Geom), P6, P6, C.c_int, C.c_int, C.POINTER(_Bunch),
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]
        L.orc_run.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads used by the sub-updates of a step (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


@dataclass
class Geom:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    cdt: float
    periodic_xy: bool = False

    @property
    def shape(self):
        return (self.nx + 1, self.ny + 1, self.nz + 1)

    def _c(self):
        return _Geom(self.nx, self.ny, self.nz, int(self.periodic_xy),
                     self.dx, self.dy, self.dz, self.cdt)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _p6(d: dict):
    return (C.POINTER(C.c_double) * 6)(*[_ptr(d[k]) for k in KEYS])


def zeros(g: Geom) -> dict:
    return {k: np.zeros(g.shape) for k in KEYS}


def vacuum_materials(g: Geom, cell_pec=None) -> dict:
    """kappa/mu for vacuum with a staircase PEC cell mask (nx, ny, nz) or None."""
    m = zeros(g)
    cp = None
    if cell_pec is not None:
        cell_pec = np.ascontiguousarray(cell_pec, dtype=np.uint8)
        assert cell_pec.shape == (g.nx, g.ny, g.nz)
        cp = cell_pec.ctypes.data
    lib().orc_vacuum_materials(C.byref(g._c()), cp, _p6(m))
    return m


def apply_pec(g: Geom, m: dict, f: dict) -> None:
    lib().orc_apply_pec(C.byref(g._c()), _p6(m), _p6(f))


def step(g: Geom, m: dict, f: dict, jx=None, jy=None, jz=None) -> None:
    """One step of the explicit scheme, in place (currents per edge or None)."""
    def p(a):
        if a is None:
            return None
        assert a.shape == g.shape and a.dtype == np.float64 and a.flags.c_contiguous
        return a.ctypes.data
    lib().orc_step(C.byref(g._c()), _p6(m), _p6(f), p(jx), p(jy), p(jz))


def step_yee(g: Geom, m: dict, f: dict, jz=None) -> None:
    """One step of Yee's scheme (7) in place: state (e^{n-1/2}, h^n)."""
    if jz is not None:
        assert jz.shape == g.shape and jz.dtype == np.float64 and jz.flags.c_contiguous
    lib().orc_step_yee(C.byref(g._c()), _p6(m), _p6(f), None if jz is None else jz.ctypes.data)


def yee_invariant(g: Geom, m: dict, f_old: dict, f_new: dict) -> float:
    """Half the leapfrog invariant <e^{n+1/2}, e^{n-1/2}> + |h^n|^2 of Yee's
    scheme, from the state before (f_old) and after (f_new) one step."""
    return lib().orc_yee_invariant(C.byref(g._c()), _p6(m), _p6(f_old), _p6(f_new))


def yee_charge(g: Geom, m: dict, f: dict) -> np.ndarray:
    """Node charges (dual divergence of e / kappa) of a Yee state."""
    q = np.zeros(g.shape)
    lib().orc_yee_charge(C.byref(g._c()), _p6(m), _p6(f), q.ctypes.data)
    return q


def energy(g: Geom, m: dict, f: dict) -> float:
    return float(lib().orc_energy(C.byref(g._c()), _p6(m), _p6(f)))


def charges(g: Geom, m: dict, f_old: dict, f_new: dict):
    """(q_e^{n+1/2} on nodes (nx+1,ny+1,nz+1), q_h^n on cells (nx,ny,nz))."""
    qe = np.zeros(g.shape)
    qh = np.zeros((g.nx, g.ny, g.nz))
    lib().orc_charges(C.byref(g._c()), _p6(m), _p6(f_old), _p6(f_new), qe.ctypes.data, qh.ctypes.data)
    return qe, qh


def bunch_cells(Q: float, sigma: float, dz: float, M: int) -> np.ndarray:
    lam = np.zeros(2 * M + 1)
    lib().orc_bunch_cells(Q, sigma, dz, M, lam.ctypes.data)
    return lam


@dataclass
class Bunch:
    Q: float
    sigma: float
    i0: int
    j0: int
    M: int
    jmin: int
    nw: int
    kend: int = 0          # wake quadrature over edges k < kend (0: all edges)


def run(g: Geom, m: dict, f: dict, nsteps: int, n0: int = 0, bunch: Bunch | None = None,
        acc: np.ndarray | None = None, want_energy: bool = False, probes=None):
    """Run nsteps steps in place.  Returns dict(energy, probes, acc, lam).

    acc accumulates -1/2 sum (e_z^{n-1/2}+e_z^{n+1/2}) per wake sample (pass the
    previous array to continue a run); W(s_j) = acc / Q in internal units.
    """
    cb = None
    lam = None
    if bunch is not None:
        lam = bunch_cells(bunch.Q, bunch.sigma, g.dz, bunch.M)
        if acc is None:
            acc = np.zeros(bunch.nw)
        cb = _Bunch(1, bunch.i0, bunch.j0, bunch.M, _ptr(lam), bunch.jmin, bunch.nw, bunch.kend)
    en = np.zeros(nsteps) if want_energy else None
    pidx = None
    pout = None
    nprobe = 0
    if probes is not None:
        pidx = np.ascontiguousarray(probes, dtype=np.int64)
        nprobe = len(pidx)
        pout = np.zeros((nsteps, nprobe))
    rc = lib().orc_run(C.byref(g._c()), _p6(m), _p6(f), n0, nsteps,
                       C.byref(cb) if cb is not None else None,
                       acc.ctypes.data if acc is not None else None,
                       en.ctypes.data if en is not None else None,
                       pidx.ctypes.data if pidx is not None else None, nprobe,
                       pout.ctypes.data if pout is not None else None)
    if rc != 0:
        raise MemoryError("oracle run failed (%d)" % rc)
    return {"energy": en, "probes": pout, "acc": acc, "lam": lam}
