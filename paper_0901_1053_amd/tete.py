"""Thin Python binding of libtete (include/tete.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides the device workspace, the device arrays handed to
the library, and the stream.  If the library is not built the import fails
loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtete.so")

FP64, FP32 = 0, 1
F_MATERIALS = 1
F_YEE = 2
F_IMPLICIT = 4
F_SKIP_STATIC = 8
MAX_BUNCH_CELLS = 8191
MAX_WAKE = 65536
MAX_PROBES = 16
KEYS = ("ex", "ey", "ez", "hx", "hy", "hz")

STATUS = {0: "TETE_OK", -1: "TETE_ERR_ARG", -2: "TETE_ERR_UNSTABLE", -3: "TETE_ERR_NOMEM",
          -4: "TETE_ERR_DEVICE", -5: "TETE_ERR_STATE", -6: "TETE_ERR_NONFINITE"}


class TeteError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(code, "?"), code))
        self.code = code
        self.status = STATUS.get(code, "?")


class GridDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("cdt", C.c_double),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("max_series", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("rows", C.c_int32), ("xchunk", C.c_int32), ("depth", C.c_int32),
                ("order", C.c_int32)]


KERNELS = {"auto": 0, "fused": 1, "split": 2, "fused2": 3, "yee": 4, "implicit": 5}


class Bunch(C.Structure):
    _fields_ = [("charge_C", C.c_double), ("sigma_z", C.c_double), ("i0", C.c_int32), ("j0", C.c_int32),
                ("half_cells", C.c_int32), ("jmin", C.c_int32), ("nw", C.c_int32)]


RZ_KEYS = ("ephi", "er", "ez", "hphi", "hr", "hz")


class RZDesc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("dr", C.c_double), ("dz", C.c_double),
                ("cdt", C.c_double), ("mode", C.c_int32), ("precision", C.c_int32)]


class RZBunch(C.Structure):
    _fields_ = [("charge_C", C.c_double), ("sigma_z", C.c_double), ("j0", C.c_int32), ("half_cells", C.c_int32),
                ("jw", C.c_int32), ("jmin", C.c_int32), ("nw", C.c_int32)]


_lib = None
P6 = C.c_void_p * 6
P3 = C.c_void_p * 3


def load(path: str = LIB_PATH):
    """Load libtete.so and declare its C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libtete.so is not built (%s); run python -m paper_0901_1053_amd.build" % path)
    # torch first: the library then binds to the HIP runtime torch already
    # loaded, so the process holds one runtime and torch's device memory and
    # streams are valid in the library's calls
    import torch  # noqa: F401
    L = C.CDLL(path)
    st = C.c_int
    vp = C.c_void_p
    sig = {
        "tete_check_desc": (st, [C.POINTER(GridDesc)]),
        "tete_workspace_bytes": (C.c_size_t, [C.POINTER(GridDesc)]),
        "tete_grid_create": (st, [C.POINTER(GridDesc), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "tete_grid_destroy": (st, [vp]),
        "tete_set_pec_cells": (st, [vp, vp]),
        "tete_set_materials": (st, [vp, P3, P3, C.c_int32]),
        "tete_set_material_classes": (st, [vp, vp, vp, C.c_int32]),
        "tete_set_fields": (st, [vp, P6, C.c_int32]),
        "tete_get_fields": (st, [vp, P6, C.c_int32]),
        "tete_set_bunch": (st, [vp, C.POINTER(Bunch)]),
        "tete_clear_bunch": (st, [vp]),
        "tete_set_open_pipes": (st, [vp, C.c_int64, C.c_int32, C.POINTER(C.c_int32)]),
        "tete_set_diagnostics": (st, [vp, C.c_int32]),
        "tete_set_probes": (st, [vp, vp, C.c_int32]),
        "tete_step": (st, [vp, C.c_int64]),
        "tete_steps_done": (st, [vp, C.POINTER(C.c_int64)]),
        "tete_grid_status": (st, [vp]),
        "tete_stream_probe": (st, [P6, P6, vp, C.c_int64, C.c_int32, vp]),
        "tete_wake": (st, [vp, vp, C.c_int32]),
        "tete_set_witness": (st, [vp, C.c_int32, C.c_int32]),
        "tete_clear_witness": (st, [vp]),
        "tete_witness_wake": (st, [vp, vp, vp, vp, C.c_int32]),
        "tete_static_tiles": (st, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
        "tete_energy": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "tete_energy_noalloc": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "tete_energy_series": (st, [vp, vp, C.c_int64, C.POINTER(C.c_int64)]),
        "tete_probes": (st, [vp, vp, C.c_int64, C.POINTER(C.c_int64)]),
        "tete_charges": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "tete_set_tuning": (st, [vp, C.POINTER(Tuning)]),
        "tete_get_tuning": (st, [vp, C.POINTER(Tuning)]),
        "tete_set_timing": (st, [vp, C.c_int64]),
        "tete_timing": (st, [vp, vp, C.c_int32, C.POINTER(C.c_int64)]),
        "tete_batch_bytes": (C.c_size_t, [C.c_int32]),
        "tete_batch_create": (st, [C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "tete_batch_destroy": (st, [vp]),
        "tete_batch_set": (st, [vp, C.c_int32, vp]),
        "tete_batch_set_launch": (st, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "tete_batch_step": (st, [vp, C.c_int64]),
        "tete_batch_count": (st, [vp, C.POINTER(C.c_int32)]),
        "tete_status_str": (C.c_char_p, [C.c_int]),
        "tete_rz_check_desc": (st, [C.POINTER(RZDesc)]),
        "tete_rz_workspace_bytes": (C.c_size_t, [C.POINTER(RZDesc)]),
        "tete_rz_create": (st, [C.POINTER(RZDesc), vp, C.c_size_t, vp, C.POINTER(vp)]),
        "tete_rz_destroy": (st, [vp]),
        "tete_rz_set_pec_cells": (st, [vp, vp]),
        "tete_rz_set_fields": (st, [vp, P6, C.c_int32]),
        "tete_rz_get_fields": (st, [vp, P6, C.c_int32]),
        "tete_rz_set_bunch": (st, [vp, C.POINTER(RZBunch)]),
        "tete_rz_step": (st, [vp, C.c_int64]),
        "tete_rz_steps_done": (st, [vp, C.POINTER(C.c_int64)]),
        "tete_rz_set_open_pipes": (st, [vp, C.c_int64, C.c_int32]),
        "tete_rz_wake": (st, [vp, vp, vp, C.c_int32]),
        "tete_rz_energy": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "tete_rz_set_tuning": (st, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "tete_rz_set_timing": (st, [vp, C.c_int64]),
        "tete_rz_timing": (st, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _chk(fn, code):
    if code != 0:
        raise TeteError(fn, code)


def make_desc(nx, ny, nz, dx, dy, dz, cdt, precision="fp64", materials=False, max_series=0,
              yee=False, implicit=False, skip_static=False) -> GridDesc:
    prec = {"fp64": FP64, "fp32": FP32}[precision]
    flags = (F_MATERIALS if materials else 0) | (F_YEE if yee else 0) | (F_IMPLICIT if implicit else 0) | \
        (F_SKIP_STATIC if skip_static else 0)
    return GridDesc(nx, ny, nz, dx, dy, dz, cdt, prec, flags, max_series)


def check_desc(desc: GridDesc) -> str:
    return STATUS[load().tete_check_desc(C.byref(desc))]


def workspace_bytes(desc: GridDesc) -> int:
    return int(load().tete_workspace_bytes(C.byref(desc)))


class Grid:
    """One explicit TE/TM grid (or, with yee=True, a grid stepped with Yee's
    scheme (7), with implicit=True one stepped with the implicit TE/TM scheme
    (16), for comparison) living in a torch-owned device workspace.
    skip_static=True lets the fused kernels (two-step, single-step and the
    materials step) leave out tiles that lie wholly in PEC (the results are
    unchanged)."""

    def __init__(self, nx, ny, nz, dx, dy, dz, cdt, precision="fp64", materials=False, max_series=0,
                 device="cuda:0", stream=None, yee=False, implicit=False, skip_static=False):
        import torch
        L = load()
        self.torch = torch
        self.desc = make_desc(nx, ny, nz, dx, dy, dz, cdt, precision, materials, max_series, yee, implicit,
                              skip_static)
        _chk("tete_check_desc", L.tete_check_desc(C.byref(self.desc)))
        self.nbytes = workspace_bytes(self.desc)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # 256-byte aligned workspace (the caching allocator aligns to 512 bytes)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _chk("tete_grid_create", L.tete_grid_create(C.byref(self.desc), C.c_void_p(self.ws.data_ptr()),
                                                        self.nbytes, C.c_void_p(self.stream.cuda_stream),
                                                        C.byref(h)))
        self.h = h
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dx, self.dy, self.dz, self.cdt = dx, dy, dz, cdt
        self.precision = precision
        self.shape = (nx + 1, ny + 1, nz + 1)
        self.np = (nx + 1) * (ny + 1) * (nz + 1)
        self.bunch = None
        self._keep = []

    # -- helpers ---------------------------------------------------------
    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def close(self):
        if self.h:
            load().tete_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up ---------------------------------------------------------
    def set_pec_cells(self, cells):
        t = self.torch
        if cells is None:
            _chk("tete_set_pec_cells", load().tete_set_pec_cells(self.h, None))
            return
        d = self._dev(cells, t.uint8)
        assert tuple(d.shape) == (self.nx, self.ny, self.nz)
        _chk("tete_set_pec_cells", load().tete_set_pec_cells(self.h, C.c_void_p(d.data_ptr())))
        self.stream.synchronize()

    def set_materials(self, mat: dict, dtype="fp64"):
        t = self.torch
        td = t.float64 if dtype == "fp64" else t.float32
        arrs = [self._dev(mat[k], td) for k in KEYS]
        pe = P3(*[a.data_ptr() for a in arrs[:3]])
        pm = P3(*[a.data_ptr() for a in arrs[3:]])
        _chk("tete_set_materials", load().tete_set_materials(self.h, pe, pm, FP64 if dtype == "fp64" else FP32))
        self.stream.synchronize()

    def set_material_classes(self, cls, table):
        """Materials by class: cls (nx+1, ny+1, nz+1) uint8 class per entry,
        table (ncls, 6) doubles kappa_x, kappa_y, kappa_z, mu_x, mu_y, mu_z."""
        t = self.torch
        d = self._dev(cls, t.uint8)
        assert d.numel() == self.np
        tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
        assert tab.ndim == 2 and tab.shape[1] == 6
        _chk("tete_set_material_classes", load().tete_set_material_classes(self.h, C.c_void_p(d.data_ptr()),
                                                                           tab.ctypes.data, tab.shape[0]))

    def set_fields(self, f: dict, dtype="fp64"):
        t = self.torch
        td = t.float64 if dtype == "fp64" else t.float32
        arrs = [self._dev(f[k], td) for k in KEYS]
        for a in arrs:
            assert a.numel() == self.np
        _chk("tete_set_fields", load().tete_set_fields(self.h, P6(*[a.data_ptr() for a in arrs]),
                                                       FP64 if dtype == "fp64" else FP32))
        self.stream.synchronize()

    def get_fields(self, dtype="fp64", numpy=True):
        t = self.torch
        td = t.float64 if dtype == "fp64" else t.float32
        arrs = [t.empty(self.shape, dtype=td, device=self.device) for _ in KEYS]
        _chk("tete_get_fields", load().tete_get_fields(self.h, P6(*[a.data_ptr() for a in arrs]),
                                                       FP64 if dtype == "fp64" else FP32))
        self.stream.synchronize()
        if numpy:
            return {k: a.cpu().numpy() for k, a in zip(KEYS, arrs)}
        return dict(zip(KEYS, arrs))

    def set_bunch(self, charge, sigma, i0, j0, half_cells, jmin, nw):
        self.bunch = Bunch(charge, sigma, i0, j0, half_cells, jmin, nw)
        _chk("tete_set_bunch", load().tete_set_bunch(self.h, C.byref(self.bunch)))

    def clear_bunch(self):
        _chk("tete_clear_bunch", load().tete_clear_bunch(self.h))
        self.bunch = None

    def set_open_pipes(self, start_step: int, kend: int = 0) -> int:
        """Open entrance and exit pipes (tete_set_open_pipes): the bunch's
        field in the uniform entrance pipe as the state of step start_step,
        and the wake quadrature ending before edge kend (0: all edges).
        Returns the conjugate-gradient iterations of the cross-section's
        potential."""
        it = C.c_int32(0)
        _chk("tete_set_open_pipes", load().tete_set_open_pipes(self.h, int(start_step), int(kend), C.byref(it)))
        return it.value

    def set_diagnostics(self, every: int):
        _chk("tete_set_diagnostics", load().tete_set_diagnostics(self.h, every))

    def set_probes(self, idx):
        a = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
        _chk("tete_set_probes", load().tete_set_probes(self.h, a.ctypes.data, len(a)))

    # -- stepping -------------------------------------------------------
    def step(self, n: int):
        _chk("tete_step", load().tete_step(self.h, int(n)))

    def steps_done(self) -> int:
        v = C.c_int64()
        _chk("tete_steps_done", load().tete_steps_done(self.h, C.byref(v)))
        return v.value

    def status(self) -> str:
        """The grid's sticky error state: "TETE_OK" or "TETE_ERR_NONFINITE"."""
        return STATUS[load().tete_grid_status(self.h)]

    # -- results --------------------------------------------------------
    def wake(self) -> np.ndarray:
        """W(s_j) in V/C for j = jmin .. jmin+nw-1."""
        nw = self.bunch.nw
        out = np.zeros(nw)
        _chk("tete_wake", load().tete_wake(self.h, out.ctypes.data, nw))
        return out

    def wake_s(self) -> np.ndarray:
        return (self.bunch.jmin + np.arange(self.bunch.nw)) * self.dz

    def set_witness(self, iw: int, jw: int):
        """Sample the wake on the node lines (iw, jw), (iw -+ 1, jw), (iw, jw -+ 1)."""
        _chk("tete_set_witness", load().tete_set_witness(self.h, int(iw), int(jw)))

    def clear_witness(self):
        _chk("tete_clear_witness", load().tete_clear_witness(self.h))

    def witness_wake(self):
        """(W (5, nw): W_par on the witness node and its neighbours -x, +x, -y,
        +y; Wx, Wy (nw): the Panofsky-Wenzel transverse wake at the node), V/C."""
        nw = self.bunch.nw
        W = np.zeros((5, nw))
        wx = np.zeros(nw)
        wy = np.zeros(nw)
        _chk("tete_witness_wake", load().tete_witness_wake(self.h, W.ctypes.data, wx.ctypes.data, wy.ctypes.data, nw))
        return W, wx, wy

    def static_tiles(self):
        """(tiles left out, tiles) of the tiling the next step takes
        (skip_static grids)."""
        a, b = C.c_int64(), C.c_int64()
        _chk("tete_static_tiles", load().tete_static_tiles(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def energy(self):
        w = C.c_double()
        n = C.c_int64()
        _chk("tete_energy", load().tete_energy(self.h, C.byref(w), C.byref(n)))
        return w.value, n.value

    def energy_noalloc(self):
        """tete_energy_noalloc: the energy with the library's static device
        scratch instead of the workspace (no allocation)."""
        w = C.c_double()
        n = C.c_int64()
        _chk("tete_energy_noalloc", load().tete_energy_noalloc(self.h, C.byref(w), C.byref(n)))
        return w.value, n.value

    def energy_series(self, max_n=1 << 20) -> np.ndarray:
        cnt = C.c_int64()
        out = np.zeros(max_n)
        _chk("tete_energy_series", load().tete_energy_series(self.h, out.ctypes.data, max_n, C.byref(cnt)))
        return out[: min(cnt.value, max_n)].copy()

    def probes(self, nprobe: int, max_steps=1 << 16) -> np.ndarray:
        cnt = C.c_int64()
        out = np.zeros(max_steps * nprobe)
        _chk("tete_probes", load().tete_probes(self.h, out.ctypes.data, out.size, C.byref(cnt)))
        n = min(cnt.value, max_steps)
        return out[: n * nprobe].reshape(n, nprobe).copy()

    def set_tuning(self, kernel="auto", rows=0, xchunk=0, depth=0, order=0):
        t = Tuning(KERNELS[kernel], rows, xchunk, depth, order)
        _chk("tete_set_tuning", load().tete_set_tuning(self.h, C.byref(t)))

    def get_tuning(self):
        t = Tuning()
        _chk("tete_get_tuning", load().tete_get_tuning(self.h, C.byref(t)))
        inv = {v: k for k, v in KERNELS.items()}
        return {"kernel": inv[t.kernel], "rows": t.rows, "xchunk": t.xchunk, "depth": t.depth, "order": t.order}

    def set_timing(self, max_steps: int):
        _chk("tete_set_timing", load().tete_set_timing(self.h, int(max_steps)))

    def timing(self):
        """(ms of the TM-like kernel, ms of the TE-like kernel, timed steps)."""
        ms = np.zeros(2)
        n = C.c_int64()
        _chk("tete_timing", load().tete_timing(self.h, ms.ctypes.data, 2, C.byref(n)))
        return float(ms[0]), float(ms[1]), n.value

    def charges(self):
        e = C.c_double()
        h = C.c_double()
        _chk("tete_charges", load().tete_charges(self.h, C.byref(e), C.byref(h)))
        return e.value, h.value


class Batch:
    """Grids of one precision stepped together by the persistent batched kernel."""

    def __init__(self, precision="fp32", device="cuda:0", stream=None):
        import torch
        L = load()
        self.torch = torch
        prec = {"fp64": FP64, "fp32": FP32}[precision]
        self.nbytes = int(L.tete_batch_bytes(prec))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.table = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _chk("tete_batch_create", L.tete_batch_create(prec, C.c_void_p(self.table.data_ptr()), self.nbytes,
                                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.members = {}

    def set(self, slot: int, grid):
        _chk("tete_batch_set", load().tete_batch_set(self.h, slot, grid.h if grid is not None else None))
        if grid is None:
            self.members.pop(slot, None)
        else:
            self.members[slot] = grid

    def set_launch(self, rows=0, depth=0, graph_steps=8, kernel="auto"):
        _chk("tete_batch_set_launch", load().tete_batch_set_launch(self.h, KERNELS[kernel], rows, depth, graph_steps))

    def step(self, n: int):
        _chk("tete_batch_step", load().tete_batch_step(self.h, int(n)))

    def count(self) -> int:
        v = C.c_int32()
        _chk("tete_batch_count", load().tete_batch_count(self.h, C.byref(v)))
        return v.value

    def close(self):
        if self.h:
            load().tete_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_probe(src: list, dst: list, code, stream=None):
    """tete_stream_probe: dst[c] = src[c] for six device tensors of one dtype
    (float32 or float64, same length n), reading the uint8 device tensor code
    (n entries) as well; asynchronous on `stream` (default: the current one)."""
    import torch
    n = src[0].numel()
    assert len(src) == 6 and len(dst) == 6 and code.numel() == n and code.dtype == torch.uint8
    for a in list(src) + list(dst):
        assert a.numel() == n and a.dtype == src[0].dtype and a.is_contiguous()
    dt = {torch.float32: FP32, torch.float64: FP64}[src[0].dtype]
    s = stream if stream is not None else torch.cuda.current_stream(src[0].device)
    _chk("tete_stream_probe", load().tete_stream_probe(P6(*[a.data_ptr() for a in src]),
                                                       P6(*[a.data_ptr() for a in dst]),
                                                       C.c_void_p(code.data_ptr()), n, dt,
                                                       C.c_void_p(s.cuda_stream)))


def make_rz_desc(nr, nz, dr, dz, cdt, mode=0, precision="fp64") -> RZDesc:
    return RZDesc(nr, nz, dr, dz, cdt, mode, {"fp64": FP64, "fp32": FP32}[precision])


def rz_check_desc(desc: RZDesc) -> str:
    return STATUS[load().tete_rz_check_desc(C.byref(desc))]


class RZGrid:
    """One r-z grid of the rotationally symmetric scheme (24) at azimuthal
    harmonic `mode`, living in a torch-owned device workspace."""

    def __init__(self, nr, nz, dr, dz, cdt, mode=0, precision="fp64", device="cuda:0", stream=None):
        import torch
        L = load()
        self.torch = torch
        self.desc = make_rz_desc(nr, nz, dr, dz, cdt, mode, precision)
        _chk("tete_rz_check_desc", L.tete_rz_check_desc(C.byref(self.desc)))
        self.nbytes = int(L.tete_rz_workspace_bytes(C.byref(self.desc)))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _chk("tete_rz_create", L.tete_rz_create(C.byref(self.desc), C.c_void_p(self.ws.data_ptr()), self.nbytes,
                                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h
        self.nr, self.nz, self.dr, self.dz, self.cdt, self.mode = nr, nz, dr, dz, cdt, mode
        self.precision = precision
        self.shape = (nr + 1, nz + 1)
        self.np = (nr + 1) * (nz + 1)
        self.bunch = None

    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a))
        return a.to(device=self.device, dtype=dtype).contiguous()

    def close(self):
        if self.h:
            load().tete_rz_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_pec_cells(self, cells):
        t = self.torch
        if cells is None:
            _chk("tete_rz_set_pec_cells", load().tete_rz_set_pec_cells(self.h, None))
            return
        d = self._dev(cells, t.uint8)
        assert tuple(d.shape) == (self.nr, self.nz)
        _chk("tete_rz_set_pec_cells", load().tete_rz_set_pec_cells(self.h, C.c_void_p(d.data_ptr())))
        self.stream.synchronize()

    def set_fields(self, f: dict, dtype="fp64"):
        t = self.torch
        td = t.float64 if dtype == "fp64" else t.float32
        arrs = [self._dev(f[k], td) for k in RZ_KEYS]
        for a in arrs:
            assert a.numel() == self.np
        _chk("tete_rz_set_fields", load().tete_rz_set_fields(self.h, P6(*[a.data_ptr() for a in arrs]),
                                                             FP64 if dtype == "fp64" else FP32))
        self.stream.synchronize()

    def get_fields(self, dtype="fp64", numpy=True):
        t = self.torch
        td = t.float64 if dtype == "fp64" else t.float32
        arrs = [t.empty(self.shape, dtype=td, device=self.device) for _ in RZ_KEYS]
        _chk("tete_rz_get_fields", load().tete_rz_get_fields(self.h, P6(*[a.data_ptr() for a in arrs]),
                                                             FP64 if dtype == "fp64" else FP32))
        if numpy:
            return {k: a.cpu().numpy() for k, a in zip(RZ_KEYS, arrs)}
        return dict(zip(RZ_KEYS, arrs))

    def set_bunch(self, charge, sigma, j0, half_cells, jw, jmin, nw):
        self.bunch = RZBunch(charge, sigma, j0, half_cells, jw, jmin, nw)
        _chk("tete_rz_set_bunch", load().tete_rz_set_bunch(self.h, C.byref(self.bunch)))

    def step(self, n: int):
        _chk("tete_rz_step", load().tete_rz_step(self.h, int(n)))

    def set_open_pipes(self, start_step: int, kend: int = 0) -> None:
        """Open entrance and exit pipes (tete_rz_set_open_pipes): the ring
        bunch's field in the uniform entrance pipe as the state of step
        start_step, and the wake quadrature ending before edge kend."""
        _chk("tete_rz_set_open_pipes", load().tete_rz_set_open_pipes(self.h, int(start_step), int(kend)))

    def steps_done(self) -> int:
        v = C.c_int64()
        _chk("tete_rz_steps_done", load().tete_rz_steps_done(self.h, C.byref(v)))
        return v.value

    def wake(self):
        """(W_par of shape (2, nw): lines jw and jw+1, W_perp of shape (nw,)) in V/C."""
        nw = self.bunch.nw
        wp = np.zeros(2 * nw)
        wt = np.zeros(nw)
        _chk("tete_rz_wake", load().tete_rz_wake(self.h, wp.ctypes.data, wt.ctypes.data, nw))
        return wp.reshape(2, nw), wt

    def wake_s(self) -> np.ndarray:
        return (self.bunch.jmin + np.arange(self.bunch.nw)) * self.dz

    def energy(self):
        w = C.c_double()
        n = C.c_int64()
        _chk("tete_rz_energy", load().tete_rz_energy(self.h, C.byref(w), C.byref(n)))
        return w.value, n.value

    def set_tuning(self, chunk_rows=0, prefetch=0, kernel="auto", order=0):
        """kernel: "auto" or "fused2" (two steps per launch), "fused" (one);
        order 1: r-chunks of a z-column consecutive, 2: z-strips of a chunk."""
        _chk("tete_rz_set_tuning", load().tete_rz_set_tuning(self.h, KERNELS[kernel], chunk_rows, prefetch, order))

    def set_timing(self, max_launches: int):
        _chk("tete_rz_set_timing", load().tete_rz_set_timing(self.h, int(max_launches)))

    def timing(self):
        """(summed kernel ms, launches timed, steps they took)."""
        ms = C.c_double()
        n = C.c_int64()
        st = C.c_int64()
        _chk("tete_rz_timing", load().tete_rz_timing(self.h, C.byref(ms), C.byref(n), C.byref(st)))
        return ms.value, n.value, st.value
