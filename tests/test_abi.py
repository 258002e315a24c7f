"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates descriptors (stability bound (25), Sec. 4.4)."""
import ctypes as C
import os
import re

import pytest

from paper_0901_1053_amd import tete

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    hdr = open(os.path.join(ROOT, "include", "tete.h")).read()
    return re.findall(r"^\s*(?:const char\*|tete_status|size_t)\s+(tete_\w+)\s*\(", hdr, re.M)


def test_exports_every_declared_symbol():
    L = tete.load()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    # the binding declares exactly the header's functions
    src = open(os.path.join(ROOT, "paper_0901_1053_amd", "tete.py")).read()
    for n in names:
        assert '"%s"' % n in src, n


def test_status_strings():
    L = tete.load()
    for code, name in tete.STATUS.items():
        assert L.tete_status_str(code).decode() == name


@pytest.mark.parametrize("dx,dy,dz,cdt,want", [
    (2e-3, 2e-3, 1e-3, 1e-3, "TETE_OK"),                 # dx = dy = 2 dz, magic step
    (1e-3, 1e-3, 1e-3, 1e-3, "TETE_ERR_UNSTABLE"),       # cubic cells at c dt = dz
    (1e-3, 1e-3, 1e-3, 0.999e-3 / 2 ** 0.5, "TETE_OK"),  # cubic cells below the transverse bound
    (2e-3, 2e-3, 1e-3, 1.001e-3, "TETE_ERR_UNSTABLE"),   # above dz
    (2 ** 0.5 * 1e-3, 2 ** 0.5 * 1e-3, 1e-3, 1e-3, "TETE_OK"),  # dx = sqrt(2) dz: both bounds equal
    (2e-3, 2e-3, 1e-3, -1e-3, "TETE_ERR_ARG"),
    (2e-3, 0.0, 1e-3, 1e-3, "TETE_ERR_ARG"),
])
def test_stability_validation(dx, dy, dz, cdt, want):
    d = tete.make_desc(24, 24, 48, dx, dy, dz, cdt)
    assert tete.check_desc(d) == want


def test_descriptor_limits():
    assert tete.check_desc(tete.make_desc(1, 4, 4, 2, 2, 1, 1)) == "TETE_ERR_ARG"
    assert tete.check_desc(tete.make_desc(2, 2, 2, 2, 2, 1, 1)) == "TETE_OK"
    assert tete.check_desc(tete.make_desc(2048, 1024, 1024, 2, 2, 1, 1)) == "TETE_ERR_ARG"   # >= 2^31 entries
    # the largest grid: 1016 x 1024 x 2048 = 2^31 - 2^24 entries (int indices
    # with room for a grid-stride loop's last step); one plane more is refused
    assert tete.check_desc(tete.make_desc(1015, 1023, 2047, 2, 2, 1, 1)) == "TETE_OK"
    assert tete.check_desc(tete.make_desc(1016, 1023, 2047, 2, 2, 1, 1)) == "TETE_ERR_ARG"
    d = tete.make_desc(8, 8, 8, 2, 2, 1, 1)
    d.precision = 7
    assert tete.check_desc(d) == "TETE_ERR_ARG"
    d = tete.make_desc(8, 8, 8, 2, 2, 1, 1)
    d.flags = 16                                           # no such flag
    assert tete.check_desc(d) == "TETE_ERR_ARG"
    for kw in ({"yee": True}, {"implicit": True}):   # the skip is for the explicit TE/TM kernels
        assert tete.check_desc(tete.make_desc(8, 8, 8, 2, 2, 1, 0.5, skip_static=True, **kw)) == "TETE_ERR_ARG"
    assert tete.check_desc(tete.make_desc(8, 8, 8, 2, 2, 1, 1, skip_static=True)) == "TETE_OK"
    assert tete.check_desc(tete.make_desc(8, 8, 8, 2, 2, 1, 1, materials=True, skip_static=True)) == "TETE_OK"
    d = tete.make_desc(8, 8, 8, 2, 2, 1, 0.5, materials=True, yee=True)     # Yee is vacuum + PEC only
    assert tete.check_desc(d) == "TETE_ERR_ARG"


@pytest.mark.parametrize("dx,dy,dz,cdt,want", [
    (2e-3, 2e-3, 1e-3, 1e-3, "TETE_ERR_UNSTABLE"),                       # TE/TM's dtau = dz is beyond (8)
    (2e-3, 2e-3, 1e-3, (0.25e6 + 0.25e6 + 1e6) ** -0.5, "TETE_OK"),      # exactly at (8)
    (2e-3, 2e-3, 1e-3, 1.001 * (0.25e6 + 0.25e6 + 1e6) ** -0.5, "TETE_ERR_UNSTABLE"),
    (1e-3, 1e-3, 1e-3, 0.999e-3 / 3 ** 0.5, "TETE_OK"),                  # cubic cells: dz / sqrt(3)
    (1e-3, 1e-3, 1e-3, 0.999e-3 / 2 ** 0.5, "TETE_ERR_UNSTABLE"),        # allowed by (25), not by (8)
])
def test_yee_stability_validation(dx, dy, dz, cdt, want):
    """Yee grids are checked against (8) instead of (25)."""
    assert tete.check_desc(tete.make_desc(24, 24, 48, dx, dy, dz, cdt, yee=True)) == want


def test_workspace_bytes():
    d64 = tete.make_desc(128, 128, 1024, 2, 2, 1, 1, "fp64")
    d32 = tete.make_desc(128, 128, 1024, 2, 2, 1, 1, "fp32")
    np_ = 129 * 129 * 1025
    b64, b32 = tete.workspace_bytes(d64), tete.workspace_bytes(d32)
    assert b64 >= 12 * 8 * np_ + np_ and b32 >= 12 * 4 * np_ + np_
    assert b64 - b32 == pytest.approx(12 * 4 * np_, rel=1e-3)
    dm = tete.make_desc(128, 128, 1024, 2, 2, 1, 1, "fp64", materials=True)
    assert tete.workspace_bytes(dm) >= b64 + 6 * 8 * np_
    assert tete.workspace_bytes(tete.make_desc(1, 1, 1, 2, 2, 1, 1)) == 0
    # the static-tile table and the active-tile list of each tiling kind (the
    # two-step kernel's and the single step's): one byte and one int32 per
    # tile of the finest tiling (single planes, 10 rows by 28 entries)
    ds = tete.make_desc(128, 128, 1024, 2, 2, 1, 1, "fp64", skip_static=True)
    cap = 129 * -(-129 // 10) * -(-1025 // 28)
    assert 10 * cap <= tete.workspace_bytes(ds) - b64 <= 10 * cap + 1024


@pytest.mark.parametrize("mode,dr,dz,cdt,want", [
    (1, 1e-3, 1e-3, 1e-3, "TETE_OK"),              # dtau = dz = dr, any m >= 1
    (40, 1e-3, 1e-3, 1e-3, "TETE_OK"),             # independent of m
    (1, 0.9e-3, 1e-3, 1e-3, "TETE_ERR_UNSTABLE"),  # above dr
    (2, 1e-3, 1e-3, 1.001e-3, "TETE_ERR_UNSTABLE"),  # above dz
    (0, 1e-3, 1e-3, 1e-3, "TETE_ERR_UNSTABLE"),    # m = 0: the on-axis cell limits dtau to 0.9089 dr
    (0, 1.1e-3, 1e-3, 1e-3, "TETE_ERR_UNSTABLE"),  # 0.9089 * 1.1 dz < dz
    (0, 1.2e-3, 1e-3, 1e-3, "TETE_OK"),
    (0, 1e-3, 1e-3, 0.9085e-3, "TETE_OK"),
    (0, 1e-3, 1e-3, 0.9095e-3, "TETE_ERR_UNSTABLE"),
    (-1, 1e-3, 1e-3, 1e-3, "TETE_ERR_ARG"),
    (1, 1e-3, 0.0, 1e-3, "TETE_ERR_ARG"),
])
def test_rz_stability_validation(mode, dr, dz, cdt, want):
    """r-z grids: dtau <= min(dz, dr) whatever m (Sec. 4.4), and 0.9089 dr for m = 0."""
    assert tete.rz_check_desc(tete.make_rz_desc(64, 256, dr, dz, cdt, mode)) == want


def test_rz_descriptor_limits_and_workspace():
    L = tete.load()
    assert tete.rz_check_desc(tete.make_rz_desc(1, 8, 1.2, 1, 1, 0)) == "TETE_ERR_ARG"
    assert tete.rz_check_desc(tete.make_rz_desc(2, 2, 1.2, 1, 1, 0)) == "TETE_OK"
    # FP64 arrays must stay below 2^31 bytes (buffer addressing); FP32 may be twice as large
    big = tete.make_rz_desc(8191, 32767, 1.2, 1, 1, 0, "fp64")
    assert tete.rz_check_desc(big) == "TETE_ERR_ARG"
    assert tete.rz_check_desc(tete.make_rz_desc(8191, 32767, 1.2, 1, 1, 0, "fp32")) == "TETE_OK"
    d = tete.make_rz_desc(100, 1000, 1.2, 1, 1, 0, "fp32")
    np_ = 101 * 1001
    b = int(L.tete_rz_workspace_bytes(C.byref(d)))
    assert b >= 12 * 4 * np_ + np_
    assert int(L.tete_rz_workspace_bytes(C.byref(big))) == 0


@pytest.mark.parametrize("dx,dz,cdt,want", [
    (0.25e-3, 1e-3, 1e-3, "TETE_OK"),             # fine transverse mesh at dtau = dz: beyond (25), fine for (16)
    (2e-3, 1e-3, 1e-3, "TETE_OK"),
    (0.25e-3, 1e-3, 1.001e-3, "TETE_ERR_UNSTABLE"),  # dtau > dz
])
def test_implicit_stability_validation(dx, dz, cdt, want):
    """Implicit grids are bounded by dtau <= dz only."""
    assert tete.check_desc(tete.make_desc(24, 24, 48, dx, dx, dz, cdt, implicit=True)) == want
    if dx < dz:
        assert tete.check_desc(tete.make_desc(24, 24, 48, dx, dx, dz, cdt)) == "TETE_ERR_UNSTABLE"


def test_implicit_flags_and_workspace():
    assert tete.check_desc(tete.make_desc(8, 8, 8, 2, 2, 1, 1, implicit=True, materials=True)) == "TETE_ERR_ARG"
    assert tete.check_desc(tete.make_desc(8, 8, 8, 2, 2, 1, 0.5, implicit=True, yee=True)) == "TETE_ERR_ARG"
    np_ = 129 * 129 * 1025
    b = tete.workspace_bytes(tete.make_desc(128, 128, 1024, 2, 2, 1, 1, "fp32"))
    bi = tete.workspace_bytes(tete.make_desc(128, 128, 1024, 2, 2, 1, 1, "fp32", implicit=True))
    # four plane-solve arrays and two row lists (int32) of np entries each
    assert bi - b == pytest.approx(4 * 4 * np_ + 2 * 4 * np_, rel=1e-3)


def test_witness_entry_points_check_handles():
    """No GPU needed: the witness calls reject a null grid."""
    L = tete.load()
    assert tete.STATUS[L.tete_set_witness(None, 1, 1)] == "TETE_ERR_ARG"
    assert tete.STATUS[L.tete_clear_witness(None)] == "TETE_ERR_ARG"
    assert tete.STATUS[L.tete_witness_wake(None, None, None, None, 1)] == "TETE_ERR_ARG"
    assert tete.STATUS[L.tete_grid_status(None)] == "TETE_ERR_ARG"
    null6 = tete.P6(*([None] * 6))
    assert tete.STATUS[L.tete_stream_probe(null6, null6, None, 16, tete.FP32, None)] == "TETE_ERR_ARG"
