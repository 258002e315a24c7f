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
    d = tete.make_desc(8, 8, 8, 2, 2, 1, 1)
    d.precision = 7
    assert tete.check_desc(d) == "TETE_ERR_ARG"
    d = tete.make_desc(8, 8, 8, 2, 2, 1, 1)
    d.flags = 4
    assert tete.check_desc(d) == "TETE_ERR_ARG"
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
