"""Edge cases and error paths of the C-ABI on the GPU."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_0901_1053_amd import inputs, tete
from tests import parity as P

pytestmark = pytest.mark.gpu


def _grid(precision="fp64", **kw):
    return tete.Grid(8, 9, 10, 2e-3, 2e-3, 1e-3, 1e-3, precision=precision, **kw)


def test_zero_steps_and_counter():
    G = _grid()
    G.step(0)
    assert G.steps_done() == 0
    G.step(3)
    assert G.steps_done() == 3
    with pytest.raises(tete.TeteError) as e:
        G.step(-1)
    assert e.value.status == "TETE_ERR_ARG"


def test_state_errors():
    G = _grid()
    with pytest.raises(tete.TeteError) as e:
        G.charges()
    assert e.value.status == "TETE_ERR_STATE"
    with pytest.raises(tete.TeteError) as e:
        G.set_materials({k: np.zeros(G.shape) for k in tete.KEYS})
    assert e.value.status == "TETE_ERR_STATE"
    L = tete.load()
    out = np.zeros(4)
    assert L.tete_wake(G.h, out.ctypes.data, 4) == -5         # no bunch
    with pytest.raises(tete.TeteError) as e:
        G.set_bunch(1e-9, 1e-3, 0, 4, 3, -3, 10)               # i0 on the wall
    assert e.value.status == "TETE_ERR_ARG"
    with pytest.raises(tete.TeteError) as e:
        G.set_bunch(1e-9, 1e-3, 4, 4, 5000, -3, 10)            # too many cells
    assert e.value.status == "TETE_ERR_ARG"
    G2 = tete.Grid(8, 9, 10, 2e-3, 2e-3, 1e-3, 0.9e-3)
    with pytest.raises(tete.TeteError) as e:
        G2.set_bunch(1e-9, 1e-3, 4, 4, 3, -3, 10)              # c dt != dz
    assert e.value.status == "TETE_ERR_STATE"


def test_series_capacity_is_checked_before_enqueueing():
    G = _grid(max_series=8)
    G.set_diagnostics(1)
    G.step(8)
    with pytest.raises(tete.TeteError) as e:
        G.step(1)
    assert e.value.status == "TETE_ERR_STATE"
    assert G.steps_done() == 8


def test_nonfinite_fields_are_reported():
    G = _grid()
    f = inputs.random_fields(G.shape, 1)
    f["hz"][3, 3, 3] = np.nan
    G.set_fields(f)
    with pytest.raises(tete.TeteError) as e:
        G.energy()
    assert e.value.status == "TETE_ERR_NONFINITE"


def test_workspace_checks():
    import torch
    L = tete.load()
    d = tete.make_desc(8, 8, 8, 2e-3, 2e-3, 1e-3, 1e-3)
    nb = tete.workspace_bytes(d)
    ws = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.tete_grid_create(C.byref(d), C.c_void_p(ws.data_ptr()), nb - 1, s, C.byref(h)) == -3
    assert L.tete_grid_create(C.byref(d), C.c_void_p(ws.data_ptr() + 8), nb, s, C.byref(h)) == -1
    bad = tete.make_desc(8, 8, 8, 1e-3, 1e-3, 1e-3, 1e-3)
    assert L.tete_grid_create(C.byref(bad), C.c_void_p(ws.data_ptr()), nb, s, C.byref(h)) == -2
    assert L.tete_grid_create(C.byref(d), C.c_void_p(ws.data_ptr()), nb, s, C.byref(h)) == 0
    assert L.tete_grid_destroy(h) == 0


def test_fp32_fp64_import_export_round_trip():
    G = _grid("fp32")
    f = inputs.random_fields(G.shape, 2)
    G.set_fields({k: v.astype(np.float32) for k, v in f.items()}, dtype="fp32")
    back = G.get_fields(dtype="fp64")
    g = O.Geom(8, 9, 10, 2e-3, 2e-3, 1e-3, 1e-3)
    m = O.vacuum_materials(g)
    fo = {k: v.astype(np.float32).astype(np.float64) for k, v in f.items()}
    O.apply_pec(g, m, fo)
    masks = P.range_masks(G.shape)
    for k in tete.KEYS:
        assert np.array_equal(back[k][masks[k]], fo[k][masks[k]]), k


def test_resume_from_fields_is_exact():
    """Checkpoint/resume of a source-free run: get_fields after n steps,
    set_fields into a fresh grid, continue: bitwise equal to the straight run."""
    f = inputs.random_fields((9, 10, 11), 3)
    A = _grid()
    A.set_fields(f)
    A.step(20)
    B = _grid()
    B.set_fields(f)
    B.step(8)
    mid = B.get_fields()
    C_ = _grid()
    C_.set_fields(mid)
    C_.step(12)
    fa, fc = A.get_fields(), C_.get_fields()
    for k in tete.KEYS:
        assert np.array_equal(fa[k], fc[k]), k


def test_minimal_grid_with_bunch():
    """2 x 2 x 2 cells with the bunch on the only interior node line."""
    case = inputs.WakeCase("tiny", 2, 2, 2, 2e-3, 2e-3, 1e-3, 1e-3, 10, Q=1e-9, sigma=0.5e-3, jmin=-4, nw=12)
    ref = P.oracle_wake(case, 10)
    got = P.gpu_wake(case, 10)
    assert np.max(np.abs(got["W"] - ref["W"])) <= 1e-12 * max(np.max(np.abs(ref["W"])), 1e-300)
