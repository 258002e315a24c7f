"""tete_energy_noalloc, the entry point that allocates nothing, against
tete_energy through the C-ABI: two calls in a row on one GPU, the second on a
smaller grid (the static scratch keeps the first call's contents), in FP64
and FP32.  Both entry points run the same kernels in the same order, so the
energies agree bitwise (the bar for FP64 is 1e-12 relative)."""
import numpy as np
import pytest

from paper_0901_1053_amd import inputs, tete

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_energy_matches_energy(precision):
    out = []
    for nt, nz, seed in ((40, 200, 3), (12, 30, 4)):
        case = inputs.scaled_wake_case(nt, nz, seed=seed, sigma_dz=2.0)
        print("noalloc", precision, nt, nz, flush=True)
        G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=precision)
        G.set_pec_cells(case.cell_mask())
        G.set_fields(inputs.random_fields(G.shape, seed))
        G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
        G.step(7)
        e_na, n_na = G.energy_noalloc()
        e, n = G.energy()
        assert n_na == n == 7
        assert abs(e_na - e) <= 1e-12 * abs(e)
        assert e_na == e
        out.append(e_na)
        G.close()
    assert out[0] != out[1]
