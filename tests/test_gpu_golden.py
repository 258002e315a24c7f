"""The single-wake workload end to end against the FP64 oracle.

The fixture ``tests/golden/single_wake_step_collimator_128x128x1024.json`` is
written by ``tests/golden/make_single_wake_golden.py``, which calls only the
oracle: the 128 x 128 x 1024 step collimator (1 nC, sigma = 1 mm, 3072
steps), with the wake W(s_j) for s in [-5, 50] sigma, the energy every 256
steps, e_z on the bunch line and all components at 17 sampled nodes after the
last step.  The GPU runs the same workload in the benchmark's launch
configuration (two steps per launch, default tiling), stopping every 256
steps to read the energy (the steps stay paired).

Tolerances: FP64 within 1e-12 (the paper's delta norm on W, relative to the
largest energy for the energies); FP32 fields with FP64 wake and energy
accumulation within 1e-5 on W and on the energy.  Final field values are
compared relative to the largest field the run holds, the bunch's own field
in the pipe (the oracle's cross-section potential times the largest value of
the current's profile): the rounding errors are made on that field, while
the fields left after the bunch has gone are about 100 times smaller.  FP64
within 1e-12 of it; FP32 after 3072 steps of FP32 rounding within 1e-4 of it
(single rounding of each of ~30 operations per step accumulating as a random
walk: sqrt(3072 * 30) * 6e-8 ~ 2e-5, with a factor 5 of margin)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pipe_oracle as PO
from paper_0901_1053_amd import inputs, tete
from tests import parity as P

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "single_wake_step_collimator_128x128x1024.json")


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _self_field_max(case):
    """Largest entry of the bunch's own field in the workload's pipe: e_x,
    e_y = -(P phi) F and h_x, h_y = (dx/dy, dy/dx)(P phi) F."""
    g = O.Geom(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt)
    m = O.vacuum_materials(g, case.cell_mask())
    phi = PO.potential(g, PO.pec_nodes(m), case.i0, case.j0)
    lam = O.bunch_cells(case.Q, case.sigma, case.dz, case.M)
    F = np.abs(PO.profile(lam, case.M, g.cdt, np.arange(-2 * case.M - 1, 1))).max()
    px = np.abs(phi[1:, :] - phi[:-1, :]).max()
    py = np.abs(phi[:, 1:] - phi[:, :-1]).max()
    return F * max(px, py, px * g.dy / g.dx, py * g.dx / g.dy)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_wake_against_oracle(golden, precision):
    case = inputs.single_wake_case()
    assert [case.nx, case.ny, case.nz] == golden["grid"] and case.steps == golden["steps"]
    assert (case.jmin, case.nw, case.M) == (golden["jmin"], golden["nw"], golden["M"])
    print("single wake", case.name, precision, flush=True)
    G = P.gpu_grid(case, precision)
    assert G.get_tuning()["kernel"] == "fused2"
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    energies = {0: G.energy()[0]}
    n = 0
    while n < case.steps:
        k = min(256, case.steps - n)
        G.step(k)
        n += k
        energies[n] = G.energy()[0]
    assert sorted(energies) == golden["energy_steps"]
    W = G.wake()
    W_ref = np.array(golden["W_V_per_C"])
    delta = P.delta_norm(W, W_ref)
    e = np.array([energies[s] for s in golden["energy_steps"]])
    e_ref = np.array(golden["energy"])
    de = float(np.max(np.abs(e - e_ref)) / np.max(np.abs(e_ref)))
    tol = 1e-12 if precision == "fp64" else 1e-5
    print("delta W %.3e  energy %.3e" % (delta, de), flush=True)
    assert delta <= tol
    assert de <= tol
    # causality: nothing ahead of the bunch head
    j = case.jmin + np.arange(case.nw)
    assert np.all(W[j < -case.M] == 0.0) and np.all(W_ref[j < -case.M] == 0.0)
    # final fields: the bunch line and the sampled nodes
    f = G.get_fields(dtype=precision, numpy=False)
    line = f["ez"][case.i0, case.j0, :case.nz].double().cpu().numpy()
    line_ref = np.array(golden["ez_bunch_line"])
    vals = np.array([[float(f[k][tuple(s["node"])].item()) for k in tete.KEYS] for s in golden["samples"]])
    vals_ref = np.array([[s[k] for k in tete.KEYS] for s in golden["samples"]])
    scale = _self_field_max(case)
    assert scale > 10 * max(np.max(np.abs(line_ref)), np.max(np.abs(vals_ref)))
    ftol = 1e-12 if precision == "fp64" else 1e-4
    dl = float(np.max(np.abs(line - line_ref)) / scale)
    dv = float(np.max(np.abs(vals - vals_ref)) / scale)
    print("fields: bunch line %.3e  samples %.3e" % (dl, dv), flush=True)
    assert dl <= ftol and dv <= ftol
    G.close()


OPEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "single_wake_open_pipes_step_collimator_128x128x1024.json")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_wake_between_open_pipes_against_oracle(precision):
    """The same workload between open pipes (tete_set_open_pipes), against the
    oracle's run of ``make_single_wake_open_golden.py``: the device solves for
    the cross-section's potential itself.  W within the delta norm 1e-12
    (FP64) / 1e-5 (FP32), the energies every 128 steps within 1e-12 / 1e-5 of
    the largest, and e_z on the bunch line within 1e-12 / 1e-4 of the bunch's
    own field (as above)."""
    with open(OPEN) as fh:
        gold = json.load(fh)
    case = inputs.single_wake_case()
    assert [case.nx, case.ny, case.nz] == gold["grid"] and (case.jmin, case.nw, case.M) == (
        gold["jmin"], gold["nw"], gold["M"])
    print("single wake, open pipes", precision, flush=True)
    G = P.gpu_grid(case, precision)
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.set_open_pipes(gold["start_step"], gold["kend"])
    n = gold["start_step"]
    energies = {n: G.energy()[0]}
    end = n + gold["steps"]
    while n < end:
        k = min(128, end - n)
        G.step(k)
        n += k
        energies[n] = G.energy()[0]
    assert sorted(energies) == gold["energy_steps"]
    W = G.wake()
    delta = P.delta_norm(W, np.array(gold["W_V_per_C"]))
    e = np.array([energies[s] for s in gold["energy_steps"]])
    e_ref = np.array(gold["energy"])
    de = float(np.max(np.abs(e - e_ref)) / np.max(np.abs(e_ref)))
    f = G.get_fields(dtype=precision, numpy=False)
    line = f["ez"][case.i0, case.j0, :case.nz].double().cpu().numpy()
    dl = float(np.max(np.abs(line - np.array(gold["ez_bunch_line"]))) / _self_field_max(case))
    print("delta W %.3e  energy %.3e  bunch line %.3e" % (delta, de, dl), flush=True)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert delta <= tol and de <= tol
    assert dl <= (1e-12 if precision == "fp64" else 1e-4)
    G.close()
