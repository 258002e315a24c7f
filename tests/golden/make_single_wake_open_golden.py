"""Write the FP64 oracle's single-wake solve between open pipes to a JSON fixture.

    python tests/golden/make_single_wake_open_golden.py [--threads N]

Workload: the step collimator of ``make_single_wake_golden.py`` (128 x 128 x
1024 cells, 1 nC, sigma = 1 mm, samples j in [-64, 640]) between open pipes
(the oracle's reading of the infinite pipes of Sec. 5, ``oracle/pipe_oracle``):
the run starts at step n0 = 383 with the bunch's own field in the uniform
entrance pipe (cell planes 0 .. 383; the collimator starts at plane 384), and
the wake quadrature ends before edge kend = nz - (M + jmax + 3) // 2 = 664,
after which no reflection from the exit wall reaches a sample; 998 steps
complete every sample.  Deterministic inputs, as the closed-box fixture.

Only ``oracle/`` computes.  Stored: the wake accumulator and W(s_j) in V/C,
the energy W^{n,e} (Sec. 4.4) at the start and every 128 steps, and e_z^{n+1/2}
on the bunch line after the last step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O                       # noqa: E402
from oracle import pipe_oracle as PO                 # noqa: E402
from paper_0901_1053_amd import inputs               # noqa: E402

OUT = os.path.join(HERE, "single_wake_open_pipes_step_collimator_128x128x1024.json")
EPS0 = 8.8541878128e-12
CHUNK = 128


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--out", default=OUT)
    args = ap.parse_args()
    if args.threads:
        O.set_threads(args.threads)
    case = inputs.single_wake_case()
    g = O.Geom(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt)
    m = O.vacuum_materials(g, case.cell_mask())
    kst = int(round(case.geometry["z0"] / case.dz))
    jmax = case.jmin + case.nw - 1
    n0 = kst - 1
    kend = case.nz - (case.M + jmax + 3) // 2
    steps = kend + case.M + jmax - n0
    assert PO.uniform_entrance(g, m, n0 + 1) and not PO.uniform_entrance(g, m, kst + 1)
    b = O.Bunch(Q=case.Q, sigma=case.sigma, i0=case.i0, j0=case.j0, M=case.M, jmin=case.jmin, nw=case.nw,
                kend=kend)
    phi = PO.potential(g, PO.pec_nodes(m), case.i0, case.j0)
    lam = O.bunch_cells(case.Q, case.sigma, case.dz, case.M)
    f = PO.self_field(g, m, phi, lam, case.M, n0)
    acc = np.zeros(case.nw)
    energy = {n0: O.energy(g, m, f)}
    t0 = time.time()
    n = n0
    while n < n0 + steps:
        k = min(CHUNK, n0 + steps - n)
        O.run(g, m, f, k, n0=n, bunch=b, acc=acc)
        n += k
        energy[n] = O.energy(g, m, f)
        print("step %d / %d  energy %.17g  %.0f s" % (n, n0 + steps, energy[n], time.time() - t0), flush=True)
    doc = {
        "what": "FP64 oracle, single wake solve between open pipes (Sec. 4.2 scheme (23), Sec. 5 wake, "
                "oracle/pipe_oracle.py)",
        "script": "tests/golden/make_single_wake_open_golden.py",
        "case": case.name,
        "grid": [case.nx, case.ny, case.nz],
        "Q": case.Q, "sigma": case.sigma, "i0": case.i0, "j0": case.j0, "M": case.M,
        "jmin": case.jmin, "nw": case.nw, "start_step": n0, "kend": kend, "steps": steps,
        "oracle_threads": O.get_threads(),
        "acc": [float(v) for v in acc],
        "W_V_per_C": [float(v) for v in acc / (case.Q * EPS0)],
        "energy_steps": sorted(energy),
        "energy": [float(energy[s]) for s in sorted(energy)],
        "ez_bunch_line": [float(v) for v in f["ez"][case.i0, case.j0, :case.nz]],
    }
    tmp = args.out + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(doc, fh, indent=0)
    os.replace(tmp, args.out)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
