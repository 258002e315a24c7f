#!/usr/bin/env python
"""Throughput of the explicit TE/TM step on one MI355X.

One "step" is one time step of the whole hot path: the TM-like half (S1-S5 with
the bunch current and the FP64 wake update) and the TE-like half (S6-S10) over
every grid entry.  Workload: tapered round-in-square collimator, 512 x 512 x
2048 cells (0.54 G cells), FP32 fields with FP64 wake accumulation, Gaussian
bunch sigma = 0.3 mm, synthetic geometry.  Inputs are resident in HBM before
the timed region; the timed region is bracketed by stream synchronisation and
measured with HIP events on the grid's stream.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

Prints one JSON line.  The headline steps every tile; the context sections
(Yee's scheme, witness lines, the implicit scheme, per-entry materials, tiles
wholly in PEC left out, the r-z scheme, batches, serving) are measured
after it and do not enter `value`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
def traffic_file(kernel_name, precision):
    return os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel_name, precision))


def measured_traffic(kernel_name, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current sources of the kernel (every file it is built
    from, by SHA-256); else None."""
    import hashlib
    try:
        with open(traffic_file(kernel_name, precision)) as fh:
            t = json.load(fh)
        for path, want in t["sources"].items():
            with open(os.path.join(ROOT, path), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest() != want:
                    return None
    except (OSError, ValueError, KeyError, AttributeError):
        return None
    if t["workload"] != workload or t["precision"] != precision:
        return None
    return t["read_bytes_per_launch"] + t["write_bytes_per_launch"]
METRIC = "Gcell-updates/s + HBM GB/s; batched wake solves/s with p50/p99 latency"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, gpu_fp64, nz_slab=32, steps_one=4, steps_all=16):
    """The FP64 oracle (plain C; OpenMP shares the planes of each sub-update,
    bitwise the single-thread result) on a z-slab of the same workload, with
    one thread and with every thread the process may use, beside the GPU's
    FP64 rate on the full workload (equal precision)."""
    from oracle import oracle as O
    g = O.Geom(case.nx, case.ny, nz_slab, case.dx, case.dy, case.dz, case.cdt)
    k0 = case.nz // 2 - nz_slab // 2
    cells = case.cell_mask()[:, :, k0:k0 + nz_slab]
    m = O.vacuum_materials(g, cells)
    b = O.Bunch(Q=case.Q, sigma=case.sigma, i0=case.i0, j0=case.j0, M=case.M, jmin=-4, nw=8)
    threads_all = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads_all = min(threads_all, int(os.environ.get("OMP_NUM_THREADS", threads_all) or threads_all))
    rates = {}
    total = 0.0
    for th, steps in ((1, steps_one), (threads_all, steps_all)):
        O.set_threads(th)
        f = O.zeros(g)
        t0 = time.perf_counter()
        O.run(g, m, f, steps, n0=nz_slab // 2 + case.M - steps // 2, bunch=b)
        dt = time.perf_counter() - t0
        total += dt
        rates[th] = case.nx * case.ny * nz_slab * steps / dt / 1e9
    O.set_threads(threads_all)
    out = {"value": rates[threads_all], "unit": "Gcell-updates/s", "cores": threads_all, "kind": "oracle",
           "single_thread_value": rates[1], "nproc": os.cpu_count(), "cpu_model": cpu_model(),
           "sample": "%dx%dx%d z-slab (cells %d..%d) of the %s workload with its geometry and bunch, FP64: "
                     "%d steps on 1 thread, %d steps on %d threads, %.1f s in all"
                     % (case.nx, case.ny, nz_slab, k0, k0 + nz_slab - 1, case.name, steps_one, steps_all,
                        threads_all, total)}
    if gpu_fp64:
        out["gpu_fp64_gcell_updates_per_s"] = gpu_fp64
        out["gpu_fp64_over_cpu_all_threads"] = round(gpu_fp64 / rates[threads_all], 1)
    return out


def gpu_fp64_rate(case, steps=10):
    """FP64 fields on the same workload (the oracle's precision): Gcell-updates/s
    of the library's default kernel, HIP events on the grid's stream."""
    import torch
    from paper_0901_1053_amd import tete
    G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision="fp64")
    G.set_pec_cells(case.cell_mask())
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.step(2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(G.stream)
    G.step(steps)
    e1.record(G.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    G.close()
    del G
    torch.cuda.empty_cache()
    return round(case.cells * steps / (ms / 1e3) / 1e9, 2)


def copy_ceiling(entries, precision, reps=5):
    """HBM rate of tete_stream_probe: the step's arrays (six read with the code
    byte, six written) streamed once with coalesced 16-byte accesses, over as
    many entries as the workload's grid; bytes per launch / mean launch time
    (HIP events on the current stream)."""
    import torch
    from paper_0901_1053_amd import tete
    td = torch.float32 if precision == "fp32" else torch.float64
    b = 4 if precision == "fp32" else 8
    src = [torch.ones(entries, dtype=td, device="cuda") for _ in range(6)]
    dst = [torch.empty(entries, dtype=td, device="cuda") for _ in range(6)]
    code = torch.zeros(entries, dtype=torch.uint8, device="cuda")
    tete.stream_probe(src, dst, code)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        tete.stream_probe(src, dst, code)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(dst[5], src[5]))
    del src, dst, code
    torch.cuda.empty_cache()
    nbytes = (12 * b + 1) * entries
    return {"kernel": "k_stream (tete_stream_probe)", "bytes_per_launch": nbytes, "ms_per_launch": round(ms, 4),
            "gbps": round(nbytes / (ms / 1e3) / 1e9, 1), "copied_correctly": ok}


def _tuned(cases, precision):
    """Autotune the launch shape for each size class present (cache in /tmp):
    x-planes per workgroup and tile order, each timed in a batch of eight
    copies (the context batch members run in; the persistent batch launch
    has one workgroup shape, 16 rows of 64 lanes, so rows are not searched
    there).  Reports each class's best shape and its gain over the default
    (x-chunk 0, order 2)."""
    from paper_0901_1053_amd.autotune import Tuner, size_class
    # FP32 batches run the two-step kernel: tune that one, in a batch of eight
    tuner = Tuner(cache_path=os.path.join("/tmp", "tete_bench_autotune.json"), xchunks=(0, 16, 32, 64, 128),
                  orders=(2, 1, 4), steps=8, warmup=1, kernel="fused2" if precision == "fp32" else "fused", batch=8)
    shapes = {}
    for c in cases:
        key = size_class(c.nx, c.ny, c.nz, precision)
        if key not in shapes:
            sh = tuner.tune(c.nx, c.ny, c.nz, c.dx, c.dy, c.dz, c.cdt, precision)
            dflt = tuner.timed.get((0, 2, 0, 0))
            # the class rounds each dimension up to a power of two; the time is
            # that of the tuned kernel on the class's first grid
            shapes[key] = {"kernel": tuner.kernel, "xchunk": sh.xchunk, "order": sh.order,
                           "ms_per_step_per_instance": round(sh.ms, 4),
                           "default_ms_per_step_per_instance": round(dflt, 4) if dflt else None,
                           "gain_over_default": round(dflt / sh.ms, 3) if dflt else None,
                           "candidates": len(tuner.timed),
                           "timed_on": "batch of %d x %dx%dx%d" % (tuner.batch, c.nx, c.ny, c.nz)}
    return tuner, shapes


def single_grid_tuning(G, steps=6):
    """Launch shapes of the two-step kernel on the headline grid (rows and
    planes loaded ahead, tile order, x-chunk; depth 0 is the shape's default),
    kernel time per step from the grid's own timing;
    the grid's shape is restored afterwards.  The headline uses the library's
    default shape."""
    saved = G.get_tuning()
    rows_ = []
    shapes = [(16, 0), (16, 2), (24, 1), (24, 0), (24, 3), (32, 0)] if G.precision == "fp32" else [(16, 0)]
    for rows, depth in shapes:
        for order in (2, 4):
            for xc in (0, 128):
                G.set_tuning("fused2", rows, xc, depth, order)
                G.step(2)
                G.set_timing(steps)
                G.step(steps)
                ms, _, n = G.timing()
                G.set_timing(0)
                rows_.append({"rows": rows, "depth": depth, "order": order, "xchunk": xc,
                              "ms_per_step": round(ms / n, 4)})
    G.set_tuning(saved["kernel"], saved["rows"], saved["xchunk"], saved["depth"], saved["order"])
    best = min(rows_, key=lambda r: r["ms_per_step"])
    return {"candidates": rows_, "best": best}


def batched_section(count):
    """All instances of the batched workload submitted at once and served by
    continuous batching (FP32 fields, FP64 wake), against FP64 one-at-a-time
    solves of every eighth instance, scaled to the whole set by their
    cell-update rate."""
    import numpy as np

    from paper_0901_1053_amd import inputs, serve
    cases = inputs.batched_cases(count)
    tuner, shapes = _tuned(cases, "fp32")
    reqs = [serve.Request(i, c, 0.0) for i, c in enumerate(cases)]
    ex = serve.GpuExecutor("fp32", batch=True, graph_steps=8, tuner=tuner)
    st = serve.Server(ex, max_slots=min(count, 256), block_steps=256).run(reqs)
    ex.close()
    cells_steps = sum(c.cells * c.steps for c in cases)
    # FP64 one at a time on every eighth instance (a sample that spans the
    # size mix); the full set's FP64 time follows from their cell-update rate
    pick = list(range(0, count, max(1, count // 8)))
    sub = [serve.Request(i, cases[i], 0.0) for i in pick]
    ex64 = serve.GpuExecutor("fp64", batch=False)
    st64 = serve.Server(ex64, max_slots=1, block_steps=10 ** 7).run(sub)
    ex64.close()
    sub_cells_steps = sum(cases[i].cells * cases[i].steps for i in pick)
    fp64_rate = sub_cells_steps / st64.makespan_s
    fp64_all_s = cells_steps / fp64_rate
    delta = max(float(np.max(np.abs(reqs[i].wake - r.wake)) / (np.max(r.wake) - np.min(r.wake)))
                for i, r in zip(pick, sub))
    return {"workload": "%d tapered-jaw collimators, 64^2x256 .. 192^2x1024" % count, "instances": count,
            "fp32_batched_solves_per_s": round(st.solves_per_s, 3), "makespan_s": round(st.makespan_s, 3),
            "gcell_updates_per_s": round(cells_steps / st.makespan_s / 1e9, 2),
            "fp64_one_at_a_time_solves_per_s": round(count / fp64_all_s, 3),
            "fp64_sample": "every %dth instance (%d of %d, %.1f%% of the set's cell-updates) solved one at a time in "
                           "FP64 at %.1f Gcell-updates/s; the set's FP64 time is its cell-updates over that rate"
                           % (max(1, count // 8), len(pick), count, 100.0 * sub_cells_steps / cells_steps,
                              fp64_rate / 1e9),
            "speedup": round(fp64_all_s / st.makespan_s, 2),
            "max_fp32_delta_vs_fp64": delta, "max_active": st.max_active, "peak_gb": round(st.peak_bytes / 1e9, 2),
            "autotuned_shapes": shapes}


def serve_section(rates, count, max_cells=None):
    """Poisson streams of serving-workload requests: FP32 continuous batching
    (p50/p99 latency, arrival to wake on host) at each rate, against FP64
    one-at-a-time FIFO serving of the same stream.  The one-at-a-time server
    solves the requests in arrival order and its behaviour does not depend on
    the arrival times otherwise, so each request is solved alone once (timed:
    set-up, steps, read-out, release) and its latencies at every rate follow
    from those solve times."""
    import numpy as np

    from paper_0901_1053_amd import inputs, serve
    cases = inputs.serve_cases(count)
    tuner, _ = _tuned(cases, "fp32")
    ex64 = serve.GpuExecutor("fp64", batch=False)
    svc64, w64 = serve.solve_alone(ex64, cases)
    ex64.close()
    res = {"workload": "%d requests, 64^2x256 .. 256^2x2048" % count, "max_cells_in_flight": max_cells,
           "fp64_one_at_a_time": "FIFO over each request's measured FP64 solve time alone "
                                 "(%.2f s for all %d)" % (sum(svc64), count),
           "rates": {}}
    for rate in rates:
        reqs = serve.make_requests(cases, rate, seed=int(rate * 1000) + 7)
        ex = serve.GpuExecutor("fp32", batch=True, graph_steps=8, tuner=tuner)
        st = serve.Server(ex, block_steps=128, max_cells=max_cells).run(reqs)
        ex.close()
        st64 = serve.one_at_a_time_stats([r.arrival for r in reqs], svc64)
        delta = max(float(np.max(np.abs(r.wake - w64[r.rid])) / (np.max(w64[r.rid]) - np.min(w64[r.rid])))
                    for r in reqs)
        res["rates"][str(rate)] = {
            "fp32_batched": {"solves_per_s": round(st.solves_per_s, 3), "p50_s": round(st.p50_s, 4),
                             "p99_s": round(st.p99_s, 4), "max_active": st.max_active},
            "fp64_one_at_a_time": {"solves_per_s": round(st64.solves_per_s, 3), "p50_s": round(st64.p50_s, 4),
                                   "p99_s": round(st64.p99_s, 4)},
            "max_fp32_delta_vs_fp64": delta}
        print("# serve rate %g done" % rate, file=sys.stderr, flush=True)
    res["tolerance"] = 1e-5
    return res


def _ms_per_step(G, steps):
    G.step(2)
    G.set_timing(steps)
    G.step(steps)
    ms, _, n = G.timing()
    G.set_timing(0)
    return ms / n


def yee_section(G, case, precision, steps=20):
    """The paper's cost comparison, measured: kernel time per step of the
    single-step and two-step TE/TM kernels (dtau = dz) and of Yee's scheme (7)
    at its stability limit (8), also with one and two steps per launch, on the
    same grid and geometry, and the time to reach the same physical time tau
    (steps scale as 1 / dtau)."""
    from paper_0901_1053_amd import tete
    tuning = G.get_tuning()
    G.set_tuning("fused2")
    t2 = _ms_per_step(G, steps)
    G.set_tuning("fused")
    t1 = _ms_per_step(G, steps)
    G.set_tuning(tuning["kernel"] if tuning["kernel"] != "yee" else "auto", tuning["rows"], tuning["xchunk"],
                 tuning["depth"], tuning["order"])
    dt_yee = (case.dx ** -2 + case.dy ** -2 + case.dz ** -2) ** -0.5
    Y = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, dt_yee, precision=precision, yee=True)
    Y.set_pec_cells(case.cell_mask())
    Y.set_tuning("fused")
    ty = _ms_per_step(Y, steps)
    Y.set_tuning("auto")
    ty2 = _ms_per_step(Y, steps)
    Y.close()
    del Y
    r = dt_yee / case.cdt
    return {"workload": case.name, "precision": precision,
            "dtau_over_dz": {"te_tm": round(case.cdt / case.dz, 4), "yee_limit_8": round(dt_yee / case.dz, 4)},
            "ms_per_step": {"te_tm_two_step": round(t2, 4), "te_tm_single_step": round(t1, 4), "yee": round(ty, 4),
                            "yee_two_step": round(ty2, 4)},
            "time_to_same_tau_vs_yee": {"te_tm_two_step": round(t2 * r / ty, 3),
                                        "te_tm_single_step": round(t1 * r / ty, 3),
                                        "te_tm_two_step_vs_yee_two_step": round(t2 * r / ty2, 3)},
            "paper": {"cost_per_step_vs_yee": round(10 / 6, 3),
                      "run_time_vs_yee_at_dx_sqrt2_dz": round((10 / 6) / 2 ** 0.5, 3)}}


def witness_section(G, case, two_step_ms, offset=32, steps=20):
    """Off-axis and transverse wakes on the large workload: a witness node
    `offset` cells from the bunch line in x.  Each two-step launch also keeps
    e_z^{n+1/2} of the five witness lines, and a small kernel over the lines
    follows it; time per step from HIP events on the grid's stream around whole
    launches, the step kernel's own time from the grid's timing, and the ratio
    to the two-step kernel without a witness; then also with an energy sample
    before every step."""
    import torch
    G.set_witness(case.i0 + offset, case.j0)
    G.step(2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(G.stream)
    G.step(steps)
    e1.record(G.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    G.set_timing(steps)
    G.step(steps)
    ms_k, _, n = G.timing()
    G.set_timing(0)
    # with an energy sample before every step as well (taken inside the
    # paired launches, which also keep the lines' values)
    G.set_diagnostics(1)
    G.step(2)
    torch.cuda.synchronize()
    e0.record(G.stream)
    G.step(steps)
    e1.record(G.stream)
    torch.cuda.synchronize()
    ms_e = e0.elapsed_time(e1) / steps
    G.set_diagnostics(0)
    G.clear_witness()
    return {"workload": case.name, "witness_offset_cells": [offset, 0], "lines": 5,
            "ms_per_step": round(ms, 4), "step_kernel_ms": round(ms_k / n, 4),
            "line_kernel_and_gap_ms": round(ms - ms_k / n, 4),
            "vs_two_step_without_witness": round(ms / two_step_ms, 3),
            "ms_per_step_with_energy_every_step": round(ms_e, 4)}


def diagnostics_section(G, case, two_step_ms, steps=16):
    """An energy sample (Sec. 4.4) before every step on the large workload:
    time per step from HIP events on the grid's stream, with the default
    kernel (paired launches take both samples, of y^n and y^{n+1}, inside the
    launch) and with single steps (the fused step, the energy kernel before
    each).  The series agree to the rounding of their FP64 sums (tests)."""
    import torch
    saved = G.get_tuning()
    res = {}
    for name, kernel in (("paired_with_samples", "auto"), ("single_steps_and_energy_kernel", "fused")):
        G.set_tuning(kernel)
        G.set_diagnostics(1)
        G.step(2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(G.stream)
        G.step(steps)
        e1.record(G.stream)
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) / steps, 4)
        G.set_diagnostics(0)
    G.set_tuning(saved["kernel"], saved["rows"], saved["xchunk"], saved["depth"], saved["order"])
    # a read-out on its own (tete_energy: the energy kernel, its fixed-order
    # finish and the copy of the value to the host), wall clock per call
    G.energy()
    t0 = time.perf_counter()
    for _ in range(5):
        G.energy()
    readout = (time.perf_counter() - t0) / 5 * 1e3
    b = 4 if G.precision == "fp32" else 8
    return {"workload": case.name, "energy_every": 1, "ms_per_step": res,
            "vs_two_step_without_samples": round(res["paired_with_samples"] / two_step_ms, 3),
            "speedup_over_single_steps": round(res["single_steps_and_energy_kernel"] / res["paired_with_samples"], 2),
            "energy_readout_ms": round(readout, 3),
            "energy_readout_gbps_algorithmic": round((6 * b + 1) * G.np / (readout / 1e3) / 1e9, 1)}


def _pec_materials(case, precision, scale=0.9, graded=False):
    """Per-entry materials carrying the workload's geometry, made on the
    device: kappa and mu `scale` of their vacuum values, kappa zero on the
    staircase PEC edges (an e edge touching a metal cell, cells outside the box
    counting as metal).  graded: each value also times 1 + 0.05 sin(0.013 k +
    0.007 i + c), a medium graded along z and x with far more distinct tuples
    than classes."""
    import numpy as np
    import torch
    from paper_0901_1053_amd import tete
    td = torch.float32 if precision == "fp32" else torch.float64
    nx, ny, nz = case.nx, case.ny, case.nz
    p = torch.ones((nx + 2, ny + 2, nz + 2), dtype=torch.bool, device="cuda")
    p[1:-1, 1:-1, 1:-1] = torch.from_numpy(np.ascontiguousarray(case.cell_mask())).to("cuda").bool()
    X, Y, Z = nx + 1, ny + 1, nz + 1
    pec = {"ex": p[1:, 0:Y, 0:Z] | p[1:, 1:, 0:Z] | p[1:, 0:Y, 1:] | p[1:, 1:, 1:],
           "ey": p[0:X, 1:Y + 1, 0:Z] | p[1:, 1:Y + 1, 0:Z] | p[0:X, 1:Y + 1, 1:] | p[1:, 1:Y + 1, 1:],
           "ez": p[0:X, 0:Y, 1:Z + 1] | p[1:, 0:Y, 1:Z + 1] | p[0:X, 1:, 1:Z + 1] | p[1:, 1:, 1:Z + 1]}
    del p
    v = {"ex": case.dx / (case.dy * case.dz), "ey": case.dy / (case.dx * case.dz),
         "ez": case.dz / (case.dx * case.dy)}
    v.update({"hx": v["ex"], "hy": v["ey"], "hz": v["ez"]})
    mat = {}
    for c, k in enumerate(tete.KEYS):
        a = torch.full((X, Y, Z), scale * v[k], device="cuda", dtype=td)
        if graded:
            kk = torch.arange(Z, device="cuda", dtype=torch.float64)[None, None, :]
            ii = torch.arange(X, device="cuda", dtype=torch.float64)[:, None, None]
            a *= (1.0 + 0.05 * torch.sin(0.013 * kk + 0.007 * ii + c)).to(td)
        if k in pec:
            a.masked_fill_(pec[k], 0.0)
        mat[k] = a
    del pec
    return mat, [scale * v[k] for k in tete.KEYS]


def materials_section(case, precision, explicit_ms_per_step, steps=6):
    """Per-entry materials on the large workload: kappa and mu 0.9 of their
    vacuum values, kappa zero on the staircase PEC edges.  Kernel time per
    step of (1) the per-entry arrays (tete_set_materials) with the fused
    materials step, single steps reading six coefficient arrays besides the
    fields (73 B per entry in FP32, 145 in FP64), and with the two-kernel step;
    (2) the same values as one material class (tete_set_material_classes):
    paired steps run the two-step kernel's class instance, reading one class
    byte per entry and the class table from LDS (one read and one write of
    the state per two steps); (3) the arrays of (1) with the default tuning,
    which finds their few tuples as classes and runs as (2); (4) a graded
    medium with far more tuples than classes, by default (FP32: the two-step
    kernel's arrays instance, six arrays read with the fields once per two
    steps) and by the materials step.  The fields of (1), (2) and (3) are the
    same, and those of (4) by either kernel (tests).  With (2) also the
    time per step with an energy sample before every step, inside the paired
    launches and with single steps."""
    import torch
    from paper_0901_1053_amd import tete
    mat, table = _pec_materials(case, precision)
    out = {}
    G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=precision,
                  materials=True)
    G.set_pec_cells(case.cell_mask())
    G.set_materials(mat, dtype=precision)
    del mat
    torch.cuda.empty_cache()
    for kernel in ("fused", "split"):
        G.set_tuning(kernel)
        G.step(2)
        G.set_timing(steps)
        G.step(steps)
        a, b, n = G.timing()
        G.set_timing(0)
        out[kernel] = (a + b) / n
    # the default: the library found the arrays' few tuples as classes
    G.set_tuning("auto")
    auto_kernel = G.get_tuning()["kernel"]
    G.step(2)
    G.set_timing(2 * steps)
    G.step(2 * steps)
    a, b, n = G.timing()
    G.set_timing(0)
    out["auto"] = (a + b) / n
    G.close()
    del G
    torch.cuda.empty_cache()
    C = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=precision,
                  materials=True)
    C.set_pec_cells(case.cell_mask())
    C.set_material_classes(torch.zeros(C.shape, dtype=torch.uint8, device="cuda"), [table])
    kernel = C.get_tuning()["kernel"]
    C.step(2)
    C.set_timing(2 * steps)
    C.step(2 * steps)
    a, _, n = C.timing()
    C.set_timing(0)
    out["classes"] = a / n
    # an energy sample before every step: taken inside the paired launches,
    # against single steps with the energy kernel; HIP events around the
    # steps on the grid's stream
    for name, kn in (("classes_energy", "auto"), ("classes_energy_single", "fused")):
        C.set_tuning(kn)
        C.set_diagnostics(1)
        C.step(2)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(C.stream)
        C.step(steps)
        e1.record(C.stream)
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
        C.set_diagnostics(0)
    C.close()
    del C
    torch.cuda.empty_cache()
    # (4) a graded medium (no classes): the arrays instance of the two-step
    # kernel (FP32) against the materials step
    mat, _ = _pec_materials(case, precision, graded=True)
    D = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=precision,
                  materials=True)
    D.set_pec_cells(case.cell_mask())
    D.set_materials(mat, dtype=precision)
    del mat
    torch.cuda.empty_cache()
    graded_kernel = D.get_tuning()["kernel"]
    for kn in ("auto", "fused"):
        D.set_tuning(kn)
        D.step(2)
        D.set_timing(2 * steps)
        D.step(2 * steps)
        a, b2, n = D.timing()
        D.set_timing(0)
        out["graded_" + kn] = (a + b2) / n
    D.close()
    del D
    torch.cuda.empty_cache()
    b = 4 if precision == "fp32" else 8
    entries = (case.nx + 1) * (case.ny + 1) * (case.nz + 1)
    nbytes = (18 * b + 1) * entries
    return {"workload": case.name, "precision": precision,
            "materials": "0.9 x vacuum kappa and mu per entry, kappa 0 on the staircase PEC edges",
            "ms_per_step": {"fused_materials": round(out["fused"], 3), "two_kernel": round(out["split"], 3),
                            "classes_two_step": round(out["classes"], 3),
                            "classes_energy_every_step": round(out["classes_energy"], 3),
                            "classes_energy_every_step_single_steps": round(out["classes_energy_single"], 3),
                            "arrays_default": round(out["auto"], 3),
                            "graded_arrays_default": round(out["graded_auto"], 3),
                            "graded_arrays_materials_step": round(out["graded_fused"], 3)},
            "graded_arrays": "each value also times 1 + 0.05 sin(0.013 k + 0.007 i + c): no classes; the default "
                             "kernel is %s" % graded_kernel,
            "classes_kernel": kernel,
            "arrays_default_kernel": auto_kernel + (" (classes found in the arrays)" if auto_kernel == "fused2" else ""),
            "fused_materials_gbps_algorithmic": round(nbytes / (out["fused"] / 1e3) / 1e9, 1),
            "classes_vs_fused_materials": round(out["fused"] / out["classes"], 2),
            "vs_vacuum_two_step": round(out["fused"] / explicit_ms_per_step, 2) if explicit_ms_per_step else None,
            "classes_vs_vacuum_two_step": round(out["classes"] / explicit_ms_per_step, 2)
            if explicit_ms_per_step else None}


def skip_section(case, precision, explicit_ms_per_step, witness_ms=None, steps=8, xchunks=(0, 257, 128, 64, 16)):
    """The two-step kernel leaving out tiles that lie wholly in PEC
    (skip_static) on the large workload, for the default x-chunk of such grids
    (32 planes), the full step's (257) and a few others (short chunks find
    more tiles wholly in the metal block around the pipe, each chunk re-reads
    seven halo planes): kernel time per step, tiles left out, and the ratio
    to the full two-step step.  Fields and wake are those
    of the full step (the skip tests); the headline counts every tile."""
    import torch
    from paper_0901_1053_amd import tete
    G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=precision,
                  skip_static=True)
    G.set_pec_cells(case.cell_mask())
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    rows = []
    for xc in xchunks:
        G.set_tuning("fused2", 0, xc)
        G.step(4)
        G.set_timing(steps)
        G.step(steps)
        a, b, n = G.timing()
        G.set_timing(0)
        ms = (a + b) / n
        sk, tot = G.static_tiles()
        rows.append({"xchunk": xc or "default (32)", "tiles": tot, "static_tiles": sk,
                     "ms_per_step": round(ms, 3),
                     "speedup_vs_full_step": round(explicit_ms_per_step / ms, 2) if explicit_ms_per_step else None})
    # the same grid with the witness node of the witness timing (32 cells off
    # the bunch line in x), default x-chunk: whole launches with the line kernel
    G.set_tuning("fused2", 0, 0)
    wit = witness_section(G, case, explicit_ms_per_step, steps=steps)
    G.close()
    del G
    torch.cuda.empty_cache()
    return {"workload": case.name, "precision": precision, "runs": rows,
            "witness": {"offset_cells": wit["witness_offset_cells"], "ms_per_step": wit["ms_per_step"],
                        "speedup_vs_full_step_with_witness":
                            round(witness_ms / wit["ms_per_step"], 2) if witness_ms else None}}


def materials_skip_section(case, precision, steps=6):
    """Per-entry materials that carry the workload's geometry (kappa and mu
    0.9 of their vacuum values, kappa zero on the staircase PEC edges).
    Kernel time per step of the fused materials step over every tile and over
    the active tiles only (skip_static); the fields are the same."""
    import torch
    from paper_0901_1053_amd import tete
    nx, ny, nz = case.nx, case.ny, case.nz
    mat, _ = _pec_materials(case, precision)
    out = {}
    for skip in (False, True):
        G = tete.Grid(nx, ny, nz, case.dx, case.dy, case.dz, case.cdt, precision=precision, materials=True,
                      skip_static=skip)
        G.set_materials(mat, dtype=precision)
        G.step(2)
        G.set_timing(steps)
        G.step(steps)
        a, b, n = G.timing()
        G.set_timing(0)
        out[skip] = (a + b) / n
        if skip:
            out["tiles"] = G.static_tiles()
        G.close()
        del G
        torch.cuda.empty_cache()
    del mat
    torch.cuda.empty_cache()
    return {"workload": case.name, "precision": precision,
            "materials": "0.9 x vacuum kappa and mu, kappa 0 on the staircase PEC edges",
            "ms_per_step": {"all_tiles": round(out[False], 3), "active_tiles": round(out[True], 3)},
            "static_tiles": out["tiles"][0], "tiles": out["tiles"][1],
            "speedup": round(out[False] / out[True], 2)}


def implicit_section(case, precision, explicit_ms_per_step, steps=4):
    """The implicit TE/TM scheme (16) on the large workload: kernel time per step
    (HIP events around the two half steps on the grid's stream), the Chebyshev
    iterations of each plane solve, and the time per step against the explicit
    two-step kernel's."""
    import math
    from paper_0901_1053_amd import tete
    G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=precision, implicit=True)
    G.set_pec_cells(case.cell_mask())
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.step(1)
    G.set_timing(steps)
    G.step(steps)
    ms_u, ms_v, n = G.timing()
    G.set_timing(0)
    G.close()
    a = 0.5 * case.cdt
    lmax = 1.0 + a * a * (4.0 / case.dx ** 2 + 4.0 / case.dy ** 2)
    rho = (math.sqrt(lmax) - 1.0) / (math.sqrt(lmax) + 1.0)
    iters = max(1, math.ceil(math.log((1e-8 if precision == "fp32" else 1e-17) / 2.0) / math.log(rho)))
    ms = (ms_u + ms_v) / n
    return {"workload": case.name, "precision": precision, "ms_per_step": round(ms, 3),
            "ms_per_half_step": {"u": round(ms_u / n, 3), "v": round(ms_v / n, 3)},
            "chebyshev_iterations_per_plane_solve": iters, "spectral_bound": round(lmax, 4),
            "vs_explicit_two_step": round(ms / explicit_ms_per_step, 2) if explicit_ms_per_step else None}


def open_pipes_section(sw, w_closed):
    """The single-wake workload between open pipes (tete_set_open_pipes): the
    bunch starts with its own field one plane before the collimator, and the
    wake quadrature ends where no reflection from the exit wall reaches any
    sample.  Set-up (the cross-section's potential by conjugate gradients and
    the state) and solve times, and the difference from the closed box's wake,
    which includes the entrance and exit wall transitions."""
    import numpy as np
    import torch
    from paper_0901_1053_amd import tete
    kst = int(round(sw.geometry["z0"] / sw.dz))          # first plane of the collimator
    jmax = sw.jmin + sw.nw - 1
    n0 = kst - 1
    kend = sw.nz - (sw.M + jmax + 3) // 2
    steps = kend + sw.M + jmax - n0
    res = {"start_step": n0, "kend": kend, "steps": steps,
           "exact_samples": "j < %d (entrance cut) and j <= %d (exit); beyond the first, at the level of the "
                            "truncated bunch's alternating charge sum" % (n0 - sw.M - 1, 2 * (sw.nz - kend) - sw.M - 2)}
    W = {}
    for prec in ("fp64", "fp32"):
        S = tete.Grid(sw.nx, sw.ny, sw.nz, sw.dx, sw.dy, sw.dz, sw.cdt, precision=prec)
        S.set_pec_cells(sw.cell_mask())
        S.set_bunch(sw.Q, sw.sigma, sw.i0, sw.j0, sw.M, sw.jmin, sw.nw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = S.set_open_pipes(n0, kend)
        t1 = time.perf_counter()
        S.step(steps)
        W[prec] = S.wake()
        t2 = time.perf_counter()
        res[prec] = {"setup_ms": round((t1 - t0) * 1e3, 2), "cg_iterations": it, "solve_s": round(t2 - t1, 4),
                     "gcell_updates_per_s": round(sw.cells * steps / (t2 - t1) / 1e9, 2)}
        del S
        torch.cuda.empty_cache()
    rng = float(np.max(w_closed) - np.min(w_closed))
    res["fp32_delta_vs_fp64_gpu"] = float(np.max(np.abs(W["fp32"] - W["fp64"])) / (np.max(W["fp64"]) - np.min(W["fp64"])))
    res["closed_box_minus_open_over_closed_range"] = float(np.max(np.abs(w_closed - W["fp64"])) / rng)
    res["W_range_V_per_C"] = {"open": float(np.ptp(W["fp64"])), "closed": rng}
    return res


def rz_section(steps=100, warmup=5):
    """The rotationally symmetric scheme (24) on the deflector-like r-z workload
    at harmonic m = 1: kernel time per step in FP32 and FP64 (HIP events on the
    grid's stream around each launch), Gcell-updates/s and the HBM roofline of
    k_rz (read and write six components plus the code byte per node), and the
    stable step against Yee's at the same m from the paper's bounds."""
    import torch
    from paper_0901_1053_amd import inputs, tete
    case = inputs.tds_case(1)
    cells = case.cells()
    jmin, nw = case.window()
    res = {"workload": case.name, "grid": [case.nr, case.nz], "cells": case.nr * case.nz, "mode": case.mode,
           "dr_m": case.dr, "dz_m": case.dz, "sigma_m": case.sigma, "steps_per_solve": case.steps()}
    for prec in ("fp32", "fp64"):
        G = tete.RZGrid(case.nr, case.nz, case.dr, case.dz, case.cdt, case.mode, prec)
        G.set_pec_cells(cells)
        G.set_bunch(case.charge, case.sigma, case.j0, case.M, case.jw, jmin, nw)
        G.step(warmup)
        G.set_timing(steps)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(G.stream)
        G.step(steps)
        e1.record(G.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kms, n, nst = G.timing()
        G.set_timing(0)
        b = 4 if prec == "fp32" else 8
        per = nst // n                                   # steps per launch (two-step kernel: 2)
        kbytes = (12 * b + 1) * G.np * per               # one cell-update per entry and step
        achieved = kbytes / (kms / n / 1e3) / 1e9
        traffic = measured_traffic("k_rz", case.name, prec)
        res[prec] = {"gcell_updates_per_s": round(case.nr * case.nz * steps / (ms / 1e3) / 1e9, 2),
                     "ms_per_step": round(ms / steps, 4),
                     "roofline": {"bound": "hbm", "kernel": "k_rz", "steps_per_launch": per,
                                  "achieved": round(achieved, 1),
                                  "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                  "frac": round(achieved / PEAK_HBM_GBPS, 4), "bytes_per_launch": kbytes,
                                  "basis": "algorithmic bytes of %d single steps per launch; the two-step launch "
                                           "reads and writes the state once, so frac can exceed 1: it is not a "
                                           "bandwidth fraction, traffic_frac is" % per,
                                  "ms_per_launch": round(kms / n, 4), "traffic": traffic,
                                  "traffic_gbps": round(traffic / (kms / n / 1e3) / 1e9, 1) if traffic else None,
                                  "traffic_frac": round(traffic / (kms / n / 1e3) / 1e9 / PEAK_HBM_GBPS, 4)
                                  if traffic else None},
                     "solve_s_estimate": round(ms / steps * case.steps() / 1e3, 2)}
        G.close()
        del G
        torch.cuda.empty_cache()
    m = case.mode
    yee = 1.0 / ((1.2 + 0.4 * m * m) / case.dr ** 2 + 1.2 / case.dz ** 2) ** 0.5
    res["stable_step_vs_yee"] = {"te_tm_dtau_over_dz": 1.0, "yee_bound_over_dz": round(yee / case.dz, 4),
                                 "steps_ratio_yee_over_te_tm": round(case.dz / yee, 3)}
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single-wake", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "fused2", "split"])
    ap.add_argument("--rows", type=int, default=0, help="fused kernel: rows per workgroup (12 or 16)")
    ap.add_argument("--xchunk", type=int, default=0, help="fused kernel: x-planes per workgroup (0: auto)")
    ap.add_argument("--depth", type=int, default=0, help="fused kernel: planes prefetched ahead (1..3)")
    ap.add_argument("--order", type=int, default=0, help="fused kernels: tile order (1..6; 0: library default)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-yee", action="store_true", help="skip the comparison with Yee's scheme")
    ap.add_argument("--no-rz", action="store_true", help="skip the rotationally symmetric workload")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit scheme (16) comparison")
    ap.add_argument("--no-witness", action="store_true", help="skip the off-axis witness timing")
    ap.add_argument("--no-materials", action="store_true", help="skip the per-entry materials timing")
    ap.add_argument("--no-skip", action="store_true", help="skip the static-tile skip timing")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape table of the headline grid")
    ap.add_argument("--no-pipes", action="store_true", help="skip the open-pipe single wake")
    ap.add_argument("--no-diag", action="store_true", help="skip the energy-every-step timing")
    ap.add_argument("--batched-count", type=int, default=64)
    ap.add_argument("--serve-rates", default="1,10,50,200", help="comma-separated request rates (req/s)")
    ap.add_argument("--serve-requests", type=int, default=48)
    ap.add_argument("--serve-max-cells", type=float, default=2 ** 28,
                    help="serving: grid cells in flight at most (0: no limit)")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="only run tete_stream_probe over six arrays of this many GiB each, 5 times (HBM "
                         "counter calibration: reads 6 x GIB + the code bytes, writes 6 x GIB per launch)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0901_1053_amd import inputs, tete

    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * 2 ** 30) // 4
        src = [torch.ones(n, dtype=torch.float32, device="cuda") for _ in range(6)]
        dst = [torch.empty_like(src[0]) for _ in range(6)]
        code = torch.zeros(n, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        for _ in range(5):
            tete.stream_probe(src, dst, code)
        torch.cuda.synchronize()
        assert torch.equal(dst[3], src[3])
        print(json.dumps({"calibration": "k_stream", "bytes_read_per_launch": 6 * 4 * n + n,
                          "bytes_written_per_launch": 6 * 4 * n}))
        return

    case = inputs.large_case()
    print("# workload %s, %s, steps %d, warmup %d" % (case.name, args.precision, args.steps, args.warmup),
          file=sys.stderr, flush=True)
    G = tete.Grid(case.nx, case.ny, case.nz, case.dx, case.dy, case.dz, case.cdt, precision=args.precision)
    G.set_pec_cells(case.cell_mask())
    G.set_bunch(case.Q, case.sigma, case.i0, case.j0, case.M, case.jmin, case.nw)
    G.set_tuning(args.kernel, args.rows, args.xchunk, args.depth, args.order)
    tuning = G.get_tuning()
    G.step(args.warmup)
    torch.cuda.synchronize()

    K = args.steps
    G.set_timing(K)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(G.stream)
    G.step(K)
    e1.record(G.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_tm, ms_te, nt = G.timing()
    G.set_timing(0)
    print("# timed %d steps in %.2f ms" % (K, ms), file=sys.stderr, flush=True)

    cells = case.cells
    entries = G.np
    b = 4 if args.precision == "fp32" else 8
    ms_step = ms / K
    value = cells * K / (ms / 1e3) / 1e9
    step_bytes = (12 * b + 1) * entries        # read + write six components, PEC code
    if tuning["kernel"] == "fused":
        kern = {"fused": ms_tm / nt}
        dom = "fused"
        kbytes = step_bytes                    # one launch per step
    elif tuning["kernel"] == "fused2":
        kern = {"fused2": 2 * ms_tm / nt}      # nt counts steps; one launch takes two
        dom = "fused2"
        kbytes = 2 * step_bytes                # two cell-updates per entry per launch
    else:
        kern = {"tm": ms_tm / nt, "te": ms_te / nt}
        dom = max(kern, key=kern.get)
        kbytes = (8 * b + 1) * entries         # each half reads five arrays + code, writes three
    achieved = kbytes / (kern[dom] / 1e3) / 1e9
    traffic = measured_traffic("k_" + dom, case.name, args.precision)
    traffic_gbps = traffic / (kern[dom] / 1e3) / 1e9 if traffic else None
    ceiling = copy_ceiling(entries, args.precision)
    print("# copy ceiling %.1f GB/s" % ceiling["gbps"], file=sys.stderr, flush=True)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": cells, "grid_entries": entries,
                   "fields": args.precision, "wake_accumulation": "fp64",
                   "geometry": "tapered round aperture in 20 mm square pipe, 10 deg, 2->10 mm diameter",
                   "bunch_sigma_m": case.sigma, "cdt_over_dz": 1.0, "dx_over_dz": 2.0,
                   "kernel": tuning},
        "hbm_gbps_algorithmic": round(step_bytes / (ms_step / 1e3) / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": "k_" + dom, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBPS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "basis": "algorithmic bytes: 12 b + 1 = %d B per grid entry per time step, %d step(s) per "
                              "launch; a launch of the two-step kernel reads and writes the state once, so it "
                              "moves about half of these bytes and frac can exceed what its DRAM traffic does"
                              % (12 * b + 1, kbytes // step_bytes),
                     "traffic": traffic,
                     "traffic_gbps": round(traffic_gbps, 1) if traffic else None,
                     "traffic_frac": round(traffic_gbps / PEAK_HBM_GBPS, 4) if traffic else None,
                     "copy_ceiling_gbps": ceiling["gbps"],
                     "traffic_vs_copy_ceiling": round(traffic_gbps / ceiling["gbps"], 4) if traffic else None,
                     "bytes_per_launch": kbytes, "ms_per_launch": round(kern[dom], 4),
                     "kernels_ms_per_launch": {k: round(v, 4) for k, v in kern.items()}},
        "copy_ceiling": ceiling,
        "paper_context": {"updates_per_step": {"explicit_te_tm": 10, "yee": 6},
                          "cost_per_step_vs_yee": round(10 / 6, 3),
                          "run_time_vs_yee_at_dx_sqrt2_dz": round((10 / 6) / 2 ** 0.5, 3),
                          "hardware": "not stated in the paper", "timings": "none reported"},
    }
    if not args.no_tune:
        out["single_grid_tuning"] = single_grid_tuning(G)
        print("# single-grid tuning done", file=sys.stderr, flush=True)
    if not args.no_yee:
        out["yee_context"] = yee_section(G, case, args.precision)
        print("# yee comparison done", file=sys.stderr, flush=True)
    if not args.no_witness:
        out["witness_context"] = witness_section(G, case, ms_step)
        print("# witness timing done", file=sys.stderr, flush=True)
    if not args.no_diag:
        out["diagnostics_context"] = diagnostics_section(G, case, ms_step)
        print("# diagnostics timing done", file=sys.stderr, flush=True)
    del G
    torch.cuda.empty_cache()
    if not args.no_implicit:
        out["implicit_context"] = implicit_section(case, args.precision, ms_step)
        torch.cuda.empty_cache()
        print("# implicit comparison done", file=sys.stderr, flush=True)
    if not args.no_materials:
        out["materials_context"] = materials_section(case, args.precision, ms_step)
        torch.cuda.empty_cache()
        print("# materials timing done", file=sys.stderr, flush=True)
    if not args.no_skip:
        out["skip_static_context"] = skip_section(case, args.precision, ms_step,
                                                  out.get("witness_context", {}).get("ms_per_step"))
        if not args.no_materials:
            out["skip_static_context"]["materials"] = materials_skip_section(case, args.precision)
        torch.cuda.empty_cache()
        print("# static-tile skip timing done", file=sys.stderr, flush=True)

    if not args.no_single_wake:
        sw = inputs.single_wake_case()
        res = {}
        for prec in ("fp64", "fp32"):
            S = tete.Grid(sw.nx, sw.ny, sw.nz, sw.dx, sw.dy, sw.dz, sw.cdt, precision=prec)
            S.set_pec_cells(sw.cell_mask())
            S.set_bunch(sw.Q, sw.sigma, sw.i0, sw.j0, sw.M, sw.jmin, sw.nw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.step(sw.steps)
            W = S.wake()
            dt = time.perf_counter() - t0
            res[prec] = {"solve_s": round(dt, 4), "gcell_updates_per_s": round(sw.cells * sw.steps / dt / 1e9, 2)}
            res[prec + "_W"] = W
            del S
            torch.cuda.empty_cache()
        import numpy as np
        w64, w32 = res.pop("fp64_W"), res.pop("fp32_W")
        res["fp32_delta_vs_fp64_gpu"] = float(np.max(np.abs(w32 - w64)) / (np.max(w64) - np.min(w64)))
        res["workload"] = sw.name
        res["steps"] = sw.steps
        out["single_wake"] = res
        print("# single wake done", file=sys.stderr, flush=True)
        if not args.no_pipes:
            out["open_pipes"] = open_pipes_section(sw, w64)
            print("# open pipes done", file=sys.stderr, flush=True)

    if not args.no_rz:
        out["rz"] = rz_section()
        print("# rz done", file=sys.stderr, flush=True)

    if not args.no_batched:
        out["batched"] = batched_section(args.batched_count)
        print("# batched done", file=sys.stderr, flush=True)
    if not args.no_serve:
        out["serve"] = serve_section([float(r) for r in args.serve_rates.split(",")], args.serve_requests,
                                     int(args.serve_max_cells) or None)
        print("# serve done", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        fp64 = gpu_fp64_rate(case) if args.precision == "fp32" else round(value, 2)
        out["cpu_baseline"] = cpu_baseline(case, fp64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
