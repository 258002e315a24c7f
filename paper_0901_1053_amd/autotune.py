"""Launch-shape autotuner for the fused steps.

For a grid size class it times one kernel (the fused single step, or the
two-step kernel that FP32 batches run) over candidate launch shapes (x-planes
per workgroup, tile order, and for single-grid stepping also rows per
workgroup and prefetch depth) with the library's live HIP-event timing, and
caches the fastest shape per class and kernel in a JSON file.  With batch = N
each shape is timed on N copies of the grid stepped as one batch, the context
batch members run in (there the instances already fill the GPU, and shorter
x-chunks only add halo planes).  Tuning changes
only the launch shape, never the results (every shape gives bitwise the same
fields).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "tete", "autotune.json")


def size_class(nx: int, ny: int, nz: int, precision: str) -> str:
    """Grids whose dimensions round to the same powers of two share a shape."""
    def b(n):
        return 1 << max(0, (n - 1).bit_length())
    return "%s:%dx%dx%d" % (precision, b(nx), b(ny), b(nz))


@dataclass
class Shape:
    xchunk: int = 0
    order: int = 0
    rows: int = 0
    depth: int = 0
    ms: float = float("nan")

    def as_dict(self):
        return {"xchunk": self.xchunk, "order": self.order, "rows": self.rows, "depth": self.depth, "ms": self.ms}

    @classmethod
    def from_dict(cls, d):
        return cls(**{k: d[k] for k in ("xchunk", "order", "rows", "depth", "ms") if k in d})

    def key(self):
        return (self.xchunk, self.order, self.rows, self.depth)


class Tuner:
    def __init__(self, cache_path: str | None = DEFAULT_CACHE, xchunks=(0, 16, 32, 64, 128), orders=(1, 2),
                 rows=(0,), depths=(0,), steps=6, warmup=2, kernel="fused", batch=0):
        if kernel not in ("fused", "fused2"):
            raise ValueError("the tuner times the fused single step or the two-step kernel")
        self.kernel = kernel
        self.batch = batch
        self.cache_path = cache_path
        self.xchunks, self.orders, self.rows, self.depths = xchunks, orders, rows, depths
        self.steps, self.warmup = steps, warmup
        # ms per step of every candidate timed for the last class tuned (or
        # read from the cache), keyed by (xchunk, order, rows, depth)
        self.timed = {}
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            try:
                with open(cache_path) as fh:
                    self.cache = json.load(fh)
            except (OSError, ValueError):
                self.cache = {}

    def save(self):
        if not self.cache_path:
            return
        os.makedirs(os.path.dirname(self.cache_path), exist_ok=True)
        tmp = self.cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def candidates(self):
        for r in self.rows:
            for d in self.depths:
                for o in self.orders:
                    for x in self.xchunks:
                        yield Shape(xchunk=x, order=o, rows=r, depth=d)

    def measure(self, nx, ny, nz, dx, dy, dz, cdt, precision, shape: Shape) -> float:
        from . import tete
        if self.batch > 0:
            return self._measure_batch(nx, ny, nz, dx, dy, dz, cdt, precision, shape)
        G = tete.Grid(nx, ny, nz, dx, dy, dz, cdt, precision=precision)
        G.set_tuning(self.kernel, shape.rows, shape.xchunk, shape.depth, shape.order)
        G.step(self.warmup)
        G.set_timing(self.steps)
        G.step(self.steps)
        ms, _, n = G.timing()
        G.close()
        return ms / max(n, 1)

    def _measure_batch(self, nx, ny, nz, dx, dy, dz, cdt, precision, shape: Shape) -> float:
        """ms per step and instance of `batch` copies stepped as one batch
        (HIP events on the batch's stream, after which its steps are ordered)."""
        import torch

        from . import tete
        B = tete.Batch(precision)
        B.set_launch(graph_steps=max(1, self.steps))
        grids = []
        for s in range(self.batch):
            G = tete.Grid(nx, ny, nz, dx, dy, dz, cdt, precision=precision)
            G.set_tuning(self.kernel, shape.rows, shape.xchunk, shape.depth, shape.order)
            B.set(s, G)
            grids.append(G)
        B.step(self.steps)                      # warm-up (and the graph's capture)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(B.stream)
        B.step(self.steps)
        e1.record(B.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (self.steps * self.batch)
        for s in range(self.batch):
            B.set(s, None)
        B.close()
        for G in grids:
            G.close()
        return ms

    def _key(self, nx, ny, nz, precision):
        return size_class(nx, ny, nz, precision) + "/" + self.kernel + ("/batch%d" % self.batch if self.batch else "")

    def tune(self, nx, ny, nz, dx, dy, dz, cdt, precision="fp32", force=False) -> Shape:
        key = self._key(nx, ny, nz, precision)
        if not force and key in self.cache:
            ent = self.cache[key]
            self.timed = {tuple(t[:4]): t[4] for t in ent.get("timed", [])}
            return Shape.from_dict(ent)
        best = None
        self.timed = {}
        for cand in self.candidates():
            cand.ms = self.measure(nx, ny, nz, dx, dy, dz, cdt, precision, cand)
            self.timed[cand.key()] = cand.ms
            if best is None or cand.ms < best.ms:
                best = cand
        ent = best.as_dict()
        ent["timed"] = [list(k) + [v] for k, v in self.timed.items()]
        self.cache[key] = ent
        self.save()
        return best

    def lookup(self, nx, ny, nz, precision) -> Shape | None:
        v = self.cache.get(self._key(nx, ny, nz, precision))
        return Shape.from_dict(v) if v else None
