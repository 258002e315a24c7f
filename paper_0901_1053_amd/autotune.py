"""Launch-shape autotuner for the fused step.

For a grid size class it times the fused kernel over candidate launch shapes
(x-planes per workgroup, tile order, and for single-grid stepping also rows per
workgroup and prefetch depth) with the library's live HIP-event timing, and
caches the fastest shape per class in a JSON file.  Tuning changes only the
launch shape, never the results (every shape gives bitwise the same fields).
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


class Tuner:
    def __init__(self, cache_path: str | None = DEFAULT_CACHE, xchunks=(0, 16, 32, 64, 128), orders=(1, 2),
                 rows=(0,), depths=(0,), steps=6, warmup=2):
        self.cache_path = cache_path
        self.xchunks, self.orders, self.rows, self.depths = xchunks, orders, rows, depths
        self.steps, self.warmup = steps, warmup
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
        G = tete.Grid(nx, ny, nz, dx, dy, dz, cdt, precision=precision)
        G.set_tuning("fused", shape.rows, shape.xchunk, shape.depth, shape.order)
        G.step(self.warmup)
        G.set_timing(self.steps)
        G.step(self.steps)
        ms, _, n = G.timing()
        G.close()
        return ms / max(n, 1)

    def tune(self, nx, ny, nz, dx, dy, dz, cdt, precision="fp32", force=False) -> Shape:
        key = size_class(nx, ny, nz, precision)
        if not force and key in self.cache:
            return Shape(**self.cache[key])
        best = None
        for cand in self.candidates():
            cand.ms = self.measure(nx, ny, nz, dx, dy, dz, cdt, precision, cand)
            if best is None or cand.ms < best.ms:
                best = cand
        self.cache[key] = best.as_dict()
        self.save()
        return best

    def lookup(self, nx, ny, nz, precision) -> Shape | None:
        v = self.cache.get(size_class(nx, ny, nz, precision))
        return Shape(**v) if v else None
