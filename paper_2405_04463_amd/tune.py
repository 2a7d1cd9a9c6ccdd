"""Autotuner for the dot-product kernel configuration.

For a given shape (rows, rotations per query) it times every candidate
configuration (`imc_set_dot_tiles` flags) on the real operands over a probe
slice of the database, keeps the fastest on the context, and remembers the
choice per (device, rows bucket, rotation count) in a JSON cache.
"""
from __future__ import annotations

import json
import os

import torch

from . import (DOT_PERSISTENT, DOT_TILES_EXPANDED_128x128, DOT_TILES_EXPANDED_256x128, DOT_TILES_EXPANDED_SHALLOW,
               DOT_TILES_ROTATION, DOT_TILES_ROTATION_DIRECT, DOT_TILES_ROTATION_LDSCOPY)

CANDIDATES_UNIFORM = [DOT_TILES_ROTATION, DOT_TILES_ROTATION_LDSCOPY, DOT_TILES_ROTATION_DIRECT,
                      DOT_TILES_EXPANDED_256x128, DOT_TILES_EXPANDED_256x128 | DOT_PERSISTENT,
                      DOT_TILES_EXPANDED_128x128, DOT_TILES_EXPANDED_SHALLOW]
CANDIDATES_ROWS = [DOT_TILES_EXPANDED_256x128, DOT_TILES_EXPANDED_256x128 | DOT_PERSISTENT,
                   DOT_TILES_EXPANDED_128x128, DOT_TILES_EXPANDED_SHALLOW]
# the fused launch of every rotation-aware group (lists of fewer rotations
# run as in the grouped mode, on the same tiles): one tile per workgroup, or
# a persistent grid
CANDIDATES_FUSED = [DOT_TILES_ROTATION, DOT_TILES_ROTATION | DOT_PERSISTENT]


def _bucket(rows: int) -> int:
    b = 32
    while b < rows:
        b *= 2
    return b


class DotTuner:
    def __init__(self, cache_path: str | None = None):
        self.cache_path = cache_path
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def key(self, rows: int, r: int) -> str:
        name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
        return f"{name}|rows<={_bucket(rows)}|r={r}"

    def tune(self, ctx, run, rows: int, r: int, candidates=None, reps: int = 2, force: bool = False):
        """`run()` enqueues the dot products of the shape on the current
        stream.  Returns (best flags, {flags: ms})."""
        k = self.key(rows, r)
        if not force and k in self.cache:
            ctx.set_dot_tiles(self.cache[k]["best"])
            return self.cache[k]["best"], self.cache[k]["ms"]
        if candidates is None:
            candidates = CANDIDATES_UNIFORM if r >= 13 else CANDIDATES_ROWS
        times = {}
        for c in candidates:
            ctx.set_dot_tiles(c)
            run()
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a, b in ev:
                a.record()
                run()
                b.record()
            torch.cuda.synchronize()
            times[c] = min(a.elapsed_time(b) for a, b in ev)
        best = min(times, key=times.get)
        ctx.set_dot_tiles(best)
        self.cache[k] = {"best": best, "ms": {str(c): t for c, t in times.items()}}
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1)
        return best, times
