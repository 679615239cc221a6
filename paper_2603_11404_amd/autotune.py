"""Workgroup-size autotuner for batched launches.

A problem's raster workgroup size (256, 512 or 1024 threads; bounded by the
LDS its image mask and the per-wave task queues need) changes speed, never
results.  The tuner times the ask-eval launch of a problem at every feasible
size and caches the fastest per (device, resolution, population, triangle
count bucket) in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import tk

SIZES = (1024, 512, 256)


class Autotuner:
    def __init__(self, path: str | None = None, reps: int = 3):
        self.path = path
        self.reps = reps
        self.cache: dict[str, int] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = {k: int(v) for k, v in json.load(f).items()}

    @staticmethod
    def key(gen) -> str:
        p = gen.p
        tri = sum(m.n_triangles for m in p.meshes)
        dev = torch.cuda.get_device_name(p.device)
        return f"{dev}|{p.cam.width}x{p.cam.height}|arms{p.n_arms}|lam{gen.lam}|tri2^{int(math.log2(max(tri, 1)))}"

    def _time(self, gen, threads: int) -> float | None:
        try:
            b = tk.Batch([gen.problem_struct(threads=threads)], device=gen.p.device)
        except tk.TkError as e:
            if e.status == tk.TK_ERR_UNSUPPORTED:
                return None
            raise
        b.ask_eval()                                  # warm-up (draws are unchanged: no update runs)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(self.reps):
            b.ask_eval()
        ev[1].record()
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / self.reps

    def choose(self, gen) -> int:
        """Workgroup size for this generation's problem (measured once per key)."""
        k = self.key(gen)
        if k not in self.cache:
            times = {t: self._time(gen, t) for t in SIZES}
            times = {t: v for t, v in times.items() if v is not None}
            self.cache[k] = min(times, key=times.get)
            self.save()
        return self.cache[k]

    def save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
