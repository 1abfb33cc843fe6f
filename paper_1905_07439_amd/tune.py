"""Autotuner: recursion depth and leaf tile per (shape, scheme, precision), from timed trials.

For C = A B (A is M x K, B is K x N) with one scheme at every level, the
candidates are the depths Q whose leaves lie in [min_leaf, max_leaf] and, for
each, the leaf tiles of the precision that pad a leaf side by at most a
quarter.  Every candidate plan runs ``reps`` products on the device (timed
with HIP events after one warm-up) and the fastest is kept.  Choices are cached
in memory and, with ``path``, in a JSON file keyed by device, shape, scheme
name and precision, so a later process reuses them without trials.

The choice changes how the product is computed (how many levels of the
randomized scheme are applied, and the leaf GEMM's tiling), not what a given
plan computes: a plan built from a cached choice is the same plan as one built
by hand with those parameters.
"""

import json
import math
import os

TILES = {"f64": (16,), "f32": (64, 128), "bf16x3": (64, 128), "f16s": (32, 64, 96, 128),
         "fp8c": (32, 64, 96, 128)}


def _ceil_div(a, b):
    return -(-a // b)


class Tuner:
    def __init__(self, path=None, reps=3, min_leaf=48, max_leaf=1024, max_pad=1.25, device="cuda:0"):
        self.path = path
        self.reps = reps
        self.min_leaf, self.max_leaf, self.max_pad = min_leaf, max_leaf, max_pad
        self.device = device
        self.cache = {}
        self.trials = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)

    def _device_name(self):
        import torch
        return torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]

    def key(self, M, K, N, name, prec):
        return "%s|%d,%d,%d|%s|%s" % (self._device_name(), M, K, N, name, prec)

    def candidates(self, M, K, N, scheme, prec, tiles=True):
        """[(Q, tile)] to try: leaves within [min_leaf, max_leaf], tiles padding a leaf side by at
        most max_pad (tile 0: the library's own choice, always included; the only one when
        ``tiles`` is false)."""
        i = scheme.info()
        b1, b2, b3 = i["b1"], i["b2"], i["b3"]
        out = []
        for q in range(1, 16):
            lm, lk, ln = _ceil_div(M, b1 ** q), _ceil_div(K, b2 ** q), _ceil_div(N, b3 ** q)
            if max(lm, lk, ln) < self.min_leaf:
                break
            if min(lm, lk, ln) < self.min_leaf // 2 or max(lm, lk, ln) > self.max_leaf:
                continue
            out.append((q, 0))
            for t in TILES[prec] if tiles else ():
                if _ceil_div(lm, t) * t <= self.max_pad * lm and _ceil_div(ln, t) * t <= self.max_pad * ln:
                    out.append((q, t))
        if not out:  # nothing in range: the depth whose leaf side is closest to the range
            q = max(1, int(round(math.log(max(M, K, N) / float(self.max_leaf), max(b1, b2, b3)))))
            out.append((q, 0))
        return out

    def _time(self, plan, A, B, C, ws):
        import torch
        plan.matmul(A, B, C=C, seed=1, workspace=ws)
        s = torch.cuda.current_stream(self.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for r in range(self.reps):
            plan.matmul(A, B, C=C, seed=r, workspace=ws)
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / self.reps

    def choose(self, M, K, N, scheme, prec, name, tiles=True):
        """{"levels": Q, "tile": t, "ms": ...} for this shape, scheme (``name`` keys the cache)."""
        k = self.key(M, K, N, name, prec) + ("" if tiles else "|depth")
        if k in self.cache:
            return self.cache[k]
        import torch
        import paper_1905_07439_amd as rbc
        dt = torch.float64 if prec == "f64" else torch.float32
        g = torch.Generator(device=self.device)
        g.manual_seed(12345)
        A = torch.randn(M, K, device=self.device, dtype=dt, generator=g)
        B = torch.randn(K, N, device=self.device, dtype=dt, generator=g)
        C = torch.empty(M, N, device=self.device, dtype=dt)
        best, tried = None, []
        for q, t in self.candidates(M, K, N, scheme, prec, tiles):
            try:
                plan = rbc.Plan(M, K, N, [scheme] * q, prec=prec, leaf_tile=t)
            except rbc.RbcError:
                continue
            tile = plan.info["tile_m"]
            if any(x["levels"] == q and x["tile"] == tile for x in tried):
                continue  # tile 0 resolved to a tile already tried
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=self.device)
            ms = self._time(plan, A, B, C, ws)
            tried.append({"levels": q, "tile": tile, "ms": ms})
            if best is None or ms < best["ms"]:
                best = {"levels": q, "tile": tile, "ms": ms}
            del plan, ws
        if best is None:
            raise RuntimeError("no candidate plan for %s" % k)
        self.trials[k] = tried
        self.cache[k] = best
        if self.path:
            self.save()
        return best

    def depth_for(self, n, scheme, prec, name, grid=(256, 512, 1024, 2048, 4096)):
        """Recursion depth for an n x n x n product without trials at n: the depth is tuned (with
        the library's tile choice) at the grid size nearest to n on a log scale, and n gets the
        depth whose leaf side is nearest, on a log scale, to the leaf side chosen there."""
        g = min(grid, key=lambda x: abs(math.log(x / float(n))))
        q_g = self.choose(g, g, g, scheme, prec, name, tiles=False)["levels"]
        b = scheme.info()["b1"]
        leaf = g / float(b ** q_g)
        q = max(1, int(round(math.log(n / leaf, b))))
        while q > 1 and _ceil_div(n, b ** q) < self.min_leaf // 2:
            q -= 1
        return q

    def plan(self, M, K, N, scheme, prec, name):
        import paper_1905_07439_amd as rbc
        c = self.choose(M, K, N, scheme, prec, name)
        return rbc.Plan(M, K, N, [scheme] * c["levels"], prec=prec, leaf_tile=c["tile"])

    def save(self):
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
