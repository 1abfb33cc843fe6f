"""Serving loop: C = A B requests of mixed sizes, schemes and seeds, continuously batched.

Requests arrive over time (a Poisson process in the load generator).  The
scheduler admits waiting requests in arrival order while their HBM footprint
(A, B, C and the plan's workspace) fits the budget and an execution slot (a
HIP stream) is free, and launches everything it admitted at that moment as
one batch: one launch of the batch engine (``Batch``, persistent or
level-synchronous), or, in ``direct`` mode, the per-stage launches of each
product.  Requests that arrive
while earlier batches run are admitted as soon as memory and a slot free up;
batches on different slots overlap on the device.  A request's latency is
its completion time (from a HIP event on its slot, on the device clock) minus
its arrival time.  Every product's result is bitwise the one it has alone.

The scheduler (admission and accounting) is independent of the device and is
exercised on the CPU with a simulated executor; the GPU executor owns plans,
operands, workspaces and streams.
"""

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

SCHEMES = ("strassen", "laderman", "approx")
APPROX_LAMBDA = 1e-3


@dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the run
    n: int
    scheme: str
    seed: int
    admitted: float = math.nan
    done: float = math.nan
    footprint: int = 0
    batch: int = -1


def make_requests(rate, duration, seed, lo=128, hi=4096, quantum=32, schemes=SCHEMES):
    """Poisson arrivals at ``rate`` per second over ``duration`` seconds, N log-uniform in
    [lo, hi] rounded to a multiple of ``quantum``, scheme uniform over ``schemes``, algorithm
    seed = request index."""
    import workloads
    arrivals = workloads.poisson_arrivals(rate, duration, seed)
    n = len(arrivals)
    sizes = workloads.log_uniform_sizes(n, seed + 1, lo, hi)
    pick = np.random.default_rng(seed + 2).integers(0, len(schemes), size=n)
    out = []
    for i in range(n):
        size = int(min(hi, max(lo, quantum * round(sizes[i] / quantum))))
        out.append(Request(i, float(arrivals[i]), size, schemes[pick[i]], i))
    return out


def levels_for(n, scheme):
    """Recursion depth: leaves of about 96..256 (at least one level)."""
    if scheme == "laderman":
        q = max(1, int(round(math.log(max(n / 192.0, 1.0), 3))))
    else:
        q = max(1, int(round(math.log2(max(n / 192.0, 1.0)))))
    return [scheme] * q


class Scheduler:
    """FIFO admission under an HBM budget, at most ``max_batch`` requests per launch."""

    def __init__(self, budget_bytes, max_batch=64):
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.in_use = 0
        self.peak = 0

    def admit(self, pending, footprint):
        """Pop from the front of ``pending`` (a deque) the requests to launch now."""
        take = []
        while pending and len(take) < self.max_batch:
            r = pending[0]
            f = footprint(r)
            if f > self.budget:
                raise ValueError("request %d needs %d bytes, more than the budget" % (r.rid, f))
            if self.in_use + f > self.budget:
                break
            pending.popleft()
            r.footprint = f
            self.in_use += f
            take.append(r)
        self.peak = max(self.peak, self.in_use)
        return take

    def release(self, reqs):
        for r in reqs:
            self.in_use -= r.footprint


def serve(requests, executor, scheduler, slots=4, clock=None, idle_sleep=2e-5):
    """Run the loop until every request is done; returns the statistics (see ``summarize``).

    ``clock``: None for real time (``time.perf_counter``); a simulated clock (with
    ``now()`` and ``advance_to(t)``) lets the CPU tests drive the loop without a device.
    """
    reqs = sorted(requests, key=lambda r: r.arrival)
    real = clock is None
    t0 = time.perf_counter()
    now = (lambda: time.perf_counter() - t0) if real else clock.now
    executor.start(t0)
    pending = deque()
    inflight = []  # (handle, slot, reqs)
    free = list(range(slots))
    nxt = 0
    n_batches = 0
    while nxt < len(reqs) or pending or inflight:
        t = now()
        while nxt < len(reqs) and reqs[nxt].arrival <= t:
            pending.append(reqs[nxt])
            nxt += 1
        progressed = False
        for item in list(inflight):
            h, slot, batch = item
            done = executor.poll(h)
            if done is not None:
                for r in batch:
                    r.done = done
                scheduler.release(batch)
                executor.finish(h)
                inflight.remove(item)
                free.append(slot)
                progressed = True
        while free and pending:
            take = scheduler.admit(pending, executor.footprint)
            if not take:
                break
            slot = free.pop(0)
            for r in take:
                r.admitted = t
                r.batch = n_batches
            inflight.append((executor.launch(take, slot), slot, take))
            n_batches += 1
            progressed = True
        if not progressed:
            if real:
                if idle_sleep:
                    time.sleep(idle_sleep)
            else:
                events = [reqs[nxt].arrival] if nxt < len(reqs) else []
                events += [executor.next_done(h) for h, _, _ in inflight]
                if events:
                    clock.advance_to(max(t, min(events)))
    executor.stop()
    return summarize(reqs, scheduler, n_batches)


def summarize(reqs, scheduler, n_batches):
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    wait = np.array([r.admitted - r.arrival for r in reqs]) * 1e3
    flops = sum(2.0 * r.n ** 3 for r in reqs)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs) if reqs else 0.0
    return {
        "requests": len(reqs), "batches": n_batches,
        "mean_batch": round(len(reqs) / max(n_batches, 1), 2),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean()), "max": float(lat.max())},
        "queue_ms": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
        "effective_tflops": flops / span / 1e12 if span > 0 else 0.0,
        "span_s": span, "peak_admitted_bytes": scheduler.peak,
    }


class GpuExecutor:
    """Runs admitted requests on the GPU: operands N(0,1) generated on the device from the
    request seed (A from 2 rid + 1, B from 2 rid + 2), plans cached per (N, scheme); the
    recursion depth from ``tuner`` when given, else ``levels_for``."""

    def __init__(self, prec="fp8c", mode="batch", device="cuda:0", keep=None, engine="levels", tuner=None):
        import torch
        import paper_1905_07439_amd as rbc
        if mode not in ("batch", "direct"):
            raise ValueError("mode must be 'batch' or 'direct'")
        self.torch, self.rbc = torch, rbc
        self.prec, self.mode, self.device, self.engine = prec, mode, device, engine
        self.tuner = tuner  # paper_1905_07439_amd.tune.Tuner: depth per size from timed trials
        self.streams = {}
        self.slot_ws = {}  # slot -> workspace buffer shared by that slot's products, in stream order
        self.plans = {}
        self.keep = keep  # dict rid -> C (and operands) for requests to keep, or None
        S = rbc.Scheme.builtin("strassen")
        self.schemes = {"strassen": S, "laderman": rbc.Scheme.builtin("laderman"),
                        "approx": rbc.Scheme.builtin("perturbed_strassen", APPROX_LAMBDA, 42)}
        self.gen = torch.Generator(device=device)

    def plan(self, r):
        key = (r.n, r.scheme)
        if key not in self.plans:
            if self.tuner is not None:
                q = self.tuner.depth_for(r.n, self.schemes[r.scheme], self.prec, r.scheme)
                lv = [self.schemes[r.scheme]] * q
            else:
                lv = [self.schemes[s] for s in levels_for(r.n, r.scheme)]
            # products that run inside a batch launch take the fewest passes
            self.plans[key] = self.rbc.Plan(r.n, r.n, r.n, lv, prec=self.prec,
                                            fusion="max" if self.mode == "batch" else "auto")
        return self.plans[key]

    def tune(self, schemes=SCHEMES, grid=(256, 512, 1024, 2048, 4096)):
        """Run the tuner's trials for every scheme and grid size now (before serving)."""
        if self.tuner is None:
            return {}
        out = {}
        for name in schemes:
            for g in grid:
                c = self.tuner.choose(g, g, g, self.schemes[name], self.prec, name, tiles=False)
                out["%s/%d" % (name, g)] = c["levels"]
        return out

    def footprint(self, r):
        return 3 * r.n * r.n * 4 + self.plan(r).workspace_bytes + (1 << 20)

    def operands(self, r):
        torch = self.torch
        self.gen.manual_seed(2 * r.rid + 1)
        A = torch.randn(r.n, r.n, device=self.device, generator=self.gen)
        self.gen.manual_seed(2 * r.rid + 2)
        B = torch.randn(r.n, r.n, device=self.device, generator=self.gen)
        return A, B

    def start(self, t0):
        torch = self.torch
        self.t0 = t0
        self.ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        self.ref_wall = time.perf_counter() - t0
        self.ref.record()
        torch.cuda.synchronize()

    def stream(self, slot):
        if slot not in self.streams:
            self.streams[slot] = self.torch.cuda.Stream(device=self.device)
        return self.streams[slot]

    def workspace(self, slot, nbytes):
        """The slot's workspace, grown (by a quarter more than asked) when a product needs more.
        Products on one slot run in its stream's order, so they can share it; a buffer
        replaced while work that uses it is queued goes back to the allocator's pool of that
        stream and is reused only by later work on it.  (Allocating a workspace per product
        left the run at the mercy of the allocator: all 1028 requests of a stream arriving at
        once took 0.11-0.17 s in most processes and up to 4 s in some.)"""
        ws = self.slot_ws.get(slot)
        if ws is None or ws.numel() < nbytes:
            ws = self.torch.empty(nbytes + nbytes // 4, dtype=self.torch.uint8, device=self.device)
            self.slot_ws[slot] = ws
        return ws

    def launch(self, reqs, slot):
        torch = self.torch
        s = self.stream(slot)
        keepalive = []
        with torch.cuda.stream(s):
            if self.mode == "direct":
                for r in reqs:
                    A, B = self.operands(r)
                    plan = self.plan(r)
                    ws = self.workspace(slot, plan.workspace_bytes)
                    C = plan.matmul(A, B, seed=r.seed, mode="full", workspace=ws, stream=s)
                    keepalive.append((A, B, C))
                    self._keep(r, A, B, C)
                batch = None
            else:
                batch = self.rbc.Batch(mode=self.engine, order="depth")
                for r in reqs:
                    A, B = self.operands(r)
                    _, C = batch.add(self.plan(r), A, B, seed=r.seed, mode="full")
                    keepalive.append((A, B, C))
                    self._keep(r, A, B, C)
                ws = self.workspace(slot, batch.workspace_bytes)
                if self.engine == "persistent":
                    batch.set_grid(min(512, max(32, batch.info()["n_tasks"] // 4)))
                batch.prepare(ws, stream=s)
                batch.launch(stream=s)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        return {"event": ev, "batch": batch, "keep": keepalive, "stream": s}

    def _keep(self, r, A, B, C):
        if self.keep is not None and r.rid in self.keep:
            self.keep[r.rid] = (A, B, C)

    def poll(self, h):
        if not h["event"].query():
            return None
        return self.ref_wall + self.ref.elapsed_time(h["event"]) * 1e-3

    def finish(self, h):
        if h["batch"] is not None:
            h["batch"].check(stream=h["stream"])
        h["keep"].clear()

    def stop(self):
        self.torch.cuda.synchronize()
