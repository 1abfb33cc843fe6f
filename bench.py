"""Benchmark: randomized Strassen F-hat^(3) on one MI355X.

Workload: C = A B with N = 4096, three Strassen levels (343 leaves of
512 x 512 x 512 on f32 MFMA, f32 accumulation), A, B i.i.d. U[-1, 1] (data
seeds 2001/2002), algorithm seed = step index mod 16, mode "full".  One step
is one full pass of the hot path: draws + fold for every level, gather of A
and B, the batched leaf GEMM, and the scatter into C, with A and B resident
in HBM.  With the plan's leaf gather on (the default at this size) the
gathers stop one level above the leaves and the leaf GEMM forms its operands
from those parent blocks while loading them.  Prints one JSON line; besides
the headline it carries, each measured outside the timed steps, the f64 N = 64
latency case, one rank-10 APA row on bf16 hi+lo leaves at N = 3072, and
compact rows of the 512-product batch (f16 leaves) and of the served request
stream (fp8 leaves, 0.5 s of arrivals).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --workload approx3072     # approximate scheme, bf16 hi+lo leaves
    python bench.py --workload batch512       # 512 products of mixed N in one persistent launch
    python bench.py --workload serve          # Poisson request stream, fp8 leaves, p50/p99 latency
    python bench.py --workload peaks          # measured ceilings: streaming copy, MFMA loops per dtype
    python bench.py --workload leaves         # reduced-precision leaf products at the configurations' shapes
    python bench.py --copy-calibration BYTES  # plain copy of known size (counter scale)
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 4096
LEVELS = 3
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3


F32_LEAF_SOURCES = ("gemm.hip", "tile_f32.hpp", "gemm_tiles.hpp", "occupancy.hpp", "devptr.hpp")


def _kernel_source_hash():
    """Hash of the sources the f32 leaf GEMM is compiled from (and nothing else)."""
    h = hashlib.sha256()
    for f in F32_LEAF_SOURCES:
        with open(os.path.join(ROOT, "paper_1905_07439_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic():
    """(HBM bytes per leaf-GEMM launch from the committed rocprofv3 counter summary, note).
    The bytes are None, with the reason in the note, when there is no summary or the
    kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "leaf_gemm_f32_n4096_counters.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except OSError:
        return None, "no counter summary at profiles/leaf_gemm_f32_n4096_counters.json"
    have, want = d.get("kernel_source_sha256_16"), _kernel_source_hash()
    if have != want:
        return None, "stale: counters taken for kernel sources %s, built from %s" % (have, want)
    return d.get("hbm_bytes_per_launch"), "FETCH_SIZE/WRITE_SIZE (rocprofv3), copy-calibrated: " + d.get("source", "")


def cpu_baseline(A, B):
    """The oracle (float64 NumPy recursion) on the same workload, one seed, timed on the host."""
    import numpy as np
    from oracle import recursion, schemes
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    S = schemes.strassen()
    t0 = time.perf_counter()
    recursion.rbc_seeded(A, B, [S] * LEVELS, 0)
    dt = time.perf_counter() - t0
    return {"value": 2.0 * N ** 3 / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": "one full F-hat^(3) product, N=4096, float64 NumPy (OpenBLAS dgemm leaves), seed 0; "
                      "%.2f s" % dt}


def _time_steps(fn, steps, warmup):
    import torch
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn(i)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def approx3072(args):
    """Approximate schemes at N = 3072, bf16 hi+lo leaves with f64 recombination, beside the
    plain f32 recursive form on the same GPU; N(0,1) inputs (seeds 3001/3002): the rank-10
    <3,2,2> APA with 1/lambda coefficients at one, two and three levels (three: 1000 leaves
    of 128 x 384 x 384, A's rows zero-padded to 27 x 128) and perturbed Strassen (Section 3.1
    recipe, sigma = lambda) at three levels (343 leaves of 384^3)."""
    import numpy as np
    import torch

    import paper_1905_07439_amd as rbc
    import workloads

    n = 3072
    dev = "cuda:0"
    A64 = workloads.gaussian((n, n), 3001)
    B64 = workloads.gaussian((n, n), 3002)
    A = torch.from_numpy(A64.astype(np.float32)).to(dev)
    B = torch.from_numpy(B64.astype(np.float32)).to(dev)
    ref = A.double() @ B.double()
    C = torch.empty((n, n), dtype=torch.float32, device=dev)
    S = rbc.Scheme.builtin("strassen")
    rows = []
    cases = [("apa322", q, lam) for q in (1, 2, 3) for lam in (1e-1, 1e-2, 1e-3, 1e-4)]
    cases += [("bini12", 3, lam) for lam in (1e-1, 3e-2, 1.5e-2, 1e-2)]
    cases += [("perturbed_strassen", 3, lam) for lam in (1e-1, 1e-2, 1e-3, 1e-4)]
    for kind, q, lam in cases:
        if kind == "apa322":
            levels = [rbc.Scheme.builtin("apa322:%r" % lam)] * q
        elif kind == "bini12":  # one step of the 12 x 12 scheme: <3,2,2>, <2,2,3>, <2,3,2>
            levels = [rbc.Scheme.builtin("%s:%r" % (k, lam)) for k in ("apa322", "apa223", "apa232")]
        else:
            levels = [rbc.Scheme.builtin("perturbed_strassen", lam, 42)] * q
        for prec in ("bf16x3", "f32"):
            plan = rbc.Plan(n, n, n, levels, prec=prec)
            ws = plan.workspace(dev)
            for mode in ("none", "full"):
                ms = _time_steps(lambda i: plan.matmul(A, B, C=C, seed=i % 16, mode=mode, workspace=ws),
                                 args.steps, args.warmup)
                errs = []
                for seed in range(4):
                    plan.matmul(A, B, C=C, seed=seed, mode=mode, workspace=ws)
                    errs.append(float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref)))
                rows.append({"scheme": kind, "levels": q, "lambda": lam, "prec": prec, "mode": mode,
                             "ms": round(ms, 4),
                             "tflops": round(2.0 * n ** 3 / ms / 1e9, 2),
                             "rel_err_vs_fp64": [float("%.3g" % e) for e in errs]})
    # The exact combination of the 12 x 12 step over lambda = 0.1..0.7 (7 products, weights
    # +-C(7, i), f64 accumulation on the device), plans built before the timed region.
    eps7 = [0.1 * k for k in range(1, 8)]
    names = ["apa322", "apa223", "apa232"]
    Cd = torch.empty((n, n), dtype=torch.float64, device=dev)
    for prec in ("bf16x3", "f32"):
        plans = rbc.apa_ebc_plans(n, n, n, names, eps7, prec=prec)
        ws = torch.empty(max(p.info["workspace_bytes"] for p in plans) + 256 + n * n * 4, dtype=torch.uint8,
                         device=dev)
        for mode in ("none", "full"):
            run = lambda i: rbc.matmul_apa_ebc(A, B, names, eps7, prec=prec, seed=i % 16, mode=mode, plans=plans,
                                               workspace=ws, out=Cd)
            ms = _time_steps(run, args.steps, args.warmup)
            errs = []
            for seed in range(4):
                run(seed)
                errs.append(float(torch.linalg.norm(Cd - ref) / torch.linalg.norm(ref)))
            rows.append({"scheme": "bini12_ebc_7", "levels": 3, "lambda": eps7, "prec": prec, "mode": mode,
                         "ms": round(ms, 4), "tflops": round(2.0 * n ** 3 / ms / 1e9, 2),
                         "rel_err_vs_fp64": [float("%.3g" % e) for e in errs]})
    std_ms = _time_steps(lambda i: torch.matmul(A, B, out=C), args.steps, args.warmup)
    out = {"metric": "effective TFLOP/s (2n³/t) at stated rel-err vs FP64 oracle; p50/p99 latency",
           "unit": "TFLOP/s", "n_gpus": 1, "dtype": "bf16x3 leaves / f32 comparator", "data": "synthetic",
           "config": {"workload": "rank-10 <3,2,2> APA (Q=1..3), rank-1000 12x12 APA "
                                  "(one step) and its exact combination over 7 lambda, perturbed Strassen (sigma=lambda, Q=3), "
                                  "N=3072, N(0,1)", "n": n},
           "rows": rows, "standard_f32_gemm_same_gpu_ms": round(std_ms, 4)}
    print(json.dumps(out), flush=True)


def peaks(args):
    """Measured ceilings on this GPU, for reading the rooflines against what the chip attains:
    the library's streaming copy over 2 x 2 GiB (HBM bytes = 2 x the size) and its register-only
    matrix-core loops per data type (2048 workgroups of 256 threads, 8 independent chains per
    wavefront).  Median of 10 timed launches after 2 warm-ups, HIP events on one stream."""
    import torch

    import paper_1905_07439_amd as rbc

    dev = "cuda:0"
    torch.cuda.set_device(0)
    s = torch.cuda.current_stream()

    def timed(fn, reps=10, warm=2):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            fn()
            e1.record(s)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return sorted(ts)[len(ts) // 2]

    nbytes = 2 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    src.fill_(1)
    ms = timed(lambda: rbc.peak_copy(src, dst))
    hbm = 2.0 * nbytes / (ms * 1e-3) / 1e9
    ms_t = timed(lambda: dst.copy_(src))
    hbm_torch = 2.0 * nbytes / (ms_t * 1e-3) / 1e9
    del src, dst
    sink = torch.empty(2048 * 256, dtype=torch.float32, device=dev)
    published = {"f32": 157.3, "f64": 78.6, "f16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "f32_32x32": 157.3,
                 "f16_32x32": 2500.0, "bf16_32x32": 2500.0}
    iters = {"f32": 4000, "f64": 4000, "f16": 2000, "bf16": 2000, "fp8": 1000, "f32_32x32": 4000,
             "f16_32x32": 2000, "bf16_32x32": 2000}
    mfma = {}
    for kind in published:
        fl = [0.0]

        def run():
            fl[0] = rbc.peak_mfma(kind, sink, iters[kind])
        ms = timed(run)
        tf = fl[0] / (ms * 1e-3) / 1e12
        mfma[kind] = {"tflops": round(tf, 1), "published": published[kind], "frac": round(tf / published[kind], 3)}
    out = {"metric": "measured ceilings (streaming copy, register-only MFMA loops)", "n_gpus": 1,
           "hbm_copy_GBs": round(hbm, 1), "hbm_published_GBs": HBM_PEAK_GBS,
           "hbm_frac": round(hbm / HBM_PEAK_GBS, 3), "hbm_torch_copy_GBs": round(hbm_torch, 1), "mfma": mfma}
    print(json.dumps(out), flush=True)


def small64_stats(reps, warmup):
    """The small case: plain randomized Strassen in f64, N = 64, two levels (49 leaves of 16^3),
    A, B ~ N(0,1) (seeds 1001/1002) and integers in [-4, 4] (seed 1003 for A, 1004 for B),
    algorithm seed 0, mode full.  Launch-latency bound: per-call latency (HIP events around
    each call) over `reps` calls, p50 and p99 in microseconds, beside the device's own time per
    product (a captured graph of 20 products replayed; the eager call is bound by the host's
    kernel-launch cost)."""
    import numpy as np
    import torch

    import paper_1905_07439_amd as rbc
    import workloads

    n, dev = 64, "cuda:0"
    S = rbc.Scheme.builtin("strassen")
    plan = rbc.Plan(n, n, n, [S, S], prec="f64")
    A = torch.from_numpy(workloads.gaussian((n, n), 1001)).to(dev)
    B = torch.from_numpy(workloads.gaussian((n, n), 1002)).to(dev)
    Ai = torch.from_numpy(workloads.integers((n, n), 1003).astype(np.float64)).to(dev)
    Bi = torch.from_numpy(workloads.integers((n, n), 1004).astype(np.float64)).to(dev)
    C = torch.empty((n, n), dtype=torch.float64, device=dev)
    ws = plan.workspace(dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.matmul(A, B, C=C, seed=0, workspace=ws)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for e0, e1 in ev:
        e0.record(stream)
        plan.matmul(A, B, C=C, seed=0, workspace=ws, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    lat = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev])  # microseconds
    p50 = float(np.percentile(lat, 50))
    ref = A @ B
    err = float(torch.linalg.norm(C - ref) / torch.linalg.norm(ref))
    Ci = plan.matmul(Ai, Bi, seed=0, workspace=ws)
    exact = bool(torch.equal(Ci, Ai @ Bi))
    # The device's own time per product: 20 products captured in a graph and replayed,
    # so that no host issue time separates the launches (the eager call is host-bound).
    C_eager = C.clone()
    device_us, replay_same = None, None
    try:
        gs = torch.cuda.Stream()
        gs.wait_stream(stream)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=gs):
            for _ in range(20):
                plan.matmul(A, B, C=C, seed=0, workspace=ws, stream=gs)
        C.zero_()
        graph.replay()
        torch.cuda.synchronize()
        replay_same = bool(torch.equal(C, C_eager))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(50):
            graph.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        replay_same = replay_same and bool(torch.equal(C, C_eager))
        device_us = round(e0.elapsed_time(e1) * 1e3 / (50 * 20), 2)
    except RuntimeError as e:  # capture unavailable: the eager figures stand alone
        print("small64: graph capture failed: %s" % e, file=sys.stderr, flush=True)
    return {"p50_us": round(p50, 2), "p99_us": round(float(np.percentile(lat, 99)), 2),
            "min_us": round(float(lat.min()), 2), "reps": reps,
            "device_us_per_product_graph": device_us, "graph_replay_bitwise_equal": replay_same,
            "tflops_at_p50": round(2.0 * n ** 3 / (p50 * 1e-6) / 1e12, 6),
            "rel_err_vs_fp64": err, "integers_exact": exact}


def small64(args):
    st = small64_stats(args.small_reps, args.warmup)
    out = {"metric": "effective TFLOP/s (2n³/t) at stated rel-err vs FP64 oracle; p50/p99 latency",
           "value": st["tflops_at_p50"], "unit": "TFLOP/s", "n_gpus": 1,
           "steps": args.small_reps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "randomized Strassen, f64, N=64, 2 levels (49 leaves of 16^3), N(0,1) and "
                                  "integers in [-4,4], algorithm seed 0, mode full", "n": 64, "levels": 2,
                      "parallelism": "single GPU"},
           "latency_us": {"p50": st["p50_us"], "p99": st["p99_us"], "min": st["min_us"],
                          "device_per_product_graph": st["device_us_per_product_graph"]},
           "graph_replay_bitwise_equal": st["graph_replay_bitwise_equal"],
           "rel_err_vs_fp64": st["rel_err_vs_fp64"], "integers_exact": st["integers_exact"]}
    print(json.dumps(out), flush=True)


def apa3072_row(steps, warmup, lam=1e-3):
    """One approximate-scheme row: the rank-10 <3,2,2> APA (1/lambda coefficients in W) at one
    level, N = 3072 (10 leaves of 1024 x 1536 x 1536), bf16 hi+lo leaves (three bf16 MFMA
    products, f32 accumulation) with the W-recombination in f64, N(0,1) inputs (seeds
    3001/3002), mode full, algorithm seeds 0..15.  Reports ms per product (HIP events), the
    relative error against the f64 product of the same (f32) inputs, and the same plan in f32."""
    import numpy as np
    import torch

    import paper_1905_07439_amd as rbc
    import workloads

    n, dev = 3072, "cuda:0"
    A = torch.from_numpy(workloads.gaussian((n, n), 3001).astype(np.float32)).to(dev)
    B = torch.from_numpy(workloads.gaussian((n, n), 3002).astype(np.float32)).to(dev)
    ref = A.double() @ B.double()
    C = torch.empty((n, n), dtype=torch.float32, device=dev)
    S = rbc.Scheme.builtin("apa322", lam)
    row = {"scheme": "apa322", "levels": 1, "lambda": lam, "mode": "full", "n": n}
    for prec in ("bf16x3", "f32"):
        plan = rbc.Plan(n, n, n, [S], prec=prec)
        ws = plan.workspace(dev)
        for i in range(warmup):
            plan.matmul(A, B, C=C, seed=i % 16, workspace=ws)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(steps):
            plan.matmul(A, B, C=C, seed=i % 16, workspace=ws, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        errs = []
        for seed in range(2):
            plan.matmul(A, B, C=C, seed=seed, workspace=ws)
            errs.append(float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref)))
        row[prec] = {"ms": round(ms, 4), "tflops": round(2.0 * n ** 3 / ms / 1e9, 2), "leaf_tile": plan.info["tile_m"],
                     "rel_err_vs_fp64": [float("%.3g" % e) for e in errs]}
        del plan, ws
    return row


def batch_levels(n):
    """Laderman at the top, then Strassen until the leaf side is at most 128."""
    m, s = n // 3, 0
    while m > 128:
        m //= 2
        s += 1
    return ["laderman"] + ["strassen"] * s


def batch512(args):
    print(json.dumps(batch512_line(args)), flush=True)


def batch512_line(args):
    """512 independent products, N_i = 96 k_i with k_i uniform on {2..24} (size seed 4000),
    Laderman then Strassen to leaves of 64..128, f16 leaves with per-leaf power-of-two scales,
    all in one persistent launch replayed from a HIP graph.  A_i, B_i are N(0,1) times one
    factor 10^U(-3,3) per matrix (factor seeds 4000+i / 14000+i, entries from torch's
    Philox generator seeded alike, on the GPU); algorithm seed i, mode full."""
    import numpy as np
    import torch

    import paper_1905_07439_amd as rbc
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)
    count = args.batch_count
    sizes = workloads.batch_sizes(count, 4000)
    L, S = rbc.Scheme.builtin("laderman"), rbc.Scheme.builtin("strassen")
    plans16, plans32 = {}, {}
    As, Bs, Cs = [], [], []
    g = torch.Generator(device=dev)
    for i, n in enumerate(sizes):
        lv = batch_levels(n)
        if n not in plans16:
            sch = [L] + [S] * (len(lv) - 1)
            plans16[n] = rbc.Plan(n, n, n, sch, prec="f16s", fusion="max")  # batch plans: fewest passes
            plans32[n] = rbc.Plan(n, n, n, sch, prec="f32")
        fa = 10.0 ** np.random.default_rng(4000 + i).uniform(-3, 3)
        fb = 10.0 ** np.random.default_rng(14000 + i).uniform(-3, 3)
        g.manual_seed(4000 + i)
        As.append(torch.randn(n, n, device=dev, generator=g) * fa)
        g.manual_seed(14000 + i)
        Bs.append(torch.randn(n, n, device=dev, generator=g) * fb)
        Cs.append(torch.empty(n, n, device=dev))
    flops = sum(2.0 * n ** 3 for n in sizes)
    traffic = sum(sum(plans16[n].traffic().values()) for n in sizes)

    batch = rbc.Batch(item_budget=args.batch_budget_gb << 30, order="depth")
    for i, n in enumerate(sizes):
        batch.add(plans16[n], As[i], Bs[i], C=Cs[i], seed=i, mode="full")
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        batch.prepare(stream=stream)
    prep_s = time.perf_counter() - t0
    info = batch.info()
    for _ in range(args.warmup):
        batch.launch(graph=True, stream=stream)
    batch.check(stream=stream)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(args.steps):
        batch.launch(graph=True, stream=stream)
        ev[k + 1].record(stream)
    batch.check(stream=stream)
    wall_ms = (time.perf_counter() - w0) * 1e3 / args.steps
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
    ms = float(np.mean(per))
    value = flops / (ms * 1e-3) / 1e12

    # the same batch through the level-synchronous executor (grouped launches in one graph)
    lb = rbc.Batch(item_budget=args.batch_budget_gb << 30, mode="levels")
    Cl = [torch.empty_like(c) for c in Cs]
    for i, n in enumerate(sizes):
        lb.add(plans16[n], As[i], Bs[i], C=Cl[i], seed=i, mode="full")
    with torch.cuda.stream(stream):
        lb.prepare(stream=stream)
    for _ in range(args.warmup):
        lb.launch(graph=True, stream=stream)
    lb.check(stream=stream)
    ev2 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev2[0].record(stream)
    for k in range(args.steps):
        lb.launch(graph=True, stream=stream)
        ev2[k + 1].record(stream)
    lb.check(stream=stream)
    ms_levels = float(np.mean([ev2[k].elapsed_time(ev2[k + 1]) for k in range(args.steps)]))
    same_bits = all(torch.equal(a, b) for a, b in zip(Cs, Cl))
    linfo = lb.info()
    del lb, Cl

    # accuracy of every product against the float64 product of the same operands
    errs = []
    for i in range(count):
        ref = As[i].double() @ Bs[i].double()
        errs.append(float(torch.linalg.norm(Cs[i].double() - ref) / torch.linalg.norm(ref)))
    errs = np.array(errs)

    # the same products one by one on the same GPU: stand-alone f16s path, the plain f32
    # recursive form, and the standard f32 product (torch -> hipBLASLt)
    def seq(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / reps

    C32 = [torch.empty_like(c) for c in Cs[:1]]
    seq16 = seq(lambda: [plans16[n].matmul(As[i], Bs[i], C=Cs[i], seed=i) for i, n in enumerate(sizes)])
    seq32 = seq(lambda: [plans32[n].matmul(As[i], Bs[i], C=Cs[i], seed=i) for i, n in enumerate(sizes)])
    errs32 = []
    for i in range(0, count, 16):
        ref = As[i].double() @ Bs[i].double()
        errs32.append(float(torch.linalg.norm(Cs[i].double() - ref) / torch.linalg.norm(ref)))
    std32 = seq(lambda: [torch.matmul(As[i], Bs[i], out=Cs[i]) for i in range(count)])
    del C32

    out = {
        "metric": "effective TFLOP/s (2n³/t) at stated rel-err vs FP64 oracle; p50/p99 latency",
        "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "wall_ms_per_step": round(wall_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16 leaves (f32 accumulate)",
        "data": "synthetic",
        "config": {"workload": "batch of %d products, N = 96k, k ~ U{2..24}, Laderman then Strassen to "
                               "leaves 64..128, f16 leaves with per-leaf 2^e scales, one persistent launch "
                               "in a HIP graph (queue in dependency-depth order)" % count,
                   "count": count, "effective_tflop": round(flops / 1e12, 4),
                   "item_budget_gb": args.batch_budget_gb, "parallelism": "single GPU"},
        "rel_err_vs_fp64": {"median": float(np.median(errs)), "max": float(errs.max())},
        "batch": {k: info[k] for k in ("n_tasks", "gather_tasks", "leaf_tasks", "scatter_tasks", "gate_tasks",
                                       "grid", "workspace_bytes")},
        "prepare_s": round(prep_s, 3),
        "levels_mode": {"ms_per_step": round(ms_levels, 4), "tflops": round(flops / ms_levels / 1e9, 3),
                        "launches": linfo["launches"], "levels": linfo["levels"],
                        "bitwise_equal_to_persistent": same_bits},
        "same_gpu": {"f16s_one_by_one_ms": round(seq16, 3), "f32_recursive_one_by_one_ms": round(seq32, 3),
                     "f32_recursive_rel_err_max": max(errs32),
                     "standard_f32_gemm_one_by_one_ms": round(std32, 3)},
        "roofline": {"bound": "hbm", "achieved": round(traffic / (ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(traffic / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "algorithmic_bytes": traffic},
    }
    return out


def serve_stream(args):
    print(json.dumps(serve_line(args)), flush=True)


def serve_line(args):
    """Requests C = A B arriving as a Poisson process at 2000 per second (seed 5000) for
    --serve-seconds, N log-uniform in [128, 4096] (multiples of 32), scheme uniform over
    Strassen, Laderman and the approximate (perturbed Strassen, lambda = 1e-3) scheme, one
    algorithm seed per request, A and B N(0,1) generated on the device; fp8 leaves with
    per-leaf power-of-two scales and one correction pass; admission under a 200 GB HBM
    budget, 4 slots, continuous batching (the products admitted together launch their stages
    on one slot's stream; batches on different slots overlap).  The same request stream is
    also served through the batch engine (level-synchronous launches, one batch per admission)
    and with the plain f32 recursive form.  The recursion depth of each (size, scheme) comes
    from the autotuner (timed trials at five size classes before the stream starts); one more
    fp8 run uses the fixed depth rule (leaves of about 192) for comparison."""
    import numpy as np
    import torch

    from paper_1905_07439_amd import serve
    from paper_1905_07439_amd.tune import Tuner

    torch.cuda.set_device(0)
    budget = 200e9

    tuners = {}

    def run(prec, mode, duration, seed, keep=None, tuned=True):
        reqs = serve.make_requests(2000, duration, seed)
        if tuned and prec not in tuners:
            tuners[prec] = Tuner()
        ex = serve.GpuExecutor(prec=prec, mode=mode, keep=keep, engine="levels",
                               tuner=tuners[prec] if tuned else None)
        depths = ex.tune()  # timed trials per scheme and size class, before the stream starts
        sch = serve.Scheduler(budget, max_batch=64)
        # warm up: plans and kernels of every size class, outside the measured stream
        warm = serve.make_requests(2000, 0.05, seed + 100)
        serve.serve(warm, ex, serve.Scheduler(budget, 64), slots=4)
        stats = serve.serve(reqs, ex, sch, slots=4)
        stats["tuned_depth"] = depths
        return stats, reqs, ex

    keep = {}
    out_rows = {}
    for prec, mode, tuned in (("fp8c", "direct", True), ("fp8c", "batch", True), ("f32", "direct", True),
                              ("fp8c", "direct", False)):
        reqs_probe = serve.make_requests(2000, args.serve_seconds, 5000)
        k = {r.rid: None for r in reqs_probe[::97]}
        stats, reqs, ex = run(prec, mode, args.serve_seconds, 5000, keep=k, tuned=tuned)
        errs = {}
        for rid, val in k.items():
            if val is None:
                continue
            A, B, C = val
            ref = A.double() @ B.double()
            e = float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref))
            errs.setdefault(reqs[rid].scheme, []).append(e)
        stats["rel_err_vs_fp64"] = {s: {"median": float(np.median(v)), "max": float(np.max(v))}
                                    for s, v in errs.items()}
        out_rows["%s_%s%s" % (prec, mode, "" if tuned else "_fixed_depth")] = stats
        del ex
        torch.cuda.empty_cache()
    # capacity: the same requests all present at time 0 (the loop runs as fast as the device
    # allows), measured on the second of two passes: the first creates the plans and uploads
    # their tables, which a long-running server has done before
    capacity = {}
    for prec in ("fp8c", "f32"):
        ex = serve.GpuExecutor(prec=prec, mode="direct", engine="levels", tuner=tuners[prec])
        ex.tune()
        for _ in range(2):
            reqs = serve.make_requests(2000, args.serve_seconds, 5000)
            for r in reqs:
                r.arrival = 0.0
            st = serve.serve(reqs, ex, serve.Scheduler(budget, max_batch=64), slots=4)
        capacity[prec] = {"tflops": round(st["effective_tflops"], 3), "span_s": round(st["span_s"], 4),
                          "requests": st["requests"]}
        del ex
        torch.cuda.empty_cache()
    head = out_rows["fp8c_direct"]
    out = {
        "metric": "effective TFLOP/s (2n³/t) at stated rel-err vs FP64 oracle; p50/p99 latency",
        "value": round(head["effective_tflops"], 3), "unit": "TFLOP/s", "n_gpus": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp8 e4m3 leaves + 1 correction pass (f32 accumulate)", "data": "synthetic",
        "config": {"workload": "serving: Poisson 2000 req/s for %.1f s, N log-uniform [128, 4096], "
                               "scheme uniform {strassen, laderman, approx lambda=1e-3}, fp8c leaves, "
                               "200 GB admission budget, 4 slots, continuous batching, recursion depth "
                               "per size class from timed trials; headline: each admitted product's "
                               "stages launched on its slot's stream" % args.serve_seconds,
                   "parallelism": "single GPU"},
        "p50_ms": round(head["latency_ms"]["p50"], 3), "p99_ms": round(head["latency_ms"]["p99"], 3),
        "runs": out_rows,
        "capacity_all_arrived_at_0": capacity,
    }
    return out


def _compact_rows(args):
    """The batched and the served configurations' headline figures, for the default line
    (each in a few seconds; a failure is reported in its row instead of ending the line)."""
    rows = {}
    try:
        b = batch512_line(argparse.Namespace(batch_count=512, batch_budget_gb=args.batch_budget_gb, steps=3,
                                             warmup=1))
        rows["batch512_f16s"] = {
            "ms_per_batch": b["ms_per_step"], "tflops": b["value"], "steps": 3,
            "rel_err_vs_fp64": b["rel_err_vs_fp64"], "levels_mode": b["levels_mode"], "same_gpu": b["same_gpu"],
            "hbm_frac_algorithmic": b["roofline"]["frac"], "workload": b["config"]["workload"]}
    except Exception as e:  # noqa: BLE001 -- reported, not fatal for the headline
        rows["batch512_f16s"] = {"error": repr(e)}
    try:
        v = serve_line(argparse.Namespace(serve_seconds=0.5))
        runs = v["runs"]
        rows["serve_fp8c"] = {
            "seconds_of_arrivals": 0.5, "p50_ms": v["p50_ms"], "p99_ms": v["p99_ms"], "tflops": v["value"],
            "rel_err_vs_fp64": runs["fp8c_direct"]["rel_err_vs_fp64"],
            "f32_recursive_same_stream": {"p50_ms": round(runs["f32_direct"]["latency_ms"]["p50"], 3),
                                          "p99_ms": round(runs["f32_direct"]["latency_ms"]["p99"], 3),
                                          "tflops": round(runs["f32_direct"]["effective_tflops"], 3)},
            "capacity_all_arrived_at_0": v["capacity_all_arrived_at_0"], "workload": v["config"]["workload"]}
    except Exception as e:  # noqa: BLE001
        rows["serve_fp8c"] = {"error": repr(e)}
    return rows


def leaves(args):
    """The reduced-precision leaf products at the configurations' shapes, one product per
    case timed stage by stage (HIP events): f16s Strassen Q = 2 at N = 4096 (49 leaves of
    1024^3), bf16x3 rank-10 <3,2,2> APA (lambda = 1e-3) Q = 1 at N = 3072 (10 leaves of
    1024 x 1536 x 1536, three bf16 products each), fp8c Strassen Q = 4 at N = 4096 (2401
    leaves of 256^3, hi/lo e4m3 with one correction pass: three fp8 products each);
    A, B ~ N(0,1) (seeds 3001/3002), mode full.  Per case: leaf kernel time, its rate against
    the dtype's dense MFMA peak, and the leaf stage's algorithmic HBM bytes per second."""
    import numpy as np
    import torch

    import paper_1905_07439_amd as rbc
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)
    S = rbc.Scheme.builtin("strassen")
    cases = [("f16s", 4096, [S] * 2, 1, 2500.0), ("bf16x3", 3072, [rbc.Scheme.builtin("apa322", 1e-3)], 3, 2500.0),
             ("fp8c", 4096, [S] * 4, 3, 5000.0)]
    rows = []
    for prec, n, levels, passes, peak in cases:
        A = torch.from_numpy(workloads.gaussian((n, n), 3001).astype(np.float32)).to(dev)
        B = torch.from_numpy(workloads.gaussian((n, n), 3002).astype(np.float32)).to(dev)
        plan = rbc.Plan(n, n, n, levels, prec=prec)
        ws = plan.workspace(dev)
        C = torch.empty((n, n), dtype=torch.float32, device=dev)
        for i in range(args.warmup):
            plan.matmul(A, B, C=C, seed=i, workspace=ws)
        plan.set_timing(True)
        for i in range(args.steps):
            plan.matmul(A, B, C=C, seed=i, workspace=ws)
        torch.cuda.synchronize()
        stage_ms, calls = plan.timing_collect()
        plan.set_timing(False)
        info = plan.info
        leaf_ms = stage_ms[2] / calls
        flops = passes * info["n_leaves"] * 2.0 * info["mM"] * info["mK"] * info["mN"]
        leaf_bytes = plan.traffic()["leaf"]
        rows.append({"prec": prec, "n": n, "levels": len(levels), "leaf": [info["mM"], info["mK"], info["mN"]],
                     "n_leaves": info["n_leaves"], "tile": info["tile_m"], "leaf_ms": round(leaf_ms, 4),
                     "leaf_tflops": round(flops / leaf_ms / 1e9, 1), "mfma_peak_tflops": peak,
                     "mfma_frac": round(flops / leaf_ms / 1e9 / peak, 3),
                     "leaf_algorithmic_GBs": round(leaf_bytes / leaf_ms / 1e6, 1),
                     "hbm_floor_ms": round(leaf_bytes / HBM_PEAK_GBS / 1e6, 4),
                     "stage_ms": [round(x / calls, 4) for x in stage_ms[:4]]})
        del plan, ws
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "reduced-precision leaf products at the configurations' shapes", "n_gpus": 1,
                      "steps": args.steps, "rows": rows}), flush=True)


def copy_calibration(nbytes):
    """A plain device copy of nbytes (for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": x.numel() * 4, "launches": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--device-warmup-ms", type=float, default=500.0,
                    help="untimed back-to-back products before the warm-up steps (clock ramp)")
    ap.add_argument("--workload", default="strassen4096",
                    choices=["strassen4096", "approx3072", "batch512", "serve", "small64", "peaks", "leaves"])
    ap.add_argument("--small-reps", type=int, default=1000)
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-budget-gb", type=int, default=24)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES")
    ap.add_argument("--headline-only", action="store_true",
                    help="the headline workload alone (no other configurations' rows): for profiler runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (requested --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.workload == "approx3072":
        return approx3072(args)
    if args.workload == "batch512":
        return batch512(args)
    if args.workload == "serve":
        return serve_stream(args)
    if args.workload == "small64":
        return small64(args)
    if args.workload == "peaks":
        return peaks(args)
    if args.workload == "leaves":
        return leaves(args)

    import numpy as np
    import torch

    import paper_1905_07439_amd as rbc
    import workloads

    dev = "cuda:0"
    torch.cuda.set_device(0)
    S = rbc.Scheme.builtin("strassen")
    plan = rbc.Plan(N, N, N, [S] * LEVELS, prec="f32")
    info = plan.info
    A64 = workloads.uniform((N, N), 2001, -1, 1)
    B64 = workloads.uniform((N, N), 2002, -1, 1)
    A = torch.from_numpy(A64.astype(np.float32)).to(dev)
    B = torch.from_numpy(B64.astype(np.float32)).to(dev)
    C = torch.empty((N, N), dtype=torch.float32, device=dev)
    ws = plan.workspace(dev)
    stream = torch.cuda.current_stream()

    # Device warm-up (untimed): the GPU's clocks take up to about a second of load to reach
    # their steady state (the same leaf product measured 0.96 ms cold and 0.80 ms warm), so the
    # product runs back to back for --device-warmup-ms before the W warm-up steps.
    t_dw = time.perf_counter()
    n_dw = 0
    while (time.perf_counter() - t_dw) * 1e3 < args.device_warmup_ms:
        for i in range(8):
            plan.matmul(A, B, C=C, seed=i % 16, workspace=ws)
        n_dw += 8
        torch.cuda.synchronize()
    for i in range(args.warmup):
        plan.matmul(A, B, C=C, seed=i % 16, workspace=ws)
    torch.cuda.synchronize()

    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.matmul(A, B, C=C, seed=i % 16, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, calls = plan.timing_collect()
    plan.set_timing(False)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = 2.0 * N ** 3 / (ms_per_step * 1e-3) / 1e12

    # the standard O(n^3) product on the same GPU (torch -> hipBLASLt/rocBLAS f32), for context
    for _ in range(3):
        torch.matmul(A, B, out=C)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    for _ in range(args.steps):
        torch.matmul(A, B, out=C)
    torch.cuda.synchronize()
    std_ms = (time.perf_counter() - g0) * 1e3 / args.steps

    # accuracy of the last step's seed against the float64 standard product
    seed = (args.steps - 1) % 16
    plan.matmul(A, B, C=C, seed=seed, workspace=ws)
    ref = A.double() @ B.double()
    rel_err = float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref))

    leaf_ms = stage_ms[2] / calls
    leaf_flops = info["n_leaves"] * 2.0 * info["mM"] * info["mN"] * info["mK"]
    achieved = leaf_flops / (leaf_ms * 1e-3) / 1e12
    traffic, traffic_note = _traffic()
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": FP32_MFMA_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4),
                "traffic": traffic, "traffic_note": traffic_note,
                "kernel": "leaf GEMM (f32 MFMA 16x16x4, operands formed from the level-2 blocks while loading)",
                "algorithmic_flops_per_launch": leaf_flops}
    tr = plan.traffic()  # algorithmic bytes of the path the plan takes
    comb_bytes = tr["gather_A"] + tr["gather_B"] + tr["scatter"]
    comb_ms = stage_ms[0] / calls + stage_ms[1] / calls + stage_ms[3] / calls

    out = {
        "metric": "effective TFLOP/s (2n³/t) at stated rel-err vs FP64 oracle; p50/p99 latency",
        "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "randomized Strassen F-hat^(3), N=4096, 343 leaves of 512^3 on f32 MFMA, "
                               "A,B ~ U[-1,1] (seeds 2001/2002), algorithm seeds 0..15, mode full",
                   "n": N, "levels": LEVELS, "scheme": "strassen", "leaf": info["mM"], "prec": "f32",
                   "leaf_gather": plan.leaf_gather[0], "parallelism": "single GPU"},
        "device_warmup": {"ms": args.device_warmup_ms, "products": n_dw},
        "rel_err_vs_fp64": rel_err,
        "stage_ms": {"gather_A": round(stage_ms[0] / calls, 4), "gather_B": round(stage_ms[1] / calls, 4),
                     "leaf": round(leaf_ms, 4), "scatter": round(stage_ms[3] / calls, 4)},
        "combination_hbm_GBs": round(comb_bytes / (comb_ms * 1e-3) / 1e9, 1),
        "standard_f32_gemm_same_gpu": {"ms": round(std_ms, 4), "tflops": round(2.0 * N ** 3 / std_ms / 1e9, 2),
                                       "lib": "torch.matmul (hipBLASLt/rocBLAS)"},
        "roofline": roofline,
    }
    # the other configurations' headline figures, cheap enough for the default line
    if not args.headline_only:
        out["small64_f64_n64_q2"] = small64_stats(1000, 20)
        out["apa322_n3072_q1_bf16x3"] = apa3072_row(max(5, args.steps // 2), 3)
        out.update(_compact_rows(args))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A64, B64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
