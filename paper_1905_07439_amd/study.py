"""Error-study harness on the GPU (the experiments of Section 3).

* ``error_of_average``: the relative error of the average of the first k
  realizations, || (1/k) sum_i F-hat_i(A, B) - A B || / || A B ||, for k up to
  K (eq. error-of-average; Figures 1 and 5): a perturbed Strassen ABC in f64
  (Section 3.1) or Strassen in f32 (Section 3.2), with the standard f32
  product's error beside it for reference.
* ``error_distribution``: the relative error of each of ``trials``
  realizations (eq. average-of-error; Figures 2, 3 and 7-12) for Q = 1..5 and
  the randomization modes: deterministic ("none"), fully randomized ("full"),
  random sign ("signs") and random permutation ("perms").

Matrices come from the seeded generators of the paper's setting (Gaussian,
uniform, adversarial types 1-3, Hilbert).  Plans use exact blocks (leaf tile
-1): the recursion splits the matrices as the unpadded problem, as in the
paper (N = 320 with Q = 5 has leaves of 10 x 10), rather than padding them to
the leaf GEMM's tile.  The truth is the float64 standard
product.  Products and averages run in the library's kernels; the float64
reference product and the norms use torch on the device.

    python -m paper_1905_07439_amd.study --experiment average --out avg.json
    python -m paper_1905_07439_amd.study --experiment distribution --out dist.json
"""

import argparse
import ctypes
import json
import sys

import numpy as np

MODES = ("none", "full", "signs", "perms")


def matrices(kind, n, seed):
    """(A, B) as float64 numpy arrays: gaussian, uniform (0, 1), adversarial1..3, hilbert."""
    import workloads
    if kind == "gaussian":
        return workloads.gaussian((n, n), seed), workloads.gaussian((n, n), seed + 1)
    if kind == "uniform":
        return workloads.uniform((n, n), seed), workloads.uniform((n, n), seed + 1)
    if kind == "hilbert":
        H = workloads.hilbert(n)
        return H, H.copy()
    if kind.startswith("adversarial"):  # a pair of Definition 14's type 1, 2 or 3
        return workloads.adversarial(int(kind[-1]), n, seed)
    raise ValueError("unknown matrix kind %r" % kind)


def _schemes(name, q):
    import paper_1905_07439_amd as rbc
    S = rbc.Scheme.builtin("strassen")
    if name == "pert":  # Section 3.1: sigma = 1e-3 on the ones and on five zeros per tensor
        return [rbc.Scheme.builtin("perturbed_strassen", 1e-3, 42)] * q
    return [rbc.Scheme.builtin(name)] * q


def _rel(C, ref):
    import torch
    return float(torch.linalg.norm(C.double() - ref) / torch.linalg.norm(ref))


def error_of_average(kind="gaussian", n=80, qs=(1, 2, 3), K=10000, checkpoints=None, scheme="pert",
                     prec="f64", seed=1, mode="full"):
    import torch
    import paper_1905_07439_amd as rbc
    from paper_1905_07439_amd import _lib
    dev = "cuda:0"
    A64, B64 = matrices(kind, n, seed)
    dt = torch.float64 if prec == "f64" else torch.float32
    A = torch.from_numpy(A64).to(dev, dt)
    B = torch.from_numpy(B64).to(dev, dt)
    ref = A.double() @ B.double()
    if checkpoints is None:
        checkpoints = sorted(set(int(round(x)) for x in np.logspace(0, np.log10(K), 25)))
    out = {"kind": kind, "n": n, "scheme": scheme, "prec": prec, "mode": mode, "K": K,
           "standard_f32_rel_err": _rel(A.float() @ B.float(), ref), "curves": {}}
    L = rbc.lib()
    for q in qs:
        plan = rbc.Plan(n, n, n, _schemes(scheme, q), prec=prec, leaf_tile=-1)
        C = torch.empty((n, n), dtype=dt, device=dev)
        acc = torch.empty((n, n), dtype=torch.float64, device=dev)
        ws = plan.workspace(dev)
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        curve = []
        for k in range(1, K + 1):
            plan.matmul(A, B, C=C, seed=k - 1, mode=mode, workspace=ws)
            _lib.check(L.rbc_accumulate(ctypes.c_void_p(acc.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                                        int(prec == "f64"), n, n, n, int(k == 1), st))
            if k in checkpoints:
                curve.append((k, _rel(acc / k, ref)))
        out["curves"]["Q%d" % q] = curve
    return out


def error_distribution(kind="gaussian", n=320, qs=(1, 2, 3, 4, 5), trials=100, modes=MODES,
                       scheme="strassen", prec="f32", seed=1):
    import torch
    import paper_1905_07439_amd as rbc
    dev = "cuda:0"
    A64, B64 = matrices(kind, n, seed)
    dt = torch.float64 if prec == "f64" else torch.float32
    A = torch.from_numpy(A64).to(dev, dt)
    B = torch.from_numpy(B64).to(dev, dt)
    ref = A.double() @ B.double()
    out = {"kind": kind, "n": n, "scheme": scheme, "prec": prec, "trials": trials,
           "standard_f32_rel_err": _rel(A.float() @ B.float(), ref), "errors": {}}
    for q in qs:
        plan = rbc.Plan(n, n, n, _schemes(scheme, q), prec=prec, leaf_tile=-1)
        C = torch.empty((n, n), dtype=dt, device=dev)
        ws = plan.workspace(dev)
        for m in modes:
            errs = []
            for t in range(trials if m != "none" else 1):
                plan.matmul(A, B, C=C, seed=t, mode=m, workspace=ws)
                errs.append(_rel(C, ref))
            out["errors"]["Q%d/%s" % (q, m)] = errs
    return out


def paper_runs(trials=100, K=10000, kinds=("gaussian", "uniform", "adversarial1", "adversarial2",
                                              "adversarial3", "hilbert"), log=None):
    """Every experiment of Section 3.1 and 3.2 at the paper's settings, on the GPU:

    * 3.1 error of average: perturbed Strassen (sigma = 1e-3), f64, 80 x 80 Gaussian,
      k = 1..K realizations, Q = 1, 2, 3 (Figure 1);
    * 3.1 distributions: the same ABC, 320 x 320, 100 realizations per Q = 1..5, deterministic
      against fully randomized, for every matrix kind (Figures 2, 3 and the appendix);
    * 3.2 error of average: Strassen in f32, 80 x 80 Gaussian and Hilbert, k up to K, Q = 1, 2, 3,
      with the standard f32 product beside it (Figures 5, 6);
    * 3.2 distributions: Strassen in f32, 320 x 320, 100 realizations per Q = 1..5 and mode
      (deterministic, full, sign, permutation), every matrix kind (Figures 7-12).

    Returns a dict of the raw results (curves and per-trial errors)."""
    out = {}

    def say(msg):
        if log:
            log(msg)

    say("3.1 error of average")
    out["s31_average"] = error_of_average("gaussian", 80, (1, 2, 3), K, scheme="pert", prec="f64")
    out["s31_dist"] = {}
    for kind in kinds:
        say("3.1 distribution " + kind)
        out["s31_dist"][kind] = error_distribution(kind, 320, (1, 2, 3, 4, 5), trials, ("none", "full"),
                                                   scheme="pert", prec="f64")
    out["s32_average"] = {}
    for kind in ("gaussian", "hilbert"):
        say("3.2 error of average " + kind)
        out["s32_average"][kind] = error_of_average(kind, 80, (1, 2, 3), K, scheme="strassen", prec="f32")
    out["s32_dist"] = {}
    for kind in kinds:
        say("3.2 distribution " + kind)
        out["s32_dist"][kind] = error_distribution(kind, 320, (1, 2, 3, 4, 5), trials, MODES, scheme="strassen",
                                                   prec="f32")
    return out


def _fmt(x):
    return "%.3g" % x


def paper_report(res):
    """Markdown summary of paper_runs: medians and quartiles of the distributions, the
    error-of-average curves at a few k."""
    lines = []
    a = res["s31_average"]
    lines.append("## Section 3.1, error of average (perturbed Strassen, sigma = 1e-3, f64, 80 x 80 Gaussian)")
    lines.append("")
    ks = [k for k, _ in a["curves"]["Q1"]]
    pick = [k for k in ks if k in (1, 10, 100, 1000, 10000)] or ks[:: max(1, len(ks) // 5)]
    lines.append("| Q | " + " | ".join("k = %d" % k for k in pick) + " |")
    lines.append("|---|" + "---|" * len(pick))
    for q, curve in sorted(a["curves"].items()):
        d = dict(curve)
        lines.append("| %s | " % q[1:] + " | ".join(_fmt(d[k]) for k in pick) + " |")
    lines.append("")
    for sec, key, modes in (("3.1", "s31_dist", ("none", "full")), ("3.2", "s32_dist", MODES)):
        what = ("perturbed Strassen (sigma = 1e-3), f64" if sec == "3.1" else "Strassen, f32 (standard f32 product "
                "for reference)")
        lines.append("## Section %s, error of %d realizations per Q, 320 x 320 (%s)" % (sec, res["trials"], what))
        lines.append("")
        lines.append("Relative Frobenius error against the f64 standard product: deterministic (one value), "
                     "then median [q1, q3] over the realizations for each randomized mode.")
        lines.append("")
        lines.append("| matrices | Q | " + " | ".join(modes) + (" | standard f32 |" if sec == "3.2" else " |"))
        lines.append("|---|---|" + "---|" * (len(modes) + (1 if sec == "3.2" else 0)))
        for kind, r in res[key].items():
            for q in (1, 2, 3, 4, 5):
                cells = []
                for m in modes:
                    e = r["errors"]["Q%d/%s" % (q, m)]
                    if m == "none":
                        cells.append(_fmt(e[0]))
                    else:
                        sm = summarize(e)
                        cells.append("%s [%s, %s]" % (_fmt(sm["median"]), _fmt(sm["q1"]), _fmt(sm["q3"])))
                std = (" | " + _fmt(r["standard_f32_rel_err"])) if sec == "3.2" else ""
                lines.append("| %s | %d | %s%s |" % (kind, q, " | ".join(cells), std))
        lines.append("")
    lines.append("## Section 3.2, error of average (Strassen, f32, 80 x 80)")
    lines.append("")
    for kind, a in res["s32_average"].items():
        ks = [k for k, _ in a["curves"]["Q1"]]
        pick = [k for k in ks if k in (1, 10, 100, 1000, 10000)] or ks
        lines.append("%s (standard f32 product: %s)" % (kind, _fmt(a["standard_f32_rel_err"])))
        lines.append("")
        lines.append("| Q | " + " | ".join("k = %d" % k for k in pick) + " |")
        lines.append("|---|" + "---|" * len(pick))
        for q, curve in sorted(a["curves"].items()):
            d = dict(curve)
            lines.append("| %s | " % q[1:] + " | ".join(_fmt(d[k]) for k in pick) + " |")
        lines.append("")
    return "\n".join(lines)


def summarize(errs):
    e = np.asarray(errs, dtype=np.float64)
    return {"median": float(np.median(e)), "q1": float(np.percentile(e, 25)), "q3": float(np.percentile(e, 75)),
            "min": float(e.min()), "max": float(e.max())}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--experiment", choices=["average", "distribution", "paper"], required=True)
    ap.add_argument("--kind", default="gaussian")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--K", type=int, default=10000)
    ap.add_argument("--trials", type=int, default=100)
    ap.add_argument("--scheme", default="")
    ap.add_argument("--prec", default="")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    if a.experiment == "paper":  # every experiment of Sections 3.1 and 3.2; markdown to --out
        res = paper_runs(trials=a.trials, K=a.K, log=lambda m: print(m, file=sys.stderr, flush=True))
        res["trials"] = a.trials
        text = paper_report(res)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
            with open(a.out + ".json", "w") as f:
                json.dump(res, f)
        else:
            print(text)
        return 0
    if a.experiment == "average":
        res = error_of_average(a.kind, a.n or 80, K=a.K, scheme=a.scheme or "pert", prec=a.prec or "f64")
    else:
        res = error_distribution(a.kind, a.n or 320, trials=a.trials, scheme=a.scheme or "strassen",
                                 prec=a.prec or "f32")
        res["summary"] = {k: summarize(v) for k, v in res["errors"].items()}
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
