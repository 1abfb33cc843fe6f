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
uniform, adversarial types 1-3, Hilbert).  The truth is the float64 standard
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
        plan = rbc.Plan(n, n, n, _schemes(scheme, q), prec=prec)
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
        plan = rbc.Plan(n, n, n, _schemes(scheme, q), prec=prec)
        C = torch.empty((n, n), dtype=dt, device=dev)
        ws = plan.workspace(dev)
        for m in modes:
            errs = []
            for t in range(trials if m != "none" else 1):
                plan.matmul(A, B, C=C, seed=t, mode=m, workspace=ws)
                errs.append(_rel(C, ref))
            out["errors"]["Q%d/%s" % (q, m)] = errs
    return out


def summarize(errs):
    e = np.asarray(errs, dtype=np.float64)
    return {"median": float(np.median(e)), "q1": float(np.percentile(e, 25)), "q3": float(np.percentile(e, 75)),
            "min": float(e.min()), "max": float(e.max())}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--experiment", choices=["average", "distribution"], required=True)
    ap.add_argument("--kind", default="gaussian")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--K", type=int, default=10000)
    ap.add_argument("--trials", type=int, default=100)
    ap.add_argument("--scheme", default="")
    ap.add_argument("--prec", default="")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
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
