"""GPU checks of averages of products (the error-of-average quantity of Section 3) and of
the error-study harness.

* Averaging every draw of one level of a perturbed-Strassen ABC (kappa != 0, with the
  (1 - kappa)^-1 factor) gives A B up to f64 rounding: the expectation result, checked by
  enumerating all 512 draws on the device.
* The device's seeded average equals the oracle's float64 average of the same seeds.
* The error of the average of K realizations falls as K grows.
"""

import sys

import numpy as np
import pytest
import torch

import paper_1905_07439_amd as rbc
import workloads
from oracle import expectation, recursion, schemes as osch
from paper_1905_07439_amd import study

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pert():
    S = rbc.Scheme.builtin("strassen")
    P = rbc.Scheme.builtin("perturbed_strassen", 1e-3, 42)
    return P, tuple(np.asarray(x) for x in P.tensors())


def test_average_over_every_draw_is_the_product():
    P, ref = _pert()
    assert abs(P.info()["kappa"]) > 0
    n = 64
    A = workloads.gaussian((n, n), 7101)
    B = workloads.gaussian((n, n), 7102)
    plan = rbc.Plan(n, n, n, [P], prec="f64")
    draws = []
    for s1, s2, s3, p1, p2, p3 in expectation.all_draws(2, 2, 2):
        draws.append((np.concatenate([s1, s2, s3]).astype(np.int32), np.concatenate([p1, p2, p3]).astype(np.int32)))
    assert len(draws) == 512
    Ad, Bd = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    avg = plan.average_over_draws(Ad, Bd, draws).cpu().numpy()
    AB = A @ B
    e = np.linalg.norm(avg - AB) / np.linalg.norm(AB)
    single = recursion.rel_err(plan.matmul_draws(Ad, Bd, draws[5][0], draws[5][1]).cpu().numpy(), AB)
    _say("mean over all draws: rel err %.3g (one draw %.3g)" % (e, single))
    assert e < 1e-12 and single > 1e-5
    want = expectation.mean_over_draws(lambda dr: recursion.rbc(A, B, [ref], [dr]), 2, 2, 2)
    assert np.linalg.norm(avg - want) / np.linalg.norm(want) < 1e-13


def test_seeded_average_matches_oracle():
    P, ref = _pert()
    n = 80
    A = workloads.gaussian((n, n), 7201)
    B = workloads.gaussian((n, n), 7202)
    plan = rbc.Plan(n, n, n, [P, P], prec="f64")
    seeds = list(range(8))
    got = plan.matmul_average(torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV), seeds).cpu().numpy()
    dims = (plan.info["mM"], plan.info["mK"], plan.info["mN"])
    want = sum(recursion.rbc_seeded(A, B, [ref, ref], s, leaf_dims=dims) for s in seeds) / len(seeds)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


def test_error_of_average_falls_with_k():
    res = study.error_of_average("gaussian", n=80, qs=(1,), K=1024, checkpoints=(1, 1024), scheme="pert",
                                 prec="f64")
    (k1, e1), (k2, e2) = res["curves"]["Q1"]
    _say("error of average: K=1 %.3g, K=1024 %.3g" % (e1, e2))
    assert (k1, k2) == (1, 1024) and e2 < e1 / 8


def test_error_distribution_harness():
    res = study.error_distribution("hilbert", n=64, qs=(1, 2), trials=4)
    assert set(res["errors"]) == {"Q%d/%s" % (q, m) for q in (1, 2) for m in study.MODES}
    for k, v in res["errors"].items():
        assert all(np.isfinite(v)) and all(0 < x < 1e-3 for x in v), k
    assert len(res["errors"]["Q1/none"]) == 1 and len(res["errors"]["Q1/full"]) == 4


def _pert_levels(q):
    return [osch.perturbed(*osch.strassen(), 1e-3, 42)] * q


@pytest.mark.parametrize("kind", ["gaussian", "adversarial1", "hilbert"])
def test_error_distribution_matches_oracle(kind):
    # The harness's per-trial errors (Section 3.1 setting: perturbed Strassen, f64) against
    # the errors of the oracle's F-hat^(Q) on the same draws (trial t = algorithm seed t),
    # for Q = 1..3 and the four modes.  The errors are ~1e-3 (algorithmic); a wrong draw,
    # mode or fold would move them far more than the 1e-12 allowed.
    # n = 80 as in the paper: exact blocks, so the oracle's own (unpadded) block structure
    n = 80
    res = study.error_distribution(kind, n=n, qs=(1, 2, 3), trials=3, scheme="pert", prec="f64")
    A, B = study.matrices(kind, n, 1)
    AB = A @ B
    for q in (1, 2, 3):
        for m in study.MODES:
            errs = res["errors"]["Q%d/%s" % (q, m)]
            assert len(errs) == (1 if m == "none" else 3)
            for t, e in enumerate(errs):
                C = recursion.rbc_seeded(A, B, _pert_levels(q), t, m)
                e_or = recursion.rel_err(C, AB)
                assert e_or > 1e-6 and abs(e - e_or) <= 1e-12, (kind, q, m, t, e, e_or)
    _say("error distribution %s matches the oracle; Q3 full %s" % (kind, res["errors"]["Q3/full"]))


@pytest.mark.parametrize("mode", ["full", "signs"])
def test_error_of_average_matches_oracle(mode):
    # The harness's error-of-average curve (eq. error-of-average) against the oracle's average
    # of F-hat over the same seeds 0..k-1, at each checkpoint k.
    n, K = 80, 8
    res = study.error_of_average("adversarial1", n=n, qs=(1, 2, 3), K=K, checkpoints=(1, 2, 5, 8), scheme="pert",
                                 prec="f64", mode=mode)
    A, B = study.matrices("adversarial1", n, 1)
    AB = A @ B
    for q in (1, 2, 3):
        acc = np.zeros((n, n))
        curve = dict(res["curves"]["Q%d" % q])
        for k in range(1, K + 1):
            acc += recursion.rbc_seeded(A, B, _pert_levels(q), k - 1, mode)
            if k in curve:
                e_or = recursion.rel_err(acc / k, AB)
                assert abs(curve[k] - e_or) <= 1e-12 * max(1.0, e_or / 1e-3), (q, k, curve[k], e_or)
