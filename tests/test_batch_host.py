"""Host-side checks of the batch engine's task table (no device work is issued).

The persistent kernel takes tasks in queue order and each task waits until
its counters reach their targets.  Executing the table sequentially on the
host must therefore meet every wait when it is reached (dependencies come
first), end with every waited counter exactly at its target, and cover every
stage's pieces exactly once.
"""

import ctypes
from collections import defaultdict

import numpy as np
import pytest

import paper_1905_07439_amd as rbc
from paper_1905_07439_amd import _lib

FAKE = 1 << 20  # never dereferenced: building the table touches no device memory


def _batch(items, **opt):
    L = rbc.lib()
    b = rbc.Batch(**opt)
    for plan, seed, mode in items:
        i = plan.info
        idx = ctypes.c_int64()
        _lib.check(L.rbc_batch_add(b._h, plan._h, ctypes.c_void_p(FAKE), i["K"], ctypes.c_void_p(FAKE),
                                   i["N"], ctypes.c_void_p(FAKE), i["N"], seed, rbc.MODES[mode], 1,
                                   ctypes.byref(idx)))
    return b


def _plan(n, names, prec):
    return rbc.Plan(n, n, n, [rbc.Scheme.builtin(s) for s in names], prec)


def _simulate(table, n_counters):
    cnt = np.zeros(n_counters, np.int64)
    needs = defaultdict(set)
    for t in table:
        for w, nd in zip(t["wait"], t["need"]):
            if w >= 0:
                assert cnt[w] >= nd, "task waits on counter %d (%d < %d) before its producers" % (w, cnt[w], nd)
                needs[int(w)].add(int(nd))
        if t["signal"] >= 0:
            cnt[t["signal"]] += t["count"]
    for w, nds in needs.items():
        assert len(nds) == 1 and cnt[w] == max(nds), (w, nds, cnt[w])
    return cnt


def _coverage(table):
    spans = defaultdict(list)
    for t in table:
        if t["kind"] in (1, 5):  # exponents and gates have no pieces
            continue
        spans[(int(t["kind"]), int(t["param"]), int(t["sub"]))].append((int(t["first"]), int(t["count"])))
    for key, sp in spans.items():
        sp.sort()
        pos = sp[0][0]
        for f, c in sp:
            assert f == pos and c >= 1, key
            pos = f + c
    return spans


F32_ITEMS = [
    (("strassen", "strassen"), 256),
    (("laderman",), 192),
    (("laderman", "strassen"), 384),
    (("strassen", "strassen", "strassen"), 512),
]
F16S_ITEMS = [
    (("laderman",), 192),
    (("laderman", "strassen"), 480),
    (("laderman", "strassen", "strassen"), 768),
    (("laderman", "strassen", "strassen", "strassen"), 1536),
]


@pytest.mark.parametrize("prec,items", [("f32", F32_ITEMS), ("f16s", F16S_ITEMS)])
@pytest.mark.parametrize("window", [1, 3])
def test_task_table_is_topological_and_complete(prec, items, window):
    plans = [_plan(n, names, prec) for names, n in items]
    b = _batch([(p, i, "full") for i, p in enumerate(plans)], window=window)
    ws = b.workspace_bytes
    info = b.info()
    table = b.task_table()
    assert info["n_items"] == len(items) and len(table) == info["n_tasks"]
    assert ws >= sum(p.workspace_bytes for p in plans)
    _simulate(table, info["n_counters"])
    spans = _coverage(table)
    # every product contributes one leaf stage whose pieces cover all its leaf tiles
    leaf_pieces = defaultdict(int)
    for (kind, param, _), sp in spans.items():
        if kind == 3:
            leaf_pieces[param] += sum(c for _, c in sp)
    tiles = sorted(leaf_pieces.values())
    expect = []
    for p in plans:
        t = 64 if prec == "f32" else p.info["tile_m"]
        expect.append(p.info["n_leaves"] * (p.info["mM"] // t) * (p.info["mN"] // t))
    assert tiles == sorted(expect)
    kinds = set(int(k) for k in table["kind"])
    assert {2, 3, 4} <= kinds and ((0 in kinds) == (prec == "f16s"))


@pytest.mark.parametrize("window", [1, 4])
def test_ring_budget_reuses_regions_behind_gates(window):
    plans = [_plan(n, names, "f16s") for names, n in F16S_ITEMS]
    items = [(plans[i % len(plans)], i, "full") for i in range(12)]
    unlimited = _batch(items, window=window)
    biggest = max(p.workspace_bytes for p in plans)
    ring = _batch(items, window=window, item_budget=int(biggest * 1.5))
    ws_u, ws_r = unlimited.workspace_bytes, ring.workspace_bytes
    assert ws_r < ws_u / 2
    iu, ir = unlimited.info(), ring.info()
    assert iu["gate_tasks"] == 0 and ir["gate_tasks"] > 0
    table = ring.task_table()
    _simulate(table, ir["n_counters"])
    _coverage(table)
    # the same work, plus the gates
    for k in (0, 2, 3, 4):
        tu = unlimited.task_table()
        assert tu[tu["kind"] == k]["count"].sum() == table[table["kind"] == k]["count"].sum()
    small = _batch(items, item_budget=biggest // 2)
    with pytest.raises(rbc.RbcError):
        small.workspace_bytes


def _check_regions(b, n_items):
    """Products whose workspace bytes overlap must be ordered: the later one's first
    tasks wait (through its gate tasks, possibly via other products) until the earlier
    one's last stage is complete."""
    table = b.task_table()
    items = [b.item(i) for i in range(n_items)]
    done_of = {it["done_counter"]: k for k, it in enumerate(items)}
    gate_of = {it["gate_counter"]: k for k, it in enumerate(items)}
    waits_on = defaultdict(set)  # item -> items whose completion it waits for directly
    for t in table[table["kind"] == 5]:
        waits_on[gate_of[int(t["signal"])]].add(done_of[int(t["wait"][0])])
    # entry tasks of an item with gates wait on its gate counter with the number of gates
    for k, it in enumerate(items):
        n = len(waits_on[k])
        entry = table[(table["wait"][:, 0] == it["gate_counter"])]
        if n:
            assert len(entry) and (entry["need"][:, 0] == n).all()
        else:
            assert len(entry) == 0

    def after(j, i, seen=None):
        seen = seen or set()
        if i in waits_on[j]:
            return True
        seen.add(j)
        return any(after(k, i, seen) for k in waits_on[j] if k not in seen)

    for i, a in enumerate(items):
        for j, c in enumerate(items):
            if i == j:
                continue
            lo, hi = a["region_offset"], a["region_offset"] + a["region_bytes"]
            lo2, hi2 = c["region_offset"], c["region_offset"] + c["region_bytes"]
            if lo < hi2 and lo2 < hi and a["first_task"] < c["first_task"]:
                assert after(j, i), "product %d reuses bytes of %d without waiting" % (j, i)


@pytest.mark.parametrize("budget_factor", [1.0, 1.3, 1.6, 2.5])
@pytest.mark.parametrize("window", [1, 3, 8])
def test_ring_regions_are_ordered(budget_factor, window):
    plans = [_plan(n, names, "f16s") for names, n in F16S_ITEMS]
    sizes = [0, 3, 1, 2, 3, 0, 2, 1, 3, 2, 0, 1, 3, 3, 1]
    items = [(plans[k], i, "full") for i, k in enumerate(sizes)]
    biggest = max(p.workspace_bytes for p in plans)
    b = _batch(items, window=window, item_budget=int(biggest * budget_factor))
    b.workspace_bytes
    _simulate(b.task_table(), b.info()["n_counters"])
    _check_regions(b, len(items))


@pytest.mark.parametrize("budget_factor", [0, 1.6])
def test_level_groups_respect_dependencies(budget_factor):
    """RBC_BATCH_LEVELS: every task runs at a larger depth than every task it waits on,
    and the grouped launches cover every piece of every working task once."""
    plans = [_plan(n, names, "f16s") for names, n in F16S_ITEMS]
    items = [(plans[i % len(plans)], i, "full") for i in range(9)]
    biggest = max(p.workspace_bytes for p in plans)
    b = _batch(items, mode="levels", item_budget=int(biggest * budget_factor))
    b.workspace_bytes
    info = b.info()
    table = b.task_table()
    assert info["launches"] >= 1 and info["levels"] >= 5
    # recompute depths from the table the same way and compare with a longest-path check
    clevel = {}
    depth = []
    for t in table:
        lv = 0
        for w in t["wait"]:
            if w >= 0:
                lv = max(lv, clevel[int(w)] + 1)
        depth.append(lv)
        if t["signal"] >= 0:
            clevel[int(t["signal"])] = max(clevel.get(int(t["signal"]), -1), lv)
    signalers = defaultdict(list)
    for i, t in enumerate(table):
        if t["signal"] >= 0:
            signalers[int(t["signal"])].append(i)
    for i, t in enumerate(table):
        for w in t["wait"]:
            if w >= 0:
                assert all(depth[j] < depth[i] for j in signalers[int(w)])
    assert max(depth) + 1 == info["levels"]
    work = int(table[table["kind"] != 5]["count"].sum())
    assert work > 0


def test_smaller_tasks_give_more_tasks_same_pieces():
    plans = [_plan(512, ("strassen", "strassen", "strassen"), "f32")]
    big = _batch([(plans[0], 0, "full")], task_bytes=1 << 22)
    small = _batch([(plans[0], 0, "full")], task_bytes=1 << 14)
    big.workspace_bytes, small.workspace_bytes
    tb, ts = big.task_table(), small.task_table()
    assert len(ts) > len(tb)
    for k in (2, 3, 4):
        assert tb[tb["kind"] == k]["count"].sum() == ts[ts["kind"] == k]["count"].sum()


def test_batch_rejects_mixed_precision_and_unsupported_plans():
    L = rbc.lib()
    b = rbc.Batch()
    p32 = _plan(256, ("strassen",), "f32")
    p16 = _plan(256, ("strassen",), "f16s")
    args = lambda p: (b._h, p._h, ctypes.c_void_p(FAKE), 256, ctypes.c_void_p(FAKE), 256,
                      ctypes.c_void_p(FAKE), 256, 0, 0, 1, None)
    _lib.check(L.rbc_batch_add(*args(p32)))
    assert L.rbc_batch_add(*args(p16)) == _lib.RBC_EINVAL
    for prec in ("f64", "bf16x3"):
        p = _plan(256, ("strassen",), prec)
        assert L.rbc_batch_add(*args(p)) == _lib.RBC_EUNSUPPORTED
    p0 = rbc.Plan(256, 256, 256, [], "f32")
    assert L.rbc_batch_add(*args(p0)) == _lib.RBC_EUNSUPPORTED
    naive = rbc.Plan(256, 256, 256, [rbc.Scheme.builtin("naive:2,2,2")], "f32")
    assert L.rbc_batch_add(*args(naive)) == _lib.RBC_EUNSUPPORTED
    assert L.rbc_batch_add(b._h, p32._h, None, 256, ctypes.c_void_p(FAKE), 256, ctypes.c_void_p(FAKE), 256,
                           0, 0, 1, None) == _lib.RBC_EINVAL
    assert L.rbc_batch_add(b._h, p32._h, ctypes.c_void_p(FAKE), 100, ctypes.c_void_p(FAKE), 256,
                           ctypes.c_void_p(FAKE), 256, 0, 0, 1, None) == _lib.RBC_EINVAL
    empty = rbc.Batch()
    assert L.rbc_batch_prepare(empty._h, ctypes.c_void_p(FAKE), 1 << 30, None) == _lib.RBC_EINVAL
    assert L.rbc_batch_launch(empty._h, None, 0) == _lib.RBC_EINVAL


@pytest.mark.parametrize("budget_factor", [0, 1.6])
def test_depth_order_is_topological_and_sorted(budget_factor):
    plans = [(_plan(n, names, "f16s"), i, "full") for i, (names, n) in enumerate(F16S_ITEMS * 2)]
    biggest = max(p.workspace_bytes for p, _, _ in plans)
    ref = _batch(plans, item_budget=int(biggest * budget_factor))
    ref.workspace_bytes
    b = _batch(plans, item_budget=int(biggest * budget_factor), order="depth")
    b.workspace_bytes
    t0, t1 = ref.task_table(), b.task_table()
    assert len(t0) == len(t1)
    # the same tasks, reordered
    key = lambda t: (int(t["kind"]), int(t["variant"]), int(t["param"]), int(t["signal"]), int(t["first"]),
                     int(t["count"]), int(t["sub"]), tuple(int(w) for w in t["wait"]))
    assert sorted(map(key, t0)) == sorted(map(key, t1))
    _simulate(t1, b.info()["n_counters"])
    _coverage(t1)
    depth, clevel = [], {}
    for t in t1:
        lv = max([clevel[int(w)] + 1 for w in t["wait"] if w >= 0] + [0])
        depth.append(lv)
        if t["signal"] >= 0:
            clevel[int(t["signal"])] = max(clevel.get(int(t["signal"]), -1), lv)
    assert depth == sorted(depth)
    for i in range(len(plans)):
        first = b.item(i)["first_task"]
        assert 0 <= first < len(t1)


def test_bad_order_rejected():
    with pytest.raises(rbc.RbcError):
        L = rbc.lib()
        opt = _lib.BatchOptions(order=7)
        h = ctypes.c_void_p()
        _lib.check(L.rbc_batch_create(ctypes.byref(opt), ctypes.byref(h)))
