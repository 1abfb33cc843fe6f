"""Host logic of the autotuner: candidate depths and tiles, depth transfer between sizes, cache."""

import json

import paper_1905_07439_amd as rbc
from paper_1905_07439_amd.tune import Tuner


def test_candidates_keep_leaves_in_range_and_pad_little():
    t = Tuner(min_leaf=48, max_leaf=1024, max_pad=1.25)
    S, L = rbc.Scheme.builtin("strassen"), rbc.Scheme.builtin("laderman")
    for n in (256, 1000, 4096):
        for sch, b in ((S, 2), (L, 3)):
            cands = t.candidates(n, n, n, sch, "fp8c")
            assert cands and all(q >= 1 for q, _ in cands)
            for q, tile in cands:
                leaf = -(-n // b ** q)
                assert leaf <= 1024 and leaf >= 24
                if tile:
                    assert tile in (32, 64, 96, 128) and -(-leaf // tile) * tile <= 1.25 * leaf
            assert {q for q, tile in cands if tile == 0} == {q for q, _ in cands}
    assert t.candidates(4096, 4096, 4096, L, "f32", tiles=False) == [(2, 0), (3, 0), (4, 0)]


def test_depth_for_transfers_the_leaf_side(monkeypatch):
    t = Tuner(min_leaf=48)
    S = rbc.Scheme.builtin("strassen")
    chosen = {256: 1, 512: 1, 1024: 1, 2048: 1, 4096: 2}  # leaves 128, 256, 512, 1024, 1024
    monkeypatch.setattr(t, "choose", lambda g, *a, **k: {"levels": chosen[g], "tile": 0, "ms": 1.0})
    assert t.depth_for(4096, S, "fp8c", "strassen") == 2
    assert t.depth_for(3000, S, "fp8c", "strassen") == 2    # nearest grid 4096: leaf 1024 -> 750
    assert t.depth_for(2048, S, "fp8c", "strassen") == 1
    assert t.depth_for(160, S, "fp8c", "strassen") == 1     # never below one level
    assert t.depth_for(700, S, "fp8c", "strassen") == 1     # nearest 512: leaf 256 -> 350


def test_cache_file_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "tune.json")
    t = Tuner(path=path)
    monkeypatch.setattr(t, "_device_name", lambda: "gfx950")
    k = t.key(512, 512, 512, "strassen", "f16s")
    t.cache[k] = {"levels": 1, "tile": 64, "ms": 0.03}
    t.save()
    assert json.load(open(path))[k]["tile"] == 64
    t2 = Tuner(path=path)
    monkeypatch.setattr(t2, "_device_name", lambda: "gfx950")
    assert t2.choose(512, 512, 512, None, "f16s", "strassen") == {"levels": 1, "tile": 64, "ms": 0.03}
