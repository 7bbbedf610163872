"""The autotuner's choice among timed launch shapes (host logic, CPU only):
candidates come in order of preference and a later one wins only when it is
faster than the current choice by more than the timing noise."""
from paper_1612_03399_amd.autotune import choose


def r(name, ms):
    return {"options": {"name": name}, "ms": ms}


def test_first_candidate_kept_within_noise():
    assert choose([r("a", 1.00), r("b", 0.99), r("c", 0.985)])["options"]["name"] == "a"


def test_clearly_faster_candidate_wins():
    assert choose([r("a", 1.00), r("b", 0.90)])["options"]["name"] == "b"


def test_comparison_is_against_the_current_choice():
    # b beats a by 5%; c is 1.5% faster than b, within noise, so b stays
    assert choose([r("a", 1.00), r("b", 0.95), r("c", 0.936)])["options"]["name"] == "b"
    # d beats b by more than the margin
    assert choose([r("a", 1.00), r("b", 0.95), r("d", 0.90)])["options"]["name"] == "d"


def test_margin_is_a_parameter():
    assert choose([r("a", 1.00), r("b", 0.99)], margin=0.0)["options"]["name"] == "b"


# ---- the staged search and its cache (host logic) ----

import json  # noqa: E402

from paper_1612_03399_amd import autotune as AT  # noqa: E402
from paper_1612_03399_amd import workload as W  # noqa: E402


def test_stage_candidates_extend_the_best_shape():
    best1 = {"threads": 384, "wg_per_cu": 2}
    c2 = AT.staged_candidates(best1)
    assert len(c2) == len(AT.STAGE2)
    assert all(c["threads"] == 384 and c["wg_per_cu"] == 2 for c in c2)
    assert {"threads": 384, "wg_per_cu": 2, "unit_nodes": 384} in c2
    best2 = c2[0]
    c3 = AT.staged_candidates(best1, best2)
    assert all(dict(c, tile_bytes=None) == dict(best2, tile_bytes=None) for c in c3)
    assert {c["tile_bytes"] for c in c3} == {s["tile_bytes"] for s in AT.STAGE3}


def test_signature_separates_workloads_and_precisions():
    a = W.small_suspension(4, 2, 32)
    b = W.small_suspension(4, 3, 32)
    c = W.small_suspension(5, 2, 32)
    sig = lambda m, p="f64": AT.signature(m, m.grid, p)
    assert sig(a) == sig(W.small_suspension(4, 2, 32))       # same shape, same key
    assert len({sig(a), sig(b), sig(c), sig(a, "f32")}) == 4


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("IPIBM_TUNE_CACHE", str(tmp_path / "tune.json"))
    assert AT.cache_load() == {}
    AT.cache_store("k1", {"options": {"threads": 384}, "results": []})
    AT.cache_store("k2", {"options": {}, "results": [{"ms": 1.0}]})
    data = json.load(open(tmp_path / "tune.json"))
    assert data["k1"]["options"] == {"threads": 384} and data["k2"]["results"] == [{"ms": 1.0}]
    assert AT.cache_load() == data
