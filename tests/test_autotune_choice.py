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
