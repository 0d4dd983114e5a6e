"""Host logic of the autotuner (no GPU): bucketing, the paper's rule as the
prior, the choice among timings, the beta-independent entry and the JSON
round trip."""
import math

from paper_2010_10039_amd import autotune as T


def test_buckets():
    assert T.alpha_class(256) == 8
    assert T.alpha_class(1000) == 10 and T.alpha_class(1024) == 10
    assert T.alpha_class(1025) == 12 and T.alpha_class(4096) == 12
    assert T.alpha_class(8192) == 13 and T.alpha_class(65536) == 16
    assert [T.beta_class(b) for b in (1.0, 1.99, 2.0, 6.4, 8.0, 17.0, 40.0)] == [0, 0, 1, 2, 3, 4, 4]
    assert T.bucket_key(2, 1024, 6.4) == "u16/a10/b2"
    assert T.bucket_key(1, 256, None) == "u8/a8/bany"


def test_paper_rule_prior():
    """floor(log2 beta) + r + 1 = 5 (Sec. 4.3), limited to r in 3..5."""
    for beta in (1.0272, 1.5, 2.7307, 3.9):
        r = T.paper_rule(beta)
        assert r == max(3, min(5, 4 - math.floor(math.log2(beta))))
    assert T.paper_rule(2.7307) == 3
    assert T.paper_rule(1.0272) == 4
    assert T.paper_rule(None) == 4
    assert T.paper_rule(0.5) == 4


def test_pick_prefers_smaller_chunk_within_two_percent():
    times = {(3, 1024): 1.015, (4, 4096): 1.0, (5, 16384): 0.999, (3, 65536): 1.5}
    assert T.Autotuner.pick(times) == (3, 1024)
    times = {(3, 1024): 1.05, (4, 4096): 1.0}
    assert T.Autotuner.pick(times) == (4, 4096)


def test_choose_falls_back_to_any_beta_then_rule(tmp_path):
    t = T.Autotuner()
    t.record("u16/a10/b2", {(3, 1024): 2.0, (4, 4096): 1.0, (5, 4096): 1.5})
    t.record("u16/a10/b1", {(3, 1024): 1.0, (4, 4096): 1.1, (5, 4096): 3.0})
    t.finish()
    assert t.choose(2, 1024, 6.0) == T.Choice(4, 4096, "timed")
    assert t.choose(2, 1024, 3.0) == T.Choice(3, 1024, "timed")
    # unknown beta: r4/c4096 scores 1 + 1.1 = 2.1, r3/c1024 scores 2 + 1 = 3
    assert t.choose(2, 1024, None) == T.Choice(4, 4096, "timed")
    # bucket never timed: the paper's rule
    assert t.choose(2, 4096, 3.0) == T.Choice(3, T.DEFAULT_CHUNK, "rule")
    p = tmp_path / "tune.json"
    t.save(str(p))
    u = T.Autotuner.load(str(p))
    assert u.choose(2, 1024, None) == t.choose(2, 1024, None)
    assert T.Autotuner.load(str(tmp_path / "missing.json")).table == {}
