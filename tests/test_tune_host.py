"""Host logic of the autotuner (no GPU): the coordinate search and the cache key."""
from paper_2208_14567_amd.tune import SPACE, cache_key, coordinate_search


def test_coordinate_search_finds_separable_minimum():
    target = {"waves32": 4, "refill_min": 16, "chunk": 64, "spread": 0, "refill64": 8, "deesc": 8, "drain32": 12,
              "sort_esc": 1, "wave64": 2}
    calls = []

    def cost(cfg):
        calls.append(dict(cfg))
        return sum((cfg[k] - target[k]) ** 2 for k in cfg)

    start = {k: v[0] for k, v in SPACE.items()}
    best, t, n = coordinate_search(cost, SPACE, start)
    assert best == target and t == 0 and n == len(calls)
    # one round over every value, plus a confirming round at most
    assert n <= 1 + 2 * sum(len(v) - 1 for v in SPACE.values())


def test_coordinate_search_keeps_start_when_nothing_helps():
    start = {k: v[0] for k, v in SPACE.items()}
    best, t, n = coordinate_search(lambda c: 1.0, SPACE, start)
    assert best == start and t == 1.0


def test_cache_key_classes():
    a = cache_key("MI355X", 20, 1_000_000, 200, 0)
    assert a == cache_key("MI355X", 20, 1_100_000, 200, 0)   # same size class
    assert a != cache_key("MI355X", 20, 4_000_000, 200, 0)
    assert a != cache_key("MI355X", 20, 1_000_000, 50, 0)
    assert a != cache_key("MI355X", 13, 1_000_000, 200, 0)
