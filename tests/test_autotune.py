"""Host logic of the launch-configuration autotuner (no GPU: the step timing is
replaced by a given function)."""
import itertools
import json

import numpy as np

import scenegen as sg
from paper_2505_13215_amd.autotune import CANDIDATES, Autotuner, workload_key


def _sets(n3, n4):
    return {"opacity": np.zeros(n3, np.float32)}, {"opacity": np.zeros(n4, np.float32)}


def _views():
    return [sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 1352, 1014),
            sg.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 2704, 2028)]


def test_candidates_are_every_built_pair():
    assert set(CANDIDATES) == set(itertools.product((8, 16, 32), (64, 128, 256, 512)))
    assert len(CANDIDATES) == 12


def test_key_buckets_counts_and_sorts_sizes():
    k1 = workload_key("gfx950", 175_000, 75_000, [(2704, 2028), (1352, 1014)], True)
    k2 = workload_key("gfx950", 200_000, 100_000, [(1352, 1014), (2704, 2028)], True)
    assert k1 == k2  # same power-of-two buckets, same multiset of sizes
    assert "n3<=262144" in k1 and "n4<=131072" in k1
    assert workload_key("gfx950", 175_000, 75_000, [(1352, 1014)], True) != k1
    assert workload_key("gfx950", 175_000, 75_000, [(2704, 2028), (1352, 1014)], False) != k1
    assert workload_key("gfx942", 175_000, 75_000, [(2704, 2028), (1352, 1014)], True) != k1
    assert "n3<=0" in workload_key("gfx950", 0, 10, [(8, 8)], False)


def test_pick_is_the_fastest_and_cached():
    calls = []
    cost = {tc: 10.0 + i for i, tc in enumerate(CANDIDATES)}
    cost[(32, 256)] = 1.5

    def timer(t, c):
        calls.append((t, c))
        return cost[(t, c)]

    tuner = Autotuner(timer=timer)
    g3, g4 = _sets(1000, 500)
    assert tuner.pick(g3, g4, _views(), True, arch="gfx950") == (32, 256)
    assert sorted(calls) == sorted(CANDIDATES)
    assert tuner.last_timings[(32, 256)] == 1.5
    # the same workload again: no new timing
    assert tuner.pick(g3, g4, _views(), True, arch="gfx950") == (32, 256)
    assert len(calls) == len(CANDIDATES)
    # another key is timed afresh
    tuner.pick(g3, g4, _views()[:1], True, arch="gfx950")
    assert len(calls) == 2 * len(CANDIDATES)


def test_ties_break_to_the_smallest_pair():
    tuner = Autotuner(timer=lambda t, c: 1.0)
    g3, g4 = _sets(10, 10)
    assert tuner.pick(g3, g4, _views(), False, arch="gfx950") == min(CANDIDATES)


def test_cache_file_round_trip(tmp_path):
    f = str(tmp_path / "tune.json")
    g3, g4 = _sets(5000, 2000)
    t1 = Autotuner(cache_file=f, timer=lambda t, c: abs(t - 8) + abs(c - 128) / 64.0)
    assert t1.pick(g3, g4, _views(), True, arch="gfx950") == (8, 128)
    data = json.load(open(f))
    assert list(data.values()) == [[8, 128]]

    def fail(t, c):
        raise AssertionError("a cached workload is not timed again")

    t2 = Autotuner(cache_file=f, timer=fail)
    assert t2.pick(g3, g4, _views(), True, arch="gfx950") == (8, 128)


def test_rejected_candidates_are_skipped():
    from paper_2505_13215_amd import H4DError
    from paper_2505_13215_amd._lib import H4D_ERR_CAPACITY

    def timer(t, c):
        if t == 8:
            raise H4DError(H4D_ERR_CAPACITY, "pair_capacity too large")
        return float(c) + t

    tuner = Autotuner(timer=timer)
    g3, g4 = _sets(10, 10)
    assert tuner.pick(g3, g4, _views(), True, arch="gfx950") == (16, 64)
    assert all(tuner.last_timings[(8, c)] == float("inf") for c in (64, 128, 256, 512))
    none = Autotuner(timer=lambda t, c: timer(8, c))
    try:
        none.pick(g3, g4, _views(), True, arch="gfx950")
    except H4DError as e:
        assert e.code == H4D_ERR_CAPACITY
    else:
        raise AssertionError("a workload no configuration fits raises")
