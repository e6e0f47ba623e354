"""Host logic of the launch-shape autotuner (no GPU): the candidate shapes, the cache key,
the choice of the minimum, reuse of a cached choice without timing, and the rejection of a
cached choice that is no longer offered.  Timing is a stand-in function."""
import json

from paper_2511_22951_amd import _native as N
from paper_2511_22951_amd import tune


def test_shapes_respect_the_tile_and_fp32_limits():
    s32, s64 = tune.shapes(N.MD_FP32), tune.shapes(N.MD_FP64)
    assert all(b >= 64 * l for l, b in s32 + s64)
    assert all(l <= 8 for l, _ in s32) and (16, 1024) in s64 and (16, 512) not in s64
    assert (2, 256) in s32 and (8, 256) not in s32 and (8, 512) in s32
    assert set(s32) < set(s64)


def test_key_classes():
    k = tune.key("eam", N.MD_FP32, 131072, 71.8)
    assert k == ("eam", "fp32", "n2^17", "nb64")
    assert tune.key("eam", N.MD_FP64, 100000, 80.1) == ("eam", "fp64", "n2^17", "nb80")


def test_pick_times_every_candidate_once_and_takes_the_minimum(tmp_path):
    path = str(tmp_path / "tune.json")
    times = {(1, 1024): 5.0, (2, 1024): 3.0, (2, 512): 2.5, (4, 1024): 2.5}
    calls = []

    def fake(c):
        calls.append(c)
        return times[c]

    cands = list(times)
    best = tune.pick(("w", "fp32"), cands, fake, device_name="dev", cache_path=path)
    assert best == (2, 512)  # ties go to the earlier candidate
    assert sorted(calls) == sorted(cands)
    d = json.load(open(path))
    assert d["dev|w|fp32"]["choice"] == [2, 512]
    # the same key again: the cached shape, no timing
    calls.clear()
    assert tune.pick(("w", "fp32"), cands, fake, device_name="dev", cache_path=path) == (2, 512)
    assert calls == []
    # another device or key is timed afresh
    tune.pick(("w", "fp32"), cands, fake, device_name="dev2", cache_path=path)
    assert len(calls) == len(cands)


def test_a_cached_choice_no_longer_offered_is_timed_again(tmp_path):
    path = str(tmp_path / "tune.json")
    json.dump({"dev|w|fp32": {"choice": [16, 1024], "times": {}}}, open(path, "w"))
    calls = []
    best = tune.pick(("w", "fp32"), [(1, 1024), (2, 1024)], lambda c: calls.append(c) or c[0],
                     device_name="dev", cache_path=path)
    assert best == (1, 1024) and len(calls) == 2
    assert json.load(open(path))["dev|w|fp32"]["choice"] == [1, 1024]


def test_use_cache_false_neither_reads_nor_writes(tmp_path):
    path = str(tmp_path / "tune.json")
    json.dump({"dev|w": {"choice": 4}}, open(path, "w"))
    assert tune.pick(("w",), [1, 2, 4], lambda c: c, use_cache=False, device_name="dev",
                     cache_path=path) == 1
    assert json.load(open(path)) == {"dev|w": {"choice": 4}}
