"""Host logic of bench.py (no GPU): the rebuild-period fallback, the algorithmic byte
model of the graded force pass, the committed HBM-traffic summary and the one-GPU rule."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_stale_runs_are_void_and_repeated_with_shorter_periods():
    used = []

    def run(k_cap):
        k = 15 if k_cap is None else min(15, k_cap)
        used.append(k)
        if k > 12:  # lists valid only up to a 12-step period
            raise bench.StaleList(k)
        return {"rebuild_every": k}

    r = bench.with_valid_period(run, "test")
    assert used == [15, 14, 13, 12]
    assert r["rebuild_every"] == 12 and r["retries"] == 3


def test_no_valid_period_is_an_error():
    def run(k_cap):
        raise bench.StaleList(1 if k_cap is None else k_cap)

    with pytest.raises(RuntimeError):
        bench.with_valid_period(run)


def test_algorithmic_bytes_of_the_force_pass():
    # per atom: length 4 + list 4 n + own record 32 + force 3 x 4 (FP32) + velocity r/w 48,
    # and with the next kick-drift fused: x_ref 24 + new position record 32
    n, nb = 131072, 71.72
    assert bench.algorithmic_force_bytes(n, nb, 4) == pytest.approx(n * (4 + 4 * nb + 32 + 12 + 48))
    assert bench.algorithmic_force_bytes(n, nb, 4, fused=True) == pytest.approx(
        n * (4 + 4 * nb + 32 + 12 + 48 + 56))
    assert bench.algorithmic_force_bytes(n, nb, 8) - bench.algorithmic_force_bytes(n, nb, 4) == \
        pytest.approx(12 * n)


def test_committed_traffic_summary_matches_the_force_pass_sources():
    # the summary under profiles/ was taken for the current sources (both paths, 2 lanes),
    # and is not offered for another configuration
    for p in ("fp32", "fp64"):
        t = bench.measured_traffic(p, 2)
        assert t is not None and 5e7 < t < 1e8
    assert bench.measured_traffic("fp32", 4) is None
    assert bench.measured_traffic("fp16", 2) is None


def test_committed_valu_counts_match_the_force_pass_sources():
    # the VALU instruction counts beside the HBM roofline come from the counter summary of the
    # current sources: per launch 4096 waves of 1.5k-3k instructions each
    for p in ("fp32", "fp64"):
        v = bench.measured_valu(p, 2)
        assert v is not None and 4096 * 1500 < v < 4096 * 3000
    assert bench.measured_valu("fp32", 4) is None
    assert 6.1e11 < bench.VALU_ISSUE_PEAK < 6.2e11


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("fused", [False, True])
def test_timed_run_is_whole_graphs(fused):
    """Every step count splits into q replays of a main graph of whole graph periods plus at
    most one tail graph, so the timed region never steps eagerly."""
    from paper_2511_22951_amd.sim import graph_period, timed_graph_plan
    for k in range(0, 21):
        P = graph_period(k, fused)
        assert P % max(1, k) == 0 and (not fused or P % 2 == 0)
        for steps in (0, 1, 3, 5, 20, 23, 48, 100, 1000, 1001):
            for gs in (1, 10, 50):
                G, q, r = timed_graph_plan(steps, k, fused, gs)
                assert G % P == 0 and G >= P
                assert q * G + r == steps
                assert (q == 0 and r == steps) or 0 <= r < G
                assert G <= max(P, steps)


def test_rebuild_period_from_the_threshold_warm_up():
    # builds before step 1 (count 1), then at steps 17, 35, 52: shortest interval 17 -> 13
    marks, c = [], 1
    for s in range(1, 121):
        c += s in (17, 35, 52)
        marks.append(c)
    k, at = bench.rebuild_period(marks, base=1)
    assert at == [17, 35, 52] and k == int(0.8 * 17)
    # the cap of a repeated (void) run
    assert bench.rebuild_period(marks, base=1, k_cap=9)[0] == 9
    # no rebuild in 120 steps: the lists stayed valid throughout -> 4/5 of it, at most 20
    assert bench.rebuild_period([1] * 120, base=1) == (20, [])
    assert bench.rebuild_period([1] * 10, base=1) == (8, [])
    # a rebuild on the first warm-up step counts
    assert bench.rebuild_period([2, 2, 2, 3], base=1)[1] == [1, 4]
