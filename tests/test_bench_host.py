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
    # the summary under profiles/ was taken for the current sources (FP32, 2 lanes), and is
    # not offered for another configuration
    t = bench.measured_traffic("fp32", 2)
    assert t is not None and 5e7 < t < 1e8
    assert bench.measured_traffic("fp64", 2) is None
    assert bench.measured_traffic("fp32", 4) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr
