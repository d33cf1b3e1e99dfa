"""CPU checks of the benchmark script's contract (no GPU needed).

`bench.py --gpus N` with N > 1 must refuse with exit status 2 (one GPU is
measured; there is no multi-GPU path), and the CPU-baseline record must carry
the fields the JSON line promises (value, unit, cores, kind "oracle", sample),
timed here on a tiny workload.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_record_fields():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1907_04834_amd import workloads as W

    w = W.ellipsoid_20k(seed=3, n=1500)
    rec = bench.cpu_baseline(w, 0.5, 16, exact_interactions=41 * 1500 ** 2,
                             bh_interactions=10 ** 6, targets=100)
    assert rec["unit"] == "pair-interactions/s" and rec["kind"] == "oracle"
    assert rec["value"] > 0 and rec["exact_pairs_per_s"] > 0 and rec["bh_interactions_per_s"] > 0
    assert isinstance(rec["cores"], int) and rec["cores"] >= 1
    assert "100 random targets x 1500 sources" in rec["sample"]
    # the step estimate is the two legs at their measured rates
    t = 41 * 1500 ** 2 / rec["exact_pairs_per_s"] + 10 ** 6 / rec["bh_interactions_per_s"]
    assert rec["step_seconds_extrapolated"] == pytest.approx(t)
