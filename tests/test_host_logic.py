"""Host-side logic that needs no GPU: the batch autotuner's candidate shapes,
the benchmark's traffic bookkeeping and its refusal of several GPUs."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytest.importorskip("torch")
from paper_1103_4887_amd import autotune  # noqa: E402

import bench  # noqa: E402


def test_batch_candidates_tile_equal_windows_only():
    equal = list(autotune.batch_candidates([4096] * 64, "fp32"))
    uneven = list(autotune.batch_candidates([4096] * 63 + [4000], "fp32"))
    assert (0, 1) in equal and (0, 1) in uneven
    assert any(T > 1 for _, T in equal)
    assert all(T == 1 for _, T in uneven)
    assert all(T == 1 and K in (0, 4) for K, T in autotune.batch_candidates([512] * 8, "fp64"))


def test_traffic_belongs_to_one_kernel_source_and_shape():
    sha = bench.kernel_source_sha256()
    assert len(sha) == 64
    shape = bench.TRAFFIC["launch"]
    per_sweep = bench.TRAFFIC["fetch_bytes_per_sweep"] + bench.TRAFFIC["write_bytes_per_sweep"]
    if sha == bench.TRAFFIC["sweep_source_sha256"]:
        assert bench.traffic_per_launch(shape, 10) == pytest.approx(10 * per_sweep)
    else:
        assert bench.traffic_per_launch(shape, 10) is None
    assert bench.traffic_per_launch((shape[0], shape[1] + 1), 10) is None


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_ncore_oracle_leg_reports_cores_and_model():
    """The N-core oracle leg of the benchmark runs one spawned process per
    core (here at most 2, for a short budget) and reports what it used."""
    import workloads as W

    probs = [W.make_hh_problem(M, 0.02, 101 + M, require_spike=False) for M in (40, 64)]
    old = bench.host_cores
    bench.host_cores = lambda: 2
    try:
        r = bench.cpu_baseline_ncore("sweep", probs, 0.5)
    finally:
        bench.host_cores = old
    assert r["cores"] == 2 and r["kind"] == "oracle"
    assert r["value"] > 0 and r["unit"] == "site-updates/s"
    assert r["cpu_model"] and "M from 40 to 64" in r["sample"]
