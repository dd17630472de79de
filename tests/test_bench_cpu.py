"""bench.py's host side, without a GPU: the algorithmic byte counts behind
`roofline.achieved`, the roofline helper, and the argument checks that must
refuse a run before anything touches a device."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FP64, FP32 = 0, 1


@pytest.mark.parametrize("prec,flat,curved", [(FP32, 64, 88), (FP64, 128, 176)])
def test_bytes_per_step_are_the_minimum_traffic_of_the_step(prec, flat, curved):
    # one state read and one write per direction; curved adds E (read once
    # thanks to the Step 5 / Step 1 seam in x) and a (read in both directions)
    per = lambda kind: sum(bench.bytes_per_point(kind, d, prec) for d in (0, 1))
    assert per("flat") == flat
    assert per("flat_pml") == flat            # 1/S is a per-axis table, not per point
    assert per("curved") == curved
    sz = 4 if prec == FP32 else 8
    assert bench.bytes_per_point("curved", 0, prec) - bench.bytes_per_point("curved", 1, prec) == 4 * sz


def test_variant_roofline_takes_the_slower_direction():
    r = bench.variant_roofline(1000, (100, 50), (10.0, 20.0), "note")
    assert r["kernel"] == "y_stage" and r["bytes_per_point"] == 50 and r["avg_launch_us"] == 20.0
    ach = 50 * 1000 / 20e-6 / 1e9
    assert r["achieved"] == pytest.approx(ach, abs=0.05)
    assert r["frac"] == pytest.approx(ach / bench.HBM_PEAK_GBS, abs=1e-4)
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s"


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_variant_names_are_refused():
    r = _run("--variants", "curved_512_fp64,no_such_variant")
    assert r.returncode == 2
    assert "no_such_variant" in r.stderr and r.stdout == ""


def test_host_baseline_runs_the_oracle_over_a_process_pool():
    from paper_1909_02894_amd import workloads as W
    r = bench.cpu_baseline_batch(W, 2, 3)
    assert r["kind"] == "oracle" and r["cores"] == 3 and r["unit"] == "grid-point*steps/s"
    assert r["value"] > 0 and r["seconds"] > 0
    sizes = [W.batch_mix(256, 4000, bench.BATCH_SIZES, 2)[i].n1 for i in range(3)]
    assert r["value"] == pytest.approx(sum(n * n * 2 for n in sizes) / r["seconds"], rel=0.02)
    assert "first 3 solves" in r["sample"]
