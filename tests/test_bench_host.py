"""Host logic of bench.py (no GPU): the committed counter summaries belong to
the current kernel sources, the traffic lookup takes the summary of the
schedule that ran, more than one GPU is refused, and the AMR method is
timed only without the CPU legs."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def summaries():
    d = os.path.join(ROOT, "profiles")
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith("_traffic.json")]


def test_counter_summaries_match_the_kernel_sources():
    """A kernel change without new counters would make the bench report no
    traffic: every committed summary carries the hash of today's sources."""
    files = summaries()
    assert files
    for f in files:
        assert json.load(open(f))["source_hash"] == bench.source_hash(), os.path.basename(f)


def test_traffic_lookup_by_schedule():
    cells = 1000.0
    for sched in (4, 5):
        t, src = bench.traffic_from_profile("quad2d_adaptive5", "fp32", "k_fv_stage", cells, sched)
        d = json.load(open(os.path.join(ROOT, "profiles", f"k_fv_stage_quad2d_adaptive5_fp32_s{sched}_traffic.json")))
        assert d["schedule"] == sched and f"_s{sched}_" in src
        assert t == pytest.approx(d["traffic_bytes_per_cell_stage"] * cells)
    # the strip kernels' summaries carry no schedule in their names
    t, src = bench.traffic_from_profile("quad2d_batch512", "fp32", "k_fv_strip", cells, 8)
    assert t is not None and src.startswith(os.path.join("profiles", "k_fv_strip_quad2d_batch512_fp32_traffic.json"))
    assert bench.traffic_from_profile("quad2d_uniform128", "fp64", "k_fv_stage", cells, 4) == (None, "no counter summary")


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_amr_scheme_needs_no_cpu():
    """The CPU baseline and the error report run the MR scheme, so timing the
    AMR method asks for --no-cpu before anything touches the GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--scheme", "amr"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "--no-cpu" in r.stderr and r.stdout == ""


def test_amr_scheme_only_where_set_up():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--scheme", "amr", "--no-cpu", "--workload",
                        "ellip3d_uniform256"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "ellip3d_uniform256" in r.stderr and r.stdout == ""
