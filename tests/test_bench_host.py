"""Host-side checks of bench.py (no GPU): the one-GPU refusal, and the use of
the committed rocprofv3 summaries for the measured HBM traffic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2404_08849_amd.profsum import read_record, source_digest  # noqa: E402

PROFILES = os.path.join(ROOT, "profiles")
RECORD_KEYS = {"workload", "kernel", "values_per_lane", "group", "profiler_avg_us",
               "traffic_bytes_per_launch", "fetch_factor", "write_factor", "source_sha256"}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert not any(line.startswith("{") for line in r.stdout.splitlines())   # no bench line


def _summaries():
    return sorted(f for f in os.listdir(PROFILES) if f.endswith(".md"))


def test_every_summary_has_a_complete_record():
    names = _summaries()
    assert names
    for f in names:
        rec = read_record(os.path.join(PROFILES, f))
        assert RECORD_KEYS <= set(rec), f
        # the copy calibration: FETCH_SIZE counts half a byte per byte read
        assert abs(float(rec["fetch_factor"]) - 0.5) < 0.01 and abs(float(rec["write_factor"]) - 1.0) < 0.01
        assert int(rec["traffic_bytes_per_launch"]) > 0
        # the summary is named for its kernel and workload
        assert f.startswith(rec["kernel"] + "_")


@pytest.mark.parametrize("name", _summaries())
def test_recorded_traffic_is_used_only_for_the_same_sources_and_instance(name):
    rec = read_record(os.path.join(PROFILES, name))
    workload = name[len(rec["kernel"]) + 1:-3].replace("_", "-")
    assert workload in bench.WORKLOADS
    vpl, grp = int(rec["values_per_lane"]), int(rec["group"])
    digest = rec["source_sha256"]
    val, src = bench.recorded_traffic(workload, rec["kernel"], (vpl, grp), digest)
    assert val == float(rec["traffic_bytes_per_launch"]) and src.endswith(name)
    # another work-group size: used, with a note
    val, src = bench.recorded_traffic(workload, rec["kernel"], (vpl, grp * 2), digest)
    assert val is not None and "work-group" in src
    # other sources or another instance: no traffic
    assert bench.recorded_traffic(workload, rec["kernel"], (vpl, grp), "0" * 64)[0] is None
    assert bench.recorded_traffic(workload, rec["kernel"], (vpl + 1, grp), digest)[0] is None
    assert bench.recorded_traffic(workload, "k_none", (vpl, grp), digest)[0] is None


def test_source_digest_is_stable():
    d = source_digest()
    assert len(d) == 64 and d == source_digest()


def test_roofline_bound_follows_the_launch_bytes():
    """A launch whose algorithmic bytes exceed the 256 MB MALL is labelled HBM-bound;
    a smaller one is cache-resident; both are read against the streaming kernels."""
    ceil = {"read": 5000.0, "write": 4000.0, "copy": 4500.0}
    kt = {"k": dict(bytes=300e6, bytes_mean=310e6, ms=0.1, ms_in_step=0.11)}
    r = bench.roofline_record(kt, "k", 3000.0, None, "none", ceil)
    assert r["bound"] == "hbm" and r["frac"] == 3000.0 / 8000.0
    assert r["frac_of_copy"] == 3000.0 / 4500.0 and r["frac_of_read"] == 3000.0 / 5000.0
    kt["k"]["bytes"] = 100e6
    assert bench.roofline_record(kt, "k", 3000.0, None, "none", ceil)["bound"] == "cache"


def test_default_workload_is_the_largest_single_gpu_ensemble():
    old = sys.argv
    sys.argv = ["bench.py"]
    try:
        a = bench.parse()
    finally:
        sys.argv = old
    w = bench.WORKLOADS[a.workload]
    assert a.workload == "ens-g7" and w["M"] == 16 and w["level"] == 7 and w["K"] == 30
    assert a.workload in bench.STORED_REFS
