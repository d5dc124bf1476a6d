"""The committed rocprofv3 summaries describe the kernels as they are.

bench.py reads the HBM traffic of its roofline kernel from
profiles/hbm_traffic.json only while the recorded hash of the kernel sources
matches; these checks keep the summaries and the sources in step, and check
that every summary states the command that produced it.
"""
import hashlib
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROF = os.path.join(ROOT, "profiles")


def _traffic():
    path = os.path.join(PROF, "hbm_traffic.json")
    if not os.path.exists(path):
        pytest.skip("no traffic summary committed")
    return json.load(open(path))


def test_stale_traffic_is_not_reported():
    """The benchmark reports counter traffic only for the kernel sources the
    counters were taken on: after any kernel change it reports null."""
    import bench
    rec = _traffic()
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    got = bench.counter_traffic(rec["workload"], rec["h"], rec["likelihood"], "propagate")
    if h.hexdigest()[:16] == rec["source_sha256_16"]:
        assert got == round(rec["per_launch"]["propagate"]["traffic_bytes"], 0)
    else:
        assert got is None


def test_traffic_summary_covers_the_roofline_kernels():
    rec = _traffic()
    for k in ("propagate", "bin_sums", "keys", "cdf_scan", "resample"):
        assert k in rec["per_launch"], k
        assert rec["per_launch"][k]["traffic_bytes"] > 0
    # calibrated by a plain copy: FETCH_SIZE reads half the bytes on this chip, WRITE_SIZE all of them
    assert 1.9 < rec["fetch_scale"] < 2.1 and 0.95 < rec["write_scale"] < 1.05


def test_summaries_state_their_commands():
    names = [f for f in os.listdir(PROF) if f.endswith(".md")]
    assert names
    for f in names:
        text = open(os.path.join(PROF, f)).read()
        assert "rocprofv3" in text and "bench.py" in text, f
