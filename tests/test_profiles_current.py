"""The committed HBM-counter summaries that bench.py reports as `traffic`
were taken on the current kernel sources: each summary records the sha256
of the sources it was taken on, and bench.py drops the figure when they
differ.  This keeps a source change from silently turning the reported
traffic into null; the fix is to re-take the counters (the commands are in
each summary)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("path,sources", [
    (bench.traffic_file("fp32c"), bench.QUAD_SOURCES),
    (bench.traffic_file("fp32"), bench.QUAD_SOURCES),
    (os.path.join(ROOT, "profiles", "fwd_stream_n2_two_level_2p24_traffic.txt"), bench.STREAM_SOURCES),
    (os.path.join(ROOT, "profiles", "fwd_tmz_n3_fp64_2d_beam_traffic.txt"), bench.TMZ_SOURCES),
    (os.path.join(ROOT, "profiles", "fwd_tmz_n3_fp32c_2d_beam_traffic.txt"), bench.TMZ_SOURCES),
])
def test_traffic_summary_matches_sources(path, sources):
    assert os.path.exists(path), path
    got = bench.measured_traffic(None, path, sources)
    assert got is not None and got > 0, f"{os.path.basename(path)} was taken on other kernel sources"
