"""CPU tests of bench.py's use of the committed counter profiles: the traffic of a
profile is reported only for the kernel sources, workload, tile size and steps
per launch that it was taken with."""
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _profile(workload):
    return open(bench.TILE_PROFILE.format(workload=workload)).read()


def _hash_current(text):
    import hashlib
    h = hashlib.sha256()
    for f in bench.TILE_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_02675_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return re.search(r"kernel-source-sha256-16:\s*([0-9a-f]{16})", text).group(1) == h.hexdigest()[:16]


@pytest.mark.parametrize("workload", ["batched_chains_4096", "batched_chains_65536"])
def test_profile_traffic_reported_only_for_the_profiled_sources(workload):
    text = _profile(workload)
    tb = int(re.search(r"tile_bodies:\s*(\d+)", text).group(1))
    spl = int(re.search(r"steps_per_launch:\s*(\d+)", text).group(1))
    t = bench.tile_traffic(spl, tb, workload)
    if _hash_current(text):
        assert t == float(re.search(r"traffic_bytes_per_launch:\s*(\d+)", text).group(1))
    else:
        assert t is None


def test_traffic_withheld_for_another_configuration():
    if not _hash_current(_profile("batched_chains_4096")):
        pytest.skip("the 4,096-chain profile predates the current kernel sources")
    assert bench.tile_traffic(10, 64, "batched_chains_4096") is not None
    assert bench.tile_traffic(10, 128, "batched_chains_4096") is None
    assert bench.tile_traffic(1, 64, "batched_chains_4096") is None
    assert bench.tile_traffic(10, 64, "batched_chains_100") is None


def test_traffic_below_algorithmic_bytes_at_the_benchmark_size():
    """The counter traffic of a launch is at most its algorithmic bytes (the stores
    of consecutive steps merge in the caches) and at least one load and one store
    of every body (which no schedule can avoid)."""
    text = _profile("batched_chains_4096")
    n = 138557
    t = float(re.search(r"traffic_bytes_per_launch:\s*(\d+)", text).group(1))
    assert (bench.TILE_LOAD_BYTES_PER_BODY + bench.TILE_STORE_BYTES_PER_BODY_STEP) * n <= t
    assert t <= bench.tile_bytes(n, 10)
    assert "k_tile_step" in text
