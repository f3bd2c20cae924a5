"""The committed rocprofv3 summaries describe the committed kernels: their source hashes
match the current kernel sources and their launch shapes match the tuned shapes the bench
launches, so the traffic and counter figures the bench reports next to its live timing
belong to the code that ran (no GPU needed)."""
import os

import bench
from paper_1802_03972_amd.autotune import lookup, lookup_batch
from paper_1802_03972_amd.build import ACCUMULATE_FILES, AUX_FILES, source_sha256

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def machine_lines(name: str) -> dict:
    out = {}
    for line in open(os.path.join(ROOT, "profiles", name)).read().splitlines():
        if ":" in line and not line.startswith(("|", "-", "#", "`", " ")):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def test_single_bunch_profile_matches_sources_and_tuned_shape():
    vals = machine_lines("k_accumulate_single_bunch_fp32.md")
    assert vals["kernel_source_sha256"] == source_sha256(ACCUMULATE_FILES)
    tile = lookup(128, 256, 0)
    assert vals["tile"] == ",".join(str(tile[k]) for k in ("w_per_lane", "dir_per_wave", "waves", "wg_per_cu"))
    got = bench.profile_values("k_accumulate_single_bunch_fp32.md", tile)
    assert got["traffic_bytes_per_launch"] > 0 and got["executed_fp32_flops_per_update"] > 0


def test_batched_profile_matches_sources_and_tuned_shape():
    vals = machine_lines("k_accumulate_batch_batched_uneven.md")
    assert vals["kernel_source_sha256"] == source_sha256(ACCUMULATE_FILES)
    tile = lookup_batch(64, 256, 0)
    assert vals["tile"] == ",".join(str(tile[k]) for k in ("w_per_lane", "dir_per_wave", "waves", "wg_per_cu"))
    got = bench.profile_values("k_accumulate_batch_batched_uneven.md", tile)
    assert got["traffic_bytes_per_launch"] > 0


def test_tracked_profile_matches_sources():
    vals = machine_lines("k_tracked_accumulate_tracked.md")
    assert vals["kernel_source_sha256"] == source_sha256(AUX_FILES)
