"""Autotuner host logic (no GPU): candidate launch shapes respect LDS and occupancy limits,
and the table lookup keys on the grid shape and arithmetic mode."""
import json

from paper_1802_03972_amd import autotune


def test_candidates_are_valid():
    for nd, no in ((16, 64), (64, 256), (128, 256), (64, 1024), (128, 512)):
        cs = autotune.candidates(nd, no)
        assert cs
        for c in cs:
            assert c["w_per_lane"] in (16, 32) and c["dir_per_wave"] in (16, 32, 64)
            assert 1 <= c["waves"] <= 8 and 1 <= c["wg_per_cu"] <= 8
            assert autotune.lds_bytes(c["w_per_lane"], c["dir_per_wave"], c["waves"]) <= autotune.LDS_LIMIT


def test_lds_formula_matches_the_kernel_layout():
    # geo float4 + tau double per (particle, direction), 11 staged doubles and (N, N^2) per
    # particle, one float per (particle, frequency); 32-particle chunks
    assert autotune.lds_bytes(32, 64, 8) == 32 * 64 * 24 + 32 * 88 + 32 * 8 + 32 * 256 * 4


def test_table_lookup(tmp_path):
    p = tmp_path / "t.json"
    tile = {"w_per_lane": 32, "dir_per_wave": 64, "waves": 8, "wg_per_cu": 1}
    p.write_text(json.dumps({autotune.key(128, 256, 0): {"tile": tile}}))
    assert autotune.lookup(128, 256, 0, str(p)) == tile
    assert autotune.lookup(128, 256, 1, str(p)) is None
    assert autotune.lookup(64, 256, 0, str(tmp_path / "missing.json")) is None


def test_variant_candidates_and_keys():
    from paper_1802_03972_amd import autotune
    for v in (1, 2, 3):
        cs = autotune.candidates(128, 256, variant=v)
        assert cs and all(c["w_per_lane"] == 16 for c in cs)
        assert autotune.key(128, 256, 0, v).endswith(f":v{v}")
    assert autotune.key(128, 256, 0) == "128x256:p0"


def test_confirm_prefers_less_partial_traffic_among_ties():
    from paper_1802_03972_amd import autotune
    a = {"w_per_lane": 16, "dir_per_wave": 16, "waves": 4, "wg_per_cu": 8}
    b = {"w_per_lane": 16, "dir_per_wave": 32, "waves": 8, "wg_per_cu": 2}
    c = {"w_per_lane": 32, "dir_per_wave": 32, "waves": 4, "wg_per_cu": 1}
    times = {str(a): 0.4943, str(b): 0.4980, str(c): 0.60}
    res = [(0.51, a, 0), (0.50, b, 0), (0.59, c, 0)]
    tb = lambda x: autotune.partial_bytes(x, 128, 256, 256)
    assert tb(b) < tb(a)
    out = autotune.confirm(res, lambda x: times[str(x)], lambda ms: 1.0 / ms, False, traffic=tb)
    assert out[0][1] == b                       # within 1 % of the fastest and half the bytes
    out = autotune.confirm(res, lambda x: times[str(x)], lambda ms: 1.0 / ms, False, traffic=tb, tie=0.001)
    assert out[0][1] == a                       # no tie: the fastest wins
