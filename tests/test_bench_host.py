"""Host-side logic of bench.py (CPU): the byte model, the choice of the
binding roof, and the kernel-source hash that ties committed counters to the
sources they were taken from."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_byte_model_per_unit():
    stats = {"steps": 10, "degree_sum": 150, "rays": 2}
    # per visited cell 16 + 8 B plus 4 texels; 16 B per neighbour; 44 B per ray
    assert bench.fwd_step_bytes(stats, 16) == 10 * (24 + 64) + 16 * 150 + 44 * 2
    assert bench.fwd_step_bytes(stats, 8) == 10 * (24 + 32) + 16 * 150 + 44 * 2
    # the adjoint replays the reads, adds 76 B of gradient updates per cell and
    # 32 B per ray instead of 44
    assert bench.bwd_step_bytes(stats, 8) == 10 * (24 + 32 + 76) + 16 * 150 + 32 * 2
    # stored exits: 8 B written per stored step; the adjoint reads them in place
    # of those steps' edge rows (the rest at the mean degree, 15 here)
    assert bench.fwd_step_bytes(stats, 8, 6) == bench.fwd_step_bytes(stats, 8) + 48
    assert bench.bwd_step_bytes(stats, 8, 6) == pytest.approx(
        10 * (24 + 32 + 76) + 16 * 15 * 4 + 8 * 6 + 32 * 2)
    assert bench.bwd_step_bytes(stats, 8, 10) == 10 * (24 + 32 + 76) + 80 + 32 * 2


def _counters(hbm, valu, busy, cycles=1.0e6):
    return {"hbm_bytes_per_launch": hbm, "valu_insts_per_launch": valu, "unit_busy": busy,
            "cycles_per_launch": cycles, "l2_hit_rate": 0.5,
            "_path": os.path.join(ROOT, "profiles", "x.json")}


def test_roofline_takes_the_most_used_roof():
    ms = 1.0
    # HBM: 4 GB in 1 ms = 4 TB/s = 0.5 of peak; VALU and units lower
    r = bench.roofline_of(_counters(4e9, 0.1e9, {"texture_data": 0.3}), ms, 8e9, "k")
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(0.5) and r["unit"] == "GB/s"
    # the texture data unit busier than HBM and VALU issue
    r = bench.roofline_of(_counters(1e9, 0.1e9, {"texture_data": 0.9, "texture_addr": 0.6}),
                          ms, 8e9, "k")
    assert r["bound"] == "texture_data" and r["frac"] == 0.9
    assert r["achieved"] == pytest.approx(0.9) and r["peak"] == pytest.approx(1.0)
    # the byte model only ever appears as the labelled effective figure
    assert r["effective"]["gbs"] == pytest.approx(8000.0)
    assert r["effective"]["frac_of_hbm_peak"] == pytest.approx(1.0)
    # the LDS busier than every other unit
    r = bench.roofline_of(_counters(1e9, 0.1e9, {"texture_data": 0.5, "lds": 0.7}), ms, 8e9, "k")
    assert r["bound"] == "lds" and r["frac"] == 0.7
    # VALU issue: 0.5 G wave instructions in 1 ms against 614.4 G/s
    r = bench.roofline_of(_counters(1e9, 0.5e9, {"texture_data": 0.2}), ms, 8e9, "k")
    assert r["bound"] == "alu" and r["frac"] == pytest.approx(0.5 / 0.6144, rel=1e-3)


def test_roofline_without_counters_reports_none():
    r = bench.roofline_of(None, 2.0, 16e9, "k")
    assert r["bound"] is None and r["frac"] is None and r["traffic"] is None
    assert r["effective"]["gbs"] == pytest.approx(8000.0)


def test_source_hash_ignores_comments_only():
    code = "int f(int x) {\n  return x + 1;\n}\n"
    commented = ("// header\n/* block\n   comment */\nint f(int x) {  // inline\n\n"
                 "  return x + 1;\n}\n")
    assert bench._code_only(code) == bench._code_only(commented)
    assert bench._code_only(code) != bench._code_only(code.replace("+ 1", "+ 2"))


def test_committed_counters_match_the_sources():
    # the roofline in the benchmark line comes from these files: they must
    # describe the kernels as they are built now
    for d in ("fwd", "bwd"):
        c = bench.load_counters(d)
        assert c is not None, f"profiles counters for {d} do not match the kernel sources"
        assert 0.0 < max(c["unit_busy"].values()) <= 1.0
