"""CPU test of the format sweep tool (compression ratios only): every
variant encodes, and more interleaved rANS states cost bytes (each state
is 4 bytes of record)."""
import json
import subprocess
import sys
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_format_sweep_ratios():
    out = subprocess.run([sys.executable, "-m", "paper_2308_16619_amd.format_sweep", "--n", "64", "--no-gpu"],
                         cwd=ROOT, capture_output=True, text=True, timeout=300, check=True).stdout
    rows = [json.loads(ln) for ln in out.splitlines() if ln.startswith("{")]
    assert len(rows) == 9
    assert {r["brick"] for r in rows} == {16, 32, 64}
    by_lanes = {r["lane_max"]: r["compressed_bytes"] for r in rows if r["brick"] == 32 and r["scale_bits"] == 10}
    assert by_lanes[1] <= by_lanes[4] <= by_lanes[16] <= by_lanes[64]
    assert all(0 < r["compression_ratio_pct"] < 100 for r in rows)
