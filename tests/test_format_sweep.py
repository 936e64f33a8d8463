"""CPU test of the format sweep tool (sizes only): every variant encodes;
the no-rANS container is the oracle's raw-nibble container; more
interleaved rANS states cost bytes (each state is 4 bytes of record)."""
import json
import os
import subprocess
import sys

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_format_sweep_ratios(orc):
    out = subprocess.run([sys.executable, "-m", "paper_2308_16619_amd.format_sweep", "--n", "64", "--no-gpu"],
                         cwd=ROOT, capture_output=True, text=True, timeout=300, check=True).stdout
    rows = [json.loads(ln) for ln in out.splitlines() if ln.startswith("{")]
    assert len(rows) == 15
    assert {r["brick"] for r in rows} == {16, 32, 64}
    assert all(0 < r["compression_ratio_pct"] < 100 for r in rows)
    table1 = {(r["brick"], r["coding"]): r["compressed_bytes"] for r in rows[:9]}
    for b in (16, 32, 64):
        assert table1[(b, "no rANS (raw nibbles)")] > max(table1[(b, "rANS, 2 tables")], table1[(b, "rANS, 1 table")])
    by_lanes = {r["lane_max"]: r["compressed_bytes"] for r in rows[9:] if r["scale_bits"] == 10}
    by_lanes[64] = table1[(32, "rANS, 2 tables")]
    assert by_lanes[1] <= by_lanes[4] <= by_lanes[16] <= by_lanes[64]
    # the no-rANS containers are the oracle's raw-nibble ones
    vol = synth.cells(n=64, grid=max(2, round(37 * 64 / 512)), seed=2)
    for log2 in (4, 5, 6):
        assert table1[(1 << log2, "no rANS (raw nibbles)")] == len(orc.encode_volume(vol, brick_log2=log2, tables=0))
