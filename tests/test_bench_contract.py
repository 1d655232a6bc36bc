"""Host checks of bench.py's reporting logic (no GPU): the one-GPU refusal,
the algorithmic bytes of the apply, and the use of committed counter
summaries only for the kernel sources they were taken on."""
import glob
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_of_the_ring_apply():
    # N = 32 ring, k = 0: 18,784,170 rows, 329,026,186 nonzeros per vector
    # (diagonal included).  Per row: 4-byte state, 2-byte stabiliser, x[r]
    # read and y[r] written (FP32); per off-diagonal term: the gathered x
    # value and one index entry (4-byte key word + 4-byte position).
    dim, nnz = 18784170, 329026186
    per_row = 4 + 2 + 2 * 4
    per_term = 4 + (4 + 4)
    want = dim * per_row + (nnz - dim) * per_term
    assert want == 3985882572
    assert bench.alg_bytes(dim, nnz, 4, 4, 1, True) == want
    # U(1) blocks read no stabiliser and no index entry from memory
    assert bench.alg_bytes(10, 30, 4, 8, 2, False) == 10 * (4 + 2 * 2 * 8) + 20 * (2 * 8)


def test_counter_summaries_apply_only_to_their_sources():
    h = bench.source_hash()
    files = glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))
    assert files, "no committed traffic summary"
    for f in files:
        t = json.load(open(f))
        w = t["workload"]
        got = bench.load_traffic(w, t["source_hash"])
        assert got == t["traffic_bytes_per_launch"]
        assert bench.load_traffic(w, "0" * 16) is None
        if t["source_hash"] != h:
            assert bench.load_traffic(w, h) is None
    for f in glob.glob(os.path.join(ROOT, "profiles", "issue_*.json")):
        t = json.load(open(f))
        got = bench.load_issue(t["workload"], t["source_hash"], 1e-3)
        assert got["valu_wave_insts"] == t["valu_wave_insts"]
        assert abs(got["issue_ms"] - t["valu_wave_insts"] / bench.VALU_PEAK_WAVE_INSTS * 1e3) < 1e-12
        assert bench.load_issue(t["workload"], "0" * 16, 1e-3) is None
