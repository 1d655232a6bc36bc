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


def test_algorithmic_bytes_model():
    """B = D (b_r + b_n + 2 nvec b_v) + T (nvec b_v + [sym] (b_p + n_probe b_k))
    with T = D x the full-space mean number of unequal-spin bonds."""
    # 6x6 J1-J2, Gamma A1: D = 31,566,122, 144 bonds, N = 36, n_up = 18:
    # T/D = 144 * 2 * 18 * 18 / (36 * 35) = 74.057...; FP32: 66.0 GB
    D = 31566122
    tbar = 144 * 2 * 18 * 18 / (36 * 35)
    assert abs(bench.mean_terms_full_space(36, 18, 144) - tbar) < 1e-12
    want = D * (8 + 1 + 2 * 4) + D * tbar * (4 + 4 + 5 * 4)
    assert bench.alg_bytes(D, 36, 18, 144, 4, 1, True) == round(want)
    assert abs(want / 1e9 - 66.0) < 0.1
    # N = 32 ring sector, FP32: 8.9 GB; FP64: 10.3 GB
    assert abs(bench.alg_bytes(18784170, 32, 16, 32, 4, 1, True) / 1e9 - 8.9) < 0.1
    assert abs(bench.alg_bytes(18784170, 32, 16, 32, 8, 1, True) / 1e9 - 10.3) < 0.1
    # U(1) blocks read no stabiliser class ... no index entry from memory
    assert bench.alg_bytes(10, 4, 2, 4, 8, 2, False) == round(
        10 * (4 + 1 + 2 * 2 * 8) + 10 * (4 * 2 * 2 * 2 / 12) * (2 * 8))


def test_roofline_bound_names_the_limiter():
    issue = {"valu_wave_insts": 0.9 * bench.VALU_PEAK_WAVE_INSTS * 1e-3, "frac_of_launch": 0.9}
    r = bench.roofline_entry(4e9, 1e-3, 4.0e9, issue)      # traffic 0.5 of peak, VALU 0.9
    assert r["bound"] == "alu" and r["unit"] == "Tops/s"
    assert abs(r["frac"] - 0.9) < 1e-9
    assert abs(r["hbm"]["frac"] - 0.5) < 1e-9
    issue2 = dict(issue, frac_of_launch=0.3)
    r = bench.roofline_entry(4e9, 1e-3, 7.2e9, issue2)    # traffic 0.9 of peak, VALU 0.3
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and abs(r["frac"] - 0.5) < 1e-9
    r = bench.roofline_entry(4e9, 1e-3, None, None)
    assert r["bound"] == "hbm" and r["limiter"].startswith("unknown")


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


def test_apply_dispatch_selection():
    """The counter summaries take the last apply dispatch and, when the terms
    read the rank-addressed x, the scatter launched just before it (both are
    inside the timed launch); a scatter before an earlier apply is not
    counted, and rows of other kernels (several counters per dispatch) are
    ignored."""
    def rows(seq):
        out = []
        for i, name in seq:
            for c in ("SQ_INSTS_VALU", "SQ_WAVES"):
                out.append({"Dispatch_Id": str(i), "Kernel_Name": name, "Counter_Name": c,
                            "Counter_Value": "1"})
        return out
    sc = "void xdg::(anonymous namespace)::k_xr_scatter<unsigned long, float>(...)"
    ap = "void xdg::k_apply<unsigned long, 3, float, double, false, 1, true, true, false, 1>(...)"
    seq = [(1, sc), (2, ap), (3, sc), (4, ap), (5, "copyBuffer"), (6, "k_count")]
    assert bench.apply_dispatches(rows(seq)) == {3, 4}
    # index form: no scatter before the last apply
    seq = [(1, sc), (2, ap), (3, ap), (4, "copyBuffer")]
    assert bench.apply_dispatches(rows(seq)) == {3}
    seq = [(7, ap)]
    assert bench.apply_dispatches(rows(seq)) == {7}
