#!/usr/bin/env python3
"""Benchmark: matrix-free H x and Lanczos on symmetry-adapted spin-1/2 sectors.

Default workload (chain32_k0_kpi): Heisenberg ring N = 32, J = 1, Sz = 0,
translation group (32 elements), momentum sectors k = 0 and k = pi
(18,784,170 states each).  One step = one Lanczos iteration (H x, the vector
operations and the scalar read-back) in each of the two sectors, with FP32
vectors and FP64 scalars.  The same steps in FP64 are timed beside it, and a
200-iteration run in both precisions gives the ground-state energies (vs the
Bethe ansatz).

Other workloads (--workload):
  chain16_u1        N = 16 ring, U(1) block only (12,870 states), FP64
  square36_j1j2_A1  6x6 J1-J2 (J2 = 0.5), T x C4v (288), Gamma A1: FP32
                    vectors + FP64 full reorthogonalisation vs FP64
  chain32_allk      all 32 momenta of the N = 32 ring x 8 vectors, batched
                    persistent launch replayed from a HIP graph (complex FP32)
                    vs sector-by-sector single-vector FP64
  tilted40_xxz      40-site tilted square lattice, T x C4 (160), 4
                    sublattices: FP32 vectors vs FP64, 100 iterations

Prints one JSON line.  Inputs are synthetic (seeded start vectors).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("H·x nonzeros/sec + Lanczos iters/sec; FP32-vector & batched vs FP64 at "
          "stated ΔE0")
HBM_PEAK_GBS = 8000.0
E0_ITERS = {"chain16_u1": 300, "chain32_k0_kpi": 200, "square36_j1j2_A1": 200,
            "chain32_allk": 100, "tilted40_xxz": 100}
DEFAULT_STEPS = {"chain16_u1": 200, "chain32_k0_kpi": 40, "square36_j1j2_A1": 10,
                 "chain32_allk": 20, "tilted40_xxz": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bethe_energy(N: int, M: int) -> float:
    """Heisenberg ring (J = 1), M magnons with consecutive Bethe quantum
    numbers: N atan(2 l_j) = pi I_j + sum_l atan(l_j - l_l); E = N/4 - sum 2/(1+4 l^2)."""
    import scipy.optimize
    I = np.arange(M) - (M - 1) / 2.0
    lam = 0.5 * np.tan(np.pi * I / N)
    for _ in range(20000):
        d = lam[:, None] - lam[None, :]
        new = 0.5 * np.tan((np.pi * I + np.arctan(d).sum(axis=1)) / N)
        done = np.max(np.abs(new - lam)) < 1e-15
        lam = new
        if done:
            break

    def F(l):
        return N * np.arctan(2 * l) - np.pi * I - np.arctan(l[:, None] - l[None, :]).sum(axis=1)
    lam = scipy.optimize.fsolve(F, lam, xtol=1e-15)
    return float(N / 4.0 - np.sum(2.0 / (1.0 + 4.0 * lam ** 2)))


def alg_bytes(dim: int, nnz: int, word: int, vec: int, nvec: int, symmetric: bool) -> int:
    """Algorithmic bytes of one application: per row the state word, the
    stabiliser (2 B, symmetric blocks), x[r] read and y[r] written; per
    off-diagonal term in the block the gathered x values and, for symmetric
    blocks, one index entry (key word + 4-byte position)."""
    T = nnz - dim
    row = word + (2 if symmetric else 0) + 2 * nvec * vec
    term = nvec * vec + ((word + 4) if symmetric else 0)
    return dim * row + T * term


def source_hash() -> str:
    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_2505_02901_amd", "csrc")
    for f in sorted(os.listdir(cs)):
        with open(os.path.join(cs, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel_hash: str):
    """HBM bytes per apply launch from the committed counter summary, if it
    was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_hash:
        return None
    return t.get("traffic_bytes_per_launch")


# VALU issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD
# every 4 cycles (16 lanes per cycle)
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def load_issue(workload: str, kernel_hash: str, launch_s: float):
    """VALU wave instructions of one apply launch from the committed counter
    summary (taken on the current kernel sources), as issue time at the peak
    rate and its share of the measured launch."""
    p = os.path.join(ROOT, "profiles", f"issue_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_hash:
        return None
    ms = t["valu_wave_insts"] / VALU_PEAK_WAVE_INSTS * 1e3
    return {"valu_wave_insts": t["valu_wave_insts"], "peak_wave_insts_per_s": VALU_PEAK_WAVE_INSTS,
            "issue_ms": ms, "frac_of_launch": ms / (launch_s * 1e3)}


def cpu_baseline(models, seconds: float = 15.0):
    """The oracle's H x on a bounded random sample of rows of the first sector."""
    import oracle
    oracle.build()
    m = models[0]
    t0 = time.perf_counter()
    basis = oracle.basis(m)
    t_basis = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    x = np.ones(len(basis), np.complex128)
    n0 = min(len(basis), 2000)
    rows = np.sort(rng.choice(len(basis), size=n0, replace=False))
    t0 = time.perf_counter()
    oracle.apply_rows(m, basis, rows, x)
    dt = time.perf_counter() - t0
    n = int(min(len(basis), max(n0, n0 * seconds / max(dt, 1e-6))))
    rows = np.sort(rng.choice(len(basis), size=n, replace=False))
    t0 = time.perf_counter()
    oracle.apply_rows(m, basis, rows, x)
    dt = time.perf_counter() - t0
    nnz = sum(1 + len(oracle.row_terms(m, int(basis[r]))[1]) for r in rows[:500])
    nnz_per_row = nnz / min(500, len(rows))
    return {"value": len(rows) * nnz_per_row / dt, "unit": "nonzeros/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{len(rows)} random rows of sector {m.name} (H x, complex128, OpenMP over "
                      f"rows); the oracle's basis enumeration of that sector ({t_basis:.1f} s) "
                      "is not included"}


class Ctx:
    def __init__(self, args):
        import torch
        import paper_2505_02901_amd as X
        import workloads as W
        self.torch, self.X, self.W, self.args = torch, X, W, args
        self.models = W.workload(args.workload)
        t0 = time.perf_counter()
        self.bases = [X.Basis.from_model(m) for m in self.models]
        self.hams = [X.Hamiltonian.from_model(b, m) for b, m in zip(self.bases, self.models)]
        torch.cuda.synchronize()
        self.t_build = time.perf_counter() - t0
        self.dims = [b.dim for b in self.bases]
        self.nnzs = [h.nnz for h in self.hams]
        self.cplx = any(b.is_complex for b in self.bases)

    def lanczos(self, prec, iters, seed0=7, sectors=None):
        out = []
        for i, h in enumerate(self.hams if sectors is None else [self.hams[s] for s in sectors]):
            out.append(h.lanczos(k=1, tol=0.0, max_iter=iters, seed=seed0 + i, prec=prec))
        return out

    def timed(self, fn):
        """W warm-up calls of fn(warm=True), then one timed call fn(warm=False)
        bracketed by device synchronisation."""
        torch = self.torch
        fn(True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn(False)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    def apply_roofline(self, nvec=1, reps=20):
        """Average duration of one apply launch of the first sector, timed with
        HIP events on the stream it is launched on, and its algorithmic bytes."""
        torch = self.torch
        h, d, n = self.hams[0], self.dims[0], self.nnzs[0]
        vdt = torch.complex64 if self.cplx else torch.float32
        shape = (d,) if nvec == 1 else (d, nvec)
        x = torch.randn(*shape, dtype=vdt, device="cuda")
        y = torch.empty_like(x)
        h.apply(x, y)
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            h.apply(x, y, stream=st)
        e1.record(st)
        e1.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / reps
        del x, y
        m = self.models[0]
        sym = m.perm is not None
        word = 8 if m.n_sites > 32 else 4
        vb = 8 if self.cplx else 4
        alg = alg_bytes(d, n, word, vb, nvec, sym)
        khash = source_hash()
        achieved = alg / sec / 1e9
        torch.cuda.empty_cache()
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": load_traffic(self.args.workload, khash),
                "valu_issue": load_issue(self.args.workload, khash, sec),
                "kernel": f"k_apply ({'complex ' if self.cplx else ''}FP32, {nvec} vector(s), "
                          f"sector {m.name})",
                "avg_launch_ms": sec * 1e3, "alg_bytes_per_launch": alg,
                "nnz_per_launch": n * nvec, "source_hash": khash}


def run_standard(c: Ctx, prec_fast, prec_ref, step_name):
    """Per-sector single-vector Lanczos steps in two precision forms."""
    X, a = c.X, c.args

    def steps(prec):
        def f(warm):
            c.lanczos(prec, a.warmup if warm else a.steps)
        return f

    el_fast = c.timed(steps(prec_fast))
    log(f"timed {a.steps} steps (fast form): {el_fast:.3f}s")
    el_ref = c.timed(steps(prec_ref))
    log(f"timed {a.steps} steps (reference form): {el_ref:.3f}s")
    nnz_step = sum(c.nnzs)
    e_fast = [r[1][0] for r in c.lanczos(prec_fast, a.e0_iters)]
    e_ref = [r[1][0] for r in c.lanczos(prec_ref, a.e0_iters)]
    log(f"E0 fast {e_fast} ref {e_ref}")
    return {
        "value": nnz_step * a.steps / el_fast,
        "ms_per_step": 1e3 * el_fast / a.steps,
        "lanczos_iters_per_s": len(c.hams) * a.steps / el_fast,
        "reference_form": {"value": nnz_step * a.steps / el_ref, "unit": "nonzeros/s",
                           "ms_per_step": 1e3 * el_ref / a.steps,
                           "lanczos_iters_per_s": len(c.hams) * a.steps / el_ref},
        "e0": {"iters": a.e0_iters, "fast": e_fast, "reference": e_ref,
               "rel_delta": [abs(p - q) / abs(q) for p, q in zip(e_fast, e_ref)]},
        "step": step_name,
    }


def run_batched(c: Ctx):
    """All sectors x nvec vectors in lockstep (batched graph) vs sector-by-sector FP64."""
    X, a = c.X, c.args
    hs = [h.handle for h in c.hams]
    nvec = 8

    def batched(warm):
        X.xdg_lanczos_eigval_batched(hs, nvec=nvec, n_iter=a.warmup if warm else a.steps, seed=4,
                                     prec=X.XDG_PREC_F32VEC)

    el = c.timed(batched)
    log(f"batched {a.steps} steps: {el:.3f}s")
    nnz_step = sum(c.nnzs) * nvec

    def single(warm):
        c.lanczos(X.XDG_PREC_F64, a.warmup if warm else a.steps)

    el_ref = c.timed(single)
    log(f"sector-by-sector FP64 {a.steps} steps: {el_ref:.3f}s")
    ev, _, _ = X.xdg_lanczos_eigval_batched(hs, nvec=nvec, n_iter=a.e0_iters, seed=4,
                                            prec=X.XDG_PREC_F32VEC)
    e_b = [float(np.min(r)) for r in ev]
    e_r = [r[1][0] for r in c.lanczos(X.XDG_PREC_F64, a.e0_iters)]
    return {
        "value": nnz_step * a.steps / el,
        "ms_per_step": 1e3 * el / a.steps,
        "lanczos_iters_per_s": len(hs) * nvec * a.steps / el,
        "reference_form": {"value": sum(c.nnzs) * a.steps / el_ref, "unit": "nonzeros/s",
                           "ms_per_step": 1e3 * el_ref / a.steps,
                           "lanczos_iters_per_s": len(hs) * a.steps / el_ref,
                           "form": "sector by sector, one vector, FP64"},
        "e0": {"iters": a.e0_iters, "batched_fp32_min_over_vectors": e_b, "fp64": e_r,
               "rel_delta": [abs(p - q) / abs(q) for p, q in zip(e_b, e_r)]},
        "step": f"one Lanczos iteration of {nvec} vectors in each of {len(hs)} sectors, "
                "complex FP32 vectors, FP64 scalars, one batched graph replay",
    }


def counters_run(args):
    """Workload for the counter runs: three applies of the first sector (FP32,
    one vector), the last of which is summarised, then a plain 1 GiB device
    copy whose FETCH_SIZE / WRITE_SIZE calibrate the counters."""
    import torch
    import paper_2505_02901_amd as X
    import workloads as W
    m = W.workload(args.workload)[0]
    b = X.Basis.from_model(m)
    h = X.Hamiltonian.from_model(b, m)
    dt = torch.complex64 if b.is_complex else torch.float32
    x = torch.randn(b.dim, dtype=dt, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        h.apply(x, y)
    torch.cuda.synchronize()
    a = torch.empty(256 << 20, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"workload": args.workload, "dim": b.dim, "nnz": h.nnz,
                      "copy_bytes": a.numel() * 4}))


def summarize_issue(args):
    """profiles/issue_<workload>.json from the CSV of the SQ_INSTS_* run (last
    apply dispatch; counts summed over the chip)."""
    import csv
    import glob
    f = glob.glob(os.path.join(args.summarize_issue, "**", "*counter_collection.csv"),
                  recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    last = [r["Dispatch_Id"] for r in rows if "k_apply" in r["Kernel_Name"]][-1]
    vals, kname = {}, ""
    for r in rows:
        if r["Dispatch_Id"] == last:
            vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            kname = r["Kernel_Name"]
    out = {"workload": args.workload, "kernel": kname, "source_hash": source_hash(),
           "valu_wave_insts": vals["SQ_INSTS_VALU"], "counters": vals}
    p = os.path.join(ROOT, "profiles", f"issue_{args.workload}.json")
    with open(p, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def summarize_counters(args):
    """profiles/traffic_<workload>.json from the CSVs of the FETCH_SIZE and
    WRITE_SIZE runs (last apply dispatch of each; counts in KiB, scaled by the
    copy calibration)."""
    import csv
    import glob

    def read(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        rows = [r for r in csv.DictReader(open(f)) if r["Counter_Name"] == counter]
        app = [r for r in rows if "k_apply" in r["Kernel_Name"]][-1]
        cp = [r for r in rows if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"]]
        cp = max(cp, key=lambda r: float(r["Counter_Value"]))
        return float(app["Counter_Value"]), float(cp["Counter_Value"]), app["Kernel_Name"]

    fetch, fetch_cp, kname = read(args.summarize_counters[0], "FETCH_SIZE")
    write, write_cp, _ = read(args.summarize_counters[1], "WRITE_SIZE")
    copy_bytes = 256 << 22
    f_scale = copy_bytes / (fetch_cp * 1024.0)
    w_scale = copy_bytes / (write_cp * 1024.0)
    traffic = fetch * 1024.0 * f_scale + write * 1024.0 * w_scale
    out = {"workload": args.workload, "kernel": kname, "source_hash": source_hash(),
           "fetch_kib": fetch, "write_kib": write, "copy_fetch_kib": fetch_cp,
           "copy_write_kib": write_cp, "fetch_scale": f_scale, "write_scale": w_scale,
           "traffic_bytes_per_launch": traffic}
    p = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.json")
    with open(p, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--counters", action="store_true",
                    help="run the profiled apply + calibration copy (under rocprofv3 --pmc)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-issue", metavar="SQ_DIR",
                    help="write profiles/issue_<workload>.json from an SQ_INSTS_* counter run")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="chain32_k0_kpi",
                    choices=sorted(E0_ITERS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--e0-iters", type=int, default=None)
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.summarize_issue:
        summarize_issue(args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    args.steps = args.steps or DEFAULT_STEPS[args.workload]
    args.warmup = args.warmup if args.warmup is not None else max(1, min(5, args.steps))
    args.e0_iters = args.e0_iters or E0_ITERS[args.workload]

    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.counters:
        counters_run(args)
        return
    c = Ctx(args)
    X = c.X
    log(f"workload {args.workload}: dims {c.dims[:4]}{'...' if len(c.dims) > 4 else ''} "
        f"nnz {sum(c.nnzs)} built in {c.t_build:.2f}s")
    w = args.workload
    if w == "chain32_allk":
        r = run_batched(c)
        dtype = "c64"
    elif w == "square36_j1j2_A1":
        r = run_standard(c, X.XDG_PREC_F32VEC_REORTH, X.XDG_PREC_F64,
                         "one Lanczos iteration, FP32 vectors with FP64 full reorthogonalisation "
                         "(reference form: FP64, no reorthogonalisation)")
        e_r2 = [q[1][0] for q in c.lanczos(X.XDG_PREC_F64_REORTH, args.e0_iters)]
        r["e0"]["fp64_reorth"] = e_r2
        dtype = "f32"
    elif w == "chain16_u1":
        r = run_standard(c, X.XDG_PREC_F64, X.XDG_PREC_F32VEC,
                         "one Lanczos iteration, FP64 (reference form: FP32 vectors)")
        dtype = "f64"
    else:
        r = run_standard(c, X.XDG_PREC_F32VEC, X.XDG_PREC_F64,
                         "one Lanczos iteration per sector, FP32 vectors, FP64 scalars "
                         "(reference form: FP64 vectors)")
        dtype = "c64" if c.cplx else "f32"
    ref = {}
    if w == "chain32_k0_kpi":
        ref = {"bethe_k0": bethe_energy(32, 16), "bethe_kpi": bethe_energy(32, 15)}
    elif w == "chain16_u1":
        ref = {"bethe": bethe_energy(16, 8)}
    if ref:
        r["e0"]["exact"] = ref
    roof = c.apply_roofline(nvec=8 if w == "chain32_allk" else 1)
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "nonzeros/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": w, "sectors": [m.name for m in c.models][:4] +
                   (["..."] if len(c.models) > 4 else []),
                   "n_sectors": len(c.models), "dims": c.dims if len(c.dims) <= 4 else
                   [min(c.dims), max(c.dims), sum(c.dims)], "nnz_per_vector": sum(c.nnzs),
                   "step": r["step"]},
        "lanczos_iters_per_s": r["lanczos_iters_per_s"],
        "reference_form": r["reference_form"],
        "e0": r["e0"],
        "basis_build_s": c.t_build,
        "roofline": roof,
    }
    # the oracle enumerates bases by brute force: feasible for the rings only
    if not args.no_cpu_baseline and w in ("chain16_u1", "chain32_k0_kpi"):
        line["cpu_baseline"] = cpu_baseline(c.models)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
