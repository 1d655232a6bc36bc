#!/usr/bin/env python3
"""Benchmark: matrix-free H x and Lanczos on symmetry-adapted spin-1/2 sectors.

Default workload (square36_j1j2_A1): J1-J2 Heisenberg model (J1 = 1,
J2 = 0.5) on the 6x6 periodic square lattice, Sz = 0, translations x C4v
(288 elements), Gamma-point A1 sector (31,566,122 states).  One step = one
Lanczos iteration with FP32 vectors and FP64 full reorthogonalisation; the
default K = 200 steps are one complete 200-iteration run, whose lowest Ritz
value is the ground-state energy.  The same run with FP64 vectors (with and
without reorthogonalisation) is timed beside it, and the energies compared.

Other workloads (--workload):
  chain16_u1        N = 16 ring, U(1) block only (12,870 states), FP64
  chain32_k0_kpi    N = 32 ring, T_32, k = 0 and pi (18,784,170 states each):
                    FP32 vectors vs FP64, 200 iterations, Bethe-ansatz energies
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
DEFAULT_STEPS = {"chain16_u1": 200, "chain32_k0_kpi": 40, "square36_j1j2_A1": 200,
                 "chain32_allk": 20, "tilted40_xxz": 3}
DEFAULT_WORKLOAD = "square36_j1j2_A1"


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


def mean_terms_full_space(n_sites: int, n_up: int, n_bonds: int) -> float:
    """Mean number of unequal-spin bonds per state over all states with n_up
    up spins: each bond has unequal spins with probability
    2 n_up (N - n_up) / (N (N - 1))."""
    N = n_sites
    return n_bonds * 2.0 * n_up * (N - n_up) / (N * (N - 1))


def alg_bytes(dim: int, n_sites: int, n_up: int, n_bonds: int, vec: int, nvec: int,
              symmetric: bool) -> int:
    """Algorithmic bytes of one application (the byte model of the method):
        B = D (b_r + b_n + 2 nvec b_v) + T (nvec b_v + [sym] (b_p + n_probe b_k))
    per row the state word b_r (4 B for N <= 32, else 8), the stabiliser
    class b_n = 1 B, x[r] read and y[r] written; per generated off-diagonal
    term (T = D x the full-space mean number of unequal-spin bonds) the
    gathered x values and, for symmetric blocks, one index lookup priced as a
    prefix-table entry (b_p = 4 B) plus n_probe = 5 postfix keys of b_k = 4 B.
    The U(1) Lin tables are cache resident and count 0."""
    b_r = 4 if n_sites <= 32 else 8
    T = dim * mean_terms_full_space(n_sites, n_up, n_bonds)
    row = b_r + 1 + 2 * nvec * vec
    term = nvec * vec + ((4 + 5 * 4) if symmetric else 0)
    return int(round(dim * row + T * term))


# The sources the apply kernels and their launcher are built from: counter
# summaries taken on other versions of these files are not used.
APPLY_SOURCES = ["include/xdg.h"] + [
    "paper_2505_02901_amd/csrc/" + f for f in (
        "xdg_internal.hpp", "device_common.hpp", "apply_impl.hpp", "apply.hip",
        "apply_u1.hip", "apply_aff.hip", "apply_sub.hip", "apply_sub_xr.hip",
        "apply_sub_xr_trivial.hip", "apply_tab.hip")]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
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
# every 4 cycles (16 lanes per cycle); as lane operations: 256 x 4 x 16 x 2.4e9
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4
VALU_PEAK_LANE_OPS = VALU_PEAK_WAVE_INSTS * 64


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


def roofline_entry(alg: int, launch_s: float, traffic, issue):
    """The roofline object of the dominant kernel.  The limiter (`bound`) is
    whichever of HBM traffic (counter bytes per launch over the launch time,
    against 8 TB/s) and VALU issue (counter instructions at the issue peak,
    as a share of the launch) is closer to its peak.  With bound "hbm" the
    figures are the algorithmic bytes over the launch time against 8 TB/s;
    with bound "alu" they are the executed VALU lane operations over the
    launch time against 256 CUs x 64 lanes x 2.4 GHz = 39.3 Tops/s, and the
    algorithmic-byte figures stay under "hbm".  Without counters for the
    current kernel sources the limiter is unknown and the HBM roofline is
    reported."""
    hbm = {"achieved": alg / launch_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": alg / launch_s / 1e9 / HBM_PEAK_GBS}
    traffic_frac = None if traffic is None else traffic / launch_s / 1e9 / HBM_PEAK_GBS
    valu_frac = None if issue is None else issue["frac_of_launch"]
    out = {"bound": "hbm", **hbm, "traffic": traffic,
           "traffic_frac_of_peak": traffic_frac, "valu_issue": issue}
    if traffic_frac is None or valu_frac is None:
        out["limiter"] = "unknown (no counters for the current kernel sources)"
        return out
    if valu_frac > traffic_frac:
        lane_ops = issue["valu_wave_insts"] * 64
        out.update({"bound": "alu", "achieved": lane_ops / launch_s / 1e12,
                    "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "Tops/s",
                    "frac": lane_ops / launch_s / VALU_PEAK_LANE_OPS, "hbm": hbm})
    out["limiter"] = (f"VALU issue {valu_frac:.2f} of the launch vs HBM traffic "
                      f"{traffic_frac:.2f} of 8 TB/s")
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(models, nvec: int = 1, target_s: float = 3.0):
    """The oracle's H x on a bounded sample of rows: per row the diagonal,
    the pull-form terms (representative search by scanning the group,
    stabiliser and character sums) and the gather of x at the target states
    (x keyed by state, so no basis list is enumerated).  Three runs on all
    host cores and three on one core; the medians are reported."""
    import oracle
    oracle.build()
    cores = oracle.num_threads()
    per = max(1, 64 // len(models))
    samples = [(m, oracle.sample_basis_states(m, per, 1000 + i)) for i, m in enumerate(models)]

    def nnz_of(rows_per_model):
        """nonzeros the sampled rows hold (diagonal + terms in the block), untimed"""
        n = 0
        for m, rows in rows_per_model:
            _, _, cnt, _, _ = oracle.rows_terms(m, rows)
            n += int(len(rows) + cnt.sum()) * nvec
        return n

    def run(rows_per_model):
        t0 = time.perf_counter()
        for m, rows in rows_per_model:
            oracle.apply_keyed(m, rows, 9, nvec=nvec, complex_=m.is_complex)
        return time.perf_counter() - t0

    def timed(threads):
        oracle.set_num_threads(threads)
        dt = run(samples)               # size the sample to ~target_s per run
        scale = max(1.0, target_s / max(dt, 1e-3))
        n_rows = int(min(200000, per * scale))
        big = [(m, oracle.sample_basis_states(m, n_rows, 2000 + i)) for i, m in enumerate(models)]
        nnz = nnz_of(big)
        times = [run(big) for _ in range(3)]
        rates = sorted(nnz / t for t in times)
        return {"value": rates[1], "runs": rates, "threads": threads,
                "rows": n_rows * len(models), "s_per_run": float(np.median(times))}

    allc = timed(cores)
    one = timed(1)
    oracle.set_num_threads(cores)
    names = ", ".join(m.name for m in models[:3]) + (" ..." if len(models) > 3 else "")
    return {"value": allc["value"], "unit": "nonzeros/s", "cores": cores, "kind": "oracle",
            "sample": f"{allc['rows']} rows drawn by the oracle from {names} (random states "
                      f"mapped to their representatives), {nvec} vector(s), median of 3 runs "
                      f"of ~{allc['s_per_run']:.1f} s; x keyed by state, so the oracle's "
                      "basis enumeration (brute force over all states) is not part of it",
            "one_core": {"value": one["value"], "runs": one["runs"], "rows": one["rows"]},
            "all_core_runs": allc["runs"], "cpu_model": cpu_model(),
            "nproc": os.cpu_count()}


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

    def apply_roofline(self, nvec=1, reps=20, batched=False):
        """Average duration of one launch of the dominant kernel (the apply of
        the first sector, or the batched apply over every sector), timed with
        HIP events on the stream it is launched on after three warm-up
        launches (an event between consecutive launches also gives the median
        launch), and its algorithmic bytes."""
        torch, X = self.torch, self.X
        vdt = torch.complex64 if self.cplx else torch.float32
        idx = range(len(self.hams)) if batched else [0]
        xs, ys = [], []
        for i in idx:
            d = self.dims[i]
            xs.append(torch.randn(*((d,) if nvec == 1 else (d, nvec)), dtype=vdt, device="cuda"))
            ys.append(torch.empty_like(xs[-1]))
        hs = [self.hams[i] for i in idx]

        def launch(st=None):
            if batched:
                X.xdg_apply_batched([h.handle for h in hs], xs, ys, stream=st)
            else:
                hs[0].apply(xs[0], ys[0], stream=st)
        for _ in range(3):
            launch()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(st)
        for r in range(reps):
            launch(st)
            ev[r + 1].record(st)
        ev[-1].synchronize()
        sec = ev[0].elapsed_time(ev[-1]) * 1e-3 / reps
        med_ms = sorted(ev[r].elapsed_time(ev[r + 1]) for r in range(reps))[reps // 2]
        del xs, ys
        vb = 8 if self.cplx else 4
        alg = 0
        for i in idx:
            m = self.models[i]
            alg += alg_bytes(self.dims[i], m.n_sites, m.n_up, len(m.jz), vb, nvec,
                             m.perm is not None)
        khash = source_hash()
        torch.cuda.empty_cache()
        roof = roofline_entry(alg, sec, load_traffic(self.args.workload, khash),
                              load_issue(self.args.workload, khash, sec))
        what = (f"batched k_apply over {len(hs)} sectors" if batched
                else f"k_apply, sector {self.models[0].name}")
        roof.update({"kernel": f"{what} ({'complex ' if self.cplx else ''}FP32 vectors, "
                               f"{nvec} per sector)",
                     "avg_launch_ms": sec * 1e3, "median_launch_ms": med_ms,
                     "alg_bytes_per_launch": alg,
                     "nnz_per_launch": sum(self.nnzs[i] for i in idx) * nvec,
                     "source_hash": khash})
        return roof


def run_standard(c: Ctx, prec_fast, prec_ref, step_name, extra_ref=None):
    """Per-sector single-vector Lanczos runs of K iterations in two precision
    forms (K = the E0 iteration count by default, so the timed runs are the
    energy runs); a third form (extra_ref: FP64 with the same
    reorthogonalisation as the fast form) is timed the same way and reported
    beside them with its energy."""
    X, a = c.X, c.args
    res = {}

    def steps(prec):
        def f(warm):
            r = c.lanczos(prec, a.warmup if warm else a.steps)
            if not warm:
                res[prec] = r
        return f

    el_fast = c.timed(steps(prec_fast))
    log(f"timed {a.steps} steps (fast form): {el_fast:.3f}s")
    el_ref = c.timed(steps(prec_ref))
    log(f"timed {a.steps} steps (reference form): {el_ref:.3f}s")
    el_x = None
    if extra_ref is not None:
        el_x = c.timed(steps(extra_ref))
        log(f"timed {a.steps} steps (FP64 form with reorthogonalisation): {el_x:.3f}s")
    nnz_step = sum(c.nnzs)

    def e0(prec):
        runs = res[prec] if a.steps == a.e0_iters and prec in res else c.lanczos(prec, a.e0_iters)
        return [r[1][0] for r in runs]
    e_fast, e_ref = e0(prec_fast), e0(prec_ref)
    log(f"E0 fast {e_fast} ref {e_ref}")
    out = {
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
    if extra_ref is not None:
        out["e0"]["reference_reorth"] = e0(extra_ref)
        out["reference_reorth_form"] = {"value": nnz_step * a.steps / el_x, "unit": "nonzeros/s",
                                        "ms_per_step": 1e3 * el_x / a.steps,
                                        "lanczos_iters_per_s": len(c.hams) * a.steps / el_x}
    return out


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
    """Workload for the counter runs: three launches of the dominant kernel
    (the FP32 apply of the first sector, one vector; for chain32_allk the
    batched apply over all 32 sectors with 8 complex vectors each), the last
    of which is summarised, then a plain 1 GiB device copy whose FETCH_SIZE /
    WRITE_SIZE calibrate the counters."""
    import torch
    import paper_2505_02901_amd as X
    import workloads as W
    batched = args.workload == "chain32_allk"
    ms = W.workload(args.workload) if batched else W.workload(args.workload)[:1]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    cplx = any(b.is_complex for b in bs)
    dt = torch.complex64 if cplx else torch.float32
    nvec = 8 if batched else 1
    xs = [torch.randn(*((b.dim,) if nvec == 1 else (b.dim, nvec)), dtype=dt, device="cuda")
          for b in bs]
    ys = [torch.empty_like(x) for x in xs]
    for _ in range(3):
        if batched:
            X.xdg_apply_batched([h.handle for h in hs], xs, ys)
        else:
            hs[0].apply(xs[0], ys[0])
    torch.cuda.synchronize()
    del xs, ys
    a = torch.empty(256 << 20, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"workload": args.workload, "dims": [b.dim for b in bs][:4],
                      "nnz": sum(h.nnz for h in hs), "nvec": nvec, "copy_bytes": a.numel() * 4}))


def apply_dispatches(rows):
    """Dispatch ids of the last apply launch in a counter CSV: the last
    k_apply dispatch and, when the terms read the rank-addressed x, the
    scatter that filled it just before (both are inside the timed launch)."""
    apply_ids = sorted({int(r["Dispatch_Id"]) for r in rows if "k_apply" in r["Kernel_Name"]})
    last = apply_ids[-1]
    scat = [int(r["Dispatch_Id"]) for r in rows
            if "k_xr_scatter" in r["Kernel_Name"] and int(r["Dispatch_Id"]) < last]
    prev = max(apply_ids[:-1] + [-1]) if len(apply_ids) > 1 else -1
    ids = {last}
    if scat and max(scat) > prev:
        ids.add(max(scat))
    return ids


def summarize_issue(args):
    """profiles/issue_<workload>.json from the CSV of the SQ_INSTS_* run (last
    apply launch: the apply dispatch and its scatter, if any; counts summed
    over the chip)."""
    import csv
    import glob
    f = glob.glob(os.path.join(args.summarize_issue, "**", "*counter_collection.csv"),
                  recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    ids = apply_dispatches(rows)
    vals, kname, scatter = {}, "", {}
    for r in rows:
        if int(r["Dispatch_Id"]) in ids:
            vals[r["Counter_Name"]] = vals.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            if "k_apply" in r["Kernel_Name"]:
                kname = r["Kernel_Name"]
            else:
                scatter[r["Counter_Name"]] = scatter.get(r["Counter_Name"], 0.0) + float(
                    r["Counter_Value"])
    out = {"workload": args.workload, "kernel": kname, "source_hash": source_hash(),
           "valu_wave_insts": vals["SQ_INSTS_VALU"], "counters": vals,
           "scatter_counters": scatter}
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
        ids = apply_dispatches(rows)
        app = [r for r in rows if int(r["Dispatch_Id"]) in ids]
        kname = [r["Kernel_Name"] for r in app if "k_apply" in r["Kernel_Name"]][0]
        sc = sum(float(r["Counter_Value"]) for r in app if "k_apply" not in r["Kernel_Name"])
        cp = [r for r in rows if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"]]
        cp = max(cp, key=lambda r: float(r["Counter_Value"]))
        return sum(float(r["Counter_Value"]) for r in app), float(cp["Counter_Value"]), kname, sc

    fetch, fetch_cp, kname, fetch_sc = read(args.summarize_counters[0], "FETCH_SIZE")
    write, write_cp, _, write_sc = read(args.summarize_counters[1], "WRITE_SIZE")
    copy_bytes = 256 << 22
    f_scale = copy_bytes / (fetch_cp * 1024.0)
    w_scale = copy_bytes / (write_cp * 1024.0)
    traffic = fetch * 1024.0 * f_scale + write * 1024.0 * w_scale
    out = {"workload": args.workload, "kernel": kname, "source_hash": source_hash(),
           "fetch_kib": fetch, "write_kib": write, "scatter_fetch_kib": fetch_sc,
           "scatter_write_kib": write_sc, "copy_fetch_kib": fetch_cp,
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
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
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
                         "(reference form: FP64, no reorthogonalisation)",
                         extra_ref=X.XDG_PREC_F64_REORTH)
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
    batched = w == "chain32_allk"
    roof = c.apply_roofline(nvec=8 if batched else 1, batched=batched, reps=5 if batched else 20)
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
        **({"reference_reorth_form": r["reference_reorth_form"]}
           if "reference_reorth_form" in r else {}),
        "e0": r["e0"],
        "basis_build_s": c.t_build,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, sampled rows) ...")
        line["cpu_baseline"] = cpu_baseline(c.models, nvec=8 if batched else 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
