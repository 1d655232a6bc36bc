#!/usr/bin/env python3
"""Benchmark: matrix-free H x and Lanczos on symmetry-adapted spin-1/2 sectors.

Default workload: Heisenberg ring N = 32, J = 1, Sz = 0, translation group
(32 elements), momentum sectors k = 0 and k = pi (18,784,170 states each).
One step = one Lanczos iteration (H x plus the vector operations and the
scalar read-back) in each of the two sectors, with FP32 vectors and FP64
scalars.  The same steps in FP64 are timed beside it, and a 200-iteration run
in both precisions gives the ground-state energies (vs the Bethe ansatz).

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
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_hash:
        return None
    return t.get("traffic_bytes_per_launch")


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
    rows = np.sort(rng.choice(len(basis), size=min(len(basis), 20000), replace=False))
    t0 = time.perf_counter()
    oracle.apply_rows(m, basis, rows[:2000], x)
    dt = time.perf_counter() - t0
    n = int(min(len(rows), max(2000, 2000 * seconds / max(dt, 1e-6))))
    rows = np.sort(rng.choice(len(basis), size=min(len(basis), n), replace=False))
    t0 = time.perf_counter()
    oracle.apply_rows(m, basis, rows, x)
    dt = time.perf_counter() - t0
    nnz = 0
    for r in rows[:500]:
        nnz += 1 + len(oracle.row_terms(m, int(basis[r]))[1])
    nnz_per_row = nnz / min(500, len(rows))
    return {"value": len(rows) * nnz_per_row / dt, "unit": "nonzeros/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{len(rows)} random rows of sector {m.name} (H x, complex128, OpenMP over "
                      f"rows); oracle basis enumeration of that sector took {t_basis:.1f} s and "
                      "is not included"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="chain32_k0_kpi")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--e0-iters", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2505_02901_amd as X
    import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    models = W.workload(args.workload)
    t0 = time.perf_counter()
    bases = [X.Basis.from_model(m) for m in models]
    hams = [X.Hamiltonian.from_model(b, m) for b, m in zip(bases, models)]
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    dims = [b.dim for b in bases]
    nnzs = [h.nnz for h in hams]
    cplx = any(b.is_complex for b in bases)
    nnz_step = sum(nnzs)

    def lanczos_steps(prec, iters, seed0=7):
        out = []
        for i, h in enumerate(hams):
            out.append(h.lanczos(k=1, tol=0.0, max_iter=iters, seed=seed0 + i, prec=prec))
        return out

    def timed(prec):
        lanczos_steps(prec, args.warmup)          # warm-up, also tunes the launch shape
        torch.cuda.synchronize()
        t = time.perf_counter()
        lanczos_steps(prec, args.steps)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    el32 = timed(X.XDG_PREC_F32VEC)
    el64 = timed(X.XDG_PREC_F64)

    # dominant kernel: the apply, timed with events on the stream it runs on
    vdt = torch.complex64 if cplx else torch.float32
    xs = [torch.randn(d, dtype=vdt, device="cuda") for d in dims]
    ys = [torch.empty_like(x) for x in xs]
    for h, x, y in zip(hams, xs, ys):
        h.apply(x, y)
    torch.cuda.synchronize()
    reps = 20
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        for h, x, y in zip(hams, xs, ys):
            h.apply(x, y, stream=st)
    e1.record(st)
    e1.synchronize()
    apply_s = e0.elapsed_time(e1) * 1e-3 / (reps * len(hams))
    sym = models[0].perm is not None
    word = 8 if models[0].n_sites > 32 else 4
    vb = 8 if cplx else 4
    alg = sum(alg_bytes(d, n, word, vb, 1, sym) for d, n in zip(dims, nnzs)) / len(hams)
    achieved = alg / apply_s / 1e9
    khash = source_hash()
    traffic = load_traffic(args.workload, khash)

    # ground-state energies after a fixed number of iterations
    e32 = [r[1][0] for r in lanczos_steps(X.XDG_PREC_F32VEC, args.e0_iters)]
    e64 = [r[1][0] for r in lanczos_steps(X.XDG_PREC_F64, args.e0_iters)]
    ref = {}
    if args.workload.startswith("chain32"):
        ref = {"k=0": bethe_energy(32, 16), "k=pi": bethe_energy(32, 15)}

    value = nnz_step * args.steps / el32
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "nonzeros/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "sectors": [m.name for m in models],
                   "dims": dims, "nnz_per_step": nnz_step,
                   "step": "one Lanczos iteration per sector, FP32 vectors, FP64 scalars"},
        "lanczos_iters_per_s": len(hams) * args.steps / el32,
        "fp64": {"value": nnz_step * args.steps / el64, "unit": "nonzeros/s",
                 "ms_per_step": 1e3 * el64 / args.steps,
                 "lanczos_iters_per_s": len(hams) * args.steps / el64},
        "e0": {"iters": args.e0_iters, "fp32vec": e32, "fp64": e64,
               "rel_delta_fp32_vs_fp64": [abs(a - b) / abs(b) for a, b in zip(e32, e64)],
               "reference": ref},
        "basis_build_s": t_build,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_apply (FP32, one vector)",
                     "avg_launch_ms": apply_s * 1e3, "alg_bytes_per_launch": alg,
                     "source_hash": khash},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(models)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
