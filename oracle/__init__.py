"""Python access to the CPU oracle (``oracle/xdg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.  It shares
nothing with the GPU library but the seeded inputs of ``workloads``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xdg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, plain IEEE double)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_act.restype = C.c_uint64
        lib.orc_act.argtypes = [C.c_int, P, C.c_uint64]
        lib.orc_rep.restype = C.c_uint64
        lib.orc_rep.argtypes = [C.c_int, C.c_int, P, C.c_uint64, P, P]
        lib.orc_basis.restype = C.c_int64
        lib.orc_basis.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, C.c_int64]
        lib.orc_basis_range.restype = C.c_int64
        lib.orc_basis_range.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_uint64, C.c_uint64,
                                        P, C.c_int64]
        lib.orc_index.restype = C.c_int64
        lib.orc_index.argtypes = [P, C.c_int64, C.c_uint64]
        lib.orc_row_terms.restype = C.c_int
        lib.orc_row_terms.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, P, P, C.c_uint64,
                                      P, P, P, C.c_int]
        lib.orc_apply.restype = C.c_int
        lib.orc_apply.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, P, P, P, C.c_int64,
                                  C.c_int64, P, P]
        lib.orc_apply_rows.restype = C.c_int
        lib.orc_apply_rows.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, P, P, P, C.c_int64,
                                       P, C.c_int64, C.c_int64, P, P]
        lib.orc_rep_many.restype = C.c_int
        lib.orc_rep_many.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int64, P, P]
        lib.orc_rows_terms.restype = C.c_int
        lib.orc_rows_terms.argtypes = [C.c_int, C.c_int, C.c_int, P, P, C.c_int, P, P, P, P,
                                       C.c_int64, P, P, P, P, P]
        lib.orc_tridiag_eigvals.restype = C.c_int
        lib.orc_tridiag_eigvals.argtypes = [C.c_int, P, P, C.c_int, P]
        lib.orc_lanczos.restype = C.c_int
        lib.orc_lanczos.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, P, P, P, C.c_int64, P,
                                    C.c_int, C.c_double, C.c_int, C.c_int, P, P, P, P]
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_num_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _model_arrays(m):
    perm = None if m.perm is None else np.ascontiguousarray(m.perm, dtype=np.int32)
    chi = m.chi_interleaved()
    sites = np.ascontiguousarray(m.sites, dtype=np.int32)
    jz = np.ascontiguousarray(m.jz, dtype=np.float64)
    jxy = np.ascontiguousarray(m.jxy, dtype=np.float64)
    return perm, chi, sites, jz, jxy


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def act(n_sites: int, g, s: int) -> int:
    g = np.ascontiguousarray(g, dtype=np.int32)
    return int(_load().orc_act(n_sites, _p(g), s))


def rep(n_sites: int, perm, s: int) -> Tuple[int, int, int]:
    """(representative, first minimising element, number of minimisers)."""
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    u = np.zeros(1, np.int32)
    n = np.zeros(1, np.int32)
    r = _load().orc_rep(n_sites, perm.shape[0], _p(perm), s, _p(u), _p(n))
    return int(r), int(u[0]), int(n[0])


def basis(m) -> np.ndarray:
    """Ascending basis list (uint64) of the model's sector."""
    perm, chi, *_ = _model_arrays(m)
    lib = _load()
    n_sym = m.n_sym
    if chi is None and n_sym:
        chi = np.zeros((n_sym, 2))
        chi[:, 0] = 1.0
    d = lib.orc_basis(m.n_sites, m.n_up, n_sym, _p(perm), _p(chi), None, 0)
    if d < 0:
        raise ValueError(f"orc_basis failed ({d})")
    out = np.empty(max(d, 1), dtype=np.uint64)
    d2 = lib.orc_basis(m.n_sites, m.n_up, n_sym, _p(perm), _p(chi), _p(out), d)
    assert d2 == d
    return out[:d]


def basis_range(m, lo: int, hi: int, cap: int = 1 << 22) -> np.ndarray:
    """Basis states s with lo <= s <= hi, ascending."""
    perm, chi, *_ = _model_arrays(m)
    n_sym = m.n_sym
    if chi is None and n_sym:
        chi = np.zeros((n_sym, 2))
        chi[:, 0] = 1.0
    out = np.empty(cap, dtype=np.uint64)
    n = _load().orc_basis_range(m.n_sites, m.n_up, n_sym, _p(perm), _p(chi), lo, hi, _p(out), cap)
    if n < 0:
        raise ValueError(f"orc_basis_range failed ({n})")
    return out[:n].copy()


def stabiliser_character_sum(m, s: int) -> complex:
    """sum of chi over the elements fixing s (zero for orbits without a symmetric state)."""
    tot = 0j
    for g, c in zip(m.perm, m.chi):
        if act(m.n_sites, g, s) == s:
            tot += c
    return tot


def index(basis_list: np.ndarray, s: int) -> int:
    b = np.ascontiguousarray(basis_list, dtype=np.uint64)
    return int(_load().orc_index(_p(b), len(b), s))


def row_terms(m, r: int):
    """(diag, targets uint64[n], amps complex128[n]) of row r (pull form)."""
    perm, chi, sites, jz, jxy = _model_arrays(m)
    cap = len(jz) + 1
    tg = np.zeros(cap, np.uint64)
    am = np.zeros(2 * cap, np.float64)
    d = np.zeros(1, np.float64)
    n = _load().orc_row_terms(m.n_sites, m.n_sym, _p(perm), _p(chi), len(jz), _p(sites), _p(jz),
                              _p(jxy), r, _p(d), _p(tg), _p(am), cap)
    if n < 0:
        raise RuntimeError("orc_row_terms failed")
    return float(d[0]), tg[:n].copy(), am[: 2 * n].view(np.complex128).copy()


def apply(m, basis_list: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = H x; x of shape [dim] or [dim, nvec], any real/complex dtype."""
    perm, chi, sites, jz, jxy = _model_arrays(m)
    b = np.ascontiguousarray(basis_list, dtype=np.uint64)
    squeeze = x.ndim == 1
    xc = np.ascontiguousarray(x.reshape(len(b), -1), dtype=np.complex128)
    nvec = xc.shape[1]
    y = np.zeros_like(xc)
    rc = _load().orc_apply(m.n_sites, m.n_sym, _p(perm), _p(chi), len(jz), _p(sites), _p(jz),
                           _p(jxy), _p(b), len(b), nvec, _p(xc), _p(y))
    if rc != 0:
        raise RuntimeError("orc_apply failed")
    return y[:, 0] if squeeze else y


def apply_rows(m, basis_list: np.ndarray, rows: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(H x)[rows]; x of shape [dim] or [dim, nvec]."""
    perm, chi, sites, jz, jxy = _model_arrays(m)
    b = np.ascontiguousarray(basis_list, dtype=np.uint64)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    squeeze = x.ndim == 1
    xc = np.ascontiguousarray(x.reshape(len(b), -1), dtype=np.complex128)
    nvec = xc.shape[1]
    y = np.zeros((len(r), nvec), np.complex128)
    rc = _load().orc_apply_rows(m.n_sites, m.n_sym, _p(perm), _p(chi), len(jz), _p(sites),
                                _p(jz), _p(jxy), _p(b), len(b), _p(r), len(r), nvec, _p(xc),
                                _p(y))
    if rc != 0:
        raise RuntimeError("orc_apply_rows failed")
    return y[:, 0] if squeeze else y


def rep_many(m, states):
    """(representatives uint64 [n], in_basis bool [n]) of host states."""
    perm, chi, *_ = _model_arrays(m)
    s = np.ascontiguousarray(states, dtype=np.uint64)
    n_sym = m.n_sym
    if chi is None and n_sym:
        chi = np.zeros((n_sym, 2))
        chi[:, 0] = 1.0
    reps = np.zeros(len(s), np.uint64)
    inb = np.zeros(len(s), np.int32)
    _load().orc_rep_many(m.n_sites, n_sym, _p(perm), _p(chi), _p(s), len(s), _p(reps), _p(inb))
    return reps, inb.astype(bool)


def sample_basis_states(m, n: int, seed: int) -> np.ndarray:
    """n distinct basis states of the model's sector, ascending, drawn without
    any basis list: random states with n_up up spins (numpy, seeded), mapped
    to their representatives, kept when the orbit carries a symmetric state.
    (Orbit-weighted, not uniform over the basis.)"""
    rng = np.random.default_rng(seed)
    out = np.zeros(0, np.uint64)
    while len(out) < n:
        k = max(64, 4 * (n - len(out)))
        bits = rng.random((k, m.n_sites)).argsort(axis=1)[:, :m.n_up].astype(np.uint64)
        states = (np.uint64(1) << bits).sum(axis=1, dtype=np.uint64)
        reps, inb = rep_many(m, states)
        out = np.unique(np.concatenate([out, reps[inb]]))
    rng.shuffle(out)
    return np.sort(out[:n])


def rows_terms(m, states):
    """Terms of several rows given by their states (no basis list needed).
    Returns (diag [n], in_basis bool [n], targets list of uint64 arrays,
    amps list of complex128 arrays)."""
    perm, chi, sites, jz, jxy = _model_arrays(m)
    s = np.ascontiguousarray(states, dtype=np.uint64)
    n, nb = len(s), len(jz)
    diag = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.int32)
    inb = np.zeros(n, np.int32)
    tg = np.zeros((n, nb), np.uint64)
    am = np.zeros((n, nb, 2), np.float64)
    n_sym = m.n_sym
    if chi is None and n_sym:
        chi = np.zeros((n_sym, 2))
        chi[:, 0] = 1.0
    rc = _load().orc_rows_terms(m.n_sites, m.n_up, n_sym, _p(perm), _p(chi), nb, _p(sites),
                                _p(jz), _p(jxy), _p(s), n, _p(diag), _p(cnt), _p(inb), _p(tg),
                                _p(am))
    if rc != 0:
        raise ValueError("orc_rows_terms: a row state has the wrong number of up spins")
    amps = am[..., 0] + 1j * am[..., 1]
    return diag, inb.astype(bool), cnt, tg, amps


def apply_keyed(m, states, seed: int, nvec: int = 1, complex_: bool = False,
                round_to_f32: bool = False) -> np.ndarray:
    """(H x) at the rows whose basis states are `states`, for the vector whose
    entry at basis state s is a fixed function of s alone
    (``workloads.keyed_values``: seeded SplitMix64 of the state, U[-1, 1]).

    Because x is keyed by the state and not by its position, the oracle needs
    no basis list: each row is the diagonal plus the pull-form terms of
    ``orc_row_terms`` weighted by x at the target states.  A device apply of
    the same x (built from the device's own basis order) must agree at every
    row; a wrong position anywhere in the device index gathers another
    state's value.  Every row state must be a basis state (checked here).
    round_to_f32: the keyed values are rounded to FP32 first (the vector as
    an FP32 device vector holds it).  Returns [n] or [n, nvec] complex128."""
    import workloads as W
    s = np.ascontiguousarray(states, dtype=np.uint64)
    diag, inb, cnt, tg, amps = rows_terms(m, s)
    if not np.all(inb):
        raise ValueError(f"{int(np.sum(~inb))} row states are not basis states of {m.name}")

    def f(q):
        v = W.keyed_values(seed, q, nvec=nvec, complex_=complex_)
        if round_to_f32:
            v = (v.astype(np.complex64) if complex_ else v.astype(np.float32)).astype(v.dtype)
        return v.astype(np.complex128).reshape(len(q), nvec)

    nb = tg.shape[1]
    valid = np.arange(nb)[None, :] < cnt[:, None]
    xt = np.zeros((len(s), nb, nvec), np.complex128)
    xt[valid] = f(tg[valid])
    y = diag[:, None] * f(s) + np.einsum("kq,kqv->kv", np.where(valid, amps, 0), xt)
    return y[:, 0] if nvec == 1 else y


def tridiag_eigvals(alpha, beta, k: int) -> np.ndarray:
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    m = len(a)
    b = np.zeros(max(m, 1), np.float64)
    b[: m - 1] = np.asarray(beta, dtype=np.float64)[: m - 1]
    out = np.zeros(k, np.float64)
    if _load().orc_tridiag_eigvals(m, _p(a), _p(b), k, _p(out)) != 0:
        raise ValueError("bad tridiagonal arguments")
    return out


def lanczos(m, basis_list: np.ndarray, x0: np.ndarray, k: int = 1, tol: float = 1e-12,
            max_iter: int = 300, reorth: bool = False):
    """Returns (status, evals[k], alpha[n], beta[n])."""
    perm, chi, sites, jz, jxy = _model_arrays(m)
    b = np.ascontiguousarray(basis_list, dtype=np.uint64)
    x = np.ascontiguousarray(x0, dtype=np.complex128)
    al = np.zeros(max_iter, np.float64)
    be = np.zeros(max_iter, np.float64)
    ev = np.zeros(k, np.float64)
    nit = np.zeros(1, np.int32)
    st = _load().orc_lanczos(m.n_sites, m.n_sym, _p(perm), _p(chi), len(jz), _p(sites), _p(jz),
                             _p(jxy), _p(b), len(b), _p(x), k, tol, max_iter, int(reorth),
                             _p(al), _p(be), _p(nit), _p(ev))
    if st < 0:
        raise RuntimeError(f"orc_lanczos failed ({st})")
    n = int(nit[0])
    return st, ev, al[:n].copy(), be[:n].copy()


# ---------------------------------------------------------------------------
# Eigenvectors and measurements (small cases only; plain definitions)
# ---------------------------------------------------------------------------

def full_states(n_sites: int, n_up: int) -> np.ndarray:
    """All product states with n_up up spins, ascending (the U(1) basis)."""
    lib = _load()
    d = lib.orc_basis(n_sites, n_up, 0, None, None, None, 0)
    out = np.empty(max(d, 1), dtype=np.uint64)
    lib.orc_basis(n_sites, n_up, 0, None, None, _p(out), d)
    return out[:d]


def expand_state(m, basis_list: np.ndarray, psi: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(product states, amplitudes) of sum_s psi_s |s~>, where the symmetric
    state of representative s is |s~> = N_s^-1 sum_g chi(g)* g|s> with
    N_s = sqrt(|G| |Stab s|) (Sec. 3.11).  Pure-Python loops: small cases."""
    full = full_states(m.n_sites, m.n_up)
    amp = np.zeros(len(full), np.complex128)
    if m.perm is None:
        return full, np.asarray(psi, np.complex128).copy()
    G = m.n_sym
    for s, c in zip(basis_list, psi):
        s = int(s)
        images = [act(m.n_sites, g, s) for g in m.perm]
        stab = sum(1 for t in images if t == s)
        ns = np.sqrt(G * stab)
        for t, ch in zip(images, m.chi):
            amp[int(np.searchsorted(full, t))] += c * np.conj(ch) / ns
    return full, amp


def szsz_definition(full: np.ndarray, amp: np.ndarray, a: int, b: int) -> float:
    """<Psi| S^z_a S^z_b |Psi> on a product-state expansion (sz = +-1/2)."""
    ba = (full >> np.uint64(a)) & np.uint64(1)
    bb = (full >> np.uint64(b)) & np.uint64(1)
    v = np.where(ba == bb, 0.25, -0.25)
    return float(np.sum(np.abs(amp) ** 2 * v))


def dense_ground_state(m, basis_list: np.ndarray) -> Tuple[float, np.ndarray]:
    """Lowest eigenpair of the block matrix built column by column from the
    oracle's H x (small cases; LAPACK eigh)."""
    D = len(basis_list)
    H = apply(m, basis_list, np.eye(D, dtype=np.complex128))
    w, v = np.linalg.eigh(H)
    return float(w[0]), v[:, 0]


def dense_sz_spectrum(m_u1, coef) -> Tuple[float, np.ndarray, np.ndarray]:
    """Full U(1) space (no symmetry): ground energy E0 and, for every
    eigenstate n, (E_n - E0, |<n| sum_j coef_j S^z_j |0>|^2).  Dense LAPACK on
    the oracle's matrix; small cases only.  The ground state must be unique."""
    b = basis(m_u1)
    D = len(b)
    H = apply(m_u1, b, np.eye(D, dtype=np.complex128))
    E, U = np.linalg.eigh(H)
    if E[1] - E[0] < 1e-9:
        raise ValueError("degenerate ground state")
    bits = ((b[:, None] >> np.arange(m_u1.n_sites, dtype=np.uint64)[None, :]) & np.uint64(1))
    o = ((bits.astype(np.float64) - 0.5) * np.asarray(coef, np.complex128)[None, :]).sum(axis=1)
    phi = o * U[:, 0]
    w = np.abs(U.conj().T @ phi) ** 2
    return float(E[0]), E - E[0], w


# ---------------------------------------------------------------------------
# Thermal pure quantum states (thermodynamics examples, Sec. 4.6)
# ---------------------------------------------------------------------------

def tpq_micro(m, basis_list: np.ndarray, x0: np.ndarray, l: float, n_steps: int):
    """Microcanonical TPQ sequence (Sugiura and Shimizu 2012) from the unit
    vector x0 / |x0|: |k+1> = (l - H/N)|k>, normalised; returns
    u[k] = <k|H|k> / N and u2[k] = <k|H^2|k> / N^2 for k < n_steps, with the
    oracle's H x in FP64."""
    N = m.n_sites
    v = np.asarray(x0, dtype=np.complex128).ravel()
    v = v / np.linalg.norm(v)
    u = np.zeros(n_steps)
    u2 = np.zeros(n_steps)
    for k in range(n_steps):
        w = apply(m, basis_list, v)
        u[k] = np.vdot(v, w).real / N
        u2[k] = np.vdot(w, w).real / N ** 2
        v = l * v - w / N
        v = v / np.linalg.norm(v)
    return u, u2


def tpq_canonical(u, u2, l: float, n_sites: int, weight, temps):
    """Canonical TPQ thermodynamics (Sugiura and Shimizu 2013) from
    microcanonical sequences u, u2 [n_rec][K]: the canonical state
    exp(-H / 2T)|psi> = exp(-x l / 2) sum_n (x / 2)^n / n! (l - h)^n |psi>,
    h = H/N, x = N/T, so every expectation value in it is a series in the
    moments M_n = <psi|(l - h)^n|psi>.  Those come from the sequence:
    |k> is (l - h)^k |psi> over its norm sqrt(q_k), hence
    M_{2k} = q_k, M_{2k+1} = q_k <k|(l - h)|k>, q_{k+1} = q_k <k|(l - h)^2|k>.
    Returns (energy, heat, log_z) per temperature; NaN where the last kept
    term of a series is not below 1e-12 of its sum.  Plain loops in log
    space (math.lgamma), one sequence at a time."""
    import math
    U = np.atleast_2d(np.asarray(u, np.float64))
    U2 = np.atleast_2d(np.asarray(u2, np.float64))
    R, K = U.shape
    wts = np.broadcast_to(np.asarray(weight, np.float64), (R,))
    logM = []
    for r in range(R):
        lm = [-math.inf] * (2 * K + 1)
        lq = 0.0
        for k in range(K):
            lm[2 * k] = lq
            a = l - U[r, k]
            lm[2 * k + 1] = lq + math.log(a) if a > 0 else -math.inf
            q = l * l - 2 * l * U[r, k] + U2[r, k]
            if q <= 0:
                break
            lq += math.log(q)
            if k == K - 1:
                lm[2 * K] = lq
        logM.append(lm)
    N = n_sites
    energy, heat, log_z = [], [], []
    for T in np.asarray(temps, np.float64):
        x = N / T
        logS, ok = [], True
        for j in range(3):
            terms, lasts = [], []
            for r in range(R):
                for n in range(2 * K - j + 1):
                    t = math.log(wts[r]) + logM[r][n + j] + n * math.log(x) - math.lgamma(n + 1)
                    terms.append(t)
                    if n == 2 * K - j:
                        lasts.append(t)
            top = max(terms)
            s = sum(math.exp(t - top) for t in terms)
            last = sum(math.exp(t - top) for t in lasts)
            if last > 1e-12 * s:
                ok = False
            logS.append(top + math.log(s))
        a1 = math.exp(logS[1] - logS[0])
        a2 = math.exp(logS[2] - logS[0])
        energy.append(N * (l - a1) if ok else math.nan)
        heat.append(x * x * (a2 - a1 * a1) if ok else math.nan)
        log_z.append(logS[0] - x * l if ok else math.nan)
    return np.array(energy), np.array(heat), np.array(log_z)
