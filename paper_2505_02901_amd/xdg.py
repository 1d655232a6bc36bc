"""ctypes binding of ``include/xdg.h`` (argument marshalling only).

Every function keeps the C name; handles are ``ctypes.c_void_p``; vectors
are torch tensors on the GPU (or raw device pointers as ints).  Every step
of the computation runs in ``libxdg.so``; if the library is not built this
module refuses to load.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxdg.so")

XDG_OK, XDG_EINVAL, XDG_EGROUP, XDG_ECHAR, XDG_ENOTSYM, XDG_ENOMEM, XDG_EHIP, XDG_ENOCONV = (
    0, -1, -2, -3, -4, -5, -6, -7)
XDG_F64, XDG_F32, XDG_C128, XDG_C64 = 0, 1, 2, 3
XDG_SEARCH_AUTO, XDG_SEARCH_U1, XDG_SEARCH_AFFINE, XDG_SEARCH_SUBLATTICE, XDG_SEARCH_TABLE = (
    0, 1, 2, 3, 4)
XDG_PREC_F64, XDG_PREC_F32VEC, XDG_PREC_F32VEC_REORTH, XDG_PREC_F64_REORTH = 0, 1, 2, 3

ERROR_NAMES = {0: "XDG_OK", -1: "XDG_EINVAL", -2: "XDG_EGROUP", -3: "XDG_ECHAR",
               -4: "XDG_ENOTSYM", -5: "XDG_ENOMEM", -6: "XDG_EHIP", -7: "XDG_ENOCONV"}


class XdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class LaunchCfg(C.Structure):
    _fields_ = [("grid", C.c_int), ("nv", C.c_int), ("occ", C.c_int), ("compact", C.c_int),
                ("sub_form", C.c_int), ("xr", C.c_int), ("reserved", C.c_int * 2)]


class BasisOpts(C.Structure):
    _fields_ = [("search", C.c_int), ("n_sublattices", C.c_int), ("flags", C.c_int),
                ("reserved", C.c_int * 5)]


XDG_FLAG_F32_ACCUMULATE = 2
XDG_FLAG_HASH_INDEX = 4
XDG_INDEX_LIN, XDG_INDEX_HASH, XDG_INDEX_RANK = 1, 2, 3


_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2505_02901_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        P, I, I64, D, U64 = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_uint64
        sig = {
            "xdg_version": (C.c_char_p, []),
            "xdg_last_error": (C.c_char_p, []),
            "xdg_check_group": (I, [I, I, P, P]),
            "xdg_check_bonds": (I, [I, I, P, I, P, P, P]),
            "xdg_plan_search": (I, [I, I, P, P, P, P]),
            "xdg_create_basis": (I, [I, I, I, P, P, P, P]),
            "xdg_destroy_basis": (None, [P]),
            "xdg_basis_dim": (I, [P, P]),
            "xdg_basis_is_complex": (I, [P, P]),
            "xdg_basis_search_kind": (I, [P, P, P]),
            "xdg_basis_index_kind": (I, [P, P, P]),
            "xdg_basis_copy_states": (I, [P, I64, I64, P]),
            "xdg_basis_copy_stabilisers": (I, [P, I64, I64, P]),
            "xdg_basis_index": (I, [P, P, I64, P]),
            "xdg_create_hamiltonian": (I, [P, I, P, P, P, P]),
            "xdg_destroy_hamiltonian": (None, [P]),
            "xdg_ham_nnz": (I, [P, P]),
            "xdg_ham_dim": (I, [P, P, P]),
            "xdg_set_device_memory_limit": (I, [I64, P]),
            "xdg_apply": (I, [P, P, P, I64, I, P]),
            "xdg_apply_batched": (I, [I, P, P, P, I64, I, P]),
            "xdg_apply_batched_noalloc": (I, [I, P, P, P, I64, I, P]),
            "xdg_apply_with_config": (I, [P, P, P, I64, I, P, P]),
            "xdg_apply_tuned_config": (I, [P, I, I64, P]),
            "xdg_random_state": (I, [I64, I64, U64, I, I, P, P]),
            "xdg_lanczos_eigval": (I, [P, P, I, D, I, U64, I, P, P, P, P, P]),
            "xdg_lanczos_eigval_batched": (I, [I, P, P, I64, I, U64, I, P, P, P, P]),
            "xdg_last_lanczos_timing": (I, [P, P]),
            "xdg_lanczos_eigvec": (I, [P, P, U64, I, I, P, P, I, P, P, P]),
            "xdg_expect_szsz": (I, [P, P, I, I, P, P, P]),
            "xdg_ftlm_thermo": (I, [I, I, P, P, P, I, P, P, P, P]),
            "xdg_tpq_micro": (I, [P, P, U64, I, D, I, P, P, P]),
            "xdg_tpq_micro_batched": (I, [I, P, P, I64, U64, I, D, I, P, P, P]),
            "xdg_tpq_thermo": (I, [I, I, P, P, D, I, P, I, P, P, P, P]),
            "xdg_apply_sz_transfer": (I, [P, P, P, P, P, I, P]),
            "xdg_spectral_cf": (I, [I, P, P, D, D, I, P, D, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return ["xdg_version", "xdg_last_error", "xdg_check_group", "xdg_check_bonds",
            "xdg_plan_search", "xdg_create_basis", "xdg_destroy_basis", "xdg_basis_dim",
            "xdg_basis_is_complex", "xdg_basis_search_kind", "xdg_basis_index_kind",
            "xdg_basis_copy_states",
            "xdg_basis_copy_stabilisers", "xdg_basis_index", "xdg_create_hamiltonian",
            "xdg_destroy_hamiltonian", "xdg_ham_nnz", "xdg_ham_dim",
            "xdg_set_device_memory_limit", "xdg_apply",
            "xdg_apply_batched", "xdg_apply_batched_noalloc", "xdg_apply_with_config",
            "xdg_apply_tuned_config",
            "xdg_random_state", "xdg_lanczos_eigval", "xdg_lanczos_eigval_batched",
            "xdg_last_lanczos_timing", "xdg_lanczos_eigvec", "xdg_expect_szsz",
            "xdg_ftlm_thermo", "xdg_tpq_micro", "xdg_tpq_micro_batched", "xdg_tpq_thermo",
            "xdg_apply_sz_transfer",
            "xdg_spectral_cf"]


def _check(rc: int, allow=(XDG_OK,)):
    if rc not in allow:
        raise XdgError(rc, xdg_last_error())
    return rc


def _arr(a, dtype):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _chi_arr(chi, n_sym):
    if chi is None:
        return None, None
    chi = np.asarray(chi)
    if np.iscomplexobj(chi) or chi.ndim == 1:
        c = np.empty((n_sym, 2), np.float64)
        c[:, 0] = np.real(chi)
        c[:, 1] = np.imag(chi)
    else:
        c = np.asarray(chi, np.float64).reshape(n_sym, 2)
    return _arr(c, np.float64)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("vectors passed to the library must be device tensors")
    if not t.is_contiguous():
        raise ValueError("vectors passed to the library must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:  # pragma: no cover
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _is_tensor(t) -> bool:
    return t is not None and not isinstance(t, int)


def _check_vec(name: str, t, dim: int, nvec: int, dtype: Optional[int] = None) -> None:
    """Refuse (ValueError, before any launch) a tensor that does not hold a
    [dim][nvec] block of the expected dtype.  Raw integer pointers are passed
    through unchecked: their size is the caller's responsibility."""
    if not _is_tensor(t):
        return
    need = dim * nvec
    if t.numel() != need:
        raise ValueError(f"{name} has {t.numel()} elements; the block needs dim {dim} x "
                         f"nvec {nvec} = {need}")
    if t.dim() > 2 or (t.dim() == 2 and int(t.shape[1]) != nvec):
        raise ValueError(f"{name} must have shape [dim] or [dim, nvec={nvec}], got "
                         f"{tuple(t.shape)}")
    if dtype is not None and _dtype_code(t) != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}; this call needs "
                         f"{_DTYPE_NAMES[dtype]}")


_DTYPE_NAMES = {XDG_F64: "float64", XDG_F32: "float32", XDG_C128: "complex128",
                XDG_C64: "complex64"}


def _prec_dtype(prec: int, cplx: bool) -> int:
    single = prec in (XDG_PREC_F32VEC, XDG_PREC_F32VEC_REORTH)
    return {(False, False): XDG_F64, (True, False): XDG_F32, (False, True): XDG_C128,
            (True, True): XDG_C64}[(single, cplx)]


def _same_storage(a, b) -> bool:
    """Both tensors hold elements and start at the same address (empty
    tensors have no storage to share)."""
    return (_is_tensor(a) and _is_tensor(b) and a.numel() > 0 and b.numel() > 0
            and a.data_ptr() == b.data_ptr())


def _dtype_code(t) -> int:
    import torch
    m = {torch.float64: XDG_F64, torch.float32: XDG_F32, torch.complex128: XDG_C128,
         torch.complex64: XDG_C64}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


# ------------------------------------------------------------------ C names --

def xdg_set_device_memory_limit(bytes_: int) -> int:
    """Cap the device memory of the library's own buffers (0 = no cap);
    returns what they hold now."""
    used = C.c_int64()
    _check(lib().xdg_set_device_memory_limit(int(bytes_), C.byref(used)))
    return used.value


def xdg_version() -> str:
    return lib().xdg_version().decode()


def xdg_last_error() -> str:
    return lib().xdg_last_error().decode()


def xdg_check_group(n_sites: int, perm, chi=None) -> int:
    perm, pp = _arr(perm, np.int32)
    n_sym = 0 if perm is None else perm.shape[0]
    chi, pc = _chi_arr(chi, n_sym)
    return lib().xdg_check_group(n_sites, n_sym, pp, pc)


def xdg_check_bonds(n_sites: int, perm, sites, jz, jxy) -> int:
    perm, pp = _arr(perm, np.int32)
    n_sym = 0 if perm is None else perm.shape[0]
    sites, ps = _arr(sites, np.int32)
    jz, pz = _arr(jz, np.float64)
    jxy, px = _arr(jxy, np.float64)
    return lib().xdg_check_bonds(n_sites, n_sym, pp, len(jz), ps, pz, px)


def xdg_plan_search(n_sites: int, perm, search: int = 0, n_sublattices: int = 0,
                    flags: int = 0):
    perm, pp = _arr(perm, np.int32)
    n_sym = 0 if perm is None else perm.shape[0]
    o = BasisOpts(search, n_sublattices, flags)
    k, ns = C.c_int(), C.c_int()
    _check(lib().xdg_plan_search(n_sites, n_sym, pp, C.byref(o), C.byref(k), C.byref(ns)))
    return k.value, ns.value


def xdg_create_basis(n_sites: int, n_up: int, perm=None, chi=None, search: int = 0,
                     n_sublattices: int = 0, flags: int = 0):
    perm, pp = _arr(perm, np.int32)
    n_sym = 0 if perm is None else perm.shape[0]
    chi, pc = _chi_arr(chi, n_sym)
    o = BasisOpts(search, n_sublattices, flags)
    h = C.c_void_p()
    _check(lib().xdg_create_basis(n_sites, n_up, n_sym, pp, pc, C.byref(o), C.byref(h)))
    return h


def xdg_destroy_basis(b) -> None:
    lib().xdg_destroy_basis(b)


def xdg_basis_dim(b) -> int:
    d = C.c_int64()
    _check(lib().xdg_basis_dim(b, C.byref(d)))
    return d.value


def xdg_basis_is_complex(b) -> bool:
    v = C.c_int()
    _check(lib().xdg_basis_is_complex(b, C.byref(v)))
    return bool(v.value)


def xdg_basis_search_kind(b) -> Tuple[int, int]:
    k, ns = C.c_int(), C.c_int()
    _check(lib().xdg_basis_search_kind(b, C.byref(k), C.byref(ns)))
    return k.value, ns.value


def xdg_basis_index_kind(b) -> Tuple[int, int]:
    """(XDG_INDEX_* kind, device bytes of the index)."""
    k, n = C.c_int(), C.c_int64()
    _check(lib().xdg_basis_index_kind(b, C.byref(k), C.byref(n)))
    return k.value, n.value


def xdg_basis_copy_states(b, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
    if count is None:
        count = xdg_basis_dim(b) - begin
    out = np.empty(max(count, 0), np.uint64)
    _check(lib().xdg_basis_copy_states(b, begin, count, out.ctypes.data_as(C.c_void_p)))
    return out


def xdg_basis_copy_stabilisers(b, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
    if count is None:
        count = xdg_basis_dim(b) - begin
    out = np.empty(max(count, 0), np.int32)
    _check(lib().xdg_basis_copy_stabilisers(b, begin, count, out.ctypes.data_as(C.c_void_p)))
    return out


def xdg_basis_index(b, states) -> np.ndarray:
    s, ps = _arr(np.atleast_1d(np.asarray(states, dtype=np.uint64)), np.uint64)
    out = np.empty(len(s), np.int64)
    _check(lib().xdg_basis_index(b, ps, len(s), out.ctypes.data_as(C.c_void_p)))
    return out


def xdg_create_hamiltonian(b, sites, jz, jxy):
    sites, ps = _arr(sites, np.int32)
    jz, pz = _arr(jz, np.float64)
    jxy, px = _arr(jxy, np.float64)
    h = C.c_void_p()
    _check(lib().xdg_create_hamiltonian(b, len(jz), ps, pz, px, C.byref(h)))
    return h


def xdg_destroy_hamiltonian(h) -> None:
    lib().xdg_destroy_hamiltonian(h)


def xdg_ham_nnz(h) -> int:
    n = C.c_int64()
    _check(lib().xdg_ham_nnz(h, C.byref(n)))
    return n.value


def xdg_ham_dim(h) -> Tuple[int, bool]:
    """(dimension of the Hamiltonian's block, whether the block is complex)."""
    d, c = C.c_int64(), C.c_int()
    _check(lib().xdg_ham_dim(h, C.byref(d), C.byref(c)))
    return d.value, bool(c.value)


def _check_apply_vectors(h, x, y, nvec: int, dtype: int, where: str = "") -> None:
    dim, _ = xdg_ham_dim(h)
    _check_vec(f"x{where}", x, dim, nvec, dtype)
    _check_vec(f"y{where}", y, dim, nvec, dtype)
    if _same_storage(x, y):
        raise ValueError(f"x{where} and y{where} must be distinct buffers")


def xdg_apply(h, x, y, nvec: Optional[int] = None, dtype: Optional[int] = None, stream=None):
    if nvec is None:
        nvec = 1 if x.dim() == 1 else int(x.shape[1])
    if dtype is None:
        dtype = _dtype_code(x)
    _check_apply_vectors(h, x, y, nvec, dtype)
    _check(lib().xdg_apply(h, _ptr(x), _ptr(y), nvec, dtype, _stream(stream)))


def xdg_apply_with_config(h, x, y, grid: int = 0, nv: int = 0, occ: int = -1, compact: int = -1,
                          nvec: Optional[int] = None, dtype: Optional[int] = None, stream=None,
                          sub_form: int = 0, xr: int = 0):
    """xdg_apply in an explicit launch shape (every shape gives the same y)."""
    if nvec is None:
        nvec = 1 if x.dim() == 1 else int(x.shape[1])
    if dtype is None:
        dtype = _dtype_code(x)
    _check_apply_vectors(h, x, y, nvec, dtype)
    cfg = LaunchCfg(grid, nv, occ, compact, sub_form, xr)
    _check(lib().xdg_apply_with_config(h, _ptr(x), _ptr(y), nvec, dtype, C.byref(cfg),
                                       _stream(stream)))


def xdg_apply_tuned_config(h, dtype: int, nvec: int = 1) -> dict:
    """The autotuner's launch shape for (dtype, nvec) on this Hamiltonian."""
    cfg = LaunchCfg()
    _check(lib().xdg_apply_tuned_config(h, dtype, nvec, C.byref(cfg)))
    return {"grid": cfg.grid, "nv": cfg.nv, "occ": cfg.occ, "compact": cfg.compact,
            "sub_form": cfg.sub_form, "xr": cfg.xr}


def xdg_apply_batched(hams: Sequence, xs: Sequence, ys: Sequence, nvec: Optional[int] = None,
                      dtype: Optional[int] = None, stream=None):
    n = len(hams)
    if len(xs) != n or len(ys) != n:
        raise ValueError("hams, xs and ys must have the same length")
    if nvec is None:
        nvec = 1 if xs[0].dim() == 1 else int(xs[0].shape[1])
    if dtype is None:
        dtype = _dtype_code(xs[0])
    for i in range(n):
        _check_apply_vectors(hams[i], xs[i], ys[i], nvec, dtype, f"[{i}]")
    H = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in hams])
    X = (C.c_void_p * n)(*[_ptr(x) for x in xs])
    Y = (C.c_void_p * n)(*[_ptr(y) for y in ys])
    _check(lib().xdg_apply_batched(n, H, X, Y, nvec, dtype, _stream(stream)))


def xdg_apply_batched_noalloc(hams: Sequence, xs: Sequence, ys: Sequence,
                              nvec: Optional[int] = None, dtype: Optional[int] = None,
                              stream=None):
    """xdg_apply_batched without any device allocation (at most 128 blocks)."""
    n = len(hams)
    if len(xs) != n or len(ys) != n:
        raise ValueError("hams, xs and ys must have the same length")
    if nvec is None:
        nvec = 1 if xs[0].dim() == 1 else int(xs[0].shape[1])
    if dtype is None:
        dtype = _dtype_code(xs[0])
    for i in range(n):
        _check_apply_vectors(hams[i], xs[i], ys[i], nvec, dtype, f"[{i}]")
    H = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in hams])
    X = (C.c_void_p * n)(*[_ptr(x) for x in xs])
    Y = (C.c_void_p * n)(*[_ptr(y) for y in ys])
    _check(lib().xdg_apply_batched_noalloc(n, H, X, Y, nvec, dtype, _stream(stream)))


def xdg_random_state(out, seed: int, kind: int = 1, nvec: Optional[int] = None, stream=None):
    nvec = nvec or (1 if out.dim() == 1 else int(out.shape[1]))
    dim = int(out.shape[0])
    _check(lib().xdg_random_state(dim, nvec, seed, kind, _dtype_code(out), _ptr(out),
                                  _stream(stream)))


def xdg_lanczos_eigval(h, k: int = 1, tol: float = 1e-12, max_iter: int = 300, seed: int = 0,
                       prec: int = XDG_PREC_F64, v0=None, stream=None):
    """Returns (status, evals, alpha, beta)."""
    if _is_tensor(v0):
        dim, cplx = xdg_ham_dim(h)
        _check_vec("v0", v0, dim, 1, _prec_dtype(prec, cplx))
    ev = np.zeros(k, np.float64)
    al = np.zeros(max_iter, np.float64)
    be = np.zeros(max_iter, np.float64)
    nit = C.c_int()
    rc = lib().xdg_lanczos_eigval(h, _ptr(v0), k, tol, max_iter, seed, prec,
                                  ev.ctypes.data_as(C.c_void_p), C.byref(nit),
                                  al.ctypes.data_as(C.c_void_p), be.ctypes.data_as(C.c_void_p),
                                  _stream(stream))
    _check(rc, allow=(XDG_OK, XDG_ENOCONV))
    n = nit.value
    return rc, ev, al[:n].copy(), be[:n].copy()


def xdg_lanczos_eigval_batched(hams: Sequence, nvec: int, n_iter: int, seed: int = 0,
                               prec: int = XDG_PREC_F32VEC, v0s=None, stream=None):
    """Returns (evals [n, nvec], alpha [n, nvec, n_iter], beta [...])."""
    n = len(hams)
    if v0s is not None:
        if len(v0s) != n:
            raise ValueError("one start block per Hamiltonian")
        info = [xdg_ham_dim(h) for h in hams]
        dt = _prec_dtype(prec, any(c for _, c in info))
        for i, (dim, _) in enumerate(info):
            _check_vec(f"v0s[{i}]", v0s[i], dim, nvec, dt)
    ev = np.zeros(n * nvec, np.float64)
    al = np.zeros(n * nvec * n_iter, np.float64)
    be = np.zeros(n * nvec * n_iter, np.float64)
    H = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in hams])
    V = None if v0s is None else (C.c_void_p * n)(*[_ptr(v) for v in v0s])
    _check(lib().xdg_lanczos_eigval_batched(n, H, V, nvec, n_iter, seed, prec,
                                            ev.ctypes.data_as(C.c_void_p),
                                            al.ctypes.data_as(C.c_void_p),
                                            be.ctypes.data_as(C.c_void_p), _stream(stream)))
    return ev.reshape(n, nvec), al.reshape(n, nvec, n_iter), be.reshape(n, nvec, n_iter)


def xdg_lanczos_eigvec(h, alpha, beta, psi, seed: int = 0, prec: int = XDG_PREC_F64, v0=None,
                       which: int = 0, stream=None) -> float:
    """Second Lanczos pass into the device tensor psi; returns the Ritz value."""
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    if len(be) < len(al):
        raise ValueError("beta needs as many entries as alpha")
    dim, cplx = xdg_ham_dim(h)
    dt = _prec_dtype(prec, cplx)
    _check_vec("psi", psi, dim, 1, dt)
    _check_vec("v0", v0, dim, 1, dt)
    if _same_storage(psi, v0):
        raise ValueError("psi may not alias v0")
    r = C.c_double()
    _check(lib().xdg_lanczos_eigvec(h, _ptr(v0), seed, prec, len(al),
                                    al.ctypes.data_as(C.c_void_p), be.ctypes.data_as(C.c_void_p),
                                    which, _ptr(psi), C.byref(r), _stream(stream)))
    return r.value


def xdg_expect_szsz(b, psi, pairs, dtype: Optional[int] = None, stream=None) -> np.ndarray:
    """<psi| (1/|G|) sum_g S^z_g(a) S^z_g(b) |psi> for each (a, b) in pairs."""
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    out = np.zeros(len(p), np.float64)
    if dtype is None:
        dtype = _dtype_code(psi)
    _check_vec("psi", psi, xdg_basis_dim(b), 1, dtype)
    _check(lib().xdg_expect_szsz(b, _ptr(psi), dtype, len(p), p.ctypes.data_as(C.c_void_p),
                                 out.ctypes.data_as(C.c_void_p), _stream(stream)))
    return out


def xdg_ftlm_thermo(alpha, beta, weight, temps):
    """(energy, heat, log_z) per temperature from Lanczos recurrences
    alpha, beta [n_rec, m] with weights [n_rec]."""
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    m = al.shape[-1]
    al = al.reshape(-1, m)
    be = be.reshape(-1, m)
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(weight, np.float64), (al.shape[0],)))
    T = np.ascontiguousarray(temps, dtype=np.float64)
    e, c, z = (np.zeros(len(T)) for _ in range(3))
    _check(lib().xdg_ftlm_thermo(al.shape[0], m, al.ctypes.data_as(C.c_void_p),
                                 be.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                                 len(T), T.ctypes.data_as(C.c_void_p), e.ctypes.data_as(C.c_void_p),
                                 c.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p)))
    return e, c, z


def xdg_tpq_micro(h, l: float, n_steps: int, seed: int = 0, prec: int = XDG_PREC_F64, v0=None,
                  stream=None):
    """(u, u2) of the microcanonical TPQ sequence |k+1> ~ (l - H/N)|k>:
    u[k] = <k|H|k>/N, u2[k] = <k|H^2|k>/N^2."""
    if _is_tensor(v0):
        dim, cplx = xdg_ham_dim(h)
        _check_vec("v0", v0, dim, 1, _prec_dtype(prec, cplx))
    u = np.zeros(n_steps, np.float64)
    u2 = np.zeros(n_steps, np.float64)
    _check(lib().xdg_tpq_micro(h, _ptr(v0), seed, prec, l, n_steps,
                               u.ctypes.data_as(C.c_void_p), u2.ctypes.data_as(C.c_void_p),
                               _stream(stream)))
    return u, u2


def xdg_tpq_micro_batched(hams: Sequence, l: float, n_steps: int, nvec: int, seed: int = 0,
                          prec: int = XDG_PREC_F32VEC, v0s=None, stream=None):
    """(u, u2) [n, nvec, n_steps] of TPQ sequences for every block and start
    vector in lockstep (one batched H x per step)."""
    n = len(hams)
    if v0s is not None:
        if len(v0s) != n:
            raise ValueError("one start block per Hamiltonian")
        info = [xdg_ham_dim(h) for h in hams]
        dt = _prec_dtype(prec, any(c for _, c in info))
        for i, (dim, _) in enumerate(info):
            _check_vec(f"v0s[{i}]", v0s[i], dim, nvec, dt)
    u = np.zeros(n * nvec * n_steps, np.float64)
    u2 = np.zeros(n * nvec * n_steps, np.float64)
    H = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in hams])
    V = None if v0s is None else (C.c_void_p * n)(*[_ptr(v) for v in v0s])
    _check(lib().xdg_tpq_micro_batched(n, H, V, nvec, seed, prec, l, n_steps,
                                       u.ctypes.data_as(C.c_void_p),
                                       u2.ctypes.data_as(C.c_void_p), _stream(stream)))
    return u.reshape(n, nvec, n_steps), u2.reshape(n, nvec, n_steps)


def xdg_tpq_thermo(u, u2, l: float, n_sites: int, weight, temps):
    """(energy, heat, log_z) per temperature from microcanonical TPQ
    sequences u, u2 [n_rec, n_steps] with weights [n_rec] (canonical TPQ)."""
    uu = np.ascontiguousarray(u, dtype=np.float64)
    K = uu.shape[-1]
    uu = uu.reshape(-1, K)
    vv = np.ascontiguousarray(u2, dtype=np.float64).reshape(-1, K)
    if vv.shape != uu.shape:
        raise ValueError("u and u2 must have the same shape")
    w = np.ascontiguousarray(np.broadcast_to(np.asarray(weight, np.float64), (uu.shape[0],)))
    T = np.ascontiguousarray(temps, dtype=np.float64)
    e, c, z = (np.zeros(len(T)) for _ in range(3))
    _check(lib().xdg_tpq_thermo(uu.shape[0], K, uu.ctypes.data_as(C.c_void_p),
                                vv.ctypes.data_as(C.c_void_p), l, n_sites,
                                w.ctypes.data_as(C.c_void_p), len(T),
                                T.ctypes.data_as(C.c_void_p), e.ctypes.data_as(C.c_void_p),
                                c.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p)))
    return e, c, z


def xdg_apply_sz_transfer(b_in, b_out, coef, x, y, dtype: Optional[int] = None, stream=None):
    """y = (sum_j coef_j S^z_j) x from block b_in to block b_out."""
    c = np.asarray(coef, dtype=np.complex128)
    ci = np.empty((len(c), 2), np.float64)
    ci[:, 0], ci[:, 1] = c.real, c.imag
    if dtype is None:
        dtype = _dtype_code(x)
    _check_vec("x", x, xdg_basis_dim(b_in), 1, dtype)
    _check_vec("y", y, xdg_basis_dim(b_out), 1, dtype)
    if _same_storage(x, y):
        raise ValueError("x and y must be distinct buffers")
    _check(lib().xdg_apply_sz_transfer(b_in, b_out, ci.ctypes.data_as(C.c_void_p), _ptr(x),
                                       _ptr(y), dtype, _stream(stream)))
    return y


def xdg_spectral_cf(alpha, beta, norm2: float, e0: float, omega, eta: float) -> np.ndarray:
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    w = np.ascontiguousarray(omega, dtype=np.float64)
    out = np.zeros(len(w))
    _check(lib().xdg_spectral_cf(len(al), al.ctypes.data_as(C.c_void_p),
                                 be.ctypes.data_as(C.c_void_p), norm2, e0, len(w),
                                 w.ctypes.data_as(C.c_void_p), eta, out.ctypes.data_as(C.c_void_p)))
    return out


def xdg_last_lanczos_timing() -> Tuple[float, float]:
    t, a = C.c_double(), C.c_double()
    _check(lib().xdg_last_lanczos_timing(C.byref(t), C.byref(a)))
    return t.value, a.value


# ----------------------------------------------------------- thin wrappers --

class Basis:
    """Owning wrapper of an ``xdg_basis`` handle."""

    def __init__(self, n_sites: int, n_up: int, perm=None, chi=None, search: int = 0,
                 n_sublattices: int = 0, flags: int = 0):
        self.handle = xdg_create_basis(n_sites, n_up, perm, chi, search, n_sublattices, flags)
        self.n_sites = n_sites
        self.n_up = n_up

    @classmethod
    def from_model(cls, m, **kw) -> "Basis":
        return cls(m.n_sites, m.n_up, m.perm, m.chi, **kw)

    @property
    def dim(self) -> int:
        return xdg_basis_dim(self.handle)

    @property
    def is_complex(self) -> bool:
        return xdg_basis_is_complex(self.handle)

    @property
    def search_kind(self) -> Tuple[int, int]:
        return xdg_basis_search_kind(self.handle)

    @property
    def index_kind(self) -> Tuple[int, int]:
        return xdg_basis_index_kind(self.handle)

    def states(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        return xdg_basis_copy_states(self.handle, begin, count)

    def stabilisers(self, begin: int = 0, count: Optional[int] = None) -> np.ndarray:
        return xdg_basis_copy_stabilisers(self.handle, begin, count)

    def index(self, states) -> np.ndarray:
        return xdg_basis_index(self.handle, states)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            xdg_destroy_basis(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hamiltonian:
    """Owning wrapper of an ``xdg_ham`` handle."""

    def __init__(self, basis: Basis, sites, jz, jxy):
        self.basis = basis
        self.handle = xdg_create_hamiltonian(basis.handle, sites, jz, jxy)

    @classmethod
    def from_model(cls, basis: Basis, m) -> "Hamiltonian":
        return cls(basis, m.sites, m.jz, m.jxy)

    @property
    def nnz(self) -> int:
        return xdg_ham_nnz(self.handle)

    def apply(self, x, y, stream=None):
        xdg_apply(self.handle, x, y, stream=stream)
        return y

    def lanczos(self, **kw):
        return xdg_lanczos_eigval(self.handle, **kw)

    def tpq(self, l: float, n_steps: int, **kw):
        return xdg_tpq_micro(self.handle, l, n_steps, **kw)

    def eig0(self, tol: float = 1e-12, max_iter: int = 300, seed: int = 0,
             prec: int = XDG_PREC_F64, v0=None, stream=None):
        """Lowest eigenvalue and normalised eigenvector (two Lanczos passes)."""
        import torch
        st, ev, al, be = xdg_lanczos_eigval(self.handle, k=1, tol=tol, max_iter=max_iter,
                                           seed=seed, prec=prec, v0=v0, stream=stream)
        single = prec in (XDG_PREC_F32VEC, XDG_PREC_F32VEC_REORTH)
        cplx = self.basis.is_complex
        dt = {(False, False): torch.float64, (True, False): torch.float32,
              (False, True): torch.complex128, (True, True): torch.complex64}[(single, cplx)]
        psi = torch.empty(self.basis.dim, dtype=dt, device="cuda")
        e = xdg_lanczos_eigvec(self.handle, al, be, psi, seed=seed, prec=prec, v0=v0,
                               stream=stream)
        return e, psi, al, be

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            xdg_destroy_hamiltonian(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
