"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark: lattices, bond lists, permutation groups, characters and random
vectors.

This module holds none of the method's arithmetic (no group action, no
representative search, no Hamiltonian): it only produces the data that the
method consumes, exactly as a user would hand it to ``Spinhalf(N, nup,
irrep)`` and an ``OpSum`` of ``SdotS``/``SzSz``/``Exchange`` terms (XDiag
Sec. 3.1, 3.2, 3.10, 3.11, Appendix A).

Permutations are given as integer rows ``perm[g][i] = g(i)`` (0-based, as in
the C++ listings of Sec. 3.10.1); characters as complex numbers per group
element, in the same order.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------
# Model container
# --------------------------------------------------------------------------


@dataclasses.dataclass
class Model:
    """A spin-1/2 XXZ problem on one symmetry sector.

    H = sum_b [ jz[b] Sz_i Sz_j + jxy[b]/2 (S+_i S-_j + S-_i S+_j) ]
    (Appendix A: ``SzSz`` plus ``Exchange``; ``SdotS`` is jz = jxy = J).
    ``perm`` is None for the U(1)-only block ``Spinhalf(N, nup)``.
    """

    name: str
    n_sites: int
    n_up: int
    sites: np.ndarray            # int32 [n_bonds, 2]
    jz: np.ndarray               # float64 [n_bonds]
    jxy: np.ndarray              # float64 [n_bonds]
    perm: Optional[np.ndarray] = None   # int32 [n_sym, n_sites]
    chi: Optional[np.ndarray] = None    # complex128 [n_sym]

    @property
    def n_sym(self) -> int:
        return 0 if self.perm is None else int(self.perm.shape[0])

    @property
    def is_complex(self) -> bool:
        return self.chi is not None and bool(np.any(np.abs(self.chi.imag) > 1e-14))

    def chi_interleaved(self) -> Optional[np.ndarray]:
        if self.chi is None:
            return None
        out = np.empty((len(self.chi), 2), dtype=np.float64)
        out[:, 0] = self.chi.real
        out[:, 1] = self.chi.imag
        return np.ascontiguousarray(out)

    def with_sector(self, perm, chi, name=None) -> "Model":
        return dataclasses.replace(self, perm=perm, chi=chi, name=name or self.name)


# --------------------------------------------------------------------------
# Chains
# --------------------------------------------------------------------------


def chain_bonds(n_sites: int, J: float = 1.0, delta: float = 1.0, periodic: bool = True):
    """Nearest-neighbour bonds (i, i+1) of a ring (Sec. 3 Heisenberg chain,
    XXZ form of the entanglement example): jz = J*delta, jxy = J."""
    n_b = n_sites if periodic else n_sites - 1
    sites = np.array([(i, (i + 1) % n_sites) for i in range(n_b)], dtype=np.int32)
    jz = np.full(n_b, J * delta, dtype=np.float64)
    jxy = np.full(n_b, J, dtype=np.float64)
    return sites, jz, jxy


def chain_translations(n_sites: int) -> np.ndarray:
    """The cyclic group {T^0, ..., T^(N-1)} with T(i) = i+1 mod N, element n
    being T^n (Sec. 3.10.1)."""
    return np.array([[(i + n) % n_sites for i in range(n_sites)] for n in range(n_sites)],
                    dtype=np.int32)


def chain_dihedral(n_sites: int) -> np.ndarray:
    """Translations followed by translations composed with the reflection
    i -> -i mod N."""
    rows = [[(i + n) % n_sites for i in range(n_sites)] for n in range(n_sites)]
    rows += [[(n - i) % n_sites for i in range(n_sites)] for n in range(n_sites)]
    return np.array(rows, dtype=np.int32)


def momentum_characters(n_sites: int, l: int) -> np.ndarray:
    """chi_k(T^n) = exp(i k n) with k = 2 pi l / N (Sec. 3.10.2)."""
    n = np.arange(n_sites)
    ang = 2.0 * np.pi * ((l * n) % n_sites) / n_sites
    chi = np.exp(1j * ang)
    # exact values where they are exact
    chi.real[np.isclose(chi.real, 0.0, atol=1e-15)] = 0.0
    chi.imag[np.isclose(chi.imag, 0.0, atol=1e-15)] = 0.0
    chi.real[np.isclose(chi.real, 1.0, atol=1e-15)] = 1.0
    chi.real[np.isclose(chi.real, -1.0, atol=1e-15)] = -1.0
    return chi


def chain_model(n_sites: int, n_up: Optional[int] = None, l: Optional[int] = None,
                J: float = 1.0, delta: float = 1.0) -> Model:
    """Heisenberg/XXZ ring; ``l`` selects the momentum sector k = 2 pi l / N
    (None = U(1) block only)."""
    if n_up is None:
        n_up = n_sites // 2
    sites, jz, jxy = chain_bonds(n_sites, J, delta)
    m = Model(f"chain{n_sites}", n_sites, n_up, sites, jz, jxy)
    if l is not None:
        m = m.with_sector(chain_translations(n_sites), momentum_characters(n_sites, l),
                          f"chain{n_sites}_k{l}")
    return m


# --------------------------------------------------------------------------
# Square-lattice tori (rectangular and tilted), J1-J2 couplings
# --------------------------------------------------------------------------


class Torus:
    """Integer points of the plane modulo the lattice spanned by two period
    vectors a1, a2.  Sites are labelled sublattice-blocked when every
    period has even components: site = q * m + w with q = (x mod 2) +
    2 (y mod 2), m = N / 4 and w the rank of the point within its
    sublattice; otherwise row-major in the order found."""

    def __init__(self, a1: Tuple[int, int], a2: Tuple[int, int], blocked: bool = True,
                 classes: Optional[Tuple[int, int, int]] = None):
        """classes = (cx, cy, n): sublattice q = (cx x + cy y) mod n instead of the
        default 2x2 classes; used for labelling when both periods lie in class 0."""
        self.a1 = tuple(a1)
        self.a2 = tuple(a2)
        self.classes = classes
        det = a1[0] * a2[1] - a1[1] * a2[0]
        if det == 0:
            raise ValueError("degenerate torus")
        self.det = abs(det)
        self._sdet = det
        pts = {}
        R = 2 * (abs(a1[0]) + abs(a1[1]) + abs(a2[0]) + abs(a2[1])) + 2
        for y in range(-R, R + 1):
            for x in range(-R, R + 1):
                key = self.key(x, y)
                if key not in pts:
                    pts[key] = (x, y)
        if len(pts) != self.det:
            raise ValueError("torus enumeration failed")
        # choose a canonical representative point: smallest (|x|+|y|, y, x) in the class
        canon = {}
        for y in range(-R, R + 1):
            for x in range(-R, R + 1):
                key = self.key(x, y)
                cand = (abs(x) + abs(y), y, x)
                if key not in canon or cand < canon[key][0]:
                    canon[key] = (cand, (x, y))
        points = [canon[k][1] for k in canon]
        if classes is None:
            even = all(c % 2 == 0 for c in (*a1, *a2))
            self.blocked = blocked and even and self.det % 4 == 0
        else:
            cx, cy, n = classes
            self.blocked = (blocked and self.det % n == 0 and
                            all((cx * a[0] + cy * a[1]) % n == 0 for a in (a1, a2)))
        if self.blocked:
            q_of = self.sublattice_of
            points.sort(key=lambda p: (q_of(p), p[1], p[0]))
        else:
            points.sort(key=lambda p: (p[1], p[0]))
        self.points: List[Tuple[int, int]] = points
        self.index = {self.key(*p): i for i, p in enumerate(points)}
        self.n_sites = len(points)

    def key(self, x: int, y: int) -> Tuple[int, int]:
        a1, a2, D = self.a1, self.a2, self._sdet
        u = (x * a2[1] - y * a2[0]) % abs(D)
        v = (-x * a1[1] + y * a1[0]) % abs(D)
        return (u, v)

    def site(self, x: int, y: int) -> int:
        return self.index[self.key(x, y)]

    def contains_vector(self, x: int, y: int) -> bool:
        return self.key(x, y) == self.key(0, 0)

    def sublattice_of(self, p) -> int:
        if self.classes is None:
            return (p[0] % 2) + 2 * (p[1] % 2)
        cx, cy, n = self.classes
        return (cx * p[0] + cy * p[1]) % n

    def sublattice(self, i: int) -> int:
        return self.sublattice_of(self.points[i])

    def bonds(self, neighbours, J: float = 1.0):
        """Bonds (i, i + d) for the neighbour vectors d, coupling J."""
        sites = []
        for i, (x, y) in enumerate(self.points):
            for dx, dy in neighbours:
                j = self.site(x + dx, y + dy)
                if j == i:
                    raise ValueError("bond onto itself")
                sites.append((i, j))
        js = np.full(len(sites), J, dtype=np.float64)
        return np.array(sites, dtype=np.int32), js.copy(), js.copy()

    def group_from(self, point_ops):
        """Translations x the given point operations (2x2 integer matrices acting
        on (x, y)) that map the torus onto itself; (perm, labels (tx, ty, op))."""
        ops = []
        for k, M in enumerate(point_ops):
            ok = True
            for a in (self.a1, self.a2):
                x, y = M[0][0] * a[0] + M[0][1] * a[1], M[1][0] * a[0] + M[1][1] * a[1]
                ok &= self.contains_vector(x, y)
            if ok:
                ops.append((k, M))
        perms, labels = [], []
        for (tx, ty) in self.points:
            for k, M in ops:
                def f(x, y, tx=tx, ty=ty, M=M):
                    return M[0][0] * x + M[0][1] * y + tx, M[1][0] * x + M[1][1] * y + ty
                perms.append(self._perm_of(f))
                labels.append((tx, ty, k))
        return np.array(perms, dtype=np.int32), labels

    def j1j2_bonds(self, J1: float = 1.0, J2: float = 0.0):
        sites, js = [], []
        for i, (x, y) in enumerate(self.points):
            for dx, dy, J in ((1, 0, J1), (0, 1, J1), (1, 1, J2), (1, -1, J2)):
                if J == 0.0:
                    continue
                j = self.site(x + dx, y + dy)
                if j == i:
                    raise ValueError("bond onto itself")
                sites.append((i, j))
                js.append(J)
        sites = np.array(sites, dtype=np.int32)
        js = np.array(js, dtype=np.float64)
        return sites, js.copy(), js.copy()

    def _perm_of(self, f) -> np.ndarray:
        return np.array([self.site(*f(x, y)) for (x, y) in self.points], dtype=np.int32)

    def symmetry_group(self, rotations: bool = True, reflections: bool = True):
        """Translations x point-group operations that map the torus onto itself.
        Returns (perm [n_sym, N], labels) with label (tx, ty, r, m): the site map
        p -> T(tx,ty) R^r M^m p, R = 90-degree rotation, M = (x,y) -> (x,-y)."""
        def rot(p, r):
            x, y = p
            for _ in range(r):
                x, y = -y, x
            return x, y

        def mir(p, m):
            return (p[0], -p[1]) if m else p

        def maps_lattice(r, m):
            for a in (self.a1, self.a2):
                x, y = rot(mir(a, m), r)
                if not self.contains_vector(x, y):
                    return False
            return True

        ops = []
        for m in ((0, 1) if reflections else (0,)):
            for r in (range(4) if rotations else (0,)):
                if maps_lattice(r, m):
                    ops.append((r, m))
        # translations: one per site, by the site's canonical point
        trans = [(x, y) for (x, y) in self.points]
        perms, labels = [], []
        for (tx, ty) in trans:
            for (r, m) in ops:
                def f(x, y, tx=tx, ty=ty, r=r, m=m):
                    xx, yy = rot(mir((x, y), m), r)
                    return xx + tx, yy + ty
                perms.append(self._perm_of(f))
                labels.append((tx, ty, r, m))
        return np.array(perms, dtype=np.int32), labels


def gamma_characters(labels, chi_rot: complex = 1.0, chi_mir: complex = 1.0) -> np.ndarray:
    """One-dimensional Gamma-point irreps of T x C4(v): the character of
    T R^r M^m is chi_rot^r chi_mir^m (A1: 1, 1; A2: 1, -1; B1: -1, 1;
    B2: -1, -1)."""
    return np.array([complex(chi_rot) ** r * complex(chi_mir) ** m for (_, _, r, m) in labels],
                    dtype=np.complex128)


IRREPS_C4V = {"A1": (1, 1), "A2": (1, -1), "B1": (-1, 1), "B2": (-1, -1)}


def torus_model(a1, a2, J1=1.0, J2=0.0, irrep: Optional[str] = "A1", n_up=None,
                rotations=True, reflections=True, name=None, delta: float = 1.0) -> Model:
    t = Torus(a1, a2)
    sites, jz, jxy = t.j1j2_bonds(J1, J2)
    jz = jz * delta
    if n_up is None:
        n_up = t.n_sites // 2
    m = Model(name or f"torus{t.n_sites}", t.n_sites, n_up, sites, jz, jxy)
    if irrep is not None:
        perm, labels = t.symmetry_group(rotations, reflections)
        cr, cm = IRREPS_C4V[irrep]
        m = m.with_sector(perm, gamma_characters(labels, cr, cm), m.name + "_" + irrep)
    return m


SQUARE_NEIGHBOURS = ((1, 0), (0, 1))
TRIANGULAR_NEIGHBOURS = ((1, 0), (0, 1), (1, -1))
ROT90 = ((0, -1), (1, 0))
ROT60_TRI = ((0, -1), (1, 1))        # (x, y) -> (-y, x + y) in triangular lattice coordinates
INVERSION = ((-1, 0), (0, -1))


def _powers(M, n):
    out, P = [], ((1, 0), (0, 1))
    for _ in range(n):
        out.append(P)
        P = ((M[0][0] * P[0][0] + M[0][1] * P[1][0], M[0][0] * P[0][1] + M[0][1] * P[1][1]),
             (M[1][0] * P[0][0] + M[1][1] * P[1][0], M[1][0] * P[0][1] + M[1][1] * P[1][1]))
    return out


def sublattice_model(kind: str, a1, a2, n_up=None, delta: float = 1.0, name=None,
                     rot_char: complex = 1.0) -> Model:
    """Heisenberg/XXZ models whose natural sublattice coding has 2, 3 or 5
    blocks (the 2-, 3- and 5-sublattice backends of Sec. 5.1), trivial
    characters of translations x point group:
      'square2'   square lattice, checkerboard classes (x + y) mod 2, T x C4;
      'triangle3' triangular lattice, classes (x + 2y) mod 3, T x C6;
      'square5'   square lattice, classes (x + 2y) mod 5, T x C4.
    Characters: 1 for translations, rot_char^r for the r-th power of the
    rotation (Gamma-point one-dimensional irreps of C4 / C6)."""
    classes, neigh, ops = {
        "square2": ((1, 1, 2), SQUARE_NEIGHBOURS, _powers(ROT90, 4)),
        "triangle3": ((1, 2, 3), TRIANGULAR_NEIGHBOURS, _powers(ROT60_TRI, 6)),
        "square5": ((1, 2, 5), SQUARE_NEIGHBOURS, _powers(ROT90, 4)),
    }[kind]
    t = Torus(a1, a2, classes=classes)
    if not t.blocked:
        raise ValueError("periods do not preserve the sublattice classes")
    sites, jz, jxy = t.bonds(neigh)
    perm, labels = t.group_from(ops)
    n_up = t.n_sites // 2 if n_up is None else n_up
    m = Model(name or f"{kind}_{t.n_sites}", t.n_sites, n_up, sites, jz * delta, jxy)
    chi = np.array([complex(rot_char) ** k for (_, _, k) in labels], dtype=np.complex128)
    return m.with_sector(perm, chi)


# --------------------------------------------------------------------------
# The benchmark workloads (sizes as in the paper's Sec. 6 family)
# --------------------------------------------------------------------------


def workload(name: str, **kw) -> List[Model]:
    """Models of the named workload (one per sector)."""
    if name == "chain16_u1":            # N=16 ring, Sz=0, no spatial symmetry
        return [chain_model(16)]
    if name == "chain32_k0_kpi":        # N=32 ring, translations, k=0 and k=pi
        return [chain_model(32, l=0), chain_model(32, l=16)]
    if name == "square36_j1j2_A1":      # 6x6 torus, J1=1, J2=0.5, T x C4v, Gamma A1
        return [torus_model((6, 0), (0, 6), 1.0, 0.5, "A1", name="square36_j1j2")]
    if name == "chain32_allk":          # all 32 momenta of the N=32 ring
        return [chain_model(32, l=l) for l in range(32)]
    if name == "tilted40_xxz":          # 40-site tilted torus, T x C4, Gamma, Jz=Jxy=1
        return [torus_model((6, 2), (-2, 6), 1.0, 0.0, "A1", reflections=False,
                            name="tilted40_xxz")]
    raise KeyError(name)


# --------------------------------------------------------------------------
# Random vectors: SplitMix64 (Steele, Lea, Flood 2014), counter based.
# Output number n >= 1 of a generator seeded with `seed` is
#   mix(seed + n * 0x9E3779B97F4A7C15 mod 2^64),
#   mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
#           z *= 0x94D049BB133111EB; z ^= z >> 31.
# Uniform [0,1): top 53 bits times 2^-53.
# Scalar q of a vector (flat index over [dim][nvec], complex = re, im
# interleaved) draws outputs n = 2q+1 and 2q+2:
#   "uniform":  2 u(2q+1) - 1                 (U[-1, 1])
#   "gauss":    sqrt(-2 ln(1 - u(2q+1))) cos(2 pi u(2q+2))   (Box-Muller)
# --------------------------------------------------------------------------

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    z = z ^ (z >> np.uint64(31))
    return z


def _uniform53(seed: int, counters: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + counters.astype(np.uint64) * _GAMMA
        z = _mix(z)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def random_scalars(seed: int, n: int, kind: str = "gauss", start: int = 0,
                   chunk: int = 1 << 24) -> np.ndarray:
    """n scalars q = start .. start+n-1 of the seeded stream (float64)."""
    out = np.empty(n, dtype=np.float64)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        q = np.arange(start + c0, start + c1, dtype=np.uint64)
        u1 = _uniform53(seed, 2 * q + 1)
        if kind == "uniform":
            out[c0:c1] = 2.0 * u1 - 1.0
        elif kind == "gauss":
            u2 = _uniform53(seed, 2 * q + 2)
            out[c0:c1] = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        else:
            raise ValueError(kind)
    return out


def random_vector(seed: int, dim: int, nvec: int = 1, kind: str = "gauss",
                  complex_: bool = False) -> np.ndarray:
    """Vector block [dim][nvec] (squeezed to [dim] when nvec == 1)."""
    n = dim * nvec * (2 if complex_ else 1)
    s = random_scalars(seed, n, kind)
    if complex_:
        v = s.view(np.complex128)
    else:
        v = s
    v = v.reshape(dim, nvec)
    return v[:, 0].copy() if nvec == 1 else v


# --------------------------------------------------------------------------
# Vectors keyed by basis state.  Entry v (column) of the vector at the basis
# state s is scalar q = (s * nvec + v) * C + c of the seeded stream above
# (C = 2 for complex, c = 0 re / 1 im), drawn as U[-1, 1]: 2 u(2q+1) - 1.
# The value depends on the state, not on its position in a basis, so a
# checker that knows only states (no basis list) can evaluate x anywhere.
# --------------------------------------------------------------------------

def keyed_values(seed: int, states, nvec: int = 1, complex_: bool = False) -> np.ndarray:
    """Keyed vector entries for host states: [n] (nvec == 1) or [n, nvec],
    float64 or complex128."""
    s = np.ascontiguousarray(states, dtype=np.uint64).reshape(-1)
    C = 2 if complex_ else 1
    q = ((s[:, None] * np.uint64(nvec) + np.arange(nvec, dtype=np.uint64)[None, :])
         * np.uint64(C))
    if complex_:
        re = 2.0 * _uniform53(seed, 2 * q + 1) - 1.0
        im = 2.0 * _uniform53(seed, 2 * (q + np.uint64(1)) + 1) - 1.0
        v = re + 1j * im
    else:
        v = 2.0 * _uniform53(seed, 2 * q + 1) - 1.0
    return v[:, 0].copy() if nvec == 1 else v


_I64 = 1 << 64


def _signed(c: int) -> int:
    return c - _I64 if c >= 1 << 63 else c


def keyed_values_torch(seed: int, states, nvec: int = 1, complex_: bool = False):
    """The same keyed entries for a torch int64 tensor of states (on any
    device), as float64 / complex128 [n] or [n, nvec].  Two's-complement
    int64 arithmetic gives the uint64 products modulo 2^64; right shifts are
    made logical by masking."""
    import torch
    s = states.to(torch.int64).reshape(-1)
    dev = s.device
    C = 2 if complex_ else 1
    v = torch.arange(nvec, dtype=torch.int64, device=dev)

    def srl(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    def u53(n):
        z = n * _signed(int(_GAMMA)) + _signed(seed & (_I64 - 1))
        z = z ^ srl(z, 30)
        z = z * _signed(int(_M1))
        z = z ^ srl(z, 27)
        z = z * _signed(int(_M2))
        z = z ^ srl(z, 31)
        return srl(z, 11).to(torch.float64) * (1.0 / 9007199254740992.0)

    q = (s[:, None] * nvec + v[None, :]) * C
    if complex_:
        out = torch.complex(2.0 * u53(2 * q + 1) - 1.0, 2.0 * u53(2 * (q + 1) + 1) - 1.0)
    else:
        out = 2.0 * u53(2 * q + 1) - 1.0
    return out[:, 0].contiguous() if nvec == 1 else out
