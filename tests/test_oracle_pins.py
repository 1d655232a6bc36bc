"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself (CPU only).

* the worked k = pi symmetric state of Sec. 3.11 (golden fixture);
* the N = 4 ring spectrum in closed form;
* the sector Hamiltonian against P^dagger H_full P, with H_full built from
  Kronecker products of spin matrices and the columns of P built from the
  definition of symmetric states (Sec. 3.11) - this checks the pull-form
  amplitude the oracle uses;
* the sector dimension against the projection-operator trace formula
  (cycle counting);
* the block sizes printed in Table 1;
* Bethe-ansatz ground-state energies of the Heisenberg ring;
* trace identity, Hermiticity, k <-> -k, ferromagnetic bound;
* Sturm bisection against LAPACK on random tridiagonal matrices.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load_gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- helpers --
# Independent constructions used only to pin the oracle.

def kron_hamiltonian(m, states):
    """H restricted to the given product states, from Kronecker products of
    2x2 spin matrices (site i = bit i, basis {|dn>, |up>} = {0, 1})."""
    N = m.n_sites
    Sz = np.diag([-0.5, 0.5])
    Sp = np.array([[0.0, 0.0], [1.0, 0.0]])
    Sm = Sp.T
    I2 = sp.identity(2, format="csr")

    def site_op(op, i):
        # np.kron puts its first factor on the most significant bit
        left = sp.identity(2 ** (N - 1 - i), format="csr")
        right = sp.identity(2 ** i, format="csr")
        return sp.kron(sp.kron(left, sp.csr_matrix(op)), right, format="csr")

    H = sp.csr_matrix((2 ** N, 2 ** N))
    for (i, j), jz, jxy in zip(m.sites, m.jz, m.jxy):
        H = H + jz * (site_op(Sz, i) @ site_op(Sz, j))
        H = H + 0.5 * jxy * (site_op(Sp, i) @ site_op(Sm, j) + site_op(Sm, i) @ site_op(Sp, j))
    idx = np.asarray(states, dtype=np.int64)
    return H[idx][:, idx]


def popcount_states(N, n):
    s = np.arange(2 ** N, dtype=np.int64)
    pc = np.zeros_like(s)
    t = s.copy()
    while np.any(t):
        pc += t & 1
        t >>= 1
    return s[pc == n]


def permute_state(g, s):
    """(g.s) has at site i the spin of s at site g(i) (Sec. 3.11)."""
    out = 0
    for i, gi in enumerate(g):
        if (s >> int(gi)) & 1:
            out |= 1 << i
    return out


def symmetric_projector(m, reps, states):
    """Columns: |r~> = N^-1 sum_g chi(g)^* g|r>, in the product basis `states`."""
    pos = {int(s): k for k, s in enumerate(states)}
    P = np.zeros((len(states), len(reps)), dtype=np.complex128)
    for c, r in enumerate(reps):
        for g, chi in zip(m.perm, m.chi):
            P[pos[permute_state(g, int(r))], c] += np.conj(chi)
        P[:, c] /= np.linalg.norm(P[:, c])
    return P


def oracle_dense(oracle, m, b):
    D = len(b)
    return oracle.apply(m, b, np.eye(D, dtype=np.complex128))


def dimension_formula(m):
    """dim = |G|^-1 sum_g chi(g)^* Fix_g, Fix_g = number of ways to choose
    whole cycles of g with n_up sites in total."""
    N, n = m.n_sites, m.n_up
    tot = 0j
    for g, chi in zip(m.perm, m.chi):
        seen = [False] * N
        lens = []
        for i in range(N):
            if not seen[i]:
                L, j = 0, i
                while not seen[j]:
                    seen[j] = True
                    j = int(g[j])
                    L += 1
                lens.append(L)
        ways = [0] * (n + 1)
        ways[0] = 1
        for L in lens:
            for t in range(n, L - 1, -1):
                ways[t] += ways[t - L]
        tot += np.conj(chi) * ways[n]
    d = tot / len(m.perm)
    assert abs(d.imag) < 1e-6 and abs(d.real - round(d.real)) < 1e-6
    return int(round(d.real))


def bethe_energy(N, M):
    """Heisenberg ring, J = 1: N atan(2 l_j) = pi I_j + sum_{l != j} atan(l_j - l_l),
    consecutive I_j centred on 0; E = N/4 - sum_j 2 / (1 + 4 l_j^2)."""
    I = np.arange(M) - (M - 1) / 2.0
    lam = 0.5 * np.tan(np.pi * I / N)

    def F(l):
        d = l[:, None] - l[None, :]
        return N * np.arctan(2 * l) - np.pi * I - np.arctan(d).sum(axis=1)

    for _ in range(20000):
        d = lam[:, None] - lam[None, :]
        new = 0.5 * np.tan((np.pi * I + np.arctan(d).sum(axis=1)) / N)
        if np.max(np.abs(new - lam)) < 1e-15:
            lam = new
            break
        lam = new
    lam = scipy.optimize.fsolve(F, lam, xtol=1e-15)
    assert np.max(np.abs(F(lam))) < 1e-11
    return N / 4.0 - np.sum(2.0 / (1.0 + 4.0 * lam ** 2))


def small_sector_models():
    out = []
    for N in (6, 8, 10):
        for l in range(N):
            out.append(W.chain_model(N, l=l))
    m = W.chain_model(8, n_up=3)
    out.append(m.with_sector(W.chain_translations(8), W.momentum_characters(8, 3), "c8n3k3"))
    # dihedral chain, both reflection parities at k = 0
    for par in (1, -1):
        perm = W.chain_dihedral(8)
        chi = np.array([1.0] * 8 + [par] * 8, dtype=np.complex128)
        out.append(W.chain_model(8).with_sector(perm, chi, f"dihedral8_{par}"))
    # XXZ with anisotropy and unequal couplings on a ring
    m = W.chain_model(10, l=3, delta=0.4, J=0.7)
    out.append(m)
    # 2-, 3- and 5-sublattice lattices (real and complex rotation characters)
    out += other_sublattice_models(small=True)
    return out


def other_sublattice_models(small=False):
    """Lattices with 2, 3 and 5 sublattice blocks (checkerboard square,
    triangular, (x + 2y) mod 5 square), trivial and complex point-group
    characters."""
    out = [W.sublattice_model("square2", (3, 1), (-1, 3)),
           W.sublattice_model("square2", (3, 1), (-1, 3), rot_char=1j, name="square2_10_E"),
           W.sublattice_model("triangle3", (4, -2), (2, 2)),
           W.sublattice_model("triangle3", (4, -2), (2, 2), rot_char=np.exp(1j * np.pi / 3),
                              name="triangle3_12_E")]
    if not small:
        out += [W.sublattice_model("square5", (2, 4), (-4, 2)),
                W.sublattice_model("square5", (2, 4), (-4, 2), rot_char=-1, name="square5_20_B"),
                W.sublattice_model("triangle3", (5, -1), (1, 4), n_up=7),
                W.sublattice_model("square2", (4, 0), (0, 4), delta=0.5)]
    return out


# ------------------------------------------------------------------ tests --

def test_worked_example_symmetric_state(oracle_lib):
    g = load_gold("worked_example_c4_kpi.json")
    N = g["n_sites"]
    T = np.array(g["translation"], dtype=np.int32)
    perm = [np.arange(N, dtype=np.int32)]
    for _ in range(N - 1):
        perm.append(T[perm[-1]])          # T^n(i) = T(T^{n-1}(i))
    perm = np.array(perm, dtype=np.int32)
    chi = np.array([complex(a, b) for a, b in g["characters_k_pi"]])

    def enc(lbl):
        return sum(1 << i for i, c in enumerate(lbl) if c == "U")

    s = enc(g["state_sites_0_to_3"])
    # symmetric state from the oracle's action and stabiliser count
    _, _, stab = oracle_lib.rep(N, perm, s)
    vec = {}
    for gg, c in zip(perm, chi):
        t = oracle_lib.act(N, gg, s)
        vec[t] = vec.get(t, 0) + np.conj(c)
    norm = math.sqrt(len(perm) * stab)
    got = {t: v / norm for t, v in vec.items()}
    want = {enc(k): v for k, v in g["coefficients"].items()}
    assert set(got) == set(want)
    for t in want:
        assert abs(got[t] - want[t]) < 1e-15
    # representative of the orbit is the smallest integer (Sec. 3.11)
    r, _, _ = oracle_lib.rep(N, perm, s)
    assert r == min(want)


def test_chain4_closed_form(oracle_lib):
    g = load_gold("chain4_spectra.json")
    ev = []
    dims = []
    for l in range(4):
        m = W.chain_model(4, l=l)
        b = oracle_lib.basis(m)
        dims.append(len(b))
        ev.extend(np.linalg.eigvalsh(oracle_dense(oracle_lib, m, b)))
    assert dims == g["momentum_dims_l0_to_l3"]
    assert np.allclose(sorted(ev), g["sz0_spectrum"], atol=1e-13)
    # U(1) block alone
    m = W.chain_model(4)
    b = oracle_lib.basis(m)
    assert np.allclose(np.linalg.eigvalsh(oracle_dense(oracle_lib, m, b)), g["sz0_spectrum"],
                       atol=1e-13)


@pytest.mark.parametrize("N", [4, 8, 10, 12])
def test_u1_block_against_kronecker(oracle_lib, N):
    m = W.chain_model(N, delta=0.7, J=1.3)
    m.jz[1] = -0.4      # break uniformity: bond order and couplings matter
    m.jxy[2] = 2.1
    b = oracle_lib.basis(m)
    states = popcount_states(N, N // 2)
    assert np.array_equal(b.astype(np.int64), states)
    Hk = kron_hamiltonian(m, states).toarray()
    Ho = oracle_dense(oracle_lib, m, b)
    assert np.max(np.abs(Ho - Hk)) < 1e-13


@pytest.mark.parametrize("idx", range(len(small_sector_models())))
def test_sector_matrix_is_projected_hamiltonian(oracle_lib, idx):
    m = small_sector_models()[idx]
    b = oracle_lib.basis(m)
    states = popcount_states(m.n_sites, m.n_up)
    H = kron_hamiltonian(m, states).toarray()
    P = symmetric_projector(m, b, states)
    assert np.allclose(P.conj().T @ P, np.eye(len(b)), atol=1e-13)
    want = P.conj().T @ H @ P
    got = oracle_dense(oracle_lib, m, b)
    assert np.max(np.abs(got - want)) < 1e-13, m.name


def test_square4x4_sectors_projected(oracle_lib):
    # non-abelian T x C4v (128 elements), J1-J2, all four Gamma irreps
    for irrep in ("A1", "A2", "B1", "B2"):
        m = W.torus_model((4, 0), (0, 4), 1.0, 0.5, irrep, n_up=6)
        b = oracle_lib.basis(m)
        assert len(b) == dimension_formula(m)
        states = popcount_states(16, 6)
        H = kron_hamiltonian(m, states)
        P = symmetric_projector(m, b, states)
        want = P.conj().T @ (H @ P)
        got = oracle_dense(oracle_lib, m, b)
        assert np.max(np.abs(got - want)) < 1e-12, irrep


def test_dimension_formula(oracle_lib):
    models = small_sector_models()
    models += [W.chain_model(14, l=l) for l in (0, 3, 7)]
    models += [W.torus_model((4, 0), (0, 4), 1.0, 0.5, ir) for ir in ("A1", "A2", "B1", "B2")]
    models += [W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False)]
    models += [W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "B1", reflections=False, n_up=8)]
    models += other_sublattice_models()
    for m in models:
        assert len(oracle_lib.basis(m)) == dimension_formula(m), m.name


def test_square4x4_dimensions():
    dims = {ir: dimension_formula(W.torus_model((4, 0), (0, 4), 1.0, 0.5, ir))
            for ir in ("A1", "A2", "B1", "B2")}
    # each symmetric block sums back to the Sz = 0 block through the irreps'
    # multiplicities: only the 1-d irreps are here, so the sum is below C(16, 8)
    assert sum(dims.values()) < math.comb(16, 8)
    assert dims == {"A1": 153, "A2": 78, "B1": 130, "B2": 95}


def test_basis_against_brute_force(oracle_lib):
    for m in (W.chain_model(10, l=5), W.chain_model(9, n_up=4, l=2),
              W.torus_model((4, 0), (0, 4), 1.0, 0.0, "B2", n_up=7)):
        N = m.n_sites
        want = []
        for s in popcount_states(N, m.n_up):
            orbit = [permute_state(g, int(s)) for g in m.perm]
            if min(orbit) != s:
                continue
            c = sum(chi for g, chi, o in zip(m.perm, m.chi, orbit) if o == s)
            if abs(c) > 0.5:
                want.append(int(s))
        got = oracle_lib.basis(m)
        assert got.tolist() == want, m.name
        for i, s in enumerate(want):
            assert oracle_lib.index(got, s) == i
        assert oracle_lib.index(got, (1 << m.n_up) - 1 + (1 << (N - 1))) in (-1,) + tuple(
            range(len(want)))


def test_basis_range_is_a_window_of_the_basis(oracle_lib):
    rng = np.random.default_rng(3)
    for m in (W.chain_model(14, l=3), W.torus_model((4, 0), (0, 4), 1.0, 0.5, "B1"),
              W.chain_model(12)):
        full = oracle_lib.basis(m)
        for _ in range(5):
            lo, hi = sorted(int(v) for v in rng.integers(0, 1 << m.n_sites, 2))
            want = full[(full >= lo) & (full <= hi)]
            assert np.array_equal(oracle_lib.basis_range(m, lo, hi), want)
        assert np.array_equal(oracle_lib.basis_range(m, 0, (1 << m.n_sites) - 1), full)


@pytest.mark.slow
def test_table1_block_sizes(oracle_lib):
    g = load_gold("table1_block_sizes.json")
    row = g["rows"][0]                 # N = 28 runs in seconds on the oracle
    N = row["n_sites"]
    # trivial irrep of translations x reflection (k = 0, even parity)
    chi = np.ones(2 * N, dtype=np.complex128)
    m = W.chain_model(N).with_sector(W.chain_dihedral(N), chi)
    d = len(oracle_lib.basis(m))
    assert d == dimension_formula(m) == 718146
    assert float(f"{d:.1e}") == row["block_size"]


def test_sector_sums_and_trace_identity(oracle_lib):
    N = 12
    n = N // 2
    dims, traces, spec = 0, 0.0, []
    for l in range(N):
        m = W.chain_model(N, l=l)
        b = oracle_lib.basis(m)
        Hk = oracle_dense(oracle_lib, m, b)
        dims += len(b)
        traces += np.trace(Hk).real
        spec.extend(np.linalg.eigvalsh(Hk))
    assert dims == math.comb(N, n)
    nb = N
    want = nb * 0.25 * (math.comb(N - 2, n - 2) + math.comb(N - 2, n) - 2 * math.comb(N - 2, n - 1))
    assert abs(traces - want) < 1e-9
    assert want == -252
    # union of the momentum spectra is the Sz = 0 spectrum
    m = W.chain_model(N)
    full = np.linalg.eigvalsh(kron_hamiltonian(m, popcount_states(N, n)).toarray())
    assert np.allclose(sorted(spec), full, atol=1e-11)


def test_k_minus_k_and_hermiticity(oracle_lib):
    N = 10
    rng = np.random.default_rng(5)
    for l in range(1, N // 2):
        a = W.chain_model(N, l=l)
        b = W.chain_model(N, l=N - l)
        ba, bb = oracle_lib.basis(a), oracle_lib.basis(b)
        Ha, Hb = oracle_dense(oracle_lib, a, ba), oracle_dense(oracle_lib, b, bb)
        assert np.allclose(np.linalg.eigvalsh(Ha), np.linalg.eigvalsh(Hb), atol=1e-12)
        assert np.max(np.abs(Ha - Ha.conj().T)) < 1e-14
    m = W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "B1", reflections=False)
    b = oracle_lib.basis(m)
    x = rng.normal(size=len(b)) + 1j * rng.normal(size=len(b))
    w = rng.normal(size=len(b)) + 1j * rng.normal(size=len(b))
    lhs = np.vdot(w, oracle_lib.apply(m, b, x))
    rhs = np.conj(np.vdot(x, oracle_lib.apply(m, b, w)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_tridiagonal_bisection_against_lapack(oracle_lib):
    rng = np.random.default_rng(1)
    for m in (1, 2, 5, 37, 120):
        a = rng.normal(size=m)
        b = rng.normal(size=m)
        T = np.diag(a) + np.diag(b[: m - 1], 1) + np.diag(b[: m - 1], -1)
        want = np.linalg.eigvalsh(T)
        k = min(m, 4)
        got = oracle_lib.tridiag_eigvals(a, b, k)
        assert np.max(np.abs(got - want[:k])) < 1e-13 * max(1, np.max(np.abs(want)))


@pytest.mark.parametrize("N", [8, 12, 16])
def test_bethe_ansatz_ground_state(oracle_lib, N):
    m = W.chain_model(N)
    b = oracle_lib.basis(m)
    x0 = W.random_vector(1, len(b), kind="uniform")
    st, ev, al, be = oracle_lib.lanczos(m, b, x0, k=1, tol=1e-14, max_iter=300)
    assert st == 0
    e_bethe = bethe_energy(N, N // 2)
    assert abs(ev[0] - e_bethe) < 1e-12 * abs(e_bethe)
    if N == 16:
        assert abs(e_bethe - (-7.142296360617)) < 5e-12


def test_bethe_momentum_pi_sector(oracle_lib):
    # the lowest k = pi level at Sz = 0 is the lowest triplet, M = N/2 - 1 magnons
    N = 12
    m = W.chain_model(N, l=N // 2)
    b = oracle_lib.basis(m)
    ev = np.linalg.eigvalsh(oracle_dense(oracle_lib, m, b))
    assert abs(ev[0] - bethe_energy(N, N // 2 - 1)) < 1e-12 * abs(ev[0])
    assert abs(np.linalg.eigvalsh(oracle_dense(oracle_lib, W.chain_model(N, l=0),
                                               oracle_lib.basis(W.chain_model(N, l=0))))[0]
               - bethe_energy(N, N // 2)) < 1e-12 * abs(ev[0])


def test_lanczos_against_dense_and_reorth(oracle_lib):
    m = W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False)
    b = oracle_lib.basis(m)
    H = oracle_dense(oracle_lib, m, b)
    want = np.linalg.eigvalsh(H)
    x0 = W.random_vector(3, len(b), kind="gauss")
    for reorth in (False, True):
        st, ev, al, be = oracle_lib.lanczos(m, b, x0, k=3, tol=1e-14, max_iter=min(len(b), 200),
                                            reorth=reorth)
        assert abs(ev[0] - want[0]) < 1e-12 * abs(want[0])
        if reorth:
            assert np.max(np.abs(ev - want[:3])) < 1e-10


def test_ferromagnetic_bound(oracle_lib):
    # J_b >= 0 and Jz = Jxy: the top level is sum_b J_b / 4, in the trivial sector
    m = W.torus_model((4, 0), (0, 4), 1.0, 0.5, "A1")
    neg = W.Model(m.name, m.n_sites, m.n_up, m.sites, -m.jz, -m.jxy, m.perm, m.chi)
    b = oracle_lib.basis(neg)
    x0 = W.random_vector(4, len(b), kind="gauss")
    st, ev, _, _ = oracle_lib.lanczos(neg, b, x0, k=1, tol=1e-14, max_iter=150)
    assert abs(-ev[0] - m.jz.sum() / 4.0) < 1e-11
    assert m.jz.sum() / 4.0 == 12.0


def test_square4x4_ground_state_equals_full_space(oracle_lib):
    m = W.torus_model((4, 0), (0, 4), 1.0, 0.5, "A1")
    b = oracle_lib.basis(m)
    assert len(b) == 153
    ev = np.linalg.eigvalsh(oracle_dense(oracle_lib, m, b))
    H = kron_hamiltonian(m, popcount_states(16, 8))
    e_full = spla.eigsh(H, k=1, which="SA", tol=1e-14)[0][0]
    assert abs(ev[0] - e_full) < 1e-11 * abs(e_full)


# --------------------------------------------------- eigenvectors, measurements
EXPAND_CASES = [
    W.chain_model(12, l=0),                                           # real, translations
    W.chain_model(12, l=5),                                           # complex characters
    W.torus_model((4, 0), (0, 4), 1.0, 0.5, "B1"),                   # non-abelian group
]


@pytest.mark.parametrize("case", range(len(EXPAND_CASES)))
def test_expanded_ground_state(oracle_lib, case):
    """The product-state expansion of the block ground state: unit norm, an
    eigenvector of the Kronecker-built U(1) Hamiltonian with the same energy,
    and g Psi = chi(g) Psi for every g (so a slip in N_s, chi or the action
    fails here)."""
    m = EXPAND_CASES[case]
    b = oracle_lib.basis(m)
    e0, psi = oracle_lib.dense_ground_state(m, b)
    full, amp = oracle_lib.expand_state(m, b, psi)
    assert abs(np.linalg.norm(amp) - 1.0) < 1e-12
    states = popcount_states(m.n_sites, m.n_up)
    assert np.array_equal(states.astype(np.uint64), full)
    H = kron_hamiltonian(m, states)
    assert np.max(np.abs(H @ amp - e0 * amp)) < 1e-10
    pos = {int(t): i for i, t in enumerate(full)}
    for g, ch in zip(m.perm, m.chi):
        moved = np.zeros_like(amp)
        for i, t in enumerate(full):
            moved[pos[oracle_lib.act(m.n_sites, g, int(t))]] = amp[i]
        assert np.max(np.abs(moved - ch * amp)) < 1e-12


def test_szsz_closed_forms(oracle_lib):
    """<S^z_0 S^z_0> = 1/4; sum_j <S^z_0 S^z_j> = <S^z_0 S^z_tot> = 0 at Sz = 0;
    the chain ground state is a translation-invariant singlet, so
    <S^z_0 S^z_1> = <S_0.S_1>/3 = E0/(3N), with E0 from the Bethe ansatz."""
    N = 16
    m = W.chain_model(N, l=0)
    b = oracle_lib.basis(m)
    e0, psi = oracle_lib.dense_ground_state(m, b)
    assert abs(e0 - bethe_energy(N, N // 2)) < 1e-11
    full, amp = oracle_lib.expand_state(m, b, psi)
    c = np.array([oracle_lib.szsz_definition(full, amp, 0, j) for j in range(N)])
    assert abs(c[0] - 0.25) < 1e-14
    assert abs(c.sum()) < 1e-13
    assert abs(c[1] - bethe_energy(N, N // 2) / (3 * N)) < 1e-12
    assert np.max(np.abs(c[1:] - c[1:][::-1])) < 1e-13        # reflection symmetry of the ring


@pytest.mark.parametrize("case", range(len(EXPAND_CASES)))
def test_symmetrised_diagonal_equals_plain_expectation(oracle_lib, case):
    """For a state of the block, <O> of the plain S^z_a S^z_b equals
    sum_s |psi_s|^2 (1/|G|) sum_g sz_s(g(a)) sz_s(g(b)): the reading of the
    symmetrised operator used for measurements."""
    m = EXPAND_CASES[case]
    b = oracle_lib.basis(m)
    rng = np.random.default_rng(case)
    psi = rng.normal(size=len(b)) + (1j * rng.normal(size=len(b)) if m.is_complex else 0)
    psi /= np.linalg.norm(psi)
    full, amp = oracle_lib.expand_state(m, b, psi)
    for a, c in ((0, 1), (0, 5), (3, 7), (2, 2)):
        plain = oracle_lib.szsz_definition(full, amp, a, c)
        sym = 0.0
        for s, p in zip(b, psi):
            o = 0.0
            for g in m.perm:
                ba = (int(s) >> int(g[a])) & 1
                bc = (int(s) >> int(g[c])) & 1
                o += 0.25 if ba == bc else -0.25
            sym += abs(p) ** 2 * o / m.n_sym
        assert abs(plain - sym) < 1e-13, (a, c)


def test_dynamical_sum_rule_matches_static_correlations(oracle_lib):
    """Sum rule of the dynamical structure factor: sum_n |<n|S^z_q|0>|^2 (full
    U(1) space, dense) = sum_j e^{iqj} <S^z_0 S^z_j> (ground state of the k = 0
    block expanded into product states), for every q of the N = 12 ring."""
    N = 12
    m_u1 = W.chain_model(N)
    m0 = W.chain_model(N, l=0)
    b = oracle_lib.basis(m0)
    e0, psi = oracle_lib.dense_ground_state(m0, b)
    full, amp = oracle_lib.expand_state(m0, b, psi)
    c = np.array([oracle_lib.szsz_definition(full, amp, 0, j) for j in range(N)])
    for l in range(N):
        q = 2 * np.pi * l / N
        coef = np.exp(1j * q * np.arange(N)) / np.sqrt(N)
        E0, dE, w = oracle_lib.dense_sz_spectrum(m_u1, coef)
        assert abs(E0 - e0) < 1e-11
        Sq = np.real(np.sum(np.exp(1j * q * np.arange(N)) * c))
        assert abs(w.sum() - Sq) < 1e-12, (l, w.sum(), Sq)
    # q = 0: S^z_tot |0> = 0 at Sz = 0, so no weight at all
    E0, dE, w = oracle_lib.dense_sz_spectrum(m_u1, np.ones(N) / np.sqrt(N))
    assert w.sum() < 1e-24


# ------------------------------------------------- row-sampled oracle forms --

def row_sample_models():
    """A real ring sector, a complex momentum sector, a dihedral sector, the
    4x4 J1-J2 torus (non-abelian T x C4v, two irreps) and a complex
    3-sublattice lattice."""
    perm = W.chain_dihedral(10)
    chi = np.array([1.0] * 10 + [-1.0] * 10, dtype=np.complex128)
    return [W.chain_model(14, l=0), W.chain_model(14, l=5),
            W.chain_model(10).with_sector(perm, chi, "dihedral10_odd"),
            W.torus_model((4, 0), (0, 4), 1.0, 0.5, "A1"),
            W.torus_model((4, 0), (0, 4), 1.0, 0.5, "B2"),
            W.sublattice_model("triangle3", (4, -2), (2, 2), rot_char=np.exp(1j * np.pi / 3),
                               name="triangle3_12_E"),
            W.chain_model(12)]


@pytest.mark.parametrize("idx", range(len(row_sample_models())))
@pytest.mark.parametrize("nvec", [1, 3])
def test_apply_rows_equals_apply(oracle_lib, idx, nvec):
    """orc_apply_rows (the form the CPU baseline times) against orc_apply,
    which the projected-Hamiltonian tests pin to the definition."""
    m = row_sample_models()[idx]
    b = oracle_lib.basis(m)
    rng = np.random.default_rng(idx)
    x = W.random_vector(11 + idx, len(b), nvec, kind="gauss", complex_=True)
    full = oracle_lib.apply(m, b, x)
    rows = np.sort(rng.choice(len(b), size=min(len(b), 97), replace=False))
    rows = np.concatenate([[0], rows, [len(b) - 1]])
    got = oracle_lib.apply_rows(m, b, rows, x)
    assert np.max(np.abs(got - full[rows])) <= 1e-14 * np.max(np.abs(full))


@pytest.mark.parametrize("idx", range(len(row_sample_models())))
@pytest.mark.parametrize("nvec,cplx,f32", [(1, False, False), (1, True, False), (3, True, True),
                                           (2, False, True)])
def test_apply_keyed_equals_apply(oracle_lib, idx, nvec, cplx, f32):
    """The basis-free form (x keyed by state, rows given by their states)
    against orc_apply on the same vector laid out in basis order."""
    m = row_sample_models()[idx]
    if m.is_complex and not cplx:
        pytest.skip("complex sector needs a complex vector")
    b = oracle_lib.basis(m)
    x = W.keyed_values(21, b, nvec=nvec, complex_=cplx)
    if f32:
        x = (x.astype(np.complex64) if cplx else x.astype(np.float32)).astype(x.dtype)
    full = oracle_lib.apply(m, b, x)
    rng = np.random.default_rng(100 + idx)
    rows = np.sort(rng.choice(len(b), size=min(len(b), 80), replace=False))
    got = oracle_lib.apply_keyed(m, b[rows], 21, nvec=nvec, complex_=cplx, round_to_f32=f32)
    assert got.shape == full[rows].shape
    assert np.max(np.abs(got - full[rows])) <= 1e-14 * np.max(np.abs(full))


def test_apply_keyed_rejects_non_basis_rows(oracle_lib):
    m = W.chain_model(12, l=0)
    b = oracle_lib.basis(m)
    full = oracle_lib.full_states(12, 6)
    nonrep = np.setdiff1d(full, b)[:3]
    with pytest.raises(ValueError):
        oracle_lib.apply_keyed(m, nonrep, 1)
    with pytest.raises(ValueError):          # wrong number of up spins
        oracle_lib.apply_keyed(m, np.array([7], np.uint64), 1)


def test_rep_many_and_sampled_states(oracle_lib):
    """The batched representative search equals the single-state one, and the
    basis-free row sampler returns basis states only."""
    for m in (W.torus_model((4, 0), (0, 4), 1.0, 0.5, "B1"), W.chain_model(14, l=5),
              W.chain_model(12)):
        rng = np.random.default_rng(3)
        full = oracle_lib.full_states(m.n_sites, m.n_up)
        states = full[rng.integers(0, len(full), 300)]
        reps, inb = oracle_lib.rep_many(m, states)
        b = oracle_lib.basis(m)
        for t, r, ok in zip(states, reps, inb):
            if m.perm is None:
                assert r == t and ok
                continue
            assert r == oracle_lib.rep(m.n_sites, m.perm, int(t))[0]
            assert ok == (abs(oracle_lib.stabiliser_character_sum(m, int(r))) > 0.5)
            assert ok == (oracle_lib.index(b, int(r)) >= 0)
        got = oracle_lib.sample_basis_states(m, min(50, len(b)), 7)
        assert len(got) == min(50, len(b)) and np.all(np.diff(got.astype(np.int64)) > 0)
        assert all(oracle_lib.index(b, int(s)) >= 0 for s in got)


# ---------------------------------------------------- thermal pure states --
# The TPQ recursion and the canonical series of the oracle against the
# eigendecomposition of the block (LAPACK): the spectral forms follow from
# |k> ~ (l - h)^k |psi> with h = H/N written in the eigenbasis.

def _spectrum(oracle, m):
    b = oracle.basis(m)
    E, U = np.linalg.eigh(oracle_dense(oracle, m, b))
    return b, E, U


def _tpq_spectral(E, c2, l, N, K):
    """u_k, u2_k from the weights |c_n|^2 (l - e_n)^(2k) (e_n = E_n / N), in
    log space."""
    e = E / N
    u, u2 = np.zeros(K), np.zeros(K)
    keep = c2 > 0
    lw0 = np.log(c2[keep])
    le = np.log(l - e[keep])
    for k in range(K):
        lw = lw0 + 2 * k * le
        p = np.exp(lw - lw.max())
        p /= p.sum()
        u[k] = p @ e[keep]
        u2[k] = p @ e[keep] ** 2
    return u, u2


def _canonical_exact(E, c2, T):
    """<psi|e^{-H/T} A|psi> forms for one vector: (energy, heat, ln sum)."""
    lw = np.log(c2[c2 > 0]) - E[c2 > 0] / T
    p = np.exp(lw - lw.max())
    s = p.sum()
    e1 = p @ E[c2 > 0] / s
    e2 = p @ E[c2 > 0] ** 2 / s
    return e1, (e2 - e1 * e1) / T ** 2, lw.max() + np.log(s)


@pytest.mark.parametrize("mi", [0, 1])
def test_tpq_micro_matches_spectral_form(oracle_lib, mi):
    m = [W.chain_model(12, l=0), W.chain_model(12, l=5)][mi]
    b, E, U = _spectrum(oracle_lib, m)
    x0 = W.random_vector(3, len(b), complex_=m.is_complex)
    c2 = np.abs(U.conj().T @ (x0 / np.linalg.norm(x0))) ** 2
    l = E.max() / m.n_sites + 0.25
    u, u2 = oracle_lib.tpq_micro(m, b, x0, l, 40)
    uw, u2w = _tpq_spectral(E, c2, l, m.n_sites, 40)
    assert np.allclose(u, uw, rtol=1e-10, atol=1e-12)
    assert np.allclose(u2, u2w, rtol=1e-10, atol=1e-12)
    assert u[-1] < u[0]                     # the sequence cools


def test_tpq_canonical_single_vector_is_exact(oracle_lib):
    m = W.chain_model(12, l=0)
    b, E, U = _spectrum(oracle_lib, m)
    D, N = len(b), m.n_sites
    x0 = W.random_vector(5, D)
    c2 = np.abs(U.T @ (x0 / np.linalg.norm(x0))) ** 2
    l = E.max() / N + 0.25
    u, u2 = _tpq_spectral(E, c2, l, N, 120)
    T = np.array([0.4, 0.7, 1.0, 2.0, 10.0])
    e, c, lz = oracle_lib.tpq_canonical(u, u2, l, N, D, T)
    for t in range(len(T)):
        ee, cc, ll = _canonical_exact(E, c2, T[t])
        assert abs(e[t] - ee) <= 1e-9 * max(1.0, abs(ee))
        assert abs(c[t] - cc) <= 1e-8 * max(1.0, abs(cc))
        assert abs(lz[t] - (np.log(D) + ll)) <= 1e-9 * max(1.0, abs(ll))
    # too few steps for a low temperature: not converged, NaN
    e, c, lz = oracle_lib.tpq_canonical(u[:4], u2[:4], l, N, D, [0.05])
    assert np.isnan(e[0]) and np.isnan(c[0]) and np.isnan(lz[0])


def test_tpq_canonical_unit_vector_ensemble_is_the_trace(oracle_lib):
    """All D basis vectors as start vectors, weight 1 each: Z = Tr e^{-H/T}
    and the canonical energy and heat of the block, exactly."""
    m = W.chain_model(10, l=0)
    b, E, U = _spectrum(oracle_lib, m)
    D, N = len(b), m.n_sites
    l = E.max() / N + 0.25
    us, u2s = [], []
    for i in range(D):
        u, u2 = _tpq_spectral(E, np.abs(U[i, :]) ** 2, l, N, 100)
        us.append(u)
        u2s.append(u2)
    T = np.array([0.5, 1.0, 3.0])
    e, c, lz = oracle_lib.tpq_canonical(np.array(us), np.array(u2s), l, N, 1.0, T)
    for t in range(len(T)):
        p = np.exp(-(E - E.min()) / T[t])
        z = p.sum()
        ee = p @ E / z
        cc = (p @ E ** 2 / z - ee ** 2) / T[t] ** 2
        assert abs(e[t] - ee) <= 1e-9 * max(1.0, abs(ee))
        assert abs(c[t] - cc) <= 1e-8 * max(1.0, abs(cc))
        assert abs(lz[t] - (np.log(z) - E.min() / T[t])) <= 1e-9 * max(1.0, abs(lz[t]))
