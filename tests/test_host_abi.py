"""Host-side behaviour of the C-ABI library (CPU only: no compute call).

* the shared library loads and exports every function include/xdg.h declares;
* group / character / bond validation and its error codes
  (Sec. 3.10.1 group axioms, Sec. 3.10.2 homomorphism, invariance of H);
* the search-kind planner on the benchmark lattices.
"""
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def X():
    import paper_2505_02901_amd as X
    X.lib()
    return X


def header_functions():
    txt = open(os.path.join(ROOT, "include", "xdg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xdg_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(X):
    names = header_functions()
    assert len(names) >= 20
    L = X.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(X.exported_names()) == names
    assert X.xdg_version().startswith("xdg-mi355x")


def test_group_validation_errors(X):
    m = W.chain_model(8, l=2)
    assert X.xdg_check_group(8, m.perm, m.chi) == X.XDG_OK
    assert X.xdg_check_group(8, m.perm, None) == X.XDG_OK
    # not a bijection
    p = m.perm.copy()
    p[3, 0] = p[3, 1]
    assert X.xdg_check_group(8, p, None) == X.XDG_EINVAL
    # site out of range
    p = m.perm.copy()
    p[2, 4] = 8
    assert X.xdg_check_group(8, p, None) == X.XDG_EINVAL
    # no identity
    assert X.xdg_check_group(8, m.perm[1:], None) == X.XDG_EGROUP
    # not closed (T^0, T^1 only)
    assert X.xdg_check_group(8, m.perm[:2], None) == X.XDG_EGROUP
    # duplicate element
    assert X.xdg_check_group(8, np.vstack([m.perm, m.perm[3:4]]), None) == X.XDG_EGROUP
    # missing inverse but closed is impossible for finite sets; a set closed
    # under products with an inverse removed is not closed either
    assert X.xdg_check_group(8, np.delete(m.perm, 3, axis=0), None) == X.XDG_EGROUP
    # characters: |chi| != 1
    c = m.chi.copy()
    c[0] = 1.5
    assert X.xdg_check_group(8, m.perm, c) == X.XDG_ECHAR
    # characters: homomorphism violated
    c = m.chi.copy()
    c[1] = np.conj(c[1])
    assert X.xdg_check_group(8, m.perm, c) == X.XDG_ECHAR
    # the k = pi characters printed in Sec. 3.10.2 pass
    chi = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    assert X.xdg_check_group(8, W.chain_translations(8), chi) == X.XDG_OK
    assert X.xdg_check_group(0, None, None) == X.XDG_EINVAL
    assert X.xdg_check_group(65, None, None) == X.XDG_EINVAL


def test_bond_validation_errors(X):
    m = W.chain_model(8, l=0)
    assert X.xdg_check_bonds(8, m.perm, m.sites, m.jz, m.jxy) == X.XDG_OK
    s = m.sites.copy()
    s[0, 1] = s[0, 0]
    assert X.xdg_check_bonds(8, m.perm, s, m.jz, m.jxy) == X.XDG_EINVAL
    s = m.sites.copy()
    s[0, 1] = 9
    assert X.xdg_check_bonds(8, m.perm, s, m.jz, m.jxy) == X.XDG_EINVAL
    jz = m.jz.copy()
    jz[2] = 0.5
    assert X.xdg_check_bonds(8, m.perm, m.sites, jz, m.jxy) == X.XDG_ENOTSYM
    # open chain is not translation invariant
    assert X.xdg_check_bonds(8, m.perm, m.sites[:-1], m.jz[:-1], m.jxy[:-1]) == X.XDG_ENOTSYM
    # reversed bond orientation and duplicated bonds with split couplings are fine
    s = m.sites[:, ::-1].copy()
    assert X.xdg_check_bonds(8, m.perm, s, m.jz, m.jxy) == X.XDG_OK
    s2 = np.vstack([m.sites, m.sites])
    assert X.xdg_check_bonds(8, m.perm, s2, np.r_[m.jz, m.jz] / 2, np.r_[m.jxy, m.jxy] / 2) == 0
    # no group: any bond list of distinct in-range sites is fine
    assert X.xdg_check_bonds(8, None, m.sites[:-1], m.jz[:-1], m.jxy[:-1]) == X.XDG_OK


def test_planner_kinds(X):
    assert X.xdg_plan_search(16, None) == (X.XDG_SEARCH_U1, 0)
    assert X.xdg_plan_search(32, W.chain_translations(32)) == (X.XDG_SEARCH_AFFINE, 0)
    assert X.xdg_plan_search(12, W.chain_dihedral(12)) == (X.XDG_SEARCH_AFFINE, 0)
    c3 = W.workload("square36_j1j2_A1")[0]
    assert c3.n_sym == 288
    assert X.xdg_plan_search(36, c3.perm) == (X.XDG_SEARCH_SUBLATTICE, 4)
    c5 = W.workload("tilted40_xxz")[0]
    assert c5.n_sym == 160
    assert X.xdg_plan_search(40, c5.perm) == (X.XDG_SEARCH_SUBLATTICE, 4)
    # forced kinds
    assert X.xdg_plan_search(32, W.chain_translations(32), X.XDG_SEARCH_TABLE)[0] == X.XDG_SEARCH_TABLE
    with pytest.raises(X.XdgError):
        X.xdg_plan_search(36, c3.perm, X.XDG_SEARCH_AFFINE)
    with pytest.raises(X.XdgError):
        X.xdg_plan_search(32, W.chain_translations(32), X.XDG_SEARCH_SUBLATTICE)
    # a random relabelling destroys the block structure: generic tables
    rng = np.random.default_rng(0)
    perm = rng.permutation(36)
    inv = np.argsort(perm)
    relab = np.array([perm[g[inv]] for g in c3.perm], dtype=np.int32)
    assert X.xdg_check_group(36, relab, None) == 0
    assert X.xdg_plan_search(36, relab)[0] == X.XDG_SEARCH_TABLE
    # 2-, 3- and 5-sublattice labellings
    for kind, a1, a2, ns in (("square2", (3, 1), (-1, 3), 2), ("triangle3", (5, -1), (1, 4), 3),
                             ("square5", (2, 4), (-4, 2), 5)):
        m = W.sublattice_model(kind, a1, a2)
        assert X.xdg_plan_search(m.n_sites, m.perm) == (X.XDG_SEARCH_SUBLATTICE, ns), kind
        assert X.xdg_check_group(m.n_sites, m.perm, m.chi) == 0
        assert X.xdg_check_bonds(m.n_sites, m.perm, m.sites, m.jz, m.jxy) == 0
    # option flags: the defined bits pass, any other bit is refused
    t16 = W.chain_translations(16)
    acc = X.XDG_FLAG_F32_ACCUMULATE | X.XDG_FLAG_HASH_INDEX
    assert X.xdg_plan_search(16, t16, flags=acc) == (X.XDG_SEARCH_AFFINE, 0)
    for bad in (1, 8, 64, acc | 16):
        with pytest.raises(X.XdgError):
            X.xdg_plan_search(16, t16, flags=bad)


def test_benchmark_lattices_are_symmetric(X):
    for name in ("chain16_u1", "chain32_k0_kpi", "square36_j1j2_A1", "tilted40_xxz"):
        for m in W.workload(name):
            assert X.xdg_check_group(m.n_sites, m.perm, m.chi) == 0, name
            assert X.xdg_check_bonds(m.n_sites, m.perm, m.sites, m.jz, m.jxy) == 0, name


def test_ftlm_quadrature_against_eigh(X):
    """Host-side thermodynamics: nodes and weights of the Lanczos quadrature
    (Ritz values, squared first components) against LAPACK's eigenvectors of
    the same tridiagonal matrices."""
    rng = np.random.default_rng(5)
    R, m = 3, 25
    al = rng.normal(size=(R, m))
    be = np.abs(rng.normal(size=(R, m))) + 0.1
    w = np.array([2.0, 1.0, 0.5])
    T = np.array([0.1, 0.5, 1.0, 3.0, 20.0])
    e, c, lz = X.xdg_ftlm_thermo(al, be, w, T)
    nodes, weights = [], []
    for r in range(R):
        Tm = np.diag(al[r]) + np.diag(be[r, :-1], 1) + np.diag(be[r, :-1], -1)
        ev, U = np.linalg.eigh(Tm)
        nodes.append(ev)
        weights.append(w[r] * U[0] ** 2)
    nodes, weights = np.concatenate(nodes), np.concatenate(weights)
    for t, T_ in enumerate(T):
        f = weights * np.exp(-(nodes - nodes.min()) / T_)
        Z = f.sum()
        E = (f * nodes).sum() / Z
        E2 = (f * nodes ** 2).sum() / Z
        assert abs(e[t] - E) < 1e-12 * max(1, abs(E))
        assert abs(c[t] - (E2 - E * E) / T_ ** 2) < 1e-10 * max(1, abs(c[t]))
        assert abs(lz[t] - (np.log(Z) - nodes.min() / T_)) < 1e-12 * max(1, abs(lz[t]))
    with pytest.raises(X.XdgError):
        X.xdg_ftlm_thermo(al, be, w, [0.0])


def test_tpq_thermo_matches_oracle_series(X):
    """Host-side canonical TPQ sums (C++) against the oracle's series (plain
    Python loops) on the same microcanonical sequences: TPQ sequences of the
    oracle from three start vectors, an unconverged low temperature (NaN on
    both sides) and the argument checks."""
    import oracle
    m = W.chain_model(12, l=0)
    b = oracle.basis(m)
    D, N = len(b), m.n_sites
    l = 1.0
    us, u2s = [], []
    for seed in (1, 2, 3):
        u, u2 = oracle.tpq_micro(m, b, W.random_vector(seed, D), l, 60)
        us.append(u)
        u2s.append(u2)
    us, u2s = np.array(us), np.array(u2s)
    w = np.array([D / 3.0] * 3)
    T = np.array([0.02, 0.3, 0.6, 1.0, 2.5, 50.0])
    e, c, lz = X.xdg_tpq_thermo(us, u2s, l, N, w, T)
    eo, co, lo = oracle.tpq_canonical(us, u2s, l, N, w, T)
    assert np.array_equal(np.isnan(e), np.isnan(eo)) and np.isnan(e[0])
    ok = ~np.isnan(eo)
    assert np.allclose(e[ok], eo[ok], rtol=1e-12, atol=1e-12)
    assert np.allclose(c[ok], co[ok], rtol=1e-10, atol=1e-12)
    assert np.allclose(lz[ok], lo[ok], rtol=1e-12, atol=1e-12)
    with pytest.raises(X.XdgError):                     # l below <k|h|k>
        X.xdg_tpq_thermo(us, u2s, float(us.min()) - 0.1, N, w, T)
    with pytest.raises(X.XdgError):
        X.xdg_tpq_thermo(us, u2s, l, N, w, [0.0])
    with pytest.raises(X.XdgError):
        X.xdg_tpq_thermo(us, u2s, l, N, [0.0, 1.0, 1.0], [1.0])


def test_ftlm_exact_at_full_krylov_dimension(X):
    """With as many (reorthogonalised) Lanczos steps as the block dimension
    the quadrature is exact: the library's thermodynamics from the oracle's
    recurrence equals <r|exp(-H/T)|r> from the oracle's dense block matrix."""
    import oracle
    m = W.chain_model(10, l=0)
    b = oracle.basis(m)
    D = len(b)
    x0 = W.random_vector(8, D, kind="gauss")
    st, ev, al, be = oracle.lanczos(m, b, x0, k=1, tol=0.0, max_iter=D, reorth=True)
    H = oracle.apply(m, b, np.eye(D, dtype=np.complex128))
    En, U = np.linalg.eigh(H)
    r = x0 / np.linalg.norm(x0)
    wts = np.abs(U.conj().T @ r) ** 2
    T = np.array([0.3, 1.0, 4.0])
    pad = np.zeros(D)
    A = pad.copy(); A[:len(al)] = al
    B = pad.copy(); B[:len(be)] = be
    e, c, lz = X.xdg_ftlm_thermo(A[None, :len(al)], B[None, :len(al)], [1.0], T)
    for t, T_ in enumerate(T):
        f = wts * np.exp(-(En - En[0]) / T_)
        Z = f.sum()
        E = (f * En).sum() / Z
        assert abs(e[t] - E) < 1e-10, (T_, e[t], E)
        assert abs(lz[t] - (np.log(Z) - En[0] / T_)) < 1e-10


def test_spectral_continued_fraction_against_eigh(X):
    """The continued fraction of a tridiagonal matrix equals its resolvent's
    (0, 0) element: sum_j w_j / (z - eps_j) with LAPACK's eigenpairs."""
    rng = np.random.default_rng(9)
    m = 30
    al = rng.normal(size=m)
    be = np.abs(rng.normal(size=m)) + 0.2
    Tm = np.diag(al) + np.diag(be[:-1], 1) + np.diag(be[:-1], -1)
    ev, U = np.linalg.eigh(Tm)
    w = U[0] ** 2
    omega = np.linspace(-3, 6, 91)
    e0, eta, norm2 = -1.5, 0.07, 2.5
    got = X.xdg_spectral_cf(al, be, norm2, e0, omega, eta)
    z = omega + e0 + 1j * eta
    want = -np.imag(norm2 * (w[None, :] / (z[:, None] - ev[None, :])).sum(axis=1)) / np.pi
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
    with pytest.raises(X.XdgError):
        X.xdg_spectral_cf(al, be, norm2, e0, omega, 0.0)
