"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bases, stabilisers and indices must be bit-exact; y = H x must agree with
the oracle to 1e-12 relative (max-norm) in FP64 / complex128 and to 2e-6 in
FP32 / complex64 (FP32 accumulation over at most ~150 terms of O(1) size;
unit round-off 6e-8).  Sizes span many 256-row tiles and a ragged tail.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def X():
    import paper_2505_02901_amd as X
    X.lib()
    assert torch.cuda.is_available()
    return X


TOL64 = 1e-12
TOL32 = 2e-6


def c4_complex_model(n_up=None):
    """20-site tilted torus, translations x C4 rotations, characters i^r:
    four blocks of five sites (the packed sublattice search) with complex
    characters."""
    m = W.torus_model((4, 2), (-2, 4), 1.0, 0.0, None, n_up=n_up)
    perm, labels = W.Torus((4, 2), (-2, 4)).symmetry_group(True, False)
    return m.with_sector(perm, W.gamma_characters(labels, 1j, 1.0), "tilted20_C4_i")


def sector_models():
    out = [W.chain_model(12), W.chain_model(20), W.chain_model(17, n_up=6)]   # U(1)
    out += [W.chain_model(12, l=l) for l in range(12)]                          # affine, real+complex
    out += [W.chain_model(24, l=l) for l in (0, 5, 12)]
    chi = np.ones(2 * 14, dtype=np.complex128)
    chi[14:] = -1
    out.append(W.chain_model(14).with_sector(W.chain_dihedral(14), chi, "dihedral14_odd"))
    # translations by even steps only: affine but not a full ring of rotations
    even = W.chain_translations(16)[::2]
    out.append(W.chain_model(16).with_sector(even, np.exp(2j * np.pi * np.arange(8) * 3 / 8),
                                             "chain16_T2_k3"))
    out += [W.torus_model((4, 0), (0, 4), 1.0, 0.5, ir) for ir in ("A1", "A2", "B1", "B2")]
    out += [W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False, n_up=n)
            for n in (10, 7)]
    out += [W.torus_model((6, 0), (0, 4), 1.0, 0.3, "A1", rotations=False, name="rect24")]
    out += [W.torus_model((6, 0), (0, 4), 1.0, 0.3, "B1", rotations=False, name="rect24b")]
    out += [c4_complex_model(n) for n in (10, 8)]
    # four blocks of eight sites (half tables of 16 entries)
    out += [W.torus_model((8, 0), (0, 4), 1.0, 0.3, ir, rotations=False, n_up=n, name="rect32")
            for ir, n in (("A1", 6), ("B2", 7))]
    # 64-bit state words: the benchmark lattices at low filling, long rings
    out += [W.torus_model((6, 0), (0, 6), 1.0, 0.5, ir, n_up=n, name="square36")
            for ir, n in (("A1", 3), ("A1", 5), ("B2", 5))]
    out += [W.torus_model((6, 2), (-2, 6), 1.0, 0.0, "A1", reflections=False, n_up=n,
                          name="tilted40") for n in (4, 5)]
    out += [W.chain_model(40, n_up=5, l=3), W.chain_model(34, n_up=4)]
    # 2-, 3- and 5-sublattice lattices (generic block count in the search)
    from test_oracle_pins import other_sublattice_models
    out += other_sublattice_models()
    return out


MODELS = sector_models()
IDS = [f"{i}-{m.name}-n{m.n_up}" for i, m in enumerate(MODELS)]
_cache = {}


def oracle_basis(m):
    # keyed by content: ids of freed temporary models are reused
    key = (m.n_sites, m.n_up, None if m.perm is None else m.perm.tobytes(),
           None if m.chi is None else np.asarray(m.chi).tobytes())
    if key not in _cache:
        _cache[key] = oracle.basis(m)
    return _cache[key]


def gpu_apply(X, H, x, dtype):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", dtype)
    yt = torch.empty_like(xt)
    H.apply(xt, yt)
    torch.cuda.synchronize()
    return yt.cpu().numpy()


def rel_err(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def test_characters_read_within_bounds(X):
    """The characters array is read for exactly n_sym entries: a large value
    stored right after it (same allocation) must not make a real sector
    complex (regression: a vectorised copy-and-test loop read one entry past
    the end)."""
    for m in (W.torus_model((4, 0), (0, 4), 1.0, 0.5, "A1"),
              W.torus_model((6, 2), (-2, 6), 1.0, 0.0, "A1", reflections=False, n_up=4),
              W.chain_model(24, l=0)):
        G = m.n_sym
        buf = np.zeros((G + 4, 2))
        buf[:G, 0] = m.chi.real
        buf[G:] = 7.0                       # poison after the last entry
        b = X.Basis(m.n_sites, m.n_up, m.perm, buf[:G])
        assert not b.is_complex, m.name
        assert b.dim == len(oracle_basis(m))


INDEXES = ["rank", "hash"]


def make_basis(X, m, index):
    """Basis with the default index (the rank bitmap for these small sectors)
    or with the hash index forced; U(1) blocks always use Lin's tables."""
    b = X.Basis.from_model(m, flags=X.XDG_FLAG_HASH_INDEX if index == "hash" else 0)
    kind, nbytes = b.index_kind
    assert b.is_complex == m.is_complex
    if m.perm is None:
        assert kind == X.XDG_INDEX_LIN
    else:
        assert kind == (X.XDG_INDEX_HASH if index == "hash" else X.XDG_INDEX_RANK)
    assert nbytes > 0
    return b


@pytest.mark.parametrize("index", INDEXES)
@pytest.mark.parametrize("m", MODELS, ids=IDS)
def test_basis_bit_exact(X, m, index):
    if m.perm is None and index == "hash":
        pytest.skip("U(1) blocks have one index")
    b = make_basis(X, m, index)
    want = oracle_basis(m)
    got = b.states()
    assert b.dim == len(want)
    assert np.array_equal(got, want)
    if m.perm is not None:
        stab = np.array([oracle.rep(m.n_sites, m.perm, int(s))[2] for s in want[:2000]])
        assert np.array_equal(b.stabilisers(0, len(stab)), stab)
    # index: every basis state maps to its position
    assert np.array_equal(b.index(want), np.arange(len(want)))
    # and random popcount-n states map to the oracle's answer (-1 if not a rep)
    rng = np.random.default_rng(7)
    probes = []
    for _ in range(3000):
        bits = rng.choice(m.n_sites, m.n_up, replace=False)
        probes.append(int(sum(1 << int(q) for q in bits)))
    probes += [(1 << m.n_sites) - 1, 0, int(want[-1]) + 1]
    # same popcount beyond the last representative (past the end of a rank
    # bitmap): the next state in numeric order and the largest one
    last = int(want[-1])
    if 0 < m.n_up < m.n_sites:
        low = last & -last
        ripple = last + low
        nxt = (((ripple ^ last) >> 2) // low) | ripple
        if nxt < (1 << m.n_sites):
            probes.append(nxt)
        probes.append(((1 << m.n_up) - 1) << (m.n_sites - m.n_up))
    want_idx = np.array([oracle.index(want, s) for s in probes])
    assert np.array_equal(b.index(probes), want_idx)


@pytest.mark.parametrize("index", INDEXES)
@pytest.mark.parametrize("m", MODELS, ids=IDS)
def test_apply_matches_oracle(X, m, index):
    if m.perm is None and index == "hash":
        pytest.skip("U(1) blocks have one index")
    b = make_basis(X, m, index)
    H = X.Hamiltonian.from_model(b, m)
    basis = oracle_basis(m)
    D = len(basis)
    cplx = m.is_complex
    for nvec in (1, 3):
        x = W.random_vector(11 + nvec, D, nvec, kind="uniform", complex_=cplx)
        y_or = oracle.apply(m, basis, x)
        if not cplx:
            assert np.max(np.abs(y_or.imag)) < 1e-12 * max(1, np.max(np.abs(y_or)))
            y_or = y_or.real
        dt64 = torch.complex128 if cplx else torch.float64
        dt32 = torch.complex64 if cplx else torch.float32
        y64 = gpu_apply(X, H, x, dt64)
        assert rel_err(y64, y_or) < TOL64, (m.name, nvec)
        y32 = gpu_apply(X, H, x, dt32)
        assert rel_err(y32, y_or) < TOL32, (m.name, nvec)
    if not cplx:
        # complex vectors on a real block: real and imaginary parts independently
        x = W.random_vector(5, D, 2, kind="gauss", complex_=True)
        yc = gpu_apply(X, H, x, torch.complex128)
        assert rel_err(yc, oracle.apply(m, basis, x)) < TOL64


@pytest.mark.parametrize("search,flags", [(4, 0), (3, 0)], ids=["table", "sublattice"])
def test_apply_other_search_kinds(X, search, flags):
    # the generic byte-table search and an explicitly requested sublattice
    # search give the same basis and the same y as the automatic choice
    for m in (W.torus_model((4, 0), (0, 4), 1.0, 0.5, "B1"),
              W.torus_model((6, 0), (0, 6), 1.0, 0.5, "A1", n_up=5, name="square36"),
              W.chain_model(16, l=5)):
        if search == 3 and m.n_sites == 16 and m.perm.shape[0] == 16:
            continue   # a ring has no block structure in its natural labelling
        b0 = X.Basis.from_model(m)
        b1 = X.Basis.from_model(m, search=search, flags=flags)
        assert b1.search_kind[0] == search
        assert np.array_equal(b0.states(), b1.states())
        assert np.array_equal(b0.stabilisers(), b1.stabilisers())
        h0 = X.Hamiltonian.from_model(b0, m)
        h1 = X.Hamiltonian.from_model(b1, m)
        x = W.random_vector(8, b0.dim, 2, kind="gauss", complex_=True)
        y0 = gpu_apply(X, h0, x, torch.complex128)
        y1 = gpu_apply(X, h1, x, torch.complex128)
        assert rel_err(y1, y0) < 1e-14
        y_or = oracle.apply(m, oracle_basis(m), x)
        assert rel_err(y1, y_or) < TOL64


def test_ring_bond_order(X):
    # a ring whose bonds are listed in order (b, b + 1 mod N) takes the
    # domain-wall mask s ^ rotr(s, 1); reversed pairs take it too, a shuffled
    # list walks the bonds one by one: all give the oracle's y, and the first
    # two give the same bits
    for m in (W.chain_model(20, l=3), W.chain_model(18), W.chain_model(36, n_up=3, l=5)):
        basis = oracle_basis(m)
        b = X.Basis.from_model(m)
        x = W.random_vector(17, len(basis), 1, kind="gauss", complex_=True)
        y_or = oracle.apply(m, basis, x)
        sites = np.asarray(m.sites, dtype=np.int32).reshape(-1, 2)
        jz = np.asarray(m.jz, dtype=np.float64)
        jxy = np.asarray(m.jxy, dtype=np.float64)
        order = np.random.default_rng(5).permutation(len(jz))
        ys = []
        for st, z, j in ((sites, jz, jxy), (sites[:, ::-1].copy(), jz, jxy),
                         (sites[order].copy(), jz[order].copy(), jxy[order].copy())):
            H = X.Hamiltonian(b, st, z, j)
            ys.append(gpu_apply(X, H, x, torch.complex128))
            assert rel_err(ys[-1], y_or) < TOL64, m.name
        assert np.array_equal(ys[0], ys[1])


def test_fp32_accumulation_modes(X):
    # FP32 vectors: by default the row is accumulated in FP64 and rounded once,
    # so y agrees with the exact product of the FP32-rounded x to one FP32
    # rounding; with XDG_FLAG_F32_ACCUMULATE the accumulation is FP32.
    for m in (W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "B1", reflections=False),
              W.chain_model(20, l=7)):
        basis = oracle_basis(m)
        x = W.random_vector(31, len(basis), 2, kind="gauss", complex_=True)
        x32 = x.astype(np.complex64)
        y_or = oracle.apply(m, basis, x32.astype(np.complex128))
        b0 = X.Basis.from_model(m)
        b1 = X.Basis.from_model(m, flags=X.XDG_FLAG_F32_ACCUMULATE)
        y0 = gpu_apply(X, X.Hamiltonian.from_model(b0, m), x32, torch.complex64)
        y1 = gpu_apply(X, X.Hamiltonian.from_model(b1, m), x32, torch.complex64)
        assert rel_err(y0, y_or) < 1.2e-7, m.name
        assert rel_err(y1, y_or) < TOL32, m.name
    # the rank-addressed x with FP32 accumulation (general and all-one characters)
    for irrep in ("B1", "A1"):
        m = W.torus_model((4, 2), (-2, 4), 1.0, 0.0, irrep, reflections=False)
        b1 = X.Basis.from_model(m, flags=X.XDG_FLAG_F32_ACCUMULATE)
        H1 = X.Hamiltonian.from_model(b1, m)
        x = torch.randn(b1.dim, 2, dtype=torch.float32, device="cuda")
        ref, y = torch.empty_like(x), torch.full_like(x, float("nan"))
        X.xdg_apply_with_config(H1.handle, x, ref, xr=0)
        X.xdg_apply_with_config(H1.handle, x, y, xr=1)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), irrep
    with pytest.raises(X.XdgError):
        X.Basis(8, 4, flags=64)


def test_apply_nvec8_and_determinism(X):
    m = W.chain_model(24, l=7)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    basis = oracle_basis(m)
    x = W.random_vector(3, len(basis), 8, kind="gauss", complex_=True)
    y1 = gpu_apply(X, H, x, torch.complex64)
    y2 = gpu_apply(X, H, x, torch.complex64)
    assert np.array_equal(y1, y2)
    assert rel_err(y1, oracle.apply(m, basis, x)) < TOL32
    # single-vector columns give bit-identical results (same per-row order)
    y_col = gpu_apply(X, H, np.ascontiguousarray(x[:, 3]), torch.complex64)
    assert np.array_equal(y_col, y1[:, 3])


def test_batched_apply_equals_single(X):
    ms = [W.chain_model(16, l=l) for l in range(16)]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    xs, ys, ref = [], [], []
    for i, (b, h) in enumerate(zip(bs, hs)):
        x = torch.from_numpy(W.random_vector(100 + i, b.dim, 4, complex_=True)).to("cuda", torch.complex64)
        xs.append(x)
        ys.append(torch.empty_like(x))
        yr = torch.empty_like(x)
        h.apply(x, yr)
        ref.append(yr)
    X.xdg_apply_batched([h.handle for h in hs], xs, ys)
    torch.cuda.synchronize()
    for y, r in zip(ys, ref):
        assert torch.equal(y, r)


def test_batched_sublattice_apply_equals_single(X):
    """The persistent batched launch over sublattice-coded sectors (four
    irreps of the 6x6 torus at n_up = 7, and of the 20-site torus; FP32 and
    FP64, one and three vectors) equals the single-sector applies bitwise."""
    for lat in (((6, 0), (0, 6), 0.5, 7), ((4, 2), (-2, 4), 0.0, 8)):
        a1, a2, j2, nu = lat
        ms = [W.torus_model(a1, a2, 1.0, j2, irrep, n_up=nu) for irrep in ("A1", "A2", "B1", "B2")]
        bs = [X.Basis.from_model(m) for m in ms]
        hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
        for dt, nv in ((torch.float32, 1), (torch.float64, 3)):
            xs = [torch.randn(b.dim, nv, dtype=dt, device="cuda") for b in bs]
            ys = [torch.full_like(x, float("nan")) for x in xs]
            X.xdg_apply_batched([h.handle for h in hs], xs, ys)
            for h, x, y in zip(hs, xs, ys):
                r = torch.empty_like(x)
                h.apply(x, r)
                torch.cuda.synchronize()
                assert torch.equal(r, y), (lat, dt, nv)


def test_random_state_matches_generator(X):
    for kind, name in ((0, "uniform"), (1, "gauss")):
        t = torch.empty(1000, 3, dtype=torch.float64, device="cuda")
        X.xdg_random_state(t, 99, kind)
        want = W.random_vector(99, 1000, 3, kind=name)
        got = t.cpu().numpy()
        if kind == 0:
            assert np.array_equal(got, want)
        else:
            assert np.max(np.abs(got - want)) < 1e-13


def test_nnz_count(X):
    m = W.chain_model(16)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    # every row has 16 bonds; off-diagonal terms = bonds with unequal spins
    basis = oracle_basis(m)
    T = sum(len(oracle.row_terms(m, int(s))[1]) for s in basis)
    assert H.nnz == len(basis) + T == 12870 + 109824


def test_empty_and_degenerate_blocks(X):
    # n_up = 0 and n_up = N: one state
    for n_up in (0, 10):
        m = W.chain_model(10, n_up=n_up, l=0)
        b = X.Basis.from_model(m)
        assert b.dim == 1
        H = X.Hamiltonian.from_model(b, m)
        x = np.ones(1)
        assert abs(gpu_apply(X, H, x, torch.float64)[0] - 10 * 0.25) < 1e-15
    # an empty sector: n_up = 1 on a ring at k != 0 has dim 1, k = 0 too; take a
    # stabiliser-incompatible sector: all-up ring at k = 1
    m = W.chain_model(6, n_up=6, l=1)
    b = X.Basis.from_model(m)
    assert b.dim == 0 == len(oracle_basis(m))
    H = X.Hamiltonian.from_model(b, m)
    e = torch.empty(0, dtype=torch.complex128, device="cuda")
    H.apply(e, torch.empty(0, dtype=torch.complex128, device="cuda"))
    # no thermal sequence on an empty block
    with pytest.raises(X.XdgError):
        H.tpq(1.0, 3)


def test_apply_argument_errors(X):
    m = W.chain_model(8, l=1)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(X.XdgError):          # real vector on a complex block
        H.apply(x, torch.zeros_like(x))
    xc = torch.zeros(b.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):          # x == y, refused by the binding
        X.xdg_apply(H.handle, xc, xc)
    with pytest.raises(X.XdgError):          # x == y as raw pointers: refused by the C ABI
        X.xdg_apply(H.handle, xc.data_ptr(), xc.data_ptr(), nvec=1, dtype=X.XDG_C128)
    with pytest.raises(X.XdgError):          # bonds not invariant
        X.Hamiltonian(b, m.sites[:-1], m.jz[:-1], m.jxy[:-1])
    with pytest.raises(X.XdgError):
        X.Basis(8, 9)


SHAPE_CASES = [
    (W.torus_model((6, 0), (0, 6), 1.0, 0.5, "A1", n_up=7), 0),          # sublattice, 4 blocks
    (W.sublattice_model("triangle3", (4, -2), (2, 2), rot_char=np.exp(1j * np.pi / 3),
                        name="triangle3_12_E"), 0),                    # sublattice, 3 blocks
    (W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False, n_up=8),
     4),                                                               # forced byte tables
    (W.chain_model(24, l=5), 0),                                       # ring search
    (W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False, n_up=8),
     0),                                                               # 4 blocks of 5 sites
    (W.torus_model((6, 0), (0, 4), 1.0, 0.3, "B1", rotations=False, name="rect24b"), 0),
    (c4_complex_model(9), 0),                                          # packed, complex chi
    (W.torus_model((8, 0), (0, 4), 1.0, 0.3, "B2", rotations=False, n_up=5, name="rect32"),
     0),                                                               # packed, 8-site blocks
]


@pytest.mark.parametrize("case", range(len(SHAPE_CASES)))
def test_every_launch_shape_gives_the_same_y(X, case):
    """The autotuner's candidates (grid, vectors per pass, occupancy copy,
    row or compacted term loop, x through the rank index or rank-addressed)
    and both forms of the sublattice search compute bitwise the same y."""
    m, search = SHAPE_CASES[case]
    b = X.Basis.from_model(m, search=search)
    H = X.Hamiltonian.from_model(b, m)
    cdt = torch.complex128 if b.is_complex else torch.float64
    for dt in ((cdt, torch.complex64) if b.is_complex else (torch.float64, torch.float32)):
        g = torch.Generator(device="cuda").manual_seed(case)
        x = torch.randn(b.dim, 2, dtype=dt, device="cuda", generator=g)
        ref = torch.empty_like(x)
        H.apply(x, ref)
        for grid in (0, 1, 5, 256):
            for nv in (1, 2, 8):
                for occ in (-1, 0, 1):
                    for compact in (0, 1):
                        for form in (0, 2):
                            for xr in (0, 1):
                                y = torch.full_like(x, float("nan"))
                                X.xdg_apply_with_config(H.handle, x, y, grid=grid, nv=nv,
                                                        occ=occ, compact=compact,
                                                        sub_form=form, xr=xr)
                                torch.cuda.synchronize()
                                assert torch.equal(y, ref), (m.name, dt, grid, nv, occ,
                                                             compact, form, xr)
        code = {torch.float64: X.XDG_F64, torch.float32: X.XDG_F32,
                torch.complex128: X.XDG_C128, torch.complex64: X.XDG_C64}[dt]
        cfg = X.xdg_apply_tuned_config(H.handle, code, 2)
        assert cfg["nv"] in (1, 2, 4, 8) and cfg["grid"] >= 1
    with pytest.raises(X.XdgError):
        X.xdg_apply_with_config(H.handle, x, torch.empty_like(x), nv=3)
    with pytest.raises(X.XdgError):
        X.xdg_apply_with_config(H.handle, x, torch.empty_like(x), sub_form=1)
    with pytest.raises(X.XdgError):
        X.xdg_apply_with_config(H.handle, x, torch.empty_like(x), xr=2)
    with pytest.raises(X.XdgError):                  # not tuned for this (dtype, nvec)
        X.xdg_apply_tuned_config(H.handle, code, 7)


XR_CASES = [0, 4, 5, 6, 7]   # the sublattice cases of SHAPE_CASES with four blocks


@pytest.mark.parametrize("case", XR_CASES)
def test_rank_addressed_x_layouts(X, case):
    """The rank-addressed copy of x through changes of its layout on one
    Hamiltonian (one vector, three vectors, FP64 / FP32, complex vectors on a
    real block, back to one vector: each change re-zeroes the slots outside
    the block) and calls alternating between two streams: every y equals the
    one through the rank index, bitwise, against the oracle's H x in FP64."""
    m, _ = SHAPE_CASES[case]
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    basis = oracle_basis(m)
    cdt = (torch.complex128, torch.complex64)
    forms = [(1, cdt[0] if b.is_complex else torch.float64),
             (3, cdt[1] if b.is_complex else torch.float32),
             (2, cdt[0]), (1, cdt[1] if b.is_complex else torch.float32),
             (1, cdt[0] if b.is_complex else torch.float64)]
    for i, (nv, dt) in enumerate(forms):
        x0 = W.random_vector(300 + i, b.dim, nv, complex_=dt.is_complex)
        x = torch.from_numpy(np.ascontiguousarray(x0)).to("cuda", dt)
        ref, y = torch.empty_like(x), torch.full_like(x, float("nan"))
        X.xdg_apply_with_config(H.handle, x, ref, xr=0)
        X.xdg_apply_with_config(H.handle, x, y, xr=1)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (m.name, nv, dt)
        if i == 0:
            want = oracle.apply(m, basis, x0.astype(np.complex128))
            got = y.cpu().numpy().astype(np.complex128)
            assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want)))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    dt = cdt[1] if b.is_complex else torch.float32
    xs = [torch.randn(b.dim, dtype=dt, device="cuda") for _ in range(4)]
    ref = [torch.empty_like(x) for x in xs]
    for x, r in zip(xs, ref):
        X.xdg_apply_with_config(H.handle, x, r, xr=0)
    torch.cuda.synchronize()
    ys = [torch.full_like(x, float("nan")) for x in xs]
    for k, (x, y) in enumerate(zip(xs, ys)):
        st = s1 if k % 2 == 0 else s2
        X.xdg_apply_with_config(H.handle, x, y, xr=1, stream=st.cuda_stream)
    torch.cuda.synchronize()
    for y, r in zip(ys, ref):
        assert torch.equal(y, r)


def test_failure_paths(X):
    """XDG_ENOMEM under a cap on the library's device memory (the call fails
    cleanly and works again once the cap is lifted), XDG_ENOCONV with the
    outputs written, and a negative cap refused."""
    m = W.chain_model(24, l=0)
    used = X.xdg_set_device_memory_limit(0)
    try:
        X.xdg_set_device_memory_limit(used + (64 << 10))
        with pytest.raises(X.XdgError) as e:
            X.Basis.from_model(m)
        assert e.value.code == X.XDG_ENOMEM
        assert "limit" in str(e.value)
    finally:
        X.xdg_set_device_memory_limit(0)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    assert X.xdg_set_device_memory_limit(0) > used
    rc, ev, al, be = H.lanczos(k=1, tol=1e-15, max_iter=3, seed=1)
    assert rc == X.XDG_ENOCONV and len(al) == 3 and np.isfinite(ev[0])
    rc, ev, al, be = H.lanczos(k=1, tol=0.0, max_iter=3, seed=1)
    assert rc == X.XDG_OK
    with pytest.raises(X.XdgError):
        X.xdg_set_device_memory_limit(-1)


def test_rank_addressed_x_out_of_memory(X):
    """The rank-addressed copy of x under a memory cap too small for it:
    XDG_ENOMEM before any launch, then the same call works once the cap is
    lifted, and y equals the form through the rank index."""
    m, _ = SHAPE_CASES[0]
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    x = torch.randn(b.dim, 3, dtype=torch.float64, device="cuda")
    ref, y = torch.empty_like(x), torch.full_like(x, float("nan"))
    X.xdg_apply_with_config(H.handle, x, ref, xr=0)
    used = X.xdg_set_device_memory_limit(0)
    try:
        X.xdg_set_device_memory_limit(used + 256)
        with pytest.raises(X.XdgError) as e:
            X.xdg_apply_with_config(H.handle, x, y, xr=1)
        assert e.value.code == X.XDG_ENOMEM
    finally:
        X.xdg_set_device_memory_limit(0)
    X.xdg_apply_with_config(H.handle, x, y, xr=1)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)


def test_batched_plans_follow_new_pointers(X):
    """Cached batched plans are keyed by the vectors: new tensors, then the
    first ones again, all give the single-block results; batched Lanczos
    runs from two different start blocks match single-vector runs from the
    same columns."""
    ms = [W.chain_model(14, l=l) for l in (0, 3, 7)]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    handles = [h.handle for h in hs]
    g = torch.Generator(device="cuda").manual_seed(5)

    def block():
        return [torch.randn(b.dim, 2, dtype=torch.complex128, device="cuda", generator=g)
                for b in bs]

    def check(xs):
        ys = [torch.full_like(x, float("nan")) for x in xs]
        X.xdg_apply_batched(handles, xs, ys)
        for h, x, y in zip(hs, xs, ys):
            r = torch.empty_like(x)
            h.apply(x, r)
            torch.cuda.synchronize()
            assert torch.equal(r, y)
    xa, xb = block(), block()
    check(xa)
    check(xb)
    check(xa)
    for v0s in (block(), block()):
        # a real block gets a real start block (the complex recurrence then
        # stays real and equals the real one)
        v0s = [v if b.is_complex else torch.complex(v.real, torch.zeros_like(v.real))
               for v, b in zip(v0s, bs)]
        ev, al, be = X.xdg_lanczos_eigval_batched(handles, nvec=2, n_iter=25, prec=0, v0s=v0s)
        for i, h in enumerate(hs):
            for c in range(2):
                col = v0s[i][:, c]
                col = (col if bs[i].is_complex else col.real).contiguous()
                st, e1, a1, b1 = h.lanczos(k=1, tol=0.0, max_iter=25, prec=0, v0=col)
                assert abs(ev[i, c] - e1[0]) < 1e-10 * abs(e1[0]), (i, c, ev[i, c], e1[0])
                assert np.max(np.abs(al[i, c, :10] - a1[:10])) < 1e-10


def test_binding_refuses_mismatched_tensors(X):
    """Sizes and dtypes are checked against the block before any launch: a
    tensor from a larger sector or an FP32 y for an FP64 x raises ValueError."""
    m = W.chain_model(10, l=0)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    big = X.Basis.from_model(W.chain_model(12, l=0))
    assert X.xdg_ham_dim(H.handle) == (b.dim, False)
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    H.apply(x, y)                                        # the right sizes pass
    bad = [
        (x, torch.zeros(big.dim, dtype=torch.float64, device="cuda")),   # y too long
        (torch.zeros(b.dim - 1, dtype=torch.float64, device="cuda"), y),  # x too short
        (x, torch.zeros(b.dim, dtype=torch.float32, device="cuda")),     # dtype mismatch
        (torch.zeros(b.dim, 3, dtype=torch.float64, device="cuda"), y),  # nvec mismatch
        (x, x.view(b.dim)),                                               # aliasing
    ]
    for xx, yy in bad:
        with pytest.raises(ValueError):
            H.apply(xx, yy)
    with pytest.raises(ValueError):
        X.xdg_apply_batched([H.handle], [x], [torch.zeros(3, dtype=torch.float64, device="cuda")])
    with pytest.raises(ValueError):                      # start vector of the wrong form
        H.lanczos(k=1, tol=0.0, max_iter=5, prec=X.XDG_PREC_F32VEC, v0=x)
    with pytest.raises(ValueError):
        H.lanczos(k=1, tol=0.0, max_iter=5, prec=X.XDG_PREC_F64, v0=x[:-1])
    with pytest.raises(ValueError):
        X.xdg_expect_szsz(b.handle, torch.zeros(big.dim, dtype=torch.float64, device="cuda"),
                          [(0, 1)])
    st, ev, al, be = H.lanczos(k=1, tol=0.0, max_iter=5, prec=X.XDG_PREC_F64)
    with pytest.raises(ValueError):
        X.xdg_lanczos_eigvec(H.handle, al, be, torch.zeros(b.dim, dtype=torch.float32,
                                                           device="cuda"))


@pytest.mark.parametrize("prec,tol", [(0, 1e-12), (1, 1e-7)])
def test_lanczos_chain16_bethe(X, prec, tol):
    m = W.chain_model(16)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    e_bethe = -7.142296360617     # Bethe ansatz, pinned in test_oracle_pins
    st, ev, al, be = H.lanczos(k=1, tol=1e-13 if prec == 0 else 1e-9, max_iter=300, seed=1,
                               prec=prec)
    assert abs(ev[0] - e_bethe) < tol * abs(e_bethe), (ev[0], len(al))


def test_lanczos_matches_oracle_sequence(X):
    m = W.chain_model(20, l=3)
    basis = oracle_basis(m)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    x0 = W.random_vector(21, len(basis), 1, kind="gauss", complex_=True)
    st_o, ev_o, al_o, be_o = oracle.lanczos(m, basis, x0, k=2, tol=0.0, max_iter=40)
    v0 = torch.from_numpy(x0).to("cuda", torch.complex128)
    st, ev, al, be = H.lanczos(k=2, tol=0.0, max_iter=40, prec=0, v0=v0)
    assert len(al) == len(al_o) == 40
    # early recurrence coefficients agree to rounding; Ritz values to 1e-12
    assert np.max(np.abs(al[:10] - al_o[:10])) < 1e-11
    assert np.max(np.abs(be[:10] - be_o[:10])) < 1e-11
    assert np.max(np.abs(ev - ev_o)) < 1e-11 * np.max(np.abs(ev_o))


def test_lanczos_reorth_and_breakdown(X):
    m = W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False)
    basis = oracle_basis(m)
    Hd = oracle.apply(m, basis, np.eye(len(basis), dtype=np.complex128)).real
    want = np.linalg.eigvalsh(Hd)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    got = {}
    for prec in (3, 2):
        st, ev, al, be = H.lanczos(k=3, tol=1e-14, max_iter=min(len(basis), 120), seed=4,
                                   prec=prec)
        tol = 1e-10 if prec == 3 else 1e-5
        assert np.max(np.abs(ev - want[:3])) < tol, (prec, ev, want[:3])
        got[prec] = ev
    # FP32 vectors (FP64 reorthogonalisation) against FP64 from the same start
    # vector: the ground-state bound |dE0| / |E0| <= 1e-7
    assert abs(got[2][0] - got[3][0]) <= 1e-7 * abs(got[3][0]), got
    # ferromagnetic state in the fully polarised sector: H v = E v at once,
    # beta_1 = 0 terminates after one step
    m2 = W.chain_model(8, n_up=8, l=0)
    b2 = X.Basis.from_model(m2)
    H2 = X.Hamiltonian.from_model(b2, m2)
    st, ev, al, be = H2.lanczos(k=1, tol=1e-12, max_iter=50, seed=3, prec=0)
    assert st == 0 and len(al) == 1 and abs(ev[0] - 2.0) < 1e-14


def test_batched_lanczos_matches_single(X):
    ms = [W.chain_model(12, l=l) for l in range(12)]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    ev, al, be = X.xdg_lanczos_eigval_batched([h.handle for h in hs], nvec=4, n_iter=60, seed=9,
                                              prec=1)
    ev64, _, _ = X.xdg_lanczos_eigval_batched([h.handle for h in hs], nvec=4, n_iter=60, seed=9,
                                              prec=0)
    for i, (m, b) in enumerate(zip(ms, bs)):
        basis = oracle_basis(m)
        e0 = np.linalg.eigvalsh(oracle.apply(m, basis, np.eye(len(basis), dtype=complex)))[0]
        assert np.max(np.abs(ev[i] - e0)) < 1e-6 * max(1, abs(e0)), (i, ev[i], e0)
        assert np.max(np.abs(ev64[i] - e0)) < 1e-11 * max(1, abs(e0)), (i, ev64[i], e0)
        # FP32 vectors against FP64 from the same start vectors: |dE0|/|E0| <= 1e-7
        assert abs(ev[i].min() - ev64[i].min()) <= 1e-7 * abs(e0), (i, ev[i], ev64[i])


# ------------------------------------------ second Lanczos pass, measurements
EIG_CASES = [W.chain_model(12), W.chain_model(12, l=0), W.chain_model(12, l=5),
             W.chain_model(16, l=0), W.torus_model((4, 0), (0, 4), 1.0, 0.5, "B1"),
             W.torus_model((4, 2), (-2, 4), 1.0, 0.0, "A1", reflections=False)]
EIG_IDS = [f"{m.name}-n{m.n_up}" for m in EIG_CASES]


@pytest.mark.parametrize("m", EIG_CASES, ids=EIG_IDS)
def test_eig0_second_pass_matches_dense(X, m):
    basis = oracle_basis(m)
    e_or, v_or = oracle.dense_ground_state(m, basis)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    D = b.dim
    for prec, tol_e, tol_v in ((0, 1e-11, 1e-9), (1, 1e-6, 1e-5)):
        e, psi, al, be = H.eig0(tol=1e-14 if prec == 0 else 1e-9, max_iter=min(D, 250), seed=5,
                                prec=prec)
        # the Ritz value of the second pass is the first pass's lowest one
        assert e == X.xdg_lanczos_eigval(H.handle, k=1, tol=0.0, max_iter=len(al), seed=5,
                                         prec=prec)[1][0]
        assert abs(e - e_or) < tol_e * abs(e_or), (prec, e, e_or)
        p = psi.cpu().numpy().astype(np.complex128)
        assert abs(np.linalg.norm(p) - 1) < tol_v
        assert 1 - abs(np.vdot(v_or, p)) < tol_v, (prec, abs(np.vdot(v_or, p)))
        # <psi|H|psi> through the apply kernel
        hp = torch.empty_like(psi)
        H.apply(psi, hp)
        torch.cuda.synchronize()
        assert abs(np.vdot(p, hp.cpu().numpy()).real - e_or) < tol_e * abs(e_or)


@pytest.mark.parametrize("m", EIG_CASES, ids=EIG_IDS)
def test_expect_szsz_matches_definition(X, m):
    """GPU symmetrised correlations against the oracle's product-state
    expansion of the same vector (plain S^z_a S^z_b)."""
    basis = oracle_basis(m)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    e, psi, _, _ = H.eig0(tol=1e-13, max_iter=min(b.dim, 200), seed=2, prec=0)
    N = m.n_sites
    pairs = [(0, j) for j in range(N)] + [(3, 1), (N - 1, 2)]
    got = X.xdg_expect_szsz(b.handle, psi, pairs)
    p = psi.cpu().numpy()
    full, amp = oracle.expand_state(m, basis, p)
    want = np.array([oracle.szsz_definition(full, amp, a, c) for a, c in pairs])
    assert np.max(np.abs(got - want)) < 1e-12, (got, want)
    assert abs(got[0] - 0.25) < 1e-12
    if 2 * m.n_up == N:
        assert abs(got[:N].sum()) < 1e-12
    # FP32 vectors: the same measurement within single-precision rounding
    got32 = X.xdg_expect_szsz(b.handle, psi.to(torch.complex64 if b.is_complex else torch.float32),
                              pairs)
    assert np.max(np.abs(got32 - want)) < 1e-6


def test_second_pass_errors(X):
    m = W.chain_model(12, l=0)
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    _, _, al, be = H.lanczos(k=1, tol=0.0, max_iter=20, seed=1, prec=0)
    psi = torch.empty(b.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(X.XdgError):      # forms with reorthogonalisation are refused
        X.xdg_lanczos_eigvec(H.handle, al, be, psi, seed=1, prec=3)
    with pytest.raises(X.XdgError):      # Ritz index out of range
        X.xdg_lanczos_eigvec(H.handle, al, be, psi, seed=1, prec=0, which=20)
    with pytest.raises(X.XdgError):      # site out of range
        X.xdg_expect_szsz(b.handle, psi, [(0, 12)])


def test_ftlm_batched_matches_oracle_quadrature(X):
    """Thermodynamics from R random vectors x M Lanczos steps in every momentum
    sector of the N = 10 ring (batched GPU recurrences, FP64): the library's
    FTLM against the oracle's recurrences from the same start vectors, with
    the quadrature taken by LAPACK."""
    N, R, M = 10, 4, 15
    ms = [W.chain_model(N, l=l) for l in range(N)]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    v0 = [W.random_vector(40 + i, b.dim, R, kind="gauss", complex_=True) for i, b in enumerate(bs)]
    v0t = [torch.from_numpy(v).to("cuda", torch.complex128) for v in v0]
    ev, al, be = X.xdg_lanczos_eigval_batched([h.handle for h in hs], nvec=R, n_iter=M, prec=0,
                                              v0s=v0t)
    weights = np.repeat([b.dim / R for b in bs], R)
    T = np.array([0.2, 0.5, 1.0, 2.0, 10.0])
    e, c, lz = X.xdg_ftlm_thermo(al.reshape(-1, M), be.reshape(-1, M), weights, T)
    nodes, wts = [], []
    for i, m in enumerate(ms):
        basis = oracle_basis(m)
        for v in range(R):
            st, _, a_o, b_o = oracle.lanczos(m, basis, v0[i][:, v], k=1, tol=0.0, max_iter=M)
            assert len(a_o) == M
            assert np.max(np.abs(al[i, v] - a_o)) < 1e-9 and np.max(np.abs(be[i, v] - b_o)) < 1e-9
            Tm = np.diag(a_o) + np.diag(b_o[:-1], 1) + np.diag(b_o[:-1], -1)
            E_, U = np.linalg.eigh(Tm)
            nodes.append(E_)
            wts.append(bs[i].dim / R * U[0] ** 2)
    nodes, wts = np.concatenate(nodes), np.concatenate(wts)
    for t, T_ in enumerate(T):
        f = wts * np.exp(-(nodes - nodes.min()) / T_)
        Z = f.sum()
        E = (f * nodes).sum() / Z
        E2 = (f * nodes ** 2).sum() / Z
        assert abs(e[t] - E) < 1e-9 * max(1, abs(E))
        assert abs(c[t] - (E2 - E * E) / T_ ** 2) < 1e-8 * max(1, abs(c[t]))
        assert abs(lz[t] - (np.log(Z) - nodes.min() / T_)) < 1e-9 * max(1, abs(lz[t]))
    # the lowest node is the ground-state energy of the ring (Bethe, N = 10)
    from test_oracle_pins import bethe_energy
    assert abs(nodes.min() - bethe_energy(N, N // 2)) < 1e-8


@pytest.mark.parametrize("mi", [0, 1])
def test_tpq_micro_matches_oracle(X, mi):
    """Microcanonical TPQ sequence on the GPU (one H x per step, FP64
    products) against the oracle's recursion from the same start vector:
    u and u2 to 1e-10 with FP64 vectors and 2e-5 with FP32 vectors; the
    canonical energy and heat of that one vector from the GPU sequence against
    <psi|e^{-H/T} H^k|psi> from the eigendecomposition of the oracle's block;
    a seeded run without a start vector cools from the middle of the band."""
    m = [W.chain_model(16, l=0), W.chain_model(14, l=3)][mi]
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    basis = oracle_basis(m)
    D, N = len(basis), m.n_sites
    x0 = W.random_vector(11, D, complex_=m.is_complex)
    l, K = 1.0, 50
    uo, u2o = oracle.tpq_micro(m, basis, x0, l, K)
    forms = ((X.XDG_PREC_F64, torch.complex128 if m.is_complex else torch.float64, 1e-10),
             (X.XDG_PREC_F32VEC, torch.complex64 if m.is_complex else torch.float32, 2e-5))
    for prec, dt, tol in forms:
        v0 = torch.from_numpy(x0).to("cuda", dt)
        u, u2 = X.xdg_tpq_micro(H.handle, l, K, prec=prec, v0=v0)
        assert np.max(np.abs(u - uo)) <= tol * np.max(np.abs(uo)), (prec, u[:3], uo[:3])
        assert np.max(np.abs(u2 - u2o)) <= tol * np.max(np.abs(u2o)), prec
        if prec == X.XDG_PREC_F64:
            E, U = np.linalg.eigh(oracle.apply(m, basis, np.eye(D, dtype=np.complex128)))
            c2 = np.abs(U.conj().T @ (x0 / np.linalg.norm(x0))) ** 2
            T = np.array([1.0, 2.0, 5.0])
            e, c, lz = X.xdg_tpq_thermo(u, u2, l, N, D, T)
            for t, T_ in enumerate(T):
                f = c2 * np.exp(-(E - E.min()) / T_)
                z = f.sum()
                ee = f @ E / z
                cc = (f @ E ** 2 / z - ee ** 2) / T_ ** 2
                assert abs(e[t] - ee) <= 1e-8 * max(1.0, abs(ee)), (T_, e[t], ee)
                assert abs(c[t] - cc) <= 1e-7 * max(1.0, abs(cc)), (T_, c[t], cc)
    u, u2 = H.tpq(l, 30, seed=4, prec=X.XDG_PREC_F32VEC)
    assert abs(u[0]) < 0.1 and u[-1] < u[0] and np.all(u2 >= u ** 2 - 1e-6)
    with pytest.raises(X.XdgError):
        X.xdg_tpq_micro(H.handle, l, 0)
    with pytest.raises(X.XdgError):
        X.xdg_tpq_micro(H.handle, l, 5, prec=X.XDG_PREC_F64_REORTH)


def test_tpq_micro_batched_matches_single(X):
    """Batched TPQ (four ring momenta, real and complex blocks, four start
    vectors each, one batched H x per step) against the oracle's recursion
    per start vector (1e-10 FP64 vectors, 2e-5 FP32) and against the
    one-vector call from the same start vector (1e-12 FP64); a seeded run
    cools every sequence from the middle of the band."""
    ms = [W.chain_model(12, l=l) for l in (0, 3, 6, 5)]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    nv, l, K = 4, 1.0, 40
    x0s = []
    for i, (m, b) in enumerate(zip(ms, bs)):
        x = W.random_vector(200 + i, b.dim, nv, complex_=m.is_complex)
        x0s.append(x.astype(np.complex128))
    forms = ((X.XDG_PREC_F64, torch.complex128, torch.float64, 1e-10),
             (X.XDG_PREC_F32VEC, torch.complex64, torch.float32, 2e-5))
    for prec, dt, rdt, tol in forms:
        v0s = [torch.from_numpy(x).to("cuda", dt) for x in x0s]
        u, u2 = X.xdg_tpq_micro_batched([h.handle for h in hs], l, K, nv, prec=prec, v0s=v0s)
        assert u.shape == (len(ms), nv, K)
        for i, m in enumerate(ms):
            basis = oracle_basis(m)
            for v in range(nv):
                uo, u2o = oracle.tpq_micro(m, basis, x0s[i][:, v], l, K)
                assert np.max(np.abs(u[i, v] - uo)) <= tol * np.max(np.abs(uo)), (prec, i, v)
                assert np.max(np.abs(u2[i, v] - u2o)) <= tol * np.max(np.abs(u2o)), (prec, i, v)
                if prec == X.XDG_PREC_F64:
                    col = x0s[i][:, v] if m.is_complex else x0s[i][:, v].real
                    v0 = torch.from_numpy(np.ascontiguousarray(col)).to(
                        "cuda", dt if m.is_complex else rdt)
                    us, u2s = X.xdg_tpq_micro(hs[i].handle, l, K, prec=prec, v0=v0)
                    assert np.max(np.abs(u[i, v] - us)) <= 1e-12 * np.max(np.abs(us)), (i, v)
                    assert np.max(np.abs(u2[i, v] - u2s)) <= 1e-12 * np.max(np.abs(u2s)), (i, v)
    u, u2 = X.xdg_tpq_micro_batched([h.handle for h in hs], l, 30, 2, seed=8)
    assert np.all(np.abs(u[:, :, 0]) < 0.15) and np.all(u[:, :, -1] < u[:, :, 0])
    assert np.all(u2 >= u ** 2 - 1e-6)
    with pytest.raises(X.XdgError):
        X.xdg_tpq_micro_batched([h.handle for h in hs], l, 5, 3)
    with pytest.raises(X.XdgError):
        X.xdg_tpq_micro_batched([h.handle for h in hs], l, 0, 2)



@pytest.mark.parametrize("lq", [3, 6])
def test_dynamical_structure_factor_matches_dense(X, lq):
    """S^zz(q, omega) of the N = 12 ring: ground state of the k = 0 block (two
    Lanczos passes), S^z_q applied into the k = q block, Lanczos from there and
    the continued fraction, against the dense full-space spectrum of the
    oracle with the same Lorentzian width."""
    N = 12
    m0, mq = W.chain_model(N, l=0), W.chain_model(N, l=lq)
    b0, bq = X.Basis.from_model(m0), X.Basis.from_model(mq)
    H0, Hq = X.Hamiltonian.from_model(b0, m0), X.Hamiltonian.from_model(bq, mq)
    e0, psi, _, _ = H0.eig0(tol=1e-14, max_iter=min(b0.dim, 200), seed=3, prec=0)
    q = 2 * np.pi * lq / N
    coef = np.exp(1j * q * np.arange(N)) / np.sqrt(N)
    phi = torch.zeros(bq.dim, dtype=torch.complex128, device="cuda")
    X.xdg_apply_sz_transfer(b0.handle, bq.handle, coef, psi.to(torch.complex128), phi)
    torch.cuda.synchronize()
    norm2 = float((phi.abs() ** 2).sum())
    v0 = phi if bq.is_complex else phi.real.contiguous()
    if not bq.is_complex:
        assert float(phi.imag.abs().max()) < 1e-14
    _, _, al, be = Hq.lanczos(k=1, tol=0.0, max_iter=min(bq.dim, 60), prec=0, v0=v0)
    omega = np.linspace(0.0, 4.0, 161)
    eta = 0.1
    got = X.xdg_spectral_cf(al, be, norm2, e0, omega, eta)
    E0, dE, w = oracle.dense_sz_spectrum(W.chain_model(N), coef)
    assert abs(E0 - e0) < 1e-10
    # the Lanczos ground state is accurate to ~sqrt(dE / gap) ~ 1e-7, so
    # quantities linear in |psi><psi| agree to that order
    assert abs(norm2 - w.sum()) < 1e-7 * w.sum()
    want = (w[None, :] * eta / np.pi / ((omega[:, None] - dE[None, :]) ** 2 + eta ** 2)).sum(axis=1)
    assert np.max(np.abs(got - want)) < 1e-6 * np.max(want), np.max(np.abs(got - want))
    # a coefficient vector that does not carry the character ratio is refused
    with pytest.raises(X.XdgError):
        X.xdg_apply_sz_transfer(b0.handle, bq.handle, np.ones(N), psi.to(torch.complex128), phi)
