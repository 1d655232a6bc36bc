"""GPU parity at the benchmark sizes (C1-C5), in the launch configuration the
benchmark times (single-vector apply through the tuned launch, FP32 and FP64).

The oracle cannot enumerate the large sectors whole, so it checks what it can
compute one by one, and properties that hold at any size check the rest:

* dimension = projection-operator trace formula (independent of both);
* the GPU basis is strictly ascending, and on windows of the state space it
  equals the oracle's brute-force enumeration of that window bit for bit;
* sampled GPU states are representatives of compatible orbits; sampled
  random states are found (or not) exactly as the oracle says;
* sampled columns H e_r: the nonzeros, mapped to states through the GPU basis,
  equal the oracle's row r (Hermitian conjugate), to 1e-12 (FP64) / 2e-6 (FP32);
* Hermiticity <w, Hx> = conj <x, Hw>, the ferromagnetic bound lambda_max =
  sum J / 4 in the trivial sector, batched = single launches bitwise;
* N = 32 ring, k = 0: the oracle enumerates the whole sector; its basis equals
  the GPU basis bit for bit, and H x on more than 1e6 random rows equals the
  oracle's rows (FP64 to 1e-12, FP32 vectors to one FP32 rounding);
* every other full-size sector (a complex N = 32 momentum, 6x6 J1-J2, 40-site
  tilted): rows sampled at random are compared with the oracle through a
  vector keyed by the basis state (``workloads.keyed_values``), which the
  oracle evaluates without a basis list, so a wrong index position anywhere
  shows up as a wrong row;
* the FP32-vector ground-state energy is within |dE0| / |E0| <= 1e-7 of FP64
  from the same start vector at 6x6 (FP64 reorthogonalisation, 200
  iterations) and at 40 sites (100 iterations), and the batched FP32 energies
  of all 32 momenta of the N = 32 ring against sector-by-sector FP64 and the
  Bethe ansatz.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle_pins import dimension_formula

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def X():
    import paper_2505_02901_amd as X
    X.lib()
    return X


_built = {}


def built(X, name, i=0):
    key = (name, i)
    if key not in _built:
        _built.clear()
        torch.cuda.empty_cache()
        m = W.workload(name)[i]
        b = X.Basis.from_model(m)
        _built[key] = (m, b, X.Hamiltonian.from_model(b, m))
    return _built[key]


def random_states(m, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        bits = rng.choice(m.n_sites, m.n_up, replace=False)
        out.append(int(sum(1 << int(q) for q in bits)))
    return out


def check_membership(X, m, b, seed, n_members=3000, n_random=3000):
    D = b.dim
    rng = np.random.default_rng(seed)
    pos = np.sort(rng.choice(D, size=min(D, n_members), replace=False))
    for p in pos[::max(1, len(pos) // 200)]:
        s = int(b.states(int(p), 1)[0])
        r, _, _ = oracle.rep(m.n_sites, m.perm, s)
        assert r == s
        assert abs(oracle.stabiliser_character_sum(m, s)) > 0.5
    probes = random_states(m, n_random, seed + 1)
    reps = []
    for t in probes:
        r, _, _ = oracle.rep(m.n_sites, m.perm, t)
        reps.append(r)
    idx = b.index(reps)
    for r, i in zip(reps, idx):
        compatible = abs(oracle.stabiliser_character_sum(m, r)) > 0.5
        if compatible:
            assert i >= 0 and int(b.states(int(i), 1)[0]) == r
        else:
            assert i == -1
    # non-representatives are never found
    nonrep = [t for t, r in zip(probes, reps) if t != r][:500]
    assert np.all(b.index(nonrep) == -1)


def check_windows(m, b, seed, n_windows=3, width=1500):
    D = b.dim
    rng = np.random.default_rng(seed)
    for p in rng.integers(0, max(1, D - width), n_windows):
        got = b.states(int(p), min(width, D - int(p)))
        assert np.all(np.diff(got.astype(np.int64) if m.n_sites < 63 else got) > 0)
        want = oracle.basis_range(m, int(got[0]), int(got[-1]))
        assert np.array_equal(got, want)


def check_columns(X, m, b, H, seed, n_cols, dtypes):
    """y = H e_r for oracle-chosen representatives r."""
    cands = [oracle.rep(m.n_sites, m.perm, t)[0] if m.perm is not None else t
             for t in random_states(m, 50, seed)]
    cols = []
    for r in cands:
        if m.perm is None or abs(oracle.stabiliser_character_sum(m, r)) > 0.5:
            cols.append(r)
        if len(cols) == n_cols:
            break
    cplx = b.is_complex
    for r in cols:
        j = int(b.index([r])[0])
        assert j >= 0 and int(b.states(j, 1)[0]) == r
        d, targets, amps = oracle.row_terms(m, r)
        want = {}
        want[r] = want.get(r, 0) + d
        for s, a in zip(targets, amps):
            want[int(s)] = want.get(int(s), 0) + a
        for dt, tol in dtypes:
            dt = {torch.float64: torch.complex128, torch.float32: torch.complex64}[dt] if cplx else dt
            x = torch.zeros(b.dim, dtype=dt, device="cuda")
            x[j] = 1
            y = torch.empty_like(x)
            H.apply(x, y)
            torch.cuda.synchronize()
            nz = torch.nonzero(y).flatten().cpu().numpy()
            vals = y[torch.from_numpy(nz).cuda()].cpu().numpy() if len(nz) else np.zeros(0)
            states = np.array([int(b.states(int(i), 1)[0]) for i in nz], dtype=np.uint64)
            got = {int(s): v for s, v in zip(states, vals)}
            nonzero_want = {s: v for s, v in want.items() if abs(v) > 1e-14}
            assert set(got) == set(nonzero_want), (r, dt)
            scale = max(abs(v) for v in nonzero_want.values())
            for s, v in nonzero_want.items():
                # y[i] = H[i, r] = conj(H[r, i])
                assert abs(got[s] - np.conj(v)) <= tol * scale, (r, s, got[s], v)


def keyed_device(b, seed, rows, cplx, dtype, nvec=1, chunk=1 << 25):
    """Device vector whose entry at basis position i is
    keyed_values(seed, state_i), built chunk by chunk from the device basis,
    and the host states at `rows` (sorted positions)."""
    D = b.dim
    x = torch.empty((D,) if nvec == 1 else (D, nvec), dtype=dtype, device="cuda")
    rows = np.asarray(rows, np.int64)
    picked = np.zeros(len(rows), np.uint64)
    for c0 in range(0, D, chunk):
        n = min(chunk, D - c0)
        st = b.states(c0, n)
        sel = (rows >= c0) & (rows < c0 + n)
        picked[sel] = st[rows[sel] - c0]
        v = W.keyed_values_torch(seed, torch.from_numpy(st.view(np.int64)).cuda(), nvec, cplx)
        x[c0:c0 + n] = v.to(dtype)
        del v
    return x, picked


def check_keyed_rows(X, m, b, H, seed, n_rows, single_too=True):
    """H x at sampled rows (the first and last included) against the oracle,
    x keyed by state: FP64 to 1e-12 of the largest row, FP32 vectors (FP64
    accumulation, one rounding on store) to 1.2e-7 of each row."""
    D = b.dim
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([[0, D - 1], rng.integers(0, D, n_rows)]))
    cplx = b.is_complex
    forms = [(torch.complex128 if cplx else torch.float64, False)]
    if single_too:
        forms.append((torch.complex64 if cplx else torch.float32, True))
    want_states = None
    for dt, f32 in forms:
        print(f"keyed rows: {m.name} dim {D} rows {len(rows)} dtype {dt}", flush=True)
        x, states = keyed_device(b, seed, rows, cplx, dt)
        if want_states is None:
            want_states = states
        assert np.array_equal(states, want_states)
        y = torch.empty_like(x)
        H.apply(x, y)
        torch.cuda.synchronize()
        got = y[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.complex128)
        del x, y
        torch.cuda.empty_cache()
        want = oracle.apply_keyed(m, states, seed, complex_=cplx, round_to_f32=f32)
        scale = np.max(np.abs(want))
        bound = (1.2e-7 * np.abs(want) + 1e-12 * scale) if f32 else np.full(len(want), 1e-12 * scale)
        err = np.abs(got - want)
        k = int(np.argmax(err / bound))
        assert np.all(err <= bound), (m.name, dt, int(rows[k]), got[k], want[k], err[k] / scale)
    return rows


def test_c1_full_oracle_parity(X):
    m = W.workload("chain16_u1")[0]
    b = X.Basis.from_model(m)
    H = X.Hamiltonian.from_model(b, m)
    basis = oracle.basis(m)
    assert np.array_equal(b.states(), basis)
    x = W.random_vector(1, len(basis), kind="uniform")
    y_or = oracle.apply(m, basis, x).real
    for dt, tol in ((torch.float64, 1e-12), (torch.float32, 2e-6)):
        xt = torch.from_numpy(x).to("cuda", dt)
        yt = torch.empty_like(xt)
        H.apply(xt, yt)
        torch.cuda.synchronize()
        y = yt.cpu().numpy()
        assert np.max(np.abs(y - y_or)) < tol * np.max(np.abs(y_or))
    assert H.nnz == 122694


@pytest.mark.parametrize("i", [0, 1], ids=["k0", "kpi"])
def test_c2_fullsize(X, i):
    m, b, H = built(X, "chain32_k0_kpi", i)
    assert b.dim == dimension_formula(m) == 18784170
    check_windows(m, b, 10 + i)
    check_membership(X, m, b, 20 + i)
    check_columns(X, m, b, H, 30 + i, 4, [(torch.float64, 1e-12), (torch.float32, 2e-6)])
    check_hermitian(b, H, 60 + i)


def test_c2_full_oracle_basis_and_rows(X):
    """The k = 0 sector of the N = 32 ring, whole: the oracle's basis (brute
    force over all C(32, 16) states) equals the GPU's bit for bit, and H x on
    more than 1e6 random rows equals orc_apply_rows on that basis."""
    m, b, H = built(X, "chain32_k0_kpi", 0)
    print("oracle basis of chain32 k = 0 ...", flush=True)
    basis = oracle.basis(m)
    assert len(basis) == b.dim == 18784170
    got = b.states()
    assert np.array_equal(got, basis)
    del got
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([[0, b.dim - 1], rng.integers(0, b.dim, 1_050_000)]))
    assert len(rows) >= 1_000_000
    x = W.random_vector(2, b.dim, kind="gauss")
    for dt in (torch.float64, torch.float32):
        xv = x if dt == torch.float64 else x.astype(np.float32).astype(np.float64)
        xt = torch.from_numpy(x).to("cuda", dt)
        yt = torch.empty_like(xt)
        H.apply(xt, yt)
        torch.cuda.synchronize()
        got = yt[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        del xt, yt
        want = oracle.apply_rows(m, basis, rows, xv).real
        scale = np.max(np.abs(want))
        bound = 1e-12 * scale if dt == torch.float64 else 1.2e-7 * np.abs(want) + 1e-12 * scale
        assert np.all(np.abs(got - want) <= bound), dt


def test_c2_complex_sector_rows(X):
    """A complex momentum sector of the N = 32 ring (l = 5) at full size:
    dimension, basis windows, and 2e5 random rows against the oracle."""
    m, b, H = built(X, "chain32_allk", 5)
    assert b.is_complex
    assert b.dim == dimension_formula(m)
    check_windows(m, b, 70, n_windows=2, width=1500)
    check_keyed_rows(X, m, b, H, 71, 200_000)


def check_hermitian(b, H, seed, fp32=True):
    """<w, H x> = <x, H w> for random real x, w over every row of the block
    (FP64 to 1e-10; FP32 vectors with FP64 row sums to 1e-5)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5))[: 2 if fp32 else 1]:
        x = torch.randn(b.dim, dtype=dt, device="cuda", generator=g)
        w = torch.randn(b.dim, dtype=dt, device="cuda", generator=g)
        hx, hw = torch.empty_like(x), torch.empty_like(w)
        H.apply(x, hx)
        H.apply(w, hw)
        lhs = torch.dot(w.double(), hx.double()).item()
        rhs = torch.dot(x.double(), hw.double()).item()
        assert abs(lhs - rhs) < tol * max(abs(lhs), torch.linalg.vector_norm(hx.double()).item()), (dt, lhs, rhs)
        del x, w, hx, hw


def test_c3_fullsize(X):
    m, b, H = built(X, "square36_j1j2_A1")
    assert b.dim == dimension_formula(m) == 31566122
    check_windows(m, b, 40, n_windows=2, width=600)
    check_membership(X, m, b, 41, n_members=1000, n_random=1000)
    check_columns(X, m, b, H, 42, 3, [(torch.float64, 1e-12), (torch.float32, 2e-6)])
    # Hermiticity at full size
    x = torch.randn(b.dim, dtype=torch.float64, device="cuda")
    w = torch.randn(b.dim, dtype=torch.float64, device="cuda")
    hx, hw = torch.empty_like(x), torch.empty_like(w)
    H.apply(x, hx)
    H.apply(w, hw)
    lhs, rhs = torch.dot(w, hx).item(), torch.dot(x, hw).item()
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    del x, w, hx, hw
    check_rank_addressed(X, b, H, 44)


def check_rank_addressed(X, b, H, seed):
    """x through the rank index and through the rank-addressed copy give
    bitwise the same y (FP32 vectors, then FP64)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    for dt in (torch.float32, torch.float64):
        x = torch.randn(b.dim, dtype=dt, device="cuda", generator=g)
        y0, y1 = torch.empty_like(x), torch.full_like(x, float("nan"))
        X.xdg_apply_with_config(H.handle, x, y0, grid=1024, occ=-1, xr=0)
        X.xdg_apply_with_config(H.handle, x, y1, grid=1024, occ=-1, xr=1)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), dt
        del x, y0, y1


def test_c3_sampled_rows(X):
    """6x6 J1-J2, Gamma A1: 1e5 random rows against the oracle (FP64 and FP32)."""
    m, b, H = built(X, "square36_j1j2_A1")
    check_keyed_rows(X, m, b, H, 43, 100_000)


def test_c3_fp32_ground_state(X):
    """FP32 vectors with FP64 reorthogonalisation against FP64, same start
    vector, 200 iterations: |dE0| / |E0| <= 1e-7."""
    m, b, H = built(X, "square36_j1j2_A1")
    e = {}
    for prec in (X.XDG_PREC_F32VEC_REORTH, X.XDG_PREC_F64, X.XDG_PREC_F64_REORTH):
        st, ev, al, be = H.lanczos(k=1, tol=0.0, max_iter=200, seed=3, prec=prec)
        assert len(al) == 200
        e[prec] = ev[0]
    print("C3 E0", e, flush=True)
    ref = e[X.XDG_PREC_F64]
    assert abs(e[X.XDG_PREC_F32VEC_REORTH] - ref) <= 1e-7 * abs(ref), e
    assert abs(e[X.XDG_PREC_F64_REORTH] - ref) <= 1e-9 * abs(ref), e


def test_c3_ferromagnetic_bound(X):
    m, b, _ = built(X, "square36_j1j2_A1")
    Hn = X.Hamiltonian(b, m.sites, -m.jz, -m.jxy)
    st, ev, al, be = Hn.lanczos(k=1, tol=1e-13, max_iter=300, seed=5, prec=0)
    assert abs(-ev[0] - m.jz.sum() / 4.0) < 1e-9
    assert m.jz.sum() / 4.0 == 27.0


def test_c4_batched_equals_single_fullsize(X):
    ms = [W.workload("chain32_allk")[l] for l in (0, 5, 16)]
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    xs = [torch.randn(b.dim, 2, dtype=torch.complex64, device="cuda") for b in bs]
    ys = [torch.empty_like(x) for x in xs]
    X.xdg_apply_batched([h.handle for h in hs], xs, ys)
    for h, x, y in zip(hs, xs, ys):
        r = torch.empty_like(x)
        h.apply(x, r)
        torch.cuda.synchronize()
        assert torch.equal(r, y)
    assert [b.dim for b in bs] == [dimension_formula(m) for m in ms]


def test_c5_fullsize(X):
    m, b, H = built(X, "tilted40_xxz")
    assert b.dim == dimension_formula(m) == 861602748
    check_windows(m, b, 50, n_windows=2, width=400)
    check_membership(X, m, b, 51, n_members=600, n_random=600)
    check_columns(X, m, b, H, 52, 2, [(torch.float64, 1e-12)])
    check_hermitian(b, H, 53, fp32=False)
    check_rank_addressed(X, b, H, 55)


def test_c5_sampled_rows(X):
    """40-site tilted XXZ, T x C4: 1e5 random rows against the oracle."""
    m, b, H = built(X, "tilted40_xxz")
    check_keyed_rows(X, m, b, H, 54, 100_000)


@pytest.mark.timeout(1200)
def test_c5_fp32_ground_state(X):
    """FP32 vectors (FP64 scalars) against FP64, same start vector, 100
    iterations: |dE0| / |E0| <= 1e-7."""
    m, b, H = built(X, "tilted40_xxz")
    e = {}
    for prec in (X.XDG_PREC_F32VEC, X.XDG_PREC_F64):
        print(f"C5 Lanczos prec {prec}", flush=True)
        st, ev, al, be = H.lanczos(k=1, tol=0.0, max_iter=100, seed=5, prec=prec)
        assert len(al) == 100
        e[prec] = ev[0]
    print("C5 E0", e, flush=True)
    ref = e[X.XDG_PREC_F64]
    assert abs(e[X.XDG_PREC_F32VEC] - ref) <= 1e-7 * abs(ref), e


@pytest.mark.timeout(1200)
def test_c4_batched_fp32_ground_states(X):
    """All 32 momenta x 8 vectors in the batched FP32 form (100 iterations):
    per sector the lowest Ritz value against the sector's own single-vector
    FP64 run (|dE0| / |E0| <= 1e-7), and k = 0 and pi against the Bethe
    ansatz."""
    from test_oracle_pins import bethe_energy
    _built.clear()
    torch.cuda.empty_cache()
    ms = W.workload("chain32_allk")
    bs = [X.Basis.from_model(m) for m in ms]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, ms)]
    print("C4 batched FP32 Lanczos", flush=True)
    ev, _, _ = X.xdg_lanczos_eigval_batched([h.handle for h in hs], nvec=8, n_iter=100, seed=4,
                                            prec=X.XDG_PREC_F32VEC)
    e_b = ev.min(axis=1)
    torch.cuda.empty_cache()
    e64 = []
    for l, h in enumerate(hs):
        st, e, al, be = h.lanczos(k=1, tol=0.0, max_iter=100, seed=400 + l, prec=X.XDG_PREC_F64)
        e64.append(e[0])
    e64 = np.array(e64)
    print("C4 E0 batched FP32", e_b.tolist(), "FP64", e64.tolist(), flush=True)
    rel = np.abs(e_b - e64) / np.abs(e64)
    assert np.all(rel <= 1e-7), (int(np.argmax(rel)), rel.max())
    for l, M in ((0, 16), (16, 15)):
        exact = bethe_energy(32, M)
        assert abs(e64[l] - exact) <= 1e-10 * abs(exact), (l, e64[l], exact)
        assert abs(e_b[l] - exact) <= 1e-7 * abs(exact), (l, e_b[l], exact)
    # k and -k have the same spectrum (to the convergence of 100 iterations
    # from different start vectors: a few 1e-9 relative in the slowest sectors)
    assert np.max(np.abs(e64[1:16] - e64[31:16:-1])) <= 1e-8 * np.max(np.abs(e64))
    del hs, bs
    torch.cuda.empty_cache()


def test_c2_ground_state_correlations(X):
    """Second Lanczos pass at full size (k = 0 sector, FP64): the sum rule
    sum_j <S^z_0 S^z_j> = 0 at Sz = 0 and, for the singlet ground state,
    <S^z_0 S^z_1> = E0 / (3N) with E0 from the Bethe ansatz."""
    from test_oracle_pins import bethe_energy
    m, b, H = built(X, "chain32_k0_kpi", 0)
    e, psi, al, be = H.eig0(tol=0.0, max_iter=200, seed=2, prec=0)
    e_bethe = bethe_energy(32, 16)
    assert abs(e - e_bethe) < 1e-12 * abs(e_bethe)
    c = X.xdg_expect_szsz(b.handle, psi, [(0, j) for j in range(32)])
    assert abs(c[0] - 0.25) < 1e-12
    assert abs(c.sum()) < 1e-11
    assert abs(c[1] - e_bethe / 96.0) < 1e-6, (c[1], e_bethe / 96.0)
    assert np.max(np.abs(c[1:] - c[1:][::-1])) < 1e-6
