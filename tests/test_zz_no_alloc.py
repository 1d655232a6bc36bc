"""The allocation-free batched apply (xdg_apply_batched_noalloc) against the
allocating one (xdg_apply_batched), through the C ABI: the same kernels, so
the outputs must be bitwise equal.  Two calls in a row, the second with a
smaller input (fewer and smaller blocks) on another stream, so that the
shared scratch array is rewritten; and the refusal beyond its limit."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def X():
    import paper_2505_02901_amd as X
    X.lib()
    return X


def blocks(X, models, nvec, dt, seed):
    bs = [X.Basis.from_model(m) for m in models]
    hs = [X.Hamiltonian.from_model(b, m) for b, m in zip(bs, models)]
    g = torch.Generator(device="cuda").manual_seed(seed)
    xs = [torch.randn(b.dim, nvec, dtype=dt, device="cuda", generator=g) for b in bs]
    return bs, hs, xs


def check_equal(X, hs, xs, stream=None):
    handles = [h.handle for h in hs]
    ref = [torch.empty_like(x) for x in xs]
    got = [torch.full_like(x, float("nan")) for x in xs]
    X.xdg_apply_batched(handles, xs, ref, stream=stream)
    X.xdg_apply_batched_noalloc(handles, xs, got, stream=stream)
    torch.cuda.synchronize()
    for i, (r, g) in enumerate(zip(ref, got)):
        assert torch.equal(r, g), i
        assert torch.isfinite(g).all()


def test_noalloc_equals_batched_on_two_calls(X):
    # call 1: five complex momentum sectors of the N = 20 ring (two fill
    # launches of descriptors), three complex FP32 vectors each
    ms1 = [W.chain_model(20, l=l) for l in (0, 3, 7, 10, 13)]
    bs1, hs1, xs1 = blocks(X, ms1, 3, torch.complex64, 1)
    print("no-alloc call 1:", [b.dim for b in bs1], flush=True)
    check_equal(X, hs1, xs1)
    # call 2, smaller: two sectors of the N = 14 ring, FP64 complex, one
    # vector, on a stream of its own
    ms2 = [W.chain_model(14, l=l) for l in (1, 7)]
    bs2, hs2, xs2 = blocks(X, ms2, 1, torch.complex128, 2)
    print("no-alloc call 2:", [b.dim for b in bs2], flush=True)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        check_equal(X, hs2, xs2, stream=st)
    st.synchronize()
    # and a sublattice-coded block (4x4 J1-J2 torus, Gamma A1), real FP32
    m3 = [W.torus_model((4, 0), (0, 4), 1.0, 0.5, "A1")]
    bs3, hs3, xs3 = blocks(X, m3, 2, torch.float32, 3)
    check_equal(X, hs3, xs3)


def test_noalloc_refuses_more_blocks_than_its_array_holds(X):
    m = W.chain_model(10, l=0)
    b = X.Basis.from_model(m)
    h = X.Hamiltonian.from_model(b, m)
    x = torch.zeros(b.dim, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(X.XdgError) as e:
        X.xdg_apply_batched_noalloc([h.handle] * 129, [x] * 129, [y] * 129)
    assert e.value.code == X.XDG_EINVAL
    X.xdg_apply_batched_noalloc([h.handle] * 3, [x] * 3, [y] * 3)   # within the limit
    torch.cuda.synchronize()


def test_noalloc_replays_from_a_captured_graph(X):
    """Allocating nothing, the call can be captured into a graph: every replay
    (with other work and a clobbered output in between) gives the eager y."""
    ms = [W.chain_model(16, l=l) for l in (0, 5, 11)]
    bs, hs, xs = blocks(X, ms, 2, torch.complex64, 7)
    handles = [h.handle for h in hs]
    ys = [torch.empty_like(x) for x in xs]
    X.xdg_apply_batched_noalloc(handles, xs, ys)      # eager (takes the array's address)
    torch.cuda.synchronize()
    ref = [y.clone() for y in ys]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        X.xdg_apply_batched_noalloc(handles, xs, ys, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        X.xdg_apply_batched_noalloc(handles, xs, ys, stream=torch.cuda.current_stream())
    for rep in range(4):
        for y in ys:
            y.fill_(float("nan"))
        z = torch.randn(1 << 16, device="cuda").sum()      # other eager work
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (y, r) in enumerate(zip(ys, ref)):
            assert torch.equal(y, r), (rep, i)
        del z
