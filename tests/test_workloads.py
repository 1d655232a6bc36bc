"""The seeded input generators (CPU): the state-keyed vector has one
definition, implemented twice (numpy for the oracle side, torch for building
device vectors); both must give the same bits."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("nvec,cplx", [(1, False), (1, True), (3, False), (2, True)])
def test_keyed_values_numpy_equals_torch(nvec, cplx):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(nvec + 2 * cplx)
    s = np.concatenate([rng.integers(0, 1 << 40, size=5000, dtype=np.uint64),
                        np.array([0, 1, (1 << 40) - 1], np.uint64)])
    a = W.keyed_values(5, s, nvec=nvec, complex_=cplx)
    b = W.keyed_values_torch(5, torch.from_numpy(s.view(np.int64)), nvec=nvec,
                             complex_=cplx).numpy()
    assert a.shape == b.shape
    assert np.array_equal(a, b)
    assert np.all(np.abs(a.real) <= 1.0) and np.all(np.abs(a.imag) <= 1.0)


def test_keyed_values_follow_the_seeded_stream():
    """Keyed by the states 0, 1, 2, ... the vector is the plain uniform stream
    (scalar q of the stream sits at state q)."""
    n = 1000
    a = W.keyed_values(7, np.arange(n, dtype=np.uint64))
    assert np.array_equal(a, W.random_scalars(7, n, kind="uniform"))
    c = W.keyed_values(7, np.arange(n, dtype=np.uint64), nvec=2, complex_=True)
    flat = W.random_scalars(7, 4 * n, kind="uniform")
    assert np.array_equal(c.view(np.float64).reshape(-1), flat)
