"""Statistics of the seeded synthetic workloads."""
import numpy as np

from workloads import generators as G


def _check_csr(c):
    rp, ci = c.rowptr, c.colind
    assert rp.dtype == np.int32 and ci.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == c.nnz
    for j in range(c.n):
        seg = ci[rp[j]:rp[j + 1]]
        assert np.all(np.diff(seg) > 0)
        assert j in seg
    A = c.to_scipy()
    assert abs(A - A.T).max() == 0.0


def test_banded_config():
    c = G.make_config(1)
    assert c.n == 1024 and c.nnz == 17336
    m = c.row_sizes()
    assert m.min() == 9 and m.max() == 17 and np.sum(m == 17) == 1024 - 16
    _check_csr(c)
    w = np.linalg.eigvalsh(c.dense())
    assert w[0] >= 1.0 - 1e-12 and w[-1] <= 1 + 2 * 8 * 0.3 + 1e-12


def test_overlap_small_reproducible_and_conditioned():
    a = G.overlap_matrix(n_atoms=64, density=0.1, nbf=13, rcut=4.14, kappa=100.0, seed=5)
    b = G.overlap_matrix(n_atoms=64, density=0.1, nbf=13, rcut=4.14, kappa=100.0, seed=5)
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.colind, b.colind)
    _check_csr(a)
    w = np.linalg.eigvalsh(a.dense())
    assert abs(w[-1] / w[0] - 100.0) < 1e-6 * 100
    # 13 columns of an atom share one row set
    m = a.row_sizes()
    assert np.all(m % 13 == 0)


def test_overlap_config2_shape():
    c = G.make_config(2)
    m = c.row_sizes()
    assert c.n == 6656
    assert 380 <= m.mean() <= 410
    assert abs(c.meta["lmax"] / c.meta["lmin"] - 100.0) < 1e-3


def test_special_cases():
    for c in (G.diagonal_spd(20), G.block_diagonal_spd((2, 3)), G.dense_spd(10),
              G.random_sparse_spd(40, 0.1), G.arrowhead_spd(12), G.explicit_zero_pattern()):
        _check_csr(c)


def test_dense_with_spectrum_has_that_spectrum():
    eigs = np.concatenate([np.full(5, 1.0), np.full(3, 2.5), np.linspace(3.0, 4.0, 4)])
    c = G.dense_with_spectrum(eigs)
    a = c.dense()
    assert np.array_equal(a, a.T)
    assert np.allclose(np.linalg.eigvalsh(a), np.sort(eigs), atol=1e-13)
    assert c.nnz == 144


def test_lanczos_shift_is_reproducible():
    """Above the dense-eigensolver size the extremes come from Lanczos with a
    seeded start vector, so generating a workload twice gives the same bits
    (the shift lands on every diagonal entry)."""
    a = G.make_config(2)
    b = G.make_config(2)
    assert a.n > 3000
    assert np.array_equal(a.vals, b.vals) and a.meta["sigma"] == b.meta["sigma"]
    assert abs(a.meta["lmax"] / a.meta["lmin"] - 1e2) <= 1e-8 * 1e2


def test_cached_extremes_match_lanczos_on_a_smaller_matrix():
    """The cached-extremes path of shift_to_kappa places the same shift as
    computing the extremes (checked where Lanczos is cheap)."""
    csr = G.overlap_matrix(n_atoms=300, nbf=13, rcut=4.14, kappa=None, seed=5)
    ext = G.extreme_eigenvalues(csr)
    a = G.shift_to_kappa(csr, 1e4)
    b = G.shift_to_kappa(csr, 1e4, ext)
    assert abs(a.meta["sigma"] - b.meta["sigma"]) <= 1e-9 * abs(b.meta["sigma"])
    assert abs(b.meta["lmax"] / b.meta["lmin"] - 1e4) <= 1e-6 * 1e4

