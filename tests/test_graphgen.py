"""Generator checks: CSR well-formedness, determinism per seed, realised
shape (average degree, k-core property, connectivity)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen as gg


def well_formed(g):
    rp, col, w = g.row_ptr, g.col, g.w
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size == w.size
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col >= 0) and np.all(col < g.n) and not np.any(col == rows)
    assert np.all(w >= 1)
    # strictly increasing columns within each row
    d = np.diff(col)
    same_row = rows[1:] == rows[:-1]
    assert np.all(d[same_row] > 0)
    A = sp.csr_matrix((w.astype(np.int64), col, rp), shape=(g.n, g.n), copy=True)
    assert (A != A.T).nnz == 0
    assert w.astype(np.int64).sum() // 2 <= 2**31 - 1


def test_planted_shape_and_determinism():
    a = gg.planted(2000, 32.0, 5, 1, 1, seed=0)
    b = gg.planted(2000, 32.0, 5, 1, 1, seed=0)
    c = gg.planted(2000, 32.0, 5, 1, 1, seed=1)
    well_formed(a)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)
    assert not np.array_equal(a.col, c.col)
    assert a.m == 2 * 16000 + 5  # round(1000*32/2) per block + 5 cross pairs
    assert connected_components(sp.csr_matrix((a.w, a.col, a.row_ptr), copy=True), directed=False)[0] == 1


def test_planted_weights_range():
    g = gg.planted(500, 9.5, 7, 1, 100, seed=4)
    well_formed(g)
    assert g.w.min() >= 1 and g.w.max() <= 100 and g.w.max() > 50


@pytest.mark.parametrize("n", [64, 65, 3])
def test_planted_small(n):
    g = gg.planted(n, 8.0, 2, 1, 3, seed=n)
    well_formed(g)


def test_rhg_degree_and_determinism():
    a = gg.rhg(1 << 14, 32.0, 5.0, seed=3)
    b = gg.rhg(1 << 14, 32.0, 5.0, seed=3)
    well_formed(a)
    assert np.array_equal(a.col, b.col)
    assert abs(a.info["avg_deg"] - 32.0) <= 0.32
    assert connected_components(sp.csr_matrix((a.w, a.col, a.row_ptr), copy=True), directed=False)[0] == 1


def test_rhg_weighted():
    g = gg.rhg(5000, 20.0, 5.0, seed=2, wlo=1, whi=100)
    well_formed(g)
    assert g.w.max() > 50


def test_rmat_core_small():
    g = gg.rmat_core(14, 16, seed=2, kcore=10)
    well_formed(g)
    assert np.all(np.diff(g.row_ptr) >= 10)  # 10-core on distinct neighbours
    assert connected_components(sp.csr_matrix((g.w, g.col, g.row_ptr), copy=True), directed=False)[0] == 1
    assert g.w.max() > 1  # duplicates merged into weights


def test_from_edges_merges_duplicates():
    g = gg.from_edges(3, [(0, 1), (1, 0), (1, 2)], [2, 3, 4])
    well_formed(g)
    assert g.col.tolist() == [1, 0, 2, 1] and g.w.tolist() == [5, 5, 4, 4]


def test_c4_params_ranges():
    ps = gg.c4_params(4096, 3)
    ns = np.array([p[0] for p in ps])
    assert ns.min() >= 64 and ns.max() <= 8192
    assert all(8.0 <= p[1] <= 64.0 and 1 <= p[2] <= 20 for p in ps)


@pytest.mark.parametrize("n,d,k", [(300, 20.0, 4), (500, 5.0, 3), (120, 100.0, 5)])
def test_clustered_er_shape(n, d, k):
    """Density d % (binomial edge count within 5 sigma), weights in [1, 100]
    between clusters and in [n, 100 n] inside them, k balanced clusters
    (the components of the heavy edges at full density), determinism."""
    g = gg.clustered_er(n, d, k, seed=7)
    well_formed(g)
    assert np.array_equal(g.col, gg.clustered_er(n, d, k, seed=7).col)
    pairs = n * (n - 1) / 2
    m = g.nnz // 2
    p = d / 100.0
    assert abs(m - pairs * p) <= 5 * np.sqrt(pairs * p * (1 - p)) + 1
    heavy = g.w >= n
    assert np.all((g.w[~heavy] >= 1) & (g.w[~heavy] <= 100))
    assert np.all((g.w[heavy] >= n) & (g.w[heavy] <= 100 * n) & (g.w[heavy] % n == 0))
    if d == 100.0:
        rows = np.repeat(np.arange(n), np.diff(g.row_ptr))
        A = sp.csr_matrix((np.ones(heavy.sum()), (rows[heavy], g.col[heavy])), shape=(n, n))
        nc, lab = connected_components(A, directed=False)
        assert nc == k
        sizes = np.bincount(lab)
        assert sizes.max() - sizes.min() <= 1
