"""The seeded synthetic inputs (graphgen) have the structure their recipes
state: valid patterns (sorted columns, no self loops or duplicates, symmetric
where undirected), the stated degree bounds, block-diagonal batches, and the
same graph for the same seed.  CPU only, small sizes."""
import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg


def _pattern(g):
    rp = g.row_ptr.astype(np.int64)
    ci = g.col_idx.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == ci.shape[0] and np.all(np.diff(rp) >= 0)
    assert np.all((ci >= 0) & (ci < g.n))
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert not np.any(rows == ci), "self loop"
    # strictly increasing columns inside every row: sorted, no duplicates
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    return sp.csr_matrix((np.ones(ci.shape[0]), ci, rp), shape=(g.n, g.n))


def _undirected(g):
    A = _pattern(g)
    assert (A != A.T).nnz == 0, "not symmetric"
    assert np.diff(g.row_ptr).min() >= 1, "isolated vertex"
    return A


def test_csr_from_edges_merges_and_symmetrizes():
    g = gg.csr_from_edges(4, np.array([0, 1, 1, 2, 3, 3]), np.array([1, 0, 2, 2, 0, 1]))
    A = _pattern(g).toarray()
    want = np.zeros((4, 4))
    for a, b in ((0, 1), (1, 2), (0, 3), (1, 3)):
        want[a, b] = want[b, a] = 1
    assert np.array_equal(A, want)


def test_chung_lu_recipe():
    g = gg.chung_lu(20000, 16, 2.1, seed=7, dmin=1.0, dmax=500.0)
    _undirected(g)
    d = np.diff(g.row_ptr)
    assert g.n == 20000 and 12 <= d.mean() <= 17
    # expected degrees fall with the label and are capped at dmax; realized
    # degrees scatter around them (Poisson-like), so the checks are loose
    assert d[:50].mean() > 10 * d[-10000:].mean()
    assert d.max() < 1.3 * 500 and d.min() >= 1
    h = gg.chung_lu(20000, 16, 2.1, seed=7, dmin=1.0, dmax=500.0)
    assert np.array_equal(g.row_ptr, h.row_ptr) and np.array_equal(g.col_idx, h.col_idx)
    k = gg.chung_lu(20000, 16, 2.1, seed=8, dmin=1.0, dmax=500.0)
    assert not (np.array_equal(g.row_ptr, k.row_ptr) and np.array_equal(g.col_idx, k.col_idx))


def test_perturbed_grid_recipe():
    side = 60
    g = gg.perturbed_grid(side, 0.05, 0.01, seed=3)
    _undirected(g)
    d = np.diff(g.row_ptr)
    assert d.max() <= 5
    lattice_edges = 2 * side * (side - 1)
    edges = g.nnz // 2
    # ~95 % of the lattice edges kept, plus 1 % of them as shortcuts
    assert 0.9 * lattice_edges < edges < 1.02 * lattice_edges
    assert g.meta["shortcuts"] == round(0.01 * lattice_edges)


def test_delaunay_is_a_planar_triangulation():
    n = 3000
    g = gg.delaunay(n, seed=11)
    _undirected(g)
    edges = g.nnz // 2
    # a triangulation of n points with h hull vertices has 3n - 3 - h edges
    assert 2 * n < edges <= 3 * n - 6
    assert 5.5 < g.nnz / n < 6.0


def test_directed_random_recipe():
    n = 20000
    g = gg.directed_random(n, 16, 0.1, seed=5)
    A = _pattern(g)                      # row u lists the sources of v -> u
    dout = np.asarray(A.sum(axis=0)).ravel()
    dangling = int(np.sum(dout == 0))
    assert dangling == g.meta["dangling"]
    assert 0.08 * n < dangling < 0.12 * n
    assert 14 <= g.nnz / n <= 17
    assert (A != A.T).nnz > 0            # really directed


def test_uneven_batch_is_block_diagonal():
    g = gg.uneven_batch(40, seed=9, n_lo=50, n_hi=400)
    _undirected(g)
    gp = g.graph_ptr.astype(np.int64)
    assert gp[0] == 0 and gp[-1] == g.n and np.all(np.diff(gp) >= 2)
    owner = np.repeat(np.arange(gp.shape[0] - 1), np.diff(gp))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert np.array_equal(owner[rows], owner[g.col_idx]), "an edge crosses two graphs"
    assert np.diff(gp).max() <= 400


@pytest.mark.parametrize("sources", [[0], [3, 9]])
def test_personalizations_are_distributions(sources):
    P = gg.source_personalization(12, sources)
    assert np.allclose(P.sum(axis=1), 1.0) and P.min() >= 0
    assert abs(gg.uniform_personalization(12).sum() - 1.0) < 1e-15
