"""Pins for the oracle on directed graphs (Sec. 2.1: dangling vertices, P' and
P'', the PageRank definition eq. 2.1).  CPU only."""
from fractions import Fraction

import numpy as np

import graphgen as gg
import oracle

C = 0.85


def _graph(n, edges):
    """CSR by targets: row u lists the sources v of the edges v -> u."""
    rows = [[] for _ in range(n)]
    for v, u in edges:
        rows[u].append(v)
    rp = np.zeros(n + 1, dtype=np.int32)
    ci = []
    for u in range(n):
        rp[u + 1] = rp[u] + len(rows[u])
        ci.extend(sorted(rows[u]))
    return gg.CSR(n=n, row_ptr=rp, col_idx=np.asarray(ci, dtype=np.int32))


def check_first_step_by_hand(power):
    """Edges 0->1, 0->2, 1->2; vertex 2 dangling.  From the uniform x_0:
    P x_0 = (0, x0/2, x0/2 + x1), d^T x_0 = x2, so
    x_1 = c (P x_0 + x2 p) + (1-c) p, in exact rationals."""
    g = _graph(3, [(0, 1), (0, 2), (1, 2)])
    c = Fraction(17, 20)
    t = Fraction(1, 3)
    px = [Fraction(0), t / 2, t / 2 + t]
    want = [c * (px[i] + t * t) + (1 - c) * t for i in range(3)]
    x1 = power(g, np.full(3, 1.0 / 3.0), float(c), 1)
    assert np.allclose(x1, [float(w) for w in want], rtol=0, atol=1e-15)


def test_first_step_by_hand():
    check_first_step_by_hand(oracle.power_method_directed)


def test_iterates_are_distributions_and_reach_the_dense_solve():
    g = gg.directed_random(400, 5, 0.15, seed=2)
    rng = np.random.default_rng(1)
    p = rng.random(g.n)
    p /= p.sum()
    pi = oracle.pagerank_directed_exact(g, p, C)
    P, d = oracle.transition_directed(g)
    # eq. 2.1: pi = P'' pi with sum 1
    Ppp = C * (P.toarray() + np.outer(p, d)) + (1 - C) * np.outer(p, np.ones(g.n))
    assert np.abs(Ppp @ pi - pi).max() < 1e-15 and abs(pi.sum() - 1) < 1e-13
    e0 = np.abs(p - pi).sum()
    seq = oracle.power_method_directed(g, p, C, 250, return_all=True)
    for t, x in enumerate(seq):
        assert abs(x.sum() - 1.0) < 1e-13
        if t in (1, 7, 30):
            assert np.abs(x - pi).sum() <= C**t * e0 * (1 + 1e-12) + 1e-15
    assert np.abs(seq[-1] - pi).sum() < 1e-13


def test_undirected_input_is_the_undirected_pagerank():
    g = gg.random_connected(300, 5, seed=3)      # symmetric: no dangling vertex, P' = P
    p = gg.source_personalization(g.n, [11])[0]
    assert np.abs(oracle.pagerank_directed_exact(g, p, C) - oracle.pagerank_exact(g, p, C)).max() \
        < 1e-14
    assert np.abs(oracle.power_method_directed(g, p, C, 9) - oracle.power_method(g, p, C, 9)).max() \
        < 1e-15


def test_mutation_dropped_dangling_mass_is_caught():
    """A planted mistake: P x without the dangling term p d^T x."""
    def wrong(g, p, c, t):
        P, _ = oracle.transition_directed(g)
        x = np.asarray(p, dtype=float).copy()
        for _ in range(t):
            x = c * (P @ x) + (1 - c) * p * x.sum()
        return x
    try:
        check_first_step_by_hand(wrong)
    except AssertionError:
        return
    raise AssertionError("mutation not caught")


def test_directed_cycle_closed_form():
    """Directed cycle 0 -> 1 -> ... -> n-1 -> 0 (every out-degree 1, nothing
    dangling), p = e_0: the walk restarts at 0 with probability 1-c per step,
    so vertex k (k steps ahead) has pi_k = (1-c) c^k / (1 - c^n)."""
    n = 7
    g = _graph(n, [(v, (v + 1) % n) for v in range(n)])
    p = np.zeros(n)
    p[0] = 1.0
    want = (1 - C) * C ** np.arange(n) / (1 - C ** n)
    assert np.abs(oracle.pagerank_directed_exact(g, p, C) - want).max() < 1e-15
    x = oracle.power_method_directed(g, p, C, 400)
    assert np.abs(x - want).max() < 1e-15


def test_graph_without_edges_returns_p():
    """Every vertex dangling: P' = p e^T, so (I - cP')pi = (1-c)p gives pi = p."""
    n = 5
    g = _graph(n, [])
    p = np.array([0.1, 0.4, 0.2, 0.0, 0.3])
    assert np.abs(oracle.pagerank_directed_exact(g, p, C) - p).max() < 1e-15
    assert np.abs(oracle.power_method_directed(g, p, C, 3) - p).max() < 1e-15
