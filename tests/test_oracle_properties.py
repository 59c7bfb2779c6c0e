"""Property-based pins for the oracle on random small graphs (hypothesis,
derandomized): CPAA and the power method converge to the dense solve, PageRank
sums to 1, the reversibility identity of undirected graphs holds, and on
directed graphs the power method converges to the fixed point of P'' with the
error bound c^t ||x_0 - pi||_1.  CPU only."""
import numpy as np
import pytest

pytest.importorskip("hypothesis")
from hypothesis import given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

import oracle  # noqa: E402
from strategies import directed_graphs, graphs  # noqa: E402


@settings(max_examples=80, deadline=None, derandomize=True, database=None)
@given(g=graphs(), c=st.floats(0.05, 0.9))
def test_series_and_power_method_reach_the_dense_solve(g, c):
    p = np.full(g.n, 1.0 / g.n)
    pi = oracle.pagerank_exact(g, p, c)
    assert abs(pi.sum() - 1.0) < 1e-12 and pi.min() > 0
    M = oracle.terms_for_mass_error(c, 1e-13) + 10
    assert np.abs(oracle.cpaa(g, (1 - c) * p, c, M) - pi).sum() < 1e-11
    t = int(np.ceil(np.log(1e-14) / np.log(c)))
    assert np.abs(oracle.power_method(g, p, c, t) - pi).sum() < 1e-11


@settings(max_examples=80, deadline=None, derandomize=True, database=None)
@given(g=graphs(), c=st.floats(0.05, 0.9), s=st.integers(0, 10**6), t=st.integers(0, 10**6))
def test_reversibility(g, c, s, t):
    """d_s pi_s(t) = d_t pi_t(s) for personalized PageRank on an undirected graph:
    pi_s(t) = (1-c) d_t [(D - cA)^{-1}]_{ts} and D - cA is symmetric."""
    s, t = s % g.n, t % g.n
    P = np.zeros((g.n, 2))
    P[s, 0] = 1.0
    P[t, 1] = 1.0
    pi = oracle.pagerank_exact(g, P, c)
    d = np.diff(g.row_ptr).astype(float)
    assert abs(d[s] * pi[t, 0] - d[t] * pi[s, 1]) < 1e-13 * max(1.0, d[s] * pi[t, 0])


@settings(max_examples=80, deadline=None, derandomize=True, database=None)
@given(g=directed_graphs(), c=st.floats(0.05, 0.9), seed=st.integers(0, 2**31 - 1))
def test_directed_power_method_contracts_to_the_fixed_point(g, c, seed):
    """Sec. 2.1 / eq. 2.1: pi = P'' pi with sum 1 and pi >= 0; P' is column
    stochastic, so ||x_t - pi||_1 <= c^t ||p - pi||_1 for the iteration from p."""
    rng = np.random.default_rng(seed)
    p = rng.random(g.n) + 1e-3
    p /= p.sum()
    pi = oracle.pagerank_directed_exact(g, p, c)
    assert abs(pi.sum() - 1.0) < 1e-12 and pi.min() > -1e-15
    P, d = oracle.transition_directed(g)
    Ppp = c * (P.toarray() + np.outer(p, d)) + (1 - c) * np.outer(p, np.ones(g.n))
    assert np.abs(Ppp @ pi - pi).max() < 1e-13
    e0 = np.abs(p - pi).sum()
    seq = oracle.power_method_directed(g, p, c, 12, return_all=True)
    for t, x in enumerate(seq):
        assert np.abs(x - pi).sum() <= c**t * e0 * (1 + 1e-10) + 1e-14
