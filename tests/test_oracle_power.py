"""Pins for the oracle's power method (the comparison method of Sec. 5, eq. 2.1
iterated from p) and for the Delaunay stand-in graph.  CPU only."""
from fractions import Fraction

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import graphgen as gg
import oracle

C = 0.85


def check_first_steps_by_hand(pm):
    """Path 0-1-2, uniform p: P p = (p_1/2, p_0 + p_2, p_1/2) = (1/6, 2/3, 1/6),
    so x_1 = c (1/6, 2/3, 1/6) + (1-c)(1/3, 1/3, 1/3), in exact rationals."""
    g = gg.path(3)
    c = Fraction(17, 20)
    third = Fraction(1, 3)
    want = [c * Fraction(1, 6) + (1 - c) * third, c * Fraction(2, 3) + (1 - c) * third,
            c * Fraction(1, 6) + (1 - c) * third]
    x1 = pm(g, np.full(3, 1.0 / 3.0), float(c), 1)
    assert np.allclose(x1, [float(w) for w in want], rtol=0, atol=1e-16)
    # and a second step from that vector
    x2 = [c * (want[1] / 2) + (1 - c) * third, c * (want[0] + want[2]) + (1 - c) * third,
          c * (want[1] / 2) + (1 - c) * third]
    assert np.allclose(pm(g, np.full(3, 1.0 / 3.0), float(c), 2),
                       [float(w) for w in x2], rtol=0, atol=1e-16)


def test_power_method_first_steps_by_hand():
    check_first_steps_by_hand(oracle.power_method)


def test_power_method_iterates_stay_distributions():
    """P is column-stochastic and p sums to 1, so every iterate sums to 1."""
    g = gg.random_connected(300, 5, seed=11)
    rng = np.random.default_rng(3)
    p = rng.random(g.n)
    p /= p.sum()
    for x in oracle.power_method(g, p, C, 30, return_all=True):
        assert abs(x.sum() - 1.0) < 1e-13
        assert x.min() > 0


def test_power_method_fixed_point_on_regular_graphs():
    """On a regular graph P e/n = e/n, so the uniform p is PageRank and every
    iterate from it equals it."""
    for g in (gg.cycle(7), gg.complete(6)):
        p = np.full(g.n, 1.0 / g.n)
        for x in oracle.power_method(g, p, C, 10, return_all=True):
            assert np.allclose(x, p, rtol=0, atol=1e-16)


def check_contraction(pm):
    """x_t - pi = (cP)^t (p - pi) and ||P||_1 = 1, so ||x_t - pi||_1 <= c^t ||p - pi||_1;
    pi from a dense LU solve."""
    g = gg.chung_lu(400, 6, 2.3, seed=5)
    p = gg.source_personalization(g.n, [7])[0]
    pi = oracle.pagerank_exact(g, p, C)
    e0 = np.abs(p - pi).sum()
    seq = pm(g, p, C, 250, return_all=True)
    for t in (1, 5, 20, 60):
        assert np.abs(seq[t] - pi).sum() <= C**t * e0 * (1 + 1e-12) + 1e-15
    assert np.abs(seq[-1] - pi).sum() < 1e-13


def test_power_method_contracts_to_the_dense_solution():
    check_contraction(oracle.power_method)


def test_delaunay_standin_is_a_planar_triangulation():
    """Symmetric pattern without self-loops; a planar graph has at most 3n - 6
    edges, and a triangulation of random points has almost exactly that many."""
    g = gg.delaunay(2000, seed=1)
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    assert (A != A.T).nnz == 0 and A.diagonal().sum() == 0
    edges = g.nnz // 2
    assert 2.9 * g.n < edges <= 3 * g.n - 6


def test_table3_iteration_counts_on_delaunay_standin():
    """Table 3, delaunay-n21 row: CPAA reaches ERR < 1e-3 (max relative error,
    Sec. 5) in 12 rounds.  On a smaller Delaunay graph of the same construction
    the oracle's CPAA needs exactly 12 too.  The power method from p needs more
    (14 here; the paper reports 20, see the design notes)."""
    g = gg.delaunay(1 << 12, seed=2112010)
    p = np.full(g.n, 1.0 / g.n)
    P = oracle.transition_matrix(g)
    pi = spl.spsolve((sp.eye(g.n) - C * P).tocsc(), (1.0 - C) * p)
    b = (1.0 - C) * p
    k_cpaa = next(M for M in range(1, 40)
                  if oracle.max_relative_error(oracle.cpaa(g, b, C, M), pi) < 1e-3)
    seq = oracle.power_method(g, p, C, 60, return_all=True)
    k_power = next(t for t, x in enumerate(seq) if oracle.max_relative_error(x, pi) < 1e-3)
    assert k_cpaa == 12
    assert k_power == 14


# ----------------------------------------------------------------------------
# planted mistakes in the power method must fail a pin
# ----------------------------------------------------------------------------

def _mutant(step=None, start=None, steps_off=0):
    def pm(g, p, c, t, return_all=False):
        P = oracle.transition_matrix(g)
        p = np.asarray(p, dtype=np.float64)
        x = start(p, c) if start else p.copy()
        seq = [x]
        for _ in range(max(t + steps_off, 0)):
            x = step(P, x, p, c) if step else c * (P @ x) + (1.0 - c) * p * x.sum(axis=0)
            seq.append(x)
        return seq if return_all else x
    return pm


def _fails(check, pm):
    try:
        check(pm)
    except AssertionError:
        return True
    return False


def test_unmutated_copy_passes_the_pins():
    assert not _fails(check_first_steps_by_hand, _mutant())
    assert not _fails(check_contraction, _mutant())


def test_mutation_transposed_transition_is_caught():
    m = _mutant(step=lambda P, x, p, c: c * (P.T @ x) + (1 - c) * p * x.sum())
    assert _fails(check_first_steps_by_hand, m)


def test_mutation_teleport_weight_swapped_is_caught():
    m = _mutant(step=lambda P, x, p, c: (1 - c) * (P @ x) + c * p * x.sum())
    assert _fails(check_first_steps_by_hand, m) and _fails(check_contraction, m)


def test_mutation_neumann_start_is_caught():
    m = _mutant(start=lambda p, c: (1 - c) * p)
    assert _fails(check_first_steps_by_hand, m)


def test_mutation_one_step_short_is_caught():
    m = _mutant(steps_off=-1)
    assert _fails(check_first_steps_by_hand, m)
