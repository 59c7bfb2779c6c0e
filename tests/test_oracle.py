"""Pins for the FP64 oracle: values the paper prints, closed forms, exact
rational arithmetic and invariants.  CPU only.

Each check is written as a plain function so the mutation tests at the end can
plant a mistake in the oracle (on the CPU) and show that some pin catches it.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import numpy.polynomial.chebyshev as npcheb
import pytest

import graphgen as gg
import oracle
import oracle.cpaa_ref as ocp

C = 0.85


# ----------------------------------------------------------------------------
# helpers independent of the oracle
# ----------------------------------------------------------------------------

def exact_pagerank_fractions(g, p, c):
    """(I - cP) x = (1-c) p solved by Gauss-Jordan elimination in exact rationals."""
    n = g.n
    rp, ci = g.row_ptr.tolist(), g.col_idx.tolist()
    deg = [rp[i + 1] - rp[i] for i in range(n)]
    c = Fraction(c).limit_denominator(10**6)
    M = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for i in range(n):               # row i of A: neighbours of vertex i
        for k in range(rp[i], rp[i + 1]):
            j = ci[k]
            M[i][j] -= c / deg[j]    # p_ij = a_ij / d_j
    rhs = [(1 - c) * Fraction(x).limit_denominator(10**9) for x in p]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        rhs[col], rhs[piv] = rhs[piv], rhs[col]
        inv = 1 / M[col][col]
        M[col] = [v * inv for v in M[col]]
        rhs[col] *= inv
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
                rhs[r] -= f * rhs[col]
    return rhs, c


def cycle_pagerank_closed_form(n, s, c):
    """PageRank personalized at s on the cycle C_n.

    P = (Z + Z^{-1})/2 is circulant; the Fourier coefficients of
    1/(1 - c cos t) are beta^{|d|}/sqrt(1-c^2), and periodizing gives
    pi_s(t) = (1-c)/sqrt(1-c^2) * (beta^d + beta^{n-d}) / (1 - beta^n), d = (t-s) mod n.
    """
    sq = math.sqrt(1 - c * c)
    b = (1 - sq) / c
    d = (np.arange(n) - s) % n
    return (1 - c) / sq * (b ** d + b ** (n - d)) / (1 - b ** n)


def complete_pagerank_closed_form(n, s, c):
    """K_n: P = (J - I)/(n-1) has eigenvalue 1 on e and -1/(n-1) on e-perp, so
    pi_s = e/n + (1-c)(n-1)/(n-1+c) (e_s - e/n)."""
    x = np.full(n, 1.0 / n)
    e_s = np.zeros(n)
    e_s[s] = 1.0
    return x + (1 - c) * (n - 1) / (n - 1 + c) * (e_s - 1.0 / n)


def small_graphs():
    return [gg.cycle(7), gg.path(6), gg.star(6), gg.complete(5),
            gg.random_connected(9, 3.0, seed=11), gg.random_connected(30, 4.0, seed=12),
            gg.random_connected(60, 6.0, seed=13)]


# ----------------------------------------------------------------------------
# checks (used directly and by the mutation tests)
# ----------------------------------------------------------------------------

def check_coefficients_vs_integral(o=ocp):
    for c in (0.3, 0.85, 0.95):
        ck = o.chebyshev_coefficients(c, 30)
        for k in range(31):
            ref = o.chebyshev_coefficient_integral(c, k)
            assert abs(ck[k] - ref) <= 1e-12 * max(1.0, abs(ref)), (c, k, ck[k], ref)


def check_series_converges_to_f(o=ocp):
    for c in (0.5, 0.85):
        x = np.linspace(-1, 1, 201)
        f = 1.0 / (1.0 - c * x)
        for M in (5, 12, 24, 40):
            ck = o.chebyshev_coefficients(c, M).copy()
            ck[0] /= 2.0               # numpy's chebval uses a_0 T_0 (not a_0/2)
            approx = npcheb.chebval(x, ck)
            err = np.max(np.abs(approx - f))
            assert err <= o.series_tail(c, M) * (1 + 1e-9) + 1e-14, (c, M, err)
            assert err >= 0.5 * o.series_tail(c, M)     # the tail is attained at x = 1


def check_dense_vs_fractions(o=ocp):
    for g in (gg.path(5), gg.star(5), gg.random_connected(6, 3.0, seed=5)):
        rng = gg.philox(7)
        p = rng.random(g.n)
        p /= p.sum()
        ref, cfrac = exact_pagerank_fractions(g, p, C)
        x = o.pagerank_exact(g, p, float(cfrac))
        assert np.max(np.abs(x - np.array([float(v) for v in ref]))) < 1e-14


def check_cycle(o=ocp):
    n, s = 11, 3
    p = np.zeros(n)
    p[s] = 1.0
    assert np.max(np.abs(o.pagerank_exact(gg.cycle(n), p, C)
                         - cycle_pagerank_closed_form(n, s, C))) < 1e-14
    # every Chebyshev term on a cycle: T_k(P) e_s = (e_{s+k} + e_{s-k}) / 2
    _, terms = o.cpaa(gg.cycle(n), p, C, 8, return_terms=True)
    for k, T in enumerate(terms):
        ref = np.zeros(n)
        ref[(s + k) % n] += 0.5
        ref[(s - k) % n] += 0.5
        assert np.max(np.abs(T - ref)) < 1e-14, k


def check_complete(o=ocp):
    n, s = 9, 4
    p = np.zeros(n)
    p[s] = 1.0
    assert np.max(np.abs(o.pagerank_exact(gg.complete(n), p, C)
                         - complete_pagerank_closed_form(n, s, C))) < 1e-14


def check_stationary(o=ocp):
    """p = d/vol is the stationary distribution of P = A D^{-1}: pi = p, and T_k(P)p = p."""
    g = gg.random_connected(40, 5.0, seed=21)
    d = np.diff(g.row_ptr).astype(float)
    p = d / d.sum()
    assert np.max(np.abs(o.pagerank_exact(g, p, C) - p)) < 1e-14
    assert np.max(np.abs(o.pagerank_power(g, p, C)[0] - p)) < 1e-14
    x = o.cpaa(g, (1 - C) * p, C, 40)
    assert np.max(np.abs(x / (1 - o.mass_error(C, 40)) - p)) < 1e-13


def check_cpaa_converges(o=ocp):
    for g in small_graphs():
        rng = gg.philox(99)
        p = rng.random(g.n)
        p /= p.sum()
        pi = o.pagerank_exact(g, p, C)
        b = (1 - C) * p
        deg = np.diff(g.row_ptr).astype(float)
        for M in (1, 2, 3, 5, 10, 20):
            x = o.cpaa(g, b, C, M)
            err = np.abs(x - pi).sum()
            assert err <= o.apriori_error_bound(deg, b, C, M) * (1 + 1e-9), (g.n, M)
            # the mass deficit is a lower bound on the L1 error and equals ERR_M
            assert abs((1 - x.sum()) - o.mass_error(C, M)) < 1e-13
            assert err >= o.mass_error(C, M) * (1 - 1e-9)
        x = o.cpaa(g, b, C, 70)
        assert np.abs(x - pi).sum() < 1e-13


def check_series_residual(o=ocp):
    g = gg.random_connected(50, 4.0, seed=31)
    rng = gg.philox(3)
    b = rng.standard_normal(g.n)
    for M in (0, 1, 2, 7, 15):
        x, terms = o.cpaa(g, b, C, M, return_terms=True)
        r = o.residual(g, b, x, C)
        r2 = o.series_residual(C, M, terms[M], terms[M + 1])
        assert np.max(np.abs(r - r2)) < 1e-13 * max(1.0, np.abs(b).max()), M


# ----------------------------------------------------------------------------
# direct tests
# ----------------------------------------------------------------------------

def test_coefficients_match_integral_definition():
    check_coefficients_vs_integral()


def test_coefficients_match_printed_closed_forms(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "paper_values.json")))
    assert "coefficients_printed" in gold
    for c in (0.2, 0.5, 0.85, 0.99):
        s = math.sqrt(1 - c * c)
        ck = ocp.chebyshev_coefficients(c, 5)
        assert ck[0] == pytest.approx(2 / s, rel=1e-15)
        assert ck[1] == pytest.approx(2 / c * (1 - s) / s, rel=1e-13)
        assert ck[2] == pytest.approx(2 / c**2 * (2 * (1 - s) - c * c) / s, rel=1e-12)
        for k in range(1, 6):
            assert ck[k - 1] / ck[k] == pytest.approx(c / (1 - s), rel=1e-14)
            if k < 5:   # c_{k-1} + c_{k+1} = (2/c) c_k (recurrence in Prop. 1's proof)
                assert ck[k - 1] + ck[k + 1] == pytest.approx(2 / c * ck[k], rel=1e-14)


def test_sigma_matches_paper(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "paper_values.json")))["sigma_c_at_0_85"]
    sig = ocp.convergence_rate(gold["c"])
    assert round(sig, gold["digits"]) == gold["value"]
    # sigma_c = 1 - c_k/B_k is the tail ratio, equal to beta (the coefficient ratio)
    assert sig == pytest.approx(ocp.beta(gold["c"]), rel=1e-13)
    for c in (0.1, 0.5, 0.9, 0.99):
        ck = ocp.chebyshev_coefficients(c, 400)
        for k in (1, 2, 10):
            B_k = ck[k:].sum()
            assert 1 - ck[k] / B_k == pytest.approx(ocp.convergence_rate(c), rel=1e-10)


def test_mass_error_formula_and_paper_claims(golden_dir):
    gold = json.load(open(os.path.join(golden_dir, "paper_values.json")))
    for M in range(0, 60):
        direct = 1 - ocp.accumulated_mass(C, M) / ocp.total_mass(C)
        assert ocp.mass_error(C, M) == pytest.approx(direct, rel=1e-9, abs=1e-15)
        # tail identity used by the a-priori bound: (1-c) sum_{k>M} c_k = ERR_M
        assert (1 - C) * ocp.series_tail(C, M) == pytest.approx(ocp.mass_error(C, M), rel=1e-12)
    e = gold["err_below_1e-4_within_rounds"]
    assert ocp.mass_error(C, e["value"]) < e["tol"]
    t = gold["cpaa_rounds_for_1e-3_mesh_graphs"]
    assert ocp.terms_for_mass_error(C, t["tol"]) == t["value"]


def test_series_converges_to_function():
    check_series_converges_to_f()


def test_dense_solve_matches_exact_rationals():
    check_dense_vs_fractions()


def test_dense_solve_matches_numpy_solve_of_definition():
    g = gg.random_connected(25, 4.0, seed=1)
    A = np.zeros((g.n, g.n))
    for i in range(g.n):
        A[i, g.col_idx[g.row_ptr[i]:g.row_ptr[i + 1]]] = 1.0
    P = A / A.sum(axis=0, keepdims=True)
    p = np.full(g.n, 1.0 / g.n)
    ref = (1 - C) * np.linalg.inv(np.eye(g.n) - C * P) @ p
    assert np.max(np.abs(ocp.pagerank_exact(g, p, C) - ref)) < 1e-14


def test_cycle_closed_forms():
    check_cycle()


def test_complete_closed_form():
    check_complete()


def test_regular_graph_uniform_is_uniform():
    for g in (gg.cycle(12), gg.complete(7)):
        p = np.full(g.n, 1.0 / g.n)
        assert np.max(np.abs(ocp.pagerank_exact(g, p, C) - p)) < 1e-15
        x = ocp.cpaa(g, (1 - C) * p, C, 60)
        assert np.max(np.abs(x - p)) < 1e-15


def test_stationary_distribution_is_fixed():
    check_stationary()


def test_power_method_matches_dense():
    for g in small_graphs():
        p = gg.source_personalization(g.n, [0, g.n - 1]).T
        x, it = ocp.pagerank_power(g, p, C, tol=1e-14)
        assert np.max(np.abs(x - ocp.pagerank_exact(g, p, C))) < 1e-14
        assert it < 250


def test_cpaa_converges_within_bounds():
    check_cpaa_converges()


def test_cpaa_matrix_rhs_equals_columnwise():
    g = gg.random_connected(30, 5.0, seed=8)
    B = gg.source_personalization(g.n, [1, 5, 29]).T * (1 - C)
    X = ocp.cpaa(g, B, C, 17)
    for j in range(3):
        assert np.max(np.abs(X[:, j] - ocp.cpaa(g, B[:, j], C, 17))) < 1e-16


def test_mass_invariant_every_term():
    """e^T T_k(P) b = e^T b for all k, since e^T P = e^T (Sec. 4.1, total mass constant)."""
    g = gg.random_connected(45, 5.0, seed=4)
    b = np.ones(g.n)
    x, terms = ocp.cpaa(g, b, C, 25, return_terms=True)
    for T in terms:
        assert T.sum() == pytest.approx(g.n, rel=1e-13)
    # accumulated mass after M rounds is S_M (Sec. 4.2.1)
    assert x.sum() == pytest.approx(ocp.accumulated_mass(C, 25, n=g.n), rel=1e-13)


def test_series_residual_identity():
    check_series_residual()


def test_residual_bound_is_an_upper_bound():
    g = gg.random_connected(40, 4.0, seed=17)
    p = gg.source_personalization(g.n, [3])[0]
    pi = ocp.pagerank_exact(g, p, C)
    for M in (3, 8, 15):
        x = ocp.cpaa(g, (1 - C) * p, C, M)
        assert np.abs(x - pi).sum() <= ocp.residual_l1_bound(g, (1 - C) * p, x, C) * (1 + 1e-12)


def test_reversibility():
    """d_s pi_s(t) = d_t pi_t(s) for undirected graphs, with pi_s personalized at s:
    (I - cAD^{-1})^{-1} = D (D - cA)^{-1} and (D - cA)^{-1} is symmetric."""
    g = gg.random_connected(35, 5.0, seed=23)
    d = np.diff(g.row_ptr).astype(float)
    Pi = ocp.pagerank_exact(g, np.eye(g.n), C)        # column s = pi_s
    lhs = d[None, :] * Pi                              # [t, s] -> d_s pi_s(t)
    assert np.max(np.abs(lhs - lhs.T)) < 1e-15
    # the same identity with the degrees swapped does not hold on a non-regular graph
    wrong = d[:, None] * Pi
    assert np.max(np.abs(wrong - wrong.T)) > 1e-3


def test_lemma2_real_spectrum_and_spd():
    for g in small_graphs():
        P = ocp.transition_dense(g)
        ev = np.linalg.eigvals(P)
        assert np.max(np.abs(ev.imag)) < 1e-10
        assert np.max(np.abs(ev)) <= 1 + 1e-12
        d = np.diff(g.row_ptr).astype(float)
        A = P * d[None, :]
        np.linalg.cholesky(np.diag(d) - C * A)       # raises if not positive definite


def test_normalized_alg1_matches_global_pagerank():
    g = gg.random_connected(50, 6.0, seed=41)
    pi = ocp.pagerank_exact(g, np.full(g.n, 1.0 / g.n), C)
    assert np.abs(ocp.cpaa_alg1_global(g, C, 60) - pi).sum() < 1e-13
    # normalization cancels the uniform mass deficit: after 12 rounds the
    # normalized result is much closer than the (1-c)-scaled one
    xn = ocp.cpaa_alg1_global(g, C, 12)
    xs = ocp.cpaa(g, (1 - C) * np.full(g.n, 1.0 / g.n), C, 12)
    assert np.abs(xn - pi).sum() < np.abs(xs - pi).sum()


def test_literal_alg1_rotation_after_round_one_is_wrong():
    """Alg. 1 read literally rotates after round 1, when T'' was never formed
    (T <- T', T' <- T'' = 0).  That reading diverges from the definition."""
    g = gg.random_connected(30, 4.0, seed=2)
    A = ocp.adjacency(g)
    d = np.diff(g.row_ptr).astype(float)
    ck = ocp.chebyshev_coefficients(C, 20)
    T = np.ones(g.n)
    Tp = np.zeros(g.n)
    Tpp = np.zeros(g.n)
    acc = ck[0] / 2 * T
    for k in range(1, 21):
        if k == 1:
            Tp = A @ (T / d)
            acc += ck[1] * Tp
        else:
            Tpp = 2 * (A @ (Tp / d)) - T
            acc += ck[k] * Tpp
        T, Tp = Tp, Tpp          # literal rotation, also at k = 1
    lit = acc / acc.sum()
    pi = ocp.pagerank_exact(g, np.full(g.n, 1.0 / g.n), C)
    assert np.abs(lit - pi).sum() > 1e-2
    assert np.abs(ocp.cpaa_alg1_global(g, C, 20) - pi).sum() < 1e-5


def test_error_measures():
    ref = np.array([0.5, 0.25, 0.25])
    x = np.array([0.5, 0.3, 0.2])
    assert ocp.l1_error(x, ref) == pytest.approx(0.1)
    assert ocp.max_error(x, ref) == pytest.approx(0.05)
    assert ocp.max_relative_error(x, ref) == pytest.approx(0.2)


def test_isolated_vertex_rejected():
    g = gg.csr_from_edges(4, np.array([0, 1]), np.array([1, 2]))   # vertex 3 isolated
    with pytest.raises(ValueError):
        ocp.transition_matrix(g)


def test_apriori_terms_examples():
    """K values of the a-priori rule on concrete inputs (used to size solves)."""
    assert ocp.terms_for_mass_error(C, 1e-10) == 39
    assert ocp.terms_for_mass_error(C, 1e-6) == 24
    g = gg.cycle(100)
    d = np.diff(g.row_ptr).astype(float)
    b = (1 - C) * np.full(100, 0.01)
    # regular graph, uniform p: sqrt(vol) ||D^{-1/2} p||_2 = 1, so the rule is eq. 4.1's
    assert ocp.terms_for_apriori(d, b, C, 1e-6) == 24


# ----------------------------------------------------------------------------
# mutation tests: a planted mistake in the oracle must fail some pin
# ----------------------------------------------------------------------------

def _fails(check, o):
    try:
        check(o)
    except AssertionError:
        return True
    return False


class _Mut:
    """A copy of the oracle module namespace with one function replaced."""

    def __init__(self, **over):
        self.__dict__.update({k: getattr(ocp, k) for k in ocp.__all__})
        self.__dict__.update(over)


def test_mutation_transposed_transition_is_caught(monkeypatch):
    orig = ocp.transition_matrix

    def transposed(g):
        return orig(g).T.tocsr()     # D^{-1} A instead of A D^{-1}
    monkeypatch.setattr(ocp, "transition_matrix", transposed)
    assert _fails(check_stationary, ocp) or _fails(check_dense_vs_fractions, ocp)


def test_mutation_gather_scaled_by_target_degree_is_caught(monkeypatch):
    def wrong(g, A, T, deg):       # divides by deg(u) instead of deg(v_i)
        return (A @ T) / (deg if T.ndim == 1 else deg[:, None])
    monkeypatch.setattr(ocp, "_gather_over_neighbours", wrong)
    assert _fails(check_cpaa_converges, ocp) or _fails(check_stationary, ocp)


def test_mutation_recurrence_sign_is_caught(monkeypatch):
    orig = ocp._gather_over_neighbours
    calls = {"n": 0}

    def flipped(g, A, T, deg):
        calls["n"] += 1
        return -orig(g, A, T, deg) if calls["n"] > 1 else orig(g, A, T, deg)
    monkeypatch.setattr(ocp, "_gather_over_neighbours", flipped)
    assert _fails(check_cycle, ocp)


def test_mutation_coefficient_off_by_one_is_caught():
    def shifted(c, M):
        return ocp.chebyshev_coefficients(c, M + 1)[1:]
    assert _fails(check_coefficients_vs_integral, _Mut(chebyshev_coefficients=shifted))


def test_mutation_dropped_first_term_is_caught(monkeypatch):
    orig = ocp.chebyshev_coefficients

    def dropped(c, M):
        ck = orig(c, M).copy()
        if M >= 1:
            ck[1] = 0.0
        return ck
    monkeypatch.setattr(ocp, "chebyshev_coefficients", dropped)
    assert _fails(check_cpaa_converges, ocp)


def test_mutation_beta_sign_in_certificate_is_caught():
    def wrong(c, M, TM, TM1):
        s = math.sqrt(1 - c * c)
        b = ocp.beta(c)
        return (1 + s) / s * b ** (M + 1) * (TM1 + b * TM)
    assert _fails(check_series_residual, _Mut(series_residual=wrong))
