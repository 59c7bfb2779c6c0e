"""Pins for the oracle's Chebyshev expansion on [a, 1] (Sec. 2.2's general
interval, used when the spectrum of P is known to lie in [a, 1]).  CPU only."""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle

C = 0.85


def _lambda_min(g):
    """Smallest eigenvalue of P (= that of D^{-1/2} A D^{-1/2}), dense."""
    d = np.diff(g.row_ptr).astype(float)
    A = oracle.adjacency(g).toarray()
    return float(np.linalg.eigvalsh(A / np.sqrt(np.outer(d, d)))[0])


@pytest.mark.parametrize("a", [-1.0, -0.75, -0.4, 0.0, 0.5])
def test_interval_coefficients_match_the_general_formula(a):
    ck = oracle.chebyshev_interval_coefficients(C, a, 12)
    q = np.array([oracle.chebyshev_interval_coefficient_integral(C, a, k) for k in range(13)])
    assert np.max(np.abs(ck - q)) < 1e-12


def test_full_interval_is_the_paper_series():
    g = gg.random_connected(200, 5, seed=2)
    b = (1 - C) * gg.source_personalization(g.n, [4])[0]
    assert np.allclose(oracle.chebyshev_interval_coefficients(C, -1.0, 20),
                       oracle.chebyshev_coefficients(C, 20), rtol=0, atol=1e-15)
    assert np.abs(oracle.cpaa_interval(g, b, C, -1.0, 17) - oracle.cpaa(g, b, C, 17)).max() < 1e-15


def check_converges_faster_on_the_spectral_interval(cpaa_interval):
    """ER graph (not bipartite): lambda_min(P) ~ -0.6.  On [lambda_min, 1] every
    |T_k(t(lambda))| <= 1, so ||x_M - x||_1 <= sqrt(vol) ||D^{-1/2} b||_2 sum_{k>M} |c'_k|,
    and the interval's coefficients decay faster than the [-1, 1] ones."""
    g = gg.erdos_renyi(400, 12, seed=3)
    lam = _lambda_min(g)
    assert -0.8 < lam < -0.3
    b = (1 - C) * gg.source_personalization(g.n, [9])[0]
    x = oracle.pagerank_exact(g, b / (1 - C), C)
    d = np.diff(g.row_ptr).astype(float)
    scale = math.sqrt(d.sum()) * math.sqrt(np.sum(b * b / d))
    ck = oracle.chebyshev_interval_coefficients(C, lam, 200)
    for M in (5, 10, 20, 30):
        err = np.abs(cpaa_interval(g, b, C, lam, M) - x).sum()
        assert err <= scale * np.abs(ck[M + 1:]).sum() * (1 + 1e-9) + 1e-15, M
        assert err < np.abs(oracle.cpaa(g, b, C, M) - x).sum(), M
    assert np.abs(cpaa_interval(g, b, C, lam, 60) - x).sum() < 1e-13


def test_converges_faster_on_the_spectral_interval():
    check_converges_faster_on_the_spectral_interval(oracle.cpaa_interval)


def test_residual_identity_on_the_interval():
    """With A = 1 - c(1+a)/2, c' = c(1-a)/(2A), beta' and s' of c':
    I - cP = A (I - c' t(P)), so the telescoping identity of the [-1, 1] series
    holds with the primed quantities and T_k(t(P)) b:
        b - (I - cP) x_M = ((1+s')/s') beta'^{M+1} (T_{M+1} - beta' T_M) b."""
    g = gg.random_connected(300, 6, seed=8)
    a = -0.5       # the identity is algebraic: it holds whatever the spectrum
    b = (1 - C) * gg.source_personalization(g.n, [0])[0]
    _, cp = oracle.interval_map(C, a)
    bp = oracle.beta(cp)
    sp_ = math.sqrt(1 - cp * cp)
    for M in (1, 4, 11):
        x, T = oracle.cpaa_interval(g, b, C, a, M, return_terms=True)
        r = oracle.residual(g, b, x, C)
        ident = (1 + sp_) / sp_ * bp ** (M + 1) * (T[M + 1] - bp * T[M])
        assert np.abs(r - ident).max() < 1e-12 * max(1.0, np.abs(r).max()), M


def test_mutation_unshifted_interval_map_is_caught():
    """A planted mistake: t(P) = 2P/(1-a) (the (1+a) shift dropped)."""
    def wrong(g, b, c, a, M):
        A = oracle.adjacency(g)
        d = np.diff(g.row_ptr).astype(float)
        ck = oracle.chebyshev_interval_coefficients(c, a, M + 1)

        def t_of(T):
            return 2.0 * (A @ (T / d)) / (1.0 - a)
        T = [np.array(b, dtype=float), None]
        T[1] = t_of(T[0])
        for _ in range(2, M + 1):
            T.append(2.0 * t_of(T[-1]) - T[-2])
        return (ck[0] / 2) * T[0] + sum(ck[k] * T[k] for k in range(1, M + 1))
    with pytest.raises(AssertionError):
        check_converges_faster_on_the_spectral_interval(wrong)
