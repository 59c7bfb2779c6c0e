"""The OpenMP C reference (oracle/cpaa_omp.c, the benchmark's multi-core CPU
baseline) against the numpy oracle, which the other oracle tests pin to the
paper: the same x_M for every pinned M and the same power-method iterates, on
one thread and on several (an OpenMP race or a missed row would show as a
difference between the two).  CPU only."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import omp

C = 0.85


@pytest.fixture(scope="module", autouse=True)
def built():
    omp.build()


@pytest.mark.parametrize("name,g", [
    ("cycle9", gg.cycle(9)),
    ("star50", gg.star(50)),
    ("chung_lu", gg.chung_lu(20000, 10, 2.1, seed=3)),
    ("grid", gg.perturbed_grid(60, 0.05, 0.01, seed=2)),
])
def test_cpaa_matches_numpy_oracle(name, g):
    rng = gg.philox(4)
    b = (1 - C) * gg.source_personalization(g.n, [g.n // 3])[0]
    b2 = rng.standard_normal(g.n)          # a residual-like right-hand side (any sign)
    for rhs in (b, b2):
        for M in (0, 1, 2, 7, 24):
            ref = oracle.cpaa(g, rhs, C, M)
            for th in (1, 4):
                x = omp.cpaa(g, rhs, C, M, threads=th)
                assert np.abs(x - ref).sum() <= 1e-12 * max(1.0, np.abs(ref).sum()), (M, th)


def test_cpaa_pinned_on_the_cycle_closed_form():
    """Independent of the numpy oracle: on the cycle every T_k(P)e_s is
    (e_{s+k} + e_{s-k})/2, so x_M has a closed form."""
    n, s, M = 31, 4, 9
    g = gg.cycle(n)
    b = np.zeros(n)
    b[s] = 1.0
    ck = oracle.chebyshev_coefficients(C, M)
    want = np.zeros(n)
    want[s] += ck[0] / 2
    for k in range(1, M + 1):
        want[(s + k) % n] += ck[k] / 2
        want[(s - k) % n] += ck[k] / 2
    assert np.abs(omp.cpaa(g, b, C, M, threads=3) - want).max() <= 1e-14


def test_power_matches_numpy_oracle():
    g = gg.chung_lu(20000, 10, 2.1, seed=5)
    p = gg.uniform_personalization(g.n)
    ref, it_ref = oracle.pagerank_power(g, p, C, tol=1e-10)
    for th in (1, 4):
        x, it = omp.power(g, p, C, 1e-10, threads=th)
        assert it == it_ref
        assert np.abs(x - ref).sum() <= 1e-13
    # the converged vector is PageRank: the dense solve on a small graph
    h = gg.random_connected(300, 5.0, seed=9)
    ph = gg.source_personalization(h.n, [7])[0]
    x, _ = omp.power(h, ph, C, 1e-13, threads=2)
    assert np.abs(x - oracle.pagerank_exact(h, ph, C)).sum() <= 1e-12
