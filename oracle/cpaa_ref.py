"""FP64 reference for CPAA (arXiv 2112.01743).  TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this
module.  It shares no code with the GPU library.

Notation follows the paper:
  * graph G, adjacency A (a_ij = 1 iff v_j -> v_i), degree matrix D,
    transition matrix P = A D^{-1} (Sec. 2.1);
  * damping c in (0, 1), personalization p, PageRank
    pi = (1-c)(I - cP)^{-1} p (Sec. 2.1);
  * Chebyshev polynomials T_k with T_{k+1}(x) = 2x T_k(x) - T_{k-1}(x)
    (Sec. 2.2, property (3));
  * coefficients c_k of f(x) = (1-cx)^{-1} (Sec. 2.2), beta and the mass
    error ERR_M (Sec. 4.2.2, eq. 4.1).
The right-hand side is written b: b = (1-c)p for a PageRank solve, or any
residual vector for a correction solve; x_M = (c_0/2) b + sum_{k=1..M} c_k T_k(P) b
(eq. 3.1 applied to b).

Readings of the paper taken here (each listed with its reason in the design
notes):
  * Alg. 1 rotates T <- T', T' <- T'' also after the first round, where T''
    was never formed; the standard recurrence is used instead (after round 1,
    T keeps T_0 and T' holds T_1).
  * Alg. 1 adds c_k T''_u into pi_i; the vertex index is u.
  * Alg. 1 starts from T_i = 1 (p = e); here T_0 = b so personalized and
    residual right-hand sides are covered; ``cpaa_alg1_global`` keeps the
    paper's all-ones start and final normalization.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
import scipy.integrate
import scipy.sparse as sp

__all__ = [
    "beta", "chebyshev_coefficients", "chebyshev_coefficient_integral",
    "interval_map", "chebyshev_interval_coefficients",
    "chebyshev_interval_coefficient_integral", "convergence_rate", "mass_error", "accumulated_mass", "total_mass",
    "series_tail", "terms_for_mass_error", "apriori_error_bound", "terms_for_apriori",
    "adjacency", "transition_matrix", "transition_dense", "pagerank_exact",
    "pagerank_power", "power_method", "transition_directed", "pagerank_directed_exact",
    "power_method_directed", "cpaa", "cpaa_interval", "cpaa_alg1_global", "residual", "residual_l1_bound",
    "series_residual", "l1_error", "max_error", "max_relative_error",
]


# ----------------------------------------------------------------------------
# Coefficients and error model (Sec. 2.2, Sec. 4.2)
# ----------------------------------------------------------------------------

def beta(c: float) -> float:
    """beta = (1 - sqrt(1 - c^2)) / c  (Sec. 4.2.2, below eq. 4.1)."""
    return (1.0 - math.sqrt(1.0 - c * c)) / c


def chebyshev_coefficients(c: float, M: int) -> np.ndarray:
    """c_0..c_M of (1 - c x)^{-1} in closed form.

    Prop. 1's proof gives c_0 = 2/sqrt(1-c^2) and a constant ratio
    c_{k-1}/c_k = c / (1 - sqrt(1-c^2)) = 1/beta, hence c_k = c_0 beta^k.
    """
    c0 = 2.0 / math.sqrt(1.0 - c * c)
    return c0 * beta(c) ** np.arange(M + 1, dtype=np.float64)


def chebyshev_coefficient_integral(c: float, k: int) -> float:
    """c_k = (2/pi) * int_0^pi cos(k t) / (1 - c cos t) dt  (Sec. 2.2), by quadrature."""
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", scipy.integrate.IntegrationWarning)
        val, _ = scipy.integrate.quad(lambda t: math.cos(k * t) / (1.0 - c * math.cos(t)),
                                      0.0, math.pi, limit=400, epsabs=1e-15, epsrel=1e-14)
    return 2.0 / math.pi * val


def interval_map(c: float, a: float) -> tuple[float, float]:
    """On x in [a, 1] write x = ((1-a)u + (1+a))/2, u in [-1, 1].  Then
    1/(1 - cx) = (1/A) / (1 - c' u) with A = 1 - c(1+a)/2 and c' = c(1-a)/(2A)
    (Sec. 2.2's general interval applied to f(x) = 1/(1-cx)).  Returns (A, c')."""
    A = 1.0 - c * (1.0 + a) / 2.0
    return A, c * (1.0 - a) / (2.0 * A)


def chebyshev_interval_coefficients(c: float, a: float, M: int) -> np.ndarray:
    """Coefficients of 1/(1-cx) in the Chebyshev polynomials of u(x) on [a, 1]:
    the [-1, 1] coefficients of 1/(1 - c'u) (Prop. 1's closed form with c') times
    1/A.  For a = -1 they are the c_k of ``chebyshev_coefficients``."""
    A, cp = interval_map(c, a)
    return chebyshev_coefficients(cp, M) / A


def chebyshev_interval_coefficient_integral(c: float, a: float, k: int) -> float:
    """The general-interval coefficient of Sec. 2.2 for f(x) = 1/(1-cx) on [a, 1],
    with the factor 2/pi that its [-1, 1] special case carries:
    c_k = (2/pi) int_0^pi f(((1-a) cos t + (1+a))/2) cos(k t) dt, by quadrature."""
    def f(t):
        x = ((1.0 - a) * math.cos(t) + (1.0 + a)) / 2.0
        return math.cos(k * t) / (1.0 - c * x)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", scipy.integrate.IntegrationWarning)
        val, _ = scipy.integrate.quad(f, 0.0, math.pi, limit=400, epsabs=1e-15, epsrel=1e-14)
    return 2.0 / math.pi * val


def convergence_rate(c: float) -> float:
    """sigma_c of Proposition 1, in the form printed there (Sec. 4.2.1)."""
    s = math.sqrt(1.0 - c * c)
    return (c * c - (2.0 - c) * (1.0 - s)) / (c * c - c * (1.0 - s))


def accumulated_mass(c: float, M: int, n: float = 1.0) -> float:
    """S_M = n c_0/2 + n sum_{i=1..M} c_i, the mass accumulated after round M (Sec. 4.2.1)."""
    ck = chebyshev_coefficients(c, M)
    return n * (ck[0] / 2.0 + ck[1:].sum())


def total_mass(c: float, n: float = 1.0) -> float:
    """S = lim S_M = n f(1) = n / (1 - c), since T_k(1) = 1 for all k (Sec. 4.2.1)."""
    return n / (1.0 - c)


def mass_error(c: float, M: int) -> float:
    """ERR_M = 1 - S_M/S = 2 beta^{M+1} / (1 + beta)  (eq. 4.1)."""
    b = beta(c)
    return 2.0 * b ** (M + 1) / (1.0 + b)


def series_tail(c: float, M: int) -> float:
    """sum_{k>M} c_k = c_0 beta^{M+1} / (1 - beta): the sup over [-1,1] of the truncation error."""
    b = beta(c)
    return 2.0 / math.sqrt(1.0 - c * c) * b ** (M + 1) / (1.0 - b)


def terms_for_mass_error(c: float, tol: float, scale: float = 1.0, m_max: int = 10000) -> int:
    """Smallest M with scale * ERR_M <= tol (eq. 4.1; scale=1 is the paper's rough rule)."""
    for M in range(m_max + 1):
        if scale * mass_error(c, M) <= tol:
            return M
    raise ValueError("tolerance not reachable")


def apriori_error_bound(deg: np.ndarray, b: np.ndarray, c: float, M: int) -> float:
    """Upper bound on ||x_M - (I-cP)^{-1} b||_1 for an undirected graph.

    P = D^{1/2} S D^{-1/2} with S = D^{-1/2} A D^{-1/2} symmetric and its
    spectrum in [-1, 1] (Lemma 2 gives a real spectrum), so
    ||(g_M - f)(P) b||_1 <= sqrt(vol) ||(g_M - f)(S) D^{-1/2} b||_2
                        <= sqrt(vol) ||D^{-1/2} b||_2 sup|g_M - f|,
    and the sup of the truncation error over [-1, 1] is the coefficient tail.
    """
    deg = np.asarray(deg, dtype=np.float64)
    vol = deg.sum()
    return math.sqrt(vol) * float(np.linalg.norm(b / np.sqrt(deg))) * series_tail(c, M)


def terms_for_apriori(deg: np.ndarray, b: np.ndarray, c: float, tol: float,
                      m_max: int = 10000) -> int:
    """Smallest M whose a-priori bound is <= tol."""
    for M in range(m_max + 1):
        if apriori_error_bound(deg, b, c, M) <= tol:
            return M
    raise ValueError("tolerance not reachable")


# ----------------------------------------------------------------------------
# The linear-system definition (Sec. 2.1)
# ----------------------------------------------------------------------------

def _deg(g) -> np.ndarray:
    return np.diff(np.asarray(g.row_ptr, dtype=np.int64)).astype(np.float64)


def adjacency(g) -> sp.csr_matrix:
    """A with a_ij = 1 iff (v_j, v_i) in E; symmetric for an undirected graph (Sec. 2.1)."""
    data = np.ones(g.col_idx.shape[0], dtype=np.float64)
    return sp.csr_matrix((data, np.asarray(g.col_idx, dtype=np.int64),
                          np.asarray(g.row_ptr, dtype=np.int64)), shape=(g.n, g.n))


def transition_matrix(g) -> sp.csr_matrix:
    """P = A D^{-1}: p_ij = a_ij / d_j, column-stochastic (Sec. 2.1)."""
    deg = _deg(g)
    if np.any(deg == 0):
        raise ValueError("isolated vertex: P = A D^{-1} needs every d_i > 0")
    return (adjacency(g) @ sp.diags(1.0 / deg)).tocsr()


def transition_dense(g) -> np.ndarray:
    return transition_matrix(g).toarray()


def pagerank_exact(g, p: np.ndarray, c: float) -> np.ndarray:
    """pi = (1 - c)(I - cP)^{-1} p by a dense FP64 solve (Sec. 2.1).

    ``p`` may be a vector or an (n, B) matrix of personalization columns.
    """
    P = transition_dense(g)
    return np.linalg.solve(np.eye(g.n) - c * P, (1.0 - c) * np.asarray(p, dtype=np.float64))


def power_method(g, p: np.ndarray, c: float, t: int, return_all: bool = False):
    """The power method of the comparison in Sec. 5: PageRank as the fixed point
    pi = P'' pi (eq. 2.1), iterated t times from x_0 = p.

    P'' = cP' + (1-c) p e^T with P' = P for an undirected graph (no dangling
    vertices), applied here as written: x_{k+1} = cPx_k + (1-c) p (e^T x_k).
    The paper does not give the start; p (the distribution the definition is
    built from) is the reading taken.  Returns x_t, or the list x_0..x_t with
    ``return_all``.
    """
    P = transition_matrix(g)
    p = np.asarray(p, dtype=np.float64)
    x = p.copy()
    seq = [x]
    for _ in range(t):
        x = c * (P @ x) + (1.0 - c) * p * x.sum(axis=0)
        seq.append(x)
    return seq if return_all else x


def transition_directed(g):
    """For a directed graph (row u of the pattern lists the v with v -> u, so
    a_uv = 1 iff v -> u as in Sec. 2.1): P = A D^{-1} on the columns of vertices
    with out-edges (D the out-degrees, column sums of A), zero columns at
    dangling vertices (sparse), and the dangling indicator d of Sec. 2.1."""
    A = adjacency(g)
    dout = np.asarray(A.sum(axis=0)).ravel()
    inv = np.zeros(g.n)
    nz = dout > 0
    inv[nz] = 1.0 / dout[nz]
    return (A @ sp.diags(inv)).tocsr(), (~nz).astype(np.float64)


def pagerank_directed_exact(g, p: np.ndarray, c: float) -> np.ndarray:
    """PageRank of a directed graph by a dense FP64 solve: with P' = P + p d^T
    (Sec. 2.1), pi = P''pi, P'' = cP' + (1-c) p e^T, sum pi = 1 (eq. 2.1) is
    (I - cP') pi = (1-c) p."""
    P, d = transition_directed(g)
    p = np.asarray(p, dtype=np.float64)
    Pp = P.toarray() + np.outer(p, d)
    return np.linalg.solve(np.eye(g.n) - c * Pp, (1.0 - c) * p)


def power_method_directed(g, p: np.ndarray, c: float, t: int, return_all: bool = False):
    """The power method on a directed graph: x_{k+1} = P'' x_k from x_0 = p with
    P'' = c(P + p d^T) + (1-c) p e^T applied as written (eq. 2.1, Sec. 2.1)."""
    P, d = transition_directed(g)
    p = np.asarray(p, dtype=np.float64)
    x = p.copy()
    seq = [x]
    for _ in range(t):
        x = c * (P @ x + p * (d @ x)) + (1.0 - c) * p * x.sum()
        seq.append(x)
    return seq if return_all else x


def pagerank_power(g, p: np.ndarray, c: float, tol: float = 1e-13,
                   max_iter: int = 100000) -> tuple[np.ndarray, int]:
    """Power iteration x <- cPx + (1-c)p (the fixed point of eq. 2.1 for undirected G).

    x_{k+1} - x_k is exactly the residual (1-c)p - (I-cP)x_k, and because
    ||(I-cP)^{-1}||_1 = 1/(1-c) for column-stochastic P the error of x_{k+1}
    is at most c ||x_{k+1} - x_k||_1 / (1-c); iteration stops once that bound
    is <= tol (for a matrix of columns: the largest column bound).
    Returns (x, iterations).
    """
    P = transition_matrix(g)
    b = (1.0 - c) * np.asarray(p, dtype=np.float64)
    x = b.copy()
    for it in range(1, max_iter + 1):
        x_new = c * (P @ x) + b
        diff = np.abs(x_new - x).sum(axis=0)
        x = x_new
        if np.max(c * diff / (1.0 - c)) <= tol:
            return x, it
    raise RuntimeError("power method did not converge")


# ----------------------------------------------------------------------------
# CPAA, Algorithm 1 (Sec. 4.1)
# ----------------------------------------------------------------------------

def _gather_over_neighbours(g, A: sp.csr_matrix, T: np.ndarray, deg: np.ndarray) -> np.ndarray:
    """For every vertex u: sum over v_i in N(u) of T_i / deg(v_i)  (the inner loop of Alg. 1)."""
    if T.ndim == 1:
        return A @ (T / deg)
    return A @ (T / deg[:, None])


def cpaa(g, b: np.ndarray, c: float, M: int, return_terms: bool = False,
         normalize: bool = False):
    """FP64 CPAA: x_M = (c_0/2) b + sum_{k=1..M} c_k T_k(P) b  (Alg. 1 with eq. 3.1).

    Rounds follow Alg. 1: round 1 forms T' = P T; round k >= 2 forms
    T'' = 2 P T' - T, adds c_k T'' to the accumulator, then rotates
    T <- T', T' <- T''.  ``b`` is a vector or an (n, B) matrix.
    With ``normalize`` the result is divided by its sum, the last step of
    Alg. 1 (only meaningful for a probability right-hand side).
    If ``return_terms`` the list [T_0 b, ..., T_{M+1} b] is returned too
    (one extra round, used by the residual certificate).
    """
    A = adjacency(g)
    deg = _deg(g)
    ck = chebyshev_coefficients(c, M + 1)
    T = np.array(b, dtype=np.float64)               # T_0 b
    acc = (ck[0] / 2.0) * T
    terms = [T.copy()] if return_terms else None
    T1 = None
    if M >= 1 or return_terms:
        T1 = _gather_over_neighbours(g, A, T, deg)  # T_1 b = P b
        if M >= 1:
            acc = acc + ck[1] * T1
        if return_terms:
            terms.append(T1.copy())
    Tm, Tc = T, T1
    last = M + 1 if return_terms else M
    for k in range(2, last + 1):
        Tn = 2.0 * _gather_over_neighbours(g, A, Tc, deg) - Tm
        if k <= M:
            acc = acc + ck[k] * Tn
        if return_terms:
            terms.append(Tn.copy())
        Tm, Tc = Tc, Tn
    if normalize:
        acc = acc / acc.sum(axis=0)
    if return_terms:
        return acc, terms
    return acc


def cpaa_alg1_global(g, c: float, M: int) -> np.ndarray:
    """Alg. 1 as printed for global PageRank: T_i = 1 start, final normalization.

    Uses the standard rotation after round 1 (see module notes).
    """
    return cpaa(g, np.ones(g.n), c, M, normalize=True)


# ----------------------------------------------------------------------------
# Residuals, certificates and error measures
# ----------------------------------------------------------------------------

def residual(g, b: np.ndarray, x: np.ndarray, c: float) -> np.ndarray:
    """r = b - (I - cP) x in FP64."""
    P = transition_matrix(g)
    return np.asarray(b, dtype=np.float64) - (x - c * (P @ x))


def residual_l1_bound(g, b: np.ndarray, x: np.ndarray, c: float) -> np.ndarray | float:
    """||x - (I-cP)^{-1} b||_1 <= ||r||_1 / (1 - c), because ||(I-cP)^{-1}||_1 = 1/(1-c)
    for a column-stochastic P (sum_k c^k ||P^k||_1 with ||P||_1 = 1)."""
    r = residual(g, b, x, c)
    return np.abs(r).sum(axis=0) / (1.0 - c)


def cpaa_interval(g, b: np.ndarray, c: float, a: float, M: int, return_terms: bool = False):
    """CPAA with the Chebyshev expansion of 1/(1-cx) on [a, 1] instead of [-1, 1]
    (Sec. 2.2's general interval; valid when the spectrum of P lies in [a, 1]):
        x_M = (c'_0/2) b + sum_{k=1..M} c'_k T_k(t(P)) b,  t(P) = (2P - (1+a)I)/(1-a),
    with the c'_k of ``chebyshev_interval_coefficients`` and T_k(t(P)) b from
    property (3): T_1 = t(P) T_0, T_{k+1} = 2 t(P) T_k - T_{k-1}.
    With ``return_terms`` also [T_0 b, ..., T_{M+1} b]."""
    A = adjacency(g)
    deg = _deg(g)
    ck = chebyshev_interval_coefficients(c, a, M + 1)

    def t_of(T):
        return (2.0 * _gather_over_neighbours(g, A, T, deg) - (1.0 + a) * T) / (1.0 - a)

    T = [np.array(b, dtype=np.float64)]
    T.append(t_of(T[0]))
    for _ in range(2, M + 2):
        T.append(2.0 * t_of(T[-1]) - T[-2])
    acc = (ck[0] / 2.0) * T[0]
    for k in range(1, M + 1):
        acc = acc + ck[k] * T[k]
    return (acc, T) if return_terms else acc


def series_residual(c: float, M: int, TM: np.ndarray, TM1: np.ndarray) -> np.ndarray:
    """Closed form of b - (I - cP) x_M from the last two Chebyshev vectors:

        b - (I-cP) x_M = ((1+s)/s) beta^{M+1} (T_{M+1}(P) b - beta T_M(P) b),  s = sqrt(1-c^2).

    Derivation: let Q(x) = 1 - 2 beta x + beta^2 and G_M = sum_{k=0..M} beta^k T_k.
    Using 2x T_k = T_{k+1} + T_{k-1} (k >= 1) and 2x T_0 = 2 T_1, the product
    telescopes: Q G_M = (1 - beta x) - beta^{M+1} (T_{M+1} - beta T_M).
    With c_k = 2 beta^k / s, g_M = (2 G_M - 1)/s, and with
    1 + beta^2 = 2/(1+s), (1 - beta^2)/(1 + beta^2) = s, 1 - cx = Q/(1 + beta^2):
        (1 - cx) g_M(x) = 1 - ((1+s)/s) beta^{M+1} (T_{M+1}(x) - beta T_M(x)).
    Applying it to P and b gives the identity (checked against the explicit
    residual in the tests).
    """
    s = math.sqrt(1.0 - c * c)
    b = beta(c)
    return (1.0 + s) / s * b ** (M + 1) * (TM1 - b * TM)


def l1_error(x: np.ndarray, ref: np.ndarray):
    return np.abs(np.asarray(x) - np.asarray(ref)).sum(axis=0)


def max_error(x: np.ndarray, ref: np.ndarray):
    return np.abs(np.asarray(x) - np.asarray(ref)).max(axis=0)


def max_relative_error(x: np.ndarray, ref: np.ndarray):
    """ERR = max_i |x_i - pi_i| / pi_i, the experimental error measure of Sec. 5.1."""
    ref = np.asarray(ref)
    return (np.abs(np.asarray(x) - ref) / ref).max(axis=0)
