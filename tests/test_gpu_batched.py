"""GPU parity of batched CPAA (cpaa_solve_batched: tiles of W right-hand sides,
one SpMM kernel per term) against the FP64 oracle, plus the undirected
reversibility identity d_s pi_s(t) = d_t pi_t(s)."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
C = 0.85


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01743_amd import binding
    binding.lib()
    return torch


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _truth_cols(g, P):
    """P: (B, n) personalizations -> (B, n) PageRank vectors."""
    if g.n <= 2500:
        return oracle.pagerank_exact(g, P.T, C).T
    return oracle.pagerank_power(g, P.T, C, tol=1e-13)[0].T


def _solve(torch, g, P, tol, X0=None, **opts):
    from paper_2112_01743_amd import Plan
    plan = Plan.from_graph(g, C, **opts)
    X, reps = plan.solve_batched(_dev(torch, P), tol, None if X0 is None else _dev(torch, X0))
    torch.cuda.synchronize()
    return X.cpu().numpy(), reps


def _check(g, P, X, reps, tol):
    ref = _truth_cols(g, P)
    for j in range(P.shape[0]):
        err = np.abs(X[j] - ref[j]).sum()
        assert reps[j]["certified"] == 1, (j, reps[j])
        assert err <= tol, (j, err, reps[j])
        assert err <= reps[j]["cert_bound"] * (1 + 1e-9) + 2e-13, (j, err, reps[j])


@pytest.mark.parametrize("B", [1, 5, 8, 13, 64, 70])
def test_small_graph_batches(torch_cuda, B):
    g = gg.random_connected(300, 5.0, seed=21)
    src = gg.random_sources(g.n, B, seed=B, replace=True)
    P = gg.source_personalization(g.n, src)
    _note(f"batch B={B}")
    X, reps = _solve(torch_cuda, g, P, 1e-8)
    _check(g, P, X, reps, 1e-8)


@pytest.mark.parametrize("W", [8, 16, 32, 64])
def test_tile_widths_agree_on_power_law(torch_cuda, W):
    """Chung-Lu graph with hubs above the long-row threshold (split rows)."""
    g = gg.chung_lu(20000, 12, 2.1, seed=3, dmax=5000)
    assert np.diff(g.row_ptr).max() > 512
    src = gg.random_sources(g.n, 40, seed=7)
    P = gg.source_personalization(g.n, src)
    P[0] = gg.uniform_personalization(g.n)
    X, reps = _solve(torch_cuda, g, P, 1e-7, tile_w=W)
    _check(g, P, X, reps, 1e-7)


@pytest.mark.parametrize("B", [5, 40, 100])
def test_autotuned_tile_width(torch_cuda, B):
    from paper_2112_01743_amd import Plan
    g = gg.chung_lu(20000, 12, 2.1, seed=3, dmax=5000)
    src = gg.random_sources(g.n, B, seed=8)
    P = gg.source_personalization(g.n, src)
    plan = Plan.from_graph(g, C, autotune=1)
    X, reps = plan.solve_batched(_dev(torch_cuda, P), 1e-7)
    W = plan.info()["tile_w"]
    _note(f"B={B}: autotuned tile_w={W}")
    assert W in (16, 32, 64)
    _check(g, P, X.cpu().numpy(), reps, 1e-7)
    X2, reps2 = plan.solve_batched(_dev(torch_cuda, P[:3]), 1e-7)
    assert plan.info()["tile_w"] == W
    _check(g, P[:3], X2.cpu().numpy(), reps2, 1e-7)


def test_power_law_batch_certified_by_main_series(torch_cuda):
    """Rows longer than a gather burst and hub chunks are summed in FP64 in the
    tiled kernel: on a power-law graph with hubs of thousands of entries every
    column is certified by its main series, without a correction series."""
    g = gg.chung_lu(300000, 16, 2.1, seed=2112005, dmax=50000)
    assert np.diff(g.row_ptr).max() > 2000
    src = gg.random_sources(g.n, 64, seed=5)
    P = gg.source_personalization(g.n, src)
    X, reps = _solve(torch_cuda, g, P, 1e-6, max_refine=0, tile_w=64)
    _note(f"bounds max {max(r['cert_bound'] for r in reps):.3e}")
    assert all(r["certified"] == 1 and r["refinements"] == 0 for r in reps)
    for j in (0, 63):
        pi = oracle.pagerank_power(g, P[j], C, tol=1e-10)[0]
        assert np.abs(X[j] - pi).sum() <= 1e-6


def test_mixed_personalizations_and_strides(torch_cuda):
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.perturbed_grid(60, 0.05, 0.01, seed=2)
    rng = gg.philox(5)
    B = 11
    P = rng.random((B, g.n))
    P /= P.sum(axis=1, keepdims=True)
    big = torch.zeros((B, g.n + 37), dtype=torch.float64, device="cuda")
    big[:, :g.n] = _dev(torch, P)
    out = torch.full((B, g.n + 5), -1.0, dtype=torch.float64, device="cuda")
    plan = Plan.from_graph(g, C, tile_w=8)
    X, reps = plan.solve_batched(big[:, :g.n], 1e-9, out=out[:, :g.n])
    Xn = out.cpu().numpy()
    assert np.all(Xn[:, g.n:] == -1.0)          # padding columns untouched
    _check(g, P, Xn[:, :g.n], reps, 1e-9)


def test_reversibility_on_grid(torch_cuda):
    """Undirected reversibility: d_s pi_s(t) = d_t pi_t(s) for sources s, t."""
    g = gg.perturbed_grid(80, 0.05, 0.01, seed=11)
    d = np.diff(g.row_ptr).astype(float)
    src = gg.random_sources(g.n, 24, seed=4)
    X, reps = _solve(torch_cuda, g, gg.source_personalization(g.n, src), 1e-9)
    M = X[:, src]                       # M[i, k] = pi_{s_i}(s_k)
    lhs = d[src][:, None] * M           # d_{s_i} pi_{s_i}(s_k)
    err_abs = np.abs(lhs - lhs.T)
    # each entry is within its solve's L1 bound; scale by the degrees
    tolm = (d[src][:, None] * 1e-9 + d[src][None, :] * 1e-9)
    assert np.all(err_abs <= tolm), err_abs.max()


def test_batched_warm_start_and_fallback(torch_cuda):
    g = gg.chung_lu(8000, 10, 2.3, seed=9)
    src = gg.random_sources(g.n, 9, seed=1)
    P = gg.source_personalization(g.n, src)
    ref = _truth_cols(g, P)
    rng = gg.philox(2)
    X0 = np.abs(ref * (1 + 1e-3 * rng.standard_normal(ref.shape)))
    X0 /= X0.sum(axis=1, keepdims=True)
    X, reps = _solve(torch_cuda, g, P, 1e-8, X0=X0)
    _check(g, P, X, reps, 1e-8)
    assert all(r["fallback_used"] == 0 for r in reps)
    _, plain = _solve(torch_cuda, g, P, 1e-8)
    assert reps[0]["terms"] < plain[0]["terms"]
    # rejected guesses restart their columns as plain solves (the tile then
    # runs until its slowest column is certified)
    X0[4] = np.nan
    X0[6] = 0.0
    X, reps = _solve(torch_cuda, g, P, 1e-8, X0=X0)
    _check(g, P, X, reps, 1e-8)
    assert [r["fallback_used"] for r in reps] == [0, 0, 0, 0, 1, 0, 1, 0, 0]


def test_batched_matches_single_solves(torch_cuda):
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(6000, 8, 2.5, seed=12)
    src = [0, 17, 500, 5999]
    P = gg.source_personalization(g.n, src)
    plan = Plan.from_graph(g, C)
    X, _ = plan.solve_batched(_dev(torch, P), 1e-9)
    for j in range(len(src)):
        x, _ = plan.solve(_dev(torch, P[j]), 1e-9)
        assert float((X[j] - x).abs().sum()) < 4e-9


def test_batched_host_io_and_normalize(torch_cuda):
    from paper_2112_01743_amd import binding as B
    g = gg.random_connected(200, 4.0, seed=3)
    P = np.ascontiguousarray(gg.source_personalization(g.n, [1, 2, 3]))
    X = np.zeros_like(P)
    plan = B.Plan.from_graph(g, C, io_device=0, normalize=1)
    st, reps = B.cpaa_solve_batched(plan.handle, 3, P.ctypes.data, g.n, 1e-9, None, g.n,
                                    X.ctypes.data, g.n)
    assert st == B.CPAA_OK, B.cpaa_last_error()
    ref = _truth_cols(g, P)
    assert np.allclose(X.sum(axis=1), 1.0, atol=1e-12)
    assert np.abs(X - ref).sum(axis=1).max() < 1e-9


def test_batched_rejects_bad_columns(torch_cuda):
    from paper_2112_01743_amd import Plan, CpaaError
    g = gg.cycle(20)
    P = gg.source_personalization(g.n, [1, 2])
    P[1, 3] = -0.5
    plan = Plan.from_graph(g, C)
    with pytest.raises(CpaaError, match="column 1"):
        plan.solve_batched(_dev(torch_cuda, P), 1e-6)
