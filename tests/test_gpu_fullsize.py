"""Parity at the full workload sizes, in the launch configuration bench.py times.

At these sizes the oracle checks the GPU result through properties that hold at
any size: its own FP64 residual r = b - (I - cP) x (one sparse product on the
CPU) gives ||x - pi||_1 <= ||r||_1 / (1 - c), which must be <= tol; sampled
columns are also compared with the oracle's power method.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
C = 0.85
TOL = 1e-6


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


def _oracle_bound(g, B, X):
    """Oracle's FP64 residual bound for each column; B, X: (cols, n)."""
    r = oracle.residual(g, B.T, X.T, C)
    return np.abs(r).sum(axis=0) / (1 - C)


@pytest.mark.timeout(600)
def test_chung_lu_4m_global(torch_cuda):
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(4_000_000, 16, 2.1, seed=2112001, dmin=1.0, dmax=50000.0)
    _note(f"chung-lu n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C, time_kernels=1)     # the bench's plan options
    p = np.full(g.n, 1.0 / g.n)
    x, rep = plan.solve(torch.as_tensor(p, device="cuda"), TOL)
    x = x.cpu().numpy()
    bound = _oracle_bound(g, ((1 - C) * p)[None, :], x[None, :])[0]
    _note(f"gpu bound {rep['cert_bound']:.3e} oracle bound {bound:.3e} terms {rep['terms']}")
    assert rep["certified"] == 1 and bound <= TOL
    assert abs(bound - rep["cert_bound"]) <= 1e-3 * bound + 1e-12
    # sampled entries against the power method (certified to 1e-9)
    pi, _ = oracle.pagerank_power(g, p, C, tol=1e-9)
    idx = gg.philox(5).choice(g.n, 2000, replace=False)
    idx = np.concatenate([idx, np.arange(50)])       # and the 50 largest-degree vertices
    assert np.max(np.abs(x[idx] - pi[idx])) <= TOL + 1e-9
    assert abs(x.sum() - 1.0) <= TOL


@pytest.mark.timeout(600)
def test_power_method_4m_global(torch_cuda):
    """The power method on the same plan (column-sliced kernels) at the full size:
    certified by the oracle's own residual, and the same vector as CPAA's."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(4_000_000, 16, 2.1, seed=2112001, dmin=1.0, dmax=50000.0)
    plan = Plan.from_graph(g, C, time_kernels=1)
    p = np.full(g.n, 1.0 / g.n)
    dp = torch.as_tensor(p, device="cuda")
    xp, rp = plan.solve_power(dp, TOL)
    xc, rc = plan.solve(dp, TOL)
    xp, xc = xp.cpu().numpy(), xc.cpu().numpy()
    bound = _oracle_bound(g, ((1 - C) * p)[None, :], xp[None, :])[0]
    _note(f"power: steps {rp['terms']}+{rp['refine_terms']} gpu bound {rp['cert_bound']:.3e} "
          f"oracle bound {bound:.3e}; cpaa terms {rc['terms']}")
    assert rp["certified"] == 1 and bound <= TOL
    assert np.abs(xp - xc).sum() <= 2 * TOL
    assert rp["terms"] > rc["terms"]


@pytest.mark.timeout(600)
def test_delaunay_2m_rcm_table3(torch_cuda):
    """The Table 3 stand-in at its full size (2^21 points, the bench's seed):
    relabelled by reverse Cuthill-McKee (auto), certified to 1e-6 by the oracle's
    residual for CPAA and the power method, and sampled entries against the
    oracle's power method."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.delaunay(1 << 21, seed=2112010)
    plan = Plan.from_graph(g, C, time_kernels=1)
    assert plan.info()["reordered"] == 2
    p = np.full(g.n, 1.0 / g.n)
    dp = torch.as_tensor(p, device="cuda")
    pi, _ = oracle.pagerank_power(g, p, C, tol=1e-9)
    idx = gg.philox(6).choice(g.n, 3000, replace=False)
    for name in ("solve", "solve_power"):
        x, rep = getattr(plan, name)(dp, TOL)
        x = x.cpu().numpy()
        bound = _oracle_bound(g, ((1 - C) * p)[None, :], x[None, :])[0]
        _note(f"{name}: terms {rep['terms']} gpu bound {rep['cert_bound']:.3e} oracle {bound:.3e}")
        assert rep["certified"] == 1 and bound <= TOL
        assert np.max(np.abs(x[idx] - pi[idx])) <= TOL + 1e-9


@pytest.mark.timeout(600)
def test_grid_256_sources(torch_cuda):
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.perturbed_grid(1000, 0.05, 0.01, seed=2112002)
    src = gg.random_sources(g.n, 256, seed=2112002)
    _note(f"grid n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C, time_kernels=1)
    P = torch.zeros((256, g.n), dtype=torch.float64, device="cuda")
    P[torch.arange(256), torch.as_tensor(src, device="cuda")] = 1.0
    X, reps = plan.solve_batched(P, TOL)
    X = X.cpu().numpy()
    assert all(r["certified"] for r in reps)
    Pn = np.zeros((256, g.n))
    Pn[np.arange(256), src] = 1.0
    bounds = _oracle_bound(g, (1 - C) * Pn, X)
    _note(f"oracle bounds max {bounds.max():.3e}")
    assert bounds.max() <= TOL
    # reversibility d_s pi_s(t) = d_t pi_t(s) among the sources, within the bounds
    d = np.diff(g.row_ptr).astype(float)
    M = X[:, src]
    lhs = d[src][:, None] * M
    tolm = d[src][:, None] * bounds[None, :] + d[src][None, :] * bounds[:, None]
    assert np.all(np.abs(lhs - lhs.T) <= tolm + 1e-15)
    # two sampled columns against the power method
    for j in (0, 255):
        pi, _ = oracle.pagerank_power(g, Pn[j], C, tol=1e-10)
        assert np.abs(X[j] - pi).sum() <= TOL


@pytest.mark.timeout(600)
def test_uneven_batch_10k_graphs(torch_cuda):
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.uneven_batch(10_000, seed=2112003)
    _, p = gg.batch_sources(g, seed=2112003)
    _note(f"batch n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C, autotune=1)          # the bench's plan options
    x, reps = plan.solve_graphs(torch.as_tensor(p, device="cuda"), TOL)
    x = x.cpu().numpy()
    assert all(r["certified"] for r in reps)
    # the block-diagonal residual separates by graph
    r = oracle.residual(g, (1 - C) * p, x, C)
    gp = g.graph_ptr.astype(np.int64)
    per_graph = np.add.reduceat(np.abs(r), gp[:-1]) / (1 - C)
    _note(f"oracle per-graph bounds max {per_graph.max():.3e}")
    assert per_graph.max() <= TOL
    for k in gg.philox(3).choice(g.num_graphs, 6, replace=False):
        sub = gg.subgraph(g, k)
        v0, v1 = gp[k], gp[k + 1]
        pi = oracle.pagerank_exact(sub, p[v0:v1], C)
        assert np.abs(x[v0:v1] - pi).sum() <= TOL


@pytest.mark.timeout(600)
def test_warm_start_network_at_1m(torch_cuda):
    """The network's forward pass on the 1M-vertex warm-start graph against the
    bf16-emulating FP64 oracle, and a warm-started solve at that size judged
    against the plain one."""
    from paper_2112_01743_amd import Plan
    from paper_2112_01743_amd.binding import Model
    from oracle import mpnn as om
    torch = torch_cuda
    g = gg.chung_lu(1_000_000, 16, 2.1, seed=2112005, dmax=50000)
    _note(f"chung-lu n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C)
    params = gg.mpnn_init(2112004)
    model = Model(plan, params)
    src = [int(s) for s in gg.random_sources(g.n, 2, seed=2112005)]
    X0 = model.predict(src)
    X0n = X0.cpu().numpy()
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    for j, s in enumerate(src):
        ref, _ = om.mpnn_forward(g, p64, s, bf16=True)
        l1 = np.abs(X0n[j] - ref).sum()
        _note(f"source {s}: forward L1 vs oracle {l1:.3e}")
        # measured 5.5e-6
        assert abs(X0n[j].sum() - 1.0) < 1e-12 and l1 <= 1e-4
    P = torch.zeros((2, g.n), dtype=torch.float64, device="cuda")
    P[torch.arange(2), torch.as_tensor(src, device="cuda")] = 1.0
    Xw, rw = plan.solve_batched(P, TOL, X0=X0)
    Xp, rp = plan.solve_batched(P, TOL)
    assert np.all(rw["certified"] == 1) and np.all(rp["certified"] == 1)
    diff = (Xw - Xp).abs().sum(dim=1).cpu().numpy()
    assert np.all(diff <= rw["cert_bound"] + rp["cert_bound"])


@pytest.mark.timeout(900)
def test_warm_start_gradients_at_1m(torch_cuda):
    """One training step with lr = 0 on the 1M-vertex training graph of the warm
    start (hub rows split over wavefronts, weight gradients summed in 1024-row
    chunks): loss and every gradient against the bf16-emulating FP64 oracle's
    forward and backward.  Targets are oracle PageRank vectors."""
    from paper_2112_01743_amd import Plan
    from paper_2112_01743_amd.binding import Model
    from oracle import mpnn as om
    torch = torch_cuda
    g = gg.chung_lu(1_000_000, 16, 2.1, seed=2112004, dmax=50000)
    _note(f"chung-lu n={g.n} nnz={g.nnz} max degree {int(np.diff(g.row_ptr).max())}")
    plan = Plan.from_graph(g, C)
    params = gg.mpnn_init(2112004)
    model = Model(plan, params)
    src = gg.random_sources(g.n, 2, seed=2112004)
    P = gg.source_personalization(g.n, src)
    T = oracle.pagerank_power(g, P.T, C, tol=1e-8)[0].T
    loss, grads = model.train_step(src, torch.as_tensor(np.ascontiguousarray(T), device="cuda"), lr=0.0,
                                   want_grads=True)
    p64 = {k: v.astype(np.float64) for k, v in params.items()}
    ref, loss_ref = None, 0.0
    for j, s in enumerate(src):
        x0, cache = om.mpnn_forward(g, p64, int(s), bf16=True)
        loss_ref += om.mpnn_l1(x0, T[j]) / len(src)
        gj = om.mpnn_backward(p64, cache, T[j], bf16=True)
        ref = gj if ref is None else {k: ref[k] + gj[k] for k in ref}
        del cache
    _note(f"loss {loss:.8f} oracle {loss_ref:.8f}")
    # the loss is an L1 distance, so |loss - loss_ref| <= ||x0_gpu - x0_oracle||_1, which
    # the forward parity at this size bounds by 1e-4 (bf16 roundings flipped by the
    # FP32 / FP64 accumulation difference; measured 5.5e-6 to 2e-5)
    assert abs(loss - loss_ref) <= 1e-4
    for k in ref:
        r = ref[k] / len(src)
        if k == "b_out":      # exactly zero in exact arithmetic (softmax shift invariance);
            # here a sum of 1M FP32 terms whose magnitudes add up to at most 2
            assert abs(grads[k][0]) <= 1e-5
            continue
        rel = np.linalg.norm(grads[k] - r) / np.linalg.norm(r)
        _note(f"grad {k}: relative difference {rel:.3e}")
        assert rel <= 1e-3, (k, rel)


@pytest.mark.timeout(600)
def test_directed_4m_sliced(torch_cuda):
    """The directed workload at its full size (the bench's graph and seed): the
    plan picks column slices by itself; the result is certified by the oracle's
    FP64 residual of (I - cP') x = (1-c) p (Sec. 2.1, ||(I - cP')^{-1}||_1 <=
    1/(1-c) for the column-stochastic P') and agrees with the row-order plan."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.directed_random(4_000_000, 16, 0.1, seed=2112020)
    _note(f"directed n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C, directed=1, time_kernels=1)
    assert plan.info()["column_slices"] == 8
    p = np.full(g.n, 1.0 / g.n)
    dp = torch.as_tensor(p, device="cuda")
    xs, rs = plan.solve_power(dp, TOL)
    xs = xs.cpu().numpy()
    del plan
    xr, rr = Plan.from_graph(g, C, directed=1, column_slices=1).solve_power(dp, TOL)
    xr = xr.cpu().numpy()
    P, d = oracle.transition_directed(g)
    r = (1 - C) * p - xs + C * (P @ xs + p * (d @ xs))
    bound = np.abs(r).sum() / (1 - C)
    _note(f"sliced: steps {rs['terms']}+{rs['refine_terms']} gpu bound {rs['cert_bound']:.3e} "
          f"oracle bound {bound:.3e}; row order steps {rr['terms']}")
    assert rs["certified"] == 1 and bound <= TOL
    assert np.abs(xs - xr).sum() <= 2 * TOL


@pytest.mark.timeout(600)
def test_column_slices_at_the_maximum_size(torch_cuda):
    """n = 8 (2^21 - 16) - 1, the largest plan the column-sliced path takes:
    a slice holds 2,097,135 vertices, so the packed entries need 21 bits of
    local column and work items hold 2^11 rows (the sliced pass's 11-row-bit
    variant, which smaller graphs never reach).  A path through all vertices
    plus n/4 random chords (42M entries); certified by the oracle's residual."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    n = 8 * (2**21 - 16) - 1
    rng = gg.philox(2112040)
    u = np.arange(n - 1, dtype=np.int64)
    a, b = rng.integers(0, n, n // 4), rng.integers(0, n, n // 4)
    g = gg.csr_from_edges(n, np.concatenate([u, a]), np.concatenate([u + 1, b]))
    _note(f"n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C, column_slices=8)
    assert plan.info()["column_slices"] == 8 and plan.info()["reordered"] == 1
    P = np.stack([np.full(n, 1.0 / n), gg.source_personalization(n, [n // 3])[0]])
    X = []
    for p in P:
        x, rep = plan.solve(torch.as_tensor(p, device="cuda"), TOL)
        _note(f"terms {rep['terms']}+{rep['refine_terms']} bound {rep['cert_bound']:.3e}")
        assert rep["certified"] == 1
        X.append(x.cpu().numpy())
    del plan
    bounds = _oracle_bound(g, (1 - C) * P, np.stack(X))
    _note(f"oracle bounds {bounds}")
    assert np.all(bounds <= TOL)


@pytest.mark.timeout(600)
def test_directed_column_slices_at_the_maximum_size(torch_cuda):
    """The directed power method at the column-sliced path's largest n (11
    row bits, 21-bit local columns) through the sliced step and the sliced
    FP64 residual; certified by the oracle's residual of (I - cP')x = (1-c)p."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    n = 8 * (2**21 - 16) - 1
    g = gg.directed_random(n, 2.5, 0.1, seed=2112041)
    _note(f"directed n={g.n} nnz={g.nnz}")
    plan = Plan.from_graph(g, C, directed=1)
    assert plan.info()["column_slices"] == 8
    p = np.full(n, 1.0 / n)
    x, rep = plan.solve(torch.as_tensor(p, device="cuda"), TOL)
    _note(f"steps {rep['terms']}+{rep['refine_terms']} method {rep['method']} "
          f"bound {rep['cert_bound']:.3e}")
    assert rep["certified"] == 1 and rep["method"] == 1
    x = x.cpu().numpy()
    del plan
    P, d = oracle.transition_directed(g)
    bound = np.abs((1 - C) * p - x + C * (P @ x + p * (d @ x))).sum() / (1 - C)
    _note(f"oracle bound {bound:.3e}")
    assert bound <= TOL
