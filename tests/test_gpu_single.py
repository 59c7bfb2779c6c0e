"""GPU parity of the single-vector CPAA path (cpaa_solve) against the FP64 oracle.

Bar: ||x - pi||_1 <= tol (1e-6 unless stated), and the library's own FP64
certificate must bound the true error.  pi comes from the oracle's dense solve
(small graphs) or its power method certified to 1e-13.
"""
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
    binding.lib()      # raises if the HIP library is missing
    return torch


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _truth(g, p):
    if g.n <= 2500:
        return oracle.pagerank_exact(g, p, C)
    return oracle.pagerank_power(g, p, C, tol=1e-13)[0]


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _solve(torch, g, p, tol=1e-6, x0=None, **opts):
    from paper_2112_01743_amd import Plan
    plan = Plan.from_graph(g, C, **opts)
    x, rep = plan.solve(_dev(torch, p), tol, None if x0 is None else _dev(torch, x0))
    torch.cuda.synchronize()
    return x.cpu().numpy(), rep, plan


def _assert_parity(g, p, x, rep, tol):
    pi = _truth(g, p)
    err = np.abs(x - pi).sum()
    assert rep["status"] == "CPAA_OK", rep
    assert rep["certified"] == 1
    assert err <= tol, (err, rep)
    # the certificate is rigorous for the returned x; 2e-13 covers the error of the truth
    assert err <= rep["cert_bound"] * (1 + 1e-9) + 2e-13, (err, rep)
    return err


SMALL = {
    "cycle7": lambda: gg.cycle(7),
    "path6": lambda: gg.path(6),
    "star6": lambda: gg.star(6),
    "complete5": lambda: gg.complete(5),
    "edge2": lambda: gg.path(2),
    "random60": lambda: gg.random_connected(60, 6.0, seed=13),
    "random777": lambda: gg.random_connected(777, 5.0, seed=14),
    "er2000": lambda: gg.erdos_renyi(2000, 10, seed=2),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_small_graphs_uniform_and_source(torch_cuda, name, tol):
    g = SMALL[name]()
    _note(f"case {name} n={g.n} nnz={g.nnz} tol={tol}")
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n // 2])[0]):
        x, rep, _ = _solve(torch_cuda, g, p, tol)
        _assert_parity(g, p, x, rep, tol)


def test_config0_er_10k_tail_1e10(torch_cuda):
    """Erdos-Renyi n=10,000, average degree 10, p = e/n; terms chosen so the
    coefficient tail is below 1e-10 and the result certified to 1e-10."""
    g = gg.erdos_renyi(10000, 10, seed=2112000)
    _note(f"config0 n={g.n} nnz={g.nnz}")
    p = gg.uniform_personalization(g.n)
    x, rep, _ = _solve(torch_cuda, g, p, 1e-10)
    pi = oracle.pagerank_power(g, p, C, tol=1e-14)[0]
    err = np.abs(x - pi).sum()
    assert rep["certified"] == 1 and err <= 1e-10, (err, rep)
    assert rep["terms"] + rep["refine_terms"] >= oracle.terms_for_mass_error(C, 1e-10) - 5


def test_series_term_parity_with_oracle_cpaa(torch_cuda):
    """With the term count pinned (k_max = M, no refinement) the GPU result is
    the FP32-recurrence value of x_M; it must match the oracle's FP64 x_M to
    the FP32 rounding level."""
    g = gg.chung_lu(5000, 8, 2.5, seed=77)
    p = gg.source_personalization(g.n, [3])[0]
    for M in (1, 2, 5, 12, 30):
        x, rep, _ = _solve(torch_cuda, g, p, 1e-14, k_max=M, max_refine=0)
        assert rep["terms"] == M and rep["refinements"] == 0
        ref = oracle.cpaa(g, (1 - C) * p, C, M)
        err = np.abs(x - ref).sum()
        _note(f"M={M} term-parity L1={err:.3e}")
        assert err <= 2e-6 * max(1.0, np.abs(ref).sum()), (M, err)


def test_hub_rows_split_across_workgroups(torch_cuda):
    """A star with 20,000 leaves plus a ring among the leaves: the hub row is
    longer than one work item and is cut into chunks (atomic fix-up)."""
    n = 20001
    leaves = np.arange(1, n)
    u = np.concatenate([np.zeros(n - 1, dtype=np.int64), leaves])
    v = np.concatenate([leaves, np.roll(leaves, 1)])
    g = gg.csr_from_edges(n, u, v)
    from paper_2112_01743_amd import Plan
    info = Plan.from_graph(g, C).info()
    assert info["split_rows"] >= 1
    for p in (gg.uniform_personalization(n), gg.source_personalization(n, [0])[0],
              gg.source_personalization(n, [17])[0]):
        for rep_i in range(2):     # second solve checks the split slots were reset
            x, rep, _ = _solve(torch_cuda, g, p, 1e-7)
            _assert_parity(g, p, x, rep, 1e-7)


def test_power_law_mid_size(torch_cuda):
    g = gg.chung_lu(200000, 16, 2.1, seed=2112001, dmax=50000)
    _note(f"chung-lu n={g.n} nnz={g.nnz} maxdeg={np.diff(g.row_ptr).max()}")
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [0])[0],
              gg.source_personalization(g.n, [g.n - 1])[0]):
        x, rep, _ = _solve(torch_cuda, g, p, 1e-6)
        _assert_parity(g, p, x, rep, 1e-6)


@pytest.mark.parametrize("npt", [4, 8, 16])
def test_work_item_sizes_agree(torch_cuda, npt):
    g = gg.chung_lu(30000, 12, 2.3, seed=5, dmax=8000)
    p = gg.uniform_personalization(g.n)
    x, rep, _ = _solve(torch_cuda, g, p, 1e-8, nnz_per_thread=npt)
    _assert_parity(g, p, x, rep, 1e-8)


@pytest.mark.parametrize("shape", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("case", ["chung_lu", "grid", "star", "path", "complete", "big_star"])
def test_column_sliced_term_agrees(torch_cuda, case, shape):
    """Column-sliced term (relabelled vertices, one column slice per XCD, a
    partial sum per row and slice with entries, combined per term), forced on
    graphs of every shape and with every launch shape of its gather pass;
    big_star's centre has more entries per slice than a wave item holds (long
    row cut into chunks), chung_lu has more rows than the LDS hub of every
    shape."""
    g = {"chung_lu": lambda: gg.chung_lu(300000, 12, 2.1, seed=5, dmax=20000),
         "grid": lambda: gg.perturbed_grid(150, 0.05, 0.01, seed=4),
         "star": lambda: gg.star(40), "path": lambda: gg.path(7),
         "complete": lambda: gg.complete(30), "big_star": lambda: gg.star(100000)}[case]()
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n // 2])[0],
              gg.source_personalization(g.n, [0])[0]):
        x, rep, plan = _solve(torch_cuda, g, p, 1e-9, column_slices=8, slice_shape=shape)
        info = plan.info()
        assert info["column_slices"] == 8 and info["reordered"] == 1
        assert info["slice_shape"] == shape
        _assert_parity(g, p, x, rep, 1e-9)


@pytest.mark.parametrize("shape", [1, 4])
def test_column_sliced_term_parity_with_oracle_cpaa(torch_cuda, shape):
    """Pinned term counts on the column-sliced path: the FP32-recurrence x_M
    against the oracle's FP64 x_M (hubs split into chunks, rows spread over
    every slice)."""
    g = gg.chung_lu(200000, 10, 2.1, seed=78, dmax=30000)
    p = gg.source_personalization(g.n, [3])[0]
    for M in (1, 2, 5, 12, 30):
        x, rep, _ = _solve(torch_cuda, g, p, 1e-14, k_max=M, max_refine=0, column_slices=8,
                           slice_shape=shape)
        assert rep["terms"] == M and rep["refinements"] == 0
        ref = oracle.cpaa(g, (1 - C) * p, C, M)
        err = np.abs(x - ref).sum()
        _note(f"shape={shape} M={M} term-parity L1={err:.3e}")
        assert err <= 2e-6 * max(1.0, np.abs(ref).sum()), (M, err)


def test_column_sliced_warm_start_and_host_io(torch_cuda):
    from paper_2112_01743_amd import Plan
    g = gg.chung_lu(30000, 10, 2.2, seed=31)
    p = gg.source_personalization(g.n, [5])[0]
    pi = _truth(g, p)
    guess = np.abs(pi * (1 + 1e-3 * gg.philox(2).standard_normal(g.n)))
    guess /= guess.sum()
    _, plain, _ = _solve(torch_cuda, g, p, 1e-9, column_slices=8)
    x, rep, _ = _solve(torch_cuda, g, p, 1e-9, x0=guess, column_slices=8)
    assert rep["fallback_used"] == 0 and rep["terms"] < plain["terms"]
    _assert_parity(g, p, x, rep, 1e-9)
    from paper_2112_01743_amd import binding as B
    plan = Plan.from_graph(g, C, column_slices=8, io_device=0)
    ph = np.ascontiguousarray(p)
    xh = np.zeros(g.n)
    st, reph = B.cpaa_solve(plan.handle, ph.ctypes.data, 1e-9, None, xh.ctypes.data)
    assert st == B.CPAA_OK, B.cpaa_last_error()
    reph = dict(reph.as_dict(), status="CPAA_OK")
    _assert_parity(g, p, xh, reph, 1e-9)


def _two_cycles():
    i = np.arange(9)
    u = np.concatenate([i, 9 + np.arange(14)])
    v = np.concatenate([(i + 1) % 9, 9 + (np.arange(14) + 1) % 14])
    return gg.csr_from_edges(23, u, v)


@pytest.mark.parametrize("case", ["delaunay", "chung_lu", "grid", "two_cycles", "star", "path"])
def test_rcm_relabelled_term_agrees(torch_cuda, case):
    """Row-order term on reverse Cuthill-McKee labels (forced), on graphs of
    every shape, disconnected ones included; p, x0 and x stay in the caller's
    labels."""
    g = {"delaunay": lambda: gg.delaunay(20000, seed=3),
         "chung_lu": lambda: gg.chung_lu(30000, 10, 2.2, seed=31),
         "grid": lambda: gg.perturbed_grid(120, 0.05, 0.01, seed=4),
         "two_cycles": _two_cycles, "star": lambda: gg.star(40), "path": lambda: gg.path(7)}[case]()
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n // 2])[0],
              gg.source_personalization(g.n, [0])[0]):
        x, rep, plan = _solve(torch_cuda, g, p, 1e-9, locality_order=2)
        info = plan.info()
        assert info["reordered"] == 2 and info["column_slices"] == 1
        _assert_parity(g, p, x, rep, 1e-9)


def test_rcm_auto_on_random_order_mesh_only(torch_cuda):
    """Auto: a Delaunay mesh in random point order (n = 300k) is relabelled and
    solved to 1e-7 (CPAA and the power method, plain and warm-started); a lattice
    in its natural row-major order (n = 360k) keeps the caller's labels."""
    from paper_2112_01743_amd import Plan
    g = gg.delaunay(300000, seed=7)
    plan = Plan.from_graph(g, C)
    assert plan.info()["reordered"] == 2
    p = gg.source_personalization(g.n, [123])[0]
    pi = _truth(g, p)
    x, rep = plan.solve(_dev(torch_cuda, p), 1e-7)
    _assert_parity(g, p, x.cpu().numpy(), rep, 1e-7)
    x, rep = plan.solve_power(_dev(torch_cuda, p), 1e-7)
    _assert_parity(g, p, x.cpu().numpy(), rep, 1e-7)
    guess = np.abs(pi * (1 + 1e-3 * gg.philox(2).standard_normal(g.n)))
    x, rep = plan.solve(_dev(torch_cuda, p), 1e-7, _dev(torch_cuda, guess))
    assert rep["fallback_used"] == 0
    _assert_parity(g, p, x.cpu().numpy(), rep, 1e-7)
    grid = gg.perturbed_grid(600, 0.05, 0.0, seed=5)
    assert Plan.from_graph(grid, C).info()["reordered"] == 0


def _lambda_min(g):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    d = np.diff(g.row_ptr).astype(float)
    A = sp.csr_matrix((np.ones(g.nnz), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    S = sp.diags(1 / np.sqrt(d)) @ A @ sp.diags(1 / np.sqrt(d))
    return float(spl.eigsh(S, k=1, which="SA", tol=1e-8, return_eigenvectors=False)[0])


@pytest.mark.parametrize("case", ["er", "delaunay", "chung_lu"])
def test_spectral_interval(torch_cuda, case):
    """Expansion on [a, 1], a from the plan's Lanczos estimate: a sits just below
    lambda_min(P) on graphs whose spectrum stays away from -1 and the solves need
    fewer terms; a graph with a bipartite component keeps [-1, 1].  Pinned-term
    results match the oracle's interval series with the same a."""
    from paper_2112_01743_amd import Plan
    g = {"er": lambda: gg.erdos_renyi(20000, 10, seed=12),
         "delaunay": lambda: gg.delaunay(30000, seed=5),
         "chung_lu": lambda: gg.chung_lu(30000, 10, 2.1, seed=2112001, dmax=3000)}[case]()
    lam = _lambda_min(g)
    plan = Plan.from_graph(g, C, spectral_interval=1)
    a = plan.info()["spectrum_lo"]
    _note(f"{case}: lambda_min {lam:.4f}, interval from {a:.4f}")
    if lam < -0.97:
        assert a == -1.0
    else:
        assert lam - 0.03 <= a <= lam
    base = Plan.from_graph(g, C)
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n // 2])[0]):
        x, rep = plan.solve(_dev(torch_cuda, p), 1e-9)
        _assert_parity(g, p, x.cpu().numpy(), rep, 1e-9)
        _, rep0 = base.solve(_dev(torch_cuda, p), 1e-9)
        tot, tot0 = rep["terms"] + rep["refine_terms"], rep0["terms"] + rep0["refine_terms"]
        _note(f"  terms {tot} (interval) vs {tot0}")
        assert tot <= tot0 if a == -1.0 else tot < tot0
    p = gg.source_personalization(g.n, [7])[0]
    for M in (3, 12):
        pm = Plan.from_graph(g, C, spectral_interval=1, k_max=M, max_refine=0)
        x, _ = pm.solve(_dev(torch_cuda, p), 1e-15)
        ref = oracle.cpaa_interval(g, (1 - C) * p, C, a, M)
        assert np.abs(x.cpu().numpy() - ref).sum() <= 2e-6, M


def test_spectral_interval_batched(torch_cuda):
    from paper_2112_01743_amd import Plan
    g = gg.erdos_renyi(3000, 12, seed=4)
    src = gg.random_sources(g.n, 70, seed=8)
    Pm = gg.source_personalization(g.n, src)
    plan = Plan.from_graph(g, C, spectral_interval=1)
    assert plan.info()["spectrum_lo"] > -0.9
    X, reps = plan.solve_batched(_dev(torch_cuda, Pm), 1e-8)
    pi = oracle.pagerank_exact(g, Pm.T, C)
    err = np.abs(X.cpu().numpy().T - pi).sum(axis=0)
    assert np.all(reps["certified"] == 1) and err.max() <= 1e-8
    assert np.all(err <= reps["cert_bound"] * (1 + 1e-9) + 2e-13)


def test_autotuned_work_items(torch_cuda):
    """The autotuner times candidate work-item sizes on the first plain solve,
    keeps the fastest, and every later solve uses it."""
    g = gg.chung_lu(60000, 12, 2.2, seed=17, dmax=10000)
    p = gg.uniform_personalization(g.n)
    x, rep, plan = _solve(torch_cuda, g, p, 1e-8, autotune=1)
    npt = plan.info()["nnz_per_thread"]
    _note(f"autotuned nnz_per_thread={npt}")
    assert npt in (8, 16, 32)
    _assert_parity(g, p, x, rep, 1e-8)
    q = gg.source_personalization(g.n, [11])[0]
    x2, rep2 = plan.solve(_dev(torch_cuda, q), 1e-8)
    assert plan.info()["nnz_per_thread"] == npt
    _assert_parity(g, q, x2.cpu().numpy(), rep2, 1e-8)


@pytest.mark.parametrize("remap", [0, 1])
def test_xcd_remap_agrees(torch_cuda, remap):
    g = gg.perturbed_grid(120, 0.05, 0.01, seed=9)
    p = gg.source_personalization(g.n, [g.n // 3])[0]
    x, rep, _ = _solve(torch_cuda, g, p, 1e-7, xcd_remap=remap)
    _assert_parity(g, p, x, rep, 1e-7)


def test_warm_start_good_guess_needs_fewer_terms(torch_cuda):
    g = gg.chung_lu(20000, 10, 2.2, seed=31)
    p = gg.source_personalization(g.n, [5])[0]
    pi = _truth(g, p)
    _, plain, _ = _solve(torch_cuda, g, p, 1e-7)
    rng = gg.philox(3)
    x0 = np.abs(pi * (1 + 1e-3 * rng.standard_normal(g.n)))
    x0 /= x0.sum()
    x, rep, _ = _solve(torch_cuda, g, p, 1e-7, x0=x0)
    _assert_parity(g, p, x, rep, 1e-7)
    assert rep["fallback_used"] == 0
    assert rep["terms"] < plain["terms"], (rep["terms"], plain["terms"])


@pytest.mark.parametrize("kind", ["nan", "zeros", "bad"])
def test_warm_start_fallback(torch_cuda, kind):
    g = gg.random_connected(300, 5.0, seed=8)
    p = gg.source_personalization(g.n, [7])[0]
    x0 = {"nan": np.full(g.n, np.nan), "zeros": np.zeros(g.n),
          "bad": np.full(g.n, 50.0)}[kind]
    x, rep, _ = _solve(torch_cuda, g, p, 1e-8, x0=x0)
    assert rep["fallback_used"] == 1
    _assert_parity(g, p, x, rep, 1e-8)


def test_normalize_matches_alg1_final_step(torch_cuda):
    g = gg.random_connected(500, 6.0, seed=4)
    p = gg.uniform_personalization(g.n)
    x, rep, _ = _solve(torch_cuda, g, p, 1e-9, normalize=1)
    assert abs(x.sum() - 1.0) < 1e-12
    assert np.abs(x - _truth(g, p)).sum() < 1e-9


def test_host_pointer_io(torch_cuda):
    from paper_2112_01743_amd import binding as B
    g = gg.random_connected(400, 5.0, seed=6)
    p = np.ascontiguousarray(gg.source_personalization(g.n, [9])[0])
    x = np.zeros(g.n)
    plan = B.Plan.from_graph(g, C, io_device=0)
    st, rep = B.cpaa_solve(plan.handle, p.ctypes.data, 1e-8, None, x.ctypes.data)
    assert st == B.CPAA_OK, B.cpaa_last_error()
    assert np.abs(x - _truth(g, p)).sum() <= 1e-8


def test_invalid_personalization_rejected(torch_cuda):
    from paper_2112_01743_amd import binding as B
    g = gg.cycle(10)
    from paper_2112_01743_amd import Plan
    plan = Plan.from_graph(g, C)
    out = torch_cuda.full((g.n,), 7.0, dtype=torch_cuda.float64, device="cuda")
    for bad in (np.full(g.n, 0.2), np.r_[-0.1, np.full(g.n - 1, 1.1 / (g.n - 1))],
                np.r_[np.nan, np.full(g.n - 1, 1.0 / (g.n - 1))]):
        st, _ = B.cpaa_solve(plan.handle, _dev(torch_cuda, bad).data_ptr(), 1e-6, None,
                             out.data_ptr())
        assert st == B.CPAA_EINVAL
        assert float(out[0]) == 7.0     # outputs untouched on error
    st, _ = B.cpaa_solve(plan.handle, _dev(torch_cuda, np.full(g.n, 0.1)).data_ptr(), -1.0, None,
                         out.data_ptr())
    assert st == B.CPAA_EINVAL


def test_term_cap_reports_noconv_with_best_effort(torch_cuda):
    g = gg.random_connected(300, 5.0, seed=12)
    p = gg.uniform_personalization(g.n)
    x, rep, _ = _solve(torch_cuda, g, p, 1e-9, k_max=3, max_refine=0)
    assert rep["status"] == "CPAA_ENOCONV" and rep["certified"] == 0
    ref = oracle.cpaa(g, (1 - C) * p, C, 3)
    assert np.abs(x - ref).sum() < 1e-6
    err = np.abs(x - _truth(g, p)).sum()
    assert err <= rep["cert_bound"] * (1 + 1e-9) + 2e-13


def test_repeated_solves_reuse_plan(torch_cuda):
    from paper_2112_01743_amd import Plan
    g = gg.chung_lu(50000, 16, 2.1, seed=44, dmax=20000)
    plan = Plan.from_graph(g, C)
    p = _dev(torch_cuda, gg.uniform_personalization(g.n))
    outs = [plan.solve(p, 1e-6)[0].cpu().numpy() for _ in range(3)]
    truth = _truth(g, gg.uniform_personalization(g.n))
    # split hub rows meet through FP32 atomics, so runs agree to rounding, not bitwise
    for o in outs:
        assert np.abs(o - truth).sum() <= 1e-6
    assert np.abs(outs[0] - outs[1]).sum() < 1e-7 and np.abs(outs[1] - outs[2]).sum() < 1e-7


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("slices", [1, 8])
def test_kernel_timing_report(torch_cuda, mode, slices):
    """time_kernels = 1 (events around every term launch) and 2 (around each
    series): both count every term launch that did work, and the series
    brackets hold the per-term ones' launches, so their total is no larger
    than the solve's."""
    g = gg.chung_lu(100000, 16, 2.1, seed=45, dmax=30000)
    p = gg.uniform_personalization(g.n)
    x, rep, _ = _solve(torch_cuda, g, p, 1e-6, time_kernels=mode, column_slices=slices)
    assert rep["term_launches"] == rep["terms"] + rep["refine_terms"]
    assert rep["ms_terms"] > 0 and rep["ms_total"] >= rep["ms_terms"]
    assert rep["edges"] == g.nnz * (rep["terms"] + rep["refine_terms"])
    _assert_parity(g, p, x, rep, 1e-6)


def test_independent_plans_on_two_streams(torch_cuda):
    """Different plans are independent: solves issued from two threads on two
    torch streams (default priority) give the same results as alone."""
    import threading
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g1 = gg.chung_lu(40000, 12, 2.2, seed=51, dmax=8000)
    g2 = gg.perturbed_grid(150, 0.05, 0.01, seed=52)
    cases = [(Plan.from_graph(g1, C), g1, gg.source_personalization(g1.n, [7])[0]),
             (Plan.from_graph(g2, C), g2, gg.uniform_personalization(g2.n))]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    out = [None, None]

    def run(i):
        plan, g, p = cases[i]
        with torch.cuda.stream(streams[i]):
            pd = _dev(torch, p)
            for _ in range(3):
                x, rep = plan.solve(pd, 1e-8, stream=streams[i])
            out[i] = (x.cpu().numpy(), rep)

    threads = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for i, (plan, g, p) in enumerate(cases):
        x, rep = out[i]
        _assert_parity(g, p, x, rep, 1e-8)


@pytest.mark.parametrize("name,g", [
    ("chung_lu", lambda: gg.chung_lu(20000, 10, 2.1, seed=9, dmax=5000)),
    ("grid", lambda: gg.perturbed_grid(80, 0.05, 0.01, seed=3)),
    ("star", lambda: gg.star(3000)),
])
def test_fp64_recurrence_matches_oracle_terms(torch_cuda, name, g):
    """fp64_recurrence = 1 (the debug mode): with the term count pinned the
    result is the oracle's FP64 x_M up to rounding order (1e-12 in L1), for
    the Chebyshev series and for the power method's iterates; the star has a
    hub split across workgroups."""
    g = g()
    p = gg.source_personalization(g.n, [g.n // 3])[0]
    for M in (1, 2, 5, 12, 30):
        x, rep, plan = _solve(torch_cuda, g, p, 1e-15, k_max=M, max_refine=0, fp64_recurrence=1)
        assert plan.info()["column_slices"] == 1
        assert rep["terms"] == M and rep["refinements"] == 0
        ref = oracle.cpaa(g, (1 - C) * p, C, M)
        err = np.abs(x - ref).sum()
        _note(f"{name} fp64 M={M} L1={err:.3e}")
        assert err <= 1e-12, (M, err)
    ref = oracle.power_method(g, p, C, 20, return_all=True)
    from paper_2112_01743_amd import Plan
    for t in (1, 7, 20):
        plan = Plan.from_graph(g, C, k_max=t, max_refine=0, fp64_recurrence=1)
        xp, rp = plan.solve_power(_dev(torch_cuda, p), 1e-15)
        assert rp["terms"] == t
        err = np.abs(xp.cpu().numpy() - ref[t]).sum()
        _note(f"{name} fp64 power t={t} L1={err:.3e}")
        assert err <= 1e-12, (t, err)


def test_fp64_recurrence_batched_and_certified(torch_cuda):
    """Batched calls on an FP64-recurrence plan solve column by column and
    certify to a tolerance the FP32 recurrence cannot reach in one series."""
    from paper_2112_01743_amd import Plan
    g = gg.chung_lu(8000, 8, 2.3, seed=21)
    src = [0, 17, 4000]
    P = gg.source_personalization(g.n, src)
    plan = Plan.from_graph(g, C, fp64_recurrence=1, max_refine=0)
    X, reps = plan.solve_batched(_dev(torch_cuda, P), 1e-11)
    ref = oracle.pagerank_power(g, P.T, C, tol=1e-14)[0].T
    errs = np.abs(X.cpu().numpy() - ref).sum(axis=1)
    _note(f"fp64 batched errors {errs}")
    assert all(r["certified"] for r in reps) and errs.max() <= 1e-11
    for j, s in enumerate(src):
        x, rep = plan.solve(_dev(torch_cuda, P[j]), 1e-11)
        assert np.abs(x.cpu().numpy() - X[j].cpu().numpy()).sum() <= 1e-14


def test_fp64_recurrence_option_checks(torch_cuda):
    from paper_2112_01743_amd import Plan, binding as B
    g = gg.chung_lu(2000, 8, 2.3, seed=3)
    with pytest.raises(B.CpaaError):
        Plan.from_graph(g, C, fp64_recurrence=1, column_slices=8)
    with pytest.raises(B.CpaaError):
        Plan.from_graph(g, C, fp64_recurrence=1, deterministic=1)


@pytest.mark.parametrize("name,g", [
    ("chung_lu", lambda: gg.chung_lu(200000, 12, 2.1, seed=41, dmax=30000)),
    ("big_star", lambda: gg.star(100000)),
])
def test_deterministic_solves_are_bitwise_equal(torch_cuda, name, g):
    """deterministic = 1: two solves of the same input, on the same plan and on
    a second plan, give identical bits (hub rows split into chunks in the
    column-sliced term and in the residual, every reduction in block order),
    and the result is certified against the oracle like any other."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = g()
    plan = Plan.from_graph(g, C, deterministic=1)
    assert plan.info()["column_slices"] == 8 and plan.info()["slice_shape"] > 0
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [1])[0]):
        pd = _dev(torch, p)
        x1, r1 = plan.solve(pd, 1e-9)
        x2, r2 = plan.solve(pd, 1e-9)
        x3, r3 = Plan.from_graph(g, C, deterministic=1).solve(pd, 1e-9)
        a, b, c = (v.cpu().numpy() for v in (x1, x2, x3))
        assert np.array_equal(a, b) and np.array_equal(a, c)
        assert r1["cert_bound"] == r2["cert_bound"] == r3["cert_bound"]
        assert r1["terms"] == r3["terms"] and r1["refine_terms"] == r3["refine_terms"]
        _assert_parity(g, p, a, r1, 1e-9)
        # a warm start and the power method are deterministic too
        xw1, _ = plan.solve(pd, 1e-9, x0=x1)
        xw2, _ = plan.solve(pd, 1e-9, x0=x1)
        assert np.array_equal(xw1.cpu().numpy(), xw2.cpu().numpy())
        xp1, _ = plan.solve_power(pd, 1e-7)
        xp2, _ = plan.solve_power(pd, 1e-7)
        assert np.array_equal(xp1.cpu().numpy(), xp2.cpu().numpy())
    # batched calls solve column by column: each column equals its single solve
    P = gg.source_personalization(g.n, [0, 5, g.n - 1])
    X, reps = plan.solve_batched(_dev(torch, P), 1e-9)
    for j in range(P.shape[0]):
        xj, _ = plan.solve(_dev(torch, P[j]), 1e-9)
        assert np.array_equal(X[j].cpu().numpy(), xj.cpu().numpy())


def test_launch_shapes_give_identical_bits_and_autotune_keeps_one(torch_cuda):
    """The launch shape of the hub-sliced gather pass (workgroup size, LDS hub
    size) changes a term's time, not its result: with
    deterministic sums every shape returns the same bits.  autotune = 1 times
    the shapes on the first solve and keeps one; later solves are unchanged."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(300000, 12, 2.1, seed=43, dmax=30000)
    pd = _dev(torch, gg.source_personalization(g.n, [7])[0])
    ref = None
    for shape in range(1, 5):
        plan = Plan.from_graph(g, C, deterministic=1, slice_shape=shape)
        assert plan.info()["slice_shape"] == shape
        x, rep = plan.solve(pd, 1e-9)
        x = x.cpu().numpy()
        if ref is None:
            ref = (x, rep)
            _assert_parity(g, pd.cpu().numpy(), x, rep, 1e-9)
        else:
            assert np.array_equal(x, ref[0]), shape
            assert rep["cert_bound"] == ref[1]["cert_bound"]
    plan = Plan.from_graph(g, C, deterministic=1, autotune=1)
    x1, _ = plan.solve(pd, 1e-9)
    kept = plan.info()["slice_shape"]
    assert 1 <= kept <= 4
    x2, _ = plan.solve(pd, 1e-9)
    assert plan.info()["slice_shape"] == kept
    assert np.array_equal(x1.cpu().numpy(), ref[0]) and np.array_equal(x2.cpu().numpy(), ref[0])


@pytest.mark.parametrize("rows", [1, 5, 64])
def test_rows_per_wave_caps_the_items(torch_cuda, rows):
    """rows_per_wave caps the present rows of a wave item of the column-sliced
    map (the default is 1,024): more, shorter items, the same solution to the
    solve's bound, and deterministic solves stay bitwise repeatable."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(200000, 12, 2.1, seed=49, dmax=30000)
    p = gg.source_personalization(g.n, [11])[0]
    plan = Plan.from_graph(g, C, column_slices=8, rows_per_wave=rows, deterministic=1)
    x1, r1 = plan.solve(_dev(torch, p), 1e-9)
    x2, _ = plan.solve(_dev(torch, p), 1e-9)
    a = x1.cpu().numpy()
    assert np.array_equal(a, x2.cpu().numpy())
    _assert_parity(g, p, a, r1, 1e-9)


def _host_residual_l1(g, p, x):
    """||(1-c) p - (I - cP) x||_1 in FP64 on the host, P x = A D^-1 x."""
    deg = np.diff(g.row_ptr).astype(np.float64)
    y = x / deg
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    ay = np.bincount(rows, weights=y[g.col_idx], minlength=g.n)
    return np.abs((1 - C) * p - x + C * ay).sum()


@pytest.mark.parametrize("deterministic", [0, 1])
def test_sliced_fp64_residual_matches_row_order_and_host(torch_cuda, deterministic):
    """The FP64 residual of hub-sliced plans (partial sums of acc per column
    slice on the term's map, long rows in chunks, then r = b - (I - cP) x per
    row) against the row-order residual of the same plan (the static-workspace
    entry point keeps it) and against r recomputed on the host; with a capped
    series the residual also drives the correction series."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(300000, 12, 2.1, seed=47, dmax=30000)
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [5])[0]):
        pd = _dev(torch, p)
        for opts in ({}, {"k_max": 10, "max_refine": 6}):
            plan = Plan.from_graph(g, C, column_slices=8, deterministic=deterministic, **opts)
            x1, r1 = plan.solve(pd, 1e-9)
            x2, r2 = plan.solve_noalloc(pd, 1e-9)
            a, b = x1.cpu().numpy(), x2.cpu().numpy()
            host = _host_residual_l1(g, p, a)
            _note(f"resid sliced {r1['resid_l1']:.6e} row-order {r2['resid_l1']:.6e} "
                  f"host {host:.6e} refinements {r1['refinements']}")
            assert abs(r1["resid_l1"] - host) <= 1e-6 * host + 1e-15
            if opts:
                assert r1["refinements"] >= 1
            if r1["refinements"] == r2["refinements"] == 0:
                assert np.array_equal(a, b)
                assert abs(r1["resid_l1"] - r2["resid_l1"]) <= 1e-9 * host + 1e-16
            else:
                assert np.abs(a - b).sum() <= 1e-12
            _assert_parity(g, p, a, r1, 1e-9)


def _with_isolated(base, n_iso, seed):
    """base plus n_iso edgeless vertices at random labels; returns (graph, kept labels)."""
    n = base.n + n_iso
    iso = np.sort(gg.philox(seed).choice(n, n_iso, replace=False))
    keep = np.setdiff1d(np.arange(n), iso)
    rows = np.repeat(np.arange(base.n), np.diff(base.row_ptr))
    u, v = keep[rows], keep[base.col_idx]
    m = u < v
    return gg.csr_from_edges(n, u[m], v[m]), keep, iso


@pytest.mark.parametrize("opts", [{}, {"column_slices": 8}, {"deterministic": 1},
                                  {"normalize": 1}])
def test_drop_isolated_matches_oracle_on_kept_vertices(torch_cuda, opts):
    """drop_isolated = 1 on a graph with edgeless vertices: P has a zero column
    there, so the kept vertices hold the PageRank of the graph without them for
    p restricted to them (the linear system (I - cP) x = (1-c) p), and each
    dropped vertex holds (1-c) p_v (Sec. 2.1); single and batched solves."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    base = gg.chung_lu(6000, 8, 2.3, seed=5)
    g, keep, iso = _with_isolated(base, 37, seed=3)
    assert np.all(np.diff(g.row_ptr)[iso] == 0)
    plan = Plan.from_graph(g, C, drop_isolated=1, **opts)
    assert plan.info()["n"] == g.n
    P = np.stack([gg.uniform_personalization(g.n),
                  gg.source_personalization(g.n, [keep[10]])[0],
                  gg.source_personalization(g.n, [iso[3]])[0]])
    X, reps = plan.solve_batched(_dev(torch, P), 1e-9)
    for j in range(P.shape[0]):
        want = np.zeros(g.n)
        want[keep] = oracle.pagerank_exact(base, P[j][keep], C) if base.n <= 2500 else \
            oracle.pagerank_power(base, P[j][keep], C, tol=1e-13)[0]
        want[iso] = (1 - C) * P[j][iso]
        if opts.get("normalize"):
            want /= want.sum()
        got = X[j].cpu().numpy()
        x1, r1 = plan.solve(_dev(torch, P[j]), 1e-9)
        assert np.abs(x1.cpu().numpy() - got).sum() <= 1e-12
        err = np.abs(got - want).sum()
        _note(f"drop_isolated {opts} column {j}: L1 {err:.2e}")
        assert reps[j]["certified"] == 1 and err <= 1e-9, (j, err)
        assert np.array_equal(got[iso], want[iso] if not opts.get("normalize") else got[iso])
    # without the option the plan refuses the graph
    from paper_2112_01743_amd import binding as B
    with pytest.raises(B.CpaaError):
        Plan.from_graph(g, C)
