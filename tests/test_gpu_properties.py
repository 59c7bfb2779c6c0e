"""Property-based parity on random small graphs (hypothesis, derandomized so
every run draws the same cases): connected or not, any damping in [0.05, 0.9],
any personalization, every plan option that changes the single-vector, batched
or power-method path.  Each GPU result must match the oracle's dense solve to
the requested tolerance and stay below the library's own certificate."""
import sys

import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402
from strategies import directed_graphs, graphs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_01743_amd import binding
    binding.lib()
    return torch


OPTIONS = [{}, {"column_slices": 8}, {"locality_order": 2}, {"spectral_interval": 1},
           {"nnz_per_thread": 4}, {"tile_w": 8}]


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@settings(max_examples=200, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(g=graphs(), c=st.floats(0.05, 0.9), opt=st.sampled_from(OPTIONS),
       pseed=st.integers(0, 2**31 - 1), method=st.sampled_from(["solve", "solve_power"]))
def test_random_graphs_match_dense_solve(torch_cuda, g, c, opt, pseed, method):
    from paper_2112_01743_amd import Plan
    rng = np.random.default_rng(pseed)
    p = rng.random(g.n) ** 3
    p /= p.sum()
    tol = 1e-9
    print(f"n={g.n} nnz={g.nnz} c={c:.3f} opt={opt} {method}", flush=True)
    sys.stdout.flush()
    plan = Plan.from_graph(g, c, **opt)
    pi = oracle.pagerank_exact(g, p, c)
    x, rep = getattr(plan, method)(_dev(torch_cuda, p), tol)
    err = np.abs(x.cpu().numpy() - pi).sum()
    assert rep["certified"] == 1 and err <= tol, (err, rep)
    assert err <= rep["cert_bound"] * (1 + 1e-9) + 1e-14
    # three columns at once through the batched path
    P = np.stack([p, gg.source_personalization(g.n, [0])[0],
                  gg.source_personalization(g.n, [g.n - 1])[0]])
    X, reps = getattr(plan, method + "_batched")(_dev(torch_cuda, P), tol)
    ref = oracle.pagerank_exact(g, P.T, c)
    errs = np.abs(X.cpu().numpy().T - ref).sum(axis=0)
    assert np.all(reps["certified"] == 1) and errs.max() <= tol, errs


@settings(max_examples=100, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(g=directed_graphs(), c=st.floats(0.05, 0.9), pseed=st.integers(0, 2**31 - 1),
       slices=st.sampled_from([1, 8]))
def test_random_directed_graphs_match_dense_solve(torch_cuda, g, c, pseed, slices):
    """Directed plans (dangling vertices, empty rows) through the power method,
    in row order or column-sliced."""
    from paper_2112_01743_amd import Plan
    rng = np.random.default_rng(pseed)
    p = rng.random(g.n) ** 3 + 1e-3
    p /= p.sum()
    print(f"directed n={g.n} nnz={g.nnz} c={c:.3f} slices={slices}", flush=True)
    plan = Plan.from_graph(g, c, directed=1, column_slices=slices)
    x, rep = plan.solve_power(_dev(torch_cuda, p), 1e-9)
    pi = oracle.pagerank_directed_exact(g, p, c)
    err = np.abs(x.cpu().numpy() - pi).sum()
    assert rep["certified"] == 1 and err <= 1e-9, (err, rep)
    assert err <= rep["cert_bound"] * (1 + 1e-9) + 1e-14
