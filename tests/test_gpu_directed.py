"""GPU parity of the power method on directed graphs with dangling vertices
(cpaa_solve_power on a plan with directed = 1) against the oracle's P''
iteration (eq. 2.1 from p) and its dense solve (Sec. 2.1's P' = P + p d^T).

Every case runs in row order (column_slices = 1, the fused k_term_dir) and
column-sliced (column_slices = 8: relabelled vertices, the sliced gather pass
and k_combine_dir).  Bar: pinned steps match the oracle's FP64 iterates to the
FP32 rounding level (step_bar below); certified solves are within tol and below
the library's bound."""
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


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _by_targets(n, edges):
    rows = [[] for _ in range(n)]
    for v, u in edges:
        rows[u].append(v)
    rp = np.zeros(n + 1, dtype=np.int32)
    for u in range(n):
        rp[u + 1] = rp[u] + len(set(rows[u]))
    ci = np.concatenate([np.asarray(sorted(set(r)), dtype=np.int32) for r in rows])
    return gg.CSR(n=n, row_ptr=rp, col_idx=ci)


def _hubs(n):
    """Most vertices point at 0 (an in-hub row longer than a work item), 0 points
    at every odd vertex, odd vertices at one more; vertices 2 mod 4 are dangling."""
    edges = [(v, 0) for v in range(1, n) if v % 4 != 2] + [(0, u) for u in range(1, n, 2)]
    edges += [(u, (u * 7 + 3) % n) for u in range(1, n, 2) if (u * 7 + 3) % n != u]
    return _by_targets(n, edges)


GRAPHS = {
    "three": lambda: _by_targets(3, [(0, 1), (0, 2), (1, 2)]),
    "random5000": lambda: gg.directed_random(5000, 6, 0.1, seed=4),
    "hubs20000": lambda: _hubs(20000),
    # in-hub of 75,000 entries: more per column slice than a sliced work item
    # holds, so the sliced term and residual passes split it too
    "hubs100000": lambda: _hubs(100000),
}


def step_bar(seq, t, c=C):
    """L1 bar for x_t of the FP32 increment path.  Step s rounds the increment
    delta_s = x_{s+1} - x_s to FP32 (z = D_out^+ delta) and sums each row in
    FP32; both errors scale with sum_v |z_v| dout_v = ||delta_s||_1, here 16
    units of 2^-24 per unit of increment mass (a blocked sum's typical error
    for rows of up to 15,000 entries; seen: under 4).  An error made at step s
    is carried by every later increment, (cP')^k e with ||cP'|| <= c in L1, so
    the accumulated x grows it at most 1/(1-c) times.  The 1e-14 floor covers
    the FP64 rounding of x_0 and of a fixed point (every delta_s = 0)."""
    mass = sum(np.abs(seq[s + 1] - seq[s]).sum() for s in range(t))
    return 16 * 2.0**-24 * mass / (1 - c) + 1e-14


def _plan(g, **opts):
    from paper_2112_01743_amd import Plan
    return Plan.from_graph(g, C, directed=1, **opts)


@pytest.mark.parametrize("slices", [1, 8])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_directed_steps_match_oracle(torch_cuda, name, slices):
    g = GRAPHS[name]()
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n - 1])[0]):
        ref = oracle.power_method_directed(g, p, C, 30, return_all=True)
        for t in (1, 2, 7, 30):
            _note(f"case {name} n={g.n} nnz={g.nnz} t={t} slices={slices}")
            plan = _plan(g, k_max=t, max_refine=0, column_slices=slices)
            assert plan.info()["column_slices"] == slices
            x, rep = plan.solve_power(_dev(torch_cuda, p), 1e-15)
            err = np.abs(x.cpu().numpy() - ref[t]).sum()
            # an earlier stop happens only at a fixed point (x_0 = p = pi when p
            # sits on a dangling vertex of the three-vertex graph), where err is 0
            bar = step_bar(ref, t)
            _note(f"  err {err:.3e} bar {bar:.3e}")
            assert rep["terms"] <= t and err <= bar, (name, t, err, bar)


@pytest.mark.parametrize("slices", [1, 8])
@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_directed_certified_solve(torch_cuda, name, tol, slices):
    g = GRAPHS[name]()
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n // 2])[0]):
        pi = (oracle.pagerank_directed_exact(g, p, C) if g.n <= 5000 else
              oracle.power_method_directed(g, p, C, int(np.log(1e-15) / np.log(C)) + 1))
        x, rep = _plan(g, column_slices=slices).solve_power(_dev(torch_cuda, p), tol)
        err = np.abs(x.cpu().numpy() - pi).sum()
        _note(f"{name} tol={tol} slices={slices}: steps {rep['terms']}+{rep['refine_terms']} "
              f"err {err:.2e} bound {rep['cert_bound']:.2e}")
        assert rep["status"] == "CPAA_OK" and rep["certified"] == 1, rep
        assert err <= tol and err <= rep["cert_bound"] * (1 + 1e-9) + 2e-13
        # the library's FP64 residual of x (row order, or the column-sliced
        # gather and combine) against the oracle's: r = (1-c)p - (I - cP')x.
        # Both round; the library's rounding allowance (the part of cert_bound
        # beyond ||r||_1) bounds its error, and the oracle's is of the same size.
        Pm, d = oracle.transition_directed(g)
        xs = x.cpu().numpy()
        rl1 = np.abs((1 - C) * p - xs + C * (Pm @ xs + p * (d @ xs))).sum()
        u = 2.0**-53
        allowance = ((rep["cert_bound"] - u * abs(rep["mass"])) * (1 - C)
                     - rep["resid_l1"] * (1 + 2 * u * g.n))
        assert 0 <= allowance and abs(rep["resid_l1"] - rl1) <= 2 * allowance + 1e-15, \
            (rep["resid_l1"], rl1, allowance)


@pytest.mark.parametrize("slices", [1, 8])
def test_directed_large_and_host_io(torch_cuda, slices):
    from paper_2112_01743_amd import Plan
    from paper_2112_01743_amd import binding as B
    g = gg.directed_random(400000, 8, 0.2, seed=9)
    p = gg.uniform_personalization(g.n)
    pi = oracle.power_method_directed(g, p, C, 230)
    x, rep = _plan(g, column_slices=slices).solve_power(_dev(torch_cuda, p), 1e-8)
    err = np.abs(x.cpu().numpy() - pi).sum()
    _note(f"n={g.n} nnz={g.nnz} slices={slices}: steps {rep['terms']}+{rep['refine_terms']} "
          f"err {err:.2e}")
    assert rep["certified"] == 1 and err <= 1e-8
    plan = Plan.from_graph(g, C, directed=1, io_device=0, column_slices=slices)
    xh = np.zeros(g.n)
    ph = np.ascontiguousarray(p)
    st, reph = B.cpaa_solve_power(plan.handle, ph.ctypes.data, 1e-8, None, xh.ctypes.data)
    assert st == B.CPAA_OK, B.cpaa_last_error()
    assert np.abs(xh - pi).sum() <= 1e-8


@pytest.mark.parametrize("slices", [1, 8])
def test_every_solve_of_a_directed_plan_runs_the_power_method(torch_cuda, slices):
    """cpaa_solve falls back to the power method (report.method = 1); the
    batched calls solve column by column; a warm start is refused."""
    from paper_2112_01743_amd import CpaaError
    g = GRAPHS["random5000"]()
    plan = _plan(g, column_slices=slices)
    assert plan.info()["directed"] == 1
    ps = [gg.uniform_personalization(g.n), gg.source_personalization(g.n, [7])[0],
          gg.source_personalization(g.n, [g.n - 2])[0]]
    pis = [oracle.pagerank_directed_exact(g, p, C) for p in ps]
    tol = 1e-9
    for name in ("solve", "solve_power"):
        x, rep = getattr(plan, name)(_dev(torch_cuda, ps[0]), tol)
        err = np.abs(x.cpu().numpy() - pis[0]).sum()
        _note(f"{name} slices={slices}: method {rep['method']} err {err:.2e}")
        assert rep["method"] == 1 and rep["certified"] == 1 and err <= tol
    P = _dev(torch_cuda, np.stack(ps))
    for name in ("solve_batched", "solve_power_batched"):
        X, reps = getattr(plan, name)(P, tol)
        errs = [np.abs(X[j].cpu().numpy() - pis[j]).sum() for j in range(3)]
        _note(f"{name} slices={slices}: errs {max(errs):.2e}")
        assert np.all(reps["method"] == 1) and np.all(reps["certified"] == 1)
        assert max(errs) <= tol
    p0 = _dev(torch_cuda, ps[0])
    for call in (lambda: plan.solve(p0, 1e-6, x0=p0),
                 lambda: plan.solve_power(p0, 1e-6, x0=p0),
                 lambda: plan.solve_batched(P, 1e-6, X0=P),
                 lambda: plan.solve_power_batched(P, 1e-6, X0=P)):
        with pytest.raises(CpaaError):
            call()


def test_directed_batched_host_io_with_padding(torch_cuda):
    """Host buffers with leading dimensions above n through the column loop."""
    from paper_2112_01743_amd import Plan
    from paper_2112_01743_amd import binding as B
    g = GRAPHS["hubs20000"]()
    plan = Plan.from_graph(g, C, directed=1, io_device=0)
    n, ldp, ldx = g.n, g.n + 3, g.n + 5
    srcs = [0, 1, 2, 17]
    P = np.zeros((len(srcs), ldp))
    for j, s in enumerate(srcs):
        P[j, :n] = gg.source_personalization(n, [s])[0]
    X = np.full((len(srcs), ldx), -7.0)
    st, reps = B.cpaa_solve_batched(plan.handle, len(srcs), P.ctypes.data, ldp, 1e-9, None, n,
                                    X.ctypes.data, ldx)
    assert st == B.CPAA_OK, B.cpaa_last_error()
    for j in range(len(srcs)):
        pi = oracle.power_method_directed(g, P[j, :n], C, 200)
        assert reps[j].method == 1 and reps[j].certified == 1
        assert np.abs(X[j, :n] - pi).sum() <= 1e-9
        assert np.all(X[j, n:] == -7.0)          # padding untouched


def test_detection_picks_the_plan(torch_cuda):
    """directed = 2: an asymmetric pattern, or a symmetric one with an isolated
    vertex (dangling: its mass goes along p, Sec. 2.1), makes a directed plan;
    a symmetric pattern without empty rows stays undirected (CPAA)."""
    from paper_2112_01743_amd import Plan
    tol = 1e-10
    asym = GRAPHS["random5000"]()
    sym = gg.random_connected(3000, 6, seed=5)
    rp = np.concatenate([sym.row_ptr, sym.row_ptr[-1:]]).astype(np.int32)   # vertex n isolated
    iso = gg.CSR(n=sym.n + 1, row_ptr=rp, col_idx=sym.col_idx.copy())
    for g, want in ((asym, 1), (sym, 0), (iso, 1)):
        plan = Plan.from_graph(g, C, directed=2)
        p = gg.uniform_personalization(g.n)
        x, rep = plan.solve(_dev(torch_cuda, p), tol)
        pi = oracle.pagerank_directed_exact(g, p, C)
        err = np.abs(x.cpu().numpy() - pi).sum()
        _note(f"n={g.n}: directed {plan.info()['directed']} method {rep['method']} err {err:.2e}")
        assert plan.info()["directed"] == want and rep["method"] == want
        assert rep["certified"] == 1 and err <= tol
