"""cpaa_solve_noalloc, the entry point that allocates nothing (its workspace is
a static device array of the library), against cpaa_solve on the same plans:
two plans in a row, the second smaller (the array keeps the first call's
contents), with the row-order and the column-sliced term, bitwise equal for
deterministic plans; a warm start; a plan that fits only with its residual in
row order; a plan whose workspace does not fit is refused without touching x."""
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


@pytest.mark.timeout(600)
def test_noalloc_matches_solve_two_calls_second_smaller(torch_cuda):
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    graphs = [gg.chung_lu(300000, 12, 2.1, seed=61, dmax=20000),
              gg.chung_lu(40000, 8, 2.3, seed=62)]
    for g in graphs:
        P = [gg.uniform_personalization(g.n), gg.source_personalization(g.n, [g.n // 7])[0]]
        truth = [oracle.pagerank_power(g, p, C, tol=1e-13)[0] for p in P]
        for det in (0, 1):
            plan = Plan.from_graph(g, C, deterministic=det)
            for p, pi in zip(P, truth):
                _note(f"n={g.n} deterministic={det} slices={plan.info()['column_slices']}")
                pd = _dev(torch, p)
                x_ref, r_ref = plan.solve(pd, 1e-9)
                x, r = plan.solve_noalloc(pd, 1e-9)
                xr, xn = x_ref.cpu().numpy(), x.cpu().numpy()
                assert r["status"] == "CPAA_OK" and r["certified"] == 1, r
                assert r["terms"] == r_ref["terms"]
                if det:
                    assert np.array_equal(xn, xr)
                else:
                    assert np.abs(xn - xr).sum() <= r["cert_bound"] + r_ref["cert_bound"]
                err = np.abs(xn - pi).sum()
                assert err <= 1e-9 and err <= r["cert_bound"] * (1 + 1e-9) + 2e-13, err
            # a warm start through the same array
            x0 = _dev(torch, truth[1] * (1 + 1e-3 * gg.philox(3).standard_normal(g.n)))
            x0 /= x0.sum()
            xw, rw = plan.solve_noalloc(_dev(torch, P[1]), 1e-9, x0=x0)
            assert rw["fallback_used"] == 0 and rw["certified"] == 1
            assert np.abs(xw.cpu().numpy() - truth[1]).sum() <= 1e-9


def test_noalloc_without_room_for_the_fp64_partials(torch_cuda):
    """A column-sliced plan whose workspace fits the 64 MiB array only without
    the FP64 partials of the sliced residual (about 36 n + 4 P bytes against
    36 n + 12 P with them, P = partials per term): the call runs its residual
    in row order and returns the same solution as cpaa_solve, to their bounds."""
    from paper_2112_01743_amd import Plan
    torch = torch_cuda
    g = gg.chung_lu(1_000_000, 16, 2.1, seed=64, dmax=50000)
    plan = Plan.from_graph(g, C, column_slices=8)
    P = plan.info()["slice_partials"]
    limit = 64 << 20
    assert 36 * g.n + 4 * P < limit < 36 * g.n + 12 * P, (g.n, P)
    for p in (gg.uniform_personalization(g.n), gg.source_personalization(g.n, [9])[0]):
        pd = _dev(torch, p)
        x_ref, r_ref = plan.solve(pd, 1e-9)
        x, r = plan.solve_noalloc(pd, 1e-9)
        assert r["status"] == "CPAA_OK" and r["certified"] == 1, r
        assert r["terms"] == r_ref["terms"]
        diff = np.abs(x.cpu().numpy() - x_ref.cpu().numpy()).sum()
        _note(f"n={g.n} partials={P} noalloc vs solve L1 {diff:.3e}")
        assert diff <= r["cert_bound"] + r_ref["cert_bound"]
        assert abs(r["resid_l1"] - r_ref["resid_l1"]) <= 1e-6 * r_ref["resid_l1"] + 1e-15


def test_noalloc_refuses_a_plan_too_large_for_the_array(torch_cuda):
    from paper_2112_01743_amd import Plan, binding as B
    torch = torch_cuda
    g = gg.erdos_renyi(2_000_000, 4, seed=63)
    plan = Plan.from_graph(g, C)
    p = _dev(torch, gg.uniform_personalization(g.n))
    x = torch.full_like(p, -7.0)
    _, rep = plan.solve_noalloc(p, 1e-6, out=x, check=False)
    assert rep["status"] == "CPAA_EINVAL"
    assert "static array" in B.cpaa_last_error()
    assert bool((x == -7.0).all())
