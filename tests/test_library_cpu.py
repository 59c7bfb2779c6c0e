"""Host-side checks of the C-ABI library: it loads, exports every function
include/cpaa.h declares, and rejects bad graphs before touching a GPU."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
from paper_2112_01743_amd import binding as B


def test_library_exports_every_declared_function():
    names = B.header_functions()
    assert {"cpaa_plan", "cpaa_solve", "cpaa_solve_batched", "cpaa_solve_graphs",
            "cpaa_solve_power", "cpaa_solve_power_batched",
            "cpaa_plan_destroy", "cpaa_last_error", "cpaa_default_opts",
            "cpaa_plan_info_get", "cpaa_model_create", "cpaa_model_predict",
            "cpaa_model_train_step", "cpaa_model_get_state", "cpaa_model_set_state",
            "cpaa_model_destroy", "cpaa_model_num_params"} <= set(names)
    L = B.lib()
    for name in names:
        assert hasattr(L, name), name


def test_library_exports_nothing_else():
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported == B.header_functions()


def test_struct_layout_matches_header(tmp_path):
    """Every ctypes structure has the size and field offsets the C compiler
    gives the header's declaration."""
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = [B.cpaa_opts, B.cpaa_report, B.cpaa_csr, B.cpaa_plan_info]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "cpaa.h"', "int main(void) {"]
    for S in structs:
        name = S.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in S._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                   check=True).stdout.splitlines())
    for S in structs:
        name = S.__name__
        assert int(got[name]) == ctypes.sizeof(S), name
        for f, _ in S._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(S, f).offset, (name, f)


def test_default_opts():
    o = B.cpaa_default_opts()
    assert o.max_refine == 2 and o.validate == 1 and o.io_device == 1 and o.xcd_remap == -1


def _plan_status(rp, ci, c=0.85, values=None, **kw):
    rp = np.asarray(rp, dtype=np.int32)
    ci = np.asarray(ci, dtype=np.int32)
    val = None if values is None else np.ascontiguousarray(values, dtype=np.float64)
    csr = B.cpaa_csr(n=len(rp) - 1, nnz=len(ci), row_ptr=rp.ctypes.data, col_idx=ci.ctypes.data,
                     num_graphs=0, graph_ptr=None, on_device=0,
                     values=None if val is None else val.ctypes.data)
    o = B.cpaa_default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    st = B.lib().cpaa_plan(ctypes.byref(csr), c, ctypes.byref(o), ctypes.byref(h))
    if st == 0:
        B.lib().cpaa_plan_destroy(h)
    return st


@pytest.mark.parametrize("case,rp,ci,status", [
    ("asymmetric", [0, 1, 2, 2], [1, 2], B.CPAA_EISOLATED),
    ("asymmetric2", [0, 1, 3, 4], [1, 0, 2, 0], B.CPAA_ENOTSYM),
    ("selfloop", [0, 2, 3], [0, 1, 0], B.CPAA_ESELFLOOP),
    ("isolated", [0, 1, 2, 2], [1, 0], B.CPAA_EISOLATED),
    ("unsorted", [0, 2, 3, 4], [2, 1, 0, 0], B.CPAA_EPATTERN),
    ("duplicate", [0, 2, 3], [1, 1, 0], B.CPAA_EPATTERN),
    ("out_of_range", [0, 1, 2], [5, 0], B.CPAA_EPATTERN),
    ("bad_rowptr", [0, 2, 1], [1, 0], B.CPAA_EPATTERN),
    ("empty", [0], [], B.CPAA_EINVAL),
    ("no_edges", [0, 0, 0], [], B.CPAA_EISOLATED),
])
def test_plan_rejects_bad_patterns(case, rp, ci, status):
    assert _plan_status(rp, ci) == status, (case, B.cpaa_last_error())


def test_plan_rejects_bad_damping_and_options():
    g = gg.cycle(5)
    assert _plan_status(g.row_ptr, g.col_idx, c=1.0) == B.CPAA_EINVAL
    assert _plan_status(g.row_ptr, g.col_idx, c=0.0) == B.CPAA_EINVAL
    assert _plan_status(g.row_ptr, g.col_idx, nnz_per_thread=3) == B.CPAA_EINVAL
    assert _plan_status(g.row_ptr, g.col_idx, tile_w=7) == B.CPAA_EINVAL
    assert "tile_w" in B.cpaa_last_error()
    assert _plan_status(g.row_ptr, g.col_idx, column_slices=4) == B.CPAA_EINVAL
    assert "column_slices" in B.cpaa_last_error()
    assert _plan_status(g.row_ptr, g.col_idx, locality_order=3) == B.CPAA_EINVAL
    assert "locality_order" in B.cpaa_last_error()
    assert _plan_status(g.row_ptr, g.col_idx, spectral_interval=2) == B.CPAA_EINVAL
    assert "spectral_interval" in B.cpaa_last_error()


def test_directed_plan_options():
    """directed = 1 accepts asymmetric patterns and empty rows (the plan then
    fails only at its first device allocation when there is no GPU), also
    with column slices, and rejects the options that need an undirected graph."""
    rp = np.array([0, 0, 1, 3], dtype=np.int32)     # edges 0->1, 0->2, 1->2; row 0 empty
    ci = np.array([0, 0, 1], dtype=np.int32)
    assert _plan_status(rp, ci) in (B.CPAA_ENOTSYM, B.CPAA_EISOLATED)
    assert _plan_status(rp, ci, directed=1) in (B.CPAA_OK, B.CPAA_ENOMEM, B.CPAA_EDEVICE)
    assert _plan_status(rp, ci, directed=1, column_slices=8) in (B.CPAA_OK, B.CPAA_ENOMEM,
                                                                 B.CPAA_EDEVICE)
    # detection (directed = 2) takes the asymmetric pattern with its empty row
    assert _plan_status(rp, ci, directed=2) in (B.CPAA_OK, B.CPAA_ENOMEM, B.CPAA_EDEVICE)
    for bad in ({"directed": 3}, {"directed": -1}, {"directed": 1, "locality_order": 2},
                {"directed": 1, "spectral_interval": 1}, {"directed": 2, "locality_order": 2}):
        assert _plan_status(rp, ci, **bad) == B.CPAA_EINVAL, bad


def test_spectral_interval_needs_one_graph():
    rp = np.array([0, 1, 2, 3, 4], dtype=np.int32)
    ci = np.array([1, 0, 3, 2], dtype=np.int32)
    gp = np.array([0, 2, 4], dtype=np.int32)
    csr = B.cpaa_csr(n=4, nnz=4, row_ptr=rp.ctypes.data, col_idx=ci.ctypes.data, num_graphs=2,
                     graph_ptr=gp.ctypes.data, on_device=0)
    o = B.cpaa_default_opts()
    o.spectral_interval = 1
    h = ctypes.c_void_p()
    st = B.lib().cpaa_plan(ctypes.byref(csr), 0.85, ctypes.byref(o), ctypes.byref(h))
    assert st == B.CPAA_EINVAL and "single-graph" in B.cpaa_last_error()


def test_plan_rejects_edge_across_graph_boundary():
    # two graphs {0,1} and {2,3} but edge 1-2 crosses
    rp = np.array([0, 1, 3, 5, 6], dtype=np.int32)
    ci = np.array([1, 0, 2, 1, 3, 2], dtype=np.int32)
    gp = np.array([0, 2, 4], dtype=np.int32)
    csr = B.cpaa_csr(n=4, nnz=6, row_ptr=rp.ctypes.data, col_idx=ci.ctypes.data, num_graphs=2,
                     graph_ptr=gp.ctypes.data, on_device=0)
    h = ctypes.c_void_p()
    st = B.lib().cpaa_plan(ctypes.byref(csr), 0.85, None, ctypes.byref(h))
    assert st == B.CPAA_EINVAL and "crosses" in B.cpaa_last_error()


def test_param_packing_roundtrip():
    import graphgen as gg
    p = gg.mpnn_init(3)
    flat = B.pack_params(p, 3)
    assert flat.size == 2 * 2 * 64 + 64 + 2 * (2 * 64 * 64 + 64) + 65
    back = B.unpack_params(flat, 3)
    for k, v in p.items():
        assert np.array_equal(back[k], v)


def test_batched_reports_become_structured_records():
    reps = (B.cpaa_report * 3)()
    reps[1].terms, reps[1].refine_terms, reps[1].cert_bound = 7, 2, 1.5e-7
    reps[2].edges, reps[2].certified = 123, 1
    rec = B._report_records(reps)
    assert rec.shape == (3,) and rec.dtype.itemsize == ctypes.sizeof(B.cpaa_report)
    assert rec[1]["terms"] + rec[1]["refine_terms"] == 9 and rec[1]["cert_bound"] == 1.5e-7
    assert rec[2]["edges"] == 123 and rec[2]["certified"] == 1 and rec[0]["terms"] == 0


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2 and "one GPU" in res.stderr and res.stdout == ""


def test_plan_checks_values_against_inverse_degrees():
    """The optional values must be the entries of P = A D^-1 (Sec. 2.1): 1/deg of
    the column (1/out-degree for a directed plan); anything else is refused
    before device work, and valid values pass the check (on a CPU-only host
    the plan then stops at its first device allocation)."""
    g = gg.chung_lu(300, 6, 2.3, seed=8)
    rp, ci = g.row_ptr, g.col_idx
    deg = np.diff(rp).astype(np.float64)
    good = 1.0 / deg[ci]
    assert _plan_status(rp, ci, values=good) in (B.CPAA_OK, B.CPAA_ENOMEM, B.CPAA_EDEVICE)
    for j in (0, len(ci) // 2, len(ci) - 1):
        bad = good.copy()
        bad[j] *= 1.0 + 1e-12
        assert _plan_status(rp, ci, values=bad) == B.CPAA_EINVAL
        assert f"values[{j}]" in B.cpaa_last_error()
    # the row's own degree instead of the column's (P transposed) is refused
    rowdeg = 1.0 / np.repeat(deg, np.diff(rp))
    assert not np.allclose(rowdeg, good)
    assert _plan_status(rp, ci, values=rowdeg) == B.CPAA_EINVAL
    # directed: out-degree of the column vertex (the number of rows listing it)
    drp = np.array([0, 0, 1, 3], dtype=np.int32)      # edges 0->1, 0->2, 1->2
    dci = np.array([0, 0, 1], dtype=np.int32)
    dout = np.bincount(dci, minlength=3).astype(np.float64)
    assert _plan_status(drp, dci, values=1.0 / dout[dci], directed=1) in (
        B.CPAA_OK, B.CPAA_ENOMEM, B.CPAA_EDEVICE)
    assert _plan_status(drp, dci, values=np.ones(3), directed=1) == B.CPAA_EINVAL


def test_drop_isolated_plan_options():
    """drop_isolated = 1 accepts edgeless vertices in an undirected graph (the
    plan then stops only at its first device allocation without a GPU), refuses
    a graph without edges and the directed and block-diagonal cases."""
    rp = np.array([0, 1, 2, 2, 2], dtype=np.int32)    # edge 0-1, vertices 2 and 3 alone
    ci = np.array([1, 0], dtype=np.int32)
    assert _plan_status(rp, ci) == B.CPAA_EISOLATED
    assert _plan_status(rp, ci, drop_isolated=1) in (B.CPAA_OK, B.CPAA_ENOMEM, B.CPAA_EDEVICE)
    assert _plan_status(rp, ci, drop_isolated=1, column_slices=8) in (
        B.CPAA_OK, B.CPAA_ENOMEM, B.CPAA_EDEVICE)
    assert _plan_status(np.zeros(4, dtype=np.int32), np.zeros(0, dtype=np.int32),
                        drop_isolated=1) == B.CPAA_EISOLATED
    assert _plan_status(rp, ci, drop_isolated=1, directed=1) == B.CPAA_EINVAL
    assert _plan_status(rp, ci, drop_isolated=2) == B.CPAA_EINVAL
    for bad in ({"fp64_recurrence": 2}, {"deterministic": 3},
                {"fp64_recurrence": 1, "column_slices": 8},
                {"fp64_recurrence": 1, "deterministic": 1},
                {"deterministic": 1, "column_slices": 1},
                {"deterministic": 1, "slice_shape": 5},
                {"slice_shape": 6}, {"slice_shape": -1},
                {"time_kernels": 3}, {"time_kernels": -1},
                {"rows_per_wave": -1}, {"rows_per_wave": 1025}):
        g = gg.cycle(6)
        assert _plan_status(g.row_ptr, g.col_idx, **bad) == B.CPAA_EINVAL, bad
