"""ctypes binding of libcpaa.so (declarations in include/cpaa.h).

Argument marshalling only: every step of a solve runs in the HIP library.
PyTorch supplies device memory (tensor.data_ptr()) and the HIP stream; the
library never sees a torch type.  If libcpaa.so is missing the binding raises
instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcpaa.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "cpaa.h")

STATUS = {0: "CPAA_OK", 1: "CPAA_EINVAL", 2: "CPAA_ENOTSYM", 3: "CPAA_EISOLATED",
          4: "CPAA_ESELFLOOP", 5: "CPAA_EPATTERN", 6: "CPAA_ENOMEM", 7: "CPAA_EDEVICE",
          8: "CPAA_ENOCONV"}
CPAA_OK, CPAA_EINVAL, CPAA_ENOTSYM, CPAA_EISOLATED, CPAA_ESELFLOOP = 0, 1, 2, 3, 4
CPAA_EPATTERN, CPAA_ENOMEM, CPAA_EDEVICE, CPAA_ENOCONV = 5, 6, 7, 8


class cpaa_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("num_graphs", ctypes.c_int32), ("graph_ptr", ctypes.c_void_p),
                ("on_device", ctypes.c_int32), ("values", ctypes.c_void_p)]


class cpaa_opts(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("normalize", ctypes.c_int32), ("nnz_per_thread", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("io_device", ctypes.c_int32), ("time_kernels", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("column_slices", ctypes.c_int32), ("locality_order", ctypes.c_int32),
                ("spectral_interval", ctypes.c_int32), ("directed", ctypes.c_int32),
                ("slice_shape", ctypes.c_int32), ("fp64_recurrence", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("drop_isolated", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32)]


class cpaa_report(ctypes.Structure):
    _fields_ = [("terms", ctypes.c_int32), ("refine_terms", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("certified", ctypes.c_int32),
                ("fallback_used", ctypes.c_int32), ("method", ctypes.c_int32),
                ("cert_bound", ctypes.c_double), ("resid_l1", ctypes.c_double),
                ("resid_max", ctypes.c_double), ("mass", ctypes.c_double),
                ("series_cert", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_terms", ctypes.c_double), ("term_launches", ctypes.c_int64),
                ("edges", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class cpaa_plan_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("num_graphs", ctypes.c_int32),
                ("reordered", ctypes.c_int32), ("max_degree", ctypes.c_int32),
                ("split_rows", ctypes.c_int32), ("nnz_per_thread", ctypes.c_int32),
                ("work_items", ctypes.c_int32), ("tile_w", ctypes.c_int32),
                ("k_cap_global", ctypes.c_int32), ("c", ctypes.c_double),
                ("beta", ctypes.c_double), ("vol", ctypes.c_double),
                ("column_slices", ctypes.c_int32), ("spectrum_lo", ctypes.c_double),
                ("directed", ctypes.c_int32), ("slice_shape", ctypes.c_int32),
                ("slice_partials", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libcpaa.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2112_01743_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.cpaa_default_opts.argtypes = [ctypes.POINTER(cpaa_opts)]
    L.cpaa_default_opts.restype = None
    L.cpaa_plan.argtypes = [ctypes.POINTER(cpaa_csr), dbl, ctypes.POINTER(cpaa_opts),
                            ctypes.POINTER(vp)]
    L.cpaa_plan.restype = ctypes.c_int
    L.cpaa_plan_destroy.argtypes = [vp]
    L.cpaa_plan_destroy.restype = None
    L.cpaa_plan_info_get.argtypes = [vp, ctypes.POINTER(cpaa_plan_info)]
    L.cpaa_plan_info_get.restype = ctypes.c_int
    L.cpaa_solve.argtypes = [vp, vp, dbl, vp, vp, ctypes.POINTER(cpaa_report), vp]
    L.cpaa_solve.restype = ctypes.c_int
    L.cpaa_solve_noalloc.argtypes = [vp, vp, dbl, vp, vp, ctypes.POINTER(cpaa_report), vp]
    L.cpaa_solve_noalloc.restype = ctypes.c_int
    L.cpaa_solve_batched.argtypes = [vp, i32, vp, i64, dbl, vp, i64, vp, i64,
                                     ctypes.POINTER(cpaa_report), vp]
    L.cpaa_solve_batched.restype = ctypes.c_int
    L.cpaa_solve_power.argtypes = [vp, vp, dbl, vp, vp, ctypes.POINTER(cpaa_report), vp]
    L.cpaa_solve_power.restype = ctypes.c_int
    L.cpaa_solve_power_batched.argtypes = [vp, i32, vp, i64, dbl, vp, i64, vp, i64,
                                           ctypes.POINTER(cpaa_report), vp]
    L.cpaa_solve_power_batched.restype = ctypes.c_int
    L.cpaa_solve_graphs.argtypes = [vp, vp, dbl, vp, ctypes.POINTER(cpaa_report), vp]
    L.cpaa_solve_graphs.restype = ctypes.c_int
    L.cpaa_last_error.argtypes = []
    L.cpaa_last_error.restype = ctypes.c_char_p
    fp = ctypes.POINTER(ctypes.c_float)
    L.cpaa_model_create.argtypes = [vp, i32, i32, fp, ctypes.POINTER(vp)]
    L.cpaa_model_create.restype = ctypes.c_int
    L.cpaa_model_destroy.argtypes = [vp]
    L.cpaa_model_destroy.restype = None
    L.cpaa_model_num_params.argtypes = [vp]
    L.cpaa_model_num_params.restype = i32
    L.cpaa_model_get_state.argtypes = [vp, fp, fp, fp, ctypes.POINTER(i64)]
    L.cpaa_model_get_state.restype = ctypes.c_int
    L.cpaa_model_set_state.argtypes = [vp, fp, fp, fp, i64]
    L.cpaa_model_set_state.restype = ctypes.c_int
    L.cpaa_model_predict.argtypes = [vp, i32, ctypes.POINTER(i32), vp, i64, vp]
    L.cpaa_model_predict.restype = ctypes.c_int
    L.cpaa_model_train_step.argtypes = [vp, i32, ctypes.POINTER(i32), vp, i64, ctypes.c_float,
                                        fp, ctypes.POINTER(dbl), vp]
    L.cpaa_model_train_step.restype = ctypes.c_int
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions declared in include/cpaa.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"CPAA_API\s+[\w\s\*]*?\b(cpaa_\w+)\s*\(", text)))


class CpaaError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        msg = lib().cpaa_last_error().decode(errors="replace")
        super().__init__(f"{where}: {self.status_name}: {msg}")


# ----------------------------------------------------------------------------
# thin wrappers with the C names
# ----------------------------------------------------------------------------

def cpaa_default_opts() -> cpaa_opts:
    o = cpaa_opts()
    lib().cpaa_default_opts(ctypes.byref(o))
    return o


def cpaa_last_error() -> str:
    return lib().cpaa_last_error().decode(errors="replace")


def cpaa_plan(csr: cpaa_csr, c: float, opts: cpaa_opts | None = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = lib().cpaa_plan(ctypes.byref(csr), c, ctypes.byref(opts) if opts is not None else None,
                         ctypes.byref(h))
    if st != CPAA_OK:
        raise CpaaError(st, "cpaa_plan")
    return h


def cpaa_plan_destroy(plan) -> None:
    lib().cpaa_plan_destroy(plan)


def cpaa_plan_info_get(plan) -> cpaa_plan_info:
    info = cpaa_plan_info()
    st = lib().cpaa_plan_info_get(plan, ctypes.byref(info))
    if st != CPAA_OK:
        raise CpaaError(st, "cpaa_plan_info_get")
    return info


def cpaa_solve(plan, p_ptr: int, tol: float, x0_ptr: int | None, x_ptr: int,
               stream: int = 0) -> tuple[int, cpaa_report]:
    rep = cpaa_report()
    st = lib().cpaa_solve(plan, p_ptr, tol, x0_ptr, x_ptr, ctypes.byref(rep), stream or None)
    return st, rep


def cpaa_solve_noalloc(plan, p_ptr: int, tol: float, x0_ptr: int | None, x_ptr: int,
                       stream: int = 0) -> tuple[int, cpaa_report]:
    rep = cpaa_report()
    st = lib().cpaa_solve_noalloc(plan, p_ptr, tol, x0_ptr, x_ptr, ctypes.byref(rep),
                                  stream or None)
    return st, rep


def cpaa_solve_batched(plan, B: int, P_ptr: int, ldp: int, tol: float, X0_ptr: int | None,
                       ldx0: int, X_ptr: int, ldx: int, stream: int = 0):
    reps = (cpaa_report * B)()
    st = lib().cpaa_solve_batched(plan, B, P_ptr, ldp, tol, X0_ptr, ldx0, X_ptr, ldx, reps,
                                  stream or None)
    return st, reps


def cpaa_solve_power(plan, p_ptr: int, tol: float, x0_ptr: int | None, x_ptr: int,
                     stream: int = 0) -> tuple[int, cpaa_report]:
    rep = cpaa_report()
    st = lib().cpaa_solve_power(plan, p_ptr, tol, x0_ptr, x_ptr, ctypes.byref(rep),
                                stream or None)
    return st, rep


def cpaa_solve_power_batched(plan, B: int, P_ptr: int, ldp: int, tol: float,
                             X0_ptr: int | None, ldx0: int, X_ptr: int, ldx: int,
                             stream: int = 0):
    reps = (cpaa_report * B)()
    st = lib().cpaa_solve_power_batched(plan, B, P_ptr, ldp, tol, X0_ptr, ldx0, X_ptr, ldx,
                                        reps, stream or None)
    return st, reps


def cpaa_solve_graphs(plan, p_ptr: int, tol: float, x_ptr: int, num_graphs: int,
                      stream: int = 0):
    reps = (cpaa_report * num_graphs)()
    st = lib().cpaa_solve_graphs(plan, p_ptr, tol, x_ptr, reps, stream or None)
    return st, reps


_CTYPE_TO_NP = {ctypes.c_int32: np.int32, ctypes.c_int64: np.int64, ctypes.c_double: np.float64}


def _report_records(reps) -> np.ndarray:
    """cpaa_report[k] -> numpy structured array (one copy; no per-record Python objects)."""
    dt = np.dtype({"names": [f for f, _ in cpaa_report._fields_],
                   "formats": [_CTYPE_TO_NP[t] for _, t in cpaa_report._fields_],
                   "offsets": [getattr(cpaa_report, f).offset for f, _ in cpaa_report._fields_],
                   "itemsize": ctypes.sizeof(cpaa_report)})
    return np.frombuffer(reps, dtype=dt).copy()


# ----------------------------------------------------------------------------
# convenience object over torch HIP tensors
# ----------------------------------------------------------------------------

def _ld(t, n: int) -> int:
    """Leading dimension of a (B, n) tensor; a single row may report any stride."""
    return int(t.stride(0)) if int(t.shape[0]) > 1 else max(int(t.stride(0)), n)


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Plan:
    """A plan for one graph (or a block-diagonal batch of graphs).

    ``row_ptr`` / ``col_idx`` are int32 arrays (numpy on the host, or torch
    device tensors); ``graph_ptr`` marks a batch of independent graphs.
    Keyword options are the fields of cpaa_opts.
    """

    def __init__(self, row_ptr, col_idx, c: float = 0.85, graph_ptr=None, values=None, **opts):
        self._keep = []
        on_device = 0
        if hasattr(row_ptr, "is_cuda"):
            on_device = int(row_ptr.is_cuda)

        def ptr(a):
            if a is None:
                return None
            if hasattr(a, "data_ptr"):
                self._keep.append(a)
                return a.data_ptr()
            a = np.ascontiguousarray(a, dtype=np.int32)
            self._keep.append(a)
            return a.ctypes.data

        n = int(len(row_ptr) - 1)
        nnz = int(len(col_idx))
        ng = 0 if graph_ptr is None else int(len(graph_ptr) - 1)
        vptr = None
        if values is not None:
            if hasattr(values, "data_ptr"):
                self._keep.append(values)
                vptr = values.data_ptr()
            else:
                va = np.ascontiguousarray(values, dtype=np.float64)
                self._keep.append(va)
                vptr = va.ctypes.data
        csr = cpaa_csr(n=n, nnz=nnz, row_ptr=ptr(row_ptr), col_idx=ptr(col_idx), num_graphs=ng,
                       graph_ptr=ptr(graph_ptr), on_device=on_device, values=vptr)
        o = cpaa_default_opts()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, int(v))
        self.opts = o
        self.n, self.nnz, self.c = n, nnz, c
        self.num_graphs = max(ng, 1)
        self.handle = cpaa_plan(csr, c, o)
        self._keep = []

    @classmethod
    def from_graph(cls, g, c: float = 0.85, **opts):
        return cls(g.row_ptr, g.col_idx, c, graph_ptr=g.graph_ptr, **opts)

    def info(self) -> dict:
        return cpaa_plan_info_get(self.handle).as_dict()

    def _single(self, fn, name, p, tol, x0, out, stream, check):
        import torch
        if out is None:
            out = torch.empty_like(p)
        st, rep = fn(self.handle, p.data_ptr(), tol, None if x0 is None else x0.data_ptr(),
                     out.data_ptr(), _stream_handle(stream))
        if check and st not in (CPAA_OK, CPAA_ENOCONV):
            raise CpaaError(st, name)
        d = rep.as_dict()
        d["status"] = STATUS.get(st, st)
        return out, d

    def _batched(self, fn, name, P, tol, X0, out, stream, check):
        import torch
        B = int(P.shape[0])
        if out is None:
            out = torch.empty_like(P)
        st, reps = fn(self.handle, B, P.data_ptr(), _ld(P, self.n), tol,
                      None if X0 is None else X0.data_ptr(),
                      _ld(X0, self.n) if X0 is not None else self.n,
                      out.data_ptr(), _ld(out, self.n), _stream_handle(stream))
        if check and st not in (CPAA_OK, CPAA_ENOCONV):
            raise CpaaError(st, name)
        return out, _report_records(reps)

    def solve(self, p, tol: float = 1e-6, x0=None, out=None, stream=None, check=True):
        """p: (n,) float64 HIP tensor.  Returns (x, report dict)."""
        return self._single(cpaa_solve, "cpaa_solve", p, tol, x0, out, stream, check)

    def solve_noalloc(self, p, tol: float = 1e-6, x0=None, out=None, stream=None, check=True):
        """cpaa_solve_noalloc: the same solve with its workspace in the library's static
        device array (nothing allocated); arguments and result as solve."""
        return self._single(cpaa_solve_noalloc, "cpaa_solve_noalloc", p, tol, x0, out, stream,
                            check)

    def solve_power(self, p, tol: float = 1e-6, x0=None, out=None, stream=None, check=True):
        """The power method (x <- cPx + (1-c)p from x = p) on the same plan and kernels;
        arguments and result as solve; report["terms"] counts power steps."""
        return self._single(cpaa_solve_power, "cpaa_solve_power", p, tol, x0, out, stream,
                            check)

    def solve_batched(self, P, tol: float = 1e-6, X0=None, out=None, stream=None, check=True):
        """P: (B, n) float64 HIP tensor, row j = personalization j.  Returns (X, reports):
        reports is a numpy structured array with one cpaa_report record per column."""
        return self._batched(cpaa_solve_batched, "cpaa_solve_batched", P, tol, X0, out, stream,
                             check)

    def solve_power_batched(self, P, tol: float = 1e-6, X0=None, out=None, stream=None,
                            check=True):
        """B power-method solves at once; arguments and result as solve_batched."""
        return self._batched(cpaa_solve_power_batched, "cpaa_solve_power_batched", P, tol, X0,
                             out, stream, check)

    def solve_graphs(self, p, tol: float = 1e-6, out=None, stream=None, check=True):
        """p: (n,) float64 HIP tensor of concatenated per-graph personalizations.  Returns
        (x, reports): one cpaa_report record per graph (numpy structured array)."""
        import torch
        if out is None:
            out = torch.empty_like(p)
        st, reps = cpaa_solve_graphs(self.handle, p.data_ptr(), tol, out.data_ptr(),
                                     self.num_graphs, _stream_handle(stream))
        if check and st not in (CPAA_OK, CPAA_ENOCONV):
            raise CpaaError(st, "cpaa_solve_graphs")
        return out, _report_records(reps)

    def close(self):
        if getattr(self, "handle", None):
            cpaa_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# warm-start network
# ----------------------------------------------------------------------------

def pack_params(params: dict, layers: int) -> np.ndarray:
    """Flatten a parameter dict into the packing order of include/cpaa.h."""
    parts = []
    for l in range(layers):
        parts += [params[f"w_self{l}"], params[f"w_nbr{l}"], params[f"b{l}"]]
    parts += [params["w_out"], params["b_out"]]
    return np.concatenate([np.asarray(a, dtype=np.float32).reshape(-1) for a in parts])


def unpack_params(flat: np.ndarray, layers: int, hidden: int = 64, in_features: int = 2) -> dict:
    out, at, fin = {}, 0, in_features
    for l in range(layers):
        for name, shape in ((f"w_self{l}", (fin, hidden)), (f"w_nbr{l}", (fin, hidden)),
                            (f"b{l}", (hidden,))):
            size = int(np.prod(shape))
            out[name] = flat[at:at + size].reshape(shape)
            at += size
        fin = hidden
    out["w_out"] = flat[at:at + hidden]
    out["b_out"] = flat[at + hidden:at + hidden + 1]
    return out


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Model:
    """The warm-start network on a Plan's graph (cpaa_model_*)."""

    def __init__(self, plan: "Plan", params: dict, layers: int = 3, hidden: int = 64):
        self.plan = plan            # the model keeps a pointer to the plan
        self.layers = layers
        flat = np.ascontiguousarray(pack_params(params, layers))
        h = ctypes.c_void_p()
        st = lib().cpaa_model_create(plan.handle, layers, hidden, _fptr(flat), ctypes.byref(h))
        if st != CPAA_OK:
            raise CpaaError(st, "cpaa_model_create")
        self.handle = h
        self.num_params = int(lib().cpaa_model_num_params(h))

    def get_state(self):
        P = self.num_params
        w, m, v = (np.zeros(P, dtype=np.float32) for _ in range(3))
        step = ctypes.c_int64()
        st = lib().cpaa_model_get_state(self.handle, _fptr(w), _fptr(m), _fptr(v),
                                        ctypes.byref(step))
        if st != CPAA_OK:
            raise CpaaError(st, "cpaa_model_get_state")
        return w, m, v, int(step.value)

    def set_state(self, w, m=None, v=None, step=0):
        w = np.ascontiguousarray(w, dtype=np.float32)
        m = None if m is None else np.ascontiguousarray(m, dtype=np.float32)
        v = None if v is None else np.ascontiguousarray(v, dtype=np.float32)
        st = lib().cpaa_model_set_state(self.handle, _fptr(w), None if m is None else _fptr(m),
                                        None if v is None else _fptr(v), int(step))
        if st != CPAA_OK:
            raise CpaaError(st, "cpaa_model_set_state")

    def params(self) -> dict:
        return unpack_params(self.get_state()[0], self.layers)

    def predict(self, sources, out=None, stream=None):
        """x0 for each source: (B, n) float64 HIP tensor."""
        import torch
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        B = int(src.shape[0])
        if out is None:
            out = torch.empty((B, self.plan.n), dtype=torch.float64, device="cuda")
        st = lib().cpaa_model_predict(self.handle, B,
                                      src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      out.data_ptr(), _ld(out, self.plan.n), _stream_handle(stream))
        if st != CPAA_OK:
            raise CpaaError(st, "cpaa_model_predict")
        return out

    def train_step(self, sources, targets, lr: float, want_grads: bool = False, stream=None):
        """targets: (B, n) float64 HIP tensor.  Returns (mean loss, grads or None)."""
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        grads = np.zeros(self.num_params, dtype=np.float32) if want_grads else None
        loss = ctypes.c_double()
        st = lib().cpaa_model_train_step(
            self.handle, int(src.shape[0]), src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            targets.data_ptr(), _ld(targets, self.plan.n), float(lr),
            None if grads is None else _fptr(grads), ctypes.byref(loss), _stream_handle(stream))
        if st != CPAA_OK:
            raise CpaaError(st, "cpaa_model_train_step")
        return loss.value, (None if grads is None else unpack_params(grads, self.layers))

    def close(self):
        if getattr(self, "handle", None):
            lib().cpaa_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
