"""Python binding of the MI355X p-multigrid library (include/pmg.h).

Argument marshalling only: every step of the solve phase runs in the HIP
kernels of libpmg.so.  Vectors are torch CUDA tensors (float64, contiguous)
or raw device pointers; streams default to torch's current stream.  The
library must be built in-tree (``python -m paper_1901_01685_amd._build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libpmg.so")

OK, EINVAL, ENOMEM, EDEVICE, EZEROPIVOT, EDIVERGED, EMAXIT, ENAN, EBUDGET = range(9)
GEOM_BOX, GEOM_QUARTER_ANNULUS = 0, 1
RHS_SINE, RHS_ANNULUS, RHS_CALLBACK = 0, 1, 2
PDE_POISSON, PDE_CDR = 0, 1
MASS_LUMPED, MASS_CONSISTENT = 0, 1
PROJ_DIRECT, PROJ_INDIRECT = 0, 1
FP64, FP32_IN_FP64 = 0, 1
ORDER_NATURAL, ORDER_NESTED_DISSECTION = 0, 1
LIMIT_PER_PART, LIMIT_PER_ROW, LIMIT_HALF_PER_PART = 0, 1, 2
OP_A, OP_L, OP_U, OP_R, OP_P, OP_A1, OP_PH = range(7)
VEC_F, VEC_MLP, VEC_ML1, VEC_COARSE_INV = range(4)
PROF_CLASSES = ("residual", "lower", "upper", "restrict", "coarse", "prolong")


class PmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pmg status {status}: {msg}")
        self.status = status


# f(x, ctx) at a physical point x[0..dim-1] (pmg_fn)
FN = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_void_p)


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("degree", C.c_int32), ("n_elem", C.c_int32),
                ("geometry", C.c_int32), ("rhs_kind", C.c_int32), ("freq", C.c_int32 * 3),
                ("pde", C.c_int32), ("knots", C.POINTER(C.c_double) * 3), ("f", FN), ("f_ctx", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("ilut_tau", C.c_double), ("ilut_fill", C.c_double), ("ilut_limit_mode", C.c_int32),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("coarse_cycles", C.c_int32),
                ("coarse_min_elems", C.c_int32), ("gs_variant", C.c_int32), ("precision", C.c_int32),
                ("max_iter", C.c_int32), ("diverge_ratio", C.c_double), ("device", C.c_int32),
                ("setup_threads", C.c_int32), ("ordering", C.c_int32), ("nd_leaf", C.c_int32),
                ("graphs", C.c_int32), ("tiled_gs", C.c_int32), ("mass_transfer", C.c_int32),
                ("projection", C.c_int32), ("poll_limit", C.c_int32), ("ilut_on_device", C.c_int32),
                ("tri_waves_per_cu", C.c_int32), ("segment_rows", C.c_int32), ("kron_residual", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("r0", C.c_double),
                ("relres", C.c_double), ("seconds", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n1", C.c_int64), ("nnz_a", C.c_int64), ("nnz_l", C.c_int64),
                ("nnz_u", C.c_int64), ("nnz_r", C.c_int64), ("nnz_p", C.c_int64), ("nlev", C.c_int32),
                ("n_coarsest", C.c_int32), ("nnz_a1", C.c_int64), ("segments", C.c_int32),
                ("seg_len", C.c_int32), ("dag_levels_l", C.c_int32), ("dag_levels_u", C.c_int32),
                ("chunks_l", C.c_int32), ("chunks_u", C.c_int32), ("chunk_levels_l", C.c_int32),
                ("chunk_levels_u", C.c_int32),
                ("bytes_vcycle", C.c_int64), ("bytes_spmv", C.c_int64), ("bytes_trisolve_l", C.c_int64),
                ("bytes_trisolve_u", C.c_int64), ("bytes_restrict", C.c_int64),
                ("bytes_prolong", C.c_int64), ("bytes_coarse", C.c_int64), ("device_bytes", C.c_int64),
                ("t_assembly", C.c_double), ("t_ilut", C.c_double), ("t_upload", C.c_double),
                ("t_schedule", C.c_double), ("ilut_on_device", C.c_int32), ("residual_layout", C.c_int32),
                ("transfer_layout", C.c_int32), ("resid_rows", C.c_int32),
                ("coarse_kron_levels", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOptions(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("max_class_bytes", C.c_int64), ("max_slots", C.c_int32),
                ("precision", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32), ("device", C.c_int32),
                ("setup_threads", C.c_int32), ("diverge_ratio", C.c_double), ("tri_waves_per_cu", C.c_int32)]


class RequestInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("relres", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_finish", C.c_double), ("n", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("failed", C.c_int64), ("evictions", C.c_int64), ("classes_resident", C.c_int32),
                ("slots_active", C.c_int32), ("queued", C.c_int32), ("bytes_in_use", C.c_int64),
                ("setup_seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported symbols and their signatures (the tests check them against include/pmg.h)
_VP, _DP, _I64P, _I32P = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
SIGNATURES = {
    "pmg_default_options": (C.c_int, [C.POINTER(Options)]),
    "pmg_setup": (C.c_int, [C.POINTER(Problem), C.POINTER(Options), C.POINTER(_VP)]),
    "pmg_setup_from_csr": (C.c_int, [C.POINTER(Problem), C.c_int64, _I64P, _I32P, _DP, C.POINTER(Options),
                                     C.POINTER(_VP)]),
    "pmg_destroy": (C.c_int, [_VP]),
    "pmg_rhs": (C.c_int, [_VP, _VP, _VP]),
    "pmg_residual": (C.c_int, [_VP, _VP, _VP, _VP, _DP, _VP]),
    "pmg_smooth": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_smooth_static": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_lower_solve": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_upper_solve": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_profile_enable": (C.c_int, [_VP, C.c_int32]),
    "pmg_profile_read": (C.c_int, [_VP, _DP, _I64P]),
    "pmg_restrict": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_coarse": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_prolong": (C.c_int, [_VP, _VP, _VP, _VP]),
    "pmg_vcycle": (C.c_int, [_VP, _VP, _VP, _VP, _DP, _VP]),
    "pmg_solve": (C.c_int, [_VP, _VP, _VP, C.c_double, C.POINTER(Result), _DP, _VP]),
    "pmg_get_info": (C.c_int, [_VP, C.POINTER(Info)]),
    "pmg_set_precision": (C.c_int, [_VP, C.c_int32]),
    "pmg_export": (C.c_int, [_VP, C.c_int32, C.c_int32, _I64P, _I64P, _I32P, _DP]),
    "pmg_export_vec": (C.c_int, [_VP, C.c_int32, _DP]),
    "pmg_export_perm": (C.c_int, [_VP, _I32P]),
    "pmg_bicgstab": (C.c_int, [_VP, _VP, _VP, C.c_double, C.POINTER(Result), _DP, _VP]),
    "pmg_export_schedule": (C.c_int, [_VP, C.c_int32, C.c_int32, _I64P, _VP]),
    "pmg_server_default_options": (C.c_int, [C.POINTER(ServerOptions)]),
    "pmg_server_create": (C.c_int, [C.POINTER(ServerOptions), C.POINTER(_VP)]),
    "pmg_server_prepare": (C.c_int, [_VP, C.POINTER(Problem)]),
    "pmg_server_submit": (C.c_int, [_VP, C.POINTER(Problem), _DP, _I64P]),
    "pmg_server_wait": (C.c_int, [_VP, C.c_int64, _DP, C.POINTER(RequestInfo)]),
    "pmg_server_poll": (C.c_int, [_VP, C.c_int64, _I32P, _DP, C.POINTER(RequestInfo)]),
    "pmg_server_configure": (C.c_int, [_VP, C.c_int32, C.c_int32]),
    "pmg_server_get_stats": (C.c_int, [_VP, C.POINTER(ServerStats)]),
    "pmg_server_clock": (C.c_double, [_VP]),
    "pmg_server_get_options": (C.c_int, [_VP, C.POINTER(ServerOptions)]),
    "pmg_server_destroy": (C.c_int, [_VP]),
    "pmg_status_str": (C.c_char_p, [C.c_int]),
    "pmg_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """Loads libpmg.so; raises if it has not been built.  torch is imported
    first when it is installed: its wheel carries its own HIP runtime, and the
    library must bind to the runtime torch uses (loaded the other way round,
    the process ends up with two runtimes and torch finds no device)."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_1901_01685_amd._build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        raise PmgError(st, lib().pmg_last_error().decode())
    return st


def _ptr(t):
    """Device pointer of a torch CUDA tensor (float64, contiguous) or a raw int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def default_options(**kw) -> Options:
    o = Options()
    _check(lib().pmg_default_options(C.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def make_problem(dim=2, degree=2, n_elem=16, geometry=GEOM_BOX, rhs_kind=RHS_SINE, freq=(1, 1, 1),
                 pde=0, knots=None, f=None):
    """pmg_problem.  knots: None or a sequence of per-direction knot vectors
    (None entries: the open uniform one); f: a Python callable f(x) -> float
    on physical points (sets rhs_kind RHS_CALLBACK).  The returned structure
    keeps the arrays and the callback alive in its _keep attribute."""
    fr = list(freq) + [1] * (3 - len(freq))
    pr = Problem(dim, degree, n_elem, geometry, rhs_kind, (C.c_int32 * 3)(*fr), pde)
    keep = []
    if knots is not None:
        for a, t in enumerate(knots):
            if t is None:
                continue
            arr = np.ascontiguousarray(t, dtype=np.float64)
            keep.append(arr)
            pr.knots[a] = arr.ctypes.data_as(_DP)
    if f is not None:
        cb = FN(lambda x, ctx: float(f(x[:dim])))
        keep.append(cb)
        pr.f = cb
        pr.rhs_kind = RHS_CALLBACK
    pr._keep = keep
    return pr


class Solver:
    """One set-up problem (pmg_setup handle) with the solve-phase entry points."""

    def __init__(self, dim=2, degree=2, n_elem=16, geometry=GEOM_BOX, rhs_kind=RHS_SINE,
                 freq=(1, 1, 1), pde=0, knots=None, f=None, operator=None, **opts):
        """operator: None, or a scipy sparse matrix that replaces the assembled
        A_p (pmg_setup_from_csr, test hook)."""
        self.problem = make_problem(dim, degree, n_elem, geometry, rhs_kind, freq, pde, knots, f)
        self.options = default_options(**opts)
        h = C.c_void_p()
        if operator is None:
            _check(lib().pmg_setup(C.byref(self.problem), C.byref(self.options), C.byref(h)))
        else:
            import scipy.sparse as sp
            A = sp.csr_matrix(operator)
            A.sort_indices()
            rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
            ci = np.ascontiguousarray(A.indices, dtype=np.int32)
            v = np.ascontiguousarray(A.data, dtype=np.float64)
            _check(lib().pmg_setup_from_csr(C.byref(self.problem), A.shape[0], rp.ctypes.data_as(_I64P),
                                            ci.ctypes.data_as(_I32P), v.ctypes.data_as(_DP),
                                            C.byref(self.options), C.byref(h)))
        self._h = h
        self.info = self.get_info()
        self.n, self.n1 = int(self.info.n), int(self.info.n1)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pmg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, precision):
        _check(lib().pmg_set_precision(self._h, precision))
        self.options.precision = precision

    def get_info(self) -> Info:
        i = Info()
        _check(lib().pmg_get_info(self._h, C.byref(i)))
        return i

    # ------------------------------------------------------------- solve phase
    def rhs(self, b, stream=None):
        _check(lib().pmg_rhs(self._h, _ptr(b), _stream(stream)))

    def residual(self, b, x, r, norm=False, stream=None):
        nv = C.c_double(0.0)
        _check(lib().pmg_residual(self._h, _ptr(b), _ptr(x), _ptr(r), C.byref(nv) if norm else None,
                                  _stream(stream)))
        return nv.value if norm else None

    def smooth(self, r, x, stream=None):
        _check(lib().pmg_smooth(self._h, _ptr(r), _ptr(x), _stream(stream)))

    def smooth_static(self, r, x, stream=None):
        _check(lib().pmg_smooth_static(self._h, _ptr(r), _ptr(x), _stream(stream)))

    def lower_solve(self, r, y, stream=None):
        _check(lib().pmg_lower_solve(self._h, _ptr(r), _ptr(y), _stream(stream)))

    def upper_solve(self, y, x, stream=None):
        _check(lib().pmg_upper_solve(self._h, _ptr(y), _ptr(x), _stream(stream)))

    def profile_enable(self, on=True):
        _check(lib().pmg_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{class: (total_ms, launches)} for the classes of PROF_CLASSES."""
        ms = np.zeros(len(PROF_CLASSES))
        cnt = np.zeros(len(PROF_CLASSES), dtype=np.int64)
        _check(lib().pmg_profile_read(self._h, ms.ctypes.data_as(_DP), cnt.ctypes.data_as(_I64P)))
        return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(PROF_CLASSES)}

    def restrict(self, r, r1, stream=None):
        _check(lib().pmg_restrict(self._h, _ptr(r), _ptr(r1), _stream(stream)))

    def coarse(self, r1, e1, stream=None):
        _check(lib().pmg_coarse(self._h, _ptr(r1), _ptr(e1), _stream(stream)))

    def prolong(self, e1, x, stream=None):
        _check(lib().pmg_prolong(self._h, _ptr(e1), _ptr(x), _stream(stream)))

    def vcycle(self, b, x, r, norm=False, stream=None):
        nv = C.c_double(0.0)
        _check(lib().pmg_vcycle(self._h, _ptr(b), _ptr(x), _ptr(r), C.byref(nv) if norm else None,
                                _stream(stream)))
        return nv.value if norm else None

    def solve(self, b, x, tol=1e-8, stream=None, check=True):
        """Returns (status, iterations, relres, r0, seconds, hist)."""
        res = Result()
        hist = np.zeros(int(self.options.max_iter) + 1)
        st = lib().pmg_solve(self._h, _ptr(b), _ptr(x), tol, C.byref(res),
                             hist.ctypes.data_as(_DP), _stream(stream))
        if check and st not in (OK, EMAXIT, EDIVERGED, ENAN):
            _check(st)
        return st, res.iterations, res.relres, res.r0, res.seconds, hist[: res.iterations + 1].copy()

    def bicgstab(self, b, x, tol=1e-8, stream=None, check=True):
        """BiCGSTAB preconditioned by one V-cycle per preconditioning phase;
        returns (status, iterations, relres, r0, seconds, hist)."""
        res = Result()
        hist = np.zeros(int(self.options.max_iter) + 1)
        st = lib().pmg_bicgstab(self._h, _ptr(b), _ptr(x), tol, C.byref(res),
                                hist.ctypes.data_as(_DP), _stream(stream))
        if check and st not in (OK, EMAXIT, EDIVERGED, ENAN):
            _check(st)
        return st, res.iterations, res.relres, res.r0, res.seconds, hist[: res.iterations + 1].copy()

    # ------------------------------------------------------------- test hooks
    def export(self, which, level=0):
        import scipy.sparse as sp
        dims = np.zeros(3, dtype=np.int64)
        _check(lib().pmg_export(self._h, which, level, dims.ctypes.data_as(_I64P), None, None, None))
        nr, nc, nnz = (int(v) for v in dims)
        rp = np.zeros(nr + 1, dtype=np.int64)
        ci = np.zeros(max(nnz, 1), dtype=np.int32)
        v = np.zeros(max(nnz, 1), dtype=np.float64)
        _check(lib().pmg_export(self._h, which, level, dims.ctypes.data_as(_I64P), rp.ctypes.data_as(_I64P),
                                ci.ctypes.data_as(_I32P), v.ctypes.data_as(_DP)))
        return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(nr, nc))

    def export_perm(self):
        out = np.zeros(self.n, dtype=np.int32)
        _check(lib().pmg_export_perm(self._h, out.ctypes.data_as(_I32P)))
        return out

    SCHEDULE_FIELDS = ("order", "wptr", "deps", "off_ptr", "off_w", "off_col",
                       "in_ptr", "in_w", "in_j", "off_val", "in_val", "diag", "chunk_row", "chunk_len",
                       "seg_start")

    def export_schedule(self, factor):
        """Schedule and chunk-sliced layout of the lower (0) or upper (1)
        triangular solve, as a dict of numpy arrays (waits as (k, 2))."""
        out = {}
        for f, name in enumerate(self.SCHEDULE_FIELDS):
            cnt = np.zeros(1, dtype=np.int64)
            _check(lib().pmg_export_schedule(self._h, factor, f, cnt.ctypes.data_as(_I64P), None))
            dt = np.float64 if 9 <= f <= 11 else np.int32
            a = np.zeros(max(int(cnt[0]), 1), dtype=dt)
            _check(lib().pmg_export_schedule(self._h, factor, f, cnt.ctypes.data_as(_I64P), a.ctypes.data_as(C.c_void_p)))
            a = a[: int(cnt[0])]
            out[name] = a
        return out

    def export_vec(self, which):
        n = {VEC_F: self.n, VEC_MLP: self.n, VEC_ML1: self.n1,
             VEC_COARSE_INV: int(self.info.n_coarsest) ** 2}[which]
        out = np.zeros(max(n, 1))
        _check(lib().pmg_export_vec(self._h, which, out.ctypes.data_as(_DP)))
        return out[:n]


class Server:
    """Continuous-batching request server (pmg_server_*): requests of any class
    are queued, admitted into device slots as slots and memory free up, and
    advanced one outer step per scheduler tick until they converge."""

    def __init__(self, **opts):
        o = ServerOptions()
        _check(lib().pmg_server_default_options(C.byref(o)))
        for k, v in opts.items():
            if not hasattr(o, k):
                raise AttributeError(k)
            setattr(o, k, v)
        self.options = o
        h = C.c_void_p()
        _check(lib().pmg_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._n = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pmg_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prepare(self, dim, degree, n_elem, geometry=GEOM_BOX, pde=0):
        """Sets up a class ahead of requests; returns the status (EBUDGET if rejected)."""
        pr = make_problem(dim, degree, n_elem, geometry, RHS_SINE, (1, 1, 1), pde)
        return lib().pmg_server_prepare(self._h, C.byref(pr))

    def submit(self, dim, degree, n_elem, geometry=GEOM_BOX, rhs_kind=RHS_SINE, freq=(1, 1, 1), b=None,
               pde=0, f=None):
        """Queues a solve (b: host right-hand side, or f: a callback whose load
        vector is computed at submit time, or neither: rhs_kind); returns
        (status, ticket)."""
        pr = make_problem(dim, degree, n_elem, geometry, rhs_kind, freq, pde, f=f)
        t = C.c_int64(-1)
        bp = None
        if b is not None:
            b = np.ascontiguousarray(b, dtype=np.float64)
            bp = b.ctypes.data_as(_DP)
        st = lib().pmg_server_submit(self._h, C.byref(pr), bp, C.byref(t))
        if st == OK:
            self._n[t.value] = (n_elem + degree - 2) ** dim
        return st, t.value

    def wait(self, ticket, want_x=True):
        """Blocks until the request is done; returns (status, info dict, x or None)."""
        n = self._n.pop(ticket, None)
        if n is None:
            raise KeyError(ticket)
        x = np.zeros(n) if want_x else None
        info = RequestInfo()
        st = lib().pmg_server_wait(self._h, ticket, x.ctypes.data_as(_DP) if want_x else None, C.byref(info))
        return st, info.as_dict(), x

    def poll(self, ticket, want_x=True):
        """Non-blocking wait: None while the request runs, else as wait()."""
        n = self._n.get(ticket)
        if n is None:
            raise KeyError(ticket)
        x = np.zeros(n) if want_x else None
        info = RequestInfo()
        done = C.c_int32(0)
        st = lib().pmg_server_poll(self._h, ticket, C.byref(done), x.ctypes.data_as(_DP) if want_x else None,
                                   C.byref(info))
        if not done.value:
            _check(st)
            return None
        self._n.pop(ticket)
        return st, info.as_dict(), x

    def configure(self, max_slots, precision):
        _check(lib().pmg_server_configure(self._h, max_slots, precision))

    def stats(self):
        st = ServerStats()
        _check(lib().pmg_server_get_stats(self._h, C.byref(st)))
        return st.as_dict()

    def clock(self):
        return lib().pmg_server_clock(self._h)

    def effective_options(self):
        """The options in force, defaults filled in (pmg_server_get_options)."""
        o = ServerOptions()
        _check(lib().pmg_server_get_options(self._h, C.byref(o)))
        return o
