"""Python binding of the FP64 CPU oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark load this module; the library and its binding never do.

The oracle is the plain, slow reference of the p-multigrid method with an
ILUT smoother (Tielen, Moeller, Goeddeke, Vuik, arXiv:1901.01685): assembly
of the B-spline Galerkin system, lumped L2 transfers between degree p and 1,
ILUT(tau, m), the h-multigrid coarse solve, the V-cycle, the stand-alone
solver and CG.  Each C function cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

OK, EINVAL, ENOMEM, EZEROPIVOT, EDIVERGED, EMAXIT, ENAN = 0, 1, 2, 4, 5, 6, 7
M_A, M_L, M_U, M_R, M_P, M_A1, M_PH, M_RH = range(8)
V_F, V_MLP, V_ML1, V_CHOL = range(4)
GEOM_BOX, GEOM_ANNULUS = 0, 1
RHS_SINE, RHS_ANNULUS = 0, 1
PDE_POISSON, PDE_CDR = 0, 1  # operator: Poisson, or the CDR coefficients of benchmark 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc, FP64, no FMA contraction."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("tau", C.c_double), ("fill", C.c_double), ("limit_mode", C.c_int),
                ("coarse_cycles", C.c_int), ("gs_variant", C.c_int), ("coarse_min", C.c_int),
                ("nu1", C.c_int), ("nu2", C.c_int), ("ordering", C.c_int), ("nd_leaf", C.c_int),
                ("mass_transfer", C.c_int), ("projection", C.c_int), ("diverge", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, dp, ip, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int64)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, ip,
                                 C.POINTER(_Opts), C.c_int, ip]
        L.orc_assemble_only.restype = vp
        L.orc_assemble_only.argtypes = [C.c_int] * 8 + [ip]
        L.orc_ilut_csr.restype = vp
        L.orc_ilut_csr.argtypes = [C.c_int, i64p, ip, dp, C.c_double, C.c_double, C.c_int, ip]
        L.orc_free.argtypes = [vp]
        L.orc_info.argtypes = [vp, i64p]
        L.orc_get_csr.argtypes = [vp, C.c_int, C.c_int, i64p, i64p, ip, dp]
        L.orc_get_vec.argtypes = [vp, C.c_int, dp]
        L.orc_get_perm.argtypes = [vp, ip]
        L.orc_solve.argtypes = [vp, dp, dp, C.c_double, C.c_int, dp, ip]
        L.orc_vcycle.argtypes = [vp, dp, dp, dp]
        L.orc_cg.argtypes = [vp, dp, dp, C.c_double, C.c_int, C.c_int, ip]
        L.orc_bicgstab.argtypes = [vp, dp, dp, C.c_double, C.c_int, C.c_int, dp, ip]
        L.orc_l2_error.restype = C.c_double
        L.orc_l2_error.argtypes = [vp, dp]
        L.orc_residual.argtypes = [vp, dp, dp, dp]
        L.orc_smooth.argtypes = [vp, dp, dp]
        L.orc_hcycle.argtypes = [vp, dp, dp]
        L.orc_restrict.argtypes = [vp, dp, dp]
        L.orc_prolong.argtypes = [vp, dp, dp]
        L.orc_coarse.argtypes = [vp, dp, dp]
        L.orc_gs.argtypes = [vp, C.c_int, dp, dp]
        L.orc_set_operator.argtypes = [vp, C.c_int, i64p, ip, dp]
        L.orc_gauss.argtypes = [C.c_int, dp, dp]
        L.orc_knots.argtypes = [C.c_int, C.c_int, dp]
        L.orc_basis.argtypes = [dp, C.c_int, C.c_int, C.c_double, dp, dp]
        L.orc_geom.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.orc_exact_u.restype = C.c_double
        L.orc_exact_u.argtypes = [C.c_int, C.c_int, ip, dp]
        L.orc_rhs_f.restype = C.c_double
        L.orc_cdr_f.restype = C.c_double
        L.orc_cdr_f.argtypes = [ip, dp]
        L.orc_rhs_f.argtypes = [C.c_int, C.c_int, ip, dp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _i64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


@dataclass
class Options:
    tau: float = 1e-12
    fill: float = 1.0
    limit_mode: int = 0      # rule 2: 0 M largest per part, 1 per row, 2 floor(M/2) per part
    coarse_cycles: int = 2
    gs_variant: int = 0      # 0: multicolour, 1: lexicographic
    coarse_min: int = 8
    nu1: int = 1
    nu2: int = 1
    ordering: int = 1        # 0: natural, 1: nested dissection over grid lines
    nd_leaf: int = 8
    mass_transfer: int = 0   # 0: lumped masses in the transfers, 1: consistent (App. B)
    projection: int = 0      # 0: direct p -> 1, 1: indirect p -> p-1 -> ... -> 1 (App. A)
    diverge: float = 1e10    # Section 5: diverged once the relative residual exceeds this

    def c(self):
        return _Opts(self.tau, self.fill, self.limit_mode, self.coarse_cycles, self.gs_variant,
                     self.coarse_min, self.nu1, self.nu2, self.ordering, self.nd_leaf, self.mass_transfer,
                     self.projection, self.diverge)


# ---------------------------------------------------------------- primitives
def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss(n, _dp(x), _dp(w))
    return x, w


def knots(p, nel):
    t = np.zeros(nel + 2 * p + 1)
    lib().orc_knots(p, nel, _dp(t))
    return t


def basis(t, p, xi):
    t = np.ascontiguousarray(t, dtype=np.float64)
    nb = len(t) - p - 1
    v = np.zeros(nb)
    d = np.zeros(nb)
    lib().orc_basis(_dp(t), len(t), p, float(xi), _dp(v), _dp(d))
    return v, d


def geom(g, dim, xi):
    xi = np.ascontiguousarray(list(xi) + [0.0] * (3 - len(xi)), dtype=np.float64)
    X = np.zeros(3)
    det = np.zeros(1)
    lib().orc_geom(g, dim, _dp(xi), _dp(X), _dp(det))
    return X[:dim], float(det[0])


def exact_u(rhs, dim, k, X):
    kk = np.ascontiguousarray(list(k) + [1] * (3 - len(k)), dtype=np.int32)
    XX = np.ascontiguousarray(list(X) + [0.0] * (3 - len(X)), dtype=np.float64)
    return lib().orc_exact_u(rhs, dim, _ip(kk), _dp(XX))


def rhs_f(rhs, dim, k, X):
    kk = np.ascontiguousarray(list(k) + [1] * (3 - len(k)), dtype=np.int32)
    XX = np.ascontiguousarray(list(X) + [0.0] * (3 - len(X)), dtype=np.float64)
    return lib().orc_rhs_f(rhs, dim, _ip(kk), _dp(XX))


def cdr_f(k, X):
    """Right-hand side of benchmark 2 (CDR operator, u = sin(k1 pi x) sin(k2 pi y))."""
    kk = np.ascontiguousarray(list(k) + [1] * (3 - len(k)), dtype=np.int32)
    XX = np.ascontiguousarray(list(X) + [0.0] * (3 - len(X)), dtype=np.float64)
    return lib().orc_cdr_f(_ip(kk), _dp(XX))


def _get_csr(h, which, lev=0):
    L = lib()
    dims = np.zeros(3, dtype=np.int64)
    rc = L.orc_get_csr(h, which, lev, _i64p(dims), None, None, None)
    if rc:
        raise ValueError(f"no operator {which} at level {lev}")
    nr, nc, nnz = (int(x) for x in dims)
    rp = np.zeros(nr + 1, dtype=np.int64)
    ci = np.zeros(max(nnz, 1), dtype=np.int32)
    v = np.zeros(max(nnz, 1), dtype=np.float64)
    L.orc_get_csr(h, which, lev, _i64p(dims), _i64p(rp), _ip(ci), _dp(v))
    return sp.csr_matrix((v[:nnz], ci[:nnz], rp), shape=(nr, nc))


def assemble_only(dim, geom_kind, nel, kind, pr, pc, nq, elim):
    st = C.c_int(0)
    h = lib().orc_assemble_only(dim, geom_kind, nel, kind, pr, pc, nq, elim, C.byref(st))
    try:
        if st.value:
            raise RuntimeError(f"assembly failed: {st.value}")
        return _get_csr(h, M_A)
    finally:
        lib().orc_free(h)


def ilut(A: sp.csr_matrix, tau=1e-12, fill=1.0, mode=0):
    """ILUT(tau, m) of a square CSR matrix; returns (L strict lower, U upper, status, bad_row)."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    v = np.ascontiguousarray(A.data, dtype=np.float64)
    st = C.c_int(0)
    h = lib().orc_ilut_csr(n, _i64p(rp), _ip(ci), _dp(v), tau, fill, mode, C.byref(st))
    try:
        info = np.zeros(32, dtype=np.int64)
        lib().orc_info(h, _i64p(info))
        if st.value:
            return None, None, st.value, int(info[8])
        return _get_csr(h, M_L), _get_csr(h, M_U), 0, -1
    finally:
        lib().orc_free(h)


# ---------------------------------------------------------------- full solver
class Oracle:
    """One problem (dim, p, n_el, geometry, right-hand side) with every operator
    of the p-multigrid method built by the oracle."""

    def __init__(self, dim, p, nel, geom=GEOM_BOX, rhs=RHS_SINE, freq=(1, 1, 1),
                 opts: Options | None = None, ilut: bool = True, pde=PDE_POISSON):
        self.dim, self.p, self.nel, self.geom, self.rhs, self.pde = dim, p, nel, geom, rhs, pde
        self.opts = opts or Options()
        fr = np.ascontiguousarray(list(freq) + [1] * (3 - len(freq)), dtype=np.int32)
        st = C.c_int(0)
        o = self.opts.c()
        self._h = lib().orc_create(dim, p, nel, geom, rhs, pde, _ip(fr), C.byref(o),
                                   0 if ilut else 1, C.byref(st))
        self.status = st.value
        if self._h is None:
            raise ValueError(f"invalid problem (status {st.value})")
        info = np.zeros(32, dtype=np.int64)
        lib().orc_info(self._h, _i64p(info))
        self.n, self.n1, self.nlev = int(info[0]), int(info[1]), int(info[2])
        self.bad_row = int(info[8])
        self.level_n = [int(info[9 + l]) for l in range(min(self.nlev, 8))]
        self.level_nel = [int(info[17 + l]) for l in range(min(self.nlev, 8))]

    def close(self):
        if self._h:
            lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # operators
    def A(self):
        return _get_csr(self._h, M_A)

    def L(self):
        return _get_csr(self._h, M_L)

    def U(self):
        return _get_csr(self._h, M_U)

    def R(self):
        return _get_csr(self._h, M_R)

    def P(self):
        return _get_csr(self._h, M_P)

    def A1(self, lev=0):
        return _get_csr(self._h, M_A1, lev)

    def Ph(self, lev=0):
        return _get_csr(self._h, M_PH, lev)

    def _vec(self, which, n):
        out = np.zeros(n)
        lib().orc_get_vec(self._h, which, _dp(out))
        return out

    def f(self):
        return self._vec(V_F, self.n)

    def perm(self):
        out = np.zeros(self.n, dtype=np.int32)
        lib().orc_get_perm(self._h, _ip(out))
        return out

    def mlp(self):
        return self._vec(V_MLP, self.n)

    def ml1(self):
        return self._vec(V_ML1, self.n1)

    def chol(self):
        nc = self.level_n[self.nlev - 1]
        return self._vec(V_CHOL, nc * nc).reshape(nc, nc)

    def set_operator(self, A):
        """Replaces A_p by A (n x n) and refactors the smoother from it (test
        hook for the failure branches); returns (status, bad_row)."""
        A = sp.csr_matrix(A)
        A.sort_indices()
        rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
        ci = np.ascontiguousarray(A.indices, dtype=np.int32)
        v = np.ascontiguousarray(A.data, dtype=np.float64)
        st = lib().orc_set_operator(self._h, self.n, _i64p(rp), _ip(ci), _dp(v))
        info = np.zeros(32, dtype=np.int64)
        lib().orc_info(self._h, _i64p(info))
        self.status = st
        return st, int(info[8])

    # solve phase
    def residual(self, b, x):
        r = np.zeros(self.n)
        lib().orc_residual(self._h, _dp(np.ascontiguousarray(b, dtype=np.float64)),
                           _dp(np.ascontiguousarray(x, dtype=np.float64)), _dp(r))
        return r

    def smooth(self, r, x):
        x = np.array(x, dtype=np.float64, copy=True)
        lib().orc_smooth(self._h, _dp(np.ascontiguousarray(r, dtype=np.float64)), _dp(x))
        return x

    def coarse(self, r1):
        e1 = np.zeros(self.n1)
        lib().orc_coarse(self._h, _dp(np.ascontiguousarray(r1, dtype=np.float64)), _dp(e1))
        return e1

    def restrict(self, r):
        """r1 = M_1^{-1} P_p^1 r with the lumped or consistent mass of the options."""
        r1 = np.zeros(self.n1)
        lib().orc_restrict(self._h, _dp(np.ascontiguousarray(r, dtype=np.float64)), _dp(r1))
        return r1

    def prolong_delta(self, e1):
        """y = M_p^{-1} P_1^p e1 (the correction added to u by the prolongation)."""
        y = np.zeros(self.n)
        lib().orc_prolong(self._h, _dp(np.ascontiguousarray(e1, dtype=np.float64)), _dp(y))
        return y

    def hcycle(self, b1, e1):
        e1 = np.array(e1, dtype=np.float64, copy=True)
        lib().orc_hcycle(self._h, _dp(np.ascontiguousarray(b1, dtype=np.float64)), _dp(e1))
        return e1

    def gs(self, lev, b, e):
        e = np.array(e, dtype=np.float64, copy=True)
        lib().orc_gs(self._h, lev, _dp(np.ascontiguousarray(b, dtype=np.float64)), _dp(e))
        return e

    def vcycle(self, b, x, r=None):
        """One V-cycle; returns (x_new, r_new) with r_new = b - A x_new."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x, dtype=np.float64, copy=True)
        r = self.residual(b, x) if r is None else np.array(r, dtype=np.float64, copy=True)
        lib().orc_vcycle(self._h, _dp(b), _dp(x), _dp(r))
        return x, r

    def solve(self, b, x0=None, tol=1e-8, maxit=100):
        """Stand-alone p-multigrid solve; returns (x, status, iters, hist)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        hist = np.zeros(maxit + 1)
        it = C.c_int(0)
        st = lib().orc_solve(self._h, _dp(b), _dp(x), tol, maxit, _dp(hist), C.byref(it))
        return x, st, it.value, hist[: it.value + 1].copy()

    def bicgstab(self, b, x0=None, tol=1e-8, maxit=100, precond=True):
        """BiCGSTAB right-preconditioned by one V-cycle (precond=False: none);
        returns (x, status, iters, hist)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
        hist = np.zeros(maxit + 1)
        it = C.c_int(0)
        st = lib().orc_bicgstab(self._h, _dp(b), _dp(x), tol, maxit, 1 if precond else 0, _dp(hist), C.byref(it))
        return x, st, it.value, hist[: it.value + 1].copy()

    def cg(self, b, tol=1e-13, maxit=100000, jacobi=True):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(self.n)
        it = C.c_int(0)
        st = lib().orc_cg(self._h, _dp(b), _dp(x), tol, maxit, 1 if jacobi else 0, C.byref(it))
        return x, st, it.value

    def l2_error(self, uh):
        return lib().orc_l2_error(self._h, _dp(np.ascontiguousarray(uh, dtype=np.float64)))
