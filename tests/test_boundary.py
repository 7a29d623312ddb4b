"""The problem statement at the C ABI (include/pmg.h, pmg_problem and
pmg_setup_from_csr), on the CPU (handles with device = -1):

  * a right-hand side given as a host callback f(x) (Section 2's model
    problem: the load vector is int f Phi_i) reproduces the built-in sine and
    annulus right-hand sides and agrees with the oracle's load vector;
  * knot vectors (Section 2, the knot vector Xi of each direction): the open
    uniform one is accepted, any other is EINVAL with a message;
  * operator injection: the smoother is factored from the given operator,
    identical to the oracle's factors of the same operator, and an operator
    with an empty row fails with PMG_EZEROPIVOT on both sides at the same row.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import paper_1901_01685_amd as P


def _rel(a, b):
    a = a.toarray() if hasattr(a, "toarray") else np.asarray(a)
    b = b.toarray() if hasattr(b, "toarray") else np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _sine(k):
    def f(x):
        return math.pi ** 2 * sum(kk * kk for kk in k[:len(x)]) * math.prod(
            math.sin(kk * math.pi * xx) for kk, xx in zip(k, x))
    return f


@pytest.mark.parametrize("dim,p,nel,k", [(2, 2, 16, (1, 1)), (2, 4, 12, (2, 3)), (3, 2, 6, (1, 2, 1))])
def test_callback_rhs_reproduces_the_sine_load_vector(dim, p, nel, k):
    """f given as a callback, integrated element by element with (p+1)^d
    Gauss points, equals the built-in separable sine load vector and the
    oracle's element-loop load vector to rounding."""
    s_cb = P.Solver(dim, p, nel, f=_sine(k), device=-1)
    s_ref = P.Solver(dim, p, nel, freq=k, device=-1)
    o = O.Oracle(dim, p, nel, freq=k, ilut=False)
    f_cb = s_cb.export_vec(P.VEC_F)
    assert _rel(f_cb, s_ref.export_vec(P.VEC_F)) < 1e-13
    assert _rel(f_cb, o.f()) < 1e-13
    # the callback changes the load vector only
    assert _rel(s_cb.export(P.OP_A), s_ref.export(P.OP_A)) == 0.0


def test_callback_rhs_on_the_annulus():
    """Benchmark 1's right-hand side passed as a callback at the physical
    points of the quarter annulus equals the built-in one and the oracle's."""
    def f(x):
        X, Y = x[0], x[1]
        return O.rhs_f(O.RHS_ANNULUS, 2, (1, 1), (X, Y))
    s_cb = P.Solver(2, 3, 16, geometry=P.GEOM_QUARTER_ANNULUS, f=f, device=-1)
    o = O.Oracle(2, 3, 16, geom=O.GEOM_ANNULUS, rhs=O.RHS_ANNULUS, ilut=False)
    assert _rel(s_cb.export_vec(P.VEC_F), o.f()) < 1e-13


def test_callback_counts_each_quadrature_point_once():
    """f = 1 gives int Phi_i, the lumped mass (partition of unity, reading R6)."""
    s = P.Solver(2, 3, 10, f=lambda x: 1.0, device=-1)
    assert _rel(s.export_vec(P.VEC_F), s.export_vec(P.VEC_MLP)) < 1e-14


def test_uniform_knot_vectors_are_accepted():
    p, nel = 3, 8
    t = np.concatenate([np.zeros(p + 1), np.arange(1, nel) / nel, np.ones(p + 1)])
    a = P.Solver(2, p, nel, knots=[t, t], device=-1)
    b = P.Solver(2, p, nel, knots=[None, t], device=-1)
    c = P.Solver(2, p, nel, device=-1)
    assert _rel(a.export(P.OP_A), c.export(P.OP_A)) == 0.0
    assert _rel(b.export_vec(P.VEC_F), c.export_vec(P.VEC_F)) == 0.0
    assert np.array_equal(t, O.knots(p, nel))


@pytest.mark.parametrize("kind", ["graded", "short_end", "repeated"])
def test_other_knot_vectors_are_rejected(kind):
    p, nel = 2, 8
    t = np.concatenate([np.zeros(p + 1), np.arange(1, nel) / nel, np.ones(p + 1)])
    if kind == "graded":
        t[p + 1:p + nel] = (np.arange(1, nel) / nel) ** 2
    elif kind == "short_end":
        t[p] = 0.05
    else:
        t[p + 3] = t[p + 2]
    with pytest.raises(P.PmgError) as e:
        P.Solver(2, p, nel, knots=[t, None], device=-1)
    assert e.value.status == P.EINVAL
    assert "knots[0]" in str(e.value)


def test_callback_requires_f():
    pr = P.make_problem(2, 2, 8)
    pr.rhs_kind = P.RHS_CALLBACK
    h = P.C.c_void_p()
    o = P.default_options(device=-1)
    assert P.lib().pmg_setup(P.C.byref(pr), P.C.byref(o), P.C.byref(h)) == P.EINVAL


def test_injected_operator_factors_match_the_oracle():
    """pmg_setup_from_csr: the smoother is ILUT of the given operator in the
    same ordering; the library's factors equal the oracle's factors of the
    same matrix (patterns identical, values to rounding)."""
    o = O.Oracle(2, 3, 16, ilut=False)
    A = o.A().tocsr()
    rng = np.random.default_rng(5)
    D = sp.diags(rng.uniform(0.5, 2.0, A.shape[0]))
    B = (D @ A @ D).tocsr()                    # same pattern, other values
    s = P.Solver(2, 3, 16, operator=B, device=-1)
    o2 = O.Oracle(2, 3, 16)
    st, _ = o2.set_operator(B)
    assert st == 0
    assert _rel(s.export(P.OP_A), B) == 0.0
    for mine, ref in ((s.export(P.OP_L), o2.L()), (s.export(P.OP_U), o2.U())):
        mine.sort_indices(); ref.sort_indices()
        assert np.array_equal(mine.indptr, ref.indptr) and np.array_equal(mine.indices, ref.indices)
        assert _rel(mine, ref) < 1e-12


def test_empty_row_is_a_zero_pivot_on_both_sides():
    """An operator whose row and column i are empty cannot be factored: both
    the library (through the C ABI) and the oracle report PMG_EZEROPIVOT at
    the position of unknown i in the ILUT ordering (reading R15)."""
    o = O.Oracle(2, 2, 16)
    A = o.A().tolil()
    i = 37
    A[i, :] = 0
    A[:, i] = 0
    A = A.tocsr()
    A.eliminate_zeros()
    with pytest.raises(P.PmgError) as e:
        P.Solver(2, 2, 16, operator=A, device=-1)
    assert e.value.status == P.EZEROPIVOT
    st, bad = o.set_operator(A)
    assert st == O.EZEROPIVOT
    pos = int(np.where(o.perm() == i)[0][0])
    assert bad == pos
    assert ("row %d" % pos) in str(e.value)


def test_injected_operator_is_checked():
    o = O.Oracle(2, 2, 8, ilut=False)
    A = o.A().tocsr()
    with pytest.raises(P.PmgError) as e:
        P.Solver(2, 2, 8, operator=A[:-1, :-1], device=-1)
    assert e.value.status == P.EINVAL
    bad = A.copy()
    bad.indices[1], bad.indices[2] = bad.indices[2], bad.indices[1]
    rp = np.ascontiguousarray(bad.indptr, dtype=np.int64)
    ci = np.ascontiguousarray(bad.indices, dtype=np.int32)
    v = np.ascontiguousarray(bad.data)
    pr = P.make_problem(2, 2, 8)
    opts = P.default_options(device=-1)
    h = P.C.c_void_p()
    st = P.lib().pmg_setup_from_csr(P.C.byref(pr), A.shape[0], rp.ctypes.data_as(P._I64P),
                                    ci.ctypes.data_as(P._I32P), v.ctypes.data_as(P._DP),
                                    P.C.byref(opts), P.C.byref(h))
    assert st == P.EINVAL and not h.value
