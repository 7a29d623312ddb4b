"""Pins of the oracle's ILUT(tau, m) (Section 3, "Smoother"): the exact-LU limit
(tau = 0, unlimited fill) against scipy's Cholesky factor, hand-worked
examples of both dropping rules (tests/golden/ilut_hand.json), and the
invariants that hold for the paper's constants tau = 1e-12, m = 1."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ilut_hand.json")


def _exact_lu_from_cholesky(A):
    """For SPD A = C^T C (C upper), the LU factorisation without pivoting is
    L = C^T diag(C)^-1 (unit lower), U = diag(C) C."""
    Cu = sla.cholesky(A, lower=False)
    d = np.diag(Cu)
    return Cu.T / d, d[:, None] * Cu


@pytest.mark.parametrize("geom,dim,p,nel", [(0, 2, 2, 6), (1, 2, 3, 5), (0, 3, 2, 4), (0, 2, 5, 4)])
def test_unlimited_ilut_is_exact_lu(geom, dim, p, nel):
    o = O.Oracle(dim, p, nel, geom=geom, rhs=geom, ilut=False)
    A = o.A()
    L, U, st, _ = O.ilut(A, tau=0.0, fill=0.0)
    assert st == 0
    n = A.shape[0]
    Ld = L.toarray() + np.eye(n)
    Ud = U.toarray()
    Ad = A.toarray()
    assert np.abs(Ld @ Ud - Ad).max() <= 1e-13 * np.abs(Ad).max()
    Lc, Uc = _exact_lu_from_cholesky(Ad)
    assert np.abs(Ld - Lc).max() < 1e-11
    assert np.abs(Ud - Uc).max() < 1e-11 * np.abs(Uc).max()


def _dense_from_triplets(trip, n):
    D = np.zeros((n, n))
    for i, j, v in trip:
        D[i, j] = v
    return D


@pytest.mark.parametrize("case", json.load(open(GOLD))["cases"], ids=lambda c: c["name"])
def test_hand_worked_examples(case):
    A = sp.csr_matrix(np.array(case["A"], dtype=float))
    n = A.shape[0]
    L, U, st, _ = O.ilut(A, tau=case["tau"], fill=case["fill"], mode=case["mode"])
    assert st == 0
    Le = _dense_from_triplets(case["L"], n)
    Ue = _dense_from_triplets(case["U"], n)
    assert np.array_equal(L.toarray() != 0, Le != 0)
    assert np.array_equal(U.toarray() != 0, Ue != 0)
    assert np.allclose(L.toarray(), Le, rtol=2e-16 * 4, atol=0)
    assert np.allclose(U.toarray(), Ue, rtol=2e-16 * 4, atol=0)


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("geom,dim,p,nel", [(0, 2, 3, 16), (1, 2, 4, 12), (0, 3, 2, 6)])
def test_invariants_paper_constants(mode, geom, dim, p, nel):
    o = O.Oracle(dim, p, nel, geom=geom, rhs=geom, opts=O.Options(limit_mode=mode))
    assert o.status == 0
    A, L, U = o.A(), o.L(), o.U()
    n = A.shape[0]
    M = int(np.floor(A.nnz / n))
    # L strictly lower, U upper with the diagonal first and positive
    Lc = L.tocoo(); Uc = U.tocoo()
    assert (Lc.row > Lc.col).all()
    assert (Uc.row <= Uc.col).all()
    assert (U.indices[U.indptr[:-1]] == np.arange(n)).all()
    assert (U.data[U.indptr[:-1]] > 0).all()
    nl = np.diff(L.indptr)
    nu = np.diff(U.indptr) - 1
    if mode == 0:
        assert nl.max() <= M and nu.max() <= M
    elif mode == 1:
        assert (nl + nu).max() <= M
    else:
        assert nl.max() <= M // 2 and nu.max() <= M // 2
        assert (nl + nu).max() <= M
    assert (L.data != 0).all() and (U.data != 0).all()
    # bit-reproducible on rerun
    o2 = O.Oracle(dim, p, nel, geom=geom, rhs=geom, opts=O.Options(limit_mode=mode))
    assert np.array_equal(o2.L().data, L.data) and np.array_equal(o2.U().indices, U.indices)
    # L U approximates the permuted A: the factorisation error is far below ||A||
    perm = o.perm()
    Ap = A[perm][:, perm]
    E = (sp.eye(n) + L) @ U - Ap
    assert abs(E).max() < 0.05 * abs(A).max()


def test_zero_pivot_is_an_error():
    A = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 2.0]]))
    L, U, st, bad = O.ilut(A, tau=0.0, fill=0.0)
    assert st == O.EZEROPIVOT and bad == 1
