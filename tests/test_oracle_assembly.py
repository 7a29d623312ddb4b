"""Pins of the oracle's Galerkin assembly, lumping and transfer operators
(Section 2, discrete system; Section 3, mass and transfer matrices, row-sum
lumping, rediscretised coarse operators) against the tensor-product
(Kronecker) identity on the box, closed forms for p = 1, exact 1-D integrals
from scipy's B-splines, conservation identities, and the h^{p+1} decay of the
L2 error of the Galerkin solution."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.interpolate import BSpline

import oracle as O


def _knots(p, nel):
    return np.concatenate([np.zeros(p), np.linspace(0, 1, nel + 1), np.ones(p)])


def _matrices_1d(p, q, nel):
    """Exact 1-D stiffness, mass and mixed (degree p x degree q) matrices from
    scipy B-splines and a 12-point Gauss rule per element (exact here)."""
    tp, tq = _knots(p, nel), _knots(q, nel)
    npf, nqf = nel + p, nel + q
    gx, gw = np.polynomial.legendre.leggauss(12)
    xs, ws = [], []
    for e in range(nel):
        a, b = e / nel, (e + 1) / nel
        xs.append(0.5 * (a + b) + 0.5 * (b - a) * gx)
        ws.append(0.5 * (b - a) * gw)
    xs, ws = np.concatenate(xs), np.concatenate(ws)

    def vals(t, k, nf):
        V = np.zeros((nf, xs.size)); D = np.zeros((nf, xs.size))
        for i in range(nf):
            c = np.zeros(nf); c[i] = 1
            bs = BSpline(t, c, k)
            V[i] = bs(xs); D[i] = bs.derivative()(xs) if k > 0 else 0
        return V, D

    Vp, Dp = vals(tp, p, npf)
    Vq, Dq = vals(tq, q, nqf)
    K = (Dp * ws) @ Dp.T
    M = (Vp * ws) @ Vp.T
    X = (Vp * ws) @ Vq.T
    return K, M, X


def _interior(M, drop_rows=True, drop_cols=True):
    r = slice(1, M.shape[0] - 1) if drop_rows else slice(None)
    c = slice(1, M.shape[1] - 1) if drop_cols else slice(None)
    return M[r, c]


@pytest.mark.parametrize("p,nel", [(1, 6), (2, 5), (3, 7), (5, 6)])
def test_box_stiffness_is_kronecker_2d(p, nel):
    K, M, _ = _matrices_1d(p, p, nel)
    Ki, Mi = _interior(K), _interior(M)
    ref = np.kron(Mi, Ki) + np.kron(Ki, Mi)          # x-fastest numbering
    A = O.assemble_only(2, O.GEOM_BOX, nel, 0, p, p, p + 1, 1).toarray()
    assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()
    # pattern: every pair of overlapping supports, nothing else
    Ao = O.assemble_only(2, O.GEOM_BOX, nel, 0, p, p, p + 1, 1)
    n1 = nel + p - 2
    for i in range(Ao.shape[0]):
        cols = Ao.indices[Ao.indptr[i]:Ao.indptr[i + 1]]
        ix, iy = i % n1, i // n1
        want = sorted(jx + n1 * jy for jy in range(n1) for jx in range(n1)
                      if abs(jx - ix) <= p and abs(jy - iy) <= p)
        assert list(cols) == want


@pytest.mark.parametrize("p,nel", [(1, 4), (2, 4), (3, 3)])
def test_box_stiffness_mass_kronecker_3d(p, nel):
    K, M, _ = _matrices_1d(p, p, nel)
    Ki, Mi = _interior(K), _interior(M)
    ref = np.kron(np.kron(Mi, Mi), Ki) + np.kron(np.kron(Mi, Ki), Mi) + np.kron(np.kron(Ki, Mi), Mi)
    A = O.assemble_only(3, O.GEOM_BOX, nel, 0, p, p, p + 1, 1).toarray()
    assert np.abs(A - ref).max() < 1e-13 * np.abs(ref).max()
    Mm = O.assemble_only(3, O.GEOM_BOX, nel, 1, p, p, p + 1, 1).toarray()
    refm = np.kron(np.kron(Mi, Mi), Mi)
    assert np.abs(Mm - refm).max() < 1e-14 * np.abs(refm).max()


@pytest.mark.parametrize("p,q,nel", [(2, 1, 6), (4, 1, 5), (3, 2, 6), (5, 4, 5)])
def test_box_transfer_is_kronecker(p, q, nel):
    """Transfer P_q^p = int phi_{i,p} phi_{j,q}: to degree 1 (direct
    projection) and to degree p-1 (indirect projection, Appendix A)."""
    _, _, X = _matrices_1d(p, q, nel)
    Xi = _interior(X)
    ref = np.kron(Xi, Xi)
    P = O.assemble_only(2, O.GEOM_BOX, nel, 1, p, q, p + 1, 1).toarray()
    assert np.abs(P - ref).max() < 1e-14 * np.abs(ref).max()


def test_p1_closed_forms():
    nel = 8
    h = 1.0 / nel
    K, M, _ = _matrices_1d(1, 1, nel)
    n = nel - 1
    Kc = (np.diag(2 * np.ones(n)) - np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / h
    Mc = (np.diag(4 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) * h / 6
    assert np.abs(_interior(K) - Kc).max() < 1e-12
    assert np.abs(_interior(M) - Mc).max() < 1e-15
    A = O.assemble_only(2, O.GEOM_BOX, nel, 0, 1, 1, 2, 1).toarray()
    assert np.abs(A - (np.kron(Mc, Kc) + np.kron(Kc, Mc))).max() < 1e-13
    # the Q1 9-point stencil of the Laplacian: 8/3 centre, -1/3 neighbours
    c = (n // 2) + n * (n // 2)
    assert abs(A[c, c] - 8 / 3) < 1e-14
    assert abs(A[c, c + 1] + 1 / 3) < 1e-14 and abs(A[c, c + n + 1] + 1 / 3) < 1e-14


@pytest.mark.parametrize("geom,dim,p,nel", [(0, 2, 3, 5), (1, 2, 2, 6), (1, 2, 4, 4), (0, 3, 2, 3)])
def test_neumann_row_sums_vanish_and_symmetry(geom, dim, p, nel):
    """Full (boundary-kept) stiffness: partition of unity gives grad(sum Phi) = 0,
    so every row sums to 0; A and M are symmetric."""
    A = O.assemble_only(dim, geom, nel, 0, p, p, p + 1, 0)
    s = np.asarray(A.sum(axis=1)).ravel()
    assert np.abs(s).max() < 1e-12 * abs(A).max()
    assert abs(A - A.T).max() < 1e-14 * abs(A).max()
    M = O.assemble_only(dim, geom, nel, 1, p, p, p + 1, 0)
    assert abs(M - M.T).max() < 1e-16 * 10


@pytest.mark.parametrize("geom,dim,p,nel,area,tol", [
    (0, 2, 3, 4, 1.0, 1e-14), (0, 3, 2, 3, 1.0, 1e-14),
    (1, 2, 2, 8, 0.75 * np.pi, 1e-6), (1, 2, 5, 16, 0.75 * np.pi, 1e-12)])
def test_mass_and_transfer_sum_to_area(geom, dim, p, nel, area, tol):
    M = O.assemble_only(dim, geom, nel, 1, p, p, p + 1, 0)
    assert abs(M.sum() - area) < tol * 10
    P = O.assemble_only(dim, geom, nel, 1, p, 1, p + 1, 0)
    assert abs(P.sum() - area) < tol * 10


@pytest.mark.parametrize("p,nel", [(2, 6), (3, 5)])
def test_lumped_masses_are_basis_integrals(p, nel):
    """Row-sum lumping over the full mass matrix equals int Phi_i (partition of
    unity); on the box this is a product of 1-D B-spline integrals."""
    o = O.Oracle(2, p, nel, ilut=False)
    tp = _knots(p, nel)
    ints = []
    for i in range(nel + p):
        c = np.zeros(nel + p); c[i] = 1
        ints.append(BSpline(tp, c, p).integrate(0, 1))
    ints = np.array(ints)[1:-1]
    assert np.allclose(o.mlp(), np.kron(ints, ints), rtol=1e-13, atol=0)
    t1 = _knots(1, nel)
    ints1 = []
    for i in range(nel + 1):
        c = np.zeros(nel + 1); c[i] = 1
        ints1.append(BSpline(t1, c, 1).integrate(0, 1))
    ints1 = np.array(ints1)[1:-1]
    assert np.allclose(o.ml1(), np.kron(ints1, ints1), rtol=1e-13, atol=0)


@pytest.mark.parametrize("geom,dim,p,nel", [(0, 2, 3, 6), (1, 2, 4, 6), (0, 3, 2, 4)])
def test_transfers_reproduce_constants_on_full_spaces(geom, dim, p, nel):
    """Without elimination, (M_p^L)^-1 P_1^p 1 = 1 and (M_1^L)^-1 P_p^1 1 = 1
    (partition of unity of both bases plus row-sum lumping)."""
    P = O.assemble_only(dim, geom, nel, 1, p, 1, p + 1, 0)   # degree p rows x degree 1 cols
    Mp = O.assemble_only(dim, geom, nel, 1, p, p, p + 1, 0)
    M1 = O.assemble_only(dim, geom, nel, 1, 1, 1, p + 1, 0)
    mlp = np.asarray(Mp.sum(axis=1)).ravel()
    ml1 = np.asarray(M1.sum(axis=1)).ravel()
    one1 = np.ones(P.shape[1]); onep = np.ones(P.shape[0])
    assert np.abs(P @ one1 / mlp - 1).max() < 1e-12
    assert np.abs(P.T @ onep / ml1 - 1).max() < 1e-12


def test_interior_operators_are_submatrices():
    """The V-cycle's interior operators are the full ones with boundary rows and
    columns removed (elimination of the boundary functions)."""
    p, nel = 3, 5
    o = O.Oracle(2, p, nel, ilut=False)
    Pf = O.assemble_only(2, 0, nel, 1, p, 1, p + 1, 0).toarray()
    nbp, nb1 = nel + p, nel + 1
    ip = [ix + nbp * iy for iy in range(1, nbp - 1) for ix in range(1, nbp - 1)]
    i1 = [ix + nb1 * iy for iy in range(1, nb1 - 1) for ix in range(1, nb1 - 1)]
    assert np.array_equal(o.P().toarray(), Pf[np.ix_(ip, i1)])
    assert np.array_equal(o.R().toarray(), Pf[np.ix_(ip, i1)].T)


@pytest.mark.parametrize("dim,nel", [(2, 32), (3, 16)])
def test_rediscretised_p1_equals_galerkin_on_box(dim, nel):
    """Nested degree-1 spaces with exact quadrature: A_{2h,1} = P^T A_{h,1} P for
    the canonical prolongation P (Section 3, coarse grid operator)."""
    o = O.Oracle(dim, 2, nel, ilut=False)
    assert o.nlev == int(np.log2(nel // 8)) + 1
    for lev in range(o.nlev - 1):
        Af, Ac, P = o.A1(lev), o.A1(lev + 1), o.Ph(lev)
        G = (P.T @ Af @ P).toarray()
        assert np.abs(G - Ac.toarray()).max() < 1e-13 * abs(Ac).max()
    assert o.level_nel[o.nlev - 1] == 8


def test_annulus_prolongation_is_exact_embedding():
    """The canonical prolongation embeds coarse degree-1 B-splines exactly in
    the fine ones, whatever the geometry map: check on sampled points."""
    o = O.Oracle(2, 2, 16, geom=O.GEOM_ANNULUS, rhs=O.RHS_ANNULUS, ilut=False)
    P = o.Ph(0).toarray()
    tf, tc = O.knots(1, 16), O.knots(1, 8)
    rng = np.random.default_rng(3)
    for _ in range(20):
        xi, eta = rng.uniform(0, 1, 2)
        vf = np.kron(O.basis(tf, 1, eta)[0][1:-1], O.basis(tf, 1, xi)[0][1:-1])
        vc = np.kron(O.basis(tc, 1, eta)[0][1:-1], O.basis(tc, 1, xi)[0][1:-1])
        assert np.abs(vf @ P - vc).max() < 1e-14


def _galerkin_l2(dim, p, nel, geom=0, rhs=0):
    o = O.Oracle(dim, p, nel, geom=geom, rhs=rhs, ilut=False)
    A = o.A().tocsc()
    u = spla.spsolve(A, o.f())
    return o.l2_error(u)


@pytest.mark.parametrize("p", [2, 3])
def test_l2_error_decays_like_h_to_p_plus_1(p):
    hs = [4, 8, 16, 32]
    errs = [_galerkin_l2(2, p, n) for n in hs]
    slopes = np.diff(np.log(errs)) / np.diff(np.log(1.0 / np.array(hs)))
    assert slopes[-1] >= p + 1 - 0.3, (errs, slopes)


def test_l2_error_decay_annulus_and_cube():
    e = [_galerkin_l2(2, 2, n, geom=1, rhs=1) for n in (8, 16, 32)]
    s = np.log(e[1] / e[2]) / np.log(2)
    assert s >= 3 - 0.3, e
    e3 = [_galerkin_l2(3, 2, n) for n in (4, 8)]
    assert np.log(e3[0] / e3[1]) / np.log(2) >= 3 - 0.5, e3
