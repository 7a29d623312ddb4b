"""Pins of the oracle's basis, quadrature and geometry against mathematics and
library routines (partition of unity, Section 2; scipy's B-splines; numpy's
Gauss-Legendre rule; the exact quarter circle)."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle as O


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6, 8, 12])
def test_gauss_matches_numpy(n):
    x, w = O.gauss(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)
    # exact for degree 2n-1
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


def test_knots_open_uniform():
    t = O.knots(3, 4)
    assert np.array_equal(t, [0, 0, 0, 0, 0.25, 0.5, 0.75, 1, 1, 1, 1])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("nel", [1, 3, 8])
def test_basis_matches_scipy_and_partition_of_unity(p, nel):
    t = O.knots(p, nel)
    nb = nel + p
    rng = np.random.default_rng(p * 100 + nel)
    pts = np.concatenate([rng.uniform(0, 1, 200), [0.0, 1.0]])
    for xi in pts:
        v, d = O.basis(t, p, xi)
        # partition of unity (Section 2) and non-negativity
        assert abs(v.sum() - 1.0) < 1e-14
        assert v.min() >= -1e-15
        # scipy's independent B-spline evaluation
        for i in range(nb):
            c = np.zeros(nb)
            c[i] = 1.0
            bs = BSpline(t, c, p, extrapolate=False)
            ref = bs(xi)
            if np.isnan(ref):
                ref = 0.0
            assert abs(v[i] - ref) < 1e-13, (i, xi)
            if p >= 1 and 0.0 < xi < 1.0:
                refd = bs.derivative()(xi)
                assert abs(d[i] - refd) < 1e-10 * max(1.0, abs(refd)), (i, xi)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_basis_support_ends_and_continuity(p):
    nel = 5
    t = O.knots(p, nel)
    nb = nel + p
    # interpolation only at the two end points
    v0, _ = O.basis(t, p, 0.0)
    v1, _ = O.basis(t, p, 1.0)
    assert v0[0] == 1.0 and abs(v0[1:]).max() == 0.0
    assert v1[-1] == 1.0 and abs(v1[:-1]).max() == 0.0
    # support [t_i, t_{i+p+1})
    for xi in np.linspace(0.01, 0.99, 37):
        v, _ = O.basis(t, p, xi)
        for i in range(nb):
            inside = t[i] <= xi < t[i + p + 1]
            if not inside:
                assert v[i] == 0.0
    # C^{p-1} at interior knots: values (and derivatives for p >= 2) agree
    # from both sides
    dlt = 1e-9
    for k in range(1, nel):
        kn = k / nel
        vl, dl = O.basis(t, p, kn - dlt)
        vr, dr = O.basis(t, p, kn + dlt)
        assert abs(vl - vr).max() < 1e-6
        if p >= 2:
            assert abs(dl - dr).max() < 1e-5 * nel * nel * p * p


def test_p1_hats_closed_form():
    nel = 4
    t = O.knots(1, nel)
    for xi in np.linspace(0, 1, 41):
        v, _ = O.basis(t, 1, xi)
        for i in range(nel + 1):
            hat = max(0.0, 1.0 - abs(xi * nel - i))
            assert abs(v[i] - hat) < 1e-15


def test_annulus_geometry():
    rng = np.random.default_rng(1)
    for _ in range(200):
        xi, eta = rng.uniform(0, 1, 2)
        X, det = O.geom(O.GEOM_ANNULUS, 2, [xi, eta])
        assert abs(np.hypot(*X) - (1.0 + xi)) < 1e-14      # |F| = 1 + xi
        assert X[0] >= -1e-15 and X[1] >= -1e-15           # first quadrant
        assert det > 0
        # Jacobian determinant by central differences
        h = 1e-6
        Xa, _ = O.geom(1, 2, [xi + h, eta]); Xb, _ = O.geom(1, 2, [xi - h, eta])
        Ya, _ = O.geom(1, 2, [xi, eta + h]); Yb, _ = O.geom(1, 2, [xi, eta - h])
        J = np.column_stack([(Xa - Xb) / (2 * h), (Ya - Yb) / (2 * h)])
        assert abs(np.linalg.det(J) - det) < 1e-7
    # end points of the arc
    X, _ = O.geom(1, 2, [0.0, 0.0]); assert np.allclose(X, [1, 0], atol=1e-15)
    X, _ = O.geom(1, 2, [1.0, 1.0]); assert np.allclose(X, [0, 2], atol=1e-15)


def test_annulus_forcing_is_minus_laplacian():
    """Benchmark 1: f = -Lap u checked by a fourth-order finite-difference
    Laplacian of the exact solution."""
    rng = np.random.default_rng(2)
    h = 1e-3
    for _ in range(50):
        r = rng.uniform(1.05, 1.95); th = rng.uniform(0.05, 1.5)
        x, y = r * np.cos(th), r * np.sin(th)
        u = lambda a, b: O.exact_u(O.RHS_ANNULUS, 2, [1, 1], [a, b])
        def d2(fa, fb, f0, fa2, fb2):
            return (-fa2 + 16 * fa - 30 * f0 + 16 * fb - fb2) / (12 * h * h)
        lap = d2(u(x + h, y), u(x - h, y), u(x, y), u(x + 2 * h, y), u(x - 2 * h, y)) + \
              d2(u(x, y + h), u(x, y - h), u(x, y), u(x, y + 2 * h), u(x, y - 2 * h))
        f = O.rhs_f(O.RHS_ANNULUS, 2, [1, 1], [x, y])
        assert abs(f + lap) < 1e-5 * max(1.0, abs(f))
    # the exact solution vanishes on the annulus boundary
    for th in np.linspace(0, np.pi / 2, 9):
        for r in (1.0, 2.0):
            assert abs(O.exact_u(1, 2, [1, 1], [r * np.cos(th), r * np.sin(th)])) < 1e-13


@pytest.mark.parametrize("k", [(1, 1, 1), (2, 3, 1), (4, 1, 2)])
def test_sine_forcing(k):
    X = [0.3, 0.7, 0.2]
    for dim in (2, 3):
        u = np.prod([np.sin(k[a] * np.pi * X[a]) for a in range(dim)])
        f = O.rhs_f(O.RHS_SINE, dim, k, X)
        assert abs(f - np.pi ** 2 * sum(kk * kk for kk in k[:dim]) * u) < 1e-12
