// Host setup: spline spaces and Galerkin assembly of every operator of the
// p-multigrid solve phase.
//
//   Section 2: open uniform knot vectors, B-splines of degree p, tensor
//     products, geometry map F, Galerkin matrix A_{h,p} and load vector.
//   Section 3, "Prolongation and restriction": mass matrices M_p, M_1, the
//     transfer matrix P_1^p (int phi_{i,p} phi_{j,1}), row-sum lumping.
//   Section 3, "Coarse grid operator": degree-1 operators by
//     rediscretisation on meshes h, 2h, 4h, ... (h-multigrid at p = 1).
//
// On the unit box every operator is a sum of Kronecker products of 1-D
// matrices (tensor basis, separable integrand, tensor Gauss rule), which is
// how it is assembled here; on the quarter annulus an element loop with the
// geometry map is used.  Quadrature: p+1 Gauss points per direction for the
// degree-p operators and the transfer matrix, 2 for degree-1 operators.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>

#include "pmg_host.hpp"

namespace pmg {

static void parallel_for(int64_t n, int threads, const std::function<void(int64_t, int64_t)>& fn) {
  if (threads <= 1 || n < 2 * threads) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> pool;
  int64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    pool.emplace_back([&, b, e] { fn(b, e); });
  }
  for (auto& th : pool) th.join();
}

// --------------------------------------------------------------- quadrature
// Golub-Welsch: the nodes of the n-point Gauss-Legendre rule are the
// eigenvalues of the symmetric tridiagonal Jacobi matrix of the Legendre
// recurrence (zero diagonal, off-diagonal b_k = k / sqrt(4 k^2 - 1)); the
// weight of a node is 2 v_0^2 / |v|^2 for its eigenvector v.  Eigenvalues
// are found by bisection on Sturm counts (the number of negative pivots of
// J - x I), eigenvector components by the matrix's own three-term
// recurrence from v_0 = 1, so w = 2 / sum_k v_k^2.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  std::vector<double> b2(n > 1 ? n - 1 : 1), bk(n > 1 ? n - 1 : 1);
  for (int k = 1; k < n; ++k) {
    bk[k - 1] = k / std::sqrt(4.0 * k * k - 1.0);
    b2[k - 1] = bk[k - 1] * bk[k - 1];
  }
  // eigenvalues of J below t
  auto below = [&](double t) {
    int cnt = 0;
    double q = -t;
    if (q < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
      if (q == 0.0) q = 1e-300;
      q = -t - b2[k - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int i = 0; i < n; ++i) {
    // the (i+1)-th smallest eigenvalue lies in [-1, 1]
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (below(mid) > i) hi = mid; else lo = mid;
    }
    const double t = 0.5 * (lo + hi);
    double vm = 0.0, v = 1.0, ss = 1.0;
    for (int k = 1; k < n; ++k) {
      const double vn = (t * v - (k > 1 ? bk[k - 2] * vm : 0.0)) / bk[k - 1];
      vm = v;
      v = vn;
      ss += v * v;
    }
    x[i] = t;
    w[i] = 2.0 / ss;
  }
}

// ------------------------------------------------------------------ splines
// Open uniform knot vector: p+1 zeros, k/nel, p+1 ones.
static std::vector<double> open_knots(int p, int nel) {
  std::vector<double> t(nel + 2 * p + 1);
  for (int i = 0; i <= p; ++i) {
    t[i] = 0.0;
    t[nel + p + i] = 1.0;
  }
  for (int k = 1; k < nel; ++k) t[p + k] = (double)k / (double)nel;
  return t;
}

// Non-zero B-splines of degree p on knot span s (t[s] <= u < t[s+1]):
// N[j] = phi_{s-p+j,p}(u), j = 0..p, by the triangular scheme on the left
// and right knot distances; dN[j] their first derivatives from the degree
// p-1 values.
static void span_basis(const std::vector<double>& t, int s, int p, double u, double* N, double* dN) {
  double left[16], right[16], Nm[16];
  auto run = [&](int q, double* out) {
    out[0] = 1.0;
    for (int j = 1; j <= q; ++j) {
      left[j] = u - t[s + 1 - j];
      right[j] = t[s + j] - u;
      double saved = 0.0;
      for (int r = 0; r < j; ++r) {
        double tmp = out[r] / (right[r + 1] + left[j - r]);
        out[r] = saved + right[r + 1] * tmp;
        saved = left[j - r] * tmp;
      }
      out[j] = saved;
    }
  };
  run(p, N);
  if (!dN) return;
  if (p == 0) {
    dN[0] = 0.0;
    return;
  }
  run(p - 1, Nm);  // Nm[j] = phi_{s-p+1+j, p-1}, j = 0..p-1
  for (int j = 0; j <= p; ++j) {
    int i = s - p + j;
    double a = 0.0, b = 0.0;
    if (j >= 1) {
      double d = t[i + p] - t[i];
      if (d > 0) a = p * Nm[j - 1] / d;
    }
    if (j <= p - 1) {
      double d = t[i + p + 1] - t[i + 1];
      if (d > 0) b = p * Nm[j] / d;
    }
    dN[j] = a - b;
  }
}

// 1-D tables on a uniform mesh: for element e and Gauss point q the values and
// derivatives of the p+1 functions e..e+p that live on it.
struct Table1D {
  int p = 0, nel = 0, nq = 0;
  std::vector<double> u, wt, val, der;
  double V(int e, int q, int a) const { return val[((size_t)e * nq + q) * (p + 1) + a]; }
  double D(int e, int q, int a) const { return der[((size_t)e * nq + q) * (p + 1) + a]; }
};

static Table1D make_table(int p, int nel, int nq) {
  Table1D T;
  T.p = p;
  T.nel = nel;
  T.nq = nq;
  std::vector<double> gx, gw;
  gauss_legendre(nq, gx, gw);
  auto t = open_knots(p, nel);
  T.u.resize((size_t)nel * nq);
  T.wt.resize((size_t)nel * nq);
  T.val.resize((size_t)nel * nq * (p + 1));
  T.der.resize((size_t)nel * nq * (p + 1));
  for (int e = 0; e < nel; ++e) {
    double a = t[p + e], b = t[p + e + 1];
    double half = 0.5 * (b - a), mid = 0.5 * (a + b);
    for (int q = 0; q < nq; ++q) {
      double u = mid + half * gx[q];
      T.u[(size_t)e * nq + q] = u;
      T.wt[(size_t)e * nq + q] = gw[q] * half;
      span_basis(t, p + e, p, u, &T.val[((size_t)e * nq + q) * (p + 1)],
                 &T.der[((size_t)e * nq + q) * (p + 1)]);
    }
  }
  return T;
}

// Banded 1-D matrix over the full function range of two degrees.
struct Band1D {
  int nr = 0, nc = 0, lo = 0, width = 0;  // entry (i, j) at i*width + (j - i + lo)
  std::vector<double> a;
  double get(int i, int j) const {
    int k = j - i + lo;
    if (k < 0 || k >= width) return 0.0;
    return a[(size_t)i * width + k];
  }
};

// kind 0: int dphi_i dphi_j; kind 1: int phi_i phi_j; kind 2: int phi_i
// dphi_j; kind 3: int dphi_i phi_j.  Rows degree pr, cols degree pc on the
// same mesh, nq Gauss points per element.
static Band1D matrix_1d(int kind, int pr, int pc, int nel, int nq) {
  Table1D Tr = make_table(pr, nel, nq), Tc = make_table(pc, nel, nq);
  Band1D B;
  B.nr = nel + pr;
  B.nc = nel + pc;
  B.lo = pr;
  B.width = pr + pc + 1;
  B.a.assign((size_t)B.nr * B.width, 0.0);
  for (int e = 0; e < nel; ++e)
    for (int q = 0; q < nq; ++q) {
      double w = Tr.wt[(size_t)e * nq + q];
      for (int a = 0; a <= pr; ++a)
        for (int b = 0; b <= pc; ++b) {
          double f = kind == 0   ? Tr.D(e, q, a) * Tc.D(e, q, b)
                     : kind == 1 ? Tr.V(e, q, a) * Tc.V(e, q, b)
                     : kind == 2 ? Tr.V(e, q, a) * Tc.D(e, q, b)
                                 : Tr.D(e, q, a) * Tc.V(e, q, b);
          int i = e + a, j = e + b;
          B.a[(size_t)i * B.width + (j - i + B.lo)] += w * f;
        }
    }
  return B;
}

// int phi_i (degree p) over (0,1), and int g phi_i for g(x) = sin(k pi x)
// (or cos(k pi x) with cosine).
static std::vector<double> integrals_1d(int p, int nel, int nq, int k, bool cosine = false) {
  Table1D T = make_table(p, nel, nq);
  std::vector<double> s(nel + p, 0.0);
  for (int e = 0; e < nel; ++e)
    for (int q = 0; q < nq; ++q) {
      double w = T.wt[(size_t)e * nq + q];
      const double x = k * M_PI * T.u[(size_t)e * nq + q];
      double g = k > 0 ? (cosine ? std::cos(x) : std::sin(x)) : 1.0;
      for (int a = 0; a <= p; ++a) s[e + a] += w * g * T.V(e, q, a);
    }
  return s;
}

// --------------------------------------------------------- tensor structure
static int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// CSR pattern of all interior pairs (i, j) with |j_a - i_a| in [-lo_a, hi]
// per direction, rows/cols numbered x fastest over interior indices.
// Interior index c corresponds to full index c + 1.
struct TensorPattern {
  int dim, nr1, nc1;  // interior functions per direction (rows, cols)
};

// Kronecker assembly on the box: value(i, j) = sum over terms of the product
// over directions of the 1-D entries (full indices), for interior rows/cols.
// `terms` lists, per term, which 1-D matrix is used in each direction.
static Csr kron_assemble(int dim, const std::vector<std::vector<const Band1D*>>& terms, int threads) {
  const Band1D* B0 = terms[0][0];
  int nr1 = B0->nr - 2, nc1 = B0->nc - 2;
  int lo = B0->lo, hi = B0->width - 1 - B0->lo;  // j - i in [-lo, hi]
  int64_t nrows = ipow(nr1, dim);
  int64_t ncols = ipow(nc1, dim);
  Csr M;
  M.nrows = (int)nrows;
  M.ncols = (int)ncols;
  M.rp.assign(nrows + 1, 0);
  auto range1 = [&](int i, int& j0, int& j1) {  // interior col range for interior row i
    j0 = std::max(0, i - lo);
    j1 = std::min(nc1 - 1, i + hi);
  };
  // counts
  std::vector<int> cnt1(nr1);
  for (int i = 0; i < nr1; ++i) {
    int j0, j1;
    range1(i, j0, j1);
    cnt1[i] = std::max(0, j1 - j0 + 1);
  }
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t t = r, c = 1;
    for (int a = 0; a < dim; ++a) {
      c *= cnt1[t % nr1];
      t /= nr1;
    }
    M.rp[r + 1] = M.rp[r] + c;
  }
  M.ci.resize(M.rp[nrows]);
  M.v.resize(M.rp[nrows]);
  parallel_for(nrows, threads, [&](int64_t rb, int64_t re) {
    for (int64_t r = rb; r < re; ++r) {
      int im[3] = {0, 0, 0}, j0[3] = {0, 0, 0}, j1[3] = {0, 0, 0};
      int64_t t = r;
      for (int a = 0; a < dim; ++a) {
        im[a] = (int)(t % nr1);
        t /= nr1;
        range1(im[a], j0[a], j1[a]);
      }
      int64_t pos = M.rp[r];
      int jz0 = dim == 3 ? j0[2] : 0, jz1 = dim == 3 ? j1[2] : 0;
      for (int jz = jz0; jz <= jz1; ++jz)
        for (int jy = j0[1]; jy <= j1[1]; ++jy)
          for (int jx = j0[0]; jx <= j1[0]; ++jx) {
            int jm[3] = {jx, jy, jz};
            double s = 0.0;
            for (const auto& term : terms) {
              double prod = 1.0;
              for (int a = 0; a < dim; ++a) prod *= term[a]->get(im[a] + 1, jm[a] + 1);
              s += prod;
            }
            int64_t col = jx + (int64_t)nc1 * (jy + (int64_t)nc1 * jz);
            M.ci[pos] = (int32_t)col;
            M.v[pos] = s;
            pos++;
          }
    }
  });
  return M;
}

// --------------------------------------------------------- CDR benchmark
// Benchmark 2 (Section 2): -div(D grad u) + v.grad u + R u on the unit
// square.  The Galerkin form int grad(phi_i).D grad(phi_j) + (v.grad phi_j)
// phi_i + R phi_j phi_i (row i the test function) is a sum of seven
// Kronecker products of 1-D matrices, x factor times y factor:
//   d11 K (x) M,  d12 G' (x) G,  d21 G (x) G',  d22 M (x) K,
//   v1 G (x) M,   v2 M (x) G,    R M (x) M,
// K = int B_i' B_j', M = int B_i B_j, G = int B_i B_j', G' = int B_i' B_j.
constexpr double kCdrD[2][2] = {{1.2, -0.7}, {-0.4, 0.9}};
constexpr double kCdrV[2] = {0.4, -0.2};
constexpr double kCdrR = 0.3;

struct CdrTerms {
  std::vector<Band1D> m;  // 14 factors, x and y of each term
  std::vector<std::vector<const Band1D*>> terms() const {
    std::vector<std::vector<const Band1D*>> t;
    for (size_t k = 0; k + 1 < m.size(); k += 2) t.push_back({&m[k], &m[k + 1]});
    return t;
  }
};

static Band1D scaled(Band1D B, double s) {
  for (double& v : B.a) v *= s;
  return B;
}

static CdrTerms cdr_terms(int p, int nel, int nq) {
  const Band1D K = matrix_1d(0, p, p, nel, nq), M = matrix_1d(1, p, p, nel, nq);
  const Band1D G = matrix_1d(2, p, p, nel, nq), Gd = matrix_1d(3, p, p, nel, nq);
  CdrTerms c;
  c.m = {scaled(K, kCdrD[0][0]), M,  scaled(Gd, kCdrD[0][1]), G, scaled(G, kCdrD[1][0]), Gd,
         scaled(M, kCdrD[1][1]), K,  scaled(G, kCdrV[0]),     M, scaled(M, kCdrV[1]),    G,
         scaled(M, kCdrR),       M};
  return c;
}

// Load vector of benchmark 2 for u = sin(k1 pi x) sin(k2 pi y): with
// a = k1 pi, b = k2 pi the right-hand side is
//   (d11 a^2 + d22 b^2 + R) sx sy - (d12 + d21) a b cx cy + v1 a cx sy + v2 b sx cy,
// separable, so f_i is a sum of products of 1-D sine / cosine integrals.
static void cdr_load(int p, int nel, const int* k, std::vector<double>& f) {
  const int nq = p + 1, np1 = nel + p - 2;
  const auto sx = integrals_1d(p, nel, nq, k[0]), cx = integrals_1d(p, nel, nq, k[0], true);
  const auto sy = integrals_1d(p, nel, nq, k[1]), cy = integrals_1d(p, nel, nq, k[1], true);
  const double a = k[0] * M_PI, b = k[1] * M_PI;
  const double css = kCdrD[0][0] * a * a + kCdrD[1][1] * b * b + kCdrR;
  const double ccc = -(kCdrD[0][1] + kCdrD[1][0]) * a * b, ccs = kCdrV[0] * a, csc = kCdrV[1] * b;
  f.resize((size_t)np1 * np1);
  for (int iy = 0; iy < np1; ++iy)
    for (int ix = 0; ix < np1; ++ix) {
      const int i = ix + 1, j = iy + 1;
      f[(size_t)iy * np1 + ix] = css * sx[i] * sy[j] + ccc * cx[i] * cy[j] + ccs * cx[i] * sy[j] + csc * sx[i] * cy[j];
    }
}

// ------------------------------------------------------------------ annulus
// F(xi, eta) = (1 + xi) C(eta), C(eta) the rational quadratic arc from (1,0)
// to (0,1) with middle control point (1,1) and weight w = sqrt(2)/2.  The arc
// lies on the unit circle, so C = (cos th, sin th) with th(eta) the angle of
// its homogeneous point (N_x, N_y) = ((1-eta)^2 + 2 w eta (1-eta),
// 2 w eta (1-eta) + eta^2); the angle's derivative is the cross product
// (N_x N_y' - N_y N_x') / (N_x^2 + N_y^2), and in polar form the Jacobian of
// F has determinant (1 + xi) th'.
struct GeoPt {
  double x, y, det, ji[2][2];  // ji = J^{-1}
};

static GeoPt annulus_map(double xi, double eta) {
  const double wm = std::sqrt(0.5);
  const double om = 1.0 - eta;
  const double nx = om * om + 2.0 * wm * eta * om, ny = 2.0 * wm * eta * om + eta * eta;
  const double dnx = -2.0 * om + 2.0 * wm * (1.0 - 2.0 * eta), dny = 2.0 * wm * (1.0 - 2.0 * eta) + 2.0 * eta;
  const double th = std::atan2(ny, nx);
  const double dth = (nx * dny - ny * dnx) / (nx * nx + ny * ny);
  const double c = std::cos(th), sn = std::sin(th), r = 1.0 + xi;
  GeoPt g;
  g.x = r * c;
  g.y = r * sn;
  // J = [[c, -r sn th'], [sn, r c th']] (columns d/dxi, d/deta)
  g.det = r * dth;
  g.ji[0][0] = c;
  g.ji[0][1] = sn;
  g.ji[1][0] = -sn / (r * dth);
  g.ji[1][1] = c / (r * dth);
  return g;
}

static double annulus_f(double x, double y) {
  double s = x * x + y * y;
  return 40.0 * x * y * y * (s - 2.0) + 2.0 * x * (s * s - 5.0 * s + 4.0);
}

static double sine_f(int dim, const int* k, const double* X) {
  double ks = 0.0, u = 1.0;
  for (int a = 0; a < dim; ++a) {
    ks += (double)k[a] * k[a];
    u *= std::sin(k[a] * M_PI * X[a]);
  }
  return M_PI * M_PI * ks * u;
}

// Element-loop assembly in 2-D with a geometry map.  Rows are interior
// degree-pr functions, columns interior degree-pc functions.  kind 0:
// stiffness, 1: mass/transfer.  Rows are split over threads by their y
// index; each thread visits the element rows that touch its functions and
// adds only into its own rows, elements in increasing order.
static Csr element_assemble_2d(int geom, int kind, int pr, int pc, int nel, int nq, int threads) {
  Table1D Tr = make_table(pr, nel, nq), Tc = make_table(pc, nel, nq);
  int nr1 = nel + pr - 2, nc1 = nel + pc - 2;
  // pattern: interior col range per interior row, per direction (overlapping supports)
  // degree-pr function i (full) lives on elements [i-pr, i]; degree-pc function
  // j on [j-pc, j]; they overlap iff j in [i - pr, i + pc].
  auto crange = [&](int ii, int& j0, int& j1) {  // interior indices
    int i = ii + 1;
    j0 = std::max(1, i - pr) - 1;
    j1 = std::min(nel + pc - 2, i + pc) - 1;
  };
  Csr M;
  M.nrows = nr1 * nr1;
  M.ncols = nc1 * nc1;
  M.rp.assign((size_t)M.nrows + 1, 0);
  std::vector<int> c1(nr1);
  for (int i = 0; i < nr1; ++i) {
    int a, b;
    crange(i, a, b);
    c1[i] = b - a + 1;
  }
  for (int r = 0; r < M.nrows; ++r) M.rp[r + 1] = M.rp[r] + (int64_t)c1[r % nr1] * c1[r / nr1];
  M.ci.resize(M.rp.back());
  M.v.assign(M.rp.back(), 0.0);
  for (int r = 0; r < M.nrows; ++r) {
    int ix = r % nr1, iy = r / nr1, x0, x1, y0, y1;
    crange(ix, x0, x1);
    crange(iy, y0, y1);
    int64_t pos = M.rp[r];
    for (int jy = y0; jy <= y1; ++jy)
      for (int jx = x0; jx <= x1; ++jx) M.ci[pos++] = jx + nc1 * jy;
  }
  int nlr = (pr + 1) * (pr + 1), nlc = (pc + 1) * (pc + 1);
  parallel_for(nr1, threads, [&](int64_t yb, int64_t ye) {
    std::vector<double> vr(nlr), gr(2 * nlr), vc(nlc), gc(2 * nlc);
    // full y-index range of owned rows: [yb+1, ye]; elements ey in [yb+1-pr, ye]
    int e0 = std::max(0, (int)yb + 1 - pr), e1 = std::min(nel - 1, (int)ye);
    for (int ey = e0; ey <= e1; ++ey)
      for (int ex = 0; ex < nel; ++ex)
        for (int qy = 0; qy < nq; ++qy)
          for (int qx = 0; qx < nq; ++qx) {
            double u = Tr.u[(size_t)ex * nq + qx], v = Tr.u[(size_t)ey * nq + qy];
            double wq = Tr.wt[(size_t)ex * nq + qx] * Tr.wt[(size_t)ey * nq + qy];
            double ji[2][2] = {{1, 0}, {0, 1}}, det = 1.0;
            if (geom == 1) {
              GeoPt g = annulus_map(u, v);
              det = g.det;
              std::memcpy(ji, g.ji, sizeof(ji));
            }
            double dw = wq * det;
            auto fill_side = [&](const Table1D& T, int p, double* vv, double* gg) {
              for (int ay = 0; ay <= p; ++ay)
                for (int ax = 0; ax <= p; ++ax) {
                  int l = ax + (p + 1) * ay;
                  double bx = T.V(ex, qx, ax), by = T.V(ey, qy, ay);
                  double hx = T.D(ex, qx, ax) * by, hy = bx * T.D(ey, qy, ay);
                  vv[l] = bx * by;
                  gg[2 * l] = ji[0][0] * hx + ji[1][0] * hy;
                  gg[2 * l + 1] = ji[0][1] * hx + ji[1][1] * hy;
                }
            };
            fill_side(Tr, pr, vr.data(), gr.data());
            fill_side(Tc, pc, vc.data(), gc.data());
            for (int ay = 0; ay <= pr; ++ay) {
              int fy = ey + ay;  // full y index of the row function
              if (fy < yb + 1 || fy > ye) continue;
              if (fy == 0 || fy == nel + pr - 1) continue;
              for (int ax = 0; ax <= pr; ++ax) {
                int fx = ex + ax;
                if (fx == 0 || fx == nel + pr - 1) continue;
                int row = (fx - 1) + nr1 * (fy - 1);
                int la = ax + (pr + 1) * ay;
                int cx0, cx1;
                crange(fx - 1, cx0, cx1);
                int rowlen = cx1 - cx0 + 1;
                for (int by = 0; by <= pc; ++by) {
                  int gy = ey + by;
                  if (gy == 0 || gy == nel + pc - 1) continue;
                  for (int bx = 0; bx <= pc; ++bx) {
                    int gx = ex + bx;
                    if (gx == 0 || gx == nel + pc - 1) continue;
                    int lb = bx + (pc + 1) * by;
                    double val = kind == 0 ? gr[2 * la] * gc[2 * lb] + gr[2 * la + 1] * gc[2 * lb + 1]
                                           : vr[la] * vc[lb];
                    int cy0, cy1;
                    crange(fy - 1, cy0, cy1);
                    int64_t pos = M.rp[row] + (int64_t)((gy - 1) - cy0) * rowlen + ((gx - 1) - cx0);
                    M.v[pos] += dw * val;
                  }
                }
              }
            }
          }
  });
  return M;
}

// f at a physical point: the built-in right-hand sides or the caller's callback.
static double rhs_value(const SetupParams& sp, int dim, const double* X) {
  if (sp.rhs == 2) return sp.fn(X, sp.fn_ctx);
  if (sp.rhs == 1) return annulus_f(X[0], X[1]);
  return sine_f(dim, sp.freq, X);
}

// Load vector and lumped mass (int Phi_i) by an element loop in 2-D.
static void element_vectors_2d(int geom, const SetupParams& sp, int p, int nel, int nq,
                               std::vector<double>* f, std::vector<double>* ml) {
  Table1D T = make_table(p, nel, nq);
  int n1 = nel + p - 2;
  if (f) f->assign((size_t)n1 * n1, 0.0);
  if (ml) ml->assign((size_t)n1 * n1, 0.0);
  for (int ey = 0; ey < nel; ++ey)
    for (int ex = 0; ex < nel; ++ex)
      for (int qy = 0; qy < nq; ++qy)
        for (int qx = 0; qx < nq; ++qx) {
          double u = T.u[(size_t)ex * nq + qx], v = T.u[(size_t)ey * nq + qy];
          double wq = T.wt[(size_t)ex * nq + qx] * T.wt[(size_t)ey * nq + qy];
          double det = 1.0, X[3] = {u, v, 0};
          if (geom == 1) {
            GeoPt g = annulus_map(u, v);
            det = g.det;
            X[0] = g.x;
            X[1] = g.y;
          }
          double fx = 0.0;
          if (f) fx = rhs_value(sp, 2, X);
          for (int ay = 0; ay <= p; ++ay) {
            int fy = ey + ay;
            if (fy == 0 || fy == nel + p - 1) continue;
            for (int ax = 0; ax <= p; ++ax) {
              int fxi = ex + ax;
              if (fxi == 0 || fxi == nel + p - 1) continue;
              double phi = T.V(ex, qx, ax) * T.V(ey, qy, ay);
              int row = (fxi - 1) + n1 * (fy - 1);
              if (f) (*f)[row] += wq * det * fx * phi;
              if (ml) (*ml)[row] += wq * det * phi;
            }
          }
        }
}

// Canonical prolongation between interior degree-1 nodes of meshes nc and
// 2 nc: coarse hat I = fine hat 2I + (fine hats 2I-1 and 2I+1) / 2, tensor
// product over directions.
static Csr canonical_prolongation(int dim, int nc) {
  int nci = nc - 1, nfi = 2 * nc - 1;
  int64_t nrows = ipow(nfi, dim);
  Csr P;
  P.nrows = (int)nrows;
  P.ncols = (int)ipow(nci, dim);
  P.rp.assign(nrows + 1, 0);
  // 1-D: fine f gets coarse c with weight 1 if f = 2c+1, 1/2 if f = 2c or 2c+2
  auto w1 = [&](int f, int* cs, double* ws) {
    int n = 0;
    if (f % 2 == 1) {
      cs[n] = (f - 1) / 2;
      ws[n++] = 1.0;
    } else {
      if (f / 2 - 1 >= 0) {
        cs[n] = f / 2 - 1;
        ws[n++] = 0.5;
      }
      if (f / 2 < nci) {
        cs[n] = f / 2;
        ws[n++] = 0.5;
      }
    }
    return n;
  };
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t t = r, m = 1;
    for (int a = 0; a < dim; ++a) {
      int cs[2];
      double ws[2];
      m *= w1((int)(t % nfi), cs, ws);
      t /= nfi;
    }
    P.rp[r + 1] = P.rp[r] + m;
  }
  P.ci.resize(P.rp.back());
  P.v.resize(P.rp.back());
  for (int64_t r = 0; r < nrows; ++r) {
    int cs[3][2], nn[3] = {1, 1, 1};
    double ws[3][2] = {{1, 0}, {1, 0}, {1, 0}};
    cs[1][0] = cs[2][0] = 0;
    int64_t t = r;
    for (int a = 0; a < dim; ++a) {
      nn[a] = w1((int)(t % nfi), cs[a], ws[a]);
      t /= nfi;
    }
    int64_t pos = P.rp[r];
    for (int c = 0; c < (dim == 3 ? nn[2] : 1); ++c)
      for (int b = 0; b < nn[1]; ++b)
        for (int a = 0; a < nn[0]; ++a) {
          int64_t col = cs[0][a] + (int64_t)nci * (cs[1][b] + (int64_t)nci * (dim == 3 ? cs[2][c] : 0));
          P.ci[pos] = (int32_t)col;
          P.v[pos] = ws[0][a] * ws[1][b] * (dim == 3 ? ws[2][c] : 1.0);
          pos++;
        }
  }
  return P;
}

Csr transpose(const Csr& A) {
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rp.assign((size_t)T.nrows + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) T.rp[A.ci[k] + 1]++;
  for (int i = 0; i < T.nrows; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.nnz());
  T.v.resize(A.nnz());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t d = pos[A.ci[k]]++;
      T.ci[d] = i;
      T.v[d] = A.v[k];
    }
  return T;
}

// Dense inverse of the (small, SPD) coarsest operator via Cholesky.
static bool dense_spd_inverse(const Csr& A, std::vector<double>& inv) {
  int n = A.nrows;
  std::vector<double> C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) C[(size_t)i * n + A.ci[k]] = A.v[k];
  for (int j = 0; j < n; ++j) {
    double s = C[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= C[(size_t)j * n + k] * C[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    double d = std::sqrt(s);
    C[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = C[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= C[(size_t)i * n + k] * C[(size_t)j * n + k];
      C[(size_t)i * n + j] = t / d;
    }
  }
  inv.assign((size_t)n * n, 0.0);
  std::vector<double> y(n), x(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= C[(size_t)i * n + k] * y[k];
      y[i] = s / C[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < n; ++k) s -= C[(size_t)k * n + i] * x[k];
      x[i] = s / C[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = x[i];
  }
  return true;
}

// Inverse of a non-singular matrix by Gaussian elimination with partial
// pivoting (the coarsest degree-1 operator of the non-symmetric problem).
static bool dense_lu_inverse(const Csr& A, std::vector<double>& inv) {
  const int n = A.nrows;
  std::vector<double> C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) C[(size_t)i * n + A.ci[k]] = A.v[k];
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int m = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(C[(size_t)i * n + k]) > std::fabs(C[(size_t)m * n + k])) m = i;
    if (!(C[(size_t)m * n + k] != 0.0) || !std::isfinite(C[(size_t)m * n + k])) return false;
    if (m != k)
      for (int j = 0; j < n; ++j) {
        std::swap(C[(size_t)k * n + j], C[(size_t)m * n + j]);
        std::swap(inv[(size_t)k * n + j], inv[(size_t)m * n + j]);
      }
    const double d = C[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      C[(size_t)k * n + j] /= d;
      inv[(size_t)k * n + j] /= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double l = C[(size_t)i * n + k];
      if (l == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        C[(size_t)i * n + j] -= l * C[(size_t)k * n + j];
        inv[(size_t)i * n + j] -= l * inv[(size_t)k * n + j];
      }
    }
  }
  return true;
}

// Load vector of a callback right-hand side on the unit cube by an element
// loop (one thread: the callback need not be thread-safe).
static void element_load_3d(const SetupParams& sp, int p, int nel, int nq, std::vector<double>& f) {
  Table1D T = make_table(p, nel, nq);
  const int n1 = nel + p - 2;
  f.assign((size_t)n1 * n1 * n1, 0.0);
  for (int ez = 0; ez < nel; ++ez)
    for (int ey = 0; ey < nel; ++ey)
      for (int ex = 0; ex < nel; ++ex)
        for (int qz = 0; qz < nq; ++qz)
          for (int qy = 0; qy < nq; ++qy)
            for (int qx = 0; qx < nq; ++qx) {
              const double X[3] = {T.u[(size_t)ex * nq + qx], T.u[(size_t)ey * nq + qy], T.u[(size_t)ez * nq + qz]};
              const double wq = T.wt[(size_t)ex * nq + qx] * T.wt[(size_t)ey * nq + qy] * T.wt[(size_t)ez * nq + qz];
              const double fw = wq * rhs_value(sp, 3, X);
              for (int az = 0; az <= p; ++az) {
                const int fz = ez + az;
                if (fz == 0 || fz == nel + p - 1) continue;
                for (int ay = 0; ay <= p; ++ay) {
                  const int fy = ey + ay;
                  if (fy == 0 || fy == nel + p - 1) continue;
                  const double vyz = T.V(ey, qy, ay) * T.V(ez, qz, az);
                  for (int ax = 0; ax <= p; ++ax) {
                    const int fxi = ex + ax;
                    if (fxi == 0 || fxi == nel + p - 1) continue;
                    f[(fxi - 1) + (size_t)n1 * ((fy - 1) + (size_t)n1 * (fz - 1))] += fw * (T.V(ex, qx, ax) * vyz);
                  }
                }
              }
            }
}

int load_vector(const SetupParams& sp, std::vector<double>& f, std::string& msg) {
  const int dim = sp.dim, p = sp.p, nel = sp.nel;
  const int64_t n = ipow(nel + p - 2, dim);
  if (sp.rhs == 2) {
    if (!sp.fn) {
      msg = "the callback right-hand side needs f";
      return 1;
    }
    if (dim == 2) element_vectors_2d(sp.geom, sp, p, nel, p + 1, &f, nullptr);
    else element_load_3d(sp, p, nel, p + 1, f);
    return 0;
  }
  if (sp.pde == 1) {
    cdr_load(p, nel, sp.freq, f);
    return 0;
  }
  if (sp.geom == 0 && sp.rhs == 0) {
    std::vector<std::vector<double>> sf(dim);
    double ks = 0.0;
    for (int a = 0; a < dim; ++a) {
      sf[a] = integrals_1d(p, nel, p + 1, sp.freq[a]);
      ks += (double)sp.freq[a] * sp.freq[a];
    }
    const int np1 = nel + p - 2;
    f.resize(n);
    for (int64_t r = 0; r < n; ++r) {
      int64_t t = r;
      double s = 1.0;
      for (int a = 0; a < dim; ++a) {
        s *= sf[a][(int)(t % np1) + 1];
        t /= np1;
      }
      f[r] = M_PI * M_PI * ks * s;
    }
    return 0;
  }
  if (dim != 2) {
    msg = "this right-hand side is two-dimensional";
    return 1;
  }
  element_vectors_2d(sp.geom, sp, p, nel, p + 1, &f, nullptr);
  return 0;
}

int assemble_all(const SetupParams& sp, HostOps& H, std::string& msg) {
  auto t0 = std::chrono::steady_clock::now();
  const int dim = sp.dim, p = sp.p, nel = sp.nel;
  H.dim = dim;
  H.p = p;
  H.nel = nel;
  H.n = (int)ipow(nel + p - 2, dim);
  // coarse space of the transfers: degree 1 (direct projection, Section 3)
  // or degree p - 1 on the same mesh (indirect projection, Appendix A)
  const int cdeg = std::max(1, sp.cdeg);
  H.n1 = (int)ipow(nel + cdeg - 2, dim);
  const int th = std::max(1, sp.threads);
  if (sp.geom == 0) {
    // ---- unit box: Kronecker products of 1-D Galerkin matrices
    Band1D K = matrix_1d(0, p, p, nel, p + 1), M = matrix_1d(1, p, p, nel, p + 1);
    std::vector<std::vector<const Band1D*>> termsA;
    for (int a = 0; a < dim; ++a) {
      std::vector<const Band1D*> t(dim, &M);
      t[a] = &K;
      termsA.push_back(t);
    }
    if (sp.pde == 1) {
      const CdrTerms c = cdr_terms(p, nel, p + 1);
      H.A = kron_assemble(dim, c.terms(), th);
    } else {
      H.A = kron_assemble(dim, termsA, th);
      // the factors as bands of their interior rows (interior index i is
      // full index i + 1)
      const int nk = nel + p - 2, w = 2 * p + 1;
      H.nk = nk;
      H.kK.assign((size_t)nk * w, 0.0);
      H.kM.assign((size_t)nk * w, 0.0);
      for (int i = 0; i < nk; ++i)
        for (int d = -p; d <= p; ++d)
          if (i + d >= 0 && i + d < nk) {
            H.kK[(size_t)i * w + d + p] = K.get(i + 1, i + d + 1);
            H.kM[(size_t)i * w + d + p] = M.get(i + 1, i + d + 1);
          }
    }
    Band1D X = matrix_1d(1, p, cdeg, nel, p + 1);
    H.P = kron_assemble(dim, {std::vector<const Band1D*>(dim, &X)}, th);
    H.xnr = X.nr;
    H.xlo = X.lo;
    H.xw = X.width;
    H.kX = X.a;
    // lumped masses = int Phi_i = product of 1-D integrals; load vector
    // f = pi^2 (sum k^2) prod_a int sin(k_a pi x) phi
    auto ip = integrals_1d(p, nel, p + 1, 0), i1 = integrals_1d(cdeg, nel, cdeg + 1, 0);
    H.mlp.resize(H.n);
    H.ml1.resize(H.n1);
    H.f.resize(H.n);
    std::vector<std::vector<double>> sf(dim);
    double ks = 0.0;
    for (int a = 0; a < dim; ++a) {
      sf[a] = integrals_1d(p, nel, p + 1, sp.freq[a]);
      ks += (double)sp.freq[a] * sp.freq[a];
    }
    int np1 = nel + p - 2, n11 = nel + cdeg - 2;
    for (int64_t r = 0; r < H.n; ++r) {
      int64_t t = r;
      double m = 1.0, s = 1.0;
      for (int a = 0; a < dim; ++a) {
        int i = (int)(t % np1) + 1;
        t /= np1;
        m *= ip[i];
        s *= sf[a][i];
      }
      H.mlp[r] = m;
      H.f[r] = M_PI * M_PI * ks * s;
    }
    if (sp.pde == 1) cdr_load(p, nel, sp.freq, H.f);
    if (sp.rhs == 2) {
      const int rc = load_vector(sp, H.f, msg);
      if (rc) return rc;
    }
    for (int64_t r = 0; r < H.n1; ++r) {
      int64_t t = r;
      double m = 1.0;
      for (int a = 0; a < dim; ++a) {
        m *= i1[(int)(t % n11) + 1];
        t /= n11;
      }
      H.ml1[r] = m;
    }
  } else {
    if (dim != 2) {
      msg = "the quarter annulus is two-dimensional";
      return 1;
    }
    H.A = element_assemble_2d(1, 0, p, p, nel, p + 1, th);
    H.P = element_assemble_2d(1, 1, p, cdeg, nel, p + 1, th);
    element_vectors_2d(1, sp, p, nel, p + 1, &H.f, &H.mlp);
    element_vectors_2d(1, sp, cdeg, nel, cdeg + 1, nullptr, &H.ml1);
  }
  H.R = transpose(H.P);
  if (sp.consistent_mass) {
    // Appendix B: consistent interior mass matrices of degree p and 1
    if (sp.geom == 0) {
      Band1D Mq = matrix_1d(1, p, p, nel, p + 1), M1q = matrix_1d(1, cdeg, cdeg, nel, cdeg + 1);
      H.Mp = kron_assemble(dim, {std::vector<const Band1D*>(dim, &Mq)}, th);
      H.M1 = kron_assemble(dim, {std::vector<const Band1D*>(dim, &M1q)}, th);
    } else {
      H.Mp = element_assemble_2d(1, 1, p, p, nel, p + 1, th);
      H.M1 = element_assemble_2d(1, 1, cdeg, cdeg, nel, cdeg + 1, th);
    }
  }
  // ---- degree-1 hierarchy by rediscretisation
  int ne = nel;
  H.A1.clear();
  H.k1K.clear();
  H.k1M.clear();
  H.Ph.clear();
  H.Rh.clear();
  H.lnel.clear();
  H.ln.clear();
  if (cdeg > 1) {
    // indirect projection: the coarse correction is a V-cycle of the degree
    // p - 1 level, set up by the caller; no degree-1 hierarchy here
    H.nlev = 0;
    H.n_coarse = 0;
    H.coarse_inv.clear();
    H.t_assembly = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return 0;
  }
  for (;;) {
    H.lnel.push_back(ne);
    H.ln.push_back((int)ipow(ne - 1, dim));
    H.k1K.emplace_back();
    H.k1M.emplace_back();
    if (sp.geom == 0 && sp.pde == 1) {
      const CdrTerms c = cdr_terms(1, ne, 2);
      H.A1.push_back(kron_assemble(dim, c.terms(), th));
    } else if (sp.geom == 0) {
      Band1D K1 = matrix_1d(0, 1, 1, ne, 2), M1 = matrix_1d(1, 1, 1, ne, 2);
      std::vector<std::vector<const Band1D*>> t1;
      for (int a = 0; a < dim; ++a) {
        std::vector<const Band1D*> t(dim, &M1);
        t[a] = &K1;
        t1.push_back(t);
      }
      H.A1.push_back(kron_assemble(dim, t1, th));
      // the 1-D factors as bands of the interior rows (interior index i is
      // full index i + 1)
      const int nk = ne - 1;
      std::vector<double>&bK = H.k1K.back(), &bM = H.k1M.back();
      bK.assign((size_t)nk * 3, 0.0);
      bM.assign((size_t)nk * 3, 0.0);
      for (int i = 0; i < nk; ++i)
        for (int d = -1; d <= 1; ++d)
          if (i + d >= 0 && i + d < nk) {
            bK[(size_t)i * 3 + d + 1] = K1.get(i + 1, i + d + 1);
            bM[(size_t)i * 3 + d + 1] = M1.get(i + 1, i + d + 1);
          }
    } else {
      H.A1.push_back(element_assemble_2d(1, 0, 1, 1, ne, 2, th));
    }
    if (ne <= sp.coarse_min || ne % 2 != 0 || H.A1.size() >= 24) break;
    H.Ph.push_back(canonical_prolongation(dim, ne / 2));
    H.Rh.push_back(transpose(H.Ph.back()));
    ne /= 2;
  }
  H.nlev = (int)H.A1.size();
  H.n_coarse = H.ln.back();
  if (H.n_coarse > 1024) {
    msg = "coarsest degree-1 level has " + std::to_string(H.n_coarse) +
          " unknowns (limit 1024): use n_elem = 2^k * m with m <= coarse_min_elems";
    return 1;
  }
  if (H.n_coarse > 0 && sp.pde == 1 && !dense_lu_inverse(H.A1.back(), H.coarse_inv)) {
    msg = "coarsest degree-1 operator is singular";
    return 4;
  }
  if (H.n_coarse > 0 && sp.pde != 1 && !dense_spd_inverse(H.A1.back(), H.coarse_inv)) {
    msg = "coarsest degree-1 operator is not positive definite";
    return 4;
  }
  H.t_assembly = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return 0;
}

}  // namespace pmg
