// Exercises the library's host setup (assembly, orderings, permutation and
// the threaded ILUT) under AddressSanitizer and UndefinedBehaviorSanitizer
// (CPU build, no device code).  Exit status 0 when every check holds; the
// sanitizers abort on the first memory or undefined-behaviour error.
#include <cmath>
#include <cstdio>
#include <string>

#include "../../paper_1901_01685_amd/csrc/pmg_host.hpp"

static double sine_cb(const double* x, void*) { return std::sin(M_PI * x[0]) * std::sin(M_PI * x[1]); }

static int run(int dim, int p, int nel, int geom, int pde, int mode, int ordering, int rhs, int threads) {
  pmg::SetupParams sp;
  sp.dim = dim;
  sp.p = p;
  sp.nel = nel;
  sp.geom = geom;
  sp.rhs = rhs;
  sp.pde = pde;
  sp.fn = sine_cb;
  sp.limit_mode = mode;
  sp.ordering = ordering;
  sp.threads = threads;
  pmg::HostOps H;
  std::string msg;
  if (int rc = pmg::assemble_all(sp, H, msg)) {
    std::printf("assemble_all failed %d: %s\n", rc, msg.c_str());
    return 1;
  }
  H.perm = pmg::line_ordering(dim, nel + p - 2, p, ordering, 8);
  pmg::Csr Ap = pmg::permute(H.A, H.perm, threads);
  int bad = -1;
  if (int rc = pmg::ilut_factor(Ap, 1e-12, 1.0, mode, threads, H.L, H.U, bad)) {
    std::printf("ilut failed %d at row %d\n", rc, bad);
    return 1;
  }
  // the threaded factorisation equals the sequential one
  pmg::Csr L1, U1;
  int bad2 = -1;
  if (int rc = pmg::ilut_factor(Ap, 1e-12, 1.0, mode, 1, L1, U1, bad2)) return rc;
  if (L1.rp != H.L.rp || L1.ci != H.L.ci || L1.v != H.L.v || U1.rp != H.U.rp || U1.ci != H.U.ci || U1.v != H.U.v) {
    std::printf("threaded ILUT differs from the sequential one\n");
    return 1;
  }
  std::vector<double> f;
  if (int rc = pmg::load_vector(sp, f, msg)) {
    std::printf("load_vector failed %d: %s\n", rc, msg.c_str());
    return 1;
  }
  const pmg::Csr T = pmg::transpose(H.A);
  std::printf("dim %d p %d nel %d geom %d pde %d mode %d ordering %d rhs %d: n %d nnz(A) %lld nnz(L) %lld nnz(U) %lld\n",
              dim, p, nel, geom, pde, mode, ordering, rhs, H.n, (long long)H.A.nnz(), (long long)H.L.nnz(),
              (long long)H.U.nnz());
  return (T.nnz() == H.A.nnz() && (int)f.size() == H.n) ? 0 : 1;
}

// The device factorisation's ticket order must put every row after the rows
// its elimination can reach: checked against the pattern of the exact LU
// (unlimited fill), which contains every pivot any ILUT meets.
static int check_ticket_order(int dim, int p, int nel, int ordering) {
  pmg::SetupParams sp;
  sp.dim = dim;
  sp.p = p;
  sp.nel = nel;
  sp.threads = 4;
  pmg::HostOps H;
  std::string msg;
  if (pmg::assemble_all(sp, H, msg)) return 1;
  const int nint = nel + p - 2;
  H.perm = pmg::line_ordering(dim, nint, p, ordering, 8);
  pmg::Csr Ap = pmg::permute(H.A, H.perm, 4);
  pmg::Csr L, U;
  int bad = -1;
  if (pmg::ilut_factor(Ap, 0.0, 0.0, 0, 4, L, U, bad)) return 1;
  const std::vector<int32_t> order = pmg::factor_ticket_order(dim, nint, p, ordering, 8);
  if ((int)order.size() != H.n) return 1;
  std::vector<int> pos(H.n, -1);
  for (int t = 0; t < H.n; ++t) {
    if (order[t] < 0 || order[t] >= H.n || pos[order[t]] >= 0) return 1;
    pos[order[t]] = t;
  }
  int64_t violations = 0;
  for (int i = 0; i < H.n; ++i)
    for (int64_t k = L.rp[i]; k < L.rp[i + 1]; ++k) violations += pos[L.ci[k]] > pos[i];
  std::printf("ticket order dim %d p %d nel %d ordering %d: n %d, exact-LU dependencies %lld, violations %lld\n", dim,
              p, nel, ordering, H.n, (long long)L.nnz(), (long long)violations);
  return violations != 0;
}

int main() {
  int bad = 0;
  bad |= check_ticket_order(2, 2, 40, 1);
  bad |= check_ticket_order(2, 5, 32, 1);
  bad |= check_ticket_order(3, 2, 12, 1);
  bad |= check_ticket_order(3, 3, 10, 1);
  bad |= check_ticket_order(2, 3, 24, 0);
  bad |= run(2, 2, 16, 0, 0, 2, 1, 0, 4);
  bad |= run(2, 3, 32, 0, 0, 0, 1, 2, 3);
  bad |= run(2, 4, 16, 1, 0, 1, 0, 1, 2);
  bad |= run(2, 3, 16, 0, 1, 2, 1, 0, 4);
  bad |= run(3, 2, 8, 0, 0, 2, 1, 0, 4);
  bad |= run(3, 3, 6, 0, 0, 0, 0, 2, 2);
  std::printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
