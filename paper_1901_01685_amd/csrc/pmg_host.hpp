// Host-side setup of the p-multigrid solver: spline spaces, Galerkin
// assembly, lumped transfers, the degree-1 hierarchy and ILUT.  Built with
// -ffp-contract=off so every sum is evaluated in the order written.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pmg {

// Host CSR with sorted columns.
struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
  int64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

struct SetupParams {
  int dim = 2, p = 2, nel = 16, geom = 0, rhs = 0, pde = 0;
  bool consistent_mass = false;  // also assemble the consistent mass matrices Mp, M1
  int cdeg = 1;  // degree of the coarse space of the p-transfers (p - 1: indirect projection)
  int freq[3] = {1, 1, 1};
  double (*fn)(const double*, void*) = nullptr;  // rhs 2: f at a physical point (caller's callback)
  void* fn_ctx = nullptr;
  double tau = 1e-12, fill = 1.0;
  int limit_mode = 0;
  int coarse_min = 8;
  int threads = 1;
  int ordering = 1, nd_leaf = 8;
};

struct HostOps {
  int dim = 2, p = 2, nel = 16;
  int n = 0, n1 = 0;           // interior unknowns at degree p and 1
  Csr A, L, U;                 // L, U: factors of P A P^T; U diagonal first
  std::vector<int32_t> perm;   // position i of the factors holds unknown perm[i]
  Csr R;                       // P_p^1 (n1 x n)
  Csr P;                       // P_1^p (n x n1)
  Csr Mp, M1;                  // consistent interior mass matrices (only when requested)
  std::vector<double> f, mlp, ml1;
  // Poisson on the unit box: A is the sum over the directions a of the
  // Kronecker product of the 1-D stiffness K in direction a and the 1-D mass
  // M in the others.  kK, kM hold the interior rows of K and M as bands (nk
  // rows of 2p+1 entries for the offsets -p..p, 0 outside the grid); empty
  // for other problems.
  int nk = 0;
  std::vector<double> kK, kM;
  // On the unit box P is the Kronecker product of one 1-D matrix X (rows the
  // degree-p functions, columns the coarse-space ones, full indices) in every
  // direction, and R its transpose: X as a band (entry (i, j) at
  // i * xw + j - i + xlo, xnr rows); empty on other geometries.
  int xnr = 0, xlo = 0, xw = 0;
  std::vector<double> kX;
  int nlev = 0;
  std::vector<int> lnel, ln;   // elements / unknowns per degree-1 level
  std::vector<Csr> A1;         // rediscretised degree-1 operators
  // Poisson on the unit box: A1[l] = K1 (x) M1 + M1 (x) K1 (+ the third term
  // in 3-D) from the level's 1-D degree-1 stiffness and mass, as bands of
  // their interior rows (3 entries per row, 0 outside the grid); empty
  // vectors for other problems.
  std::vector<std::vector<double>> k1K, k1M;
  std::vector<Csr> Ph, Rh;     // canonical prolongation level l <- l+1, and transpose
  std::vector<double> coarse_inv;  // dense inverse of the coarsest A1 (row-major)
  int n_coarse = 0;
  double t_assembly = 0, t_ilut = 0;
};

// Gauss-Legendre rule on [-1,1], increasing nodes.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Builds everything but ILUT.  Returns 0 or a pmg_status code; msg on error.
int assemble_all(const SetupParams& sp, HostOps& H, std::string& msg);

// Load vector f_i = int f Phi_i of the problem's right-hand side (interior
// functions of degree sp.p), as assemble_all computes it.
int load_vector(const SetupParams& sp, std::vector<double>& f, std::string& msg);

// ILUT(tau, m) of A in its given row order; returns 0, or PMG_EZEROPIVOT with
// the failing row in bad_row.
int ilut_factor(const Csr& A, double tau, double fill, int mode, int threads, Csr& L, Csr& U,
                int& bad_row);

Csr transpose(const Csr& A);

// ILUT ordering over grid lines (natural or nested dissection).
std::vector<int32_t> line_ordering(int dim, int nint, int p, int ordering, int leaf);

// An order of the rows of P A P^T (P the ordering above) in which every row
// comes after the rows its factorisation can depend on: the blocks of the
// nested dissection by height in the dissection tree (uncut boxes first,
// then separators level by level), the rows of the blocks of one height
// interleaved, each block's rows in increasing order.  Rows of independent
// blocks are therefore factored side by side.  Natural order: the rows in
// order.
std::vector<int32_t> factor_ticket_order(int dim, int nint, int p, int ordering, int leaf);

// Segments of the triangular-solve schedules: runs of whole grid lines of at
// most max_rows rows (at least one line) that never cross a block of the
// nested dissection, as row starts in the ordering (plus the row count).
std::vector<int32_t> line_segments(int dim, int nint, int p, int ordering, int leaf, int max_rows);

// B = P A P^T, B_ij = A_{perm[i], perm[j]}, columns sorted.
Csr permute(const Csr& A, const std::vector<int32_t>& perm, int threads);

}  // namespace pmg
