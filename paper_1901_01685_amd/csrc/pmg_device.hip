// Device operators, V-cycle orchestration and the C ABI (include/pmg.h).
//
// The solve phase of the p-multigrid method (Section 3: two-grid correction
// steps 1-5 with direct projection to p = 1, lumped L2 transfers, ILUT
// smoothing, h-multigrid coarse solve; Section 5: stand-alone iteration) runs
// entirely in the kernels of kernels.hpp on the caller's HIP stream; the host
// only sequences launches and reads back one FP64 norm per V-cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "pmg_internal.hpp"

using pmgdev::DevMat;
using pmgdev::TriSched;
using pmgdev::Workspace;
using pmgdev::fail;

namespace pmgdev {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

pmg_status fail(pmg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

pmg_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? PMG_ENOMEM : PMG_EDEVICE;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

}  // namespace pmgdev

pmg_handle_s::~pmg_handle_s() {
  if (on_device) {
    hipSetDevice(device);
    hipDeviceSynchronize();
    ops.release();
    for (auto& v : ev)
      for (hipEvent_t e : v) hipEventDestroy(e);
  }
}

namespace {

constexpr int kMaxCsrBlocks = 4096;

int pick_group(double avg) {
  if (avg >= 128) return 64;
  if (avg >= 48) return 32;
  if (avg >= 20) return 16;
  if (avg >= 8) return 8;
  return 4;
}

unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

unsigned csr_grid(int nrows, int G) { return std::min<unsigned>(nblocks(nrows, 256 / G), kMaxCsrBlocks); }

// Wait lists of the segment-ordered triangular solves.  Forward: chunk
// (s, c) reads rows of segments < s; for each such segment the number of its
// leading rows that must be final.  Backward (upper == true): segments are
// taken from the last, chunks from the end of the segment, and a segment's
// progress counts rows final from its end.
void build_schedule(const pmg::Csr& T, int seg_len, bool upper, TriSched& S) {
  const int n = T.nrows;
  S.seg_len = seg_len;
  S.nseg = n / seg_len;
  S.nch = (seg_len + 63) / 64;
  S.wptr.assign((size_t)S.nseg * S.nch + 1, 0);
  S.waits.clear();
  std::vector<int> need(S.nseg, 0), touched;
  for (int q = 0; q < S.nseg; ++q) {
    const int s = upper ? S.nseg - 1 - q : q;
    for (int cc = 0; cc < S.nch; ++cc) {
      const int c = upper ? S.nch - 1 - cc : cc;
      const int r0 = s * seg_len + c * 64;
      const int r1 = std::min(s * seg_len + seg_len, r0 + 64);
      touched.clear();
      for (int row = r0; row < r1; ++row) {
        const int64_t kb = T.rp[row] + (upper ? 1 : 0);
        for (int64_t k = kb; k < T.rp[row + 1]; ++k) {
          const int col = T.ci[k];
          const int sc = col / seg_len;
          if (sc == s) continue;
          const int req = upper ? (sc * seg_len + seg_len - col) : (col - sc * seg_len + 1);
          if (need[sc] == 0) touched.push_back(sc);
          need[sc] = std::max(need[sc], req);
        }
      }
      std::sort(touched.begin(), touched.end());
      for (int sc : touched) {
        S.waits.push_back(make_int2(sc, need[sc]));
        need[sc] = 0;
      }
      S.wptr[(size_t)q * S.nch + cc + 1] = (int)S.waits.size();
    }
  }
  S.nwaits = (int)S.waits.size();
  // split index per row: lower -> first entry with column >= chunk start;
  // upper -> first entry (after the diagonal) with column >= chunk end
  S.ks.assign(n, 0);
  for (int row = 0; row < n; ++row) {
    const int s = row / seg_len, c = (row - s * seg_len) / 64;
    const int cs = s * seg_len + c * 64, ce = std::min(s * seg_len + seg_len, cs + 64);
    int64_t k = T.rp[row] + (upper ? 1 : 0);
    if (!upper) {
      while (k < T.rp[row + 1] && T.ci[k] < cs) ++k;
    } else {
      while (k < T.rp[row + 1] && T.ci[k] < ce) ++k;
    }
    S.ks[row] = (int)k;
  }
  // depth of the dependency DAG (for the record)
  std::vector<int> lev(n, 0);
  int mx = 0;
  if (!upper) {
    for (int i = 0; i < n; ++i) {
      int l = 0;
      for (int64_t k = T.rp[i]; k < T.rp[i + 1]; ++k) l = std::max(l, lev[T.ci[k]]);
      lev[i] = l + 1;
      mx = std::max(mx, l + 1);
    }
  } else {
    for (int i = n - 1; i >= 0; --i) {
      int l = 0;
      for (int64_t k = T.rp[i] + 1; k < T.rp[i + 1]; ++k) l = std::max(l, lev[T.ci[k]]);
      lev[i] = l + 1;
      mx = std::max(mx, l + 1);
    }
  }
  S.dag_levels = mx;
}

pmg_status upload_mat(pmgdev::DevArena& mem, const pmg::Csr& M, DevMat& D, bool with32) {
  D.nrows = M.nrows;
  D.ncols = M.ncols;
  D.nnz = M.nnz();
  if (D.nnz >= (int64_t)INT32_MAX) return fail(PMG_EINVAL, "operator has more than 2^31 non-zeros");
  std::vector<int> rp32(M.rp.begin(), M.rp.end());
  pmg_status s;
  if ((s = mem.upload(&D.rp, rp32.data(), rp32.size()))) return s;
  if ((s = mem.upload(&D.ci, M.ci.data(), M.ci.size()))) return s;
  if ((s = mem.upload(&D.v, M.v.data(), M.v.size()))) return s;
  if (with32) {
    std::vector<float> v32(M.v.begin(), M.v.end());
    if ((s = mem.upload(&D.v32, v32.data(), v32.size()))) return s;
  }
  D.G = pick_group(D.nrows ? (double)D.nnz / D.nrows : 1.0);
  return PMG_OK;
}

// Per-step timing with HIP events on the launch stream (pmg_profile_*).
struct ProfScope {
  pmg_handle h;
  int cls;
  hipStream_t st;
  ProfScope(pmg_handle h_, int c, hipStream_t s) : h(h_), cls(c), st(s) {
    if (h->profiling) h->prof_mark(cls, st);
  }
  ~ProfScope() {
    if (h->profiling) h->prof_mark(cls, st);
  }
};

// ------------------------------------------------------------ launch helpers
template <typename T, int G>
void csr_launch_g(int mode, int nrows, const int* rows, const DevMat& M, const T* v, const T* x,
                  const T* b, const T* d, T* out, double* partial, hipStream_t st) {
  if (nrows <= 0) return;
  const unsigned grid = csr_grid(nrows, G);
  switch (mode) {
    case pmg::kResid:
      pmg::csr_kernel<T, G, pmg::kResid><<<grid, 256, 0, st>>>(nrows, rows, M.rp, M.ci, v, x, b, d, out, partial);
      break;
    case pmg::kPlain:
      pmg::csr_kernel<T, G, pmg::kPlain><<<grid, 256, 0, st>>>(nrows, rows, M.rp, M.ci, v, x, b, d, out, partial);
      break;
    case pmg::kScale:
      pmg::csr_kernel<T, G, pmg::kScale><<<grid, 256, 0, st>>>(nrows, rows, M.rp, M.ci, v, x, b, d, out, partial);
      break;
    case pmg::kScaleAdd:
      pmg::csr_kernel<T, G, pmg::kScaleAdd><<<grid, 256, 0, st>>>(nrows, rows, M.rp, M.ci, v, x, b, d, out, partial);
      break;
    case pmg::kAdd:
      pmg::csr_kernel<T, G, pmg::kAdd><<<grid, 256, 0, st>>>(nrows, rows, M.rp, M.ci, v, x, b, d, out, partial);
      break;
    case pmg::kGS:
      pmg::csr_kernel<T, G, pmg::kGS><<<grid, 256, 0, st>>>(nrows, rows, M.rp, M.ci, v, x, b, d, out, partial);
      break;
  }
}

template <typename T>
void csr_launch(int mode, int nrows, const int* rows, const DevMat& M, const T* v, const T* x, const T* b,
                const T* d, T* out, double* partial, hipStream_t st) {
  switch (M.G) {
    case 4: csr_launch_g<T, 4>(mode, nrows, rows, M, v, x, b, d, out, partial, st); break;
    case 8: csr_launch_g<T, 8>(mode, nrows, rows, M, v, x, b, d, out, partial, st); break;
    case 16: csr_launch_g<T, 16>(mode, nrows, rows, M, v, x, b, d, out, partial, st); break;
    case 32: csr_launch_g<T, 32>(mode, nrows, rows, M, v, x, b, d, out, partial, st); break;
    default: csr_launch_g<T, 64>(mode, nrows, rows, M, v, x, b, d, out, partial, st); break;
  }
}

template <typename T>
void fill(T* p, int64_t n, T val, hipStream_t st) {
  if (n > 0) pmg::fill_kernel<T><<<nblocks(n, 256), 256, 0, st>>>(n, p, val);
}

double read_norm(Workspace& ws, hipStream_t st) {
  pmgdev::enqueue_norm_readback(ws, st);
  hipStreamSynchronize(st);
  return std::sqrt(ws.host_scalar[0]);
}

template <typename T>
void lower_impl(pmg_handle h, Workspace& ws, const T* r, T* y, bool fp32, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_LOWER, st);
  const T* lv = fp32 ? (const T*)h->L.v32 : (const T*)h->L.v;
  pmg::trisolve_lower<T><<<h->tl.nseg, 64, 0, st>>>(h->tl.nseg, h->tl.seg_len, h->L.rp, h->L.ci, lv, h->tl.d_ks,
                                                     h->d_perm, r, y, h->tl.d_wptr, h->tl.d_waits, ws.prog_l,
                                                     ws.tickets);
}

template <typename T>
void upper_impl(pmg_handle h, Workspace& ws, T* y, T* x, bool fp32, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_UPPER, st);
  const T* uv = fp32 ? (const T*)h->U.v32 : (const T*)h->U.v;
  pmg::trisolve_upper<T><<<h->tu.nseg, 64, 0, st>>>(h->tu.nseg, h->tu.seg_len, h->U.rp, h->U.ci, uv, h->tu.d_ks,
                                                     h->d_perm, y, x, h->tu.d_wptr, h->tu.d_waits, ws.prog_u,
                                                     ws.tickets + 2);
}

template <typename T>
void smooth_impl(pmg_handle h, Workspace& ws, const T* r, T* x, T* y, bool fp32, hipStream_t st) {
  lower_impl<T>(h, ws, r, y, fp32, st);
  upper_impl<T>(h, ws, y, x, fp32, st);
}

void gs_sweeps(pmg_handle h, int l, const double* b, double* e, int nsweep, hipStream_t st) {
  for (int s = 0; s < nsweep; ++s)
    for (int c = 0; c < h->colors; ++c)
      csr_launch<double>(pmg::kGS, h->color_cnt[l][c], h->color_rows[l][c], h->A1[l], h->A1[l].v, nullptr, b,
                         nullptr, e, nullptr, st);
}

void hcycle(pmg_handle h, Workspace& ws, int l, const double* b, double* e, hipStream_t st) {
  const pmg::HostOps& H = h->H;
  if (l == H.nlev - 1) {
    pmg::dense_matvec<<<1, 256, 0, st>>>(H.n_coarse, h->coarse_inv, b, e);
    return;
  }
  gs_sweeps(h, l, b, e, h->opt.nu1, st);
  double* r = ws.hr[l];
  csr_launch<double>(pmg::kResid, h->A1[l].nrows, nullptr, h->A1[l], h->A1[l].v, e, b, nullptr, r, ws.partial, st);
  double* bc = ws.hb[l + 1];
  double* ec = ws.he[l + 1];
  csr_launch<double>(pmg::kPlain, h->Rh[l].nrows, nullptr, h->Rh[l], h->Rh[l].v, r, nullptr, nullptr, bc, nullptr,
                     st);
  fill<double>(ec, H.ln[l + 1], 0.0, st);
  hcycle(h, ws, l + 1, bc, ec, st);
  csr_launch<double>(pmg::kAdd, h->Ph[l].nrows, nullptr, h->Ph[l], h->Ph[l].v, ec, nullptr, nullptr, e, nullptr,
                     st);
  gs_sweeps(h, l, b, e, h->opt.nu2, st);
}

void coarse_impl(pmg_handle h, Workspace& ws, const double* r1, double* e1, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_COARSE, st);
  fill<double>(e1, h->H.n1, 0.0, st);
  for (int c = 0; c < h->opt.coarse_cycles; ++c) hcycle(h, ws, 0, r1, e1, st);
}

void restrict64(pmg_handle h, const double* r, double* r1, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_RESTRICT, st);
  csr_launch<double>(pmg::kScale, h->R.nrows, nullptr, h->R, h->R.v, r, nullptr, h->ml1_inv, r1, nullptr, st);
}

void prolong64(pmg_handle h, const double* e1, double* x, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_PROLONG, st);
  csr_launch<double>(pmg::kScaleAdd, h->P.nrows, nullptr, h->P, h->P.v, e1, nullptr, h->mlp_inv, x, nullptr, st);
}

// One FP32 V-cycle on A c = r32 from c = 0 (inner step of defect
// correction): pre-smoothing, residual, restriction, FP64 h-multigrid at
// p = 1, prolongation, residual, post-smoothing.  Result in ws.c32.
void vcycle32(pmg_handle h, Workspace& ws, hipStream_t st) {
  const int n = h->H.n, n1 = h->H.n1;
  float* c = ws.c32;
  float* t = ws.t32;  // inner residual r32 - A c
  fill<float>(c, n, 0.0f, st);
  const int nu1 = h->opt.nu1, nu2 = h->opt.nu2;
  const float* cur = ws.r32;  // residual of the correction equation at c = 0
  for (int k = 0; k < nu1; ++k) {
    smooth_impl<float>(h, ws, cur, c, ws.y32, true, st);
    csr_launch<float>(pmg::kResid, n, nullptr, h->A, h->A.v32, c, ws.r32, nullptr, t, ws.partial, st);
    cur = t;
  }
  if (n1 > 0) {
    csr_launch<float>(pmg::kScale, h->R.nrows, nullptr, h->R, h->R.v32, cur, nullptr, h->ml1_inv32, ws.q32,
                      nullptr, st);
    pmg::cast_kernel<float, double><<<nblocks(n1, 256), 256, 0, st>>>(n1, ws.q32, ws.r1);
    coarse_impl(h, ws, ws.r1, ws.e1, st);
    pmg::cast_kernel<double, float><<<nblocks(n1, 256), 256, 0, st>>>(n1, ws.e1, ws.q32);
    csr_launch<float>(pmg::kScaleAdd, h->P.nrows, nullptr, h->P, h->P.v32, ws.q32, nullptr, h->mlp_inv32, c,
                      nullptr, st);
    csr_launch<float>(pmg::kResid, n, nullptr, h->A, h->A.v32, c, ws.r32, nullptr, t, ws.partial, st);
    cur = t;
  }
  for (int k = 0; k < nu2; ++k) {
    smooth_impl<float>(h, ws, cur, c, ws.y32, true, st);
    if (k + 1 < nu2) {
      csr_launch<float>(pmg::kResid, n, nullptr, h->A, h->A.v32, c, ws.r32, nullptr, t, ws.partial, st);
      cur = t;
    }
  }
}

bool valid_problem(const pmg_problem* p, std::string& msg) {
  if (!p) { msg = "problem is NULL"; return false; }
  if (p->dim != 2 && p->dim != 3) { msg = "dim must be 2 or 3"; return false; }
  if (p->degree < 1 || p->degree > 10) { msg = "degree must be in 1..10"; return false; }
  if (p->n_elem < 2) { msg = "n_elem must be >= 2"; return false; }
  if (p->geometry != PMG_GEOM_BOX && p->geometry != PMG_GEOM_QUARTER_ANNULUS) { msg = "unknown geometry"; return false; }
  if (p->geometry == PMG_GEOM_QUARTER_ANNULUS && p->dim != 2) { msg = "the quarter annulus is 2-D"; return false; }
  if (p->rhs_kind != PMG_RHS_SINE && p->rhs_kind != PMG_RHS_ANNULUS) { msg = "unknown rhs_kind"; return false; }
  if (p->rhs_kind == PMG_RHS_ANNULUS && p->dim != 2) { msg = "the annulus right-hand side is 2-D"; return false; }
  if (p->dim == 3 && p->geometry != PMG_GEOM_BOX) { msg = "3-D supports the unit cube only"; return false; }
  for (int a = 0; a < p->dim; ++a)
    if (p->freq[a] < 1 && p->rhs_kind == PMG_RHS_SINE) { msg = "freq must be >= 1"; return false; }
  double n = std::pow((double)(p->n_elem + p->degree - 2), p->dim);
  if (n < 1 || n > 2.0e9) { msg = "problem size out of range"; return false; }
  return true;
}

}  // namespace

// ----------------------------------------------------------- shared internals
namespace pmgdev {

size_t workspace_bytes(pmg_handle h, bool mixed, bool request_vectors) {
  const pmg::HostOps& H = h->H;
  size_t b = 8 * (2 * (size_t)H.n + 2 * (size_t)std::max(H.n1, 1)) + 8 * (size_t)h->partial_cap + 32;
  for (int l = 0; l < H.nlev; ++l) b += 8 * (size_t)H.ln[l] * (l == 0 ? 1 : 3);
  b += 4 * (size_t)(h->tl.nseg + h->tu.nseg + 2) + 16;
  if (mixed) b += 4 * (4 * (size_t)H.n + (size_t)std::max(H.n1, 1));
  if (request_vectors) b += 16 * (size_t)H.n;
  return b;
}

void zero(double* p, int64_t n, hipStream_t st) { fill<double>(p, n, 0.0, st); }

pmg_status alloc_workspace(pmg_handle h, Workspace& ws, bool mixed, bool request_vectors, hipStream_t st) {
  const pmg::HostOps& H = h->H;
  const int64_t n = H.n, n1 = std::max(H.n1, 1);
  ws.n = H.n;
  ws.n1 = H.n1;
  ws.mixed = mixed;
  pmg_status s;
  DevArena& m = ws.mem;
  if ((s = m.alloc(&ws.y, n))) return s;
  if ((s = m.alloc(&ws.r, n))) return s;
  if ((s = m.alloc(&ws.r1, n1))) return s;
  if ((s = m.alloc(&ws.e1, n1))) return s;
  if ((s = m.alloc(&ws.partial, h->partial_cap))) return s;
  if ((s = m.alloc(&ws.scalar, 4))) return s;
  ws.hb.assign(H.nlev, nullptr);
  ws.he.assign(H.nlev, nullptr);
  ws.hr.assign(H.nlev, nullptr);
  for (int l = 1; l < H.nlev; ++l) {
    if ((s = m.alloc(&ws.hb[l], H.ln[l]))) return s;
    if ((s = m.alloc(&ws.he[l], H.ln[l]))) return s;
  }
  for (int l = 0; l < H.nlev; ++l)
    if ((s = m.alloc(&ws.hr[l], H.ln[l]))) return s;
  if ((s = m.alloc(&ws.prog_l, h->tl.nseg + 1))) return s;
  if ((s = m.alloc(&ws.prog_u, h->tu.nseg + 1))) return s;
  if ((s = m.alloc(&ws.tickets, 4))) return s;
  fill<int>(ws.prog_l, h->tl.nseg + 1, 0, st);
  fill<int>(ws.prog_u, h->tu.nseg + 1, 0, st);
  fill<unsigned>(ws.tickets, 4, 0u, st);
  PMG_HIP_OK(hipGetLastError());
  if (mixed) {
    if ((s = m.alloc(&ws.r32, n))) return s;
    if ((s = m.alloc(&ws.c32, n))) return s;
    if ((s = m.alloc(&ws.y32, n))) return s;
    if ((s = m.alloc(&ws.t32, n))) return s;
    if ((s = m.alloc(&ws.q32, n1))) return s;
  }
  if (request_vectors) {
    if ((s = m.alloc(&ws.b, n))) return s;
    if ((s = m.alloc(&ws.x, n))) return s;
  }
  PMG_HIP_OK(hipHostMalloc((void**)&ws.host_scalar, 4 * sizeof(double), hipHostMallocDefault));
  if (!st) PMG_HIP_OK(hipDeviceSynchronize());
  return PMG_OK;
}

void residual64(pmg_handle h, Workspace& ws, const double* b, const double* x, double* r, bool norm,
                hipStream_t st) {
  ProfScope ps(h, PMG_PROF_RESIDUAL, st);
  csr_launch<double>(pmg::kResid, h->A.nrows, nullptr, h->A, h->A.v, x, b, nullptr, r, ws.partial, st);
  if (norm) pmg::reduce_partials<<<1, 256, 0, st>>>((int)csr_grid(h->A.nrows, h->A.G), ws.partial, ws.scalar);
}

void enqueue_norm_readback(Workspace& ws, hipStream_t st) {
  hipMemcpyAsync(ws.host_scalar, ws.scalar, sizeof(double), hipMemcpyDeviceToHost, st);
}

// One FP64 V-cycle; r holds b - A x on entry and exit.
void vcycle64(pmg_handle h, Workspace& ws, const double* b, double* x, double* r, bool norm, hipStream_t st) {
  const int nu1 = h->opt.nu1, nu2 = h->opt.nu2;
  for (int k = 0; k < nu1; ++k) {
    smooth_impl<double>(h, ws, r, x, ws.y, false, st);
    residual64(h, ws, b, x, r, false, st);
  }
  if (h->H.n1 > 0) {
    restrict64(h, r, ws.r1, st);
    coarse_impl(h, ws, ws.r1, ws.e1, st);
    prolong64(h, ws.e1, x, st);
    residual64(h, ws, b, x, r, nu2 == 0 && norm, st);
  }
  for (int k = 0; k < nu2; ++k) {
    smooth_impl<double>(h, ws, r, x, ws.y, false, st);
    residual64(h, ws, b, x, r, k == nu2 - 1 && norm, st);
  }
  if (nu2 == 0 && h->H.n1 == 0) residual64(h, ws, b, x, r, norm, st);
}

void mixed_step(pmg_handle h, Workspace& ws, const double* b, double* x, hipStream_t st) {
  const int n = h->H.n;
  pmg::cast_kernel<double, float><<<nblocks(n, 256), 256, 0, st>>>(n, ws.r, ws.r32);
  vcycle32(h, ws, st);
  pmg::add_cast_kernel<float><<<nblocks(n, 256), 256, 0, st>>>(n, ws.c32, x);
  residual64(h, ws, b, x, ws.r, true, st);
}

}  // namespace pmgdev

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* pmg_status_str(pmg_status s) {
  switch (s) {
    case PMG_OK: return "ok";
    case PMG_EINVAL: return "invalid argument";
    case PMG_ENOMEM: return "out of memory";
    case PMG_EDEVICE: return "device error";
    case PMG_EZEROPIVOT: return "zero pivot in ILUT";
    case PMG_EDIVERGED: return "diverged";
    case PMG_EMAXIT: return "maximum iterations reached";
    case PMG_ENAN: return "non-finite residual";
    case PMG_EBUDGET: return "device memory budget exceeded";
  }
  return "unknown status";
}

const char* pmg_last_error(void) { return pmgdev::last_error_cstr(); }

pmg_status pmg_default_options(pmg_options* o) {
  if (!o) return fail(PMG_EINVAL, "options pointer is NULL");
  std::memset(o, 0, sizeof(*o));
  o->ilut_tau = 1e-12;
  o->ilut_fill = 1.0;
  o->ilut_limit_mode = PMG_LIMIT_PER_PART;
  o->nu1 = 1;
  o->nu2 = 1;
  o->coarse_cycles = 2;
  o->coarse_min_elems = 8;
  o->gs_variant = PMG_GS_MULTICOLOR;
  o->precision = PMG_FP64;
  o->max_iter = 100;
  o->diverge_ratio = 1e10;
  o->device = 0;
  o->setup_threads = 0;
  o->ordering = PMG_ORDER_NESTED_DISSECTION;
  o->nd_leaf = 8;
  return PMG_OK;
}

pmg_status pmg_setup(const pmg_problem* prob, const pmg_options* opt, pmg_handle* out) {
  pmgdev::set_error("");
  if (!out) return fail(PMG_EINVAL, "out pointer is NULL");
  *out = nullptr;
  std::string msg;
  if (!valid_problem(prob, msg)) return fail(PMG_EINVAL, msg);
  pmg_options o;
  if (opt) o = *opt; else pmg_default_options(&o);
  if (o.nu1 < 0 || o.nu2 < 0 || o.coarse_cycles < 1 || o.coarse_min_elems < 1 || o.max_iter < 0 ||
      !(o.ilut_tau >= 0) || o.gs_variant != PMG_GS_MULTICOLOR ||
      (o.precision != PMG_FP64 && o.precision != PMG_FP32_IN_FP64) ||
      (o.ilut_limit_mode != PMG_LIMIT_PER_PART && o.ilut_limit_mode != PMG_LIMIT_PER_ROW) || o.device < -1 ||
      (o.ordering != PMG_ORDER_NATURAL && o.ordering != PMG_ORDER_NESTED_DISSECTION) || o.nd_leaf < 1)
    return fail(PMG_EINVAL, "invalid options");
  std::unique_ptr<pmg_handle_s> h(new pmg_handle_s());
  h->prob = *prob;
  h->opt = o;
  pmg::SetupParams sp;
  sp.dim = prob->dim;
  sp.p = prob->degree;
  sp.nel = prob->n_elem;
  sp.geom = prob->geometry;
  sp.rhs = prob->rhs_kind;
  for (int a = 0; a < 3; ++a) sp.freq[a] = prob->freq[a] > 0 ? prob->freq[a] : 1;
  sp.tau = o.ilut_tau;
  sp.fill = o.ilut_fill;
  sp.limit_mode = o.ilut_limit_mode;
  sp.coarse_min = o.coarse_min_elems;
  sp.ordering = o.ordering;
  sp.nd_leaf = o.nd_leaf;
  int hw = (int)std::thread::hardware_concurrency();
  sp.threads = o.setup_threads > 0 ? o.setup_threads : std::max(1, std::min(hw, 16));
  int rc = pmg::assemble_all(sp, h->H, msg);
  if (rc) return fail((pmg_status)rc, msg);
  pmg::HostOps& H = h->H;
  {
    auto t0 = std::chrono::steady_clock::now();
    int bad = -1;
    H.perm = pmg::line_ordering(prob->dim, prob->n_elem + prob->degree - 2, prob->degree, o.ordering, o.nd_leaf);
    pmg::Csr Ap = pmg::permute(H.A, H.perm, sp.threads);
    rc = pmg::ilut_factor(Ap, o.ilut_tau, o.ilut_fill, o.ilut_limit_mode, sp.threads, H.L, H.U, bad);
    H.t_ilut = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc) return fail(PMG_EZEROPIVOT, "ILUT: zero or non-finite pivot in row " + std::to_string(bad));
  }
  const int seg_len = prob->n_elem + prob->degree - 2;
  build_schedule(H.L, seg_len, false, h->tl);
  build_schedule(H.U, seg_len, true, h->tu);
  h->colors = 1 << prob->dim;
  h->partial_cap = (int)csr_grid(H.n, pick_group((double)H.A.nnz() / std::max(H.n, 1))) + 16;
  for (int l = 0; l < H.nlev; ++l) {
    const int G1 = pick_group((double)H.A1[l].nnz() / std::max(H.ln[l], 1));
    h->partial_cap = std::max(h->partial_cap, (int)csr_grid(H.ln[l], G1) + 16);
  }

  // info
  pmg_info& I = h->info;
  I.n = H.n;
  I.n1 = H.n1;
  I.nnz_a = H.A.nnz();
  I.nnz_l = H.L.nnz();
  I.nnz_u = H.U.nnz();
  I.nnz_r = H.R.nnz();
  I.nnz_p = H.P.nnz();
  I.nlev = H.nlev;
  I.n_coarsest = H.n_coarse;
  I.nnz_a1 = H.A1.empty() ? 0 : H.A1[0].nnz();
  I.segments = h->tl.nseg;
  I.seg_len = seg_len;
  I.dag_levels_l = h->tl.dag_levels;
  I.dag_levels_u = h->tu.dag_levels;
  const int64_t n = H.n, n1 = H.n1;
  I.bytes_spmv = 12 * I.nnz_a + 4 * (n + 1) + 24 * n;
  I.bytes_trisolve_l = 12 * I.nnz_l + 4 * (n + 1) + 16 * n;
  I.bytes_trisolve_u = 12 * I.nnz_u + 4 * (n + 1) + 32 * n;
  I.bytes_restrict = 12 * I.nnz_r + 4 * (n1 + 1) + 8 * n + 16 * n1;
  I.bytes_prolong = 12 * I.nnz_p + 4 * (n + 1) + 8 * n1 + 24 * n;
  int64_t bc = 0;
  for (int l = 0; l < H.nlev; ++l) {
    const int64_t nl = H.ln[l];
    if (l == H.nlev - 1) {
      bc += 8 * (int64_t)H.n_coarse * H.n_coarse + 16 * nl;
      continue;
    }
    const int64_t a1 = H.A1[l].nnz() * 12 + 4 * (nl + 1);
    const int64_t sweeps = o.nu1 + o.nu2;
    bc += sweeps * (a1 + 24 * nl) + (a1 + 24 * nl) + (12 * H.Rh[l].nnz() + 8 * nl + 8 * H.ln[l + 1]) +
          (12 * H.Ph[l].nnz() + 16 * nl + 8 * H.ln[l + 1]) + 8 * H.ln[l + 1];
  }
  I.bytes_coarse = o.coarse_cycles * bc + 8 * n1;
  I.bytes_vcycle = (o.nu1 + o.nu2 + (n1 > 0 ? 1 : 0)) * I.bytes_spmv +
                   (o.nu1 + o.nu2) * (I.bytes_trisolve_l + I.bytes_trisolve_u) +
                   (n1 > 0 ? I.bytes_restrict + I.bytes_coarse + I.bytes_prolong : 0);
  I.t_assembly = H.t_assembly;
  I.t_ilut = H.t_ilut;

  if (o.device >= 0) {
    auto t0 = std::chrono::steady_clock::now();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= o.device)
      return fail(PMG_EDEVICE, "no HIP device " + std::to_string(o.device));
    PMG_HIP_OK(hipSetDevice(o.device));
    h->device = o.device;
    h->on_device = true;
    const bool mixed = o.precision == PMG_FP32_IN_FP64;
    pmgdev::DevArena& m = h->ops;
    pmg_status s;
    if ((s = upload_mat(m, H.A, h->A, mixed))) return s;
    if ((s = upload_mat(m, H.L, h->L, mixed))) return s;
    if ((s = upload_mat(m, H.U, h->U, mixed))) return s;
    if (n1 > 0) {
      if ((s = upload_mat(m, H.R, h->R, mixed))) return s;
      if ((s = upload_mat(m, H.P, h->P, mixed))) return s;
    }
    h->A1.resize(H.nlev);
    h->Ph.resize(H.Ph.size());
    h->Rh.resize(H.Rh.size());
    for (int l = 0; l < H.nlev; ++l)
      if ((s = upload_mat(m, H.A1[l], h->A1[l], false))) return s;
    for (size_t l = 0; l < H.Ph.size(); ++l) {
      if ((s = upload_mat(m, H.Ph[l], h->Ph[l], false))) return s;
      if ((s = upload_mat(m, H.Rh[l], h->Rh[l], false))) return s;
    }
    // multicolour row lists per level
    h->color_rows.assign(H.nlev, std::vector<int*>(h->colors, nullptr));
    h->color_cnt.assign(H.nlev, std::vector<int>(h->colors, 0));
    for (int l = 0; l < H.nlev; ++l) {
      const int n1d = H.lnel[l] - 1;
      std::vector<std::vector<int>> lists(h->colors);
      for (int i = 0; i < H.ln[l]; ++i) {
        int t = i, col = 0;
        for (int a = 0; a < prob->dim; ++a) {
          col |= ((t % n1d) & 1) << a;
          t /= n1d;
        }
        lists[col].push_back(i);
      }
      for (int c = 0; c < h->colors; ++c) {
        h->color_cnt[l][c] = (int)lists[c].size();
        if ((s = m.upload(&h->color_rows[l][c], lists[c].data(), lists[c].size()))) return s;
      }
    }
    std::vector<double> inv(H.n), inv1(std::max<int64_t>(n1, 1));
    for (int64_t i = 0; i < n; ++i) inv[i] = 1.0 / H.mlp[i];
    for (int64_t i = 0; i < n1; ++i) inv1[i] = 1.0 / H.ml1[i];
    if ((s = m.upload(&h->f, H.f.data(), H.f.size()))) return s;
    if ((s = m.upload(&h->mlp_inv, inv.data(), inv.size()))) return s;
    if ((s = m.upload(&h->ml1_inv, inv1.data(), inv1.size()))) return s;
    if ((s = m.upload(&h->coarse_inv, H.coarse_inv.data(), H.coarse_inv.size()))) return s;
    if (mixed) {
      std::vector<float> a(inv.begin(), inv.end()), b(inv1.begin(), inv1.end());
      if ((s = m.upload(&h->mlp_inv32, a.data(), a.size()))) return s;
      if ((s = m.upload(&h->ml1_inv32, b.data(), b.size()))) return s;
    }
    if ((s = m.upload(&h->tl.d_wptr, h->tl.wptr.data(), h->tl.wptr.size()))) return s;
    if ((s = m.upload(&h->tl.d_waits, h->tl.waits.data(), h->tl.waits.size()))) return s;
    if ((s = m.upload(&h->tu.d_wptr, h->tu.wptr.data(), h->tu.wptr.size()))) return s;
    if ((s = m.upload(&h->tu.d_waits, h->tu.waits.data(), h->tu.waits.size()))) return s;
    if ((s = m.upload(&h->tl.d_ks, h->tl.ks.data(), h->tl.ks.size()))) return s;
    if ((s = m.upload(&h->tu.d_ks, h->tu.ks.data(), h->tu.ks.size()))) return s;
    if ((s = m.upload(&h->d_perm, H.perm.data(), H.perm.size()))) return s;
    if ((s = pmgdev::alloc_workspace(h.get(), h->ws, mixed, false))) return s;
    PMG_HIP_OK(hipDeviceSynchronize());
    I.t_upload = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    I.device_bytes = (int64_t)(h->ops.bytes + h->ws.mem.bytes);
  }
  *out = h.release();
  return PMG_OK;
}

pmg_status pmg_destroy(pmg_handle h) {
  delete h;
  return PMG_OK;
}

pmg_status pmg_get_info(pmg_handle h, pmg_info* info) {
  if (!h || !info) return fail(PMG_EINVAL, "NULL argument");
  *info = h->info;
  return PMG_OK;
}

static const pmg::Csr* pick_csr(pmg_handle h, int which, int lev) {
  const pmg::HostOps& H = h->H;
  switch (which) {
    case 0: return &H.A;
    case 1: return &H.L;
    case 2: return &H.U;
    case 3: return &H.R;
    case 4: return &H.P;
    case 5: return (lev >= 0 && lev < H.nlev) ? &H.A1[lev] : nullptr;
    case 6: return (lev >= 0 && lev < (int)H.Ph.size()) ? &H.Ph[lev] : nullptr;
  }
  return nullptr;
}

pmg_status pmg_export(pmg_handle h, int32_t which, int32_t level, int64_t* dims, int64_t* rp, int32_t* ci,
                      double* v) {
  if (!h || !dims) return fail(PMG_EINVAL, "NULL argument");
  const pmg::Csr* M = pick_csr(h, which, level);
  if (!M) return fail(PMG_EINVAL, "unknown operator or level");
  dims[0] = M->nrows;
  dims[1] = M->ncols;
  dims[2] = M->nnz();
  if (rp) std::memcpy(rp, M->rp.data(), sizeof(int64_t) * M->rp.size());
  if (ci) std::memcpy(ci, M->ci.data(), sizeof(int32_t) * M->ci.size());
  if (v) std::memcpy(v, M->v.data(), sizeof(double) * M->v.size());
  return PMG_OK;
}

pmg_status pmg_export_vec(pmg_handle h, int32_t which, double* out) {
  if (!h || !out) return fail(PMG_EINVAL, "NULL argument");
  const pmg::HostOps& H = h->H;
  const std::vector<double>* v = nullptr;
  switch (which) {
    case 0: v = &H.f; break;
    case 1: v = &H.mlp; break;
    case 2: v = &H.ml1; break;
    case 3: v = &H.coarse_inv; break;
    default: return fail(PMG_EINVAL, "unknown vector");
  }
  std::memcpy(out, v->data(), sizeof(double) * v->size());
  return PMG_OK;
}

pmg_status pmg_export_perm(pmg_handle h, int32_t* out) {
  if (!h || !out) return fail(PMG_EINVAL, "NULL argument");
  std::memcpy(out, h->H.perm.data(), sizeof(int32_t) * h->H.perm.size());
  return PMG_OK;
}

#define NEED_DEVICE(h)                                                              \
  do {                                                                              \
    if (!(h)) return fail(PMG_EINVAL, "handle is NULL");                            \
    if (!(h)->on_device) return fail(PMG_EDEVICE, "handle was set up host-only");   \
    PMG_HIP_OK(hipSetDevice((h)->device));                                          \
  } while (0)

pmg_status pmg_rhs(pmg_handle h, double* b, void* stream) {
  NEED_DEVICE(h);
  if (!b) return fail(PMG_EINVAL, "b is NULL");
  PMG_HIP_OK(hipMemcpyAsync(b, h->f, sizeof(double) * h->H.n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PMG_OK;
}

pmg_status pmg_residual(pmg_handle h, const double* b, const double* x, double* r, double* rnorm, void* stream) {
  NEED_DEVICE(h);
  if (!b || !x || !r) return fail(PMG_EINVAL, "NULL vector");
  hipStream_t st = (hipStream_t)stream;
  pmgdev::residual64(h, h->ws, b, x, r, rnorm != nullptr, st);
  PMG_HIP_OK(hipGetLastError());
  if (rnorm) *rnorm = read_norm(h->ws, st);
  return PMG_OK;
}

pmg_status pmg_smooth(pmg_handle h, const double* r, double* x, void* stream) {
  NEED_DEVICE(h);
  if (!r || !x) return fail(PMG_EINVAL, "NULL vector");
  smooth_impl<double>(h, h->ws, r, x, h->ws.y, false, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_lower_solve(pmg_handle h, const double* r, double* y, void* stream) {
  NEED_DEVICE(h);
  if (!r || !y) return fail(PMG_EINVAL, "NULL vector");
  lower_impl<double>(h, h->ws, r, y, false, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_upper_solve(pmg_handle h, double* y, double* x, void* stream) {
  NEED_DEVICE(h);
  if (!y || !x) return fail(PMG_EINVAL, "NULL vector");
  upper_impl<double>(h, h->ws, y, x, false, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_profile_enable(pmg_handle h, int32_t on) {
  NEED_DEVICE(h);
  PMG_HIP_OK(hipDeviceSynchronize());
  for (auto& u : h->ev_used) u = 0;
  h->profiling = on != 0;
  return PMG_OK;
}

pmg_status pmg_profile_read(pmg_handle h, double* ms, int64_t* count) {
  NEED_DEVICE(h);
  if (!ms || !count) return fail(PMG_EINVAL, "NULL argument");
  for (int c = 0; c < PMG_PROF_NCLASS; ++c) {
    double tot = 0.0;
    const size_t pairs = h->ev_used[c] / 2;
    for (size_t i = 0; i < pairs; ++i) {
      PMG_HIP_OK(hipEventSynchronize(h->ev[c][2 * i + 1]));
      float t = 0.0f;
      PMG_HIP_OK(hipEventElapsedTime(&t, h->ev[c][2 * i], h->ev[c][2 * i + 1]));
      tot += t;
    }
    ms[c] = tot;
    count[c] = (int64_t)pairs;
  }
  return PMG_OK;
}

pmg_status pmg_restrict(pmg_handle h, const double* r, double* r1, void* stream) {
  NEED_DEVICE(h);
  if (!r || !r1) return fail(PMG_EINVAL, "NULL vector");
  if (h->H.n1 == 0) return PMG_OK;
  restrict64(h, r, r1, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_coarse(pmg_handle h, const double* r1, double* e1, void* stream) {
  NEED_DEVICE(h);
  if (!r1 || !e1) return fail(PMG_EINVAL, "NULL vector");
  if (h->H.n1 == 0) return PMG_OK;
  coarse_impl(h, h->ws, r1, e1, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_prolong(pmg_handle h, const double* e1, double* x, void* stream) {
  NEED_DEVICE(h);
  if (!e1 || !x) return fail(PMG_EINVAL, "NULL vector");
  if (h->H.n1 == 0) return PMG_OK;
  prolong64(h, e1, x, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_vcycle(pmg_handle h, const double* b, double* x, double* r, double* rnorm, void* stream) {
  NEED_DEVICE(h);
  if (!b || !x || !r) return fail(PMG_EINVAL, "NULL vector");
  hipStream_t st = (hipStream_t)stream;
  pmgdev::vcycle64(h, h->ws, b, x, r, rnorm != nullptr, st);
  PMG_HIP_OK(hipGetLastError());
  if (rnorm) *rnorm = read_norm(h->ws, st);
  return PMG_OK;
}

pmg_status pmg_solve(pmg_handle h, const double* b, double* x, double tol, pmg_result* res, double* hist,
                     void* stream) {
  NEED_DEVICE(h);
  if (!b || !x || !(tol >= 0)) return fail(PMG_EINVAL, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = h->ws;
  auto t0 = std::chrono::steady_clock::now();
  pmg_result R{};
  pmgdev::residual64(h, ws, b, x, ws.r, true, st);
  PMG_HIP_OK(hipGetLastError());
  const double r0 = read_norm(ws, st);
  R.r0 = r0;
  R.relres = 1.0;
  if (hist) hist[0] = 1.0;
  pmg_status status = PMG_EMAXIT;
  if (!std::isfinite(r0)) {
    status = PMG_ENAN;
  } else if (r0 == 0.0) {
    status = PMG_OK;
    R.relres = 0.0;
  } else {
    const bool mixed = h->opt.precision == PMG_FP32_IN_FP64;
    for (int it = 1; it <= h->opt.max_iter; ++it) {
      if (!mixed)
        pmgdev::vcycle64(h, ws, b, x, ws.r, true, st);
      else
        pmgdev::mixed_step(h, ws, b, x, st);
      PMG_HIP_OK(hipGetLastError());
      const double rel = read_norm(ws, st) / r0;
      R.iterations = it;
      R.relres = rel;
      if (hist) hist[it] = rel;
      if (!std::isfinite(rel) || rel > h->opt.diverge_ratio) {
        status = PMG_EDIVERGED;
        break;
      }
      if (rel <= tol) {
        status = PMG_OK;
        break;
      }
    }
  }
  R.status = status;
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (res) *res = R;
  if (status != PMG_OK) pmgdev::set_error(pmg_status_str(status));
  return status;
}

}  // extern "C"
