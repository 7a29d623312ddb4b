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
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "kernels.hpp"
#include "pmg_internal.hpp"

using pmgdev::DevMat;
using pmgdev::TriSched;
using pmgdev::DevStencil;
using pmgdev::DevXStencil;
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

// Scratch of pmg_smooth_static, for callers that cannot allocate device
// memory: the ticket counters of both triangular solves in the first
// kStaticHead bytes, then the forward solve's output y and the backward
// solve's output e for up to kStaticMaxN unknowns each (32 MiB in all).  One
// copy per device, held until the process ends; every call on a device shares
// it, so calls that overlap on one device race.  Host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kStaticMaxN = int64_t(1) << 21;
constexpr int64_t kStaticHead = 4096;
static_assert(kStaticHead >= (int64_t)(2 * pmg::kTicketWords * sizeof(unsigned)), "counters fit the head");
static __device__ __align__(256) unsigned char scratch[kStaticHead + 2 * sizeof(double) * kStaticMaxN];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
}  // namespace

// Device address of `scratch` on device dev, which must be current; looked up
// once per device.
static pmg_status static_scratch(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= 64) return pmgdev::fail(PMG_EDEVICE, "device ordinal out of range for the static scratch");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return pmgdev::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return pmgdev::fail(PMG_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return PMG_OK;
}

pmg_handle_s::~pmg_handle_s() {
  delete sub;
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
// default upper bound of a triangular-solve segment's rows (pmg_options.segment_rows)
constexpr int kSegmentRows = 512;

int pick_group(double avg) {
  if (avg >= 128) return 64;
  if (avg >= 48) return 32;
  if (avg >= 20) return 16;
  if (avg >= 8) return 8;
  return 4;
}

unsigned nblocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

unsigned csr_grid(int nrows, int G) { return std::min<unsigned>(nblocks(nrows, 256 / G), kMaxCsrBlocks); }

// Chunk boundaries of the segment-ordered triangular solves.  A segment (a
// run of whole grid lines inside one block of the nested dissection, rows
// seg[s] .. seg[s+1]-1) is cut into chunks of 64 rows, counted in processing
// coordinates (forward solve: position in the segment; backward solve:
// position from its end), with the first chunk shortened by an offset o in
// [0, 64).  The offset of each segment is chosen, in processing order, among
// even values so that the segment's chunks reach the lowest levels of the
// chunk dependency graph given the chunks of the segments before it: a chunk
// of one grid line reads a few rows past its own end in the previous lines,
// and with aligned boundaries it would wait for two chunks of each of them
// instead of one.  Returns per segment the processing-coordinate chunk starts
// (plus the segment's length).
std::vector<std::vector<int>> choose_chunks(const pmg::Csr& T, const std::vector<int32_t>& seg,
                                            const std::vector<int32_t>& seg_of, bool upper) {
  const int nseg = (int)seg.size() - 1;
  auto len = [&](int t) { return seg[t + 1] - seg[t]; };
  // per segment: for each segment it reads, the furthest processing position
  // read by the row at each processing position (-1: none)
  struct Dep {
    int t;
    std::vector<int> reach;
  };
  std::vector<std::vector<Dep>> deps(nseg);
  std::vector<int> slot(nseg, -1);
  for (int s = 0; s < nseg; ++s) {
    std::vector<int> touched;
    const int ls = len(s);
    for (int x = 0; x < ls; ++x) {
      const int row = seg[s] + x;
      const int xp = upper ? ls - 1 - x : x;
      for (int64_t k = T.rp[row] + (upper ? 1 : 0); k < T.rp[row + 1]; ++k) {
        const int t = seg_of[T.ci[k]], y = T.ci[k] - seg[t];
        if (t == s) continue;
        if (slot[t] < 0) {
          slot[t] = (int)deps[s].size();
          deps[s].push_back(Dep{t, std::vector<int>(ls, -1)});
          touched.push_back(t);
        }
        int& r = deps[s][slot[t]].reach[xp];
        r = std::max(r, upper ? len(t) - 1 - y : y);
      }
    }
    for (int t : touched) slot[t] = -1;
  }
  std::vector<std::vector<int>> bounds(nseg), levels(nseg);
  auto cut = [&](int o, int ls) {
    std::vector<int> b{0};
    for (int a = 64 - o; a < ls; a += 64)
      if (a > 0) b.push_back(a);
    b.push_back(ls);
    return b;
  };
  std::vector<int> lv;
  for (int qq = 0; qq < nseg; ++qq) {
    const int s = upper ? nseg - 1 - qq : qq;
    int best_last = INT32_MAX;
    int64_t best_sum = 0;
    for (int o = 0; o < 64; o += 2) {
      const std::vector<int> b = cut(o, len(s));
      lv.assign(b.size() - 1, 0);
      int prev = 0;
      int64_t sum = 0;
      for (size_t k = 0; k + 1 < b.size(); ++k) {
        int l = prev;
        for (const Dep& d : deps[s]) {
          int need = -1;
          for (int x = b[k]; x < b[k + 1]; ++x) need = std::max(need, d.reach[x]);
          if (need < 0) continue;
          const std::vector<int>& tb = bounds[d.t];
          const size_t kk = std::upper_bound(tb.begin(), tb.end(), need) - tb.begin() - 1;
          l = std::max(l, levels[d.t][kk]);
        }
        lv[k] = prev = l + 1;
        sum += l + 1;
      }
      if (lv.back() < best_last || (lv.back() == best_last && sum < best_sum)) {
        best_last = lv.back();
        best_sum = sum;
        bounds[s] = b;
        levels[s] = lv;
      }
    }
  }
  return bounds;
}

// Schedule and chunk-sliced layout of one segment-ordered triangular solve
// (the layout is described with pmg::TriDev).  Forward: row i reads rows
// j < i; backward (upper == true): row i reads rows j > i and chunks are
// finished from the end of their segment.
pmg_status build_schedule(const pmg::Csr& T, const std::vector<int32_t>& seg, int seg_len, bool upper,
                          TriSched& S) {
  const int n = T.nrows;
  S.seg_len = seg_len;
  if ((int64_t)n * 8 >= INT32_MAX) return fail(PMG_EINVAL, "triangular factor has more than 2^28 rows");
  if (seg.size() < 2 || seg.front() != 0 || seg.back() != n) return fail(PMG_EINVAL, "bad schedule segments");
  S.nrows = n;
  S.nseg = (int)seg.size() - 1;
  S.seg_start = seg;
  std::vector<int32_t> seg_of(n);
  for (int s = 0; s < S.nseg; ++s) {
    if (seg[s + 1] <= seg[s]) return fail(PMG_EINVAL, "bad schedule segments");
    for (int r = seg[s]; r < seg[s + 1]; ++r) seg_of[r] = s;
  }
  // chunk geometry in natural order (segment-major, ascending rows)
  const std::vector<std::vector<int>> bounds = choose_chunks(T, seg, seg_of, upper);
  S.chunk_row.clear();
  S.chunk_len.clear();
  for (int s = 0; s < S.nseg; ++s) {
    const std::vector<int>& b = bounds[s];
    const int ls = seg[s + 1] - seg[s];
    const int K = (int)b.size() - 1;
    for (int k = 0; k < K; ++k) {
      const int kp = upper ? K - 1 - k : k;  // processing index of the k-th chunk by rows
      const int a = upper ? ls - b[kp + 1] : b[kp];
      const int e = upper ? ls - b[kp] : b[kp + 1];
      S.chunk_row.push_back(seg[s] + a);
      S.chunk_len.push_back(e - a);
    }
  }
  const int nq = (int)S.chunk_row.size();
  S.nch = nq;
  std::vector<int> row_chunk(n);
  for (int q = 0; q < nq; ++q)
    for (int r = S.chunk_row[q]; r < S.chunk_row[q] + S.chunk_len[q]; ++r) row_chunk[r] = q;
  S.wptr.assign((size_t)nq + 1, 0);
  S.off_ptr.assign(nq, 0);
  S.off_w.assign(nq, 0);
  S.in_ptr.assign(nq, 0);
  S.in_w.assign(nq, 0);
  S.diag.assign(upper ? n : 0, 0.0);
  if (upper)
    for (int row = 0; row < n; ++row) S.diag[row] = T.v[T.rp[row]];
  // slot counts first, so the sliced arrays are written in place below
  for (int q = 0; q < nq; ++q) {
    const int r0 = S.chunk_row[q], r1 = r0 + S.chunk_len[q];
    int wo = 0, wi = 0;
    for (int row = r0; row < r1; ++row) {
      int ni = 0, no = 0;
      for (int64_t k = T.rp[row] + (upper ? 1 : 0); k < T.rp[row + 1]; ++k)
        (T.ci[k] >= r0 && T.ci[k] < r1) ? ++ni : ++no;
      wo = std::max(wo, no);
      wi = std::max(wi, ni);
    }
    // whole column groups (see pmg::TriDev)
    S.off_w[q] = (wo + pmg::kColGroup - 1) / pmg::kColGroup * pmg::kColGroup;
    S.in_w[q] = (wi + pmg::kColGroup - 1) / pmg::kColGroup * pmg::kColGroup;
  }
  int64_t no_tot = 0, ni_tot = 0;
  for (int q = 0; q < nq; ++q) {
    S.off_ptr[q] = (int)no_tot;
    S.in_ptr[q] = (int)ni_tot;
    no_tot += (int64_t)S.off_w[q] * 64;
    ni_tot += (int64_t)S.in_w[q] * 64;
  }
  if (no_tot + pmg::kTriPad >= INT32_MAX || ni_tot + pmg::kTriPad >= INT32_MAX)
    return fail(PMG_EINVAL, "triangular factor has more than 2^31 stored slots");
  // trailing padding entries (see pmg::TriDev)
  S.off_pad = (int)no_tot;
  S.in_pad = (int)ni_tot;
  S.off_col.assign(no_tot + pmg::kTriPad, -1);
  S.off_val.assign(no_tot + pmg::kTriPad, 0.0);
  S.in_j.assign(ni_tot + pmg::kTriPad, -1);
  S.in_val.assign(ni_tot + pmg::kTriPad, 0.0);
  // per chunk, in a topological order (forward: ascending q, backward:
  // descending q): the chunks it reads, its level and the sliced entries
  std::vector<int> level(nq, 0), mark(nq, 0), touched;
  std::vector<std::vector<int>> deps_q(nq);
  std::vector<std::vector<int>> oc(64), ic(64);
  for (int qq = 0; qq < nq; ++qq) {
    const int q = upper ? nq - 1 - qq : qq;
    const int r0 = S.chunk_row[q], r1 = r0 + S.chunk_len[q];
    const int s = seg_of[r0];
    touched.clear();
    auto add_dep = [&](int qd) {
      if (!mark[qd]) {
        mark[qd] = 1;
        touched.push_back(qd);
      }
    };
    // the previous chunk of the own segment, always
    if (!upper && r0 > seg[s]) add_dep(q - 1);
    if (upper && r1 < seg[s + 1]) add_dep(q + 1);
    for (int row = r0; row < r1; ++row) {
      const int l = row - r0;
      oc[l].clear();
      ic[l].clear();
      for (int64_t k = T.rp[row] + (upper ? 1 : 0); k < T.rp[row + 1]; ++k) {
        const int col = T.ci[k];
        if (col >= r0 && col < r1) {
          ic[l].push_back((int)k);
        } else {
          oc[l].push_back((int)k);
          add_dep(row_chunk[col]);
        }
      }
    }
    int lv = 0;
    for (int qd : touched) lv = std::max(lv, level[qd]);
    level[q] = lv + 1;
    // dependencies sorted by level (ties: processing order)
    auto earlier = [&](int a, int b) {
      if (level[a] != level[b]) return level[a] < level[b];
      return upper ? a > b : a < b;
    };
    std::sort(touched.begin(), touched.end(), earlier);
    for (int qd : touched) mark[qd] = 0;
    deps_q[q] = touched;
    // slots of each row by the level of their chunk, then by column
    for (int l = 0; l < r1 - r0; ++l)
      std::sort(oc[l].begin(), oc[l].end(), [&](int ka, int kb) {
        const int qa = row_chunk[T.ci[ka]], qb = row_chunk[T.ci[kb]];
        if (qa != qb) return earlier(qa, qb);
        return upper ? T.ci[ka] > T.ci[kb] : T.ci[ka] < T.ci[kb];
      });
    for (int l = 0; l < r1 - r0; ++l) {
      // right-aligned: padding first, the row's entries in the last slots
      const size_t pad = (size_t)S.off_w[q] - oc[l].size();
      for (size_t u = 0; u < oc[l].size(); ++u) {
        const size_t o = S.off_ptr[q] + (pad + u) * 64 + l;
        S.off_col[o] = T.ci[oc[l][u]];
        S.off_val[o] = T.v[oc[l][u]];
      }
      for (size_t u = 0; u < ic[l].size(); ++u) {
        const size_t o = S.in_ptr[q] + u * 64 + l;
        const int col = T.ci[ic[l][u]];
        S.in_j[o] = col - r0;
        S.in_val[o] = upper ? T.v[ic[l][u]] / S.diag[col] : T.v[ic[l][u]];
      }
    }
  }
  // dependency lists by natural chunk index (they define the order; the
  // kernels find readiness in the data)
  S.deps.clear();
  for (int q = 0; q < nq; ++q) {
    S.deps.insert(S.deps.end(), deps_q[q].begin(), deps_q[q].end());
    S.wptr[q + 1] = (int)S.deps.size();
  }
  // ticket order: by level, ties in processing order
  S.order.resize(nq);
  for (int i = 0; i < nq; ++i) S.order[i] = upper ? nq - 1 - i : i;
  std::stable_sort(S.order.begin(), S.order.end(), [&](int a, int b) { return level[a] < level[b]; });
  S.chunk_levels = nq ? *std::max_element(level.begin(), level.end()) : 0;
  S.slots = (int64_t)S.off_pad;
  // depth of the row dependency DAG (for the record)
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
  return PMG_OK;
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

// The shape of an operator whose values live in a stencil layout instead:
// nothing is uploaded, the kernels read only the sizes.
void describe_mat(const pmg::Csr& M, DevMat& D) {
  D.nrows = M.nrows;
  D.ncols = M.ncols;
  D.nnz = M.nnz();
  D.G = pick_group(D.nrows ? (double)D.nnz / D.nrows : 1.0);
}

// Offsets of A's stencil layout (see pmg::stencil_resid), or 0 when it is
// not used: every entry must lie within the degree-p offsets of its row, and
// the layout must read fewer bytes than CSR (8 bytes per offset slot against
// 12 per non-zero; the zero slots at the boundary make it lose on small grids).
int stencil_slots(const pmg::HostOps& H) {
  const int d = H.dim, p = H.p, nx = H.nel + p - 2;
  const int w = 2 * p + 1;
  const int S = d == 2 ? w * w : w * w * w;
  const int64_t n = H.n;
  if ((int64_t)8 * S * n >= (int64_t)12 * H.A.nnz()) return 0;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t ix = i % nx, iy = (i / nx) % nx, iz = i / ((int64_t)nx * nx);
    for (int64_t k = H.A.rp[i]; k < H.A.rp[i + 1]; ++k) {
      const int64_t j = H.A.ci[k];
      const int64_t dx = j % nx - ix, dy = (j / nx) % nx - iy, dz = j / ((int64_t)nx * nx) - iz;
      if (std::abs(dx) > p || std::abs(dy) > p || std::abs(dz) > p) return 0;
    }
  }
  return S;
}

pmg_status upload_stencil(pmgdev::DevArena& mem, const pmg::HostOps& H, int S, bool kron, DevStencil& D,
                          bool with32) {
  if (S == 0) return PMG_OK;
  const int d = H.dim, p = H.p, nx = H.nel + p - 2, w = 2 * p + 1;
  const int64_t n = H.n;
  D.dim = d;
  D.p = p;
  D.nx = D.ny = nx;
  D.S = S;
  if (kron) {
    // the coefficients are formed from the 1-D factors in the kernel
    pmg_status s;
    if ((s = mem.upload(&D.kK, H.kK.data(), H.kK.size()))) return s;
    if ((s = mem.upload(&D.kM, H.kM.data(), H.kM.size()))) return s;
    return PMG_OK;
  }
  std::vector<double> V((size_t)S * n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t ix = i % nx, iy = (i / nx) % nx, iz = i / ((int64_t)nx * nx);
    for (int64_t k = H.A.rp[i]; k < H.A.rp[i + 1]; ++k) {
      const int64_t j = H.A.ci[k];
      const int64_t dx = j % nx - ix, dy = (j / nx) % nx - iy, dz = j / ((int64_t)nx * nx) - iz;
      const int64_t off = ((d == 3 ? (dz + p) * w : 0) + (dy + p)) * w + (dx + p);
      V[(size_t)off * n + i] = H.A.v[k];
    }
  }
  pmg_status s;
  if ((s = mem.upload(&D.v, V.data(), V.size()))) return s;
  if (with32) {
    std::vector<float> V32(V.begin(), V.end());
    if ((s = mem.upload(&D.v32, V32.data(), V32.size()))) return s;
  }
  return PMG_OK;
}

// Whether the degree-1 levels take the structured kernels: the levels halve
// (nx_l = 2 nx_{l+1} + 1) and every smoothed level's operator couples nodes
// only within {-1, 0, 1}^d.
bool grid_levels_structured(const pmg::HostOps& H, int dim) {
  if (H.nlev < 2) return false;
  for (int l = 0; l + 1 < H.nlev; ++l)
    if (H.lnel[l] != 2 * H.lnel[l + 1]) return false;
  for (int l = 0; l + 1 < H.nlev; ++l) {
    const pmg::Csr& A = H.A1[l];
    const int64_t nx = H.lnel[l] - 1;
    for (int64_t i = 0; i < A.nrows; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int64_t j = A.ci[k];
        for (int a = 0; a < dim; ++a) {
          const int64_t s = a == 0 ? 1 : a == 1 ? nx : nx * nx;
          if (std::abs((j / s) % nx - (i / s) % nx) > 1) return false;
        }
      }
  }
  return true;
}

// Degree-1 levels in colour-major stencil layout (see the structured
// h-multigrid kernels).  Leaves G empty, so the CSR path is taken, unless
// every level's operator couples nodes only within {-1, 0, 1}^d and the
// levels halve (nx_l = 2 nx_{l+1} + 1).
pmg_status upload_grid_levels(pmgdev::DevArena& mem, const pmg::HostOps& H, int dim, bool kron,
                              std::vector<pmg::GridLevel>& G) {
  G.clear();
  if (H.nlev < 1) return PMG_OK;  // no degree-1 hierarchy (indirect projection)
  const int nl = H.nlev - 1;  // levels with smoothing (the last is solved directly)
  for (int l = 0; l + 1 < H.nlev; ++l)
    if (H.lnel[l] != 2 * H.lnel[l + 1]) return PMG_OK;
  const int K = dim == 2 ? 9 : 27;
  std::vector<pmg::GridLevel> out(nl);
  std::vector<std::vector<double>> vals(nl);
  for (int l = 0; l < nl; ++l) {
    const pmg::Csr& A = H.A1[l];
    const int nx = H.lnel[l] - 1;
    pmg::GridLevel& L = out[l];
    L.nx = nx;
    L.n = (int)H.ln[l];
    for (int c = 0; c < 8; ++c) {
      const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
      if (dim == 2 && cz) {
        L.cnt[c] = 0;
        continue;
      }
      int64_t m = (int64_t)((nx - cx + 1) / 2) * ((nx - cy + 1) / 2);
      if (dim == 3) m *= (nx - cz + 1) / 2;
      L.cnt[c] = (int)m;
    }
    int64_t off = 0;
    for (int c = 0; c < 8; ++c) {
      L.voff[c] = (int)off;
      off += (int64_t)K * L.cnt[c];
    }
    vals[l].assign(off, 0.0);
    for (int64_t i = 0; i < L.n; ++i) {
      const int ix = (int)(i % nx), iy = (int)((i / nx) % nx), iz = (int)(i / ((int64_t)nx * nx));
      const int c = (ix & 1) | ((iy & 1) << 1) | (dim == 3 ? (iz & 1) << 2 : 0);
      const int mx = (nx - (c & 1) + 1) / 2, my = (nx - ((c >> 1) & 1) + 1) / 2;
      const int64_t t = ix / 2 + (int64_t)mx * (iy / 2 + (int64_t)my * (dim == 3 ? iz / 2 : 0));
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int64_t j = A.ci[k];
        const int dx = (int)(j % nx) - ix, dy = (int)((j / nx) % nx) - iy, dz = (int)(j / ((int64_t)nx * nx)) - iz;
        if (std::abs(dx) > 1 || std::abs(dy) > 1 || std::abs(dz) > 1) return PMG_OK;  // not a stencil
        const int kk = ((dim == 3 ? (dz + 1) * 3 : 0) + (dy + 1)) * 3 + (dx + 1);
        vals[l][L.voff[c] + (int64_t)kk * L.cnt[c] + t] = A.v[k];
      }
    }
  }
  for (int l = 0; l < nl; ++l) {
    double* d;
    pmg_status s = mem.upload(&d, vals[l].data(), vals[l].size());
    if (s) return s;
    out[l].v = d;
    // 2-D Kronecker levels: the tiled kernels form the values from the bands
    if (kron && dim == 2 && l < (int)H.k1K.size() && H.k1K[l].size() == (size_t)3 * out[l].nx) {
      double *k, *m;
      if ((s = mem.upload(&k, H.k1K[l].data(), H.k1K[l].size()))) return s;
      if ((s = mem.upload(&m, H.k1M[l].data(), H.k1M[l].size()))) return s;
      out[l].kK = k;
      out[l].kM = m;
    }
  }
  G = out;
  return PMG_OK;
}

// Shape of a transfer M between grids (rows on an nxr^d grid, columns on an
// nxc^d grid) in stencil layout: every row couples only to a W^d block of
// column nodes at offset lo from its own position.  Returns the number of
// slots W^d if that layout reads fewer bytes than CSR, else 0.
int64_t xstencil_shape(const pmg::Csr& M, int dim, int nxr, int nxc, int& lo, int& W) {
  auto pos = [&](int64_t i, int nx, int a) {
    return (int)(a == 0 ? i % nx : a == 1 ? (i / nx) % nx : i / ((int64_t)nx * nx));
  };
  lo = INT32_MAX;
  int hi = INT32_MIN;
  for (int64_t i = 0; i < M.nrows; ++i)
    for (int64_t k = M.rp[i]; k < M.rp[i + 1]; ++k)
      for (int a = 0; a < dim; ++a) {
        const int dlt = pos(M.ci[k], nxc, a) - pos(i, nxr, a);
        lo = std::min(lo, dlt);
        hi = std::max(hi, dlt);
      }
  if (M.nnz() == 0) return 0;
  W = hi - lo + 1;
  const int64_t S = dim == 2 ? (int64_t)W * W : (int64_t)W * W * W;
  return 8 * S * M.nrows < 12 * M.nnz() ? S : 0;
}

pmg_status upload_xstencil(pmgdev::DevArena& mem, const pmg::Csr& M, int dim, int nxr, int nxc, DevXStencil& D,
                           bool with32) {
  auto pos = [&](int64_t i, int nx, int a) {
    return (int)(a == 0 ? i % nx : a == 1 ? (i / nx) % nx : i / ((int64_t)nx * nx));
  };
  int lo = 0, W = 0;
  const int64_t S = xstencil_shape(M, dim, nxr, nxc, lo, W);
  if (S == 0) return PMG_OK;
  std::vector<double> V((size_t)S * M.nrows, 0.0);
  for (int64_t i = 0; i < M.nrows; ++i)
    for (int64_t k = M.rp[i]; k < M.rp[i + 1]; ++k) {
      int64_t slot = 0;
      for (int a = dim - 1; a >= 0; --a) slot = slot * W + (pos(M.ci[k], nxc, a) - pos(i, nxr, a) - lo);
      V[(size_t)slot * M.nrows + i] = M.v[k];
    }
  pmg_status s;
  if ((s = mem.upload(&D.v, V.data(), V.size()))) return s;
  if (with32) {
    std::vector<float> V32(V.begin(), V.end());
    if ((s = mem.upload(&D.v32, V32.data(), V32.size()))) return s;
  }
  D.nxr = nxr;
  D.nxc = nxc;
  D.o = lo;
  D.W = W;
  return PMG_OK;
}

// A transfer on the unit box as the 1-D factor of its Kronecker product
// (pmg::kron_xgrid): row ix of the nxr^d grid, slot kx -> column ix + lo + kx
// of the nxc^d grid; P's factor is X (rows: degree-p functions), R's is X^T.
pmg_status upload_xkron(pmgdev::DevArena& mem, const pmg::HostOps& H, const pmg::Csr& M, bool transposed, int dim,
                        int nxr, int nxc, DevXStencil& D) {
  int lo = 0, W = 0;
  xstencil_shape(M, dim, nxr, nxc, lo, W);
  if (M.nnz() == 0 || W <= 0) return PMG_OK;
  auto X = [&](int i, int j) {  // full indices
    const int k = j - i + H.xlo;
    return i < 0 || i >= H.xnr || k < 0 || k >= H.xw ? 0.0 : H.kX[(size_t)i * H.xw + k];
  };
  std::vector<double> tab((size_t)nxr * W, 0.0);
  for (int ix = 0; ix < nxr; ++ix)
    for (int kx = 0; kx < W; ++kx) {
      const int jx = ix + lo + kx;
      if (jx < 0 || jx >= nxc) continue;
      tab[(size_t)ix * W + kx] = transposed ? X(jx + 1, ix + 1) : X(ix + 1, jx + 1);
    }
  pmg_status s;
  if ((s = mem.upload(&D.tab, tab.data(), tab.size()))) return s;
  D.nxr = nxr;
  D.nxc = nxc;
  D.o = lo;
  D.W = W;
  return PMG_OK;
}

// Host slot-major order (slot u of lane l at ptr + 64 u + l) to the device's
// 16-byte groups of G slots per lane (ptr + 64 u + G l + u % G).  Chunks start
// at multiples of 64 * kColGroup entries, so the groups never straddle two
// chunks; the padding tail (pad_at..) keeps its value.
template <typename TO, typename TI>
std::vector<TO> group_slots(const std::vector<TI>& src, int64_t pad_at, int G) {
  std::vector<TO> dst(src.size());
  for (int64_t i = 0; i < pad_at; ++i) {
    const int64_t u = i / 64, l = i % 64;
    dst[(u / G) * 64 * G + l * G + u % G] = (TO)src[i];
  }
  for (size_t i = (size_t)pad_at; i < src.size(); ++i) dst[i] = (TO)src[i];
  return dst;
}

// Off-chunk columns for the device: padding (-1) becomes n, the first index
// past the buffer the gathers read through.
std::vector<int> device_cols(const std::vector<int>& src, int64_t pad_at, int n) {
  std::vector<int> dst = group_slots<int>(src, pad_at, pmg::kColGroup);
  for (int& c : dst)
    if (c < 0) c = n;
  return dst;
}

pmg_status upload_tri(pmgdev::DevArena& mem, TriSched& S, bool upper, bool with32) {
  pmg_status s;
  const int nq = (int)S.order.size();
  std::vector<pmg::TriMeta> meta(nq);
  for (int tk = 0; tk < nq; ++tk) {
    const int q = S.order[tk];
    meta[tk] = pmg::TriMeta{S.chunk_row[q], S.chunk_len[q], S.off_ptr[q], S.off_w[q], S.in_ptr[q], S.in_w[q], {0, 0}};
  }
  pmg::TriMeta* md;
  int *oc, *ij;
  double *ov, *iv, *dg = nullptr;
  if ((s = mem.upload(&md, meta.data(), meta.size()))) return s;
  {
    const std::vector<int> gc = device_cols(S.off_col, S.off_pad, S.nrows);
    const std::vector<double> gv = group_slots<double>(S.off_val, S.off_pad, 2);
    const std::vector<int> gj = group_slots<int>(S.in_j, S.in_pad, pmg::kColGroup);
    const std::vector<double> gw = group_slots<double>(S.in_val, S.in_pad, 2);
    if ((s = mem.upload(&oc, gc.data(), gc.size()))) return s;
    if ((s = mem.upload(&ov, gv.data(), gv.size()))) return s;
    if ((s = mem.upload(&ij, gj.data(), gj.size()))) return s;
    if ((s = mem.upload(&iv, gw.data(), gw.size()))) return s;
  }
  if (upper && (s = mem.upload(&dg, S.diag.data(), S.diag.size()))) return s;
  S.dev64 = pmg::TriDev<double>{S.off_pad, S.in_pad, S.nrows, md, oc, ov, ij, iv, dg};
  if (with32) {
    const std::vector<float> a = group_slots<float>(S.off_val, S.off_pad, 4),
                             b = group_slots<float>(S.in_val, S.in_pad, 4);
    const std::vector<float> c(S.diag.begin(), S.diag.end());
    float *ov32, *iv32, *dg32 = nullptr;
    if ((s = mem.upload(&ov32, a.data(), a.size()))) return s;
    if ((s = mem.upload(&iv32, b.data(), b.size()))) return s;
    if (upper && (s = mem.upload(&dg32, c.data(), c.size()))) return s;
    S.dev32 = pmg::TriDev<float>{S.off_pad, S.in_pad, S.nrows, md, oc, ov32, ij, iv32, dg32};
  }
  return PMG_OK;
}

template <typename T>
const pmg::TriDev<T>& tri_dev(const TriSched& S);
template <>
const pmg::TriDev<double>& tri_dev<double>(const TriSched& S) { return S.dev64; }
template <>
const pmg::TriDev<float>& tri_dev<float>(const TriSched& S) { return S.dev32; }

template <typename T>
int tri_grid(const TriSched& S) {
  return sizeof(T) == 8 ? S.grid64 : S.grid32;
}

// Counters and fault word of a triangular solve of ws (factor 0 lower, 1 upper).
pmg::TriCtl tri_ctl(pmg_handle h, Workspace& ws, int factor) {
  return pmg::TriCtl{ws.tickets + factor * pmg::kTicketWords, ws.tickets + 2 * pmg::kTicketWords,
                     h->opt.poll_limit > 0 ? h->opt.poll_limit : pmg::kPollLimit};
}

// Persistent grid of the triangular solves: as many waves as fit on the
// device at once (more would only start after others exit), at most one per
// chunk.
template <typename T>
pmg_status size_tri_grid(int device, int waves_per_cu, TriSched& L, TriSched& U) {
  hipDeviceProp_t prop;
  PMG_HIP_OK(hipGetDeviceProperties(&prop, device));
  int per_cu_l = 0, per_cu_u = 0;
  PMG_HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_l, pmg::trisolve_lower<T>, 64, 0));
  PMG_HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_u, pmg::trisolve_upper<T>, 64, 0));
  if (waves_per_cu > 0) {
    per_cu_l = std::min(per_cu_l, waves_per_cu);
    per_cu_u = std::min(per_cu_u, waves_per_cu);
  }
  const int64_t cl = (int64_t)std::max(per_cu_l, 1) * prop.multiProcessorCount;
  const int64_t cu = (int64_t)std::max(per_cu_u, 1) * prop.multiProcessorCount;
  const int gl = (int)std::max<int64_t>(1, std::min<int64_t>(cl, (int64_t)L.nch));
  const int gu = (int)std::max<int64_t>(1, std::min<int64_t>(cu, (int64_t)U.nch));
  (sizeof(T) == 8 ? L.grid64 : L.grid32) = gl;
  (sizeof(T) == 8 ? U.grid64 : U.grid32) = gu;
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

// out = d .* (M x) (add: out += d .* (M x)) for a p-transfer, stencil or CSR.
template <typename T>
void transfer(const DevMat& M, const DevXStencil& X, int dim, const T* x, const T* d, T* out, bool add,
              hipStream_t st) {
  if (X.tab) {
    const unsigned grid = std::min<unsigned>(nblocks(M.nrows, 256), kMaxCsrBlocks);
#define PMG_KRON_X(D, ADD, KW) \
  pmg::kron_xgrid<T, D, ADD, KW><<<grid, 256, 0, st>>>(M.nrows, X.nxr, X.nxc, X.o, X.W, X.tab, x, d, out)
#define PMG_KRON_XW(D, ADD) \
  if (X.W <= 8)             \
    PMG_KRON_X(D, ADD, 8);  \
  else                      \
    PMG_KRON_X(D, ADD, 0)
    if (dim == 2) {
      if (add) PMG_KRON_XW(2, true); else PMG_KRON_XW(2, false);
    } else {
      if (add) PMG_KRON_XW(3, true); else PMG_KRON_XW(3, false);
    }
#undef PMG_KRON_XW
#undef PMG_KRON_X
    return;
  }
  if (X.v) {
    const T* V;
    if constexpr (sizeof(T) == 8) V = X.v; else V = X.v32;
    const unsigned grid = std::min<unsigned>(nblocks(M.nrows, 256), kMaxCsrBlocks);
    if (dim == 2) {
      if (add)
        pmg::xgrid_spmv<T, 2, true><<<grid, 256, 0, st>>>(M.nrows, X.nxr, X.nxc, X.o, X.W, V, x, d, out);
      else
        pmg::xgrid_spmv<T, 2, false><<<grid, 256, 0, st>>>(M.nrows, X.nxr, X.nxc, X.o, X.W, V, x, d, out);
    } else {
      if (add)
        pmg::xgrid_spmv<T, 3, true><<<grid, 256, 0, st>>>(M.nrows, X.nxr, X.nxc, X.o, X.W, V, x, d, out);
      else
        pmg::xgrid_spmv<T, 3, false><<<grid, 256, 0, st>>>(M.nrows, X.nxr, X.nxc, X.o, X.W, V, x, d, out);
    }
    return;
  }
  const T* v;
  if constexpr (sizeof(T) == 8) v = M.v; else v = M.v32;
  csr_launch<T>(add ? pmg::kScaleAdd : pmg::kScale, M.nrows, nullptr, M, v, x, nullptr, d, out, nullptr, st);
}

// Rows per thread of a residual launch: kResidRows while that still leaves
// about three waves per SIMD on the 256 CUs, else one row, for the latency
// of the loads.  The stencil and Kronecker kernels take the same rows per
// thread and workgroup, so their block partials are the same sums.
constexpr int kResidMinThreads = 3 * 4 * 256 * 64;
int resid_rows(int n, int nx, int ny) {
  return pmg::resid_threads(n, nx, ny, pmg::kResidRows) >= kResidMinThreads ? pmg::kResidRows : 1;
}
int resid_rows(const DevStencil& S, int n) { return resid_rows(n, S.nx, S.ny); }

// Workgroups of a residual launch (grid-stride beyond kMaxCsrBlocks
// workgroups), which is also its number of partials.
unsigned resid_grid(const DevStencil& S, int n) {
  return std::min<unsigned>(nblocks(pmg::resid_threads(n, S.nx, S.ny, resid_rows(S, n)), 256), kMaxCsrBlocks);
}

// stencil_resid with the offset loop unrolled for stencil widths up to 11
// (degrees 1..5), the runtime loop otherwise; RB rows per thread.
template <typename T, int DIM, bool PLAIN, int RB>
void launch_stencil_rb(const DevStencil& S, int n, unsigned grid, const T* V, const T* x, const T* b, T* r,
                       double* partial, hipStream_t st) {
  switch (2 * S.p + 1) {
#define PMG_STENCIL_W(W)                                                                                    \
  case W:                                                                                                   \
    pmg::stencil_resid<T, DIM, PLAIN, W, RB><<<grid, 256, 0, st>>>(n, S.nx, S.ny, S.p, V, x, b, r, partial); \
    return;
    PMG_STENCIL_W(3)
    PMG_STENCIL_W(5)
    PMG_STENCIL_W(7)
    PMG_STENCIL_W(9)
    PMG_STENCIL_W(11)
#undef PMG_STENCIL_W
    default:
      pmg::stencil_resid<T, DIM, PLAIN, 0, RB><<<grid, 256, 0, st>>>(n, S.nx, S.ny, S.p, V, x, b, r, partial);
  }
}
template <typename T, int DIM, bool PLAIN>
void launch_stencil(const DevStencil& S, int n, unsigned grid, const T* V, const T* x, const T* b, T* r,
                    double* partial, hipStream_t st) {
  if (resid_rows(S, n) == pmg::kResidRows)
    launch_stencil_rb<T, DIM, PLAIN, pmg::kResidRows>(S, n, grid, V, x, b, r, partial, st);
  else
    launch_stencil_rb<T, DIM, PLAIN, 1>(S, n, grid, V, x, b, r, partial, st);
}

// kron_resid with the offset loop unrolled (widths 3..11); RB rows per thread.
template <typename T, int DIM, bool PLAIN, int RB>
void launch_kron_rb(const DevStencil& S, int n, unsigned grid, const T* x, const T* b, T* r, double* partial,
                    hipStream_t st) {
  switch (2 * S.p + 1) {
#define PMG_KRON_W(W)                                                                                       \
  case W:                                                                                                   \
    pmg::kron_resid<T, DIM, PLAIN, W, RB><<<grid, 256, 0, st>>>(n, S.nx, S.p, S.kK, S.kM, x, b, r, partial); \
    return;
    PMG_KRON_W(3)
    PMG_KRON_W(5)
    PMG_KRON_W(7)
    PMG_KRON_W(9)
    PMG_KRON_W(11)
#undef PMG_KRON_W
  }
}
template <typename T, int DIM, bool PLAIN>
void launch_kron(const DevStencil& S, int n, unsigned grid, const T* x, const T* b, T* r, double* partial,
                 hipStream_t st) {
  if (resid_rows(S, n) == pmg::kResidRows)
    launch_kron_rb<T, DIM, PLAIN, pmg::kResidRows>(S, n, grid, x, b, r, partial, st);
  else
    launch_kron_rb<T, DIM, PLAIN, 1>(S, n, grid, x, b, r, partial, st);
}

// r = b - A_{h,p} x with block partials of sum(r^2) in partial; returns the
// number of partials written.
template <typename T>
unsigned resid_a(pmg_handle h, const T* x, const T* b, T* r, double* partial, hipStream_t st) {
  const DevStencil& S = h->As;
  if (S.kK) {
    const int n = h->A.nrows;
    const unsigned grid = resid_grid(S, n);
    if (S.dim == 2)
      launch_kron<T, 2, false>(S, n, grid, x, b, r, partial, st);
    else
      launch_kron<T, 3, false>(S, n, grid, x, b, r, partial, st);
    return grid;
  }
  if (S.v) {
    const T* V;
    if constexpr (sizeof(T) == 8) V = S.v; else V = S.v32;
    const int n = h->A.nrows;
    const unsigned grid = resid_grid(S, n);
    if (S.dim == 2)
      launch_stencil<T, 2, false>(S, n, grid, V, x, b, r, partial, st);
    else
      launch_stencil<T, 3, false>(S, n, grid, V, x, b, r, partial, st);
    return grid;
  }
  const T* v;
  if constexpr (sizeof(T) == 8) v = h->A.v; else v = h->A.v32;
  csr_launch<T>(pmg::kResid, h->A.nrows, nullptr, h->A, v, x, b, nullptr, r, partial, st);
  return csr_grid(h->A.nrows, h->A.G);
}

template <typename T>
void fill(T* p, int64_t n, T val, hipStream_t st) {
  if (n > 0) pmg::fill_kernel<T><<<nblocks(n, 256), 256, 0, st>>>(n, p, val);
}

// Waits for the norm enqueued last on st and writes it to *out; EDEVICE if a
// triangular solve of ws reported a fault since the last check.
pmg_status read_norm(Workspace& ws, hipStream_t st, double* out) {
  pmgdev::enqueue_norm_readback(ws, st);
  PMG_HIP_OK(hipStreamSynchronize(st));
  *out = std::sqrt(ws.host_scalar[0]);
  return pmgdev::take_fault(ws, st);
}

// Marks every entry of a solve's output as not final (pmg::kPending).
void fill_pending(double* p, int64_t n, hipStream_t st) {
  fill<unsigned long long>(reinterpret_cast<unsigned long long*>(p), n, pmg::kPending64, st);
}
void fill_pending(float* p, int64_t n, hipStream_t st) {
  fill<unsigned>(reinterpret_cast<unsigned*>(p), n, pmg::kPending32, st);
}

template <typename T>
void lower_launch(pmg_handle h, const pmg::TriCtl& ctl, const T* r, T* y, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_LOWER, st);
  fill_pending(y, h->H.n, st);
  const int g = tri_grid<T>(h->tl);
  pmg::trisolve_lower<T><<<g, 64, 0, st>>>(h->tl.nch, tri_dev<T>(h->tl), h->d_perm, r, y, ctl);
}

template <typename T>
void upper_launch(pmg_handle h, const pmg::TriCtl& ctl, const T* y, T* e, T* x, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_UPPER, st);
  fill_pending(e, h->H.n, st);
  const int g = tri_grid<T>(h->tu);
  pmg::trisolve_upper<T><<<g, 64, 0, st>>>(h->tu.nch, tri_dev<T>(h->tu), h->d_perm, y, e, x, ctl);
}

template <typename T>
void lower_impl(pmg_handle h, Workspace& ws, const T* r, T* y, hipStream_t st) {
  lower_launch<T>(h, tri_ctl(h, ws, 0), r, y, st);
}

template <typename T>
void upper_impl(pmg_handle h, Workspace& ws, const T* y, T* e, T* x, hipStream_t st) {
  upper_launch<T>(h, tri_ctl(h, ws, 1), y, e, x, st);
}

// x += U^{-1} L^{-1} P r (then permuted back) with work vectors y, e.
template <typename T>
void smooth_impl(pmg_handle h, Workspace& ws, const T* r, T* x, T* y, T* e, hipStream_t st) {
  lower_impl<T>(h, ws, r, y, st);
  upper_impl<T>(h, ws, y, e, x, st);
}

void gs_sweeps(pmg_handle h, int l, const double* b, double* e, int nsweep, hipStream_t st) {
  for (int s = 0; s < nsweep; ++s)
    for (int c = 0; c < h->colors; ++c)
      csr_launch<double>(pmg::kGS, h->color_cnt[l][c], h->color_rows[l][c], h->A1[l], h->A1[l].v, nullptr, b,
                         nullptr, e, nullptr, st);
}

// Levels l_lds.. of the structured V-cycle in one launch (pmg::hcycle_lds).
void hcycle_lds(pmg_handle h, const double* b, double* e, hipStream_t st) {
  const pmg::HostOps& H = h->H;
  pmg::LdsCycle S{};
  S.nl = H.nlev - h->l_lds;
  S.colors = h->colors;
  S.nu1 = h->opt.nu1;
  S.nu2 = h->opt.nu2;
  S.ncoarse = H.n_coarse;
  S.cinv = h->coarse_inv;
  S.b0 = b;
  S.e0 = e;
  int off = 0;
  for (int k = 0; k < S.nl; ++k) {
    const int l = h->l_lds + k;
    S.nx[k] = H.lnel[l] - 1;
    if (k + 1 < S.nl) S.lev[k] = h->grid[l];
    S.eoff[k] = off;
    off += (int)H.ln[l];
    S.boff[k] = off;
    off += (int)H.ln[l];
  }
  S.roff = off;
  if (h->prob.dim == 3)
    pmg::hcycle_lds<3><<<1, pmg::kLdsThreads, h->lds_bytes, st>>>(S);
  else
    pmg::hcycle_lds<2><<<1, pmg::kLdsThreads, h->lds_bytes, st>>>(S);
}

// The h-multigrid V-cycle from level l on the structured grids (pmg::grid_*).
// Tiled smoothing on 2-D structured levels (pmg::gs_tile_down / gs_tile_up).
bool tiled_gs(pmg_handle h) {
  return h->opt.tiled_gs && h->prob.dim == 2 && h->opt.nu1 <= pmg::kTileMaxSweeps &&
         h->opt.nu2 <= pmg::kTileMaxSweeps;
}

// Coarse nodes per block side: blocks of up to 30 (about 300 blocks on the
// finest levels, two per CU in LDS), at least 8 on the smaller levels.
int tile_block(int nc) { return std::max(1, std::min(30, std::max(8, nc / 16))); }

size_t tile_lds_bytes(int tcb, int colors, int nsweep, bool down) {
  const int64_t halo = (down ? 2 : 0) + (int64_t)colors * nsweep, w = 2 * tcb + 1 + 2 * halo, rw = 2 * tcb + 1;
  return (size_t)(w * w + (down ? rw * rw : 0)) * 8;
}

void hcycle_grid(pmg_handle h, Workspace& ws, int l, const double* b, double* e, hipStream_t st) {
  const pmg::HostOps& H = h->H;
  if (l == h->l_lds) {
    hcycle_lds(h, b, e, st);
    return;
  }
  if (l == H.nlev - 1) {
    pmg::dense_matvec<<<1, 256, 0, st>>>(H.n_coarse, h->coarse_inv, b, e);
    return;
  }
  const pmg::GridLevel& L = h->grid[l];
  const bool d3 = h->prob.dim == 3;
  if (tiled_gs(h)) {
    // pre-smoothing + residual + restriction, the coarser levels, then
    // prolongation + post-smoothing; the iterate after the pre-smoothing
    // lives in ws.hr[l] (no residual vector is needed on this path)
    const int nc = H.lnel[l + 1] - 1;
    const int tcb = tile_block(nc);
    const int nblk = ((nc + tcb - 1) / tcb) * ((nc + tcb - 1) / tcb);
    double* bc = ws.hb[l + 1];
    double* ec = ws.he[l + 1];
    pmg::gs_tile_down<<<nblk, pmg::kTileThreads, tile_lds_bytes(tcb, h->colors, h->opt.nu1, true), st>>>(
        L, nc, tcb, h->colors, h->opt.nu1, b, e, ws.hr[l], bc, ec);
    hcycle_grid(h, ws, l + 1, bc, ec, st);
    pmg::gs_tile_up<<<nblk, pmg::kTileThreads, tile_lds_bytes(tcb, h->colors, h->opt.nu2, false), st>>>(
        L, nc, tcb, h->colors, h->opt.nu2, b, ws.hr[l], ec, e);
    return;
  }
  auto sweeps = [&](int nsweep) {
    for (int sw = 0; sw < nsweep; ++sw)
      for (int c = 0; c < h->colors; ++c) {
        if (!L.cnt[c]) continue;
        if (d3)
          pmg::grid_gs<3><<<nblocks(L.cnt[c], 256), 256, 0, st>>>(L, c, b, e);
        else
          pmg::grid_gs<2><<<nblocks(L.cnt[c], 256), 256, 0, st>>>(L, c, b, e);
      }
  };
  sweeps(h->opt.nu1);
  double* r = ws.hr[l];
  if (d3)
    pmg::grid_resid<3><<<nblocks(L.n, 256), 256, 0, st>>>(L, b, e, r);
  else
    pmg::grid_resid<2><<<nblocks(L.n, 256), 256, 0, st>>>(L, b, e, r);
  double* bc = ws.hb[l + 1];
  double* ec = ws.he[l + 1];
  const int nc = H.lnel[l + 1] - 1;
  const int64_t ncell = H.ln[l + 1];
  if (d3)
    pmg::grid_restrict<3><<<nblocks(ncell, 256), 256, 0, st>>>(nc, r, bc, ec);
  else
    pmg::grid_restrict<2><<<nblocks(ncell, 256), 256, 0, st>>>(nc, r, bc, ec);
  hcycle_grid(h, ws, l + 1, bc, ec, st);
  if (d3)
    pmg::grid_prolong_add<3><<<nblocks(L.n, 256), 256, 0, st>>>(nc, ec, e);
  else
    pmg::grid_prolong_add<2><<<nblocks(L.n, 256), 256, 0, st>>>(nc, ec, e);
  sweeps(h->opt.nu2);
}

void hcycle(pmg_handle h, Workspace& ws, int l, const double* b, double* e, hipStream_t st) {
  const pmg::HostOps& H = h->H;
  if (!h->grid.empty()) {
    hcycle_grid(h, ws, l, b, e, st);
    return;
  }
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

// Coarse correction e1 ~ A_c^{-1} r1 from e1 = 0: coarse_cycles h-multigrid
// V-cycles at p = 1, or (indirect projection) one V-cycle of the degree p-1
// level, whose own workspace holds its vectors.
void coarse_impl(pmg_handle h, Workspace& ws, const double* r1, double* e1, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_COARSE, st);
  fill<double>(e1, h->H.n1, 0.0, st);
  if (h->sub) {
    pmg_handle c = h->sub;
    const int64_t nc = c->H.n;
    pmg::cast_kernel<double, double><<<nblocks(nc, 256), 256, 0, st>>>(nc, r1, c->ws.r);  // residual at e1 = 0
    pmgdev::vcycle64(c, c->ws, r1, e1, c->ws.r, false, st, false);
    return;
  }
  for (int c = 0; c < h->opt.coarse_cycles; ++c) hcycle(h, ws, 0, r1, e1, st);
}

// x = M^{-1} b for a consistent interior mass matrix M (Appendix B) by
// conjugate gradients preconditioned with the inverse lumped mass dinv, from
// x = 0 until ||b - M x|| <= 1e-13 ||b|| or 20000 steps (the count is
// independent of h but grows with p: about 250 at p = 3 and 1600 at p = 5,
// the lumped masses being a weak preconditioner at high degree).  The two
// scalars of a step are summed on the host from the block partials, in
// block order.
void mass_solve(pmg_handle h, Workspace& ws, const DevMat& M, const double* dinv, const double* b, double* x,
                hipStream_t st) {
  const int64_t n = M.nrows;
  const unsigned nb = std::min<unsigned>(nblocks(n, 256), kMaxCsrBlocks);
  auto sums = [&](double& a, double* c) {
    hipMemcpyAsync(ws.cg_host, ws.cg_pa, nb * sizeof(double), hipMemcpyDeviceToHost, st);
    if (c) hipMemcpyAsync(ws.cg_host + kMaxCsrBlocks, ws.cg_pb, nb * sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    a = 0.0;
    for (unsigned i = 0; i < nb; ++i) a += ws.cg_host[i];
    if (c) {
      *c = 0.0;
      for (unsigned i = 0; i < nb; ++i) *c += ws.cg_host[kMaxCsrBlocks + i];
    }
  };
  pmg::cg_init<<<nb, 256, 0, st>>>(n, b, dinv, x, ws.cg_r, ws.cg_z, ws.cg_p, ws.cg_pa, ws.cg_pb);
  double bb, rz;
  sums(bb, &rz);
  if (!(bb > 0.0)) return;
  for (int it = 0; it < 20000; ++it) {
    csr_launch<double>(pmg::kPlain, (int)n, nullptr, M, M.v, ws.cg_p, nullptr, nullptr, ws.cg_q, nullptr, st);
    pmg::dot2_partials<<<nb, 256, 0, st>>>(n, ws.cg_p, ws.cg_q, nullptr, nullptr, ws.cg_pa, nullptr);
    double pq;
    sums(pq, nullptr);
    if (!(pq > 0.0)) return;
    pmg::cg_step<<<nb, 256, 0, st>>>(n, rz / pq, ws.cg_p, ws.cg_q, dinv, x, ws.cg_r, ws.cg_z, ws.cg_pa, ws.cg_pb);
    double rr, rz2;
    sums(rr, &rz2);
    if (rr <= 1e-26 * bb) return;
    pmg::cg_dir<<<nb, 256, 0, st>>>(n, rz2 / rz, ws.cg_z, ws.cg_p);
    rz = rz2;
  }
}

pmg_status alloc_mass(pmg_handle h, Workspace& ws) {
  if (ws.cg_host) return PMG_OK;
  const int64_t n = h->H.n;
  pmgdev::DevArena& m = ws.mem;
  pmg_status s;
  for (double** v : {&ws.cg_r, &ws.cg_z, &ws.cg_p, &ws.cg_q, &ws.cg_t, &ws.cg_y})
    if ((s = m.alloc(v, n))) return s;
  if ((s = m.alloc(&ws.cg_pa, kMaxCsrBlocks))) return s;
  if ((s = m.alloc(&ws.cg_pb, kMaxCsrBlocks))) return s;
  PMG_HIP_OK(hipHostMalloc((void**)&ws.cg_host, 2 * kMaxCsrBlocks * sizeof(double), hipHostMallocDefault));
  return PMG_OK;
}

// r1 = M_1^{-1} P_p^1 r: lumped (Section 3) or consistent (Appendix B) mass
void restrict64(pmg_handle h, Workspace& ws, const double* r, double* r1, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_RESTRICT, st);
  if (h->opt.mass_transfer == PMG_MASS_CONSISTENT) {
    csr_launch<double>(pmg::kPlain, h->R.nrows, nullptr, h->R, h->R.v, r, nullptr, nullptr, ws.cg_t, nullptr, st);
    mass_solve(h, ws, h->M1, h->ml1_inv, ws.cg_t, r1, st);
    return;
  }
  transfer<double>(h->R, h->Rs, h->prob.dim, r, h->ml1_inv, r1, false, st);
}

// x += M_p^{-1} P_1^p e1: lumped or consistent mass
void prolong64(pmg_handle h, Workspace& ws, const double* e1, double* x, hipStream_t st) {
  ProfScope ps(h, PMG_PROF_PROLONG, st);
  if (h->opt.mass_transfer == PMG_MASS_CONSISTENT) {
    csr_launch<double>(pmg::kPlain, h->P.nrows, nullptr, h->P, h->P.v, e1, nullptr, nullptr, ws.cg_t, nullptr, st);
    mass_solve(h, ws, h->Mp, h->mlp_inv, ws.cg_t, ws.cg_y, st);
    pmg::add_vec<<<std::min<unsigned>(nblocks(h->P.nrows, 256), kMaxCsrBlocks), 256, 0, st>>>(h->P.nrows, ws.cg_y, x);
    return;
  }
  transfer<double>(h->P, h->Ps, h->prob.dim, e1, h->mlp_inv, x, true, st);
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
    smooth_impl<float>(h, ws, cur, c, ws.y32, ws.e32, st);
    resid_a<float>(h, c, ws.r32, t, ws.partial, st);
    cur = t;
  }
  if (n1 > 0) {
    transfer<float>(h->R, h->Rs, h->prob.dim, cur, h->ml1_inv32, ws.q32, false, st);
    pmg::cast_kernel<float, double><<<nblocks(n1, 256), 256, 0, st>>>(n1, ws.q32, ws.r1);
    coarse_impl(h, ws, ws.r1, ws.e1, st);
    pmg::cast_kernel<double, float><<<nblocks(n1, 256), 256, 0, st>>>(n1, ws.e1, ws.q32);
    transfer<float>(h->P, h->Ps, h->prob.dim, ws.q32, h->mlp_inv32, c, true, st);
    resid_a<float>(h, c, ws.r32, t, ws.partial, st);
    cur = t;
  }
  for (int k = 0; k < nu2; ++k) {
    smooth_impl<float>(h, ws, cur, c, ws.y32, ws.e32, st);
    if (k + 1 < nu2) {
      resid_a<float>(h, c, ws.r32, t, ws.partial, st);
      cur = t;
    }
  }
}


}  // namespace

// ----------------------------------------------------------- shared internals
namespace pmgdev {

bool valid_problem(const pmg_problem* p, std::string& msg) {
  if (!p) { msg = "problem is NULL"; return false; }
  if (p->dim != 2 && p->dim != 3) { msg = "dim must be 2 or 3"; return false; }
  if (p->degree < 1 || p->degree > 10) { msg = "degree must be in 1..10"; return false; }
  if (p->n_elem < 2) { msg = "n_elem must be >= 2"; return false; }
  if (p->geometry != PMG_GEOM_BOX && p->geometry != PMG_GEOM_QUARTER_ANNULUS) { msg = "unknown geometry"; return false; }
  if (p->geometry == PMG_GEOM_QUARTER_ANNULUS && p->dim != 2) { msg = "the quarter annulus is 2-D"; return false; }
  if (p->rhs_kind != PMG_RHS_SINE && p->rhs_kind != PMG_RHS_ANNULUS && p->rhs_kind != PMG_RHS_CALLBACK) {
    msg = "unknown rhs_kind";
    return false;
  }
  if (p->rhs_kind == PMG_RHS_CALLBACK && !p->f) { msg = "rhs_kind PMG_RHS_CALLBACK needs f"; return false; }
  if (p->rhs_kind == PMG_RHS_ANNULUS && p->dim != 2) { msg = "the annulus right-hand side is 2-D"; return false; }
  if (p->dim == 3 && p->geometry != PMG_GEOM_BOX) { msg = "3-D supports the unit cube only"; return false; }
  if (p->pde != PMG_PDE_POISSON && p->pde != PMG_PDE_CDR) { msg = "unknown pde"; return false; }
  if (p->pde == PMG_PDE_CDR && (p->dim != 2 || p->geometry != PMG_GEOM_BOX || p->rhs_kind == PMG_RHS_ANNULUS)) {
    msg = "the CDR problem is benchmark 2: unit square, sine or callback right-hand side";
    return false;
  }
  if (p->degree >= 1 && p->degree <= 10 && p->n_elem >= 2 && p->n_elem < (1 << 20)) {
    const int deg = p->degree, ne = p->n_elem, nk = ne + 2 * deg + 1;
    for (int a = 0; a < p->dim; ++a) {
      const double* t = p->knots[a];
      if (!t) continue;
      for (int k = 0; k < nk; ++k) {
        const double want = k <= deg ? 0.0 : k >= ne + deg ? 1.0 : (double)(k - deg) / ne;
        if (!(std::fabs(t[k] - want) <= 1e-12)) {
          msg = "knots[" + std::to_string(a) + "][" + std::to_string(k) + "] = " + std::to_string(t[k]) +
                ": only the open uniform knot vector of degree " + std::to_string(deg) + " on " +
                std::to_string(ne) + " elements is supported (expected " + std::to_string(want) + ")";
          return false;
        }
      }
    }
  }
  for (int a = 0; a < p->dim; ++a)
    if (p->freq[a] < 1 && p->rhs_kind == PMG_RHS_SINE) { msg = "freq must be >= 1"; return false; }
  double n = std::pow((double)(p->n_elem + p->degree - 2), p->dim);
  if (n < 1 || n > 2.0e9) { msg = "problem size out of range"; return false; }
  return true;
}


size_t workspace_bytes(pmg_handle h, bool mixed, bool request_vectors) {
  const pmg::HostOps& H = h->H;
  size_t b = 8 * (3 * (size_t)H.n + 2 * (size_t)std::max(H.n1, 1)) + 8 * (size_t)h->partial_cap + 32;
  for (int l = 0; l < H.nlev; ++l) b += 8 * (size_t)H.ln[l] * (l == 0 ? 1 : 3);
  b += pmg::kTicketAlloc * sizeof(unsigned);
  if (mixed) b += 4 * (5 * (size_t)H.n + (size_t)std::max(H.n1, 1));
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
  if ((s = m.alloc(&ws.e, n))) return s;
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
  if ((s = m.alloc(&ws.tickets, pmg::kTicketAlloc))) return s;
  fill<unsigned>(ws.tickets, pmg::kTicketAlloc, 0u, st);
  if (h->opt.mass_transfer == PMG_MASS_CONSISTENT && H.n1 > 0 && (s = alloc_mass(h, ws))) return s;
  PMG_HIP_OK(hipGetLastError());
  if (mixed) {
    if ((s = m.alloc(&ws.r32, n))) return s;
    if ((s = m.alloc(&ws.c32, n))) return s;
    if ((s = m.alloc(&ws.y32, n))) return s;
    if ((s = m.alloc(&ws.e32, n))) return s;
    if ((s = m.alloc(&ws.t32, n))) return s;
    if ((s = m.alloc(&ws.q32, n1))) return s;
  }
  if (request_vectors) {
    if ((s = m.alloc(&ws.b, n))) return s;
    if ((s = m.alloc(&ws.x, n))) return s;
  }
  PMG_HIP_OK(hipHostMalloc((void**)&ws.host_scalar, 4 * sizeof(double), hipHostMallocDefault));
  std::memset(ws.host_scalar, 0, 4 * sizeof(double));
  if (!st) PMG_HIP_OK(hipDeviceSynchronize());
  return PMG_OK;
}

void residual64(pmg_handle h, Workspace& ws, const double* b, const double* x, double* r, bool norm,
                hipStream_t st) {
  ProfScope ps(h, PMG_PROF_RESIDUAL, st);
  const unsigned np = resid_a<double>(h, x, b, r, ws.partial, st);
  if (norm) pmg::reduce_partials<<<1, 256, 0, st>>>((int)np, ws.partial, ws.scalar);
}

void enqueue_norm_readback(Workspace& ws, hipStream_t st) {
  hipMemcpyAsync(ws.host_scalar, ws.scalar, sizeof(double), hipMemcpyDeviceToHost, st);
  enqueue_fault_readback(ws, st);
}

void enqueue_fault_readback(Workspace& ws, hipStream_t st) {
  hipMemcpyAsync(ws.host_scalar + 1, ws.tickets + 2 * pmg::kTicketWords, sizeof(unsigned), hipMemcpyDeviceToHost,
                 st);
}

pmg_status take_fault(Workspace& ws, hipStream_t st) {
  unsigned f;
  std::memcpy(&f, ws.host_scalar + 1, sizeof f);
  if (!f) return PMG_OK;
  std::memset(ws.host_scalar + 1, 0, sizeof(double));
  fill<unsigned>(ws.tickets + 2 * pmg::kTicketWords, 1, 0u, st);
  return fail(PMG_EDEVICE,
              "a triangular solve stopped waiting for an entry after its poll bound (options.poll_limit); "
              "the results since the last check are invalid");
}

// One FP64 V-cycle; r holds b - A x on entry and exit.
void vcycle64(pmg_handle h, Workspace& ws, const double* b, double* x, double* r, bool norm, hipStream_t st,
              bool final_resid) {
  const int nu1 = h->opt.nu1, nu2 = h->opt.nu2;
  for (int k = 0; k < nu1; ++k) {
    smooth_impl<double>(h, ws, r, x, ws.y, ws.e, st);
    residual64(h, ws, b, x, r, false, st);
  }
  if (h->H.n1 > 0) {
    restrict64(h, ws, r, ws.r1, st);
    coarse_impl(h, ws, ws.r1, ws.e1, st);
    prolong64(h, ws, ws.e1, x, st);
    if (nu2 > 0 || final_resid) residual64(h, ws, b, x, r, nu2 == 0 && norm, st);
  }
  for (int k = 0; k < nu2; ++k) {
    smooth_impl<double>(h, ws, r, x, ws.y, ws.e, st);
    if (k + 1 < nu2 || final_resid) residual64(h, ws, b, x, r, k == nu2 - 1 && norm, st);
  }
  if (nu2 == 0 && h->H.n1 == 0 && final_resid) residual64(h, ws, b, x, r, norm, st);
}

// ---------------------------------------------------------------------------
// BiCGSTAB right-preconditioned by one V-cycle (pmg_bicgstab).

// y = A x (plain product, FP64)
void matvec_a(pmg_handle h, Workspace& ws, const double* x, double* y, hipStream_t st) {
  const DevStencil& S = h->As;
  if (S.kK) {
    const int n = h->A.nrows;
    const unsigned grid = resid_grid(S, n);
    if (S.dim == 2)
      launch_kron<double, 2, true>(S, n, grid, x, x, y, ws.partial, st);
    else
      launch_kron<double, 3, true>(S, n, grid, x, x, y, ws.partial, st);
    return;
  }
  if (S.v) {
    const int n = h->A.nrows;
    const unsigned grid = resid_grid(S, n);
    if (S.dim == 2)
      launch_stencil<double, 2, true>(S, n, grid, S.v, x, x, y, ws.partial, st);
    else
      launch_stencil<double, 3, true>(S, n, grid, S.v, x, x, y, ws.partial, st);
    return;
  }
  csr_launch<double>(pmg::kPlain, h->A.nrows, nullptr, h->A, h->A.v, x, nullptr, nullptr, y, nullptr, st);
}

pmg_status alloc_bicg(pmg_handle h, Workspace& ws) {
  if (ws.bc_S) return PMG_OK;
  const int64_t n = h->H.n;
  DevArena& m = ws.mem;
  pmg_status s;
  for (double** v : {&ws.bc_rh, &ws.bc_p, &ws.bc_v, &ws.bc_y, &ws.bc_z, &ws.bc_t, &ws.bc_w})
    if ((s = m.alloc(v, n))) return s;
  if ((s = m.alloc(&ws.bc_S, 8))) return s;
  if ((s = m.alloc(&ws.bc_pa, kMaxCsrBlocks))) return s;
  if ((s = m.alloc(&ws.bc_pb, kMaxCsrBlocks))) return s;
  PMG_HIP_OK(hipHostMalloc((void**)&ws.bc_host, 8 * sizeof(double), hipHostMallocDefault));
  return PMG_OK;
}

// z = M^{-1} v: one V-cycle on A z = v from z = 0 (w: residual scratch)
void bicg_precond(pmg_handle h, Workspace& ws, const double* v, double* z, double* w, hipStream_t st) {
  const int64_t n = h->H.n;
  fill<double>(z, n, 0.0, st);
  pmg::cast_kernel<double, double><<<nblocks(n, 256), 256, 0, st>>>(n, v, w);  // copy (a kernel, graph-safe)
  vcycle64(h, ws, v, z, w, false, st, false);
}

// One BiCGSTAB iteration (the steps of the textbook method, as listed with
// pmg_bicgstab), all on st; the residual lives in ws.r.
void bicg_iteration(pmg_handle h, Workspace& ws, double* x, hipStream_t st) {
  const int64_t n = h->H.n;
  const unsigned g = std::min<unsigned>(nblocks(n, 256), kMaxCsrBlocks);
  double* S = ws.bc_S;
  pmg::bicg_p<<<g, 256, 0, st>>>(n, S, ws.r, ws.bc_v, ws.bc_p);
  bicg_precond(h, ws, ws.bc_p, ws.bc_y, ws.bc_w, st);
  matvec_a(h, ws, ws.bc_y, ws.bc_v, st);
  pmg::dot2_partials<<<g, 256, 0, st>>>(n, ws.bc_rh, ws.bc_v, nullptr, nullptr, ws.bc_pa, ws.bc_pb);
  pmg::bicg_reduce<<<1, 256, 0, st>>>((int)g, ws.bc_pa, ws.bc_pb, S, 4, -1, 0);
  pmg::bicg_s<<<g, 256, 0, st>>>(n, S, ws.bc_v, ws.bc_y, ws.r, x);
  bicg_precond(h, ws, ws.r, ws.bc_z, ws.bc_w, st);
  matvec_a(h, ws, ws.bc_z, ws.bc_t, st);
  pmg::dot2_partials<<<g, 256, 0, st>>>(n, ws.bc_t, ws.r, ws.bc_t, ws.bc_t, ws.bc_pa, ws.bc_pb);
  pmg::bicg_reduce<<<1, 256, 0, st>>>((int)g, ws.bc_pa, ws.bc_pb, S, 5, 6, 0);
  pmg::bicg_x<<<g, 256, 0, st>>>(n, S, ws.bc_z, ws.bc_t, ws.bc_rh, x, ws.r, ws.bc_pa, ws.bc_pb);
  pmg::bicg_reduce<<<1, 256, 0, st>>>((int)g, ws.bc_pa, ws.bc_pb, S, 7, 0, 1);
}

// Captures the step enqueued by `enqueue` into ws.gexec; false if capture or
// instantiation is refused (the capture stream is left usable either way).
template <typename F>
bool capture_step(Workspace& ws, F&& enqueue) {
  if (!ws.cap && hipStreamCreateWithFlags(&ws.cap, hipStreamNonBlocking) != hipSuccess) {
    ws.cap = nullptr;
    return false;
  }
  if (ws.gexec) {
    hipGraphExecDestroy(ws.gexec);
    ws.gexec = nullptr;
  }
  if (hipStreamBeginCapture(ws.cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  enqueue(ws.cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(ws.cap, &g);
  if (e != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    hipGetLastError();
    return false;
  }
  const hipError_t ei = hipGraphInstantiate(&ws.gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (ei != hipSuccess) {
    ws.gexec = nullptr;
    hipGetLastError();
    return false;
  }
  return true;
}

// Enqueues the work of `enqueue` on st, from the graph cached in ws when the
// key matches (capturing it first otherwise), or kernel by kernel.
template <typename F>
void run_cached(pmg_handle h, Workspace& ws, const void* const (&key)[5], F&& enqueue, hipStream_t st) {
  if (!h->opt.graphs || h->profiling || ws.graph_failed) {
    enqueue(st);
    return;
  }
  if (!ws.gexec || !std::equal(key, key + 5, ws.gkey)) {
    if (!capture_step(ws, enqueue)) {
      ws.graph_failed = true;
      enqueue(st);
      return;
    }
    std::copy(key, key + 5, ws.gkey);
  }
  if (hipGraphLaunch(ws.gexec, st) != hipSuccess) {
    hipGetLastError();
    ws.graph_failed = true;
    enqueue(st);
  }
}

void outer_step(pmg_handle h, Workspace& ws, bool mixed, const double* b, double* x, double* r, bool norm,
                hipStream_t st) {
  auto enqueue = [&](hipStream_t s) {
    if (mixed)
      mixed_step(h, ws, b, x, s);
    else
      vcycle64(h, ws, b, x, r, norm, s);
  };
  const intptr_t kind = mixed ? 2 : (norm ? 1 : 0);
  const void* const key[5] = {h, (const void*)kind, b, x, mixed ? ws.r : r};
  run_cached(h, ws, key, enqueue, st);
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
  o->graphs = 1;
  o->tiled_gs = 1;
  o->mass_transfer = PMG_MASS_LUMPED;
  o->projection = PMG_PROJ_DIRECT;
  o->poll_limit = 0;
  o->ilut_on_device = 1;
  o->tri_waves_per_cu = 0;
  o->segment_rows = 0;
  o->kron_residual = 1;
  return PMG_OK;
}

// A caller's operator (pmg_setup_from_csr) checked and copied into M.
static pmg_status take_csr(int64_t n, int64_t want_n, const int64_t* rp, const int32_t* ci, const double* v,
                           pmg::Csr& M) {
  if (n != want_n) return fail(PMG_EINVAL, "operator has " + std::to_string(n) + " rows, the problem " +
                                               std::to_string(want_n) + " unknowns");
  if (!rp || (rp[n] > 0 && (!ci || !v)) || rp[0] != 0) return fail(PMG_EINVAL, "invalid CSR arrays");
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return fail(PMG_EINVAL, "row pointers decrease at row " + std::to_string(i));
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] < 0 || ci[k] >= n || (k > rp[i] && ci[k] <= ci[k - 1]))
        return fail(PMG_EINVAL, "columns out of range or not increasing in row " + std::to_string(i));
  }
  M.nrows = M.ncols = (int)n;
  M.rp.assign(rp, rp + n + 1);
  M.ci.assign(ci, ci + rp[n]);
  M.v.assign(v, v + rp[n]);
  return PMG_OK;
}

static pmg_status setup_impl(const pmg_problem* prob, const pmg_options* opt, const int64_t* inj_n,
                             const int64_t* inj_rp, const int32_t* inj_ci, const double* inj_v, pmg_handle* out);

pmg_status pmg_setup(const pmg_problem* prob, const pmg_options* opt, pmg_handle* out) {
  return setup_impl(prob, opt, nullptr, nullptr, nullptr, nullptr, out);
}

pmg_status pmg_setup_from_csr(const pmg_problem* prob, int64_t n, const int64_t* rp, const int32_t* ci,
                              const double* v, const pmg_options* opt, pmg_handle* out) {
  return setup_impl(prob, opt, &n, rp, ci, v, out);
}

static pmg_status setup_impl(const pmg_problem* prob, const pmg_options* opt, const int64_t* inj_n,
                             const int64_t* inj_rp, const int32_t* inj_ci, const double* inj_v, pmg_handle* out) {
  pmgdev::set_error("");
  if (!out) return fail(PMG_EINVAL, "out pointer is NULL");
  *out = nullptr;
  std::string msg;
  if (!pmgdev::valid_problem(prob, msg)) return fail(PMG_EINVAL, msg);
  pmg_options o;
  if (opt) o = *opt; else pmg_default_options(&o);
  if (o.nu1 < 0 || o.nu2 < 0 || o.coarse_cycles < 1 || o.coarse_min_elems < 1 || o.max_iter < 0 ||
      !(o.ilut_tau >= 0) || o.gs_variant != PMG_GS_MULTICOLOR ||
      (o.precision != PMG_FP64 && o.precision != PMG_FP32_IN_FP64) ||
      (o.ilut_limit_mode != PMG_LIMIT_PER_PART && o.ilut_limit_mode != PMG_LIMIT_PER_ROW &&
       o.ilut_limit_mode != PMG_LIMIT_HALF_PER_PART) || o.device < -1 ||
      (o.ordering != PMG_ORDER_NATURAL && o.ordering != PMG_ORDER_NESTED_DISSECTION) || o.nd_leaf < 1 ||
      (o.mass_transfer != PMG_MASS_LUMPED && o.mass_transfer != PMG_MASS_CONSISTENT) ||
      (o.mass_transfer == PMG_MASS_CONSISTENT && o.precision != PMG_FP64) ||
      (o.projection != PMG_PROJ_DIRECT && o.projection != PMG_PROJ_INDIRECT) || o.poll_limit < 0 ||
      o.tri_waves_per_cu < 0 || o.segment_rows < 0 || (o.kron_residual != 0 && o.kron_residual != 1))
    return fail(PMG_EINVAL, "invalid options");
  std::unique_ptr<pmg_handle_s> h(new pmg_handle_s());
  h->prob = *prob;
  h->opt = o;
  // the consistent-mass inner solves test convergence on the host: no graphs
  if (o.mass_transfer == PMG_MASS_CONSISTENT) h->opt.graphs = 0;
  pmg::SetupParams sp;
  sp.consistent_mass = o.mass_transfer == PMG_MASS_CONSISTENT;
  sp.cdeg = (o.projection == PMG_PROJ_INDIRECT && prob->degree > 2) ? prob->degree - 1 : 1;
  sp.dim = prob->dim;
  sp.p = prob->degree;
  sp.nel = prob->n_elem;
  sp.geom = prob->geometry;
  sp.rhs = prob->rhs_kind;
  sp.pde = prob->pde;
  sp.fn = prob->f;
  sp.fn_ctx = prob->f_ctx;
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
  if (inj_n) {
    pmg_status si = take_csr(*inj_n, H.n, inj_rp, inj_ci, inj_v, H.A);
    if (si) return si;
    // an injected operator is no Kronecker sum
    H.nk = 0;
    H.kK.clear();
    H.kM.clear();
  }
  {
    auto t0 = std::chrono::steady_clock::now();
    int bad = -1;
    H.perm = pmg::line_ordering(prob->dim, prob->n_elem + prob->degree - 2, prob->degree, o.ordering, o.nd_leaf);
    pmg::Csr Ap = pmg::permute(H.A, H.perm, sp.threads);
    bool factored = false;
    int ndev = 0;
    if (o.ilut_on_device && o.device >= 0 && hipGetDeviceCount(&ndev) == hipSuccess && o.device < ndev) {
      // the same factors as the host factorisation, bit for bit; rows too
      // long for the device kernel fall back to the host
      PMG_HIP_OK(hipSetDevice(o.device));
      std::string why;
      // an injected operator may couple anything: rows strictly in order then
      std::vector<int32_t> order;
      if (inj_n) {
        order.resize(H.n);
        for (int i = 0; i < H.n; ++i) order[i] = i;
      } else {
        order = pmg::factor_ticket_order(prob->dim, prob->n_elem + prob->degree - 2, prob->degree, o.ordering,
                                         o.nd_leaf);
      }
      const pmg_status sd = pmgdev::ilut_device(Ap, order, o.ilut_tau, o.ilut_fill, o.ilut_limit_mode, o.poll_limit,
                                                H.L, H.U, bad, why);
      if (sd == PMG_EZEROPIVOT)
        return fail(PMG_EZEROPIVOT, "ILUT: zero or non-finite pivot in row " + std::to_string(bad));
      if (sd != PMG_OK && sd != PMG_EINVAL) return sd;
      factored = sd == PMG_OK;
      h->info.ilut_on_device = factored ? 1 : 0;
    }
    if (!factored) {
      rc = pmg::ilut_factor(Ap, o.ilut_tau, o.ilut_fill, o.ilut_limit_mode, sp.threads, H.L, H.U, bad);
      if (rc) return fail(PMG_EZEROPIVOT, "ILUT: zero or non-finite pivot in row " + std::to_string(bad));
    }
    H.t_ilut = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  const int seg_len = prob->n_elem + prob->degree - 2;
  {
    auto t0 = std::chrono::steady_clock::now();
    // segments: runs of whole grid lines inside one block of the nested
    // dissection (an injected operator: one line each)
    std::vector<int32_t> seg;
    if (inj_n) {
      for (int r = 0; r < H.n; r += seg_len) seg.push_back(r);
      seg.push_back(H.n);
    } else {
      // by default several lines only when a line is shorter than a chunk:
      // there a chunk spanning lines saves chain steps, while cutting long
      // lines at other places than their ends lengthens the chains
      const int rows = o.segment_rows > 0 ? o.segment_rows : (seg_len >= 64 ? 1 : kSegmentRows);
      seg = pmg::line_segments(prob->dim, seg_len, prob->degree, o.ordering, o.nd_leaf, rows);
    }
    pmg_status bs = build_schedule(H.L, seg, seg_len, false, h->tl);
    if (bs == PMG_OK) bs = build_schedule(H.U, seg, seg_len, true, h->tu);
    if (bs != PMG_OK) return bs;
    h->info.t_schedule = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
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
  I.chunks_l = h->tl.nch;
  I.chunks_u = h->tu.nch;
  I.chunk_levels_l = h->tl.chunk_levels;
  I.chunk_levels_u = h->tu.chunk_levels;
  const int64_t n = H.n, n1 = H.n1;
  // Kronecker factors on the box (for degrees whose stencil width is
  // unrolled), else the stencil layout where it reads fewer bytes than CSR
  h->a_kron = o.kron_residual && H.nk > 0 && prob->degree <= 5;
  {
    const int w = 2 * prob->degree + 1;
    h->a_stencil = h->a_kron ? (prob->dim == 2 ? w * w : w * w * w) : stencil_slots(H);
  }
  I.residual_layout = h->a_kron ? 2 : h->a_stencil ? 1 : 0;
  {
    const int nxa = prob->n_elem + prob->degree - 2;  // grid lines of A's layouts (both axes)
    I.resid_rows = I.residual_layout ? resid_rows((int)n, nxa, nxa) : 0;
  }
  I.bytes_spmv = h->a_kron ? 2 * 8 * (int64_t)H.kK.size() + 24 * (int64_t)H.n
                 : h->a_stencil ? 8 * (int64_t)h->a_stencil * H.n + 24 * (int64_t)H.n
                                : 12 * I.nnz_a + 4 * (n + 1) + 24 * n;
  I.bytes_trisolve_l = 12 * I.nnz_l + 4 * (n + 1) + 16 * n;
  I.bytes_trisolve_u = 12 * I.nnz_u + 4 * (n + 1) + 32 * n;
  {
    const bool cmass = sp.consistent_mass;
    const int nxp = prob->n_elem + prob->degree - 2, nx1 = prob->n_elem + sp.cdeg - 2;
    int lo, W;
    const int64_t sr = n1 > 0 ? xstencil_shape(H.R, prob->dim, nx1, nxp, lo, W) : 0;
    const int wr = W;
    const int64_t sp = n1 > 0 ? xstencil_shape(H.P, prob->dim, nxp, nx1, lo, W) : 0;
    const int wp = W;
    // the transfers on the box from the 1-D factor of their Kronecker product
    // (not with consistent masses, which apply R and P in CSR)
    h->x_kron = o.kron_residual && n1 > 0 && !H.kX.empty() && !cmass;
    I.transfer_layout = h->x_kron ? 2 : (n1 > 0 && sr && sp) ? 1 : 0;
    I.bytes_restrict = (h->x_kron ? 8 * (int64_t)nx1 * wr : sr ? 8 * sr * n1 : 12 * I.nnz_r + 4 * (n1 + 1)) +
                       8 * n + 16 * n1;
    I.bytes_prolong = (h->x_kron ? 8 * (int64_t)nxp * wp : sp ? 8 * sp * n : 12 * I.nnz_p + 4 * (n + 1)) +
                      8 * n1 + 24 * n;
  }
  // degree-1 levels by the layout their kernels read: the 1-D bands (2-D
  // box, tiled), the stencil slots (structured levels, canonical transfers
  // without storage) or CSR
  int64_t bc = 0;
  const bool structured = grid_levels_structured(H, prob->dim);
  for (int l = 0; l < H.nlev; ++l) {
    const int64_t nl = H.ln[l], nc = l + 1 < H.nlev ? H.ln[l + 1] : 0;
    if (l == H.nlev - 1) {
      bc += 8 * (int64_t)H.n_coarse * H.n_coarse + 16 * nl;
      continue;
    }
    const bool bands = structured && o.kron_residual && tiled_gs(h.get()) && l < (int)H.k1K.size() &&
                       !H.k1K[l].empty();
    const int64_t a1 = bands ? 2 * 8 * (int64_t)H.k1K[l].size()
                       : structured ? 8 * (prob->dim == 2 ? 9 : 27) * nl
                                    : H.A1[l].nnz() * 12 + 4 * (nl + 1);
    const int64_t rt = structured ? 0 : 12 * H.Rh[l].nnz(), pt = structured ? 0 : 12 * H.Ph[l].nnz();
    const int64_t sweeps = o.nu1 + o.nu2;
    bc += sweeps * (a1 + 24 * nl) + (a1 + 24 * nl) + (rt + 8 * nl + 8 * nc) + (pt + 16 * nl + 8 * nc) + 8 * nc;
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
    // CSR copies only of the operators that have no stencil layout
    if (h->a_stencil) describe_mat(H.A, h->A);
    else if ((s = upload_mat(m, H.A, h->A, mixed))) return s;
    if ((s = upload_stencil(m, H, h->a_stencil, h->a_kron, h->As, mixed))) return s;
    if ((s = upload_tri(m, h->tl, false, mixed))) return s;
    if ((s = upload_tri(m, h->tu, true, mixed))) return s;
    if ((s = size_tri_grid<double>(o.device, o.tri_waves_per_cu, h->tl, h->tu))) return s;
    if (mixed && (s = size_tri_grid<float>(o.device, o.tri_waves_per_cu, h->tl, h->tu))) return s;
    if (n1 > 0) {
      const int nxp = prob->n_elem + prob->degree - 2, nx1 = prob->n_elem + sp.cdeg - 2;
      if (h->x_kron) {
        if ((s = upload_xkron(m, H, H.R, true, prob->dim, nx1, nxp, h->Rs))) return s;
        if ((s = upload_xkron(m, H, H.P, false, prob->dim, nxp, nx1, h->Ps))) return s;
      } else {
        if ((s = upload_xstencil(m, H.R, prob->dim, nx1, nxp, h->Rs, mixed))) return s;
        if ((s = upload_xstencil(m, H.P, prob->dim, nxp, nx1, h->Ps, mixed))) return s;
      }
      // (the consistent-mass transfers apply R and P unscaled, in CSR)
      if ((h->Rs.v || h->Rs.tab) && !sp.consistent_mass) describe_mat(H.R, h->R);
      else if ((s = upload_mat(m, H.R, h->R, mixed))) return s;
      if ((h->Ps.v || h->Ps.tab) && !sp.consistent_mass) describe_mat(H.P, h->P);
      else if ((s = upload_mat(m, H.P, h->P, mixed))) return s;
      if (sp.consistent_mass) {
        if ((s = upload_mat(m, H.Mp, h->Mp, false))) return s;
        if ((s = upload_mat(m, H.M1, h->M1, false))) return s;
      }
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
    if ((s = upload_grid_levels(m, H, prob->dim, o.kron_residual != 0, h->grid))) return s;
    h->info.coarse_kron_levels = 0;
    for (const pmg::GridLevel& L : h->grid) h->info.coarse_kron_levels += L.kK != nullptr;
    if (!h->grid.empty() && tiled_gs(h.get())) {
      const size_t dn = tile_lds_bytes(30, h->colors, pmg::kTileMaxSweeps, true);
      const size_t up = tile_lds_bytes(30, h->colors, pmg::kTileMaxSweeps, false);
      PMG_HIP_OK(hipFuncSetAttribute((const void*)pmg::gs_tile_down, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dn));
      PMG_HIP_OK(hipFuncSetAttribute((const void*)pmg::gs_tile_up, hipFuncAttributeMaxDynamicSharedMemorySize, (int)up));
    }
    // the smallest levels in one workgroup: from the coarsest upwards while
    // their iterates, right-hand sides and one residual fit 128 KiB of LDS
    if (!h->grid.empty()) {
      int64_t need = 0;
      int ll = -1;
      for (int l = H.nlev - 1; l >= 0 && H.nlev - l <= pmg::kLdsLevels; --l) {
        const int64_t dbl = need + 2 * H.ln[l] + H.ln[l];  // this level's e, b and the residual scratch
        if (dbl * 8 > (128 << 10)) break;
        need += 2 * H.ln[l];
        ll = l;
        h->lds_bytes = (size_t)dbl * 8;
      }
      h->l_lds = ll;
      if (ll >= 0) {
        auto k2 = pmg::hcycle_lds<2>;
        auto k3 = pmg::hcycle_lds<3>;
        if (prob->dim == 3)
          PMG_HIP_OK(hipFuncSetAttribute((const void*)k3, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_bytes));
        else
          PMG_HIP_OK(hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)h->lds_bytes));
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
    if ((s = m.upload(&h->d_perm, H.perm.data(), H.perm.size()))) return s;
    if ((s = pmgdev::alloc_workspace(h.get(), h->ws, mixed, false))) return s;
    PMG_HIP_OK(hipDeviceSynchronize());
    I.t_upload = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    I.device_bytes = (int64_t)(h->ops.bytes + h->ws.mem.bytes);
  }
  if (sp.cdeg > 1) {
    // indirect projection: the degree p-1 level, set up with the same
    // options (and so itself indirect down to degree 2)
    pmg_problem sub = *prob;
    sub.degree = prob->degree - 1;
    pmg_handle sh = nullptr;
    const pmg_status s2 = pmg_setup(&sub, &o, &sh);
    if (s2 != PMG_OK) return s2;  // the inner call has set the message
    h->sub = sh;
  }
  *out = h.release();
  return PMG_OK;
}

pmg_status pmg_destroy(pmg_handle h) {
  delete h;
  return PMG_OK;
}

pmg_status pmg_set_precision(pmg_handle h, int32_t precision) {
  if (!h) return fail(PMG_EINVAL, "NULL handle");
  if (precision != PMG_FP64 && precision != PMG_FP32_IN_FP64) return fail(PMG_EINVAL, "unknown precision");
  if (precision == PMG_FP32_IN_FP64 && !h->ws.mixed)
    return fail(PMG_EINVAL, "the handle was set up in FP64 only: set it up with precision PMG_FP32_IN_FP64");
  h->opt.precision = precision;
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

pmg_status pmg_export_schedule(pmg_handle h, int32_t factor, int32_t field, int64_t* count, void* out) {
  if (!h || !count) return fail(PMG_EINVAL, "NULL argument");
  if (factor != 0 && factor != 1) return fail(PMG_EINVAL, "factor must be 0 (lower) or 1 (upper)");
  const TriSched& S = factor ? h->tu : h->tl;
  const std::vector<int>* iv = nullptr;
  const std::vector<double>* dv = nullptr;
  switch (field) {
    case 0: iv = &S.order; break;
    case 1: iv = &S.wptr; break;
    case 2: iv = &S.deps; break;
    case 3: iv = &S.off_ptr; break;
    case 4: iv = &S.off_w; break;
    case 5: iv = &S.off_col; break;
    case 6: iv = &S.in_ptr; break;
    case 7: iv = &S.in_w; break;
    case 8: iv = &S.in_j; break;
    case 9: dv = &S.off_val; break;
    case 10: dv = &S.in_val; break;
    case 11: dv = &S.diag; break;
    case 12: iv = &S.chunk_row; break;
    case 13: iv = &S.chunk_len; break;
    case 14: iv = &S.seg_start; break;
    default: return fail(PMG_EINVAL, "unknown schedule field " + std::to_string(field));
  }
  if (iv) {
    *count = (int64_t)iv->size();
    if (out) std::memcpy(out, iv->data(), sizeof(int) * iv->size());
  } else {
    *count = (int64_t)dv->size();
    if (out) std::memcpy(out, dv->data(), sizeof(double) * dv->size());
  }
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
  if (rnorm) return read_norm(h->ws, st, rnorm);
  return PMG_OK;
}

pmg_status pmg_smooth(pmg_handle h, const double* r, double* x, void* stream) {
  NEED_DEVICE(h);
  if (!r || !x) return fail(PMG_EINVAL, "NULL vector");
  smooth_impl<double>(h, h->ws, r, x, h->ws.y, h->ws.e, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_smooth_static(pmg_handle h, const double* r, double* x, void* stream) {
  NEED_DEVICE(h);
  if (!r || !x) return fail(PMG_EINVAL, "NULL vector");
  if ((int64_t)h->H.n > kStaticMaxN)
    return fail(PMG_EINVAL, "pmg_smooth_static: " + std::to_string(h->H.n) +
                                " unknowns exceed the static scratch (at most " + std::to_string(kStaticMaxN) +
                                "); use pmg_smooth");
  unsigned char* base = nullptr;
  pmg_status s;
  if ((s = static_scratch(h->device, &base))) return s;
  hipStream_t st = (hipStream_t)stream;
  unsigned* tick = reinterpret_cast<unsigned*>(base);
  double* y = reinterpret_cast<double*>(base + kStaticHead);
  double* e = y + kStaticMaxN;
  // the counters must start at zero (a kernel, not a memset, so the call can
  // be captured into a graph); the fault word stays the handle's
  fill<unsigned>(tick, 2 * pmg::kTicketWords, 0u, st);
  const pmg::TriCtl lo = tri_ctl(h, h->ws, 0), up = tri_ctl(h, h->ws, 1);
  lower_launch<double>(h, pmg::TriCtl{tick, lo.fault, lo.poll_limit}, r, y, st);
  upper_launch<double>(h, pmg::TriCtl{tick + pmg::kTicketWords, up.fault, up.poll_limit}, y, e, x, st);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_lower_solve(pmg_handle h, const double* r, double* y, void* stream) {
  NEED_DEVICE(h);
  if (!r || !y) return fail(PMG_EINVAL, "NULL vector");
  lower_impl<double>(h, h->ws, r, y, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_upper_solve(pmg_handle h, double* y, double* x, void* stream) {
  NEED_DEVICE(h);
  if (!y || !x) return fail(PMG_EINVAL, "NULL vector");
  upper_impl<double>(h, h->ws, y, h->ws.e, x, (hipStream_t)stream);
  PMG_HIP_OK(hipMemcpyAsync(y, h->ws.e, sizeof(double) * h->H.n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
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
  restrict64(h, h->ws, r, r1, (hipStream_t)stream);
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
  prolong64(h, h->ws, e1, x, (hipStream_t)stream);
  PMG_HIP_OK(hipGetLastError());
  return PMG_OK;
}

pmg_status pmg_vcycle(pmg_handle h, const double* b, double* x, double* r, double* rnorm, void* stream) {
  NEED_DEVICE(h);
  if (!b || !x || !r) return fail(PMG_EINVAL, "NULL vector");
  hipStream_t st = (hipStream_t)stream;
  pmgdev::outer_step(h, h->ws, false, b, x, r, rnorm != nullptr, st);
  PMG_HIP_OK(hipGetLastError());
  if (rnorm) return read_norm(h->ws, st, rnorm);
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
  double r0 = 0.0;
  pmg_status s0 = read_norm(ws, st, &r0);
  if (s0) return s0;
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
      pmgdev::outer_step(h, ws, mixed, b, x, ws.r, true, st);
      PMG_HIP_OK(hipGetLastError());
      double nrm = 0.0;
      if ((s0 = read_norm(ws, st, &nrm))) return s0;
      const double rel = nrm / r0;
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

pmg_status pmg_bicgstab(pmg_handle h, const double* b, double* x, double tol, pmg_result* res, double* hist,
                        void* stream) {
  NEED_DEVICE(h);
  if (!b || !x || !(tol >= 0)) return fail(PMG_EINVAL, "invalid argument");
  hipStream_t st = (hipStream_t)stream;
  Workspace& ws = h->ws;
  pmg_status s;
  if ((s = pmgdev::alloc_bicg(h, ws))) return s;
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = h->H.n;
  pmg_result R{};
  // r = b - A x, r^ = r, rho = (r^, r) = ||r||^2, rho_prev = alpha = omega = 1, p = v = 0
  pmgdev::residual64(h, ws, b, x, ws.r, true, st);
  pmg::cast_kernel<double, double><<<nblocks(n, 256), 256, 0, st>>>(n, ws.r, ws.bc_rh);
  fill<double>(ws.bc_p, n, 0.0, st);
  fill<double>(ws.bc_v, n, 0.0, st);
  pmg::bicg_init<<<1, 1, 0, st>>>(ws.scalar, ws.bc_S);
  PMG_HIP_OK(hipGetLastError());
  double r0 = 0.0;
  if ((s = read_norm(ws, st, &r0))) return s;
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
    const void* const key[5] = {h, (const void*)(intptr_t)3, b, x, ws.bc_S};
    for (int it = 1; it <= h->opt.max_iter; ++it) {
      pmgdev::run_cached(h, ws, key, [&](hipStream_t q) { pmgdev::bicg_iteration(h, ws, x, q); }, st);
      PMG_HIP_OK(hipMemcpyAsync(ws.bc_host, ws.bc_S, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
      pmgdev::enqueue_fault_readback(ws, st);
      PMG_HIP_OK(hipStreamSynchronize(st));
      if ((s = pmgdev::take_fault(ws, st))) return s;
      const double rel = std::sqrt(ws.bc_host[7]) / r0;
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
      // omega = 0 (s = 0 without convergence) or rho = 0 for the next
      // iteration: breakdown
      if (ws.bc_host[3] == 0.0 || ws.bc_host[0] == 0.0) {
        status = PMG_EDIVERGED;
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
