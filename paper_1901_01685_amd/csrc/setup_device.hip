// Setup on the device: ILUT(tau, m) of P A_p P^T by the kernel of
// ilut_kernels.hpp (Section 3, "Smoother"), giving the same factors as the
// host factorisation (setup_ilut.cpp) bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "ilut_kernels.hpp"
#include "pmg_internal.hpp"

namespace {

// Largest working-row table in LDS (slots, log2); the first global-memory
// tables are sized for working rows of this many times the longest row of
// A (the longest working rows measured on the host: 99 times at p = 5,
// h = 1/512 in 2-D, 215 times at p = 3, h = 1/64 on the cube); the most
// global memory the tables may take together.
constexpr int kLdsBitsMax = 12;
constexpr int64_t kGlobalRowsPerEntry = 300;
constexpr double kGlobalTableBytes = 16.0e9;

template <typename T>
__global__ void fill_words(int64_t n, T* __restrict__ p, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
void fill(T* p, int64_t n, T v) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  fill_words<T><<<(unsigned)blocks, 256>>>(n, p, v);
}

}  // namespace

namespace pmgdev {

pmg_status ilut_device(const pmg::Csr& Ap, const std::vector<int32_t>& order, double tau, double fill_factor, int mode,
                       int poll_limit, pmg::Csr& L, pmg::Csr& U, int& bad_row, std::string& why) {
  const int n = Ap.nrows;
  const int64_t nnzA = Ap.nnz();
  bad_row = -1;
  if (n <= 0 || !(fill_factor > 0)) {
    why = "unlimited fill is factored on the host";
    return PMG_EINVAL;
  }
  const int64_t M = (int64_t)std::floor(fill_factor * (double)nnzA / (double)n);
  int64_t keep_l, keep_u;
  if (mode == 1) {
    keep_l = keep_u = M;
  } else {
    keep_l = keep_u = mode == 2 ? M / 2 : M;
  }
  const int64_t cl = std::max<int64_t>(keep_l, 1), cu = keep_u + 1;
  int64_t maxrow = 1;
  for (int i = 0; i < n; ++i) maxrow = std::max<int64_t>(maxrow, Ap.rp[i + 1] - Ap.rp[i]);
  // working row in LDS: 20 slots per entry of the longest row of A (rows
  // with fill reach about 16 times their length; a table counts as full at
  // 7/8), at most 2^12 slots so that three waves share a compute unit.  A
  // row that outgrows it is factored again in its wave's table in global
  // memory, which is sized for the longest working rows of the largest
  // problems and doubled (the factorisation run again) if a row outgrows it.
  int tbits = 9;
  while ((int64_t(1) << tbits) < 20 * std::max(maxrow, cu) && tbits < kLdsBitsMax) ++tbits;
  auto lds_of = [&](int tb) { return 12 * (size_t(1) << tb) + 256 * sizeof(int); };
  auto full_of = [](int tb) { return (int)((int64_t(1) << tb) - (int64_t(1) << tb) / 8); };
  int gbits = 0;
  const int64_t nw0 = ((int64_t)n + 63) / 64;  // level-0 words of the lower-part bitmap
  if (n > full_of(tbits)) {
    gbits = tbits + 1;
    while (full_of(gbits) < std::min<int64_t>(n, kGlobalRowsPerEntry * maxrow)) ++gbits;
    // the level-1 words of that bitmap take the LDS of the table
    while (8 * ((nw0 + 63) / 64) > 12 * (int64_t(1) << tbits) && tbits < kLdsBitsMax) ++tbits;
    if (8 * ((nw0 + 63) / 64) > 12 * (int64_t(1) << tbits)) {
      why = "too many unknowns for the device factorisation's bitmaps";
      return PMG_EINVAL;
    }
  }
  if ((int64_t)order.size() != n || cu > pmg::ilut::kMaxChunks * pmg::ilut::kWave ||
      (double)n * (double)(cl + cu) > 4.0e9) {
    why = "rows too long for the device factorisation";
    return PMG_EINVAL;
  }
  DevArena mem;
  struct Release {
    DevArena& m;
    ~Release() { m.release(); }
  } rel{mem};
  int64_t *rp = nullptr;
  int *ci = nullptr, *Lc = nullptr, *Ln = nullptr, *Uc = nullptr, *Un = nullptr, *flags = nullptr, *ord = nullptr;
  double *v = nullptr, *Lv = nullptr, *Uv = nullptr;
  unsigned *state = nullptr, *fault = nullptr;
  pmg_status s;
  if ((s = mem.upload(&rp, Ap.rp.data(), Ap.rp.size()))) return s;
  if ((s = mem.upload(&ci, Ap.ci.data(), Ap.ci.size()))) return s;
  if ((s = mem.upload(&v, Ap.v.data(), Ap.v.size()))) return s;
  if ((s = mem.upload(&ord, order.data(), order.size()))) return s;
  {
    std::vector<char> seen((size_t)n, 0);
    for (int t = 0; t < n; ++t) {
      if (order[t] < 0 || order[t] >= n || seen[order[t]]) {
        why = "the ticket order is not a permutation";
        return PMG_EINVAL;
      }
      seen[order[t]] = 1;
    }
  }
  if ((s = mem.alloc(&Lc, (size_t)n * cl))) return s;
  if ((s = mem.alloc(&Lv, (size_t)n * cl))) return s;
  if ((s = mem.alloc(&Ln, n))) return s;
  if ((s = mem.alloc(&Uc, (size_t)n * cu))) return s;
  if ((s = mem.alloc(&Uv, (size_t)n * cu))) return s;
  if ((s = mem.alloc(&Un, n))) return s;
  if ((s = mem.alloc(&state, pmg::kTicketWords))) return s;
  if ((s = mem.alloc(&fault, 1))) return s;
  if ((s = mem.alloc(&flags, 2))) return s;
  int hflags[2] = {0, 0};
  int dev = 0;
  PMG_HIP_OK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  PMG_HIP_OK(hipGetDeviceProperties(&prop, dev));
  const size_t lds = lds_of(tbits);
  PMG_HIP_OK(hipFuncSetAttribute((const void*)pmg::ilut::ilut_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
  int per_cu = 0;
  PMG_HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pmg::ilut::ilut_rows, 64, lds));
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(per_cu, 1) * prop.multiProcessorCount, n));
  int* gkeys = nullptr;
  double* gvals = nullptr;
  unsigned long long* gb0 = nullptr;
  DevArena gmem;
  struct ReleaseG {
    DevArena& m;
    ~ReleaseG() { m.release(); }
  } relg{gmem};
  for (;;) {
    if (gbits) {
      if ((double)grid * (12.0 * (double)(int64_t(1) << gbits) + 8.0 * (double)nw0) > kGlobalTableBytes) {
        why = "a working row outgrew the largest global-memory table";
        return PMG_EINVAL;
      }
      gmem.release();
      if ((s = gmem.alloc(&gkeys, (size_t)grid << gbits))) return s;
      if ((s = gmem.alloc(&gvals, (size_t)grid << gbits))) return s;
      if ((s = gmem.alloc(&gb0, (size_t)grid * (size_t)nw0))) return s;
      fill<unsigned long long>(gb0, grid * nw0, 0ull);
    }
    fill<int>(Un, n, -1);
    fill<int>(Uc, (int64_t)n * cu, -1);
    fill<unsigned long long>(reinterpret_cast<unsigned long long*>(Uv), (int64_t)n * cu, pmg::kPending64);
    fill<unsigned>(state, pmg::kTicketWords, 0u);
    fill<unsigned>(fault, 1, 0u);
    fill<int>(flags, 1, n);
    fill<int>(flags + 1, 1, 0);
    PMG_HIP_OK(hipGetLastError());
    pmg::ilut::Args A{};
    A.n = n;
    A.rp = rp;
    A.ci = ci;
    A.v = v;
    A.tau = tau;
    A.mode = mode == 1 ? 1 : 0;
    A.keep_l = (int)keep_l;
    A.keep_u = (int)keep_u;
    A.cl = (int)cl;
    A.cu = (int)cu;
    A.Lc = Lc;
    A.Lv = Lv;
    A.Ln = Ln;
    A.Uc = Uc;
    A.Uv = Uv;
    A.Un = Un;
    A.state = state;
    A.fault = fault;
    A.flags = flags;
    // a row can wait for most of the factorisation's critical path: a wider
    // default bound than the triangular solves'
    A.poll_limit = poll_limit > 0 ? poll_limit : (1 << 26);
    A.tbits = tbits;
    A.full = full_of(tbits);
    A.order = ord;
    A.gkeys = gkeys;
    A.gvals = gvals;
    A.gbits = gbits;
    A.gfull = gbits ? full_of(gbits) : 0;
    A.gbits0 = gb0;
    A.nw0 = (int)nw0;
    pmg::ilut::ilut_rows<<<(unsigned)grid, 64, lds>>>(A);
    PMG_HIP_OK(hipGetLastError());
    PMG_HIP_OK(hipDeviceSynchronize());
    unsigned hfault = 0;
    PMG_HIP_OK(hipMemcpy(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost));
    PMG_HIP_OK(hipMemcpy(&hfault, fault, sizeof hfault, hipMemcpyDeviceToHost));
    if (hfault) return fail(PMG_EDEVICE, "device ILUT: a row waited past its poll bound");
    if (hflags[1] & 2) {
      why = "device ILUT met an inconsistent working row";
      return PMG_EINVAL;
    }
    if (!hflags[1]) break;
    gbits = gbits ? gbits + 1 : tbits + 1;
  }
  if (hflags[0] < n) {
    bad_row = hflags[0];
    return PMG_EZEROPIVOT;
  }
  std::vector<int> ln(n), un(n);
  PMG_HIP_OK(hipMemcpy(ln.data(), Ln, sizeof(int) * n, hipMemcpyDeviceToHost));
  PMG_HIP_OK(hipMemcpy(un.data(), Un, sizeof(int) * n, hipMemcpyDeviceToHost));
  std::vector<int> lc((size_t)n * cl), uc((size_t)n * cu);
  std::vector<double> lv((size_t)n * cl), uv((size_t)n * cu);
  PMG_HIP_OK(hipMemcpy(lc.data(), Lc, sizeof(int) * lc.size(), hipMemcpyDeviceToHost));
  PMG_HIP_OK(hipMemcpy(lv.data(), Lv, sizeof(double) * lv.size(), hipMemcpyDeviceToHost));
  PMG_HIP_OK(hipMemcpy(uc.data(), Uc, sizeof(int) * uc.size(), hipMemcpyDeviceToHost));
  PMG_HIP_OK(hipMemcpy(uv.data(), Uv, sizeof(double) * uv.size(), hipMemcpyDeviceToHost));
  L = pmg::Csr();
  U = pmg::Csr();
  L.nrows = L.ncols = U.nrows = U.ncols = n;
  L.rp.assign((size_t)n + 1, 0);
  U.rp.assign((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i) {
    if (ln[i] < 0 || ln[i] > cl || un[i] < 1 || un[i] > cu) return fail(PMG_EDEVICE, "device ILUT: bad row counts");
    L.rp[i + 1] = L.rp[i] + ln[i];
    U.rp[i + 1] = U.rp[i] + un[i];
  }
  L.ci.resize(L.rp[n]);
  L.v.resize(L.rp[n]);
  U.ci.resize(U.rp[n]);
  U.v.resize(U.rp[n]);
  // rows were stored in the order their entries were found: sort each by
  // column (U keeps its diagonal first)
  auto place = [&](int lo, int hi) {
    std::vector<std::pair<int, double>> row;
    for (int i = lo; i < hi; ++i) {
      row.clear();
      for (int t = 0; t < ln[i]; ++t) row.emplace_back(lc[(size_t)i * cl + t], lv[(size_t)i * cl + t]);
      std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      for (int t = 0; t < ln[i]; ++t) {
        L.ci[L.rp[i] + t] = row[t].first;
        L.v[L.rp[i] + t] = row[t].second;
      }
      row.clear();
      for (int t = 1; t < un[i]; ++t) row.emplace_back(uc[(size_t)i * cu + t], uv[(size_t)i * cu + t]);
      std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      U.ci[U.rp[i]] = uc[(size_t)i * cu];
      U.v[U.rp[i]] = uv[(size_t)i * cu];
      for (int t = 1; t < un[i]; ++t) {
        U.ci[U.rp[i] + t] = row[t - 1].first;
        U.v[U.rp[i] + t] = row[t - 1].second;
      }
    }
  };
  const int nth = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  const int chunk = (n + nth - 1) / nth;
  for (int t = 0; t < nth; ++t) {
    const int lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo < hi) pool.emplace_back(place, lo, hi);
  }
  for (auto& th : pool) th.join();
  return PMG_OK;
}

}  // namespace pmgdev
