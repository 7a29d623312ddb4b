// Setup on the device: ILUT(tau, m) of P A_p P^T by the kernel of
// ilut_kernels.hpp (Section 3, "Smoother"), giving the same factors as the
// host factorisation (setup_ilut.cpp) bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ilut_kernels.hpp"
#include "pmg_internal.hpp"

namespace {

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

pmg_status ilut_device(const pmg::Csr& Ap, double tau, double fill_factor, int mode, int poll_limit, pmg::Csr& L,
                       pmg::Csr& U, int& bad_row, std::string& why) {
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
  // working-row table: 8 slots per entry of the longest row to start with,
  // doubled while a row outgrows three quarters of it and LDS allows
  int tbits = 9;
  while ((int64_t(1) << tbits) < 8 * std::max(maxrow, cu) && tbits < 14) ++tbits;
  int64_t list_cap = cl + cu;
  list_cap += list_cap & 1;
  auto lds_of = [&](int tb) { return 12 * (size_t(1) << tb) + 12 * (size_t)list_cap; };
  const size_t kLdsMax = size_t(152) << 10;
  if (lds_of(tbits) > kLdsMax || (double)n * (double)(cl + cu) > 4.0e9) {
    why = "rows too long for the device factorisation";
    return PMG_EINVAL;
  }
  DevArena mem;
  struct Release {
    DevArena& m;
    ~Release() { m.release(); }
  } rel{mem};
  int64_t *rp = nullptr;
  int *ci = nullptr, *Lc = nullptr, *Ln = nullptr, *Uc = nullptr, *Un = nullptr, *flags = nullptr;
  double *v = nullptr, *Lv = nullptr, *Uv = nullptr;
  unsigned *state = nullptr, *fault = nullptr;
  pmg_status s;
  if ((s = mem.upload(&rp, Ap.rp.data(), Ap.rp.size()))) return s;
  if ((s = mem.upload(&ci, Ap.ci.data(), Ap.ci.size()))) return s;
  if ((s = mem.upload(&v, Ap.v.data(), Ap.v.size()))) return s;
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
  for (;;) {
    const size_t lds = lds_of(tbits);
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
    A.list_cap = (int)list_cap;
    PMG_HIP_OK(hipFuncSetAttribute((const void*)pmg::ilut::ilut_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
    int dev = 0, per_cu = 0;
    PMG_HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    PMG_HIP_OK(hipGetDeviceProperties(&prop, dev));
    PMG_HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pmg::ilut::ilut_rows, 64, lds));
    const int64_t grid =
        std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(per_cu, 1) * prop.multiProcessorCount, n));
    pmg::ilut::ilut_rows<<<(unsigned)grid, 64, lds>>>(A);
    PMG_HIP_OK(hipGetLastError());
    PMG_HIP_OK(hipDeviceSynchronize());
    unsigned hfault = 0;
    PMG_HIP_OK(hipMemcpy(hflags, flags, sizeof hflags, hipMemcpyDeviceToHost));
    PMG_HIP_OK(hipMemcpy(&hfault, fault, sizeof hfault, hipMemcpyDeviceToHost));
    if (hfault) return fail(PMG_EDEVICE, "device ILUT: a row waited past its poll bound");
    if (!hflags[1]) break;
    if (lds_of(tbits + 1) > kLdsMax) {
      why = "a working row outgrew the largest table";
      return PMG_EINVAL;
    }
    ++tbits;
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
  for (int i = 0; i < n; ++i) {
    std::copy(lc.begin() + (size_t)i * cl, lc.begin() + (size_t)i * cl + ln[i], L.ci.begin() + L.rp[i]);
    std::copy(lv.begin() + (size_t)i * cl, lv.begin() + (size_t)i * cl + ln[i], L.v.begin() + L.rp[i]);
    std::copy(uc.begin() + (size_t)i * cu, uc.begin() + (size_t)i * cu + un[i], U.ci.begin() + U.rp[i]);
    std::copy(uv.begin() + (size_t)i * cu, uv.begin() + (size_t)i * cu + un[i], U.v.begin() + U.rp[i]);
  }
  return PMG_OK;
}

}  // namespace pmgdev
