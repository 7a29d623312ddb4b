// ILUT(tau, m) on the device (Section 3, "Smoother": the dual-threshold
// incomplete LU of the stiffness matrix), the same algorithm and the same
// arithmetic as the host factorisation in setup_ilut.cpp, so both give
// identical factors:
//   for row i, w = row i of P A P^T;  tau_i = tau * (sum_j |a_ij|) / nnz_i;
//   for k < i in increasing order with w_k != 0: w_k /= u_kk; drop it if
//     |w_k| < tau_i, else w_j -= w_k u_kj for the entries of row k of U
//     (product and difference rounded separately, as the host computes them);
//   drop the remaining |w_j| < tau_i (never the diagonal); keep the largest
//   entries per rule 2 (magnitudes ranked in single precision, ties to the
//   smaller column) and store them sorted by column, the diagonal first in U.
//
// One wave factors one row at a time; rows are drawn from a ticket counter in
// an order in which every row comes after the rows it can depend on (the
// blocks of the nested dissection by height, independent blocks interleaved),
// so the smallest unfinished ticket only waits for finished rows and is held
// by a running wave (the argument of the triangular solves).  The working row lives in LDS as an open-addressing hash table
// keyed by column.  A row of U is published entry by entry with device-scope
// stores into slots that hold a marker until written (column -1, value the
// signalling-NaN marker, count -1): a wave waiting for row k reloads the
// count and the entries it needs until no marker is left, so readiness
// travels with the data and no fence is needed.  Waits are bounded as in the
// triangular solves (poll_limit, fault word).  Each pivot row is fetched in
// one round of loads (count and slots together); the entries kept by rule 2
// are found by a radix select on their rank keys and stored in the order they
// are found (the host sorts each row by column afterwards; the factorisation
// itself does not depend on the order of a row's entries).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tri_layout.hpp"

namespace pmg {
namespace ilut {

constexpr int kWave = 64;

struct Args {
  int n;
  const int64_t* rp;  // P A P^T: row pointers, columns ascending within a row
  const int* ci;
  const double* v;
  double tau;
  int mode;      // 0: keep_l in L and keep_u in U; 1: keep_l in the whole row
  int keep_l, keep_u;
  int cl, cu;    // slots per row of L, and of U with the diagonal first
  int* Lc;       // n * cl
  double* Lv;
  int* Ln;       // entries of each row of L
  int* Uc;       // n * cu, -1 until written
  double* Uv;    // n * cu, kPending64 until written
  int* Un;       // entries of each row of U (with the diagonal), -1 until written
  unsigned* state;  // [0] ticket counter, [kTicketStride] exited waves
  unsigned* fault;  // set when a wait reached poll_limit
  int* flags;       // [0] smallest row with a zero or non-finite pivot (n: none), [1] table overflow
  int poll_limit;
  int tbits;         // working row: 1 << tbits slots
  const int* order;  // ticket -> row: every row after the rows it can depend on
};

__device__ __forceinline__ int ld_dev(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool is_marker(double v) {
  return (unsigned long long)__double_as_longlong(v) == kPending64;
}

__device__ __forceinline__ int wave_min(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ unsigned slot_of(int j, int tbits) { return ((unsigned)j * 2654435761u) >> (32 - tbits); }

// Slot of column j in the working row, or -1.
__device__ __forceinline__ int find(const int* keys, int j, int tbits) {
  const unsigned mask = (1u << tbits) - 1;
  unsigned s = slot_of(j, tbits);
  for (unsigned t = 0; t <= mask; ++t, s = (s + 1) & mask) {
    const int k = keys[s];
    if (k == j) return (int)s;
    if (k == -1) return -1;
  }
  return -1;
}

// Slot of column j, inserted with value 0 if absent; -1 when the table is
// full (*used counts the occupied slots).  Lanes insert distinct columns.
__device__ __forceinline__ int insert(int* keys, double* vals, int j, int tbits, int* used) {
  const unsigned mask = (1u << tbits) - 1;
  unsigned s = slot_of(j, tbits);
  for (unsigned t = 0; t <= mask; ++t, s = (s + 1) & mask) {
    const int k = keys[s];
    if (k == j) return (int)s;
    if (k == -1) {
      const int old = atomicCAS(&keys[s], -1, j);
      if (old == -1) {
        vals[s] = 0.0;
        atomicAdd(used, 1);
        return (int)s;
      }
      if (old == j) return (int)s;
    }
  }
  return -1;
}

// Rank key of rule 2: ascending order = magnitude (in single precision)
// descending, then column ascending.
__device__ __forceinline__ unsigned long long rank_key(double v, int j) {
  const float m = (float)fabs(v);
  const unsigned bits = __float_as_uint(m);
  return ((unsigned long long)(~bits) << 32) | (unsigned)j;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Whether slot s of the working row of row i holds a candidate of rule 2 in
// `part` (0 lower, 1 upper, 2 both) after rule 1.
__device__ __forceinline__ bool candidate(int j, double x, int i, double taui, int part) {
  if (j < 0 || j == i || x == 0.0 || fabs(x) < taui) return false;
  if (part == 0) return j < i;
  if (part == 1) return j > i;
  return true;
}

// The rank key K such that exactly `want` candidates of `part` have a key
// <= K (all of them when there are at most `want`): a radix select on the
// 64-bit key, 8 bits per pass from the top, over a 256-bin histogram in LDS;
// it stops at the first pass whose boundary bin holds exactly the entries
// still wanted (keys are unique, so the last pass always does).
__device__ __forceinline__ unsigned long long select_key(const int* keys, const double* vals, int* hist, int T,
                                                         int lane, int i, double taui, int part, int want,
                                                         int total) {
  if (total <= want) return ~0ull;
  if (want <= 0) return 0ull;  // no finite entry has the key 0
  unsigned long long prefix = 0;
  int remaining = want;
  for (int shift = 56;; shift -= 8) {
    for (int b = lane; b < 256; b += kWave) hist[b] = 0;
    __syncthreads();
    const unsigned long long himask = shift == 56 ? 0ull : (~0ull << (shift + 8));
    for (int s = lane; s < T; s += kWave) {
      const int j = keys[s];
      const double x = vals[s];
      if (!candidate(j, x, i, taui, part)) continue;
      const unsigned long long key = rank_key(x, j);
      if ((key & himask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
    }
    __syncthreads();
    int h[4], loc = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      h[q] = hist[4 * lane + q];
      loc += h[q];
    }
    const int incl = wave_incl_scan(loc, lane);
    // the lane whose bins hold the remaining-th entry
    int c = incl - loc, bsel = -1, before = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (bsel < 0 && c + h[q] >= remaining) {
        bsel = 4 * lane + q;
        before = c;
      }
      c += h[q];
    }
    const unsigned long long owner = __ballot(bsel >= 0 && incl - loc < remaining);
    const int src = __ffsll((long long)owner) - 1;
    const int b = __shfl(bsel, src), bef = __shfl(before, src);
    const int inb = hist[b];
    __syncthreads();
    prefix |= (unsigned long long)b << shift;
    remaining -= bef;
    if (inb == remaining || shift == 0) return prefix | (shift == 0 ? 0ull : ((1ull << shift) - 1));
  }
}

// U rows of up to kMaxChunks * 64 slots are fetched in one round of loads.
constexpr int kMaxChunks = 12;

// Row k of U (count, and slot c * 64 + lane in chunk c), waiting until the
// count and every slot below it are written; all loads of a round are in
// flight together.
__device__ __forceinline__ int fetch_u(const Args& A, int k, int nch, int lane, int (&uc)[kMaxChunks],
                                       double (&uv)[kMaxChunks], bool& gave_up) {
  const int64_t base = (int64_t)k * A.cu;
  int cnt = ld_dev(A.Un + k);
#pragma unroll
  for (int c = 0; c < kMaxChunks; ++c) {
    const int s = c * kWave + lane;
    const bool act = c < nch && s < A.cu;
    uc[c] = act ? ld_dev(A.Uc + base + s) : 0;
    uv[c] = act ? ld_dev(A.Uv + base + s) : 0.0;
  }
  for (int polls = 0;; ++polls) {
    const int lim = cnt >= 1 ? cnt : A.cu;
    bool miss = cnt < 1;
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int s = c * kWave + lane;
      miss |= c < nch && s < lim && (uc[c] == -1 || is_marker(uv[c]));
    }
    if (__ballot(miss) == 0) break;
    if (gave_up || polls >= A.poll_limit ||
        ((polls & 15) == 15 && ld_dev(reinterpret_cast<const int*>(A.fault)) != 0)) {
      gave_up = true;
      st_dev(A.fault, 1u);
      return cnt >= 1 ? cnt : 1;
    }
    __builtin_amdgcn_s_sleep(2);
    if (cnt < 1) cnt = ld_dev(A.Un + k);
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int s = c * kWave + lane;
      if (c < nch && s < A.cu && (uc[c] == -1 || is_marker(uv[c]))) {
        uc[c] = ld_dev(A.Uc + base + s);
        uv[c] = ld_dev(A.Uv + base + s);
      }
    }
  }
  return cnt;
}

__global__ __launch_bounds__(64) void ilut_rows(Args A) {
  // every product and difference rounded on its own, as on the host (hipcc
  // would otherwise fuse w_j - l_k u_kj into one FMA)
#pragma clang fp contract(off)
  extern __shared__ unsigned char lds[];
  const int T = 1 << A.tbits;
  int* keys = reinterpret_cast<int*>(lds);
  double* vals = reinterpret_cast<double*>(lds + sizeof(int) * T);
  int* hist = reinterpret_cast<int*>(lds + 12 * (size_t)T);  // 256 bins
  const int nch = (A.cu + kWave - 1) / kWave;
  __shared__ int used, nkl, nku;
  const int lane = threadIdx.x & 63;
  bool gave_up = false;
  for (;;) {
    const int tk = __builtin_amdgcn_readfirstlane((int)atomicAdd(A.state, lane == 0 ? 1u : 0u));
    if (tk >= A.n) break;
    const int i = A.order[tk];
    for (int s = lane; s < T; s += kWave) keys[s] = -1;
    if (lane == 0) used = 0;
    __syncthreads();
    // the row of P A P^T into the table; tau_i from the sum of |a_ij| in
    // column order (one lane adds them, in the host's order)
    const int64_t r0 = A.rp[i], r1 = A.rp[i + 1];
    double rs = 0.0;
    for (int64_t b = r0; b < r1; b += kWave) {
      const int64_t k = b + lane;
      const bool act = k < r1;
      const int j = act ? A.ci[k] : -1;
      const double a = act ? A.v[k] : 0.0;
      if (act) {
        const int s = insert(keys, vals, j, A.tbits, &used);
        if (s >= 0) vals[s] = a;
      }
      const int m = (int)(r1 - b < kWave ? r1 - b : kWave);
      for (int t = 0; t < m; ++t) {
        const double at = __shfl(a, t);
        rs = rs + fabs(at);
      }
    }
    __syncthreads();
    const int64_t nzi = r1 - r0;
    const double taui = nzi > 0 ? A.tau * (rs / (double)nzi) : 0.0;
    bool over = used > (7 * T) / 8;
    // elimination with the rows k < i, in increasing k
    int kprev = -1;
    while (!over) {
      int cand = 0x7fffffff;
      for (int s = lane; s < T; s += kWave) {
        const int j = keys[s];
        if (j > kprev && j < i && vals[s] != 0.0) cand = min(cand, j);
      }
      const int k = wave_min(cand);
      if (k == 0x7fffffff) break;
      kprev = k;
      const int sk = find(keys, k, A.tbits);
      const double wk = vals[sk];
      int uc[kMaxChunks];
      double uv[kMaxChunks];
      const int cntk = fetch_u(A, k, nch, lane, uc, uv, gave_up);
      // the diagonal first: the multiplier decides whether row k is used
      const double ukk = __shfl(uv[0], 0);
      const double lk = wk / ukk;
      __syncthreads();
      if (fabs(lk) < taui) {
        if (lane == 0) vals[sk] = 0.0;
        __syncthreads();
        continue;
      }
      if (lane == 0) vals[sk] = lk;
      __syncthreads();
#pragma unroll
      for (int c = 0; c < kMaxChunks; ++c) {
        if (c >= nch) break;
        const int s = c * kWave + lane;
        const int j = uc[c];
        if (s >= 1 && s < cntk && s < A.cu && j >= 0 && j < A.n) {
          const int t = insert(keys, vals, j, A.tbits, &used);
          if (t >= 0) {
            const double prod = lk * uv[c];
            vals[t] = vals[t] - prod;
          } else {
            atomicOr(&A.flags[1], 1);
          }
        }
        __syncthreads();
      }
      over = used > (7 * T) / 8;
    }
    if (over && lane == 0) atomicOr(&A.flags[1], 1);
    // pivot
    const int si = find(keys, i, A.tbits);
    const double d = si >= 0 ? vals[si] : 0.0;
    if (lane == 0 && (!(d != 0.0) || !isfinite(d))) atomicMin(&A.flags[0], i);
    // rule 1 on the final row, then rule 2
    int nlo = 0, nup = 0;
    for (int s = lane; s < T; s += kWave) {
      const int j = keys[s];
      if (j < 0 || j == i) continue;
      const double x = vals[s];
      if (x == 0.0 || fabs(x) < taui) continue;
      if (j < i) ++nlo; else ++nup;
    }
    nlo = wave_sum(nlo);
    nup = wave_sum(nup);
    unsigned long long kl, ku;
    if (A.mode == 1) {
      kl = ku = select_key(keys, vals, hist, T, lane, i, taui, 2, A.keep_l, nlo + nup);
    } else {
      kl = select_key(keys, vals, hist, T, lane, i, taui, 0, A.keep_l, nlo);
      ku = select_key(keys, vals, hist, T, lane, i, taui, 1, A.keep_u, nup);
    }
    // store the kept entries as they are found
    if (lane == 0) nkl = nku = 0;
    __syncthreads();
    const int64_t lb = (int64_t)i * A.cl, ub = (int64_t)i * A.cu;
    for (int s = lane; s < T; s += kWave) {
      const int j = keys[s];
      const double x = vals[s];
      if (!candidate(j, x, i, taui, 2)) continue;
      if (rank_key(x, j) > (j < i ? kl : ku)) continue;
      if (j < i) {
        const int q = atomicAdd(&nkl, 1);
        if (q < A.cl) {
          A.Lc[lb + q] = j;
          A.Lv[lb + q] = x;
        }
      } else {
        const int q = atomicAdd(&nku, 1);
        if (q + 1 < A.cu) {
          st_dev(A.Uc + ub + 1 + q, j);
          st_dev(A.Uv + ub + 1 + q, x);
        }
      }
    }
    __syncthreads();
    const int keepL = nkl < A.cl ? nkl : A.cl;
    const int keepU = nku < A.cu - 1 ? nku : A.cu - 1;
    if (lane == 0) {
      A.Ln[i] = keepL;
      st_dev(A.Uc + ub, i);
      // a value with the marker's bits would look unwritten: store a quiet NaN
      st_dev(A.Uv + ub, is_marker(d) ? __builtin_nan("") : d);
      st_dev(A.Un + i, keepU + 1);
    }
    __syncthreads();
  }
  // the last wave out clears the counters for the next launch
  unsigned* exited = A.state + kTicketStride;
  const unsigned prev = atomicAdd(exited, lane == 0 ? 1u : 0u);
  if ((unsigned)__builtin_amdgcn_readfirstlane((int)prev) == gridDim.x - 1 && lane == 0) {
    st_dev(A.state, 0u);
    st_dev(exited, 0u);
  }
}

}  // namespace ilut
}  // namespace pmg
