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
// One wave factors one row at a time; rows are drawn in increasing order from
// a ticket counter, so the smallest unfinished row only waits for finished
// rows and is held by a running wave (the argument of the triangular
// solves).  The working row lives in LDS as an open-addressing hash table
// keyed by column.  A row of U is published entry by entry with device-scope
// stores into slots that hold a marker until written (column -1, value the
// signalling-NaN marker, count -1): a wave waiting for row k reloads the
// count and the entries it needs until no marker is left, so readiness
// travels with the data and no fence is needed.  Waits are bounded as in the
// triangular solves (poll_limit, fault word).
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
  int tbits;     // working row: 1 << tbits slots
  int list_cap;  // kept entries staged per row (>= cl + cu)
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

// The smallest key K with count(key <= K) >= want over the candidates of
// this lane's slots (part: 0 lower, 1 upper, 2 both), by bisection on the
// 64-bit key; all candidates are kept when there are at most `want`.
__device__ __forceinline__ unsigned long long kth_key(const int* keys, const double* vals, int T, int lane, int i,
                                                      double taui, int part, int want, int total) {
  if (total <= want) return ~0ull;
  unsigned long long lo = 0, hi = ~0ull;  // invariant: count(<= hi) >= want
  while (lo < hi) {
    const unsigned long long mid = lo + (hi - lo) / 2;
    int c = 0;
    for (int s = lane; s < T; s += kWave) {
      const int j = keys[s];
      if (j < 0 || j == i) continue;
      const double x = vals[s];
      if (x == 0.0 || fabs(x) < taui) continue;
      if (part == 0 && j > i) continue;
      if (part == 1 && j < i) continue;
      c += rank_key(x, j) <= mid ? 1 : 0;
    }
    c = wave_sum(c);
    if (c >= want) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Waits (bounded) until *p is not `bad` for the lanes with `need`, reloading
// with device-scope loads; returns the value.  A wave that gives up marks the
// fault word and every later wait of any wave returns at once.
template <typename T>
__device__ __forceinline__ T wait_value(const T* p, bool need, const Args& A, bool& gave_up) {
  T val = need ? ld_dev(p) : T(0);
  int polls = 0;
  for (;;) {
    bool miss;
    if constexpr (sizeof(T) == 8) miss = need && is_marker(val);
    else miss = need && val == T(-1);
    if (__ballot(miss) == 0) break;
    if (gave_up || polls >= A.poll_limit || ld_dev(reinterpret_cast<const int*>(A.fault)) != 0) {
      gave_up = true;
      st_dev(A.fault, 1u);
      break;
    }
    ++polls;
    __builtin_amdgcn_s_sleep(2);
    if (miss) val = ld_dev(p);
  }
  return val;
}

__global__ __launch_bounds__(64) void ilut_rows(Args A) {
  // every product and difference rounded on its own, as on the host (hipcc
  // would otherwise fuse w_j - l_k u_kj into one FMA)
#pragma clang fp contract(off)
  extern __shared__ unsigned char lds[];
  const int T = 1 << A.tbits;
  int* keys = reinterpret_cast<int*>(lds);
  double* vals = reinterpret_cast<double*>(lds + sizeof(int) * T);
  int* kc = reinterpret_cast<int*>(lds + 12 * (size_t)T);                       // kept columns
  double* kv = reinterpret_cast<double*>(lds + 12 * (size_t)T + 4 * (size_t)A.list_cap);  // kept values
  __shared__ int used, nkept;
  const int lane = threadIdx.x & 63;
  bool gave_up = false;
  for (;;) {
    const int i = __builtin_amdgcn_readfirstlane((int)atomicAdd(A.state, lane == 0 ? 1u : 0u));
    if (i >= A.n) break;
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
    bool over = used > (3 * T) / 4;
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
      const int cnt = wait_value(A.Un + k, true, A, gave_up);
      const int cntk = gave_up && cnt < 1 ? 1 : cnt;
      const int64_t base = (int64_t)k * A.cu;
      // the diagonal first: the multiplier decides whether row k is used
      const double ukk = __shfl(wait_value(A.Uv + base, lane == 0, A, gave_up), 0);
      const double lk = wk / ukk;
      __syncthreads();
      if (fabs(lk) < taui) {
        if (lane == 0) vals[sk] = 0.0;
        __syncthreads();
        continue;
      }
      if (lane == 0) vals[sk] = lk;
      __syncthreads();
      for (int b = 1; b < cntk; b += kWave) {
        const int s = b + lane;
        const bool act = s < cntk && s < A.cu;
        const int j = wait_value(A.Uc + base + (act ? s : 0), act, A, gave_up);
        const double u = wait_value(A.Uv + base + (act ? s : 0), act, A, gave_up);
        if (act && j >= 0 && j < A.n) {
          const int t = insert(keys, vals, j, A.tbits, &used);
          if (t >= 0) {
            const double prod = lk * u;
            vals[t] = vals[t] - prod;
          }
          else atomicOr(&A.flags[1], 1);
        }
        __syncthreads();
      }
      over = used > (3 * T) / 4;
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
    int keepL, keepU;
    if (A.mode == 1) {
      kl = ku = kth_key(keys, vals, T, lane, i, taui, 2, A.keep_l, nlo + nup);
      keepL = keepU = -1;  // counted below
    } else {
      kl = kth_key(keys, vals, T, lane, i, taui, 0, A.keep_l, nlo);
      ku = kth_key(keys, vals, T, lane, i, taui, 1, A.keep_u, nup);
      keepL = nlo < A.keep_l ? nlo : A.keep_l;
      keepU = nup < A.keep_u ? nup : A.keep_u;
    }
    // stage the kept entries (lower first, upper after), unordered
    if (lane == 0) nkept = 0;
    __syncthreads();
    for (int s = lane; s < T; s += kWave) {
      const int j = keys[s];
      if (j < 0 || j == i) continue;
      const double x = vals[s];
      if (x == 0.0 || fabs(x) < taui) continue;
      const unsigned long long key = rank_key(x, j);
      if (key <= (j < i ? kl : ku)) {
        const int q = atomicAdd(&nkept, 1);
        if (q < A.list_cap) {
          kc[q] = j;
          kv[q] = x;
        }
      }
    }
    __syncthreads();
    const int nk = nkept < A.list_cap ? nkept : A.list_cap;
    if (A.mode == 1) {
      int c = 0;
      for (int q = lane; q < nk; q += kWave) c += kc[q] < i ? 1 : 0;
      keepL = wave_sum(c);
      keepU = nk - keepL;
    }
    // each kept entry's place: the kept entries of its part with a smaller column
    const int64_t lb = (int64_t)i * A.cl, ub = (int64_t)i * A.cu;
    for (int q = lane; q < nk; q += kWave) {
      const int j = kc[q];
      int pos = 0;
      for (int t = 0; t < nk; ++t) {
        const int jt = kc[t];
        pos += ((jt < i) == (j < i) && jt < j) ? 1 : 0;
      }
      if (j < i) {
        if (pos < A.cl) {
          A.Lc[lb + pos] = j;
          A.Lv[lb + pos] = kv[q];
        }
      } else if (pos + 1 < A.cu) {
        st_dev(A.Uc + ub + 1 + pos, j);
        st_dev(A.Uv + ub + 1 + pos, kv[q]);
      }
    }
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
