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
// by a running wave (the argument of the triangular solves).  The working
// row is an open-addressing hash table keyed by column, in LDS; a row that
// outgrows it (rows of the top separators collect tens of thousands of
// entries before rule 2 trims them) is factored again from the start in a
// larger table of its wave in global memory.  A row of U is published entry by entry with device-scope
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
  int* flags;       // [0] smallest row with a zero or non-finite pivot (n: none), [1] bit 0: table
                    // overflow, bit 1: a pivot missing from the working row (the host factors instead)
  int poll_limit;
  int tbits;         // working row in LDS: 1 << tbits slots
  int full;          // occupied slots beyond which that table overflows
  const int* order;  // ticket -> row: every row after the rows it can depend on
  // rows that outgrow the LDS table are factored again in a table of
  // 1 << gbits slots in global memory, one per wave (gbits 0: none)
  int* gkeys;        // gridDim.x << gbits
  double* gvals;
  int gbits;
  int gfull;
  unsigned long long* gbits0;  // gridDim.x * nw0 level-0 words of the lower-part bitmaps, zero
  int nw0;                     // ceil(n / 64); the level-1 words, ceil(n / 4096), fit the LDS table
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

// The working row is touched only by the wave that owns it, in LDS or in
// its own part of global memory.  Its accesses are relaxed atomics at
// workgroup scope (plain accesses on LDS); the inserting atomics
// (compare-and-swap of a key, OR into the pivot bitmap) are at agent scope,
// which includes the workgroup, and the workgroup barriers between the
// phases of a row order them all.
__device__ __forceinline__ int tk_ld(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void tk_st(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ double tv_ld(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void tv_st(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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
    const int k = tk_ld(keys + s);
    if (k == j) return (int)s;
    if (k == -1) return -1;
  }
  return -1;
}

// Slot of column j, inserted with value 0 if absent (then `fresh` is set);
// -1 when the table is full (*used counts the occupied slots).  Lanes insert
// distinct columns.
__device__ __forceinline__ int insert(int* keys, double* vals, int j, int tbits, int* used, bool& fresh) {
  const unsigned mask = (1u << tbits) - 1;
  unsigned s = slot_of(j, tbits);
  fresh = false;
  for (unsigned t = 0; t <= mask; ++t, s = (s + 1) & mask) {
    const int k = tk_ld(keys + s);
    if (k == j) return (int)s;
    if (k == -1) {
      const int old = atomicCAS(&keys[s], -1, j);
      if (old == -1) {
        tv_st(vals + s, 0.0);
        atomicAdd(used, 1);
        fresh = true;
        return (int)s;
      }
      if (old == j) return (int)s;
    }
  }
  return -1;
}

// w_j -= prod for column j: the entry is found, or inserted as 0 - prod as
// the host computes a new entry; the key and value of each probed slot are
// loaded together, so an existing entry costs one round trip.  Returns the
// slot, or -1 when the table is full; `fresh` as for insert.
__device__ __forceinline__ int subtract(int* keys, double* vals, int j, double prod, int tbits, int* used,
                                        bool& fresh) {
#pragma clang fp contract(off)
  const unsigned mask = (1u << tbits) - 1;
  unsigned s = slot_of(j, tbits);
  fresh = false;
  for (unsigned t = 0; t <= mask; ++t, s = (s + 1) & mask) {
    const int k = tk_ld(keys + s);
    const double v = tv_ld(vals + s);
    if (k == j) {
      tv_st(vals + s, v - prod);
      return (int)s;
    }
    if (k == -1) {
      const int old = atomicCAS(&keys[s], -1, j);
      if (old == -1) {
        const double zero = 0.0;
        tv_st(vals + s, zero - prod);
        atomicAdd(used, 1);
        fresh = true;
        return (int)s;
      }
      if (old == j) {
        tv_st(vals + s, tv_ld(vals + s) - prod);
        return (int)s;
      }
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

// Scans of the working row load this many slots per lane before using any.
constexpr int kScanBatch = 8;

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
    for (int s0 = 0; s0 < T; s0 += kScanBatch * kWave) {
      int jj[kScanBatch];
      double xx[kScanBatch];
#pragma unroll
      for (int u = 0; u < kScanBatch; ++u) {
        const int s = s0 + u * kWave + lane;
        jj[u] = s < T ? tk_ld(keys + s) : -1;
        xx[u] = s < T ? tv_ld(vals + s) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kScanBatch; ++u) {
        if (!candidate(jj[u], xx[u], i, taui, part)) continue;
        const unsigned long long key = rank_key(xx[u], jj[u]);
        if ((key & himask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1);
      }
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

// Columns of the strict lower part of a working row in global memory, as a
// two-level bitmap: bit j of the wave's level-0 words (global memory) and bit
// j / 64 of the level-1 words (in the LDS that the row's table would
// otherwise use).  Pivots are taken in increasing column order and fill only
// adds columns beyond the current pivot, so the next pivot is the first set
// bit past it: one level-0 word, or a scan of 64 level-1 words per round.
struct LowerBits {
  unsigned long long* l0;  // ceil(n / 64) words, zero between rows
  unsigned long long* l1;  // ceil(n / 4096) words, cleared at the start of a row
};

__device__ __forceinline__ unsigned long long bits_ld(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void mark_lower(const LowerBits& B, int j) {
  atomicOr(B.l0 + (j >> 6), 1ull << (j & 63));
  atomicOr(B.l1 + (j >> 12), 1ull << ((j >> 6) & 63));
}

// The smallest marked column in (kprev, i), or 0x7fffffff.
__device__ __forceinline__ int next_lower(const LowerBits& B, int kprev, int i, int lane) {
  const int c = kprev + 1;
  if (c >= i) return 0x7fffffff;
  const int w = c >> 6;
  unsigned long long bits = bits_ld(B.l0 + w) & (~0ull << (c & 63));
  int word = w;
  if (bits == 0) {
    word = -1;
    const int last = (i - 1) >> 6;  // last level-0 word that can hold a lower column
    for (int q = w + 1; q <= last;) {
      const int b1 = q >> 6;
      const int wi = b1 + lane;
      unsigned long long m = wi <= (last >> 6) ? bits_ld(B.l1 + wi) : 0ull;
      if (lane == 0) m &= ~0ull << (q & 63);
      const unsigned long long any = __ballot(m != 0ull);
      if (any) {
        const int l = __ffsll((long long)any) - 1;
        const unsigned long long ml = __shfl(m, l);
        word = ((b1 + l) << 6) + __ffsll((long long)ml) - 1;
        break;
      }
      q = (b1 + kWave) << 6;
    }
    if (word < 0) return 0x7fffffff;
    bits = bits_ld(B.l0 + word);
  }
  const int k = (word << 6) + __ffsll((long long)bits) - 1;
  return k < i ? k : 0x7fffffff;
}

// Clears the level-0 words a row marked, then its level-1 words.
__device__ __forceinline__ void clear_lower(const LowerBits& B, int i, int lane) {
  const int n1 = i > 0 ? ((i - 1) >> 12) + 1 : 0;
  for (int wi = lane; wi < n1; wi += kWave) {
    unsigned long long m = bits_ld(B.l1 + wi);
    while (m) {
      const int b = __ffsll((long long)m) - 1;
      __hip_atomic_store(B.l0 + (wi << 6) + b, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      m &= m - 1;
    }
    __hip_atomic_store(B.l1 + wi, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Row i with the working row in `keys`/`vals` (1 << tbits slots, counted
// full beyond `full`; in LDS or in the wave's global table, only this wave
// touches it).  sh: used, kept in L, kept in U, insert failed (LDS).  Returns
// false, having published nothing, when the row outgrew the table and `last`
// is false (the caller factors it again in a larger table); with `last` true
// an overflow is flagged for the host, which factors everything again with
// larger tables, and a truncated row is published so that no wave waits
// forever on it.
// GLOBAL: the table is the wave's in global memory and the pivots are found
// through the bitmaps B; otherwise (LDS) by a scan of the table.
template <bool GLOBAL>
__device__ __forceinline__ bool factor_row(const Args& A, int i, int* keys, double* vals, int tbits,
                                           int full, int* hist, int* sh, int lane, int nch, bool& gave_up, bool last,
                                           const LowerBits& B) {
  // every product and difference rounded on its own, as on the host (hipcc
  // would otherwise fuse w_j - l_k u_kj into one FMA)
#pragma clang fp contract(off)
  const int T = 1 << tbits;
  for (int s = lane; s < T; s += kWave) tk_st(keys + s, -1);
  if (GLOBAL) {
    const int n1 = i > 0 ? ((i - 1) >> 12) + 1 : 0;
    for (int wi = lane; wi < n1; wi += kWave) B.l1[wi] = 0ull;
  }
  if (lane == 0) sh[0] = sh[3] = 0;
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
      bool fresh;
      const int s = insert(keys, vals, j, tbits, &sh[0], fresh);
      if (s >= 0) tv_st(vals + s, a);
      else sh[3] = 1;
      if (GLOBAL && fresh && j < i) mark_lower(B, j);
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
  bool over = sh[0] > full || sh[3] != 0;
  if (over && !last) return false;  // (LDS only: the global table is the last resort)
  // elimination with the rows k < i, in increasing k
  int kprev = -1;
  while (!over) {
    int k;
    if (GLOBAL) {
      k = next_lower(B, kprev, i, lane);
    } else {
      int cand = 0x7fffffff;
      for (int s = lane; s < T; s += kWave) {
        const int j = tk_ld(keys + s);
        if (j > kprev && j < i && tv_ld(vals + s) != 0.0) cand = min(cand, j);
      }
      k = wave_min(cand);
    }
    if (k == 0x7fffffff) break;
    kprev = k;
    // the first probe for w_k travels with the loads of row k of U
    const unsigned s0 = slot_of(k, tbits);
    const int k0 = tk_ld(keys + s0);
    const double v0 = tv_ld(vals + s0);
    int uc[kMaxChunks];
    double uv[kMaxChunks];
    const int cntk = fetch_u(A, k, nch, lane, uc, uv, gave_up);
    int sk = (int)s0;
    double wk = v0;
    if (k0 != k) {
      sk = find(keys, k, tbits);
      if (sk < 0) {
        if (lane == 0) atomicOr(&A.flags[1], 2);
        break;
      }
      wk = tv_ld(vals + sk);
    }
    if (GLOBAL && wk == 0.0) continue;  // the scan skips these
    // the diagonal first: the multiplier decides whether row k is used
    const double ukk = __shfl(uv[0], 0);
    const double lk = wk / ukk;
    __syncthreads();
    if (fabs(lk) < taui) {
      if (lane == 0) tv_st(vals + sk, 0.0);
      __syncthreads();
      continue;
    }
    if (lane == 0) tv_st(vals + sk, lk);
    __syncthreads();
    // w -= l_k (row k of U): the columns of row k are distinct, so all its
    // slots are updated together; the first probe of every slot is loaded
    // before any is used
    int pk[kMaxChunks];
    double pv[kMaxChunks];
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int s = c * kWave + lane;
      const int j = uc[c];
      const bool act = c < nch && s >= 1 && s < cntk && s < A.cu && j >= 0 && j < A.n;
      uc[c] = act ? j : -1;
      const unsigned q = act ? slot_of(j, tbits) : 0u;
      pk[c] = act ? tk_ld(keys + q) : -2;
      pv[c] = act ? tv_ld(vals + q) : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kMaxChunks; ++c) {
      const int j = uc[c];
      if (j < 0) continue;
      const double prod = lk * uv[c];
      if (pk[c] == j) {
        tv_st(vals + slot_of(j, tbits), pv[c] - prod);
        continue;
      }
      bool fresh;
      const int t = subtract(keys, vals, j, prod, tbits, &sh[0], fresh);
      if (t < 0) sh[3] = 1;
      if (GLOBAL && fresh && j < i) mark_lower(B, j);
    }
    __syncthreads();
    over = sh[0] > full || sh[3] != 0;
    if (over && !last) return false;
  }
  if (over && lane == 0) atomicOr(&A.flags[1], 1);
  if (GLOBAL) {
    __syncthreads();
    clear_lower(B, i, lane);
  }
  // pivot
  const int si = find(keys, i, tbits);
  const double d = si >= 0 ? tv_ld(vals + si) : 0.0;
  if (lane == 0 && (!(d != 0.0) || !isfinite(d))) atomicMin(&A.flags[0], i);
  // rule 1 on the final row: the candidates of rule 2 counted by part; in
  // the global table they are also moved to its front (in place: a round's
  // slots are all loaded before any is written, and the front never passes
  // the slots already loaded), so the passes of rule 2 read only them
  int nlo = 0, nup = 0, Tc = T;
  {
    int base = 0;
    for (int s0 = 0; s0 < T; s0 += kScanBatch * kWave) {
      int jj[kScanBatch];
      double xx[kScanBatch];
#pragma unroll
      for (int u = 0; u < kScanBatch; ++u) {
        const int s = s0 + u * kWave + lane;
        jj[u] = s < T ? tk_ld(keys + s) : -1;
        xx[u] = s < T ? tv_ld(vals + s) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kScanBatch; ++u) {
        const bool c = candidate(jj[u], xx[u], i, taui, 2);
        if (c) {
          if (jj[u] < i) ++nlo; else ++nup;
        }
        if (GLOBAL) {
          const unsigned long long m = __ballot(c);
          if (c) {
            const int pos = base + __popcll(m & ((1ull << lane) - 1));
            tk_st(keys + pos, jj[u]);
            tv_st(vals + pos, xx[u]);
          }
          base += __popcll(m);
        }
      }
    }
    if (GLOBAL) Tc = base;
  }
  nlo = wave_sum(nlo);
  nup = wave_sum(nup);
  __syncthreads();
  unsigned long long kl, ku;
  if (A.mode == 1) {
    kl = ku = select_key(keys, vals, hist, Tc, lane, i, taui, 2, A.keep_l, nlo + nup);
  } else {
    kl = select_key(keys, vals, hist, Tc, lane, i, taui, 0, A.keep_l, nlo);
    ku = select_key(keys, vals, hist, Tc, lane, i, taui, 1, A.keep_u, nup);
  }
  // store the kept entries as they are found
  if (lane == 0) sh[1] = sh[2] = 0;
  __syncthreads();
  const int64_t lb = (int64_t)i * A.cl, ub = (int64_t)i * A.cu;
  for (int s0 = 0; s0 < Tc; s0 += kScanBatch * kWave) {
    int jj[kScanBatch];
    double xx[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      const int s = s0 + u * kWave + lane;
      jj[u] = s < Tc ? tk_ld(keys + s) : -1;
      xx[u] = s < Tc ? tv_ld(vals + s) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      const int j = jj[u];
      const double x = xx[u];
      if (!candidate(j, x, i, taui, 2)) continue;
      if (rank_key(x, j) > (j < i ? kl : ku)) continue;
      if (j < i) {
        const int q = atomicAdd(&sh[1], 1);
        if (q < A.cl) {
          A.Lc[lb + q] = j;
          A.Lv[lb + q] = x;
        }
      } else {
        const int q = atomicAdd(&sh[2], 1);
        if (q + 1 < A.cu) {
          st_dev(A.Uc + ub + 1 + q, j);
          st_dev(A.Uv + ub + 1 + q, x);
        }
      }
    }
  }
  __syncthreads();
  const int keepL = sh[1] < A.cl ? sh[1] : A.cl;
  const int keepU = sh[2] < A.cu - 1 ? sh[2] : A.cu - 1;
  if (lane == 0) {
    A.Ln[i] = keepL;
    st_dev(A.Uc + ub, i);
    // a value with the marker's bits would look unwritten: store a quiet NaN
    st_dev(A.Uv + ub, is_marker(d) ? __builtin_nan("") : d);
    st_dev(A.Un + i, keepU + 1);
  }
  __syncthreads();
  return true;
}

__global__ __launch_bounds__(64) void ilut_rows(Args A) {
  extern __shared__ unsigned char lds[];
  const int T = 1 << A.tbits;
  int* keys = reinterpret_cast<int*>(lds);
  double* vals = reinterpret_cast<double*>(lds + sizeof(int) * T);
  int* hist = reinterpret_cast<int*>(lds + 12 * (size_t)T);  // 256 bins
  const int nch = (A.cu + kWave - 1) / kWave;
  __shared__ int sh[4];
  const int lane = threadIdx.x & 63;
  int* gk = A.gbits ? A.gkeys + ((size_t)blockIdx.x << A.gbits) : nullptr;
  double* gv = A.gbits ? A.gvals + ((size_t)blockIdx.x << A.gbits) : nullptr;
  const LowerBits B{A.gbits ? A.gbits0 + (size_t)blockIdx.x * (size_t)A.nw0 : nullptr,
                    reinterpret_cast<unsigned long long*>(lds)};
  bool gave_up = false;
  for (;;) {
    const int tk = __builtin_amdgcn_readfirstlane((int)atomicAdd(A.state, lane == 0 ? 1u : 0u));
    if (tk >= A.n) break;
    const int i = A.order[tk];
    if (!factor_row<false>(A, i, keys, vals, A.tbits, A.full, hist, sh, lane, nch, gave_up, A.gbits == 0, B))
      factor_row<true>(A, i, gk, gv, A.gbits, A.gfull, hist, sh, lane, nch, gave_up, true, B);
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
