// HIP kernels of the p-multigrid solve phase, written for gfx950 (CDNA4,
// wave64).  Everything here is sparse and bandwidth- or latency-bound; no
// matrix cores are involved.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmg {

constexpr int kWave = 64;

enum CsrMode : int {
  kResid = 0,     // out = b - A x, block partial of sum(out^2)
  kPlain = 1,     // out = A x
  kScale = 2,     // out = d .* (A x)
  kScaleAdd = 3,  // out += d .* (A x)
  kAdd = 4,       // out += A x
  kGS = 5         // rows from a list: out_i = (b_i - sum_{j != i} a_ij out_j) / a_ii
};

template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// CSR kernel with G lanes per row (G divides 64), 256 threads per block,
// grid-stride over row groups (the grid is capped, so a residual produces at
// most one partial sum per block).  Consecutive lanes of a group read
// consecutive non-zeros (coalesced); x is gathered through the caches.  Row
// sums are reduced in a fixed tree, so results are bit-reproducible.
template <typename T, int G, int MODE>
__global__ __launch_bounds__(256) void csr_kernel(int nrows, const int* __restrict__ rows,
                                                  const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const T* __restrict__ v, const T* x,
                                                  const T* __restrict__ b, const T* __restrict__ d, T* out,
                                                  double* __restrict__ partial) {
  const int tid = threadIdx.x;
  const int g = tid / G, l = tid % G;
  const int rpb = 256 / G;
  double sq = 0.0;
  for (int idx = blockIdx.x * rpb + g; idx < nrows; idx += gridDim.x * rpb) {
    const int row = rows ? rows[idx] : idx;
    const int k0 = rp[row], k1 = rp[row + 1];
    T acc = 0, diag = 0;
    for (int k = k0 + l; k < k1; k += G) {
      const int c = ci[k];
      const T a = v[k];
      if (MODE == kGS) {
        if (c == row) {
          diag = a;
          continue;
        }
        acc += a * out[c];
      } else {
        acc += a * x[c];
      }
    }
    acc = group_sum(acc, G);
    if (MODE == kGS) diag = group_sum(diag, G);
    if (l == 0) {
      if (MODE == kResid) {
        const T res = b[row] - acc;
        out[row] = res;
        sq += (double)res * (double)res;
      } else if (MODE == kPlain) {
        out[row] = acc;
      } else if (MODE == kScale) {
        out[row] = d[row] * acc;
      } else if (MODE == kScaleAdd) {
        out[row] = out[row] + d[row] * acc;
      } else if (MODE == kAdd) {
        out[row] = out[row] + acc;
      } else if (MODE == kGS) {
        out[row] = (b[row] - acc) / diag;
      }
    }
  }
  if (MODE == kResid) {
    __shared__ double red[256];
    red[tid] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = red[0];
  }
}

// Sums n block partials in a fixed order into out[0] (one block).
__global__ __launch_bounds__(256) void reduce_partials(int n, const double* __restrict__ partial,
                                                       double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

template <typename T>
__global__ void fill_kernel(int64_t n, T* __restrict__ y, T val) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = val;
}

template <typename TI, typename TO>
__global__ void cast_kernel(int64_t n, const TI* __restrict__ x, TO* __restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (TO)x[i];
}

// y += (double) c
template <typename TI>
__global__ void add_cast_kernel(int64_t n, const TI* __restrict__ c, double* __restrict__ y) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += (double)c[i];
}

// e = Ainv b for the coarsest degree-1 level (dense, row-major, n <= 1024),
// one block; threads own rows.
__global__ __launch_bounds__(256) void dense_matvec(int n, const double* __restrict__ Ainv,
                                                    const double* __restrict__ b, double* __restrict__ e) {
  __shared__ double bs[1024];
  for (int i = threadIdx.x; i < n; i += 256) bs[i] = b[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    const double* a = Ainv + (size_t)i * n;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += a[j] * bs[j];
    e[i] = s;
  }
}

// ---------------------------------------------------------------------------
// Sparse triangular solves with the ILUT factors (Section 3, "Smoother").
//
// Rows are grouped in segments (grid lines of the tensor numbering, seg_len
// consecutive rows).  One wave owns one segment and walks it in chunks of 64
// rows, lane = row.  Waves take segments in increasing dependency order
// through an atomic ticket, so a wave only ever waits for segments already
// owned by running waves (no deadlock, whatever the launch order).  Each
// segment publishes how many of its rows are final in prog[segment].  Before
// a chunk, the wave waits until every segment it reads from has progressed
// far enough (precomputed (segment, rows needed) pairs per chunk), then each
// lane accumulates its row's products with rows outside the chunk in
// parallel, and the rows inside the chunk are finished in order, the newest
// value broadcast from its lane.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Values of y published by other waves are read and written with device-scope
// (agent) atomic accesses: a wave may read part of a cache line of another
// segment while the rest of that line is not final yet, and a plain load
// could later hit that stale copy in this XCD's L2.
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wave_ticket(unsigned* ticket) {
  int t = 0;
  if ((threadIdx.x & 63) == 0) t = (int)atomicAdd(ticket, 1u);
  return __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
}

__device__ __forceinline__ void wait_chunk(const int* __restrict__ wptr, const int2* __restrict__ waits,
                                           int chunk, int lane, int* prog) {
  const int w0 = wptr[chunk], w1 = wptr[chunk + 1];
  for (int w = w0 + lane; w < w1; w += kWave) {
    const int2 pr = waits[w];
    while (__hip_atomic_load(prog + pr.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < pr.y)
      __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void publish(int* prog, int seg, int val, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (lane == 0) __hip_atomic_store(prog + seg, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every wave once its segment is final.  The last wave to finish
// clears the progress counters and the ticket for the next launch (all other
// waves are past their last read of them), so a solve needs no separate
// reset launch.  state[0] = ticket, state[1] = finished waves.
__device__ __forceinline__ void finish_segment(int nseg, int* prog, unsigned* state, int lane) {
  unsigned prev = 0;
  if (lane == 0) prev = atomicAdd(state + 1, 1u);
  prev = __builtin_amdgcn_readfirstlane(__shfl((int)prev, 0, 64));
  if (prev == (unsigned)(nseg - 1)) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int i = lane; i < nseg; i += kWave) st_dev(prog + i, 0);
    if (lane == 0) {
      st_dev(state, 0u);
      st_dev(state + 1, 0u);
    }
  }
}

// Off-chunk part of a row: t -= sum_{k in [k0, k1)} v[k] y[ci[k]], in k order,
// with the loads issued in batches of 8 so that they are in flight together.
template <typename T>
__device__ __forceinline__ T gather_sub(T t, int k0, int k1, const int* __restrict__ ci,
                                        const T* __restrict__ v, const T* y) {
  int k = k0;
  for (; k + 8 <= k1; k += 8) {
    int c[8];
    T a[8], yy[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      c[u] = ci[k + u];
      a[u] = v[k + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) yy[u] = ld_dev(y + c[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) t -= a[u] * yy[u];
  }
  for (; k < k1; ++k) t -= v[k] * ld_dev(y + ci[k]);
  return t;
}

// y = L^{-1} P r, L unit lower (strict part stored, sorted columns), P the
// ILUT ordering ((P r)_i = r[perm[i]]).  ks[row]
// is the first entry of the row whose column lies in the row's own chunk.
// The in-chunk entries are staged in a dense 64 x 64 LDS tile (source row j,
// target lane) before the wait, so the ordered part touches no global memory.
template <typename T>
__global__ __launch_bounds__(64) void trisolve_lower(int nseg, int seg_len, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const T* __restrict__ v,
                                                     const int* __restrict__ ks,
                                                     const int* __restrict__ perm, const T* __restrict__ r,
                                                     T* y, const int* __restrict__ wptr,
                                                     const int2* __restrict__ waits, int* prog,
                                                     unsigned* ticket) {
  __shared__ T tile[kWave * kWave];
  const int lane = threadIdx.x & 63;
  const int s = wave_ticket(ticket);
  if (s >= nseg) return;
  const int seg0 = s * seg_len;
  const int nch = (seg_len + kWave - 1) / kWave;
  for (int c = 0; c < nch; ++c) {
    const int r0 = seg0 + c * kWave;
    const int nrow = min(kWave, seg_len - c * kWave);
    const int row = r0 + lane;
    const bool act = lane < nrow;
#pragma unroll 8
    for (int j = 0; j < kWave; ++j) tile[j * kWave + lane] = 0;
    int k0 = 0, k1 = 0, kin = 0;
    T t = 0;
    if (act) {
      k0 = rp[row];
      k1 = rp[row + 1];
      kin = ks[row];
      t = r[perm[row]];
      for (int k = kin; k < k1; ++k) tile[(ci[k] - r0) * kWave + lane] = v[k];
    }
    wait_chunk(wptr, waits, s * nch + c, lane, prog);
    if (act) t = gather_sub(t, k0, kin, ci, v, y);
    // rows inside the chunk, in order
    for (int j = 0; j < nrow - 1; ++j) {
      const T yj = lane_bcast(t, j);
      t -= tile[j * kWave + lane] * yj;
    }
    if (act) st_dev(y + row, t);
    publish(prog, s, c * kWave + nrow, lane);
  }
  finish_segment(nseg, prog, ticket, lane);
}

// e = U^{-1} y (diagonal first in each row, then the strict upper part
// sorted), written over y, and x += P^T e.  ks[row] is the first entry whose
// column lies beyond the row's own chunk.
template <typename T>
__global__ __launch_bounds__(64) void trisolve_upper(int nseg, int seg_len, const int* __restrict__ rp,
                                                     const int* __restrict__ ci, const T* __restrict__ v,
                                                     const int* __restrict__ ks,
                                                     const int* __restrict__ perm, T* y, T* __restrict__ x,
                                                     const int* __restrict__ wptr,
                                                     const int2* __restrict__ waits, int* prog,
                                                     unsigned* ticket) {
  __shared__ T tile[kWave * kWave];
  const int lane = threadIdx.x & 63;
  const int sr = wave_ticket(ticket);
  if (sr >= nseg) return;
  const int s = nseg - 1 - sr;
  const int seg0 = s * seg_len;
  const int nch = (seg_len + kWave - 1) / kWave;
  int done = 0;
  for (int c = nch - 1; c >= 0; --c) {
    const int r0 = seg0 + c * kWave;
    const int nrow = min(kWave, seg_len - c * kWave);
    const int row = r0 + lane;
    const bool act = lane < nrow;
#pragma unroll 8
    for (int j = 0; j < kWave; ++j) tile[j * kWave + lane] = 0;
    T t = 0, dg = 1;
    int kout = 0, k1 = 0;
    if (act) {
      const int k0 = rp[row];
      k1 = rp[row + 1];
      kout = ks[row];
      t = y[row];
      dg = v[k0];
      for (int k = k0 + 1; k < kout; ++k) tile[(ci[k] - r0) * kWave + lane] = v[k];
    }
    wait_chunk(wptr, waits, sr * nch + (nch - 1 - c), lane, prog);
    if (act) t = gather_sub(t, kout, k1, ci, v, y);
    // rows inside the chunk, last to first
    T e = 0;
    for (int j = nrow - 1; j >= 0; --j) {
      if (lane == j) e = t / dg;
      const T ej = lane_bcast(e, j);
      t -= tile[j * kWave + lane] * ej;
    }
    if (act) {
      st_dev(y + row, e);
      x[perm[row]] += e;
    }
    done += nrow;
    publish(prog, s, done, lane);
  }
  finish_segment(nseg, prog, ticket, lane);
}

}  // namespace pmg
