// HIP kernels of the p-multigrid solve phase, written for gfx950 (CDNA4,
// wave64).  Everything here is sparse and bandwidth- or latency-bound; no
// matrix cores are involved.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tri_layout.hpp"
#include "grid_layout.hpp"

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

// Rows of the residual kernels per thread: RB (1 or kResidRows) consecutive
// rows in y of one grid column (ix, iz), so a line of x is loaded once for
// all of them (2p + RB lines instead of (2p + 1) RB); the lanes of a wave
// hold consecutive ix, so every load and store is contiguous across the wave.
constexpr int kResidRows = 4;

__host__ __device__ inline int resid_threads(int n, int nx, int ny, int rb) {
  return nx * ((ny + rb - 1) / rb) * (n / (nx * ny));
}

// Block partials of sum(r^2) for the residual kernels (threads' sums in
// order, then a tree over the block).
__device__ __forceinline__ void resid_partial(double sq, double* partial) {
  __shared__ double red[256];
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Residual r = b - A x (PLAIN: r = A x) with A in stencil layout.  With the tensor-product
// B-spline basis of degree p, row i (grid position (ix, iy, iz), x fastest,
// nx * ny per plane) couples only to the rows at offsets |dx|, |dy|, |dz| <=
// p; the value of offset k of row i is V[k * n + i] (k lexicographic in
// (dz, dy, dx), 0 where the offset leaves the grid), so no column indices
// are stored and both V and x are read contiguously across a wave's rows.
// Each row's sum runs over dz, dy, dx ascending, whatever line of x is
// loaded first; a thread takes RB rows (resid_threads threads).
// WX > 0: the stencil width 2 p + 1 known at compile time, so the offsets of
// a stencil row are unrolled and all their loads issued together (offsets
// outside the grid read offset 0 with weight 0, which adds an exact zero).
template <typename T, int DIM, bool PLAIN, int WX, int RB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 4))) void stencil_resid(int n, int nx, int ny, int p, const T* __restrict__ V,
                                                     const T* __restrict__ x, const T* __restrict__ b,
                                                     T* __restrict__ r, double* __restrict__ partial) {
  const int w = 2 * p + 1;
  const int nz = DIM == 3 ? n / (nx * ny) : 1;
  const int nyb = (ny + RB - 1) / RB, nt = nx * nyb * nz;
  double sq = 0.0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nt; t += gridDim.x * 256) {
    const int ix = t % nx, u = t / nx, iy0 = (u % nyb) * RB, iz = u / nyb;
    const int nr = min(RB, ny - iy0);
    const int dx0 = max(-p, -ix), dx1 = min(p, nx - 1 - ix);
    const int dz0 = DIM == 3 ? max(-p, -iz) : 0, dz1 = DIM == 3 ? min(p, nz - 1 - iz) : 0;
    const int i0 = (iz * ny + iy0) * nx + ix;  // row (ix, iy0, iz)
    const int y0 = max(0, iy0 - p), y1 = min(ny - 1, iy0 + nr - 1 + p);
    T acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = 0;
    for (int dz = dz0; dz <= dz1; ++dz)
      for (int y = y0; y <= y1; ++y) {
        const T* xr = x + ((iz + dz) * ny + y) * nx + ix;
        if constexpr (WX > 0) {
          T xx[WX];
#pragma unroll
          for (int k = 0; k < WX; ++k) {
            const int dx = k - WX / 2;
            xx[k] = xr[dx >= dx0 && dx <= dx1 ? dx : 0];
          }
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const int dy = y - iy0 - q;
            if (q < nr && dy >= -p && dy <= p) {
              const int k0 = ((DIM == 3 ? (dz + p) * w : 0) + (dy + p)) * w + p;  // offset index of dx = 0
              const T* vr = V + (size_t)k0 * n + i0 + q * nx;
              T vv[WX];
#pragma unroll
              for (int k = 0; k < WX; ++k) {
                const int dx = k - WX / 2;
                vv[k] = vr[(int64_t)(dx >= dx0 && dx <= dx1 ? dx : 0) * n];
              }
#pragma unroll
              for (int k = 0; k < WX; ++k) {
                const int dx = k - WX / 2;
                acc[q] += (dx >= dx0 && dx <= dx1 ? vv[k] : (T)0) * xx[k];
              }
            }
          }
        } else {
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const int dy = y - iy0 - q;
            if (q < nr && dy >= -p && dy <= p) {
              const int k0 = ((DIM == 3 ? (dz + p) * w : 0) + (dy + p)) * w + p;
              const T* vr = V + (size_t)k0 * n + i0 + q * nx;
              for (int dx = dx0; dx <= dx1; ++dx) acc[q] += vr[(int64_t)dx * n] * xr[dx];
            }
          }
        }
      }
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) {
        const int i = i0 + q * nx;
        const T res = PLAIN ? acc[q] : b[i] - acc[q];  // PLAIN: r = A x
        r[i] = res;
        sq += (double)res * (double)res;
      }
  }
  resid_partial(sq, partial);
}

// Coefficient of A = sum over directions a of (K in direction a) (x) (M in
// the others) at one offset, from the 1-D factors' entries in each
// direction: the products and sums of the assembly in its order, each
// rounded on its own, so the value is the stored A_ij bit for bit.
__device__ __forceinline__ double kron2(double Kx, double Mx, double Ky, double My) {
#pragma clang fp contract(off)
  double s = 0.0;
  s = s + Kx * My;
  s = s + Mx * Ky;
  return s;
}
__device__ __forceinline__ double kron3(double Kx, double Mx, double Ky, double My, double Kz, double Mz) {
#pragma clang fp contract(off)
  double s = 0.0;
  s = s + (Kx * My) * Mz;
  s = s + (Mx * Ky) * Mz;
  s = s + (Mx * My) * Kz;
  return s;
}

// Residual r = b - A x (PLAIN: r = A x) for Poisson on the unit box, where A
// is a Kronecker sum: the coefficients are formed from the bands kK, kM of
// the 1-D stiffness and mass (nx interior rows of WX = 2p+1 entries, 0
// outside the grid) instead of read, so only the vectors come from HBM.  The
// rows of a thread, the loop order, the masking of offsets outside the grid
// and the block partials are those of stencil_resid, and the coefficients
// equal the stored values, so both kernels give the same results bit for
// bit.  The row's x-factors stay in registers; the y- and z-factors are
// loaded per offset line (the same for the lanes of one grid line).
template <typename T, int DIM, bool PLAIN, int WX, int RB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void kron_resid(
    int n, int nx, int p, const double* __restrict__ kK, const double* __restrict__ kM, const T* __restrict__ x,
    const T* __restrict__ b, T* __restrict__ r, double* __restrict__ partial) {
  const int ny = nx;
  const int nz = DIM == 3 ? n / (nx * ny) : 1;
  const int nyb = (ny + RB - 1) / RB, nt = nx * nyb * nz;
  double sq = 0.0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < nt; t += gridDim.x * 256) {
    const int ix = t % nx, u = t / nx, iy0 = (u % nyb) * RB, iz = u / nyb;
    const int nr = min(RB, ny - iy0);
    const int dx0 = max(-p, -ix), dx1 = min(p, nx - 1 - ix);
    const int dz0 = DIM == 3 ? max(-p, -iz) : 0, dz1 = DIM == 3 ? min(p, nz - 1 - iz) : 0;
    const int i0 = (iz * ny + iy0) * nx + ix;
    const int y0 = max(0, iy0 - p), y1 = min(ny - 1, iy0 + nr - 1 + p);
    double Kx[WX], Mx[WX];
#pragma unroll
    for (int k = 0; k < WX; ++k) {
      Kx[k] = kK[ix * WX + k];
      Mx[k] = kM[ix * WX + k];
    }
    T acc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[q] = 0;
    for (int dz = dz0; dz <= dz1; ++dz) {
      const double Kz = DIM == 3 ? kK[iz * WX + dz + p] : 0.0, Mz = DIM == 3 ? kM[iz * WX + dz + p] : 0.0;
      for (int y = y0; y <= y1; ++y) {
        const T* xr = x + ((iz + dz) * ny + y) * nx + ix;
        T xx[WX];
#pragma unroll
        for (int k = 0; k < WX; ++k) {
          const int dx = k - WX / 2;
          xx[k] = xr[dx >= dx0 && dx <= dx1 ? dx : 0];
        }
        // the y-factors of every row of the thread for this line, loaded with
        // the line (clamped in range; unused where the line is not a neighbour)
        double Ky[RB], My[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const int iy = min(iy0 + q, ny - 1), ky = min(max(y - iy0 - q + p, 0), WX - 1);
          Ky[q] = kK[iy * WX + ky];
          My[q] = kM[iy * WX + ky];
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const int dy = y - iy0 - q;
          if (q < nr && dy >= -p && dy <= p) {
#pragma unroll
            for (int k = 0; k < WX; ++k) {
              const int dx = k - WX / 2;
              const T c = (T)(DIM == 3 ? kron3(Kx[k], Mx[k], Ky[q], My[q], Kz, Mz) : kron2(Kx[k], Mx[k], Ky[q], My[q]));
              acc[q] += (dx >= dx0 && dx <= dx1 ? c : (T)0) * xx[k];
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if (q < nr) {
        const int i = i0 + q * nx;
        const T res = PLAIN ? acc[q] : b[i] - acc[q];  // PLAIN: r = A x
        r[i] = res;
        sq += (double)res * (double)res;
      }
  }
  resid_partial(sq, partial);
}

// y = d .* (M x) (or y += d .* (M x) with ADD) for a transfer M between the
// degree-p and degree-1 grids (nxr nodes per axis for the rows, nxc for the
// columns).  Row i at grid position (ix, iy, iz) couples only to the column
// nodes (ix + o + kx, iy + o + ky, iz + o + kz), 0 <= k < W per axis; the
// value of slot k (lexicographic in (kz, ky, kx)) is V[k * nrow + i], 0 where
// the column node leaves its grid.
template <typename T, int DIM, bool ADD>
__global__ __launch_bounds__(256) void xgrid_spmv(int nrow, int nxr, int nxc, int o, int W, const T* __restrict__ V,
                                                  const T* __restrict__ x, const T* __restrict__ d, T* out) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nrow; i += gridDim.x * 256) {
    const int ix = i % nxr, t = i / nxr, iy = t % nxr, iz = t / nxr;
    const int jx = ix + o, jy = iy + o, jz = DIM == 3 ? iz + o : 0;
    const int kx0 = max(0, -jx), kx1 = min(W, nxc - jx);
    const int ky0 = max(0, -jy), ky1 = min(W, nxc - jy);
    const int kz0 = DIM == 3 ? max(0, -jz) : 0, kz1 = DIM == 3 ? min(W, nxc - jz) : 1;
    T acc = 0;
    for (int kz = kz0; kz < kz1; ++kz)
      for (int ky = ky0; ky < ky1; ++ky) {
        const T* vr = V + (size_t)((DIM == 3 ? kz * W : 0) + ky) * W * nrow + i;
        const T* xr = x + ((size_t)(jz + kz) * nxc + (jy + ky)) * nxc + jx;
        for (int kx = kx0; kx < kx1; ++kx) acc += vr[(int64_t)kx * nrow] * xr[kx];
      }
    out[i] = ADD ? out[i] + d[i] * acc : d[i] * acc;
  }
}

// xgrid_spmv for a transfer that is the Kronecker product of one 1-D matrix
// in every direction (P on the unit box, and R = P^T): the value of slot
// (kz, ky, kx) of row (ix, iy, iz) is formed from the 1-D factor's entries
// tab[ix W + kx] * tab[iy W + ky] (* tab[iz W + kz]), in the assembly's order
// and rounding, so it equals the stored value; same loops and sums as
// xgrid_spmv, so the results agree bit for bit.  KW > 0: W <= KW, and the
// row's x-factors are held in registers (loaded once, not per ky and kz);
// KW = 0: any W, the factors read in the loop.
__device__ __forceinline__ double kron_prod(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
template <typename T, int DIM, bool ADD, int KW>
__global__ __launch_bounds__(256) void kron_xgrid(int nrow, int nxr, int nxc, int o, int W,
                                                  const double* __restrict__ tab, const T* __restrict__ x,
                                                  const T* __restrict__ d, T* out) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < nrow; i += gridDim.x * 256) {
    const int ix = i % nxr, t = i / nxr, iy = t % nxr, iz = t / nxr;
    const int jx = ix + o, jy = iy + o, jz = DIM == 3 ? iz + o : 0;
    const int kx0 = max(0, -jx), kx1 = min(W, nxc - jx);
    const int ky0 = max(0, -jy), ky1 = min(W, nxc - jy);
    const int kz0 = DIM == 3 ? max(0, -jz) : 0, kz1 = DIM == 3 ? min(W, nxc - jz) : 1;
    double fx[KW > 0 ? KW : 1];
    if constexpr (KW > 0) {
#pragma unroll
      for (int k = 0; k < KW; ++k) fx[k] = k < W ? tab[ix * W + k] : 0.0;
    }
    T acc = 0;
    for (int kz = kz0; kz < kz1; ++kz)
      for (int ky = ky0; ky < ky1; ++ky) {
        const double ty = tab[iy * W + ky], tz = DIM == 3 ? tab[iz * W + kz] : 1.0;
        const T* xr = x + ((size_t)(jz + kz) * nxc + (jy + ky)) * nxc + jx;
        if constexpr (KW > 0) {
#pragma unroll
          for (int k = 0; k < KW; ++k)
            if (k >= kx0 && k < kx1) {
              const double c = DIM == 3 ? kron_prod(kron_prod(fx[k], ty), tz) : kron_prod(fx[k], ty);
              acc += (T)c * xr[k];
            }
        } else {
          for (int kx = kx0; kx < kx1; ++kx) {
            const double tx = tab[ix * W + kx];
            const double c = DIM == 3 ? kron_prod(kron_prod(tx, ty), tz) : kron_prod(tx, ty);
            acc += (T)c * xr[kx];
          }
        }
      }
    out[i] = ADD ? out[i] + d[i] * acc : d[i] * acc;
  }
}

// ---------------------------------------------------------------------------
// BiCGSTAB vector steps.  The method's scalars live in device memory
// (S[0] rho, S[1] previous rho, S[2] alpha, S[3] omega, S[4] (r^, v),
// S[5] (t, s), S[6] (t, t), S[7] ||r||^2); each kernel derives the scalars it
// needs from them, so an iteration needs the host only for the stopping test.
// Dot products are block partials in a fixed tree order (bit-reproducible).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void block_sum2(double a, double b, double* pa, double* pb) {
  __shared__ double ra[256], rb[256];
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      ra[threadIdx.x] += ra[threadIdx.x + k];
      rb[threadIdx.x] += rb[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pa[blockIdx.x] = ra[0];
    if (pb) pb[blockIdx.x] = rb[0];
  }
}

// S[0] = rho = ||r_0||^2 (from the residual norm), S[1..3] = 1 (one thread)
__global__ void bicg_init(const double* __restrict__ rr, double* S) {
  S[0] = rr[0];
  S[1] = S[2] = S[3] = 1.0;
  S[4] = S[5] = S[6] = 0.0;
  S[7] = rr[0];
}

// partials of (a, b) and, if c, of (c, d)
__global__ __launch_bounds__(256) void dot2_partials(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                     const double* __restrict__ c, const double* __restrict__ d,
                                                     double* __restrict__ pa, double* __restrict__ pb) {
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    s1 += a[i] * b[i];
    if (c) s2 += c[i] * d[i];
  }
  block_sum2(s1, s2, pa, c ? pb : nullptr);
}

// Conjugate gradients for the consistent-mass transfers (Appendix B), with
// the inverse lumped mass dinv as preconditioner.  cg_init: x = 0, r = b,
// z = dinv .* b, p = z, partials of b.b and b.z; cg_step: x += a p,
// r -= a q, z = dinv .* r, partials of r.r and r.z; cg_dir: p = z + c p.
__global__ __launch_bounds__(256) void cg_init(int64_t n, const double* __restrict__ b, const double* __restrict__ dinv,
                                               double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                               double* __restrict__ p, double* __restrict__ pa, double* __restrict__ pb) {
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double bi = b[i], zi = dinv[i] * bi;
    x[i] = 0.0;
    r[i] = bi;
    z[i] = zi;
    p[i] = zi;
    s1 += bi * bi;
    s2 += bi * zi;
  }
  block_sum2(s1, s2, pa, pb);
}

__global__ __launch_bounds__(256) void cg_step(int64_t n, double a, const double* __restrict__ p,
                                               const double* __restrict__ q, const double* __restrict__ dinv,
                                               double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                               double* __restrict__ pa, double* __restrict__ pb) {
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i], zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    s1 += ri * ri;
    s2 += ri * zi;
  }
  block_sum2(s1, s2, pa, pb);
}

__global__ __launch_bounds__(256) void cg_dir(int64_t n, double c, const double* __restrict__ z, double* __restrict__ p) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = z[i] + c * p[i];
}

// x += y
__global__ __launch_bounds__(256) void add_vec(int64_t n, const double* __restrict__ y, double* __restrict__ x) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) x[i] += y[i];
}

// S[ia] = sum of pa (and S[ib] = sum of pb if ib >= 0); with shift_rho the
// old S[0] is first saved in S[1].  One block.
__global__ __launch_bounds__(256) void bicg_reduce(int nb, const double* __restrict__ pa, const double* __restrict__ pb,
                                                   double* S, int ia, int ib, int shift_rho) {
  __shared__ double ra[256], rb[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += pa[i];
    if (ib >= 0) b += pb[i];
  }
  ra[threadIdx.x] = a;
  rb[threadIdx.x] = b;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      ra[threadIdx.x] += ra[threadIdx.x + k];
      rb[threadIdx.x] += rb[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (shift_rho) S[1] = S[0];
    S[ia] = ra[0];
    if (ib >= 0) S[ib] = rb[0];
  }
}

// p = r + beta (p - omega v), beta = (rho / rho_prev) (alpha / omega)
__global__ __launch_bounds__(256) void bicg_p(int64_t n, const double* __restrict__ S, const double* __restrict__ r,
                                              const double* __restrict__ v, double* __restrict__ p) {
  const double beta = (S[0] / S[1]) * (S[2] / S[3]), omega = S[3];
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// alpha = rho / (r^, v); s = r - alpha v (over r); x += alpha y
__global__ __launch_bounds__(256) void bicg_s(int64_t n, double* S, const double* __restrict__ v,
                                              const double* __restrict__ y, double* __restrict__ r,
                                              double* __restrict__ x) {
  const double alpha = S[0] / S[4];
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    r[i] -= alpha * v[i];
    x[i] += alpha * y[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) S[2] = alpha;
}

// omega = (t, s) / (t, t) (0 if t = 0); x += omega z; r = s - omega t (s is
// in r); partials of (r, r) and (r^, r) for the stopping test and next rho
__global__ __launch_bounds__(256) void bicg_x(int64_t n, double* S, const double* __restrict__ z,
                                              const double* __restrict__ t, const double* __restrict__ rh,
                                              double* __restrict__ x, double* __restrict__ r, double* __restrict__ pa,
                                              double* __restrict__ pb) {
  const double omega = S[6] > 0.0 ? S[5] / S[6] : 0.0;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] += omega * z[i];
    const double ri = r[i] - omega * t[i];
    r[i] = ri;
    s1 += ri * ri;
    s2 += rh[i] * ri;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) S[3] = omega;
  block_sum2(s1, s2, pa, pb);
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
// Degree-1 h-multigrid on the structured grids of its levels.
//
// A level's interior nodes form an nx^d grid (x fastest).  Its operator
// couples a node only to the nodes at offsets in {-1, 0, 1}^d, stored per
// colour (parity of the grid position along each axis: colour bit a = parity
// along axis a): the t-th node of colour c (x fastest within the colour) has
// the value of offset k (lexicographic in (dz, dy, dx)) at
// V[voff[c] + k * cnt[c] + t].  A colour's nodes are not coupled to each
// other, so a Gauss-Seidel half-sweep over one colour is one parallel pass
// reading its values contiguously.  The canonical transfers (weights 1/2, 1,
// 1/2 per axis: coarse node c sits on fine node 2c + 1) are applied from
// their definition, without a matrix.
// ---------------------------------------------------------------------------

template <int DIM>
__device__ __forceinline__ void colour_node(const GridLevel& L, int c, int t, int& ix, int& iy, int& iz) {
  const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
  const int mx = (L.nx - cx + 1) / 2, my = (L.nx - cy + 1) / 2;
  const int tx = t % mx, r = t / mx;
  ix = 2 * tx + cx;
  iy = 2 * (DIM == 3 ? r % my : r) + cy;
  iz = DIM == 3 ? 2 * (r / my) + cz : 0;
}

// sum over the offsets of node (ix, iy, iz), the centre left out when
// skip_centre (its value returned in *centre)
template <int DIM>
__device__ __forceinline__ double grid_dot(const GridLevel& L, const double* vc, int cnt, int t, int ix, int iy,
                                           int iz, const double* x, bool skip_centre, double* centre) {
  const int nx = L.nx;
  const int i = (iz * nx + iy) * nx + ix;
  double acc = 0.0;
  int k = 0;
#pragma unroll
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx, ++k) {
        const bool ok = ix + dx >= 0 && ix + dx < nx && iy + dy >= 0 && iy + dy < nx &&
                        (DIM == 2 || (iz + dz >= 0 && iz + dz < nx));
        const double a = vc[(size_t)k * cnt + t];
        if (dx == 0 && dy == 0 && dz == 0 && skip_centre) {
          *centre = a;
        } else {
          // branch-free, so all loads of the node are in flight together: a
          // neighbour outside the grid reads the node itself with weight 0
          // (acc + 0 * x is acc for finite x, and acc is never -0)
          const double xv = x[ok ? i + (dz * nx + dy) * nx + dx : i];
          acc += (ok ? a : 0.0) * xv;
        }
      }
  return acc;
}

// One multicolour Gauss-Seidel half-sweep: e_i = (b_i - sum_{j != i} a_ij e_j) / a_ii
// for the nodes of colour c.
template <int DIM>
__global__ __launch_bounds__(256) void grid_gs(GridLevel L, int c, const double* __restrict__ b, double* e) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= L.cnt[c]) return;
  int ix, iy, iz;
  colour_node<DIM>(L, c, t, ix, iy, iz);
  const int i = (iz * L.nx + iy) * L.nx + ix;
  double centre = 1.0;
  const double acc = grid_dot<DIM>(L, L.v + L.voff[c], L.cnt[c], t, ix, iy, iz, e, true, &centre);
  e[i] = (b[i] - acc) / centre;
}

// r = b - A e over all nodes (threads in colour-major order).
template <int DIM>
__global__ __launch_bounds__(256) void grid_resid(GridLevel L, const double* __restrict__ b,
                                                  const double* __restrict__ e, double* __restrict__ r) {
  int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= L.n) return;
  int c = 0;
  while (g >= L.cnt[c]) g -= L.cnt[c++];
  int ix, iy, iz;
  colour_node<DIM>(L, c, g, ix, iy, iz);
  const int i = (iz * L.nx + iy) * L.nx + ix;
  r[i] = b[i] - grid_dot<DIM>(L, L.v + L.voff[c], L.cnt[c], g, ix, iy, iz, e, false, nullptr);
}

// Coarse right-hand side bc = R_h r (R_h = P_h^T: coarse node c collects fine
// nodes 2c, 2c+1, 2c+2 with weights 1/2, 1, 1/2 per axis) and the coarse
// iterate ec = 0.  nf = 2 nc + 1 fine nodes per axis.
template <int DIM>
__global__ __launch_bounds__(256) void grid_restrict(int nc, const double* __restrict__ r, double* __restrict__ bc,
                                                     double* __restrict__ ec) {
  const int C = blockIdx.x * 256 + threadIdx.x;
  const int ncell = DIM == 3 ? nc * nc * nc : nc * nc;
  if (C >= ncell) return;
  const int nf = 2 * nc + 1;
  const int cx = C % nc, cy = (C / nc) % nc, cz = DIM == 3 ? C / (nc * nc) : 0;
  const double w[3] = {0.5, 1.0, 0.5};
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < (DIM == 3 ? 3 : 1); ++a)
#pragma unroll
    for (int bb = 0; bb < 3; ++bb)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const int fz = DIM == 3 ? 2 * cz + a : 0;
        const double wz = DIM == 3 ? w[a] : 1.0;
        acc += (wz * w[bb] * w[cc]) * r[((size_t)fz * nf + 2 * cy + bb) * nf + 2 * cx + cc];
      }
  bc[C] = acc;
  ec[C] = 0.0;
}

// (P_h ec) at fine node F: along an axis fine node f takes coarse (f-1)/2 with
// weight 1 if f is odd, else coarse f/2 - 1 and f/2 (those that exist) with
// 1/2.  Written with two parents per axis (a missing one has weight 0 and adds
// an exact zero), so the indices stay in registers.
template <int DIM>
__device__ __forceinline__ double prolong_at(int nc, int F, const double* ec) {
  const int nf = 2 * nc + 1;
  const int f[3] = {F % nf, (F / nf) % nf, DIM == 3 ? F / (nf * nf) : 0};
  int c0[3], c1[3];
  double w0[3], w1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == 2 && DIM == 2) {
      c0[a] = c1[a] = 0;
      w0[a] = 1.0;
      w1[a] = 0.0;
    } else if (f[a] & 1) {
      c0[a] = c1[a] = (f[a] - 1) / 2;
      w0[a] = 1.0;
      w1[a] = 0.0;
    } else {
      const int lo = f[a] / 2 - 1, hi = f[a] / 2;
      c0[a] = lo >= 0 ? lo : 0;
      w0[a] = lo >= 0 ? 0.5 : 0.0;
      c1[a] = hi < nc ? hi : 0;
      w1[a] = hi < nc ? 0.5 : 0.0;
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int kz = 0; kz < (DIM == 3 ? 2 : 1); ++kz)
#pragma unroll
    for (int ky = 0; ky < 2; ++ky)
#pragma unroll
      for (int kx = 0; kx < 2; ++kx) {
        const double w = (kz ? w1[2] : w0[2]) * (ky ? w1[1] : w0[1]) * (kx ? w1[0] : w0[0]);
        const int c = ((kz ? c1[2] : c0[2]) * nc + (ky ? c1[1] : c0[1])) * nc + (kx ? c1[0] : c0[0]);
        acc += w * ec[c];
      }
  return acc;
}

// e_f += P_h ec (canonical prolongation, see prolong_at); nf = 2 nc + 1 fine
// nodes per axis.
template <int DIM>
__global__ __launch_bounds__(256) void grid_prolong_add(int nc, const double* __restrict__ ec, double* __restrict__ ef) {
  const int nf = 2 * nc + 1;
  const int F = blockIdx.x * 256 + threadIdx.x;
  const int nfine = DIM == 3 ? nf * nf * nf : nf * nf;
  if (F >= nfine) return;
  ef[F] += prolong_at<DIM>(nc, F, ec);
}

// ---------------------------------------------------------------------------
// Tiled smoothing on 2-D structured degree-1 levels.
//
// The launch-per-colour path costs a launch per colour phase, which on the
// middle levels is most of the time.  Here a workgroup owns the fine nodes
// 2 C0 .. 2 C1 - 1 per axis under a block C0 .. C1 - 1 of coarse nodes (the
// last block also the last fine node) and runs all colour phases of the
// sweeps in LDS on that block widened by a halo: each phase updates a region
// one node narrower than the one before, so the nodes the block needs at the
// end hold exactly the values of the launch-per-colour sweeps (halo nodes are
// computed again by the neighbouring blocks, from the same inputs with the
// same arithmetic).  The iterate is read from one buffer and written to
// another, so no block reads a value another block has already replaced.
// gs_tile_down fuses the pre-smoothing sweeps with the residual and the
// restriction after them, gs_tile_up the prolongation with the
// post-smoothing sweeps after it.  Results are identical to the
// launch-per-phase kernels.
// ---------------------------------------------------------------------------

constexpr int kTileThreads = 512;
constexpr int kTileMaxSweeps = 2;  // sweeps per launch (the halo grows with them)

struct TileBox {
  int f0x, f1x, f0y, f1y;  // owned fine nodes [f0, f1)
  int c0x, c1x, c0y, c1y;  // coarse nodes of the block [c0, c1)
  int ox, oy, w;           // LDS origin and row length of the iterate tile
};

__device__ __forceinline__ TileBox tile_box(int nc, int tcb, int halo) {
  const int ntx = (nc + tcb - 1) / tcb;
  const int bx = blockIdx.x % ntx, by = blockIdx.x / ntx;
  const int nf = 2 * nc + 1;
  TileBox B;
  B.c0x = bx * tcb;
  B.c1x = min(B.c0x + tcb, nc);
  B.c0y = by * tcb;
  B.c1y = min(B.c0y + tcb, nc);
  B.f0x = 2 * B.c0x;
  B.f1x = B.c1x == nc ? nf : 2 * B.c1x;
  B.f0y = 2 * B.c0y;
  B.f1y = B.c1y == nc ? nf : 2 * B.c1y;
  B.ox = B.f0x - halo;
  B.oy = B.f0y - halo;
  B.w = 2 * tcb + 1 + 2 * halo;
  return B;
}

// The stencil sum of grid_dot for node (ix, iy), neighbours from the LDS tile.
// KRON: the coefficients formed from the level's 1-D bands (kron2, the
// assembly's products and sums), equal to the stored values bit for bit.
template <bool KRON>
__device__ __forceinline__ double tile_dot_t(const GridLevel& L, int ix, int iy, const double* el, const TileBox& B,
                                             bool skip_centre, double* centre) {
  const int c = (ix & 1) | ((iy & 1) << 1);
  const int mx = (L.nx - (c & 1) + 1) / 2;
  const int t = (iy >> 1) * mx + (ix >> 1);
  const int cnt = L.cnt[c];
  const double* vc = L.v + L.voff[c];
  const int nx = L.nx;
  const double* x = el + (iy - B.oy) * B.w + (ix - B.ox);
  double Kx[3], Mx[3], Ky[3], My[3];
  if constexpr (KRON) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      Kx[u] = L.kK[ix * 3 + u];
      Mx[u] = L.kM[ix * 3 + u];
      Ky[u] = L.kK[iy * 3 + u];
      My[u] = L.kM[iy * 3 + u];
    }
  }
  double acc = 0.0;
  int k = 0;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx, ++k) {
      const bool ok = ix + dx >= 0 && ix + dx < nx && iy + dy >= 0 && iy + dy < nx;
      const double a = KRON ? kron2(Kx[dx + 1], Mx[dx + 1], Ky[dy + 1], My[dy + 1]) : vc[(size_t)k * cnt + t];
      if (dx == 0 && dy == 0 && skip_centre) {
        *centre = a;
      } else {
        // branch-free as in grid_dot: a neighbour outside the grid reads the
        // node itself with weight 0
        const double xv = x[ok ? dy * B.w + dx : 0];
        acc += (ok ? a : 0.0) * xv;
      }
    }
  return acc;
}
__device__ __forceinline__ double tile_dot(const GridLevel& L, int ix, int iy, const double* el, const TileBox& B,
                                           bool skip_centre, double* centre) {
  return L.kK ? tile_dot_t<true>(L, ix, iy, el, B, skip_centre, centre)
              : tile_dot_t<false>(L, ix, iy, el, B, skip_centre, centre);
}

// Colour phases of nsweep sweeps; after them the nodes within `hend` of the
// owned range hold their final values.
__device__ __forceinline__ void tile_sweeps(const GridLevel& L, int colors, int nsweep, int hend,
                                            const double* __restrict__ b, double* el, const TileBox& B) {
  const int nf = L.nx, K = colors * nsweep;
  for (int k = 0; k < K; ++k) {
    const int c = k % colors, h = hend + K - 1 - k;
    const int x0 = max(B.f0x - h, 0), x1 = min(B.f1x + h, nf);
    const int y0 = max(B.f0y - h, 0), y1 = min(B.f1y + h, nf);
    const int xs = x0 + ((x0 & 1) != (c & 1)), ys = y0 + ((y0 & 1) != ((c >> 1) & 1));
    const int mxr = xs < x1 ? (x1 - xs + 1) / 2 : 0, myr = ys < y1 ? (y1 - ys + 1) / 2 : 0;
#pragma unroll 2
    for (int t = threadIdx.x; t < mxr * myr; t += kTileThreads) {
      const int ix = xs + 2 * (t % mxr), iy = ys + 2 * (t / mxr);
      double centre = 1.0;
      const double acc = tile_dot(L, ix, iy, el, B, true, &centre);
      el[(iy - B.oy) * B.w + (ix - B.ox)] = (b[iy * nf + ix] - acc) / centre;
    }
    __syncthreads();
  }
}

// Pre-smoothing (nsweep sweeps of e_in, result in e_out), then bc = R_h (b - A e)
// and ec = 0 on the coarse level.  tcb coarse nodes per block side.
__global__ __launch_bounds__(kTileThreads) void gs_tile_down(GridLevel L, int nc, int tcb, int colors, int nsweep,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ e_in,
                                                             double* __restrict__ e_out, double* __restrict__ bc,
                                                             double* __restrict__ ec) {
  extern __shared__ double sm[];
  constexpr int hend = 2;  // the residual reaches one node past the block and reads one further
  const int halo = hend + colors * nsweep;
  const TileBox B = tile_box(nc, tcb, halo);
  const int nf = L.nx;
  double* el = sm;
  double* rl = sm + B.w * B.w;
  const int rw = 2 * tcb + 1;
  {
    const int x0 = max(B.ox, 0), x1 = min(B.f1x + halo, nf), y0 = max(B.oy, 0), y1 = min(B.f1y + halo, nf);
    const int mw = x1 - x0;
    for (int t = threadIdx.x; t < mw * (y1 - y0); t += kTileThreads) {
      const int ix = x0 + t % mw, iy = y0 + t / mw;
      el[(iy - B.oy) * B.w + (ix - B.ox)] = e_in[iy * nf + ix];
    }
  }
  __syncthreads();
  tile_sweeps(L, colors, nsweep, hend, b, el, B);
  // residual at fine nodes 2 C0 .. 2 C1 (the block's restriction stencils)
  {
    const int x1 = min(2 * B.c1x + 1, nf), y1 = min(2 * B.c1y + 1, nf);
    const int mw = x1 - B.f0x;
    for (int t = threadIdx.x; t < mw * (y1 - B.f0y); t += kTileThreads) {
      const int ix = B.f0x + t % mw, iy = B.f0y + t / mw;
      rl[(iy - B.f0y) * rw + (ix - B.f0x)] = b[iy * nf + ix] - tile_dot(L, ix, iy, el, B, false, nullptr);
    }
  }
  __syncthreads();
  {
    const double w[3] = {0.5, 1.0, 0.5};
    const int mc = B.c1x - B.c0x;
    for (int t = threadIdx.x; t < mc * (B.c1y - B.c0y); t += kTileThreads) {
      const int cx = B.c0x + t % mc, cy = B.c0y + t / mc;
      const double* r = rl + 2 * (cy - B.c0y) * rw + 2 * (cx - B.c0x);
      const double wz = 1.0;
      double acc = 0.0;
#pragma unroll
      for (int bb = 0; bb < 3; ++bb)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) acc += (wz * w[bb] * w[cc]) * r[bb * rw + cc];
      bc[cy * nc + cx] = acc;
      ec[cy * nc + cx] = 0.0;
    }
    const int mw = B.f1x - B.f0x;
    for (int t = threadIdx.x; t < mw * (B.f1y - B.f0y); t += kTileThreads) {
      const int ix = B.f0x + t % mw, iy = B.f0y + t / mw;
      e_out[iy * nf + ix] = el[(iy - B.oy) * B.w + (ix - B.ox)];
    }
  }
}

// e_out = nsweep post-smoothing sweeps of (e_in + P_h ec).
__global__ __launch_bounds__(kTileThreads) void gs_tile_up(GridLevel L, int nc, int tcb, int colors, int nsweep,
                                                           const double* __restrict__ b,
                                                           const double* __restrict__ e_in,
                                                           const double* __restrict__ ec,
                                                           double* __restrict__ e_out) {
  extern __shared__ double sm[];
  const int halo = colors * nsweep;
  const TileBox B = tile_box(nc, tcb, halo);
  const int nf = L.nx;
  double* el = sm;
  {
    const int x0 = max(B.ox, 0), x1 = min(B.f1x + halo, nf), y0 = max(B.oy, 0), y1 = min(B.f1y + halo, nf);
    const int mw = x1 - x0;
    for (int t = threadIdx.x; t < mw * (y1 - y0); t += kTileThreads) {
      const int ix = x0 + t % mw, iy = y0 + t / mw;
      const int F = iy * nf + ix;
      el[(iy - B.oy) * B.w + (ix - B.ox)] = e_in[F] + prolong_at<2>(nc, F, ec);
    }
  }
  __syncthreads();
  tile_sweeps(L, colors, nsweep, 0, b, el, B);
  const int mw = B.f1x - B.f0x;
  for (int t = threadIdx.x; t < mw * (B.f1y - B.f0y); t += kTileThreads) {
    const int ix = B.f0x + t % mw, iy = B.f0y + t / mw;
    e_out[iy * nf + ix] = el[(iy - B.oy) * B.w + (ix - B.ox)];
  }
}

// ---------------------------------------------------------------------------
// The smallest levels of the structured h-multigrid V-cycle in one workgroup.
//
// Below a few thousand nodes a level's phases are too short to fill the GPU,
// and a launch per phase costs more than the phase.  This kernel runs the
// V-cycle from level 0 of its list down to the coarsest and back (the same
// steps as the launch-per-phase path) with every level's iterate and
// right-hand side in LDS; only the stencil values (L2-resident) and the
// coarsest inverse are read from global memory.  Phases are separated by
// workgroup barriers.
// ---------------------------------------------------------------------------

constexpr int kLdsLevels = 6;
constexpr int kLdsThreads = 1024;

struct LdsCycle {
  int nl;               // levels in the list, the last solved directly
  int colors, nu1, nu2;
  int ncoarse;          // unknowns of the coarsest level
  const double* cinv;   // its inverse, row-major
  const double* b0;     // right-hand side of the first level (global)
  double* e0;           // iterate of the first level (global, read and written)
  GridLevel lev[kLdsLevels - 1];  // smoothing levels
  int nx[kLdsLevels];   // nodes per axis of every level
  int eoff[kLdsLevels], boff[kLdsLevels], roff;  // LDS offsets (doubles)
};

template <int DIM>
__device__ __forceinline__ int grid_index(int nx, int ix, int iy, int iz) {
  return (iz * nx + iy) * nx + ix;
}

// sum over the offsets of node (ix, iy, iz) of a level held in LDS (x), the
// centre left out when skip_centre
template <int DIM>
__device__ __forceinline__ double lds_dot(const GridLevel& L, const double* vc, int cnt, int t, int ix, int iy, int iz,
                                          const double* x, bool skip_centre, double* centre) {
  const int nx = L.nx;
  double a[DIM == 3 ? 27 : 9];
  int k = 0;
#pragma unroll
  for (int q = 0; q < (DIM == 3 ? 27 : 9); ++q) a[q] = vc[(size_t)q * cnt + t];
  double acc = 0.0;
#pragma unroll
  for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx, ++k) {
        const bool ok = ix + dx >= 0 && ix + dx < nx && iy + dy >= 0 && iy + dy < nx &&
                        (DIM == 2 || (iz + dz >= 0 && iz + dz < nx));
        if (dx == 0 && dy == 0 && dz == 0 && skip_centre) {
          *centre = a[k];
        } else {
          const double xv = x[ok ? grid_index<DIM>(nx, ix + dx, iy + dy, iz + dz) : grid_index<DIM>(nx, ix, iy, iz)];
          acc += (ok ? a[k] : 0.0) * xv;  // as in grid_dot
        }
      }
  return acc;
}

template <int DIM>
__device__ void lds_sweeps(const LdsCycle& S, int k, double* sm, int nsweep) {
  const GridLevel& L = S.lev[k];
  double* e = sm + S.eoff[k];
  const double* b = sm + S.boff[k];
  for (int sw = 0; sw < nsweep; ++sw)
    for (int c = 0; c < S.colors; ++c) {
      for (int t = threadIdx.x; t < L.cnt[c]; t += kLdsThreads) {
        int ix, iy, iz;
        colour_node<DIM>(L, c, t, ix, iy, iz);
        double centre = 1.0;
        const double acc = lds_dot<DIM>(L, L.v + L.voff[c], L.cnt[c], t, ix, iy, iz, e, true, &centre);
        const int i = grid_index<DIM>(L.nx, ix, iy, iz);
        e[i] = (b[i] - acc) / centre;
      }
      __syncthreads();
    }
}

template <int DIM>
__global__ __launch_bounds__(kLdsThreads) void hcycle_lds(LdsCycle S) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x;
  const int n0 = DIM == 3 ? S.nx[0] * S.nx[0] * S.nx[0] : S.nx[0] * S.nx[0];
  for (int i = tid; i < n0; i += kLdsThreads) {
    sm[S.boff[0] + i] = S.b0[i];
    sm[S.eoff[0] + i] = S.e0[i];
  }
  __syncthreads();
  for (int k = 0; k + 1 < S.nl; ++k) {
    const GridLevel& L = S.lev[k];
    lds_sweeps<DIM>(S, k, sm, S.nu1);
    // residual into the scratch, all nodes in colour-major order
    double* r = sm + S.roff;
    const double* e = sm + S.eoff[k];
    const double* b = sm + S.boff[k];
    for (int g0 = tid; g0 < L.n; g0 += kLdsThreads) {
      int g = g0, c = 0;
      while (g >= L.cnt[c]) g -= L.cnt[c++];
      int ix, iy, iz;
      colour_node<DIM>(L, c, g, ix, iy, iz);
      const int i = grid_index<DIM>(L.nx, ix, iy, iz);
      r[i] = b[i] - lds_dot<DIM>(L, L.v + L.voff[c], L.cnt[c], g, ix, iy, iz, e, false, nullptr);
    }
    __syncthreads();
    // restriction (weights 1/2, 1, 1/2 per axis) and a zero coarse iterate
    const int nc = S.nx[k + 1], nf = 2 * nc + 1;
    const int ncell = DIM == 3 ? nc * nc * nc : nc * nc;
    double* bc = sm + S.boff[k + 1];
    double* ec = sm + S.eoff[k + 1];
    const double w[3] = {0.5, 1.0, 0.5};
    for (int C = tid; C < ncell; C += kLdsThreads) {
      const int cx = C % nc, cy = (C / nc) % nc, cz = DIM == 3 ? C / (nc * nc) : 0;
      double acc = 0.0;
      for (int a = 0; a < (DIM == 3 ? 3 : 1); ++a)
        for (int bb = 0; bb < 3; ++bb)
          for (int cc = 0; cc < 3; ++cc) {
            const int fz = DIM == 3 ? 2 * cz + a : 0;
            const double wz = DIM == 3 ? w[a] : 1.0;
            acc += (wz * w[bb] * w[cc]) * r[(fz * nf + 2 * cy + bb) * nf + 2 * cx + cc];
          }
      bc[C] = acc;
      ec[C] = 0.0;
    }
    __syncthreads();
  }
  {  // coarsest: e = A^{-1} b
    const int kc = S.nl - 1;
    const double* bc = sm + S.boff[kc];
    double* ec = sm + S.eoff[kc];
    for (int i = tid; i < S.ncoarse; i += kLdsThreads) {
      const double* a = S.cinv + (size_t)i * S.ncoarse;
      double acc = 0.0;
      for (int j = 0; j < S.ncoarse; ++j) acc += a[j] * bc[j];
      ec[i] = acc;
    }
    __syncthreads();
  }
  for (int k = S.nl - 2; k >= 0; --k) {
    const int nc = S.nx[k + 1], nf = 2 * nc + 1;
    const int nfine = DIM == 3 ? nf * nf * nf : nf * nf;
    const double* ec = sm + S.eoff[k + 1];
    double* ef = sm + S.eoff[k];
    for (int F = tid; F < nfine; F += kLdsThreads) ef[F] += prolong_at<DIM>(nc, F, ec);
    __syncthreads();
    lds_sweeps<DIM>(S, k, sm, S.nu2);
  }
  for (int i = tid; i < n0; i += kLdsThreads) S.e0[i] = sm[S.eoff[0] + i];
}

// ---------------------------------------------------------------------------
// Sparse triangular solves with the ILUT factors (Section 3, "Smoother").
//
// Rows are grouped in segments (grid lines of the tensor numbering, seg_len
// consecutive rows) and segments in chunks of 64 rows, lane = row.  A grid of
// persistent waves takes chunks through an atomic ticket in a topological
// order of the chunk dependency graph, so a wave only ever waits for chunks
// already owned by running waves (no deadlock, whatever the launch order or
// the number of resident waves).
//
// Readiness travels with the data: the output vector starts filled with the
// kPending marker, and a wave that reads an entry of another chunk reloads it
// until the marker is gone.  Per chunk: the in-chunk entries are staged in
// LDS, the off-chunk slots are gathered batch by batch (entries that are
// final early first), then the rows inside the chunk are finished in order,
// the newest value broadcast from its lane, and stored.  Every load of a batch
// is issued before the first is consumed, so a chunk costs a few memory round
// trips, and the chain from one level to the next is one store and one load.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Entries written by other waves during the solve are read and written with
// device-scope (agent) atomic accesses, which are coherent across the XCDs'
// L2 caches: every reload sees the newest stored value.
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool pending(double v) {
  return (unsigned long long)__double_as_longlong(v) == kPending64;
}
__device__ __forceinline__ bool pending(float v) { return (unsigned)__float_as_int(v) == kPending32; }

// A computed value never has the marker's bits (it is a signalling NaN);
// should one arrive anyway it is stored as the canonical quiet NaN.
template <typename T>
__device__ __forceinline__ T publishable(T v) {
  return pending(v) ? (T)__builtin_nan("") : v;
}

// Counters and fault word of one triangular solve.  state: the ticket
// counter and the exited-wave count (kTicketWords words); fault: set to 1
// by a wave that polled a batch poll_limit times, and left for the host to
// read and clear.
struct TriCtl {
  unsigned* state;
  unsigned* fault;
  int poll_limit;
};

// Draws the wave's next ticket: every lane takes part in the atomic (lane 0
// adds 1, the others 0) and lane 0's old value is the ticket.  No branch
// depends on the lane here: inside a loop, a lane-dependent branch around the
// atomic followed by a cross-lane read lets the compiler send lane 0 and the
// other lanes round different loops.
//
// Why no wave waits forever, whatever the number of resident waves: tickets
// follow a topological order of the chunk graph, so the smallest unfinished
// ticket only waits for finished chunks, and it is held by a wave that is
// running (a wave draws a ticket only once it runs, and tickets are drawn in
// increasing order from the one counter).  That wave finishes its chunk, and
// by induction every chunk is finished.  The poll bound (TriCtl) turns a
// schedule that breaks this order into a reported fault instead of a hang.
__device__ __forceinline__ int wave_ticket(unsigned* state) {
  const unsigned v = atomicAdd(state, (threadIdx.x & 63) == 0 ? 1u : 0u);
  return __builtin_amdgcn_readfirstlane((int)v);
}

// Called by every wave of the grid once it has drawn a ticket past the last
// chunk.  The last wave to get here clears the counters for the next launch
// (all other waves have exited), so a solve needs no separate reset launch.
__device__ __forceinline__ void finish_grid(unsigned* state, int lane) {
  unsigned* exited = state + kTicketStride;
  const unsigned prev = atomicAdd(exited, lane == 0 ? 1u : 0u);
  if ((unsigned)__builtin_amdgcn_readfirstlane((int)prev) == gridDim.x - 1 && lane == 0) {
    st_dev(state, 0u);
    st_dev(exited, 0u);
  }
}

// Read-only data with a wave-uniform address through the scalar cache (the
// constant address space): such loads are counted apart from the vector
// loads in flight, so waiting for them does not drain the gathers.
__device__ __forceinline__ TriMeta ld_meta(const TriMeta* p) {
  const auto* w = (const __attribute__((address_space(4))) int*)p;
  TriMeta m;
  m.row0 = w[0];
  m.nrow = w[1];
  m.off_ptr = w[2];
  m.off_w = w[3];
  m.in_ptr = w[4];
  m.in_w = w[5];
  return m;
}

constexpr int kStage = 16;  // in-chunk slots loaded per round trip
static_assert(kStage % kColGroup == 0 && kTriBatch % kColGroup == 0, "slot loads come in whole groups");
static_assert(kTriPad >= 64 * kColGroup, "one padding group per lane");

// 16-byte groups of a lane's slots (see pmg::TriDev): kColGroup column
// indices, or 16 / sizeof(T) values.
typedef int ColGroup __attribute__((ext_vector_type(kColGroup)));
template <typename T>
struct ValGroup;
template <>
struct ValGroup<double> {
  static constexpr int G = 2;
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct ValGroup<float> {
  static constexpr int G = 4;
  typedef float type __attribute__((ext_vector_type(4)));
};

// Slots u0 .. u0 + N - 1 of one lane (u0 a multiple of kColGroup) from the
// grouped arrays at `base`; slots outside [0, w) and lanes past the end of a
// partial chunk (act false) read the padding group at `pad` instead, which
// stays cached, so padding lanes cost no memory traffic.  The factor is read
// once per solve, so its loads are non-temporal and leave the caches to the
// solution vector.
template <int N>
__device__ __forceinline__ void load_cols(int (&c)[N], int u0, int w, int base, int pad, int lane, const int* cols,
                                          bool act) {
#pragma unroll
  for (int g = 0; g < N / kColGroup; ++g) {
    const int v = u0 + g * kColGroup;
    const int i = act && v >= 0 && v < w ? base + v * kWave + lane * kColGroup : pad + lane * kColGroup;
    const ColGroup q = __builtin_nontemporal_load(reinterpret_cast<const ColGroup*>(cols + i));
#pragma unroll
    for (int k = 0; k < kColGroup; ++k) c[g * kColGroup + k] = q[k];
  }
}

template <typename T, int N>
__device__ __forceinline__ void load_vals(T (&a)[N], int u0, int w, int base, int pad, int lane, const T* vals,
                                          bool act) {
  constexpr int G = ValGroup<T>::G;
#pragma unroll
  for (int g = 0; g < N / G; ++g) {
    const int v = u0 + g * G;
    const int i = act && v >= 0 && v < w ? base + v * kWave + lane * G : pad + lane * G;
    const typename ValGroup<T>::type q =
        __builtin_nontemporal_load(reinterpret_cast<const typename ValGroup<T>::type*>(vals + i));
#pragma unroll
    for (int k = 0; k < G; ++k) a[g * G + k] = q[k];
  }
}

template <typename T, int N>
__device__ __forceinline__ void load_slots(int (&c)[N], T (&a)[N], int u0, int w, int base, int pad, int lane,
                                           const int* cols, const T* vals, bool act) {
  load_cols<N>(c, u0, w, base, pad, lane, cols, act);
  load_vals<T, N>(a, u0, w, base, pad, lane, vals, act);
}

template <typename T>
__device__ __forceinline__ void load_in(int (&jj)[kStage], T (&vv)[kStage], int u0, int w, int base, int lane,
                                        const TriDev<T>& F, bool act) {
  load_slots<T, kStage>(jj, vv, u0, w, base, F.in_pad, lane, F.in_j, F.in_val, act);
}

// Stage the in-chunk entries of this lane's row in column `lane` of the tile
// (each lane only ever touches its own column); the first kStage slots were
// loaded into jj/vv by the caller.  Padding slots write 0 on the diagonal,
// which holds no entry of a strictly triangular part.
template <typename T>
__device__ __forceinline__ void stage_tile(T* tile, int (&jj)[kStage], T (&vv)[kStage], int base, int w,
                                           int lane, const TriDev<T>& F, bool act) {
#pragma unroll
  for (int j = 0; j < kWave; ++j) tile[j * kWave + lane] = 0;
  for (int u0 = 0;;) {
#pragma unroll
    for (int u = 0; u < kStage; ++u) tile[(jj[u] >= 0 ? jj[u] : lane) * kWave + lane] = jj[u] >= 0 ? vv[u] : (T)0;
    u0 += kStage;
    if (u0 >= w) break;
    load_in(jj, vv, u0, w, base, lane, F, act);
  }
}

// Off-chunk batches end at the last slot, so the last batch holds every
// row's latest entries; the first may start before slot 0 (those read
// padding).  With w a multiple of kColGroup every batch starts on a group.
__device__ __forceinline__ int first_batch(int w) { return w - (w + kTriBatch - 1) / kTriBatch * kTriBatch; }

template <typename T>
__device__ __forceinline__ void load_batch_cols(int (&c)[kTriBatch], int u0, const TriMeta& m, int lane,
                                                const TriDev<T>& F, bool act) {
  load_cols<kTriBatch>(c, u0, m.off_w, m.off_ptr, F.off_pad, lane, F.off_col, act);
}

// The solution vector as a buffer resource of n entries: a gather of a
// padding column (stored as n) falls outside it and reads 0 without a memory
// access, and each gather needs only a 32-bit offset.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const T* y, int n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(y), (short)0, n * (int)sizeof(T), 0x00020000);
}
__device__ __forceinline__ double ld_buf(__amdgpu_buffer_rsrc_t r, int col, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, col * 8, 0, 0));
}
__device__ __forceinline__ float ld_buf(__amdgpu_buffer_rsrc_t r, int col, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, col * 4, 0, 0));
}

// One off-chunk batch, slots u0 .. u0 + kTriBatch - 1: gathers y for the
// columns in cc, loads the batch's values and the next batch's columns (into
// cn), then subtracts the batch in slot order.  The values load with the
// gathers rather than a batch ahead: the batch waits for the next columns'
// memory round trip anyway, and the registers they would hold keep the
// gather's state out of the accumulation registers.  The first gathers are
// plain loads: within one solve an entry only ever changes from the marker to
// its final value, so a cached copy is either final or the marker.  The batch
// is summed first; only if the sum is a NaN (some entry still the marker, or
// a NaN in the data) are the marker entries reloaded with device-scope loads
// until they are final (only those lanes load), and the batch summed again
// from the same start, so the result does not depend on which path was taken.
template <typename T>
__device__ __forceinline__ T gather_batch(T t, const int (&cc)[kTriBatch], int (&cn)[kTriBatch], int u0,
                                          const TriMeta& m, int lane, const TriDev<T>& F, const T* y,
                                          __amdgpu_buffer_rsrc_t yr, const TriCtl& ctl) {
  const bool act = lane < m.nrow;
  T yy[kTriBatch];
#pragma unroll
  for (int u = 0; u < kTriBatch; ++u) yy[u] = ld_buf(yr, cc[u], T());
  T aa[kTriBatch];
  load_vals<T, kTriBatch>(aa, u0, m.off_w, m.off_ptr, F.off_pad, lane, F.off_val, act);
  load_batch_cols(cn, u0 + kTriBatch, m, lane, F, act);
  T s = t;
#pragma unroll
  for (int u = 0; u < kTriBatch; ++u) s -= aa[u] * yy[u];  // padding: 0 * 0
  if (__ballot(s != s) == 0) return s;
  // The fault word is reloaded with the pending entries, so checking it adds
  // no round trip; after poll_limit polls, or once another wave has set it,
  // the wave stops waiting and its sums turn NaN (the marker is a NaN), which
  // it stores as a quiet NaN, so no later wave waits on it either.
  unsigned fault = 0;
  for (int polls = 0;; ++polls) {
    bool pend = false;
#pragma unroll
    for (int u = 0; u < kTriBatch; ++u) pend |= pending(yy[u]);
    if (__ballot(pend) == 0) break;
    if (polls >= ctl.poll_limit || __builtin_amdgcn_readfirstlane((int)fault) != 0) {
      st_dev(ctl.fault, 1u);
      break;
    }
    __builtin_amdgcn_s_sleep(2);
#pragma unroll
    for (int u = 0; u < kTriBatch; ++u)
      if (pending(yy[u])) yy[u] = ld_dev(y + cc[u]);
    fault = ld_dev(ctl.fault);
  }
#pragma unroll
  for (int u = 0; u < kTriBatch; ++u) t -= aa[u] * yy[u];
  return t;
}

// t -= sum over the off-chunk slots of this lane of val * y[col], batch by
// batch in slot order.  The first batch's columns (from first_batch) were
// loaded into cc by the caller; the two column sets take turns as current and
// next batch, so none is copied.  A row's entries fill its last slots, so the
// entries that become final last all sit in the last batch and, once they
// arrive, no further batch has to be loaded.
template <typename T>
__device__ __forceinline__ T gather_off(T t, int (&cc)[kTriBatch], const TriMeta& m, int lane,
                                        const TriDev<T>& F, const T* y, const TriCtl& ctl) {
  const __amdgpu_buffer_rsrc_t yr = vec_rsrc(y, F.n);
  int cn[kTriBatch];
  for (int u0 = first_batch(m.off_w);;) {
    t = gather_batch(t, cc, cn, u0, m, lane, F, y, yr, ctl);
    u0 += kTriBatch;
    if (u0 >= m.off_w) break;
    t = gather_batch(t, cn, cc, u0, m, lane, F, y, yr, ctl);
    u0 += kTriBatch;
    if (u0 >= m.off_w) break;
  }
  return t;
}

// Rows inside the chunk, first to last: after step j the value of row j
// (lane j) is final and is subtracted, times column j of the tile, from the
// later rows.  Lanes past the chunk's end hold zeros and change nothing.
template <typename T>
__device__ __forceinline__ T serial_forward(T t, const T* tile, int lane) {
#pragma unroll
  for (int j0 = 0; j0 < kWave; j0 += 16) {
    T cf[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) cf[u] = tile[(j0 + u) * kWave + lane];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (j0 + u < kWave - 1) t -= cf[u] * lane_bcast(t, j0 + u);
  }
  return t;
}

// Rows inside the chunk, last to first, on undivided partial sums (the tile
// holds U_ij / U_jj).
template <typename T>
__device__ __forceinline__ T serial_backward(T t, const T* tile, int lane) {
#pragma unroll
  for (int j0 = kWave - 16; j0 >= 0; j0 -= 16) {
    T cf[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) cf[u] = tile[(j0 + u) * kWave + lane];
#pragma unroll
    for (int u = 15; u >= 0; --u)
      if (j0 + u > 0) t -= cf[u] * lane_bcast(t, j0 + u);
  }
  return t;
}

// y = L^{-1} P r, L unit lower, P the ILUT ordering ((P r)_i = r[perm[i]]).
// y must hold kPending in every entry at launch.
template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void trisolve_lower(
    int nq, TriDev<T> F, const int* __restrict__ perm, const T* __restrict__ r, T* y, TriCtl ctl) {
  __shared__ T tile[kWave * kWave];
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int tk = wave_ticket(ctl.state);
    if (tk >= nq) break;
    const TriMeta m = ld_meta(F.meta + tk);
    const int row = m.row0 + lane;
    const bool act = lane < m.nrow;
    // every independent load of the chunk first
    const int pr = perm[act ? row : row - lane];  // lanes past the end read the chunk's first row
    int cc[kTriBatch];
    load_batch_cols(cc, first_batch(m.off_w), m, lane, F, act);
    int jj[kStage];
    T vv[kStage];
    load_in(jj, vv, 0, m.in_w, m.in_ptr, lane, F, act);
    T t = r[pr];
    t = act ? t : (T)0;
    stage_tile(tile, jj, vv, m.in_ptr, m.in_w, lane, F, act);
    t = gather_off(t, cc, m, lane, F, y, ctl);
    t = serial_forward(t, tile, lane);
    if (act) st_dev(y + row, publishable(t));
  }
  finish_grid(ctl.state, lane);
}

// e = U^{-1} y (diagonal in F.diag) and x += P^T e.  e must hold kPending in
// every entry at launch; y is only read.
template <typename T>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void trisolve_upper(
    int nq, TriDev<T> F, const int* __restrict__ perm, const T* __restrict__ y, T* e, T* __restrict__ x,
    TriCtl ctl) {
  __shared__ T tile[kWave * kWave];
  const int lane = threadIdx.x & 63;
  for (;;) {
    const int tk = wave_ticket(ctl.state);
    if (tk >= nq) break;
    const TriMeta m = ld_meta(F.meta + tk);
    const int row = m.row0 + lane;
    const bool act = lane < m.nrow;
    const int ra = act ? row : row - lane;  // lanes past the end read the chunk's first row
    const T t0 = y[ra];
    const T d0 = F.diag[ra];
    const int pr = perm[ra];
    int cc[kTriBatch];
    load_batch_cols(cc, first_batch(m.off_w), m, lane, F, act);
    int jj[kStage];
    T vv[kStage];
    load_in(jj, vv, 0, m.in_w, m.in_ptr, lane, F, act);
    const T xv = x[pr];  // each entry of x is updated by one row only
    stage_tile(tile, jj, vv, m.in_ptr, m.in_w, lane, F, act);
    T t = act ? t0 : (T)0;
    const T dg = act ? d0 : (T)1;
    t = gather_off(t, cc, m, lane, F, (const T*)e, ctl);
    t = serial_backward(t, tile, lane);
    const T ev = t / dg;
    if (act) {
      st_dev(e + row, publishable(ev));
      x[pr] = xv + ev;
    }
  }
  finish_grid(ctl.state, lane);
}

}  // namespace pmg
