// Internal device-side structures shared by the C ABI (pmg_device.hip) and
// the request server (pmg_serve.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pmg.h"
#include "tri_layout.hpp"
#include "grid_layout.hpp"
#include "pmg_host.hpp"

namespace pmgdev {

// thread-local error detail behind pmg_last_error()
void set_error(const std::string& msg);
pmg_status fail(pmg_status s, const std::string& msg);
pmg_status hip_fail(hipError_t e, const char* what);
const char* last_error_cstr();

#define PMG_HIP_OK(call)                                        \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return pmgdev::hip_fail(e_, #call);   \
  } while (0)

// Device allocations owned together and released together.
struct DevArena {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename T>
  pmg_status alloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    ptrs.push_back(*p);
    bytes += count * sizeof(T);
    return PMG_OK;
  }
  template <typename T>
  pmg_status upload(T** p, const T* src, size_t count) {
    pmg_status s = alloc(p, count);
    if (s) return s;
    if (count) PMG_HIP_OK(hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice));
    return PMG_OK;
  }
  void release() {
    for (void* q : ptrs) hipFree(q);
    ptrs.clear();
    bytes = 0;
  }
};

struct DevMat {
  int nrows = 0, ncols = 0;
  int64_t nnz = 0;
  int* rp = nullptr;
  int* ci = nullptr;
  double* v = nullptr;
  float* v32 = nullptr;
  int G = 8;
};

// A_{h,p} in stencil layout (pmg::stencil_resid), used instead of CSR when
// it reads fewer bytes.
struct DevStencil {
  int dim = 0, p = 0, nx = 0, ny = 0, S = 0;  // S = (2p+1)^dim offsets
  double* v = nullptr;
  float* v32 = nullptr;
  double* kK = nullptr;  // Kronecker factors (pmg::kron_resid) instead of v
  double* kM = nullptr;
};

// A transfer between the degree-p and degree-1 grids in stencil layout
// (pmg::xgrid_spmv); v == nullptr: CSR is used.
struct DevXStencil {
  int nxr = 0, nxc = 0, o = 0, W = 0;
  double* v = nullptr;
  float* v32 = nullptr;
  double* tab = nullptr;  // Kronecker factor (pmg::kron_xgrid) instead of v: nxr x W
};

// Schedule and chunk-sliced factor of one triangular solve (see TriDev).
struct TriSched {
  int nrows = 0, nseg = 0, seg_len = 0, dag_levels = 0, chunk_levels = 0;
  std::vector<int32_t> seg_start;  // first row of each segment, then nrows
  int nch = 0;  // chunks in all
  int grid64 = 1, grid32 = 1;  // persistent waves per launch (all resident)
  // all by natural chunk index
  std::vector<int> chunk_row, chunk_len;  // first row and rows of each chunk
  std::vector<int> wptr, deps, order;     // chunks read by each chunk; ticket -> chunk
  std::vector<int> off_ptr, off_w, off_col, in_ptr, in_w, in_j;
  std::vector<double> off_val, in_val, diag;
  int64_t slots = 0;  // stored off-chunk slots (entries + padding)
  int off_pad = 0, in_pad = 0;  // start of the 64 padding entries
  pmg::TriDev<double> dev64{};
  pmg::TriDev<float> dev32{};
};

// Everything one solve in flight writes: vectors, norm partials, the
// triangular-solve counters.  Several workspaces may use one operator set
// concurrently on different streams.
struct Workspace {
  DevArena mem;
  int n = 0, n1 = 0;
  // y, e: outputs of the lower and upper triangular solves
  double *y = nullptr, *e = nullptr, *r = nullptr, *r1 = nullptr, *e1 = nullptr, *partial = nullptr,
         *scalar = nullptr;
  double *b = nullptr, *x = nullptr;  // request vectors (server slots only)
  double* host_scalar = nullptr;      // pinned
  std::vector<double*> hb, he, hr;
  unsigned* tickets = nullptr;  // pmg::kTicketAlloc words: lower and upper solve counters, fault word
  float *r32 = nullptr, *c32 = nullptr, *y32 = nullptr, *e32 = nullptr, *t32 = nullptr, *q32 = nullptr;
  bool mixed = false;
  // BiCGSTAB (pmg_bicgstab): shadow residual, direction, A y, preconditioned
  // vectors, A z, a residual scratch for the preconditioner, the device
  // scalars (see pmg::bicg_*), block partials and a pinned host copy
  double *bc_rh = nullptr, *bc_p = nullptr, *bc_v = nullptr, *bc_y = nullptr, *bc_z = nullptr, *bc_t = nullptr,
         *bc_w = nullptr, *bc_S = nullptr, *bc_pa = nullptr, *bc_pb = nullptr, *bc_host = nullptr;
  // conjugate gradients of the consistent-mass transfers: residual, preconditioned
  // residual, direction, M p, the transferred right-hand side and solution,
  // block partials and a pinned host copy of them
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr, *cg_t = nullptr, *cg_y = nullptr,
         *cg_pa = nullptr, *cg_pb = nullptr, *cg_host = nullptr;
  // cached graph of one outer step (outer_step), captured on `cap` and valid
  // for the handle and vectors it was captured with
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec = nullptr;
  const void* gkey[5] = {};
  bool graph_failed = false;
  ~Workspace() {
    if (gexec) hipGraphExecDestroy(gexec);
    if (cap) hipStreamDestroy(cap);
    mem.release();
    if (host_scalar) hipHostFree(host_scalar);
    if (bc_host) hipHostFree(bc_host);
    if (cg_host) hipHostFree(cg_host);
  }
};

}  // namespace pmgdev

struct pmg_handle_s {
  pmg_problem prob{};
  pmg_options opt{};
  pmg_handle_s* sub = nullptr;  // indirect projection: the degree p-1 level (owned)
  pmg::HostOps H;
  int device = -1;
  bool on_device = false;
  int colors = 4;
  pmgdev::DevArena ops;  // operators (read-only during solves)
  pmgdev::DevMat A, L, U, R, P;
  pmgdev::DevMat Mp, M1;  // consistent masses (mass_transfer = consistent)
  pmgdev::DevStencil As;  // A in stencil layout (As.v == nullptr: CSR is used)
  int a_stencil = 0;      // offsets of that layout, 0 if CSR is used
  bool a_kron = false;    // residual from the Kronecker factors (As.kK, As.kM)
  bool x_kron = false;    // p-transfers from their Kronecker factor (Rs.tab, Ps.tab)
  pmgdev::DevXStencil Rs, Ps;  // P_p^1 and P_1^p in stencil layout
  std::vector<pmgdev::DevMat> A1, Ph, Rh;
  std::vector<pmg::GridLevel> grid;  // degree-1 levels in stencil layout (empty: CSR path)
  int l_lds = -1;                    // levels l_lds.. run in one workgroup from LDS (-1: none)
  size_t lds_bytes = 0;              // its dynamic LDS
  std::vector<std::vector<int*>> color_rows;
  std::vector<std::vector<int>> color_cnt;
  double *f = nullptr, *mlp_inv = nullptr, *ml1_inv = nullptr, *coarse_inv = nullptr;
  float *mlp_inv32 = nullptr, *ml1_inv32 = nullptr;
  int* d_perm = nullptr;
  pmgdev::TriSched tl, tu;
  int partial_cap = 0;
  pmgdev::Workspace ws;  // the workspace of the single-handle entry points
  pmg_info info{};
  // per-step event timing
  bool profiling = false;
  std::vector<hipEvent_t> ev[PMG_PROF_NCLASS];
  size_t ev_used[PMG_PROF_NCLASS] = {};
  void prof_mark(int cls, hipStream_t st) {
    auto& v = ev[cls];
    size_t& u = ev_used[cls];
    if (u >= v.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      v.push_back(e);
    }
    hipEventRecord(v[u], st);
    ++u;
  }
  ~pmg_handle_s();
};

namespace pmgdev {

// Workspace for one solve on handle h (mixed: FP32 vectors as well).  Its
// counters are cleared by a kernel on `st`; work later enqueued on `st` is
// ordered after that (with st == nullptr the device is synchronised).
pmg_status alloc_workspace(pmg_handle h, Workspace& ws, bool mixed, bool request_vectors,
                           hipStream_t st = nullptr);
// ILUT(tau, m) of Ap (rows in factorisation order, columns ascending) on the
// current device, with the host factorisation's arithmetic (identical
// factors).  OK with L (strict lower) and U (diagonal first) on the host;
// EZEROPIVOT with bad_row; EINVAL (reason in why) when the rows are too long
// for the device kernel or the fill is unlimited, the caller then factoring
// on the host; EDEVICE on a HIP error or a wait past the poll bound.
// order: pmg::factor_ticket_order of the problem (rows after their dependencies).
pmg_status ilut_device(const pmg::Csr& Ap, const std::vector<int32_t>& order, double tau, double fill, int mode,
                       int poll_limit, pmg::Csr& L, pmg::Csr& U, int& bad_row, std::string& why);
// Checks a problem description (sizes, kinds, knot vectors, callback); false
// with the reason in msg.
bool valid_problem(const pmg_problem* p, std::string& msg);
// p[0..n) = 0 on stream st
void zero(double* p, int64_t n, hipStream_t st);
// Bytes a workspace of h would take.
size_t workspace_bytes(pmg_handle h, bool mixed, bool request_vectors);

// Solve-phase steps on stream st with workspace ws.
void residual64(pmg_handle h, Workspace& ws, const double* b, const double* x, double* r, bool norm,
                hipStream_t st);
// final_resid = false leaves r stale after the last smoothing step (a
// V-cycle used as a preconditioner needs only x).
void vcycle64(pmg_handle h, Workspace& ws, const double* b, double* x, double* r, bool norm, hipStream_t st,
              bool final_resid = true);
// One defect-correction step: r (FP64 residual, in ws.r) -> FP32 V-cycle ->
// x += c -> r = b - A x and its norm (device scalar).
void mixed_step(pmg_handle h, Workspace& ws, const double* b, double* x, hipStream_t st);
// Enqueues the copy of the last norm^2 into ws.host_scalar[0] and of the
// triangular solves' fault word into ws.host_scalar[1] (enqueue_fault_readback).
void enqueue_norm_readback(Workspace& ws, hipStream_t st);
void enqueue_fault_readback(Workspace& ws, hipStream_t st);
// After the stream has passed the readback: EDEVICE (with a message) if a
// triangular solve of ws stopped at its poll bound, and then the word is
// cleared on st; PMG_OK otherwise.
pmg_status take_fault(Workspace& ws, hipStream_t st);
// One outer step of the solve on st: the FP64 V-cycle (vcycle64 with b, x,
// r, norm) or, with mixed, the defect-correction step (mixed_step; r is
// ws.r and the norm is always taken).  With the handle's graphs option the
// step's kernels are captured once into a HIP graph cached in ws (keyed by
// the handle, the kind of step and the vectors) and replayed; while
// profiling, or if capture fails, they are launched one by one.
void outer_step(pmg_handle h, Workspace& ws, bool mixed, const double* b, double* x, double* r, bool norm,
                hipStream_t st);

}  // namespace pmgdev
