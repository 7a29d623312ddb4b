/*
 * pmg.h -- C ABI of the MI355X p-multigrid library.
 *
 * Solves the B-spline Galerkin (isogeometric) discretisation of Poisson's
 * equation -Lap u = f with homogeneous Dirichlet conditions by the
 * p-multigrid method with an ILUT smoother of Tielen, Moeller, Goeddeke and
 * Vuik (arXiv:1901.01685):
 *   - problem statement: Section 2 (model problem, B-spline basis, geometry
 *     map F, Galerkin system A_{h,p} u = f_{h,p}); benchmarks 1 (quarter
 *     annulus) and 4 (unit cube), and the unit square;
 *   - solve phase: Section 3 (two-grid correction steps 1-5, V-cycle with
 *     direct projection to p = 1, lumped L2 transfers, ILUT smoothing,
 *     h-multigrid coarse solve) and Section 5 (stand-alone solver protocol).
 *
 * Conventions (every entry point):
 *   - Vectors b, x, r, r1, e1 are DEVICE pointers (hipMalloc'd or torch CUDA
 *     tensors) to FP64 arrays owned by the caller.  Degree-p vectors have
 *     length info.n, degree-1 vectors length info.n1.  Unknowns are the
 *     interior tensor B-splines (boundary functions eliminated), numbered
 *     0-based with x fastest: i = ix + n*iy (+ n*n*iz), n = n_elem + p - 2.
 *   - stream is a hipStream_t (NULL = the null stream).  Calls are ordered
 *     on that stream; pmg_solve and any call returning a norm synchronise it.
 *   - A handle owns all device operators and work buffers; it is used by one
 *     host thread at a time, and calls on one handle must not overlap.
 *   - Errors are return codes; nothing is thrown across the ABI.  A
 *     thread-local message is available from pmg_last_error().  On a failed
 *     pmg_setup *out is set to NULL.
 */
#ifndef PMG_H
#define PMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmg_handle_s *pmg_handle;

typedef enum {
  PMG_OK = 0,
  PMG_EINVAL = 1,     /* invalid argument or unsupported configuration */
  PMG_ENOMEM = 2,     /* host or device allocation failed */
  PMG_EDEVICE = 3,    /* HIP runtime error, no device for a device call, or a
                         triangular solve or device ILUT row that stopped at its
                         poll bound (see pmg_options.poll_limit) */
  PMG_EZEROPIVOT = 4, /* ILUT met a zero or non-finite pivot */
  PMG_EDIVERGED = 5,  /* relative residual above the divergence ratio */
  PMG_EMAXIT = 6,     /* max_iter V-cycles without reaching tol */
  PMG_ENAN = 7,       /* non-finite initial residual (NaN/Inf in b or x) */
  PMG_EBUDGET = 8     /* device-memory budget exceeded (serving) */
} pmg_status;

enum { PMG_GEOM_BOX = 0, PMG_GEOM_QUARTER_ANNULUS = 1 };
enum { PMG_RHS_SINE = 0, PMG_RHS_ANNULUS = 1, PMG_RHS_CALLBACK = 2 };
enum { PMG_PDE_POISSON = 0, PMG_PDE_CDR = 1 };
enum { PMG_MASS_LUMPED = 0, PMG_MASS_CONSISTENT = 1 };
enum { PMG_PROJ_DIRECT = 0, PMG_PROJ_INDIRECT = 1 };
enum { PMG_FP64 = 0, PMG_FP32_IN_FP64 = 1 };
enum { PMG_LIMIT_PER_PART = 0, PMG_LIMIT_PER_ROW = 1, PMG_LIMIT_HALF_PER_PART = 2 };
enum { PMG_GS_MULTICOLOR = 0 };
enum { PMG_ORDER_NATURAL = 0, PMG_ORDER_NESTED_DISSECTION = 1 };

/* The problem (Section 2): -div(D grad u) + v.grad u + R u = f on
 * Omega = F((0,1)^dim), u = 0 on the boundary, discretised with tensor
 * B-splines of degree `degree` on the open uniform knot vector with n_elem
 * elements per direction (h = 1/n_elem).
 *   pde PMG_PDE_POISSON: D = I, v = 0, R = 0 (benchmarks 1 and 4);
 *   pde PMG_PDE_CDR (dim 2, unit square, rhs_kind sine): benchmark 2,
 *     D = [1.2 -0.7; -0.4 0.9], v = (0.4, -0.2), R = 0.3, a non-symmetric
 *     operator at every level; the sine right-hand side is then this
 *     operator applied to u = sin(k1 pi x) sin(k2 pi y).
 *   geometry PMG_GEOM_BOX: unit square / cube (F = identity);
 *   geometry PMG_GEOM_QUARTER_ANNULUS (dim 2): radii 1 and 2, F(xi, eta) =
 *     (1 + xi) C(eta), C the rational quadratic quarter circle (benchmark 1).
 *   rhs_kind PMG_RHS_SINE: f = pi^2 (sum_a k_a^2) prod_a sin(k_a pi x_a),
 *     k = freq[0..dim-1] (manufactured u = prod sin(k_a pi x_a));
 *   rhs_kind PMG_RHS_ANNULUS: f = -Lap u for benchmark 1's
 *     u = -(x^2+y^2-1)(x^2+y^2-4) x y^2;
 *   rhs_kind PMG_RHS_CALLBACK: f is the caller's function `f` (any pde and
 *     geometry); the load vector f_i = int f Phi_i is integrated element by
 *     element with (p+1)^dim Gauss points per element through the geometry
 *     map, f evaluated at the physical points.
 * Knot vectors (Section 2, "B-spline basis functions": the knot vector Xi of
 * each direction): knots[a] may point to the caller's knot vector of
 * direction a, length n_elem + 2 degree + 1 (host memory, read during the
 * call only), or be NULL for the open uniform one.  The solve phase is built
 * for the paper's meshes, so a given vector must be that one: degree + 1
 * zeros, the interior knots i / n_elem (to 1e-12), degree + 1 ones; any
 * other vector (graded, periodic, repeated interior knots) is EINVAL with a
 * message saying which knot differs. */
typedef double (*pmg_fn)(const double *x, void *ctx); /* f at the physical point x[0..dim-1] */
typedef struct {
  int32_t dim;      /* 2 or 3 */
  int32_t degree;   /* p >= 1 (polynomial degree, C^{p-1} splines) */
  int32_t n_elem;   /* elements per direction, >= 2 */
  int32_t geometry; /* PMG_GEOM_* */
  int32_t rhs_kind; /* PMG_RHS_* */
  int32_t freq[3];  /* sine frequencies (>= 1) */
  int32_t pde;      /* PMG_PDE_* (0: Poisson) */
  const double *knots[3]; /* per direction: NULL or the open uniform knot vector (see above) */
  pmg_fn f;         /* rhs_kind PMG_RHS_CALLBACK: called on the calling thread during
                       pmg_setup / pmg_server_submit only, one point at a time */
  void *f_ctx;      /* passed to f unchanged */
} pmg_problem;

/* Solver options.  Defaults (pmg_default_options) are the paper's constants
 * (Section 3: tau = 1e-12, m = 1, two h-multigrid V-cycles as the p = 1
 * solve; Section 5: nu1 = nu2 = 1, divergence above 1e10). */
typedef struct {
  double ilut_tau;          /* ILUT drop tolerance tau (rule 1) */
  double ilut_fill;         /* ILUT fill factor m (rule 2); <= 0: unlimited */
  int32_t ilut_limit_mode;  /* ILUT rule 2, M = floor(m nnz(A) / n): PMG_LIMIT_PER_PART
                               (default: the M largest of the strict lower and of the strict
                               upper part, as in the cited ILUT; the only reading that
                               converges on every configuration of Table 4), PMG_LIMIT_PER_ROW
                               (M largest of the whole row) or PMG_LIMIT_HALF_PER_PART
                               (floor(M/2) in each part) */
  int32_t nu1, nu2;         /* pre/post ILUT smoothing steps */
  int32_t coarse_cycles;    /* h-multigrid V-cycles at p = 1 */
  int32_t coarse_min_elems; /* direct solve once n_elem <= this (or odd) */
  int32_t gs_variant;       /* PMG_GS_MULTICOLOR */
  int32_t precision;        /* PMG_FP64 or PMG_FP32_IN_FP64 (defect correction) */
  int32_t max_iter;         /* V-cycles (outer steps in mixed precision) */
  double diverge_ratio;     /* PMG_EDIVERGED above this relative residual */
  int32_t device;           /* HIP device ordinal; -1 = host-only setup (export) */
  int32_t setup_threads;    /* host threads for setup; 0 = hardware concurrency */
  int32_t ordering;         /* ILUT permutation: PMG_ORDER_* (default nested dissection) */
  int32_t nd_leaf;          /* nested dissection: lines per undivided block (default 8) */
  int32_t graphs;           /* 1 (default): each outer step of pmg_vcycle / pmg_solve is
                               enqueued as a cached HIP graph; 0: kernel by kernel */
  int32_t tiled_gs;         /* 1 (default): on 2-D degree-1 levels the Gauss-Seidel sweeps
                               before the restriction run with the residual and the
                               restriction as one tiled launch, and the prolongation with
                               the sweeps after it (up to 2 sweeps each); 0: one launch
                               per colour and per transfer.  Results are identical. */
  int32_t mass_transfer;    /* PMG_MASS_LUMPED (default, Section 3): the transfers divide by
                               the row-sum lumped masses; PMG_MASS_CONSISTENT (Appendix B):
                               they solve with the consistent interior mass matrices M_1 and
                               M_p instead (conjugate gradients preconditioned by the lumped
                               masses, to 1e-13 relative).  Consistent: FP64 only, and the
                               steps run kernel by kernel (graphs off), as the inner solves
                               test convergence on the host. */
  int32_t projection;       /* PMG_PROJ_DIRECT (default, Section 3): transfers between degree p
                               and the degree-1 space; PMG_PROJ_INDIRECT (Appendix A): degree p
                               transfers to degree p-1 on the same mesh and its coarse
                               correction is one V-cycle (ILUT smoothing) of an internal
                               degree-(p-1) handle, recursively down to degree 2, whose coarse
                               space is degree 1 with the h-multigrid.  Setup builds one
                               operator, ILUT factorisation and transfer per degree. */
  int32_t poll_limit;       /* bound on the polls of one wave of a triangular solve waiting
                               for one batch of entries (0: the default, 1 << 22, seconds of
                               waiting).  A wave that reaches it marks the solve as faulted
                               and stops waiting, and so does every other wave of the solve:
                               the kernels always end.  The next call that synchronises
                               (pmg_residual or pmg_vcycle with a norm, pmg_solve,
                               pmg_bicgstab, a server step) returns PMG_EDEVICE, and the
                               results since the previous such call are invalid.  A
                               correct schedule never reaches the default bound; small
                               values force the fault path (test hook).  The same bound
                               applies to a row of the device ILUT waiting for an earlier
                               row of U (default there 1 << 26): pmg_setup then returns
                               PMG_EDEVICE and builds no handle. */
  int32_t ilut_on_device;   /* 1 (default): ILUT is factored on the device (one wave per row,
                               rows of independent nested-dissection blocks side by side), with
                               the host factorisation's arithmetic, so the factors are
                               identical.  Problems the kernel does not take (fill <= 0, more
                               than 767 entries per row of U, working rows beyond its largest
                               tables) are factored on the host (reported in
                               pmg_info.ilut_on_device).  0: on the host threads. */
  int32_t tri_waves_per_cu; /* waves per compute unit of the triangular solves' persistent
                               grid; 0 (default): as many as fit at once */
  int32_t segment_rows;     /* the triangular-solve schedules cut the rows into segments,
                               runs of whole grid lines inside one block of the nested
                               dissection holding at most this many rows (one line at
                               least), and each segment into chunks of 64 rows; 0 (default):
                               one line per segment when a line holds 64 rows or more,
                               otherwise up to 512 rows */
  int32_t kron_residual;    /* 1 (default): on the unit box the residual (Poisson, degree
                               <= 5) forms A's coefficients from the 1-D stiffness and mass
                               factors of its Kronecker sum, and the p-transfers (lumped
                               masses) form theirs from the 1-D factor of theirs, instead of
                               reading them (the assembled values, bit for bit); 0: the
                               stencil layouts */
} pmg_options;

typedef struct {
  int32_t status;     /* pmg_status of the solve */
  int32_t iterations; /* V-cycles (FP64) or outer defect-correction steps */
  double r0;          /* ||b - A x0||_2 */
  double relres;      /* final ||b - A x||_2 / r0, FP64 */
  double seconds;     /* wall time of the solve on the host clock */
} pmg_result;

typedef struct {
  int64_t n, n1;              /* unknowns at degree p and at p = 1 */
  int64_t nnz_a, nnz_l, nnz_u, nnz_r, nnz_p;
  int32_t nlev;               /* levels of the p = 1 hierarchy incl. the direct one */
  int32_t n_coarsest;         /* unknowns of the direct solve */
  int64_t nnz_a1;             /* nnz of the finest p = 1 operator */
  int32_t segments;           /* segments of the triangular-solve schedule (pmg_options.segment_rows) */
  int32_t seg_len;            /* rows per grid line */
  int32_t dag_levels_l, dag_levels_u; /* depth of the L and U dependency DAGs (rows) */
  int32_t chunks_l, chunks_u;             /* chunks of the triangular-solve schedules */
  int32_t chunk_levels_l, chunk_levels_u; /* depth of their chunk dependency graphs */
  int64_t bytes_vcycle;       /* algorithmic HBM bytes of one FP64 V-cycle */
  int64_t bytes_spmv, bytes_trisolve_l, bytes_trisolve_u, bytes_restrict, bytes_prolong,
      bytes_coarse;           /* per step, each operator counted in the layout its kernels read
                                 (1-D factors, stencil slots or CSR) and every vector once */
  int64_t device_bytes;       /* device memory held by the handle */
  double t_assembly, t_ilut, t_upload; /* setup phase times, seconds */
  double t_schedule;          /* triangular-solve schedules and sliced layouts (host), seconds */
  int32_t ilut_on_device;     /* 1 if the ILUT factors were computed on the device */
  int32_t residual_layout;    /* how the residual reads A: 0 CSR, 1 stencil layout, 2 Kronecker
                                 factors (pmg_options.kron_residual) */
  int32_t transfer_layout;    /* the same for the p-transfers R and P */
  int32_t resid_rows;         /* rows in y that one thread of the residual kernels takes (4 on
                                 grids that still fill the device that way, else 1; 0 with CSR) */
  int32_t coarse_kron_levels; /* 2-D degree-1 levels whose tiled smoothing forms the operator's
                                 values from the 1-D stiffness and mass of the level (unit box,
                                 Poisson, pmg_options.kron_residual) instead of reading them */
} pmg_info;

/* ILUT ordering (Section 3, "Smoother": the factorisation follows a
 * fill-reducing permutation the paper does not name).  Unknowns are grouped
 * in grid lines along x; PMG_ORDER_NESTED_DISSECTION cuts the grid of lines
 * recursively across its longest side with separators p lines wide (the two
 * halves are then uncoupled), orders each half first and the separator
 * last, and keeps blocks of at most nd_leaf lines in natural order.  The
 * factors are those of P A P^T and one smoothing step is
 * x <- x + P^T U^{-1} L^{-1} P r. */

/* Fills *o with the defaults listed above. */
pmg_status pmg_default_options(pmg_options *o);

/* Setup (timed separately, not the hot path): host assembly of A_p, f_p,
 * the lumped masses M_p^L and M_1^L, the transfer matrix P_1^p (Section 3,
 * "Prolongation and restriction"), the rediscretised degree-1 hierarchy
 * ("Coarse grid operator"), ILUT(tau, m) of P A_p P^T with P the ordering of
 * o->ordering, nested dissection by default ("Smoother"), the
 * triangular-solve schedule, then upload to device
 * `o->device`.  With o->device == -1 nothing touches a GPU and only
 * pmg_get_info / pmg_export work.  o may be NULL (defaults).
 * Errors: EINVAL (bad problem/options), ENOMEM, EZEROPIVOT, EDEVICE. */
pmg_status pmg_setup(const pmg_problem *prob, const pmg_options *o, pmg_handle *out);

/* Operator injection (test hook): as pmg_setup, but the degree-p operator
 * A_{h,p} is the caller's n x n matrix instead of the assembled one, given in
 * host CSR (rp: n + 1 int64 row pointers from 0; ci: int32 columns, strictly
 * increasing within each row; v: values), copied during the call.  The ILUT
 * factors of the smoother are computed from it (Section 3, "Smoother"); the
 * transfers, the degree-1 hierarchy and the load vector still come from
 * prob.  n must equal the problem's number of unknowns.  Any sparsity is
 * accepted (entries outside the B-spline coupling pattern make the residual
 * use CSR).  Drives the solver into the branches of its status codes, e.g.
 * PMG_EZEROPIVOT for an operator with an empty row, PMG_EDIVERGED for -A.
 * Errors: as pmg_setup, and EINVAL for a wrong size or malformed CSR. */
pmg_status pmg_setup_from_csr(const pmg_problem *prob, int64_t n, const int64_t *rp, const int32_t *ci,
                              const double *v, const pmg_options *o, pmg_handle *out);

/* Releases every resource of h (device memory included).  NULL is a no-op. */
pmg_status pmg_destroy(pmg_handle h);

/* Copies the load vector f_{h,p} (Section 2) into b (device, length n). */
pmg_status pmg_rhs(pmg_handle h, double *b, void *stream);

/* Step a1: r = b - A_{h,p} x (Section 3, step 2 defect); if rnorm != NULL the
 * 2-norm of r is written there (host) and the stream is synchronised. */
pmg_status pmg_residual(pmg_handle h, const double *b, const double *x, double *r, double *rnorm,
                        void *stream);

/* Steps a2 + a3: one ILUT smoothing step (Section 3, "Smoother"):
 * x <- x + U^{-1} L^{-1} r, r given (normally b - A x).  r is not modified. */
pmg_status pmg_smooth(pmg_handle h, const double *r, double *x, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pmg_smooth
 * with its work vectors and counters in a static device array instead of the
 * handle's workspace.  Same kernels and results as pmg_smooth (bit for bit).
 * Limit: h's unknowns <= 2^21 (2,097,152); larger problems return EINVAL
 * (use pmg_smooth).  The array (32 MiB + 4 KiB) exists once per device for
 * the life of the process and is shared by every call on that device, so
 * calls that overlap on one device race (calls on one stream are ordered).
 * Allocates nothing: no hipMalloc, hipFree or allocating library call.  A
 * poll-bound fault is recorded in h and reported by the next synchronising
 * call on h, as for pmg_smooth.  r, x device, length n, distinct. */
pmg_status pmg_smooth_static(pmg_handle h, const double *r, double *x, void *stream);

/* Step a2 alone: y = L^{-1} r (forward substitution with the unit lower ILUT
 * factor, Section 3, "Smoother").  r, y device, length n, distinct. */
pmg_status pmg_lower_solve(pmg_handle h, const double *r, double *y, void *stream);

/* Step a3 alone: e = U^{-1} y (backward substitution with the upper ILUT
 * factor), written over y, and x <- x + P^T e (P the ILUT ordering).  y, x
 * device, length n. */
pmg_status pmg_upper_solve(pmg_handle h, double *y, double *x, void *stream);

/* Step a4: r1 = (M_1^L)^{-1} P_p^1 r (lumped L2 restriction, Section 3). */
pmg_status pmg_restrict(pmg_handle h, const double *r, double *r1, void *stream);

/* Step a5: e1 = coarse_cycles h-multigrid V-cycles on A_{h,1} e1 = r1 from
 * e1 = 0 (multicolour Gauss-Seidel, canonical transfers, direct solve on the
 * coarsest mesh; Section 3 and Figure 1).  r1, e1 device, length n1. */
pmg_status pmg_coarse(pmg_handle h, const double *r1, double *e1, void *stream);

/* Step a6: x <- x + (M_p^L)^{-1} P_1^p e1 (lumped L2 prolongation, Section 3). */
pmg_status pmg_prolong(pmg_handle h, const double *e1, double *x, void *stream);

/* One FP64 p-multigrid V-cycle (steps a1-a6): on entry r must hold b - A x
 * (e.g. from pmg_residual); on exit x is updated and r = b - A x.  If rnorm
 * != NULL, ||r||_2 is written there and the stream is synchronised. */
pmg_status pmg_vcycle(pmg_handle h, const double *b, double *x, double *r, double *rnorm,
                      void *stream);

/* Stand-alone solver (Section 5): V-cycles from the initial guess in x until
 * ||b - A x|| <= tol ||b - A x0|| (step a7).  With precision PMG_FP32_IN_FP64
 * each outer step is an FP32 V-cycle on the FP64 residual (defect
 * correction; outer residual, update and p = 1 solve in FP64).  x holds the
 * last iterate also on EDIVERGED / EMAXIT.  hist (host, may be NULL,
 * length max_iter + 1) receives ||r_k|| / ||r_0||.  res may be NULL.
 * Returns the solve status (also in res->status); ENAN if r0 is not finite;
 * r0 == 0 returns OK after 0 iterations. */
pmg_status pmg_solve(pmg_handle h, const double *b, double *x, double tol, pmg_result *res,
                     double *hist, void *stream);

/* BiCGSTAB on A u = f, right-preconditioned by one p-multigrid V-cycle (from
 * a zero initial guess) in each preconditioning phase (Section 5, the method
 * as a preconditioner of a Krylov solver suited to its non-symmetric coarse
 * correction; two V-cycles per iteration).  Textbook BiCGSTAB with shadow
 * residual r_0:
 *   rho = (r^, r); beta = (rho / rho_prev)(alpha / omega); p = r + beta (p - omega v)
 *   y = M^{-1} p; v = A y; alpha = rho / (r^, v); s = r - alpha v; x += alpha y
 *   z = M^{-1} s; t = A z; omega = (t, s)/(t, t) (0 if t = 0); x += omega z; r = s - omega t.
 * FP64 throughout; the method's scalars stay on the device and the host
 * reads ||r|| once per iteration.  Stops when ||r|| / ||r_0|| <= tol; hist
 * (host, length max_iter + 1, or NULL) receives that ratio per iteration.
 * Status as pmg_solve; a breakdown (rho = 0, or omega = 0 before
 * convergence) and a non-finite residual give PMG_EDIVERGED. */
pmg_status pmg_bicgstab(pmg_handle h, const double *b, double *x, double tol, pmg_result *res,
                        double *hist, void *stream);

/* Selects the precision of later pmg_solve calls on h: PMG_FP64 (plain FP64
 * V-cycles) or PMG_FP32_IN_FP64 (FP32 V-cycles in FP64 defect correction).
 * A handle set up with PMG_FP32_IN_FP64 holds both copies of its operators
 * and may switch either way; one set up in FP64 cannot switch to mixed
 * (EINVAL).  Lets one set of operators serve both forms of the solve. */
pmg_status pmg_set_precision(pmg_handle h, int32_t precision);

/* Sizes, DAG depths, algorithmic bytes and setup times. */
pmg_status pmg_get_info(pmg_handle h, pmg_info *info);

/* Host copies of setup operators (test hook).  which: 0 A_p, 1 L (strict
 * lower, permuted numbering), 2 U (diagonal first, permuted numbering), 3 P_p^1 (n1 x n), 4 P_1^p (n x n1),
 * 5 A_{2^k h,1} (level k), 6 canonical prolongation level k -> k+1.
 * dims[0..2] = rows, cols, nnz are always written; rp (rows+1), ci, v are
 * filled when non-NULL.  EINVAL for an unknown operator or level. */
pmg_status pmg_export(pmg_handle h, int32_t which, int32_t level, int64_t *dims, int64_t *rp,
                      int32_t *ci, double *v);

/* Host copies of setup vectors: 0 f_p (n), 1 M_p^L (n), 2 M_1^L (n1),
 * 3 inverse of the coarsest A_1 (n_coarsest^2, row-major). */
pmg_status pmg_export_vec(pmg_handle h, int32_t which, double *out);

/* The ILUT ordering: out[i] = unknown placed at position i (length n). */
pmg_status pmg_export_perm(pmg_handle h, int32_t *out);

/* Host copies of the schedule and chunk-sliced layout of a triangular solve
 * (test hook; layout of each field as the kernels read it).  factor: 0 lower,
 * 1 upper.  field: 0 chunk order (ticket -> chunk), 1 wptr and 2 deps (per
 * chunk, the chunks it reads), 3 off_ptr, 4 off_w, 5 off_col, 6 in_ptr,
 * 7 in_w, 8 in_j (int32 elements), 9 off_val, 10 in_val, 11 diag (double
 * elements; diag for the upper factor only), 12 chunk_row, 13 chunk_len
 * (first row and rows of each chunk, int32), 14 segment starts (first row
 * of each segment, then n; int32).  *count receives the number of
 * elements; out, when non-NULL, must hold that many.  Chunks are numbered
 * by first row.  EINVAL for an unknown factor or field. */
pmg_status pmg_export_schedule(pmg_handle h, int32_t factor, int32_t field, int64_t *count, void *out);

/* Per-step timing with HIP events recorded on the launch stream around each
 * step of the solve phase (classes below; the coarse class spans the whole
 * h-multigrid solve).  pmg_profile_enable(h, 1) synchronises the device,
 * clears the records and starts recording; 0 stops.  pmg_profile_read
 * waits for the recorded events and writes, per class, the total time in
 * milliseconds (ms[PMG_PROF_NCLASS]) and the number of timed launches
 * (count[PMG_PROF_NCLASS]). */
enum {
  PMG_PROF_RESIDUAL = 0,
  PMG_PROF_LOWER = 1,
  PMG_PROF_UPPER = 2,
  PMG_PROF_RESTRICT = 3,
  PMG_PROF_COARSE = 4,
  PMG_PROF_PROLONG = 5,
  PMG_PROF_NCLASS = 6
};
pmg_status pmg_profile_enable(pmg_handle h, int32_t on);
pmg_status pmg_profile_read(pmg_handle h, double *ms, int64_t *count);

const char *pmg_status_str(pmg_status s);
/* Detail of the last error on the calling thread ("" if none). */
const char *pmg_last_error(void);

/* ---------------------------------------------------------------------------
 * Request server: many Poisson solves of different classes (dim, degree,
 * n_elem, geometry) on one device, with continuous batching.  Each class's
 * operators and ILUT factors are set up once and stay resident while the
 * device-memory budget allows (least recently used idle classes are evicted).
 * A scheduler thread admits queued requests into slots as slots and memory
 * free up and advances every active request by one outer step per tick (one
 * FP32 V-cycle plus the FP64 residual in mixed precision, one FP64 V-cycle
 * otherwise), each slot on its own stream, so the work of concurrent
 * requests overlaps on the device.  Results do not depend on what else runs:
 * every reduction has a fixed order, and each slot has its own workspace.
 * The server object is thread-safe. */
typedef struct pmg_server_s *pmg_server;

typedef struct {
  int64_t budget_bytes;    /* device memory for operators and slot workspaces; 0 (default):
                              70 % of the device's memory (about 200 GB on an MI355X) */
  int64_t max_class_bytes; /* classes estimated above this are rejected; 0: budget/4 (with the
                              default budget this rejects the 3-D classes with n_elem = 256 and
                              those with n_elem = 128 at p >= 4) */
  int32_t max_slots;       /* requests in flight on the device */
  int32_t precision;       /* PMG_FP32_IN_FP64 (default) or PMG_FP64 */
  double tol;              /* relative FP64 residual target, default 1e-10 */
  int32_t max_iter;        /* outer steps per request, default 100 */
  int32_t device;          /* HIP device ordinal */
  int32_t setup_threads;   /* host threads per class setup; 0 = default */
  double diverge_ratio;    /* PMG_EDIVERGED above this relative residual, default 1e10 */
  int32_t tri_waves_per_cu; /* pmg_options.tri_waves_per_cu of every class handle: waves per
                               compute unit of each slot's triangular-solve grid; default 1,
                               so that the grids of several slots are resident together
                               (0: as many as fit, and the slots' grids take turns) */
} pmg_server_options;

typedef struct {
  int32_t status;     /* pmg_status of the solve */
  int32_t iterations; /* outer steps (V-cycles) */
  double relres;      /* final ||b - A x|| / ||b - A x0||, FP64, x0 = 0 */
  double t_submit, t_admit, t_finish; /* seconds on the server clock */
  int64_t n;          /* unknowns */
} pmg_request_info;

typedef struct {
  int64_t submitted, completed, rejected, failed, evictions;
  int32_t classes_resident, slots_active, queued;
  int64_t bytes_in_use;
  double setup_seconds; /* total host setup time of all classes so far */
} pmg_server_stats;

pmg_status pmg_server_default_options(pmg_server_options *o);
/* Starts the scheduler and setup threads.  Errors: EINVAL, EDEVICE. */
pmg_status pmg_server_create(const pmg_server_options *o, pmg_server *out);
/* Sets up the class of prob now (blocking) so that later requests find it
 * resident.  EBUDGET if the class can never fit (estimate above
 * max_class_bytes or the budget) or does not fit now. */
pmg_status pmg_server_prepare(pmg_server s, const pmg_problem *prob);
/* Queues one solve of prob with zero initial guess.  b_host (host, length n,
 * copied) is the right-hand side, or NULL for the load vector of prob's
 * rhs_kind and freq.  *ticket identifies the request.  EBUDGET at once if
 * the class can never fit; EINVAL for an invalid problem. */
pmg_status pmg_server_submit(pmg_server s, const pmg_problem *prob, const double *b_host, int64_t *ticket);
/* Blocks until the request is done; copies the solution into x_host (length
 * n) if non-NULL and its record into *info if non-NULL, then forgets the
 * ticket.  Returns the solve status; EINVAL for an unknown ticket. */
pmg_status pmg_server_wait(pmg_server s, int64_t ticket, double *x_host, pmg_request_info *info);
/* Non-blocking form of pmg_server_wait: *done = 0 and PMG_OK while the
 * request is queued or running; once it is done, *done = 1 and the call acts
 * as pmg_server_wait (copies, forgets the ticket, returns the solve status).
 * EINVAL for an unknown ticket or a NULL done. */
pmg_status pmg_server_poll(pmg_server s, int64_t ticket, int32_t *done, double *x_host, pmg_request_info *info);
/* Changes slots and precision; waits until no request is queued or active. */
pmg_status pmg_server_configure(pmg_server s, int32_t max_slots, int32_t precision);
pmg_status pmg_server_get_stats(pmg_server s, pmg_server_stats *st);
/* The options in force, with the defaults filled in (budget_bytes and
 * max_class_bytes as taken from the device at pmg_server_create). */
pmg_status pmg_server_get_options(pmg_server s, pmg_server_options *o);
/* Seconds since the server was created (the clock of pmg_request_info). */
double pmg_server_clock(pmg_server s);
/* Stops the threads (waiting for active requests) and frees everything. */
pmg_status pmg_server_destroy(pmg_server s);

#ifdef __cplusplus
}
#endif
#endif /* PMG_H */
