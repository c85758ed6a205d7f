/*
 * hlp.h -- restarted reflected Halpern PDHG for linear programming on one
 *          AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Problem (arXiv 2507.14051, Sec. 2.1, eq. (lp)):
 *
 *     min  c^T x   s.t.   lc <= A x <= uc,   lv <= x <= uv
 *
 * with A an m x n sparse matrix in CSR form and IEEE +-INFINITY for absent
 * bounds.  The solver is the paper's method: the PDHG step of eq. (pdhg)
 * (Sec. 2.2) with tau = eta/omega, sigma = eta*omega; reflected Halpern
 * anchoring (Sec. 3, "Halpern scheme", "Reflection"); restarts driven by the
 * fixed-point residual ||z - PDHG(z)||_P (Sec. 3, "Adaptive restart"); the
 * constant stepsize eta = 0.998/||A||_2 from power iteration (Sec. 3,
 * "Stepsize"); the PID update of the primal weight (Sec. 3, "Primal weight
 * update"); all-zero start and termination on the relative KKT error of the
 * original LP (Sec. 4).  Two extensions sit on the same kernels: an FP32
 * iteration with FP64 iterative refinement (HLP_MIXED) and the reverse mode
 * of K unrolled iterations (hlp_unrolled_forward / hlp_unrolled_backward).
 *
 * Conventions for every entry point:
 *   - Return value: HLP_OK (0) or a negative hlp_err.  No C++ exception
 *     crosses the ABI.  After a non-OK return, hlp_last_error() gives a
 *     message (thread-local, valid until the next call on the thread).
 *   - "device" pointers are HIP device memory on the current device;
 *     "host" pointers are ordinary host memory.  Sizes are element counts
 *     unless the name ends in _bytes.
 *   - Ownership: the caller owns every buffer.  The library allocates no
 *     device memory: all of its device state lives in the caller's
 *     workspace, sized by hlp_workspace_bytes().  The handle must not
 *     outlive the workspace.
 *   - Streams: all device work is enqueued on the hip_stream given to
 *     hlp_lp_create (a hipStream_t; NULL means the default stream).  Every
 *     entry point returns only after that stream has finished its work.
 *   - Calls on one handle must not overlap; distinct handles are independent.
 */
#ifndef HLP_H
#define HLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hlp_lp hlp_lp; /* opaque */

typedef enum {
  HLP_OK = 0,
  HLP_EINVAL = -1,       /* invalid argument or input data (message says which) */
  HLP_ENOMEM = -2,       /* workspace or tape too small */
  HLP_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  HLP_EUNSUPPORTED = -4  /* valid input outside what the library supports */
} hlp_err;

typedef enum {
  HLP_OPTIMAL = 0,     /* relative KKT error <= tol (Sec. 4) */
  HLP_ITER_LIMIT = 1,  /* max_iter iterations done */
  HLP_TIME_LIMIT = 2,  /* time_limit_s exceeded (Sec. 4, time limit) */
  HLP_NUMERICAL = 3    /* a NaN or Inf appeared in the check quantities */
} hlp_status;

typedef enum { HLP_FP64 = 0, HLP_MIXED = 1 } hlp_precision;

/*
 * Parameters.  Fields marked [setup] are read by hlp_lp_create only; the rest
 * by hlp_solve / hlp_unrolled_forward.  hlp_params_default() fills in the
 * defaults listed here.  Where the paper gives no value the default is this
 * library's reading, noted per field.
 */
typedef struct {
  double tol;              /* relative KKT tolerance epsilon (Sec. 4); 1e-8 */
  int64_t max_iter;        /* iteration limit (>= 1); 10,000,000 */
  double time_limit_s;     /* wall-clock limit in seconds; 3600 */
  int32_t eval_freq;       /* restart and termination tests every this many iterations
                              (and at max_iter); 64 -- the paper checks "at each
                              iteration", which is eval_freq = 1 */
  int32_t precision;       /* hlp_precision [setup and solve]; HLP_FP64 */
  double gamma;            /* reflection coefficient in [0,1] (Sec. 3); 1.0 */
  double beta_sufficient;  /* restart: r <= b_s r0 (Sec. 3); 0.2 */
  double beta_necessary;   /* restart: r <= b_n r0 and r > r_prev; 0.8 */
  double beta_artificial;  /* restart: k >= b_a T; 0.36 */
  double kp, ki, kd;       /* PID gains (Sec. 3); 0.99, 0.01, 0.0 */
  double omega0;           /* initial primal weight (Sec. 3); 1.0 */
  double eta_override;     /* [setup] > 0: use this eta and skip power iteration; 0 */
  int32_t ruiz_iters;      /* [setup] Ruiz infinity-norm passes; 10 */
  int32_t pock_chambolle;  /* [setup] 1: one Pock-Chambolle (alpha = 1) pass after Ruiz; 1 */
  int32_t power_max_iter;  /* [setup] power iteration cap; 5000 */
  int32_t restart_to_current; /* 0: new anchor = PDHG(z); 1: the Halpern iterate z; 0 */
  double power_tol;        /* [setup] relative change of the norm estimate that stops it; 1e-8 */
  double pid_min_norm;     /* skip the PID update if ||dx|| or ||dy|| is below this; 1e-10 */
  int32_t trace_iters;     /* > 0: record the first trace_iters iterates (see hlp_solve); 0 */
  int32_t debug_poison_iter; /* > 0: write NaN into x after that iteration (tests the
                                HLP_NUMERICAL path from the host); 0 */
  int32_t graphs;          /* 1: replay each run of eval_freq iterations (and its check)
                              from a captured HIP graph; 0: launch every kernel; 1.
                              Results are bitwise identical either way. */
  int32_t stream_matrix;   /* [setup] -1: automatic; 1: load the matrix arrays in the
                              half-steps as non-temporal (streaming) data; 0: cached.
                              Automatic streams when both matrices exceed 128 MB.
                              Results are bitwise identical either way; -1 */
  int32_t column_panels;   /* [setup] column panels for the dual half-step's A~ xbar:
                              the nonzeros of long rows (more than panel_row_min) are
                              also stored grouped by panels of consecutive columns,
                              each panel reduced by blocks of one XCD so that its slice
                              of xbar stays in that XCD's L2; the per-panel partial row
                              sums are added in panel order.  -1: automatic (on when
                              8n bytes exceed 8 MiB and long rows hold at least half of
                              the nonzeros; then 8 ceil(n / 2^20) panels, so a panel's
                              slice of xbar takes at most 1 MiB); 0: off;
                              k > 0: 8 ceil(k / 8) panels, at most 1024.  Changes only the
                              order in which the row sums are added; -1 */
  int32_t panel_row_min;   /* [setup] rows with more nonzeros than this are "long"
                              (>= 1); 16 */
  int32_t dense_row_min;   /* [setup] with column panels on, long rows with at least
                              this many nonzeros are "dense": their nonzeros are also
                              grouped by narrow panels of 2048 columns, whose slice of
                              xbar a block stages in LDS; the per-panel partial row sums
                              are added in panel order.  When the dense rows hold at
                              least half of the nonzeros, their entries of A~^T are
                              split off the same way for the primal half-step.  At
                              most 65,536 dense rows (and at most nnz / dense_row_min):
                              with more, the threshold is doubled until they fit.
                              0: no dense rows; otherwise > panel_row_min; 2048 */
} hlp_params;

/* Outcome of a solve.  Objectives and relative errors refer to the original
 * (unscaled) LP and are those of the returned point. */
typedef struct {
  int32_t status;          /* hlp_status */
  int32_t power_iters;     /* power iterations run at setup (0 with eta_override) */
  int64_t iters;           /* PDHG iterations (applications of the PDHG operator) */
  int64_t restarts;
  int64_t checks;          /* restart/termination tests done */
  double rel_kkt;          /* max of the three ratios below */
  double rel_gap;          /* |pobj - dobj| / (1 + |pobj| + |dobj|) */
  double rel_primal;       /* ||Ax - proj_[lc,uc](Ax)||_2 / (1 + ||(lc,uc) finite||_2) */
  double rel_dual;         /* ||c - A^T y - r||_2 / (1 + ||c||_2) */
  double pobj, dobj;       /* c^T x and -p(-y;lc,uc) - p(-r;lv,uv) */
  double omega, eta;       /* final primal weight, stepsize */
  double setup_s, solve_s; /* wall seconds in hlp_lp_create / hlp_solve */
} hlp_info;

/* One restart/termination test of a solve (Sec. 3, "Adaptive restart";
 * Sec. 4).  Values refer to the state the test saw. */
typedef struct {
  int64_t iter;            /* T: PDHG iterations done when the test ran */
  int64_t k;               /* k: iterations of the current epoch, counted after the increment */
  double r;                /* fixed-point residual ||z - PDHG(z)||_P at this iteration */
  double r0;               /* the epoch's r(z^{n,0}), measured at its first iteration */
  double rel_kkt, rel_gap, rel_primal, rel_dual;  /* of the PDHG output zhat, original LP */
  double omega;            /* primal weight in force during the iterations before the test
                              (before the PID update that a restart here applies) */
  double seconds;          /* wall seconds since hlp_solve began */
  int32_t restart;         /* 1: the test restarted (anchor reset, PID update) */
  int32_t reserved;        /* 0 */
} hlp_check;

/* Fill *p with the defaults above.  Errors: HLP_EINVAL if p is NULL. */
hlp_err hlp_params_default(hlp_params* p);

/*
 * Device workspace needed by hlp_lp_create for an m x n matrix with nnz
 * nonzeros under the [setup] fields of *p (precision decides whether FP32
 * mirrors are kept).  Writes the byte count to *bytes (host).
 * Errors: HLP_EINVAL for negative sizes or NULL pointers; HLP_EUNSUPPORTED if
 * nnz or a dimension does not fit int32 indexing (nnz >= 2^31, m or n >= 2^31 - 1).
 */
hlp_err hlp_workspace_bytes(int32_t m, int32_t n, int64_t nnz, const hlp_params* p, size_t* bytes);

/*
 * Device workspace for this particular matrix: as hlp_workspace_bytes, but
 * the column-panel layout is sized for the rows row_ptr describes (host
 * int64[m+1], the CSR row pointers of the matrix that will be passed to
 * hlp_lp_create) instead of for the worst rows (m, n, nnz) allow.  At most
 * hlp_workspace_bytes.  hlp_lp_create accepts a workspace of this size for
 * that matrix and parameters (it reads the row pointers back to lay it out).
 * Errors: HLP_EINVAL for NULL pointers or row pointers that do not start at 0,
 * end at nnz and never decrease; HLP_EUNSUPPORTED as hlp_workspace_bytes.
 */
hlp_err hlp_workspace_bytes_csr(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const hlp_params* p,
                                size_t* bytes);

/*
 * Build a handle: validate, canonical CSR copy, explicit transpose, diagonal
 * rescaling (Ruiz then Pock-Chambolle; the paper's Sec. 4 notes that the
 * iteration runs on a preconditioned LP while termination is judged on the
 * original one), the scaled vectors, and eta (power iteration, Sec. 3).
 *
 *   row_ptr  device int64[m+1]  CSR row pointers, row_ptr[0] = 0, nondecreasing
 *   col_idx  device int32[nnz]  column of each nonzero; strictly increasing within a row
 *   val      device double[nnz] finite values
 *   c        device double[n]   finite objective
 *   lc, uc   device double[m]   row bounds, lc <= uc, lc != +inf, uc != -inf
 *   lv, uv   device double[n]   column bounds, same rules
 *   p        host               [setup] fields are used; NULL = defaults
 *   workspace, workspace_bytes  device buffer of at least hlp_workspace_bytes() (or
 *                               hlp_workspace_bytes_csr() of this matrix), 256-byte aligned
 *   hip_stream                  hipStream_t all work goes to (NULL = default stream)
 *   out      host               receives the handle
 *
 * The input arrays are copied (the caller may free or reuse them after the
 * call).  workspace_bytes may be the hlp_workspace_bytes_csr size of this
 * matrix.  Errors: HLP_EINVAL for any violated rule above (NaN anywhere
 * included) or a misaligned/small workspace (HLP_ENOMEM if small);
 * HLP_EHIP on a HIP failure.  On error *out is NULL.
 */
hlp_err hlp_lp_create(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr,
                      const int32_t* col_idx, const double* val, const double* c,
                      const double* lc, const double* uc, const double* lv,
                      const double* uv, const hlp_params* p, void* workspace,
                      size_t workspace_bytes, void* hip_stream, hlp_lp** out);

/*
 * Replace c and the bounds (same rules and layout as hlp_lp_create) while
 * keeping A, its scaling and eta.  Errors as hlp_lp_create.
 */
hlp_err hlp_lp_update_vectors(hlp_lp* lp, const double* c, const double* lc,
                              const double* uc, const double* lv, const double* uv);

/*
 * Solve to the relative KKT tolerance (Sec. 4) with restarted reflected
 * Halpern PDHG (Secs. 2.2 and 3).
 *
 *   x0, y0   device double[n], double[m]  warm start in the original space; NULL = zeros
 *   x, y, r  device double[n], [m], [n]   outputs: the PDHG output zhat at the last
 *            check, unscaled, and the reduced costs r = proj_R(c - A^T y) (Sec. 4);
 *            any may be NULL
 *   info     host, may be NULL
 *   trace    device double[trace_iters * (2n + 2m)] or NULL: for t = 1..trace_iters,
 *            block t-1 holds [xhat (n), yhat (m), x (n), y (m)] in the scaled space,
 *            xhat/yhat = PDHG(z^t), x/y the iterate after the Halpern update.
 *            In HLP_MIXED mode these are the FP64 values centre + correction/scale.
 *
 * p->precision must match the handle's (a handle created for HLP_FP64 holds no
 * FP32 mirror).  The solver outcome is info->status; a limit or a numerical
 * breakdown is not an error.  Errors: HLP_EINVAL (bad parameters, NULL lp),
 * HLP_EUNSUPPORTED (precision mismatch), HLP_EHIP.
 */
hlp_err hlp_solve(hlp_lp* lp, const hlp_params* p, const double* x0, const double* y0,
                  double* x, double* y, double* r, hlp_info* info, double* trace);

/*
 * The check log of the last hlp_solve on this handle: one hlp_check per
 * restart/termination test, in order (kept in host memory by the handle,
 * replaced by the next hlp_solve).  Writes the number of records to *count
 * (host, required) and copies the first min(cap, *count) of them to out (host
 * array, may be NULL with cap = 0 to query the count).
 * Errors: HLP_EINVAL for a NULL handle or count, cap < 0, or out NULL with cap > 0.
 */
hlp_err hlp_check_log(const hlp_lp* lp, hlp_check* out, int64_t cap, int64_t* count);

/* Copy the scaling diagonals (device double[m], double[n]; either may be NULL)
 * and return eta and the power iterations through the host pointers (may be NULL). */
hlp_err hlp_lp_scaling(const hlp_lp* lp, double* d_r, double* d_c, double* eta, int32_t* power_iters);

/* Copy the explicit transpose built at setup: col_ptr device int32[n+1],
 * row_idx device int32[nnz], val device double[nnz] (the scaled values of the
 * transpose).  Any pointer may be NULL. */
hlp_err hlp_lp_transpose(const hlp_lp* lp, int32_t* col_ptr, int32_t* row_idx, double* val);

/* The column-panel layout chosen at setup (hlp_params::column_panels,
 * dense_row_min): the panel count (0: not used), the number of long rows in
 * those panels, the number of narrow panels and of dense rows, through host
 * pointers (any may be NULL).  Errors: HLP_EINVAL for a NULL handle. */
hlp_err hlp_lp_panels(const hlp_lp* lp, int32_t* panels, int32_t* long_rows, int32_t* dense_panels,
                      int32_t* dense_rows);

/*
 * Unrolled iterations with a tape for the reverse mode (an extension: the
 * derivative of the frozen iteration map, not part of the paper).
 *
 * hlp_tape_bytes: device bytes a tape for K iterations with a checkpoint
 * every ckpt_every iterations needs (K >= 1, 1 <= ckpt_every).
 *
 * hlp_unrolled_forward runs exactly K iterations from the all-zero start
 * (or x0, y0 in the original space, device, NULL = zeros; treated as
 * constants), with the restart/PID controller live (tests every eval_freq
 * iterations, no termination test) when replay = 0, or replaying the
 * controller decisions already on the tape when replay = 1.  It writes
 * x = D_c xhat_K and y = D_r yhat_K (device double[n], [m]) and records on the
 * tape: eta, the primal weight and Halpern index of every iteration, the
 * restart iterations, and the state (x, y, anchors) every ckpt_every
 * iterations.  p->precision must be HLP_FP64.
 *
 * hlp_unrolled_backward: given gx, gy (device double[n], [m]; either may be
 * NULL = 0), the derivative of the loss with respect to the outputs, writes
 * the gradient with respect to c (double[n]), lc, uc (double[m]), lv, uv
 * (double[n]) of the map recorded on the tape, with the vectors the handle
 * holds now (any output may be NULL).  Clamp ties count as active, the lower
 * bound first; infinite bounds get 0.  Recomputes each segment from its
 * checkpoint.
 * Errors: HLP_EINVAL, HLP_ENOMEM (tape too small), HLP_EUNSUPPORTED, HLP_EHIP.
 */
hlp_err hlp_tape_bytes(const hlp_lp* lp, int32_t K, int32_t ckpt_every, size_t* bytes);
hlp_err hlp_unrolled_forward(hlp_lp* lp, const hlp_params* p, int32_t K, int32_t ckpt_every,
                             int32_t replay, const double* x0, const double* y0,
                             double* x, double* y, void* tape, size_t tape_bytes);
hlp_err hlp_unrolled_backward(hlp_lp* lp, const void* tape, size_t tape_bytes,
                              const double* gx, const double* gy, double* gc, double* glc,
                              double* guc, double* glv, double* guv);

/*
 * Measurement: run `iters` iterations of the hot loop from a zero start (no
 * checks, the two half-steps alternating as in a solve) on the handle's
 * stream.  Each half-step is launched with a pair of HIP events that take the
 * kernel's own start and end timestamps; ms_out (host double[4]) receives the
 * mean duration in milliseconds of
 *   [0] the primal half-step (transpose SpMV fused with the primal update),
 *   [1] the dual half-step (SpMV fused with the dual update),
 *   [2] one iteration, from two plain events around the whole run,
 *   [3] the number of iterations timed.
 * precision selects the FP64 or the FP32 kernels (the handle must hold them).
 */
hlp_err hlp_profile_iterations(hlp_lp* lp, const hlp_params* p, int32_t iters, double* ms_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hlp_lp_create
 * followed by hlp_solve in one call, with the library's own static device
 * scratch as the workspace.  It allocates no device memory and calls no
 * allocating HIP or torch routine; HIP graphs are not used (p->graphs is
 * ignored), no trace is recorded and no check log is kept.
 *
 *   m, n, nnz, row_ptr, col_idx, val, c, lc, uc, lv, uv   as hlp_lp_create (device)
 *   p            host, NULL = defaults ([setup] fields and solve fields both apply)
 *   hip_stream   hipStream_t for all work (NULL = default stream)
 *   x, y, r, info  outputs as hlp_solve (device double[n], [m], [n]; host info; any may be NULL)
 *
 * The scratch is a file-scope device array of HLP_STATIC_SCRATCH_BYTES (160 MiB):
 * each GPU the library runs on holds its own copy until the process ends, and
 * every call on a GPU uses that GPU's copy, so calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the caller.
 * An LP whose workspace (hlp_workspace_bytes with *p) exceeds it gets
 * HLP_ENOMEM before any device work.  Results are bitwise those of
 * hlp_lp_create + hlp_solve with graphs off.
 * Errors: as hlp_lp_create and hlp_solve; HLP_ENOMEM when the LP does not fit.
 */
#define HLP_STATIC_SCRATCH_BYTES ((size_t)160 << 20)
hlp_err hlp_solve_static(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                         const double* val, const double* c, const double* lc, const double* uc,
                         const double* lv, const double* uv, const hlp_params* p, void* hip_stream,
                         double* x, double* y, double* r, hlp_info* info);

/* Destroy a handle (does not touch the workspace).  NULL is ignored. */
void hlp_lp_destroy(hlp_lp* lp);

/* Message for the last non-OK return on this thread ("" if none). */
const char* hlp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HLP_H */
