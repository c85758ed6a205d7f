// Internal declarations shared by the host controller and the kernel files.
// Host-side only: no device code here.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hlp.h"

namespace hlp {

// Quantities reduced at a check.  The primal and dual half-steps in their
// "residual" variants and the transpose KKT kernel each write per-block
// partial sums of their own subset; finalize kernels sum them in block order.
enum Q : int {
  Q_DX2 = 0,     // ||x - xhat||^2                       (primal kernel)
  Q_XA2 = 1,     // ||xhat - x0||^2                      (primal kernel, PID)
  Q_DY2 = 2,     // ||y - yhat||^2                       (dual kernel)
  Q_DYADX = 3,   // (y - yhat)^T A~ (x - xhat)           (dual kernel)
  Q_YA2 = 4,     // ||yhat - y0||^2                      (dual kernel, PID)
  Q_RP2 = 5,     // ||A x - proj(A x)||^2, unscaled      (dual kernel)
  Q_DOBJ_R = 6,  // row part of the dual objective       (dual kernel)
  Q_RD2 = 7,     // ||g - proj_R(g)||^2, unscaled        (transpose KKT kernel)
  Q_DOBJ_C = 8,  // column part of the dual objective    (transpose KKT kernel)
  Q_POBJ = 9,    // c^T x                                (transpose KKT kernel)
  Q_VP = 10,     // max primal violation, scaled space    (mixed: dual kernel; max)
  Q_VD = 11,     // max dual violation, scaled space      (mixed: KKT kernel; max)
  Q_VX = 12,     // max bound violation of x, scaled      (mixed: KKT kernel; max)
  NQ = 13
};

// Result slots (each NQ doubles) in the device results array.
enum Slot : int { SLOT_CHECK = 0, SLOT_R0 = 1, SLOT_TMP = 2, NSLOT = 3 };

// Power-iteration state kept on the device.
struct PowerState {
  double s;          // ||A~^T A~ v|| of the last pass
  double root;       // sqrt(s)
  double prev_root;
  double estimate;   // final ||A~||_2 estimate
  int32_t it;        // passes done
  int32_t done;
  int32_t has_prev;
  int32_t pad;
};

// Step scalars read by the half-step kernels from device memory.
struct StepDev {
  double tau, sigma, gamma;
  int64_t k0;  // Halpern index of launch offset j = 0
  double P, D; // refinement scales of the FP32 path (x = xc + x'/P, y = yc + y'/D)
};

}  // namespace hlp

struct hlp_lp {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  hipStream_t stream = nullptr;
  int32_t precision = HLP_FP64;
  // CSR of A~ (scaled) and its explicit transpose
  int32_t *rp = nullptr, *col = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  int32_t *cp = nullptr, *row = nullptr;
  double* tval = nullptr;
  float* tval32 = nullptr;
  double* val0 = nullptr;   // unscaled CSR values (input of the scaling statistics)
  double* tval0 = nullptr;  // unscaled transpose values
  int32_t Lr = 8, Lc = 8;   // lanes per row for A~ and A~^T (setup and check-only kernels)
  // row blocks (see device.h) of A~ (rbA, nbA blocks) and of A~^T (rbT, nbT)
  int32_t *rbA = nullptr, *rbT = nullptr, *rbtmp = nullptr;
  // the same blocks as {first row, end row, first nonzero, end nonzero}
  // (int4 per block), so a half-step block needs a single table load
  int32_t *rbxA = nullptr, *rbxT = nullptr;
  int32_t nbA = 0, nbT = 0;
  // stream the matrix arrays with non-temporal loads (set when the two
  // matrices exceed half of the 256 MB Infinity Cache, so they do not evict
  // the gathered vectors)
  bool nt = false;
  // Column panels of the long rows (dual half-step, see hlp_params::column_panels).
  // AS: A~ without the long rows (they are empty rows there); AP: the nonzeros
  // of the long rows grouped panel-major, AP row p*nL + l = the part of long
  // row lrow[l] in panel p (columns [p*panel_w, (p+1)*panel_w)).
  int32_t panels = 0, panel_w = 0, nL = 0, nL_cap = 0;
  int32_t *lrow = nullptr, *plid = nullptr;
  uint32_t* lbits = nullptr;          // bit i: row i is long
  int32_t *sp = nullptr, *scol = nullptr;
  double* sval = nullptr;
  float* sval32 = nullptr;
  int32_t *pp = nullptr, *pcol = nullptr;
  double* pval = nullptr;
  float* pval32 = nullptr;
  double* ppart = nullptr;            // partial row sums, P*nL (float in the FP32 path)
  // A~^T's row indices with the long rows redirected to the compact copy of
  // their y entries (index m + l); gathered by the plain primal half-steps
  int32_t* rowc = nullptr;
  int32_t *rbS = nullptr, *rbxS = nullptr, *rbP = nullptr, *rbxP = nullptr, *tabP = nullptr;
  int32_t *pscrA = nullptr, *pscrB = nullptr, *pscrC = nullptr;  // setup scratch
  // Dense rows (at least dense_min nonzeros; a subset of the rows taken out of
  // AS, listed after the long rows in lrow): AD = their nonzeros grouped by
  // narrow panels of dense_w columns, row q*nD + d = the part of dense row
  // lrow[nL + d] in narrow panel q.  A tile = consecutive row blocks of one
  // narrow panel, reduced by one block with the panel's slice of xbar in LDS.
  int32_t dense_min = 0, dense_P = 0, dense_w = 0, nD = 0, nD_cap = 0;
  int32_t nD_limit = 0;  // more dense rows than this: the threshold is doubled
  // the layout was sized for this matrix's rows (long + dense, dense, short
  // nonzeros and dense nonzeros exactly what build_panels must find)
  bool exact_layout = false;
  int64_t cap_nnz_short = 0, cap_nnz_dense = 0;
  int32_t *dlid = nullptr, *ppD = nullptr;
  uint16_t* pcolD = nullptr;  // column offset in the narrow panel
  double* pvalD = nullptr;
  float* pval32D = nullptr;
  double* partD = nullptr;   // dense_P * nD partial sums (float in the FP32 path)
  double* part2D = nullptr;  // group sums of 64 narrow panels: ceil(dense_P / 64) * nD
  int32_t *rbD = nullptr, *rbxD = nullptr, *tilesD = nullptr;
  int32_t nbD = 0, ntilesD = 0, nbCD = 0;
  // The primal side of the dense rows: ATR = A~^T without the dense rows'
  // entries (indices remapped like rowc), ATD = those entries grouped by
  // slices of dense_wT entries of the compact copy of y (row r*n + j = the
  // entries of column j whose dense index lies in slice r), with its tiles.
  int32_t dense_PT = 0, dense_PT_cap = 0, dense_wT = 0;
  int32_t *cpR = nullptr, *rowR = nullptr, *ppT = nullptr;
  uint16_t* rowT = nullptr;  // offset of the dense index in its slice
  double *tvalR = nullptr, *tvalT = nullptr;
  float *tval32R = nullptr, *tval32T = nullptr;
  double* partT = nullptr;  // dense_PT * n partial sums (float in the FP32 path)
  int32_t *rbR = nullptr, *rbxR = nullptr, *rbT2 = nullptr, *rbxT2 = nullptr, *tilesT = nullptr;
  int32_t nbR = 0, nbT2 = 0, ntilesT = 0;
  int64_t capD_blocks = 0, capT_blocks = 0;  // row blocks (and tiles) reserved for AD and ATD
  double* rsum = nullptr;       // check iterations: 3 x (nL + nD) panel row sums (A~ xbar, A~ dx, A~ xh)
  int64_t nb_dual_region = 0;   // blocks of the last check dual launch (its partials region)
  int64_t nb_primal_region = 0; // blocks of the last check primal launch (its partials region)
  int64_t nb_rows_region = 0;   // blocks of the last KKT-rows launch (its partials region)
  int64_t nb_kkt_region = 0;    // blocks of the last KKT-columns launch (its partials region)
  int32_t nbS = 0, nbP = 0, nbPgrid = 0, nbC = 0;
  int32_t poff[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // blocks of XCD x: tabP[poff[x] .. poff[x+1])
  int64_t rbtmp_rows = 0;             // capacity of the row-block scratch (rows)
  hlp::StepDev* step = nullptr;
  // captured runs of eval_freq iterations (see controller.cpp)
  void* graph_exec[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t graph_len = 0;
  hipStream_t capture_stream = nullptr;
  // scaling diagonals and scaled vectors
  double *dr = nullptr, *dc = nullptr;
  double *ct = nullptr, *lct = nullptr, *uct = nullptr, *lvt = nullptr, *uvt = nullptr;
  double norm_c = 0.0, norm_b = 0.0;  // ||c||_2 and ||(lc,uc) finite||_2, original space
  double eta = 1.0;
  int32_t power_iters = 0;
  // FP64 iteration state
  double *x = nullptr, *y = nullptr, *xa = nullptr, *ya = nullptr, *xbar = nullptr;
  double *xh = nullptr, *yh = nullptr, *dxv = nullptr, *rbuf = nullptr;
  // FP32 iteration state (mixed precision) and FP64 centre
  float *x32 = nullptr, *y32 = nullptr, *xa32 = nullptr, *ya32 = nullptr, *xbar32 = nullptr;
  float *xh32 = nullptr, *yh32 = nullptr, *dx32 = nullptr;
  float *c32 = nullptr, *lv32 = nullptr, *uv32 = nullptr, *lc32 = nullptr, *uc32 = nullptr,
        *b32 = nullptr;
  double *xcen = nullptr, *ycen = nullptr, *axc = nullptr, *atyc = nullptr;
  // reductions
  double* partials = nullptr;
  int64_t partial_blocks = 0;  // capacity in blocks (each NQ doubles)
  double* results = nullptr;   // NSLOT * NQ
  double* fin_scratch = nullptr;  // first-pass chunk results of large finalizes: 4 x 256 x 8
  hlp::PowerState* pstate = nullptr;
  int32_t* flags = nullptr;   // 8 ints: validation flags and setup counts
  // setup scratch (transpose)
  int32_t *kA = nullptr, *kB = nullptr, *vA = nullptr, *vB = nullptr, *rowof = nullptr;
  int32_t *hist = nullptr, *scan_tmp = nullptr;
  int64_t hist_len = 0, scan_tmp_len = 0;
  double* pv = nullptr;  // power iteration vectors (aliases)
  double* pu = nullptr;
  double* pw = nullptr;
  double setup_s = 0.0;
  // one record per check of the last hlp_solve (host memory); not kept when
  // keep_log is false (the allocation-free entry point)
  std::vector<hlp_check> check_log;
  bool keep_log = true;
};

namespace hlp {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
hlp_err hip_fail(hipError_t e, const char* what);
#define HLP_HIP(call)                                         \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::hlp::hip_fail(e_, #call);  \
  } while (0)
#define HLP_TRY(call)                   \
  do {                                  \
    hlp_err r_ = (call);                \
    if (r_ != HLP_OK) return r_;        \
  } while (0)

// ---------------------------------------------------------------- setup
// hlp_lp_create's work into a fresh handle object owned by the caller.
hlp_err setup_into(hlp_lp* lp, int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                   const double* val, const double* c, const double* lc, const double* uc, const double* lv,
                   const double* uv, const hlp_params* p, void* workspace, size_t workspace_bytes,
                   void* hip_stream, bool size_to_rows);

// ---------------------------------------------------------------- layout
// Capacities of the column-panel layout that the workspace reserves.
struct Caps {
  int32_t panels = 0;        // wide panels reserved (0: no panel layout)
  int64_t rows = 0;          // long and dense rows together
  int64_t long_rows = 0;     // long rows (wide panels)
  int64_t dense_rows = 0;    // dense rows (narrow panels); 0: none
  int64_t dense_limit = 0;   // more dense rows than this double the threshold
  int64_t slices = 0;        // slices of the primal split (0: not reserved)
  int64_t nnz_short = 0, nnz_long = 0, nnz_dense = 0;  // nonzeros of AS, AP, AD (and ATD)
  int64_t nnz_rest = 0;      // nonzeros of ATR
};
// For any rows an (m, n, nnz) matrix can have.
Caps worst_caps(int32_t m, int32_t n, int64_t nnz, int32_t panels, int32_t panel_row_min, int32_t dense_row_min);
// For the rows of this matrix (host row pointers, already validated): what
// hlp_lp_create's layout rules (thresholds, the automatic rule, the primal
// split) will build from them.
Caps exact_caps(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, int32_t panels, int32_t panel_row_min,
                int32_t dense_row_min, bool automatic);
// Carve the workspace.  With lp->... == nullptr base, only computes the size.
size_t carve(hlp_lp* lp, void* base, int32_t m, int32_t n, int64_t nnz, int32_t precision, const Caps& caps);
constexpr int32_t kDenseW = 2048;     // columns per narrow panel (its FP64 slice: 16 KB of LDS; < 65536)
// Compact dense indices per slice of the primal split (< 65536).  4096 halves
// the slice partials but its 32 KB slice leaves three blocks per CU, and the
// primal half-step of the largest LP got slower (2.21 -> 2.29 ms).
constexpr int32_t kDenseWT = 2048;
constexpr int32_t kDenseGroup = 64;   // narrow panels summed per group
constexpr int32_t kTileBlocks = 32;   // row blocks per tile
constexpr int32_t kMaxDense = 65536;  // dense rows at most (more: no dense class)
// Upper bound on the row blocks of a CSR with `rows` rows and nnz nonzeros
// (see the row-block rules in device.h), with panels of `period` rows.
inline int64_t row_block_bound(int64_t rows, int64_t nnz, int64_t panels) {
  return rows / 256 + nnz / 2048 + 3 * (nnz / 65) + panels + 4;
}
// Panels reserved for these sizes and parameters (0: none).
int32_t panel_count(int32_t n, const hlp_params* p);

int lanes_for(double mean_row_len);

// ---------------------------------------------------------------- kernel launchers (kernels_*.hip)
// Validation: returns bit flags through *flags (device), see kernels_setup.hip.
hipError_t launch_validate_rowptr(const int64_t* rp, int32_t m, int64_t nnz, int32_t* flags, hipStream_t s);
hipError_t launch_validate_rows(const int64_t* rp, const int32_t* col, const double* val, int32_t m,
                                int32_t n, int32_t* flags, hipStream_t s);
hipError_t launch_validate_vectors(const double* c, const double* lc, const double* uc,
                                   const double* lv, const double* uv, int32_t m, int32_t n,
                                   int32_t* flags, hipStream_t s);
hipError_t launch_copy_csr(const int64_t* rp64, const int32_t* col, const double* val, int32_t m,
                           int64_t nnz, int32_t* rp, int32_t* col_out, double* val_out, hipStream_t s);
hipError_t launch_transpose(hlp_lp* lp);
hipError_t launch_rescale(hlp_lp* lp, int32_t ruiz_iters, int32_t pock_chambolle);
hipError_t launch_scale_vectors(hlp_lp* lp, const double* c, const double* lc, const double* uc,
                                const double* lv, const double* uv);
hipError_t launch_power(hlp_lp* lp, int32_t passes, int32_t first_pass, int32_t max_iter, double tol);
// One power pass with the panel layout (kernels_iter.hip); *nb: partial blocks written.
hipError_t launch_power_pass_panels(hlp_lp* lp, int64_t* nb);
hipError_t launch_fill(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill32(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);

// Iteration (kernels_iter.hip).
// The step scalars (tau, sigma, gamma, k0) are set on the device by
// launch_set_step; each half-step launch carries its offset j from k0.
struct StepArgs {
  int32_t j = 0;
  int32_t residual = 0;      // compute the check quantities and write xhat / yhat
  uint8_t* mask_x = nullptr; // if set (FP64 only): write xhat and the clamp codes of v
  uint8_t* mask_y = nullptr; // if set (FP64 only): write yhat and the clamp codes of w
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // if set: timestamps of the kernel itself
};
// rbx holds rbx_cap blocks (-1: one per row); the caller checks *count <= rbx_cap.
hipError_t launch_build_row_blocks(hlp_lp* lp, const int32_t* ptr, int32_t rows, int32_t* rb, int32_t* rbx,
                                   int32_t* count, int32_t period = 0, int64_t rbx_cap = -1);
// Column panels: long-row split (returns nL and the short-part nonzero count
// through counts[0..1] on the device), then the panel layout and its blocks.
// counts[0] = long rows, counts[1] = nonzeros of the short part, counts[2] = dense rows.
hipError_t launch_panel_split(hlp_lp* lp, int32_t T, int32_t Ld, int32_t* counts);
// AS, the long rows' layout (if nL > 0) and the dense rows' layout (if nD > 0);
// block counts of AS, AP and AD go to counts[3], counts[4], counts[5].
hipError_t launch_panel_layout(hlp_lp* lp, int32_t* counts);
hipError_t launch_panel_starts(const int32_t* rbx, int32_t nb, int32_t rows_per_panel, int32_t* pstart,
                               hipStream_t s);
hipError_t launch_panel_remap(hlp_lp* lp);
// ATR and ATD (needs nD > 0, dense_PT set); block counts to counts[6], counts[7].
hipError_t launch_dense_transpose(hlp_lp* lp, int32_t* counts);
hipError_t launch_set_step(hlp_lp* lp, double tau, double sigma, double gamma, int64_t k0, double P = 1.0,
                           double D = 1.0);
hipError_t launch_primal(hlp_lp* lp, const StepArgs& s);
hipError_t launch_dual(hlp_lp* lp, const StepArgs& s);
hipError_t launch_kkt_cols(hlp_lp* lp, double* r_out);
hipError_t launch_finalize(hlp_lp* lp, int32_t which /*0 primal,1 dual,2 kkt*/, int32_t slot);
hipError_t launch_restart_copy(hlp_lp* lp, int32_t to_current);
hipError_t launch_warm_start(hlp_lp* lp, const double* x0, const double* y0);
hipError_t launch_unscale(hlp_lp* lp, double* x, double* y);
hipError_t launch_trace(hlp_lp* lp, double* dst);
hipError_t launch_poison(hlp_lp* lp);

// Mixed precision (kernels_iter.hip).
hipError_t launch_primal32(hlp_lp* lp, const StepArgs& s);
hipError_t launch_dual32(hlp_lp* lp, const StepArgs& s);
hipError_t launch_combine(hlp_lp* lp);  // xh <- xcen + xh32/P, yh <- ycen + yh32/D (P, D from the step)
hipError_t launch_kkt_rows(hlp_lp* lp);                      // A~ xh (FP64) and row KKT terms
hipError_t launch_recentre(hlp_lp* lp, double P, double D);  // rebuild the correction data
hipError_t launch_trace32(hlp_lp* lp, double* dst);

// Adjoint (kernels_adjoint.hip).  Reverse mode of one iteration; mode of the
// iteration: 0 Halpern update after it, 1 restart after it, 2 the last one.
struct AdjVecs {
  double *gxn, *gxa, *gct, *glv, *guv, *u;   // n
  double *gyn, *gya, *glc, *guc, *gw, *py;   // m
};
struct AdjIter {
  double tau, sigma, a, gamma;
  int32_t mode;
};
hipError_t launch_bwd_prep(hlp_lp* lp, const AdjVecs& v, const AdjIter& it, const uint8_t* my, const double* Gy);
hipError_t launch_bwd_cols(hlp_lp* lp, const AdjVecs& v, const AdjIter& it, const uint8_t* mx, const double* Gx);
hipError_t launch_bwd_rows(hlp_lp* lp, const AdjVecs& v, int32_t do_prev, const AdjIter& prev,
                           const uint8_t* my_prev, const double* Gy);
hipError_t launch_bwd_out(hlp_lp* lp, const AdjVecs& v, double* gc, double* glc, double* guc, double* glv,
                          double* guv);
hipError_t launch_zero_adj(hlp_lp* lp, const AdjVecs& v);


}  // namespace hlp
