// Hot-loop kernels of restarted reflected Halpern PDHG (paper Secs. 2.2, 3).
//
// One iteration is two launches:
//   primal half-step: g = A~^T y over the explicit transpose (L lanes per
//     column), fused with xhat = clamp(x - tau (c~ - g), lv~, uv~),
//     xbar = 2 xhat - x and the reflected Halpern update of x;
//   dual half-step: h = A~ xbar over the CSR (L lanes per row), fused with
//     w = h - y/sigma, yhat = sigma (clamp(w, lc~, uc~) - w) and the reflected
//     Halpern update of y.
// Their "residual" variants also write xhat, yhat, x - xhat and per-block
// partial sums of the check quantities (fixed-point residual in the P-norm of
// Sec. 2.2, the PID distances, the row side of the KKT error of Sec. 4).  A
// transpose kernel adds the column side of the KKT error.  All reductions are
// per-block partials summed in block order: results are bit-reproducible.
#include <hip/hip_ext.h>

#include <algorithm>

#include <cmath>

#include "device.h"
#include "hlp_internal.h"

namespace hlp {

namespace {

inline int nblocks(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

// partial regions inside lp->partials, each `cap` blocks x 8 doubles
constexpr int kRegionStride = 8;
constexpr int64_t kFinDirect = 4096;  // regions up to this many blocks: one finalize pass
constexpr int kFinChunks = 256;       // chunks of the first pass otherwise (hlp_lp::fin_scratch)
inline double* region(hlp_lp* lp, int r) { return lp->partials + (int64_t)r * lp->partial_blocks * kRegionStride; }
enum { R_PRIMAL = 0, R_DUAL = 1, R_KKT = 2, R_ROWS = 3 };

// ============================================================================ step scalars
// tau, sigma, gamma and the Halpern index k0 at the start of the current run
// of launches live in device memory, so a run of iterations can be replayed
// from a HIP graph; each launch carries only its offset j (a = (k0+j+1)/(k0+j+2)).
__global__ void k_set_step(StepDev* s, double tau, double sigma, double gamma, int64_t k0, double P, double D) {
  s->tau = tau;
  s->sigma = sigma;
  s->gamma = gamma;
  s->k0 = k0;
  s->P = P;
  s->D = D;
}

__device__ __forceinline__ double halpern_a(const StepDev* s, int32_t j) {
  const int64_t k = s->k0 + j;
  return (double)(k + 1) / (double)(k + 2);
}

// ============================================================================ FP64 half-steps
struct PrimalArgs {
  const int4* rb; const int32_t* cp; const int32_t* row; const double* tval;
  const double* y; double* x; const double* xa; const double* ct; const double* lv; const double* uv;
  double* xbar; double* xh; double* dx; double* partials; uint8_t* mask; const StepDev* step;
  int32_t j;
  const double* partT;  // if PT > 0: the dense rows' part of A~^T y, PT slice sums per column
  int32_t PT, n;
};

// sum over r < cnt of a[r*stride + i], added in order of r; the loads go out
// eight at a time (one load at a time would cost a memory round trip per term).
template <typename T>
__device__ __forceinline__ T strided_sum(const T* __restrict__ a, int32_t cnt, int64_t stride, int i) {
  T h = T(0);
  for (int r = 0; r < cnt; r += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = r + u < cnt ? a[(int64_t)(r + u) * stride + i] : T(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r + u < cnt) h += v[u];
  }
  return h;
}

// The dense rows' part of column j's product: its slice sums in slice order.
template <typename T>
__device__ __forceinline__ T slice_sum(const T* __restrict__ partT, int32_t PT, int32_t n, int j) {
  return strided_sum(partT, PT, n, j);
}

// MODE 0: plain step; 1: also xhat, x - xhat and the check partials;
// 2: also xhat and the clamp code of v (for the reverse mode).
// NT: stream the matrix arrays (large matrices, see hlp_lp::nt).
template <int MODE, bool NT>
__global__ __launch_bounds__(kBlock) void k_primal(PrimalArgs p) {
  constexpr bool RES = MODE == 1;
  __shared__ double lds[kRbLds];
  const int4 blk = p.rb[blockIdx.x];
  const int s = blk.x, e = blk.y, ps = blk.z, pe = blk.w;
  const int j = s + threadIdx.x;
  const bool own = j < e;
  double xj = 0.0, cj = 0.0, lo = 0.0, hi = 0.0, xaj = 0.0;
  int a0 = 0, a1 = 0;
  if (own) {
    xj = p.x[j]; cj = p.ct[j]; lo = p.lv[j]; hi = p.uv[j]; xaj = p.xa[j];
    a0 = p.cp[j]; a1 = p.cp[j + 1];
  }
  double g = rb_dot<double, NT>(p.row, p.tval, p.y, ps, pe, a0, a1, own, e - s, lds);
  if (p.PT > 0 && own) g += slice_sum(p.partT, p.PT, p.n, j);
  double q0 = 0.0, q1 = 0.0;
  if (own) {
    const double tau = p.step->tau, gam = p.step->gamma, a = halpern_a(p.step, p.j);
    const double v = xj - tau * (cj - g);
    const double xh = clampv(v, lo, hi);
    p.xbar[j] = 2.0 * xh - xj;
    p.x[j] = a * ((1.0 + gam) * xh - gam * xj) + (1.0 - a) * xaj;
    if (MODE == 2) {
      p.xh[j] = xh;
      p.mask[j] = clamp_code(v, lo, hi);
    }
    if (RES) {
      p.xh[j] = xh;
      const double d = xj - xh;
      p.dx[j] = d;
      q0 = d * d;
      const double e2 = xh - xaj;
      q1 = e2 * e2;
    }
  }
  if (RES) {
    double v[2] = {q0, q1};
    block_reduce_store<2>(v, p.partials + (int64_t)blockIdx.x * kRegionStride);
  }
}

struct DualArgs {
  const int4* rb; const int32_t* rp; const int32_t* col; const double* val;
  const double* xbar; const double* dx; const double* xh;
  double* y; const double* ya; const double* lc; const double* uc; const double* dr;
  double* yh; double* partials; uint8_t* mask; const StepDev* step;
  int32_t j;
};

// MODE and NT as for k_primal (the code is that of w against the row bounds).
template <int MODE, bool NT>
__global__ __launch_bounds__(kBlock) void k_dual(DualArgs p) {
  constexpr bool RES = MODE == 1;
  __shared__ double lds[kRbLds];
  const int4 blk = p.rb[blockIdx.x];
  const int s = blk.x, e = blk.y, ps = blk.z, pe = blk.w;
  const int i = s + threadIdx.x;
  const bool own = i < e;
  double yi = 0.0, lo = 0.0, hi = 0.0, yai = 0.0, dri = 1.0;
  int a0 = 0, a1 = 0;
  if (own) {
    yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i];
    if (RES) dri = p.dr[i];
    a0 = p.rp[i]; a1 = p.rp[i + 1];
  }
  const double h = rb_dot<double, NT>(p.col, p.val, p.xbar, ps, pe, a0, a1, own, e - s, lds);
  double adx = 0.0, axh = 0.0;
  if (RES) {
    adx = rb_dot<double>(p.col, p.val, p.dx, ps, pe, a0, a1, own, e - s, lds);
    axh = rb_dot<double>(p.col, p.val, p.xh, ps, pe, a0, a1, own, e - s, lds);
  }
  double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (own) {
    const double sigma = p.step->sigma, gam = p.step->gamma, a = halpern_a(p.step, p.j);
    const double w = h - yi / sigma;
    const double yh = sigma * (clampv(w, lo, hi) - w);
    p.y[i] = a * ((1.0 + gam) * yh - gam * yi) + (1.0 - a) * yai;
    if (MODE == 2) {
      p.yh[i] = yh;
      p.mask[i] = clamp_code(w, lo, hi);
    }
    if (RES) {
      p.yh[i] = yh;
      const double dy = yi - yh;
      q[0] = dy * dy;
      q[1] = dy * adx;
      const double e2 = yh - yai;
      q[2] = e2 * e2;
      const double pr = (axh - clampv(axh, lo, hi)) / dri;
      q[3] = pr * pr;
      q[4] = (finite(lo) ? lo * fmax(yh, 0.0) : 0.0) - (finite(hi) ? hi * fmax(-yh, 0.0) : 0.0);
    }
  }
  if (RES) block_reduce_store<5>(q, p.partials + (int64_t)blockIdx.x * kRegionStride);
}

// ---------------------------------------------------------------------------- column panels
// y[m + l] <- y[lrow[l]]: the compact copy of the long rows' entries.
template <typename T>
__global__ void k_refresh_long_y(T* __restrict__ y, const int32_t* __restrict__ lrow, int32_t nL, int32_t m) {
  const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (l < nL) y[m + l] = y[lrow[l]];
}

// A run of row blocks reduced one after another by one workgroup.  For the
// staged kind (short rows, at most kRbLds nonzeros) the next block's entries
// and row pointers are loaded while the current block is reduced, so their
// latency overlaps the gathers and the LDS work.  The sums are those of
// rb_dot: products staged at their position, each row added serially.
constexpr int kStagedSlots = (kRbLds + kBlock - 1) / kBlock;  // per thread, at stride kBlock

__device__ __forceinline__ bool staged_kind(int4 blk) {
  const int nrows = blk.y - blk.x;
  return nrows > 1 && blk.w - blk.z <= nrows * kRbSerial;
}

template <typename T>
struct StagedRegs {
  int ix[kStagedSlots];
  T v[kStagedSlots];
  int a0, a1;
};

template <bool NT, typename T, typename I>
__device__ __forceinline__ void staged_load(const I* __restrict__ idx, const T* __restrict__ val,
                                            const int32_t* __restrict__ ptr, int4 blk, StagedRegs<T>& R) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kStagedSlots; ++u) {
    const int q = blk.z + tid + u * kBlock;
    R.ix[u] = 0;
    R.v[u] = T(0);
    if (q < blk.w) {
      R.ix[u] = (int)ld<NT>(idx + q);
      R.v[u] = ld<NT>(val + q);
    }
  }
  const int r = blk.x + tid;
  R.a0 = R.a1 = 0;
  if (r < blk.y) { R.a0 = ptr[r]; R.a1 = ptr[r + 1]; }
}

// tb: the nbk row blocks (in LDS); out[r] = row r's sum of val .* vec[idx],
// products and sums in T (the values and the vector are V).
// cur: the first block's loads if it is of the staged kind (the caller issues
// them, so they can overlap its own set-up).
template <typename T, bool NT, typename I, typename V>
__device__ __forceinline__ void row_block_run(const int4* tb, int nbk, const I* __restrict__ idx,
                                              const V* __restrict__ val, const int32_t* __restrict__ ptr,
                                              const V* __restrict__ vec, T* __restrict__ out, T* lds,
                                              StagedRegs<V>& cur) {
  const int tid = threadIdx.x;
  StagedRegs<V> nxt;
  for (int b = 0; b < nbk; ++b) {  // uniform over the workgroup
    const int4 blk = tb[b];
    const int r = blk.x + tid;
    const bool own = r < blk.y;
    const bool pre = b + 1 < nbk && staged_kind(tb[b + 1]);
    if (staged_kind(blk)) {
      const int len = blk.w - blk.z;
      V g[kStagedSlots];
#pragma unroll
      for (int u = 0; u < kStagedSlots; ++u) g[u] = tid + u * kBlock < len ? vec[cur.ix[u]] : V(0);
      if (pre) staged_load<NT>(idx, val, ptr, tb[b + 1], nxt);
#pragma unroll
      for (int u = 0; u < kStagedSlots; ++u) {
        const int q = tid + u * kBlock;
        if (q < len) lds[q] = (T)cur.v[u] * (T)g[u];
      }
      __syncthreads();
      const T acc = own ? lds_row_sum(lds, cur.a0 - blk.z, cur.a1 - blk.z) : T(0);
      __syncthreads();
      if (own) out[r] = acc;
      if (pre) cur = nxt;
    } else {
      int a0 = 0, a1 = 0;
      if (own) { a0 = ptr[r]; a1 = ptr[r + 1]; }
      const T acc = rb_dot<T, NT>(idx, val, vec, blk.z, blk.w, a0, a1, own, blk.y - blk.x, lds);
      if (own) out[r] = acc;
      if (pre) staged_load<NT>(idx, val, ptr, tb[b + 1], cur);
    }
  }
}

// Dual half-step with the long rows split into column panels.  A panel block
// reduces (panel, long row) segments; the blocks of panel p run on XCD p mod 8
// (workgroups are dealt to the XCDs in turn), so an XCD gathers from one
// panel's slice of xbar at a time and the slice stays in its L2.  In plain
// iterations k_dual_ps runs them beside the short rows' blocks; k_dual_pn then
// adds, for each long row, the panel partials in panel order (h) and runs its
// update.  (One row block per workgroup: these gathers go to L2 and want many
// waves in flight, more than row_block_run's register budget leaves.)
// (T: products and sums; V: the values and the vector.)
template <typename T, typename V = T>
struct PanelDotArgs {
  const int4* tab; const int32_t* pp; const int32_t* pcol; const V* pval; const V* vec; T* out;
  int32_t off[9];
};

// Block k of the (panel, long row) table.
template <typename T, bool NT, typename V>
__device__ __forceinline__ void panel_dot_block(const PanelDotArgs<T, V>& p, int k, T* lds) {
  const int4 blk = p.tab[k];
  const int r = blk.x + threadIdx.x;
  const bool own = r < blk.y;
  int a0 = 0, a1 = 0;
  if (own) { a0 = p.pp[r]; a1 = p.pp[r + 1]; }
  const T acc = rb_dot<T, NT>(p.pcol, p.pval, p.vec, blk.z, blk.w, a0, a1, own, blk.y - blk.x, lds);
  if (own) p.out[r] = acc;
}

// (The power iteration's and the check iterations' products; the plain
// half-step runs these blocks in k_dual_ps.)
template <typename T, bool NT, typename V = T>
__global__ __launch_bounds__(kBlock) void k_panel_dot(PanelDotArgs<T, V> p) {
  __shared__ T lds[kRbLds];
  const int x = blockIdx.x & 7;
  const int k = p.off[x] + (int)(blockIdx.x >> 3);
  if (k >= p.off[x + 1]) return;  // uniform over the block
  panel_dot_block<T, NT>(p, k, lds);
}

template <typename T>
__device__ __forceinline__ T panel_sum(const T* __restrict__ part, int32_t P, int32_t nL, int l) {
  T h = T(0);
  for (int q = 0; q < P; q += 8) {  // P is a multiple of 8
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(q + u) * nL + l];
#pragma unroll
    for (int u = 0; u < 8; ++u) h += v[u];
  }
  return h;
}

// Dense rows: a tile is up to kTileBlocks row blocks of one narrow panel of
// AD; the block stages the panel's slice of the vector in LDS once and
// gathers from there (the indices are 16-bit offsets in the slice).
template <typename T, typename V = T>
struct DenseDotArgs {
  const int4* tiles; const int4* rbx; const int32_t* pp; const uint16_t* pcol; const V* pval; const V* vec;
  T* out; int32_t n;
};

// W: the slice width (kDenseW columns for AD, kDenseWT dense indices for
// ATD).  (The register budget is that of four waves per SIMD, at most what
// the LDS allows for T = double.)
template <typename T, bool NT, int W, typename V = T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_dense_dot(DenseDotArgs<T, V> p) {
  __shared__ V xs[W];
  __shared__ T lds[kRbLds];
  __shared__ int4 tb[kTileBlocks];
  const int4 tile = p.tiles[blockIdx.x];
  const int c0 = tile.z * W;
  const int nc = min(W, p.n - c0);
  const int nbk = tile.y - tile.x;  // 1 to kTileBlocks
  if (nbk <= 0) return;             // uniform over the block
  const int tid = threadIdx.x;
  // the first row block's loads go out with the staging of the slice
  const int4 blk0 = p.rbx[tile.x];
  StagedRegs<V> cur;
  if (staged_kind(blk0)) staged_load<NT>(p.pcol, p.pval, p.pp, blk0, cur);
  if (tid < nbk) tb[tid] = p.rbx[tile.x + tid];
  for (int c = tid; c < nc; c += kBlock) xs[c] = p.vec[c0 + c];
  __syncthreads();
  row_block_run<T, NT>(tb, nbk, p.pcol, p.pval, p.pp, xs, p.out, lds, cur);
}

// Group sums of kDenseGroup narrow panels, in panel order:
// out[g*nD + d] = sum over q in group g of part[q*nD + d].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_combine(const T* __restrict__ part, int32_t nD, int32_t P,
                                                          T* __restrict__ out) {
  const int d = blockIdx.x * kBlock + threadIdx.x;
  const int g = blockIdx.y;
  if (d >= nD) return;
  const int q0 = g * kDenseGroup, q1 = min(P, q0 + kDenseGroup);
  T h = T(0);
  int q = q0;
  for (; q + 8 <= q1; q += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(q + u) * nD + d];
#pragma unroll
    for (int u = 0; u < 8; ++u) h += v[u];
  }
  for (; q < q1; ++q) h += part[(int64_t)q * nD + d];
  out[(int64_t)g * nD + d] = h;
}

template <typename T>
__device__ __forceinline__ T group_sum(const T* __restrict__ part2, int32_t G, int32_t nD, int d) {
  return strided_sum(part2, G, nD, d);
}

__device__ __forceinline__ bool is_long(const uint32_t* __restrict__ bits, int i) {
  return (bits[i >> 5] >> (i & 31)) & 1u;
}

// The host sizes the long-row part of the grid as ceil(nL / 256).
static_assert(kBlock == 256, "k_dual_pn: one long row per thread of 256-thread blocks");

struct DualPanelArgs {
  const int4* rb; const int32_t* sp; const int32_t* scol; const double* sval; const double* xbar;
  double* y; const double* ya; const double* lc; const double* uc; const StepDev* step;
  const uint32_t* lbits; const int32_t* lrow; const double* part; const double* part2;
  int32_t P, nL, nbS, j, m, nbC, nD, G;
};

// The dual update of row i (l >= 0: row l of lrow, whose compact copy the
// primal half-step gathers).
__device__ __forceinline__ void dual_pn_update(const DualPanelArgs& p, int i, int l, double h, double yi, double lo,
                                               double hi, double yai) {
  const double sigma = p.step->sigma, gam = p.step->gamma, a = halpern_a(p.step, p.j);
  const double w = h - yi / sigma;
  const double yh = sigma * (clampv(w, lo, hi) - w);
  const double yn = a * ((1.0 + gam) * yh - gam * yi) + (1.0 - a) * yai;
  p.y[i] = yn;
  if (l >= 0) p.y[p.m + l] = yn;
}

// Row block b of AS: the short rows' products and updates.
template <bool NT>
__device__ __forceinline__ void short_block(const DualPanelArgs& p, int b, double* lds) {
  const int4 blk = p.rb[b];
  const int i = blk.x + threadIdx.x;
  const bool in = i < blk.y;
  bool own = false;
  double yi = 0.0, lo = 0.0, hi = 0.0, yai = 0.0;
  int a0 = 0, a1 = 0;
  if (in) {
    a0 = p.sp[i]; a1 = p.sp[i + 1];
    own = !is_long(p.lbits, i);
    if (own) { yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; }
  }
  const double h = rb_dot<double, NT>(p.scol, p.sval, p.xbar, blk.z, blk.w, a0, a1, in, blk.y - blk.x, lds);
  if (own) dual_pn_update(p, i, -1, h, yi, lo, hi, yai);
}

// Blocks [0, nbS): short rows; then the long rows from their panel partials
// (h = sum in panel order) and the dense rows from their group sums.
template <bool NT>
__global__ __launch_bounds__(kBlock) void k_dual_pn(DualPanelArgs p) {
  __shared__ double lds[kRbLds];
  int i = 0, l = -1;
  bool own = false;
  double h = 0.0, yi = 0.0, lo = 0.0, hi = 0.0, yai = 0.0;
  if ((int)blockIdx.x < p.nbS) {
    short_block<NT>(p, blockIdx.x, lds);
    return;
  } else if ((int)blockIdx.x < p.nbS + p.nbC) {
    l = ((int)blockIdx.x - p.nbS) * kBlock + threadIdx.x;
    own = l < p.nL;
    if (own) {
      i = p.lrow[l];
      yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i];
      h = panel_sum(p.part, p.P, p.nL, l);
    }
  } else {
    const int d = ((int)blockIdx.x - p.nbS - p.nbC) * kBlock + threadIdx.x;
    own = d < p.nD;
    if (own) {
      l = p.nL + d;
      i = p.lrow[l];
      yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i];
      h = group_sum(p.part2, p.G, p.nD, d);
    }
  }
  if (own) dual_pn_update(p, i, l, h, yi, lo, hi, yai);
}

// Check iterations with panels: the long and dense rows' sums of one product
// (out[l] for long row l, out[nL + d] for dense row d), from the partials of
// the panel kernels, in the same order as k_dual_pn.
// (T: the partials' type, summed in T as the half-steps do; out in FP64.)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pn_rowsums(const T* __restrict__ part, const T* __restrict__ part2,
                                                      int32_t P, int32_t nL, int32_t nD, int32_t G,
                                                      double* __restrict__ out) {
  const int l = blockIdx.x * kBlock + threadIdx.x;
  if (l < nL) out[l] = (double)panel_sum(part, P, nL, l);
  else if (l < nL + nD) out[l] = (double)group_sum(part2, G, nD, l - nL);
}

// The check-iteration dual half-step with panels: h = A~ xbar, A~ dx and
// A~ xh from AS for the short rows and from the row sums for the others, the
// update of k_dual (xhat, the restart and KKT partials), and the compact copy.
struct DualResArgs {
  const int4* rb; const int32_t* sp; const int32_t* scol; const double* sval;
  const double* xbar; const double* dx; const double* xh;
  double* y; const double* ya; const double* lc; const double* uc; const double* dr;
  double* yh; double* partials; const StepDev* step;
  const uint32_t* lbits; const int32_t* lrow; const double* rsum;
  int32_t nbS, j, m, nL, nD;
};

__global__ __launch_bounds__(kBlock) void k_dual_pn_res(DualResArgs p) {
  __shared__ double lds[kRbLds];
  int i = 0, l = -1;
  bool own = false;
  double h = 0.0, adx = 0.0, axh = 0.0, yi = 0.0, lo = 0.0, hi = 0.0, yai = 0.0, dri = 1.0;
  if ((int)blockIdx.x < p.nbS) {
    const int4 blk = p.rb[blockIdx.x];
    i = blk.x + threadIdx.x;
    const bool in = i < blk.y;
    int a0 = 0, a1 = 0;
    if (in) {
      a0 = p.sp[i]; a1 = p.sp[i + 1];
      own = !is_long(p.lbits, i);
      if (own) { yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; dri = p.dr[i]; }
    }
    const int nr = blk.y - blk.x;
    h = rb_dot<double>(p.scol, p.sval, p.xbar, blk.z, blk.w, a0, a1, in, nr, lds);
    adx = rb_dot<double>(p.scol, p.sval, p.dx, blk.z, blk.w, a0, a1, in, nr, lds);
    axh = rb_dot<double>(p.scol, p.sval, p.xh, blk.z, blk.w, a0, a1, in, nr, lds);
  } else {
    l = ((int)blockIdx.x - p.nbS) * kBlock + threadIdx.x;
    const int nc = p.nL + p.nD;
    own = l < nc;
    if (own) {
      i = p.lrow[l];
      yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; dri = p.dr[i];
      h = p.rsum[l]; adx = p.rsum[nc + l]; axh = p.rsum[2 * nc + l];
    }
  }
  double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (own) {
    const double sigma = p.step->sigma, gam = p.step->gamma, a = halpern_a(p.step, p.j);
    const double w = h - yi / sigma;
    const double yh = sigma * (clampv(w, lo, hi) - w);
    const double yn = a * ((1.0 + gam) * yh - gam * yi) + (1.0 - a) * yai;
    p.y[i] = yn;
    if (l >= 0) p.y[p.m + l] = yn;
    p.yh[i] = yh;
    const double dy = yi - yh;
    q[0] = dy * dy;
    q[1] = dy * adx;
    const double e2 = yh - yai;
    q[2] = e2 * e2;
    const double pr = (axh - clampv(axh, lo, hi)) / dri;
    q[3] = pr * pr;
    q[4] = (finite(lo) ? lo * fmax(yh, 0.0) : 0.0) - (finite(hi) ? hi * fmax(-yh, 0.0) : 0.0);
  }
  block_reduce_store<5>(q, p.partials + (int64_t)blockIdx.x * kRegionStride);
}

// The FP32 path's check-iteration dual half-step with panels: h in FP32 and
// A~ dx accumulated in FP64 (as k_dual32's check variant computes them) from
// AS for the short rows and from the row sums for the others; the update,
// yhat, the restart partials and the compact copy.
struct Dual32ResArgs {
  const int4* rb; const int32_t* sp; const int32_t* scol; const float* sval;
  const float* xbar; const float* dx;
  float* y; const float* ya; const float* lc; const float* uc; const float* b;
  float* yh; double* partials; const StepDev* step;
  const uint32_t* lbits; const int32_t* lrow; const double* rsum;
  int32_t nbS, j, m, nL, nD;
};

__global__ __launch_bounds__(kBlock) void k_dual32_pn_res(Dual32ResArgs p) {
  __shared__ double lds[kRbLds];
  int i = 0, l = -1;
  bool own = false;
  float h = 0.0f, yi = 0.0f, lo = 0.0f, hi = 0.0f, yai = 0.0f, bi = 0.0f;
  double adx = 0.0;
  if ((int)blockIdx.x < p.nbS) {
    const int4 blk = p.rb[blockIdx.x];
    i = blk.x + threadIdx.x;
    const bool in = i < blk.y;
    int a0 = 0, a1 = 0;
    if (in) {
      a0 = p.sp[i]; a1 = p.sp[i + 1];
      own = !is_long(p.lbits, i);
      if (own) { yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; bi = p.b[i]; }
    }
    const int nr = blk.y - blk.x;
    h = rb_dot<float>(p.scol, p.sval, p.xbar, blk.z, blk.w, a0, a1, in, nr, reinterpret_cast<float*>(lds));
    adx = rb_dot<double>(p.scol, p.sval, p.dx, blk.z, blk.w, a0, a1, in, nr, lds);
  } else {
    l = ((int)blockIdx.x - p.nbS) * kBlock + threadIdx.x;
    const int nc = p.nL + p.nD;
    own = l < nc;
    if (own) {
      i = p.lrow[l];
      yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; bi = p.b[i];
      h = (float)p.rsum[l];
      adx = p.rsum[nc + l];
    }
  }
  double q[3] = {0.0, 0.0, 0.0};
  if (own) {
    const float sigma = (float)p.step->sigma, gam = (float)p.step->gamma, a = (float)halpern_a(p.step, p.j);
    const float w = h - (bi + yi) / sigma;
    const float yh = yi + sigma * (clampv(w, lo, hi) - h);
    const float yn = a * ((1.0f + gam) * yh - gam * yi) + (1.0f - a) * yai;
    p.y[i] = yn;
    if (l >= 0) p.y[p.m + l] = yn;
    p.yh[i] = yh;
    const double dy = (double)(yi - yh);
    q[0] = dy * dy;
    q[1] = dy * adx;
    const double e2 = (double)(yh - yai);
    q[2] = e2 * e2;
  }
  block_reduce_store<3>(q, p.partials + (int64_t)blockIdx.x * kRegionStride);
}

// Row side of the KKT error (mixed mode, FP64) with panels: A~ xh from AS for
// the short rows and from the row sums for the long and dense rows.
struct KktRowPanelArgs {
  const int4* rb; const int32_t* sp; const int32_t* scol; const double* sval;
  const double* xh; const double* yh; const double* lc; const double* uc; const double* dr;
  double* ax_out; double* partials; const uint32_t* lbits; const int32_t* lrow; const double* rsum;
  int32_t nbS, nL, nD;
};

__global__ __launch_bounds__(kBlock) void k_kkt_rows_pn(KktRowPanelArgs p) {
  __shared__ double lds[kRbLds];
  int i = 0;
  bool own = false;
  double acc = 0.0;
  if ((int)blockIdx.x < p.nbS) {
    const int4 blk = p.rb[blockIdx.x];
    i = blk.x + threadIdx.x;
    const bool in = i < blk.y;
    int a0 = 0, a1 = 0;
    if (in) {
      a0 = p.sp[i]; a1 = p.sp[i + 1];
      own = !is_long(p.lbits, i);
    }
    acc = rb_dot<double>(p.scol, p.sval, p.xh, blk.z, blk.w, a0, a1, in, blk.y - blk.x, lds);
  } else {
    const int l = ((int)blockIdx.x - p.nbS) * kBlock + threadIdx.x;
    own = l < p.nL + p.nD;
    if (own) {
      i = p.lrow[l];
      acc = p.rsum[l];
    }
  }
  double q[3] = {0.0, 0.0, 0.0};
  if (own) {
    const double lo = p.lc[i], hi = p.uc[i];
    const double viol = acc - clampv(acc, lo, hi);
    const double pr = viol / p.dr[i];
    q[0] = pr * pr;
    const double yh = p.yh[i];
    q[1] = (finite(lo) ? lo * fmax(yh, 0.0) : 0.0) - (finite(hi) ? hi * fmax(-yh, 0.0) : 0.0);
    q[2] = fabs(viol);
    p.ax_out[i] = acc;
  }
  block_reduce_store<3>(q, p.partials + (int64_t)blockIdx.x * kRegionStride, 4u);
}

// Power iteration with panels (setup): w = A~ v from AS for the short rows
// and from the panel row sums for the long and dense rows, with its compact
// copy w[m + l]; then u = A~^T w and the block partial sums of u_j^2.
__global__ __launch_bounds__(kBlock) void k_pw_rows(const int4* __restrict__ rb, const int32_t* __restrict__ sp,
                                                   const int32_t* __restrict__ scol, const double* __restrict__ sval,
                                                   const double* __restrict__ v, const uint32_t* __restrict__ lbits,
                                                   const int32_t* __restrict__ lrow, const double* __restrict__ rsum,
                                                   int32_t nbS, int32_t m, int32_t nc, double* __restrict__ w,
                                                   const PowerState* __restrict__ ps) {
  if (ps->done) return;
  __shared__ double lds[kRbLds];
  if ((int)blockIdx.x < nbS) {
    const int4 blk = rb[blockIdx.x];
    const int i = blk.x + threadIdx.x;
    const bool in = i < blk.y;
    int a0 = 0, a1 = 0;
    if (in) { a0 = sp[i]; a1 = sp[i + 1]; }
    const double h = rb_dot<double>(scol, sval, v, blk.z, blk.w, a0, a1, in, blk.y - blk.x, lds);
    if (in && !is_long(lbits, i)) w[i] = h;
  } else {
    const int l = ((int)blockIdx.x - nbS) * kBlock + threadIdx.x;
    if (l < nc) {
      const double h = rsum[l];
      w[lrow[l]] = h;
      w[m + l] = h;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_pw_cols(const int4* __restrict__ rb, const int32_t* __restrict__ cp,
                                                   const int32_t* __restrict__ row, const double* __restrict__ tval,
                                                   const double* __restrict__ w, const double* __restrict__ partT,
                                                   int32_t PT, int32_t n, double* __restrict__ u,
                                                   double* __restrict__ partials, const PowerState* __restrict__ ps) {
  if (ps->done) return;
  __shared__ double lds[kRbLds];
  const int4 blk = rb[blockIdx.x];
  const int j = blk.x + threadIdx.x;
  const bool own = j < blk.y;
  int a0 = 0, a1 = 0;
  if (own) { a0 = cp[j]; a1 = cp[j + 1]; }
  double g = rb_dot<double>(row, tval, w, blk.z, blk.w, a0, a1, own, blk.y - blk.x, lds);
  if (PT > 0 && own) g += slice_sum(partT, PT, n, j);
  double q[1] = {0.0};
  if (own) {
    u[j] = g;
    q[0] = g * g;
  }
  block_reduce_store<1>(q, partials + blockIdx.x);
}

struct Dual32PanelArgs {
  const int4* rb; const int32_t* sp; const int32_t* scol; const float* sval; const float* xbar;
  float* y; const float* ya; const float* lc; const float* uc; const float* b; const StepDev* step;
  const uint32_t* lbits; const int32_t* lrow; const float* part; const float* part2;
  int32_t P, nL, nbS, j, m, nbC, nD, G;
};

__device__ __forceinline__ void dual32_pn_update(const Dual32PanelArgs& p, int i, int l, float h, float yi, float lo,
                                                 float hi, float yai, float bi) {
  const float sigma = (float)p.step->sigma, gam = (float)p.step->gamma, a = (float)halpern_a(p.step, p.j);
  const float w = h - (bi + yi) / sigma;
  const float yh = yi + sigma * (clampv(w, lo, hi) - h);
  const float yn = a * ((1.0f + gam) * yh - gam * yi) + (1.0f - a) * yai;
  p.y[i] = yn;
  if (l >= 0) p.y[p.m + l] = yn;
}

template <bool NT>
__device__ __forceinline__ void short_block(const Dual32PanelArgs& p, int b, float* lds) {
  const int4 blk = p.rb[b];
  const int i = blk.x + threadIdx.x;
  const bool in = i < blk.y;
  bool own = false;
  float yi = 0.0f, lo = 0.0f, hi = 0.0f, yai = 0.0f, bi = 0.0f;
  int a0 = 0, a1 = 0;
  if (in) {
    a0 = p.sp[i]; a1 = p.sp[i + 1];
    own = !is_long(p.lbits, i);
    if (own) { yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; bi = p.b[i]; }
  }
  const float h = rb_dot<float, NT>(p.scol, p.sval, p.xbar, blk.z, blk.w, a0, a1, in, blk.y - blk.x, lds);
  if (own) dual32_pn_update(p, i, -1, h, yi, lo, hi, yai, bi);
}

template <bool NT>
__global__ __launch_bounds__(kBlock) void k_dual32_pn(Dual32PanelArgs p) {
  __shared__ float lds[kRbLds];
  int i = 0, l = -1;
  bool own = false;
  float h = 0.0f, yi = 0.0f, lo = 0.0f, hi = 0.0f, yai = 0.0f, bi = 0.0f;
  if ((int)blockIdx.x < p.nbS) {
    short_block<NT>(p, blockIdx.x, lds);
    return;
  } else if ((int)blockIdx.x < p.nbS + p.nbC) {
    l = ((int)blockIdx.x - p.nbS) * kBlock + threadIdx.x;
    own = l < p.nL;
    if (own) {
      i = p.lrow[l];
      yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; bi = p.b[i];
      h = panel_sum(p.part, p.P, p.nL, l);
    }
  } else {
    const int d = ((int)blockIdx.x - p.nbS - p.nbC) * kBlock + threadIdx.x;
    own = d < p.nD;
    if (own) {
      l = p.nL + d;
      i = p.lrow[l];
      yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; bi = p.b[i];
      h = group_sum(p.part2, p.G, p.nD, d);
    }
  }
  if (own) dual32_pn_update(p, i, l, h, yi, lo, hi, yai, bi);
}

// The plain dual half-step's latency-bound blocks in one launch: the long
// rows' panel blocks and the short rows' blocks (with their update), so the
// short rows run beside the panels instead of after them.  Block b runs on
// XCD x = b mod 8 (workgroups are dealt to the XCDs in turn); of XCD x's R
// slots t = b / 8, the np_x panel blocks of its panels take the slots with
// floor((t+1) np_x / R) > floor(t np_x / R), spread evenly, so each panel
// keeps its XCD; the u-th other slot of XCD x takes short block u*8 + x.
// R = max over x of np_x + ceil((nbS - x) / 8) (host), so every block has a slot.
template <typename T, typename SA>
struct DualPsArgs {
  PanelDotArgs<T> pn;
  SA s;
  int32_t R;
};

template <typename T, bool NT, typename SA>
__global__ __launch_bounds__(kBlock) void k_dual_ps(DualPsArgs<T, SA> a) {
  __shared__ T lds[kRbLds];
  const int x = blockIdx.x & 7, t = blockIdx.x >> 3;
  const int np = a.pn.off[x + 1] - a.pn.off[x];
  const int c0 = (int)((int64_t)t * np / a.R), c1 = (int)((int64_t)(t + 1) * np / a.R);
  if (c1 > c0) {  // uniform over the block
    panel_dot_block<T, NT>(a.pn, a.pn.off[x] + c0, lds);
    return;
  }
  const int g = (t - c0) * 8 + x;
  if (g < a.s.nbS) short_block<NT>(a.s, g, lds);
}

// Column side of the KKT error at (xhat, yhat): g~ = c~ - A~^T yhat,
// r~ = proj_R(g~), ||(g~ - r~)/d_c||^2, the column part of the dual objective,
// c~^T xhat; in mixed mode also the max dual violation |g~ - r~| and the max
// bound violation of xhat (scaled space), and A~^T yhat itself.
struct KktColArgs {
  const int32_t* rb; const int32_t* cp; const int32_t* row; const double* tval;
  const double* yh; const double* xh; const double* ct; const double* lv; const double* uv;
  const double* dc; double* r_out; double* aty_out; double* partials;
  const double* partT;  // if PT > 0: the dense rows' part of A~^T yhat, PT slice sums per column
  int32_t PT, n;
};

template <bool MIXED>
__global__ __launch_bounds__(kBlock) void k_kkt_cols(KktColArgs p) {
  __shared__ double lds[kRbLds];
  const int s = p.rb[blockIdx.x], e = p.rb[blockIdx.x + 1];
  const int j = s + threadIdx.x;
  const bool own = j < e;
  int a0 = 0, a1 = 0;
  if (own) {
    a0 = p.cp[j];
    a1 = p.cp[j + 1];
  }
  double acc = rb_dot<double>(p.row, p.tval, p.yh, p.cp[s], p.cp[e], a0, a1, own, e - s, lds);
  if (p.PT > 0 && own) acc += slice_sum(p.partT, p.PT, p.n, j);
  double q[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (own) {
    const double g = p.ct[j] - acc;
    const double lo = p.lv[j], hi = p.uv[j];
    const bool fl = finite(lo), fu = finite(hi);
    const double r = (fl && fu) ? g : (fl ? fmax(g, 0.0) : (fu ? fmin(g, 0.0) : 0.0));
    const double d = p.dc[j];
    const double e2 = (g - r) / d;
    q[0] = e2 * e2;
    q[1] = (fl ? lo * fmax(r, 0.0) : 0.0) - (fu ? hi * fmax(-r, 0.0) : 0.0);
    const double xj = p.xh[j];
    q[2] = p.ct[j] * xj;
    if (p.r_out) p.r_out[j] = r / d;
    if (MIXED) {
      q[3] = fabs(g - r);
      q[4] = fabs(xj - clampv(xj, lo, hi));
      p.aty_out[j] = acc;
    }
  }
  if constexpr (MIXED) {
    block_reduce_store<5>(q, p.partials + (int64_t)blockIdx.x * kRegionStride, 8u | 16u);
  } else {
    double q3[3] = {q[0], q[1], q[2]};
    block_reduce_store<3>(q3, p.partials + (int64_t)blockIdx.x * kRegionStride);
  }
}

// Row side of the KKT error for a point given in FP64 (mixed mode):
// A~ xh, ||(A~xh - proj)/d_r||^2, the row dual-objective part, the max
// primal violation (scaled); stores A~ xh.
struct KktRowArgs {
  const int32_t* rb; const int32_t* rp; const int32_t* col; const double* val;
  const double* xh; const double* yh; const double* lc; const double* uc; const double* dr;
  double* ax_out; double* partials;
};

__global__ __launch_bounds__(kBlock) void k_kkt_rows(KktRowArgs p) {
  __shared__ double lds[kRbLds];
  const int s = p.rb[blockIdx.x], e = p.rb[blockIdx.x + 1];
  const int i = s + threadIdx.x;
  const bool own = i < e;
  int a0 = 0, a1 = 0;
  if (own) {
    a0 = p.rp[i];
    a1 = p.rp[i + 1];
  }
  const double acc = rb_dot<double>(p.col, p.val, p.xh, p.rp[s], p.rp[e], a0, a1, own, e - s, lds);
  double q[3] = {0.0, 0.0, 0.0};
  if (own) {
    const double lo = p.lc[i], hi = p.uc[i];
    const double viol = acc - clampv(acc, lo, hi);
    const double pr = viol / p.dr[i];
    q[0] = pr * pr;
    const double yh = p.yh[i];
    q[1] = (finite(lo) ? lo * fmax(yh, 0.0) : 0.0) - (finite(hi) ? hi * fmax(-yh, 0.0) : 0.0);
    q[2] = fabs(viol);
    p.ax_out[i] = acc;
  }
  block_reduce_store<3>(q, p.partials + (int64_t)blockIdx.x * kRegionStride, 4u);
}

// ============================================================================ FP32 (mixed)
// Shifted coordinates x = xc + x'/P, y = yc + y'/D; the step on (x', y') is
// the same PDHG step with tau' = tau P/D, sigma' = sigma D/P and data
// (c', lv', uv', lc', uc', b):  yhat' = y' + sigma'(clamp(h - (b + y')/sigma') - h).
// Products and sums in FP32; the check partials accumulate in FP64.
struct Primal32Args {
  const int4* rb; const int32_t* cp; const int32_t* row; const float* tval;
  const float* y; float* x; const float* xa; const float* c; const float* lv; const float* uv;
  float* xbar; float* xh; float* dx; double* partials; const StepDev* step;
  int32_t j;
  const float* partT;
  int32_t PT, n;
};

template <bool RES, bool NT>
__global__ __launch_bounds__(kBlock) void k_primal32(Primal32Args p) {
  __shared__ float lds[kRbLds];
  const int4 blk = p.rb[blockIdx.x];
  const int s = blk.x, e = blk.y, ps = blk.z, pe = blk.w;
  const int j = s + threadIdx.x;
  const bool own = j < e;
  float xj = 0.0f, cj = 0.0f, lo = 0.0f, hi = 0.0f, xaj = 0.0f;
  int a0 = 0, a1 = 0;
  if (own) {
    xj = p.x[j]; cj = p.c[j]; lo = p.lv[j]; hi = p.uv[j]; xaj = p.xa[j];
    a0 = p.cp[j]; a1 = p.cp[j + 1];
  }
  float g = rb_dot<float, NT>(p.row, p.tval, p.y, ps, pe, a0, a1, own, e - s, lds);
  if (p.PT > 0 && own) g += slice_sum(p.partT, p.PT, p.n, j);
  double q0 = 0.0, q1 = 0.0;
  if (own) {
    const float tau = (float)p.step->tau, gam = (float)p.step->gamma, a = (float)halpern_a(p.step, p.j);
    const float v = xj - tau * (cj - g);
    const float xh = clampv(v, lo, hi);
    p.xbar[j] = 2.0f * xh - xj;
    p.x[j] = a * ((1.0f + gam) * xh - gam * xj) + (1.0f - a) * xaj;
    if (RES) {
      p.xh[j] = xh;
      const float d = xj - xh;
      p.dx[j] = d;
      q0 = (double)d * (double)d;
      const double e2 = (double)(xh - xaj);
      q1 = e2 * e2;
    }
  }
  if (RES) {
    double v[2] = {q0, q1};
    block_reduce_store<2>(v, p.partials + (int64_t)blockIdx.x * kRegionStride);
  }
}

struct Dual32Args {
  const int4* rb; const int32_t* rp; const int32_t* col; const float* val;
  const float* xbar; const float* dx;
  float* y; const float* ya; const float* lc; const float* uc; const float* b;
  float* yh; double* partials; const StepDev* step;
  int32_t j;
};

template <bool RES, bool NT>
__global__ __launch_bounds__(kBlock) void k_dual32(Dual32Args p) {
  __shared__ double lds[kRbLds];
  const int4 blk = p.rb[blockIdx.x];
  const int s = blk.x, e = blk.y, ps = blk.z, pe = blk.w;
  const int i = s + threadIdx.x;
  const bool own = i < e;
  float yi = 0.0f, lo = 0.0f, hi = 0.0f, yai = 0.0f, bi = 0.0f;
  int a0 = 0, a1 = 0;
  if (own) {
    yi = p.y[i]; lo = p.lc[i]; hi = p.uc[i]; yai = p.ya[i]; bi = p.b[i];
    a0 = p.rp[i]; a1 = p.rp[i + 1];
  }
  const float h = rb_dot<float, NT>(p.col, p.val, p.xbar, ps, pe, a0, a1, own, e - s, reinterpret_cast<float*>(lds));
  double adx = 0.0;
  if (RES) adx = rb_dot<double>(p.col, p.val, p.dx, ps, pe, a0, a1, own, e - s, lds);
  double q[3] = {0.0, 0.0, 0.0};
  if (own) {
    const float sigma = (float)p.step->sigma, gam = (float)p.step->gamma, a = (float)halpern_a(p.step, p.j);
    const float w = h - (bi + yi) / sigma;
    const float yh = yi + sigma * (clampv(w, lo, hi) - h);
    p.y[i] = a * ((1.0f + gam) * yh - gam * yi) + (1.0f - a) * yai;
    if (RES) {
      p.yh[i] = yh;
      const double dy = (double)(yi - yh);
      q[0] = dy * dy;
      q[1] = dy * adx;
      const double e2 = (double)(yh - yai);
      q[2] = e2 * e2;
    }
  }
  if (RES) block_reduce_store<3>(q, p.partials + (int64_t)blockIdx.x * kRegionStride);
}

// ============================================================================ elementwise
__global__ void k_restart_copy(double* x, double* xa, const double* xh, double* y, double* ya,
                               const double* yh, int32_t n, int32_t m, int32_t to_current) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    double v = to_current ? x[i] : xh[i];
    xa[i] = v;
    x[i] = v;
  }
  if (i < m) {
    double v = to_current ? y[i] : yh[i];
    ya[i] = v;
    y[i] = v;
  }
}

__global__ void k_warm_start(const double* x0, const double* y0, const double* dr, const double* dc,
                             double* x, double* xa, double* y, double* ya, int32_t n, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    double v = x0 ? x0[i] / dc[i] : 0.0;
    x[i] = v;
    xa[i] = v;
  }
  if (i < m) {
    double v = y0 ? y0[i] / dr[i] : 0.0;
    y[i] = v;
    ya[i] = v;
  }
}

__global__ void k_unscale(const double* xh, const double* yh, const double* dr, const double* dc,
                          double* x, double* y, int32_t n, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (x && i < n) x[i] = dc[i] * xh[i];
  if (y && i < m) y[i] = dr[i] * yh[i];
}

__global__ void k_trace(const double* xh, const double* yh, const double* x, const double* y,
                        double* dst, int32_t n, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    dst[i] = xh[i];
    dst[(int64_t)n + m + i] = x[i];
  }
  if (i < m) {
    dst[(int64_t)n + i] = yh[i];
    dst[2 * (int64_t)n + m + i] = y[i];
  }
}

__global__ void k_trace32(const float* xh, const float* yh, const float* x, const float* y,
                          const double* xc, const double* yc, const StepDev* st, double* dst,
                          int32_t n, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const double P = st->P, D = st->D;
  if (i < n) {
    dst[i] = xc[i] + (double)xh[i] / P;
    dst[(int64_t)n + m + i] = xc[i] + (double)x[i] / P;
  }
  if (i < m) {
    dst[(int64_t)n + i] = yc[i] + (double)yh[i] / D;
    dst[2 * (int64_t)n + m + i] = yc[i] + (double)y[i] / D;
  }
}

__global__ void k_poison(double* x) { x[0] = __builtin_nan(""); }

// xh <- xc + xh32/P, yh <- yc + yh32/D (the FP64 point of the shifted iterate)
__global__ void k_combine(const float* xh32, const float* yh32, const double* xc, const double* yc,
                          const StepDev* st, double* xh, double* yh, int32_t n, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const double P = st->P, D = st->D;
  if (i < n) xh[i] = xc[i] + (double)xh32[i] / P;
  if (i < m) yh[i] = yc[i] + (double)yh32[i] / D;
}

// New centre (xc, yc) <- (xh, yh) and the correction data from FP64 residuals
// A~ xc (ax) and A~^T yc (aty), both computed at the last check.
__global__ void k_recentre(const double* xh, const double* yh, const double* ax, const double* aty,
                           const double* ct, const double* lvt, const double* uvt, const double* lct,
                           const double* uct, double P, double D, double* xc, double* yc, float* c32,
                           float* lv32, float* uv32, float* lc32, float* uc32, float* b32, float* x32,
                           float* xa32, float* y32, float* ya32, int32_t n, int32_t m) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const double v = xh[i];
    xc[i] = v;
    c32[i] = (float)(D * (ct[i] - aty[i]));
    lv32[i] = (float)(P * (lvt[i] - v));
    uv32[i] = (float)(P * (uvt[i] - v));
    x32[i] = 0.0f;
    xa32[i] = 0.0f;
  }
  if (i < m) {
    const double v = yh[i];
    yc[i] = v;
    lc32[i] = (float)(P * (lct[i] - ax[i]));
    uc32[i] = (float)(P * (uct[i] - ax[i]));
    b32[i] = (float)(D * v);
    y32[i] = 0.0f;
    ya32[i] = 0.0f;
  }
}

// ============================================================================ finalize
struct Region {
  const double* p;
  int64_t nb;
  int32_t nq;
  uint32_t max_mask;
  int8_t q[8];
};
struct FinArgs {
  Region r[4];
  double* dst;
};

// One block per region; each quantity summed (or maxed) over blocks in order.
__global__ void k_finalize(FinArgs a) {
  const Region R = a.r[blockIdx.x];
  for (int k = 0; k < R.nq; ++k) {
    const bool mx = (R.max_mask >> k) & 1u;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < R.nb; b += kBlock) {
      const double v = R.p[b * kRegionStride + k];
      s = mx ? (v > s ? v : s) : s + v;
    }
    double v[1] = {s};
    __shared__ double tot[1];
    block_reduce_store<1>(v, tot, mx ? 1u : 0u);
    __syncthreads();
    if (threadIdx.x == 0) a.dst[R.q[k]] = tot[0];
    __syncthreads();
  }
}

// Large regions first go through this: block (c, r) reduces blocks
// [c*chunk, (c+1)*chunk) of region r, all its quantities in one pass over
// whole rows of partials, into out[(r*G + c)*kRegionStride + k]; k_finalize
// then reduces the G chunk results in order.
__global__ void k_finalize_chunks(FinArgs a, int64_t chunk, int32_t G, double* out) {
  const Region R = a.r[blockIdx.y];
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = min(R.nb, b0 + chunk);
  double acc[kRegionStride];
#pragma unroll
  for (int k = 0; k < kRegionStride; ++k) acc[k] = 0.0;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += kBlock) {
    const double2* row = reinterpret_cast<const double2*>(R.p + b * kRegionStride);
#pragma unroll
    for (int h = 0; h < kRegionStride / 2; ++h) {
      const double2 v = row[h];
      const bool m0 = (R.max_mask >> (2 * h)) & 1u, m1 = (R.max_mask >> (2 * h + 1)) & 1u;
      acc[2 * h] = m0 ? (v.x > acc[2 * h] ? v.x : acc[2 * h]) : acc[2 * h] + v.x;
      acc[2 * h + 1] = m1 ? (v.y > acc[2 * h + 1] ? v.y : acc[2 * h + 1]) : acc[2 * h + 1] + v.y;
    }
  }
  block_reduce_store<kRegionStride>(acc, out + ((int64_t)blockIdx.y * G + blockIdx.x) * kRegionStride, R.max_mask);
}

// ============================================================================ dispatch helpers
Region make_region(const double* p, int64_t nb, std::initializer_list<int> qs, uint32_t max_mask) {
  Region r{};
  r.p = p;
  r.nb = nb;
  r.nq = (int32_t)qs.size();
  r.max_mask = max_mask;
  int k = 0;
  for (int q : qs) r.q[k++] = (int8_t)q;
  return r;
}

// A half-step launch; with events in s, they take the kernel's own start and
// end timestamps (for the per-kernel timing of hlp_profile_iterations).
template <typename K, typename A>
hipError_t launch_step_kernel(K kernel, int32_t nblk, const StepArgs& s, hipStream_t st, const A& a) {
  if (s.ev_start || s.ev_stop)
    hipExtLaunchKernelGGL(kernel, dim3(nblk), dim3(kBlock), 0, st, s.ev_start, s.ev_stop, 0, a);
  else
    hipLaunchKernelGGL(kernel, dim3(nblk), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

// The launches of a panel half-step: the dense tiles (if dense rows), the
// panel and short blocks (k_dual_ps), the dense rows' group sums, then the
// long and dense rows' updates (kdual over its blocks past nbS).  With events,
// the start event takes the first kernel's start and the stop event the last
// kernel's end.
template <typename T, typename KD, typename AD>
hipError_t launch_panel_dual(hlp_lp* lp, const T* pval, const T* pvalD, const T* vec, KD kdual, const AD& ad,
                             const StepArgs& s) {
  const bool finish = lp->nbC + lp->nbCD > 0;
  StepArgs first = s, mid = s, last = s;
  first.ev_stop = nullptr;
  mid.ev_start = mid.ev_stop = nullptr;
  last.ev_start = nullptr;
  bool started = false;
  auto take = [&](bool is_last) -> StepArgs {
    StepArgs a = started ? (is_last ? last : mid) : (is_last ? s : first);
    started = true;
    return a;
  };
  hipError_t e;
  if (lp->nD > 0) {
    DenseDotArgs<T> da{reinterpret_cast<const int4*>(lp->tilesD), reinterpret_cast<const int4*>(lp->rbxD), lp->ppD,
                       lp->pcolD, pvalD, vec, reinterpret_cast<T*>(lp->partD), lp->n};
    e = lp->nt ? launch_step_kernel(k_dense_dot<T, true, kDenseW>, lp->ntilesD, take(false), lp->stream, da)
               : launch_step_kernel(k_dense_dot<T, false, kDenseW>, lp->ntilesD, take(false), lp->stream, da);
    if (e != hipSuccess) return e;
  }
  DualPsArgs<T, AD> pa{{reinterpret_cast<const int4*>(lp->tabP), lp->pp, lp->pcol, pval, vec,
                        reinterpret_cast<T*>(lp->ppart), {}},
                       ad, 0};
  int64_t R = 0;
  for (int x = 0; x < 8; ++x) {
    pa.pn.off[x] = lp->nL > 0 ? lp->poff[x] : 0;
    const int64_t np = lp->nL > 0 ? lp->poff[x + 1] - lp->poff[x] : 0;
    R = std::max<int64_t>(R, np + std::max<int64_t>(0, ((int64_t)ad.nbS - x + 7) / 8));
  }
  pa.pn.off[8] = lp->nL > 0 ? lp->poff[8] : 0;
  pa.R = (int32_t)R;
  if (R > 0) {
    e = lp->nt ? launch_step_kernel(k_dual_ps<T, true, AD>, (int32_t)(8 * R), take(!finish && lp->nD == 0), lp->stream, pa)
               : launch_step_kernel(k_dual_ps<T, false, AD>, (int32_t)(8 * R), take(!finish && lp->nD == 0), lp->stream, pa);
    if (e != hipSuccess) return e;
  }
  if (lp->nD > 0) {
    const int32_t G = (lp->dense_P + kDenseGroup - 1) / kDenseGroup;
    const StepArgs ev = take(!finish);
    if (ev.ev_start || ev.ev_stop)
      hipExtLaunchKernelGGL(k_dense_combine<T>, dim3(lp->nbCD, G), dim3(kBlock), 0, lp->stream, ev.ev_start,
                            ev.ev_stop, 0, reinterpret_cast<const T*>(lp->partD), lp->nD, lp->dense_P,
                            reinterpret_cast<T*>(lp->part2D));
    else
      hipLaunchKernelGGL(k_dense_combine<T>, dim3(lp->nbCD, G), dim3(kBlock), 0, lp->stream,
                         reinterpret_cast<const T*>(lp->partD), lp->nD, lp->dense_P, reinterpret_cast<T*>(lp->part2D));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!finish) return hipSuccess;
  AD f = ad;
  f.nbS = 0;
  return launch_step_kernel(kdual, lp->nbC + lp->nbCD, take(true), lp->stream, f);
}

// The primal half-step with dense rows: the tiles of ATD (slices of the
// compact copy of y in LDS) write the slice sums, then the row-block kernel
// over ATR adds them.  Events as for launch_panel_dual.
template <typename T, typename A, typename K>
hipError_t launch_primal_pair(hlp_lp* lp, const T* tvalT, const T* y, const A& a, K kprimal, const StepArgs& s) {
  StepArgs first = s, last = s;
  first.ev_stop = nullptr;
  last.ev_start = nullptr;
  DenseDotArgs<T> da{reinterpret_cast<const int4*>(lp->tilesT), reinterpret_cast<const int4*>(lp->rbxT2), lp->ppT,
                     lp->rowT, tvalT, y + lp->m + lp->nL, reinterpret_cast<T*>(lp->partT), lp->nD};
  hipError_t e = lp->nt ? launch_step_kernel(k_dense_dot<T, true, kDenseWT>, lp->ntilesT, first, lp->stream, da)
                        : launch_step_kernel(k_dense_dot<T, false, kDenseWT>, lp->ntilesT, first, lp->stream, da);
  if (e != hipSuccess) return e;
  return launch_step_kernel(kprimal, lp->nbR, last, lp->stream, a);
}

// The panel pipeline of one product A~ v for the long and dense rows, into
// out[0, nL + nD) (no events): products and sums in T over values and a
// vector of type V (pval, pvalD: the AP and AD values of that type).
template <typename T, typename V>
hipError_t panel_rowsums_t(hlp_lp* lp, const V* pval, const V* pvalD, const V* v, double* out) {
  hipError_t e;
  const int32_t G = (lp->dense_P + kDenseGroup - 1) / kDenseGroup;
  T* partD = reinterpret_cast<T*>(lp->partD);
  T* part2D = reinterpret_cast<T*>(lp->part2D);
  T* ppart = reinterpret_cast<T*>(lp->ppart);
  if (lp->nD > 0) {
    DenseDotArgs<T, V> da{reinterpret_cast<const int4*>(lp->tilesD), reinterpret_cast<const int4*>(lp->rbxD),
                          lp->ppD, lp->pcolD, pvalD, v, partD, lp->n};
    hipLaunchKernelGGL((k_dense_dot<T, false, kDenseW, V>), dim3(lp->ntilesD), dim3(kBlock), 0, lp->stream, da);
    hipLaunchKernelGGL(k_dense_combine<T>, dim3(lp->nbCD, G), dim3(kBlock), 0, lp->stream, (const T*)partD, lp->nD,
                       lp->dense_P, part2D);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (lp->nL > 0) {
    PanelDotArgs<T, V> pa{reinterpret_cast<const int4*>(lp->tabP), lp->pp, lp->pcol, pval, v, ppart, {}};
    for (int k = 0; k < 9; ++k) pa.off[k] = lp->poff[k];
    hipLaunchKernelGGL((k_panel_dot<T, false, V>), dim3(lp->nbPgrid), dim3(kBlock), 0, lp->stream, pa);
  }
  hipLaunchKernelGGL(k_pn_rowsums<T>, dim3(nblocks((int64_t)lp->nL + lp->nD)), dim3(kBlock), 0, lp->stream,
                     (const T*)ppart, (const T*)part2D, lp->panels, lp->nL, lp->nD, G, out);
  return hipGetLastError();
}

hipError_t panel_rowsums(hlp_lp* lp, const double* v, double* out) {
  return panel_rowsums_t<double, double>(lp, lp->pval, lp->pvalD, v, out);
}

// The FP32 path's check dual half-step with panels: h as the plain FP32
// panel half-step sums it (FP32 partials in panel order), A~ dx in FP64.
hipError_t launch_dual32_res_panels(hlp_lp* lp, const StepArgs& s) {
  const int64_t nc = (int64_t)lp->nL + lp->nD;
  hipError_t e;
  if ((e = panel_rowsums_t<float, float>(lp, lp->pval32, lp->pval32D, lp->xbar32, lp->rsum)) != hipSuccess) return e;
  if ((e = panel_rowsums_t<double, float>(lp, lp->pval32, lp->pval32D, lp->dx32, lp->rsum + nc)) != hipSuccess)
    return e;
  Dual32ResArgs d{reinterpret_cast<const int4*>(lp->rbxS), lp->sp, lp->scol, lp->sval32, lp->xbar32, lp->dx32,
                  lp->y32, lp->ya32, lp->lc32, lp->uc32, lp->b32, lp->yh32, region(lp, R_DUAL), lp->step,
                  lp->lbits, lp->lrow, lp->rsum, lp->nbS, s.j, lp->m, lp->nL, lp->nD};
  const int32_t nb = lp->nbS + (int32_t)((nc + kBlock - 1) / kBlock);
  lp->nb_dual_region = nb;
  return launch_step_kernel(k_dual32_pn_res, nb, s, lp->stream, d);
}

hipError_t launch_dual_res_panels(hlp_lp* lp, const StepArgs& s) {
  const int64_t nc = (int64_t)lp->nL + lp->nD;
  hipError_t e;
  if ((e = panel_rowsums(lp, lp->xbar, lp->rsum)) != hipSuccess) return e;
  if ((e = panel_rowsums(lp, lp->dxv, lp->rsum + nc)) != hipSuccess) return e;
  if ((e = panel_rowsums(lp, lp->xh, lp->rsum + 2 * nc)) != hipSuccess) return e;
  DualResArgs d{reinterpret_cast<const int4*>(lp->rbxS), lp->sp, lp->scol, lp->sval, lp->xbar, lp->dxv, lp->xh,
                lp->y, lp->ya, lp->lct, lp->uct, lp->dr, lp->yh, region(lp, R_DUAL), lp->step, lp->lbits, lp->lrow,
                lp->rsum, lp->nbS, s.j, lp->m, lp->nL, lp->nD};
  const int32_t nb = lp->nbS + (int32_t)((nc + kBlock - 1) / kBlock);
  lp->nb_dual_region = nb;
  return launch_step_kernel(k_dual_pn_res, nb, s, lp->stream, d);
}

}  // namespace

// One power pass u = A~^T (A~ v) with the panel layout; block partial sums of
// u_j^2 into lp->partials, their count into *nb.
hipError_t launch_power_pass_panels(hlp_lp* lp, int64_t* nb) {
  const int32_t nc = lp->nL + lp->nD;
  hipError_t e;
  if ((e = panel_rowsums(lp, lp->pv, lp->rsum)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pw_rows, dim3(lp->nbS + (nc + kBlock - 1) / kBlock), dim3(kBlock), 0, lp->stream,
                     reinterpret_cast<const int4*>(lp->rbxS), lp->sp, lp->scol, lp->sval, lp->pv, lp->lbits, lp->lrow,
                     lp->rsum, lp->nbS, lp->m, nc, lp->pu, (const PowerState*)lp->pstate);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (lp->ntilesT > 0) {
    DenseDotArgs<double> da{reinterpret_cast<const int4*>(lp->tilesT), reinterpret_cast<const int4*>(lp->rbxT2),
                            lp->ppT, lp->rowT, lp->tvalT, lp->pu + lp->m + lp->nL, lp->partT, lp->nD};
    hipLaunchKernelGGL((k_dense_dot<double, false, kDenseWT>), dim3(lp->ntilesT), dim3(kBlock), 0, lp->stream, da);
    hipLaunchKernelGGL(k_pw_cols, dim3(lp->nbR), dim3(kBlock), 0, lp->stream, reinterpret_cast<const int4*>(lp->rbxR),
                       lp->cpR, lp->rowR, lp->tvalR, (const double*)lp->pu, (const double*)lp->partT, lp->dense_PT,
                       lp->n, lp->pw, lp->partials, (const PowerState*)lp->pstate);
    *nb = lp->nbR;
  } else {
    hipLaunchKernelGGL(k_pw_cols, dim3(lp->nbT), dim3(kBlock), 0, lp->stream, reinterpret_cast<const int4*>(lp->rbxT),
                       lp->cp, lp->rowc, lp->tval, (const double*)lp->pu, (const double*)nullptr, 0, lp->n, lp->pw,
                       lp->partials, (const PowerState*)lp->pstate);
    *nb = lp->nbT;
  }
  return hipGetLastError();
}

namespace {

template <typename T>
hipError_t refresh_long_y(hlp_lp* lp, T* y) {
  const int32_t nc = lp->nL + lp->nD;  // long rows, then dense rows
  if (!lp->panels || nc == 0 || !y) return hipSuccess;
  hipLaunchKernelGGL(k_refresh_long_y<T>, dim3(nblocks(nc)), dim3(kBlock), 0, lp->stream, y, lp->lrow, nc, lp->m);
  return hipGetLastError();
}

}  // namespace

// ============================================================================ launchers
hipError_t launch_set_step(hlp_lp* lp, double tau, double sigma, double gamma, int64_t k0, double P, double D) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, lp->stream, lp->step, tau, sigma, gamma, k0, P, D);
  return hipGetLastError();
}

hipError_t launch_primal(hlp_lp* lp, const StepArgs& s) {
  if (lp->nbT == 0) return hipSuccess;
  PrimalArgs a{reinterpret_cast<const int4*>(lp->rbxT), lp->cp, lp->row, lp->tval, lp->y, lp->x, lp->xa, lp->ct, lp->lvt, lp->uvt,
               lp->xbar, lp->xh, lp->dxv, region(lp, R_PRIMAL), s.mask_x, lp->step, s.j};
  if (s.mask_x) return launch_step_kernel(k_primal<2, false>, lp->nbT, s, lp->stream, a);
  const bool split = lp->panels && lp->ntilesT > 0;
  if (split) {
    // dense rows' part first (slices of y staged in LDS), then the rest
    a.rb = reinterpret_cast<const int4*>(lp->rbxR);
    a.cp = lp->cpR;
    a.row = lp->rowR;
    a.tval = lp->tvalR;
    a.partT = lp->partT;
    a.PT = lp->dense_PT;
    a.n = lp->n;
  }
  if (s.residual) {
    lp->nb_primal_region = split ? lp->nbR : lp->nbT;
    if (split) return launch_primal_pair(lp, lp->tvalT, lp->y, a, k_primal<1, false>, s);
    return launch_step_kernel(k_primal<1, false>, lp->nbT, s, lp->stream, a);
  }
  if (split) return launch_primal_pair(lp, lp->tvalT, lp->y, a, lp->nt ? k_primal<0, true> : k_primal<0, false>, s);
  if (lp->panels) a.row = lp->rowc;  // long rows' y entries from the compact copy
  if (lp->nt) return launch_step_kernel(k_primal<0, true>, lp->nbT, s, lp->stream, a);
  return launch_step_kernel(k_primal<0, false>, lp->nbT, s, lp->stream, a);
}

hipError_t launch_dual(hlp_lp* lp, const StepArgs& s) {
  if (lp->nbA == 0) return hipSuccess;
  DualArgs a{reinterpret_cast<const int4*>(lp->rbxA), lp->rp, lp->col, lp->val, lp->xbar, lp->dxv, lp->xh, lp->y, lp->ya, lp->lct, lp->uct,
             lp->dr, lp->yh, region(lp, R_DUAL), s.mask_y, lp->step, s.j};
  if (s.residual && !s.mask_y && lp->panels) return launch_dual_res_panels(lp, s);
  if (s.mask_y || s.residual) {
    lp->nb_dual_region = lp->nbA;
    hipError_t e = s.mask_y ? launch_step_kernel(k_dual<2, false>, lp->nbA, s, lp->stream, a)
                            : launch_step_kernel(k_dual<1, false>, lp->nbA, s, lp->stream, a);
    return e != hipSuccess ? e : refresh_long_y(lp, lp->y);
  }
  if (lp->panels) {
    const int32_t G = (lp->dense_P + kDenseGroup - 1) / kDenseGroup;
    DualPanelArgs d{reinterpret_cast<const int4*>(lp->rbxS), lp->sp, lp->scol, lp->sval, lp->xbar, lp->y, lp->ya,
                    lp->lct, lp->uct, lp->step, lp->lbits, lp->lrow, lp->ppart, lp->part2D, lp->panels, lp->nL,
                    lp->nbS, s.j, lp->m, lp->nbC, lp->nD, G};
    return lp->nt ? launch_panel_dual<double>(lp, lp->pval, lp->pvalD, lp->xbar, k_dual_pn<true>, d, s)
                  : launch_panel_dual<double>(lp, lp->pval, lp->pvalD, lp->xbar, k_dual_pn<false>, d, s);
  }
  if (lp->nt) return launch_step_kernel(k_dual<0, true>, lp->nbA, s, lp->stream, a);
  return launch_step_kernel(k_dual<0, false>, lp->nbA, s, lp->stream, a);
}

hipError_t launch_kkt_cols(hlp_lp* lp, double* r_out) {
  if (lp->nbT == 0) return hipSuccess;
  KktColArgs a{lp->rbT, lp->cp, lp->row, lp->tval, lp->yh, lp->xh, lp->ct, lp->lvt, lp->uvt, lp->dc, r_out,
               lp->atyc, region(lp, R_KKT), nullptr, 0, lp->n};
  int32_t nb = lp->nbT;
  if (lp->panels && lp->ntilesT > 0) {
    // as the primal half-step: the dense rows' entries of A~^T yhat by the
    // tiles of ATD (slices of yhat's compact copy in LDS), then ATR adds them
    hipError_t e = refresh_long_y(lp, lp->yh);
    if (e != hipSuccess) return e;
    DenseDotArgs<double> da{reinterpret_cast<const int4*>(lp->tilesT), reinterpret_cast<const int4*>(lp->rbxT2),
                            lp->ppT, lp->rowT, lp->tvalT, lp->yh + lp->m + lp->nL, lp->partT, lp->nD};
    hipLaunchKernelGGL((k_dense_dot<double, false, kDenseWT>), dim3(lp->ntilesT), dim3(kBlock), 0, lp->stream, da);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    a.rb = lp->rbR;
    a.cp = lp->cpR;
    a.row = lp->rowR;
    a.tval = lp->tvalR;
    a.partT = lp->partT;
    a.PT = lp->dense_PT;
    nb = lp->nbR;
  }
  lp->nb_kkt_region = nb;
  if (nb == 0) return hipSuccess;
  if (lp->precision == HLP_MIXED) hipLaunchKernelGGL(k_kkt_cols<true>, dim3(nb), dim3(kBlock), 0, lp->stream, a);
  else hipLaunchKernelGGL(k_kkt_cols<false>, dim3(nb), dim3(kBlock), 0, lp->stream, a);
  return hipGetLastError();
}

hipError_t launch_kkt_rows(hlp_lp* lp) {
  if (lp->nbA == 0) return hipSuccess;
  if (lp->panels) {
    const int64_t nc = (int64_t)lp->nL + lp->nD;
    hipError_t e = panel_rowsums(lp, lp->xh, lp->rsum);
    if (e != hipSuccess) return e;
    KktRowPanelArgs a{reinterpret_cast<const int4*>(lp->rbxS), lp->sp, lp->scol, lp->sval, lp->xh, lp->yh,
                      lp->lct, lp->uct, lp->dr, lp->axc, region(lp, R_ROWS), lp->lbits, lp->lrow, lp->rsum,
                      lp->nbS, lp->nL, lp->nD};
    const int32_t nb = lp->nbS + (int32_t)((nc + kBlock - 1) / kBlock);
    lp->nb_rows_region = nb;
    hipLaunchKernelGGL(k_kkt_rows_pn, dim3(nb), dim3(kBlock), 0, lp->stream, a);
    return hipGetLastError();
  }
  lp->nb_rows_region = lp->nbA;
  KktRowArgs a{lp->rbA, lp->rp, lp->col, lp->val, lp->xh, lp->yh, lp->lct, lp->uct, lp->dr, lp->axc,
               region(lp, R_ROWS)};
  hipLaunchKernelGGL(k_kkt_rows, dim3(lp->nbA), dim3(kBlock), 0, lp->stream, a);
  return hipGetLastError();
}

// which: bit 0 primal region, bit 1 dual region, bit 2 KKT-cols region,
// bit 3 KKT-rows region (mixed); bit 4 selects the FP32 layouts.
hipError_t launch_finalize(hlp_lp* lp, int32_t which, int32_t slot) {
  FinArgs a{};
  a.dst = lp->results + (int64_t)slot * NQ;
  int nr = 0;
  const bool f32 = (which & 16) != 0;
  const int64_t nbp = lp->nb_kkt_region > 0 ? lp->nb_kkt_region : lp->nbT;
  const int64_t nbd = lp->nb_dual_region > 0 ? lp->nb_dual_region : lp->nbA;
  const int64_t nbx = lp->nb_primal_region > 0 ? lp->nb_primal_region : lp->nbT;
  if (which & 1) a.r[nr++] = make_region(region(lp, R_PRIMAL), nbx, {Q_DX2, Q_XA2}, 0u);
  if (which & 2) {
    if (f32) a.r[nr++] = make_region(region(lp, R_DUAL), nbd, {Q_DY2, Q_DYADX, Q_YA2}, 0u);
    else a.r[nr++] = make_region(region(lp, R_DUAL), nbd, {Q_DY2, Q_DYADX, Q_YA2, Q_RP2, Q_DOBJ_R}, 0u);
  }
  if (which & 4) {
    if (lp->precision == HLP_MIXED)
      a.r[nr++] = make_region(region(lp, R_KKT), nbp, {Q_RD2, Q_DOBJ_C, Q_POBJ, Q_VD, Q_VX}, 8u | 16u);
    else a.r[nr++] = make_region(region(lp, R_KKT), nbp, {Q_RD2, Q_DOBJ_C, Q_POBJ}, 0u);
  }
  const int64_t nbr = lp->nb_rows_region > 0 ? lp->nb_rows_region : lp->nbA;
  if (which & 8) a.r[nr++] = make_region(region(lp, R_ROWS), nbr, {Q_RP2, Q_DOBJ_R, Q_VP}, 4u);
  if (nr == 0) return hipSuccess;
  int64_t nbmax = 0;
  for (int r = 0; r < nr; ++r) nbmax = std::max(nbmax, a.r[r].nb);
  if (nbmax > kFinDirect) {
    const int64_t chunk = std::max<int64_t>(kFinDirect, (nbmax + kFinChunks - 1) / kFinChunks);
    const int32_t G = (int32_t)((nbmax + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_finalize_chunks, dim3(G, nr), dim3(kBlock), 0, lp->stream, a, chunk, G, lp->fin_scratch);
    for (int r = 0; r < nr; ++r) {
      a.r[r].p = lp->fin_scratch + (int64_t)r * G * kRegionStride;
      a.r[r].nb = std::min<int64_t>(G, (a.r[r].nb + chunk - 1) / chunk);
    }
  }
  hipLaunchKernelGGL(k_finalize, dim3(nr), dim3(kBlock), 0, lp->stream, a);
  return hipGetLastError();
}

hipError_t launch_restart_copy(hlp_lp* lp, int32_t to_current) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_restart_copy, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->x, lp->xa, lp->xh,
                     lp->y, lp->ya, lp->yh, lp->n, lp->m, to_current);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : refresh_long_y(lp, lp->y);
}

hipError_t launch_warm_start(hlp_lp* lp, const double* x0, const double* y0) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_warm_start, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, x0, y0, lp->dr, lp->dc,
                     lp->x, lp->xa, lp->y, lp->ya, lp->n, lp->m);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : refresh_long_y(lp, lp->y);
}

hipError_t launch_unscale(hlp_lp* lp, double* x, double* y) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unscale, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->xh, lp->yh, lp->dr,
                     lp->dc, x, y, lp->n, lp->m);
  return hipGetLastError();
}

hipError_t launch_trace(hlp_lp* lp, double* dst) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->xh, lp->yh, lp->x, lp->y,
                     dst, lp->n, lp->m);
  return hipGetLastError();
}

hipError_t launch_trace32(hlp_lp* lp, double* dst) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_trace32, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->xh32, lp->yh32, lp->x32,
                     lp->y32, lp->xcen, lp->ycen, (const StepDev*)lp->step, dst, lp->n, lp->m);
  return hipGetLastError();
}

hipError_t launch_poison(hlp_lp* lp) {
  if (lp->n == 0 || lp->precision == HLP_MIXED) return hipSuccess;
  hipLaunchKernelGGL(k_poison, dim3(1), dim3(1), 0, lp->stream, lp->x);
  return hipGetLastError();
}

hipError_t launch_primal32(hlp_lp* lp, const StepArgs& s) {
  if (lp->nbT == 0) return hipSuccess;
  Primal32Args a{reinterpret_cast<const int4*>(lp->rbxT), lp->cp, lp->row, lp->tval32, lp->y32, lp->x32, lp->xa32, lp->c32, lp->lv32, lp->uv32,
                 lp->xbar32, lp->xh32, lp->dx32, region(lp, R_PRIMAL), lp->step, s.j};
  const bool split = lp->panels && lp->ntilesT > 0;
  if (split) {
    a.rb = reinterpret_cast<const int4*>(lp->rbxR);
    a.cp = lp->cpR;
    a.row = lp->rowR;
    a.tval = lp->tval32R;
    a.partT = reinterpret_cast<const float*>(lp->partT);
    a.PT = lp->dense_PT;
    a.n = lp->n;
  }
  if (s.residual) {
    lp->nb_primal_region = split ? lp->nbR : lp->nbT;
    if (split) return launch_primal_pair(lp, lp->tval32T, lp->y32, a, k_primal32<true, false>, s);
    return launch_step_kernel(k_primal32<true, false>, lp->nbT, s, lp->stream, a);
  }
  if (split)
    return launch_primal_pair(lp, lp->tval32T, lp->y32, a, lp->nt ? k_primal32<false, true> : k_primal32<false, false>,
                              s);
  if (lp->panels) a.row = lp->rowc;
  if (lp->nt) return launch_step_kernel(k_primal32<false, true>, lp->nbT, s, lp->stream, a);
  return launch_step_kernel(k_primal32<false, false>, lp->nbT, s, lp->stream, a);
}

hipError_t launch_dual32(hlp_lp* lp, const StepArgs& s) {
  if (lp->nbA == 0) return hipSuccess;
  Dual32Args a{reinterpret_cast<const int4*>(lp->rbxA), lp->rp, lp->col, lp->val32, lp->xbar32, lp->dx32, lp->y32, lp->ya32, lp->lc32, lp->uc32,
               lp->b32, lp->yh32, region(lp, R_DUAL), lp->step, s.j};
  if (s.residual) {
    if (lp->panels) return launch_dual32_res_panels(lp, s);
    lp->nb_dual_region = lp->nbA;
    hipError_t e = launch_step_kernel(k_dual32<true, false>, lp->nbA, s, lp->stream, a);
    return e != hipSuccess ? e : refresh_long_y(lp, lp->y32);
  }
  if (lp->panels) {
    const float* part = reinterpret_cast<const float*>(lp->ppart);
    const float* part2 = reinterpret_cast<const float*>(lp->part2D);
    const int32_t G = (lp->dense_P + kDenseGroup - 1) / kDenseGroup;
    Dual32PanelArgs d{reinterpret_cast<const int4*>(lp->rbxS), lp->sp, lp->scol, lp->sval32, lp->xbar32, lp->y32,
                      lp->ya32, lp->lc32, lp->uc32, lp->b32, lp->step, lp->lbits, lp->lrow, part, part2, lp->panels,
                      lp->nL, lp->nbS, s.j, lp->m, lp->nbC, lp->nD, G};
    return lp->nt ? launch_panel_dual<float>(lp, lp->pval32, lp->pval32D, lp->xbar32, k_dual32_pn<true>, d, s)
                  : launch_panel_dual<float>(lp, lp->pval32, lp->pval32D, lp->xbar32, k_dual32_pn<false>, d, s);
  }
  if (lp->nt) return launch_step_kernel(k_dual32<false, true>, lp->nbA, s, lp->stream, a);
  return launch_step_kernel(k_dual32<false, false>, lp->nbA, s, lp->stream, a);
}

hipError_t launch_combine(hlp_lp* lp) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->xh32, lp->yh32, lp->xcen,
                     lp->ycen, (const StepDev*)lp->step, lp->xh, lp->yh, lp->n, lp->m);
  return hipGetLastError();
}

hipError_t launch_recentre(hlp_lp* lp, double P, double D) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_recentre, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->xh, lp->yh, lp->axc,
                     lp->atyc, lp->ct, lp->lvt, lp->uvt, lp->lct, lp->uct, P, D, lp->xcen, lp->ycen, lp->c32,
                     lp->lv32, lp->uv32, lp->lc32, lp->uc32, lp->b32, lp->x32, lp->xa32, lp->y32, lp->ya32,
                     lp->n, lp->m);
  hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : refresh_long_y(lp, lp->y32);
}

}  // namespace hlp
