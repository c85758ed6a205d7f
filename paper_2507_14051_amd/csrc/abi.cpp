// C ABI entry points: argument checks, workspace layout, setup (validation,
// CSR copy, transpose, rescaling, power iteration) and error reporting.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hlp_internal.h"

namespace hlp {

namespace {
thread_local std::string g_err;
constexpr size_t kAlign = 256;

inline size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    size_t bytes = up(sizeof(T) * (size_t)std::max<int64_t>(count, 1));
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

const char* flag_message(int f) {
  if (f & 1) return "row_ptr must start at 0 and end at nnz";
  if (f & 2) return "row_ptr must be nondecreasing";
  if (f & 4) return "column index out of range";
  if (f & 8) return "column indices must be strictly increasing within each row";
  if (f & 16) return "matrix values must be finite";
  if (f & 32) return "c must be finite";
  if (f & 64) return "a bound is NaN";
  if (f & 128) return "a lower bound exceeds its upper bound";
  if (f & 256) return "a lower bound is +inf or an upper bound is -inf";
  return "invalid input";
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

void set_error(const std::string& msg) { g_err = msg; }

hlp_err hip_fail(hipError_t e, const char* what) {
  g_err = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what;
  return HLP_EHIP;
}

int lanes_for(double mean) {
  int L = 1;
  while (L < 64 && L < mean) L <<= 1;
  return L;
}

int32_t panel_count(int32_t n, const hlp_params* p) {
  int64_t P = 0;
  if (p->column_panels > 0) P = 8 * (((int64_t)p->column_panels + 7) / 8);
  else if (p->column_panels == -1 && n > (1 << 20)) P = 8 * (((int64_t)n + (1 << 20) - 1) >> 20);
  return (int32_t)std::min<int64_t>(P, 1024);
}

// Capacities of the panel layout for the worst row-length pattern that
// (m, n, nnz) allow: at most nnz / (T + 1) rows longer than T, at most
// min(m, nnz / Ld, kMaxDense) dense rows, every part of the matrix as large
// as the whole.
Caps worst_caps(int32_t m, int32_t n, int64_t nnz, int32_t panels, int32_t panel_row_min, int32_t dense_row_min) {
  Caps k;
  int64_t nLmax = 0, R = 0;
  if (panels > 0 && panel_row_min >= 1) {
    nLmax = std::min<int64_t>(m, nnz / ((int64_t)panel_row_min + 1));
    R = (int64_t)panels * nLmax;
    if (R + 2 >= (int64_t(1) << 30)) nLmax = R = 0;  // int32 device indexing of the panel rows
  }
  if (nLmax == 0) panels = 0;
  k.panels = panels;
  k.rows = nLmax;
  k.long_rows = nLmax;
  int64_t nDmax = 0, PT = 0;
  if (panels > 0 && dense_row_min > panel_row_min) {
    const int64_t PD = ((int64_t)n + kDenseW - 1) / kDenseW;
    nDmax = std::min<int64_t>(std::min<int64_t>(m, nnz / dense_row_min), kMaxDense);
    PT = (nDmax + kDenseWT - 1) / kDenseWT;
    if (nDmax == 0 || PD * nDmax + PD + 2 >= (int64_t(1) << 30) || PT * n + PT + 2 >= (int64_t(1) << 30))
      nDmax = PT = 0;
  }
  k.dense_rows = nDmax;
  k.dense_limit = nDmax;
  k.slices = PT;
  k.nnz_short = k.nnz_long = k.nnz_dense = k.nnz_rest = nnz;
  return k;
}

Caps exact_caps(int32_t m, int32_t n, int64_t nnz, const int64_t* rp, int32_t panels, int32_t panel_row_min,
                int32_t dense_row_min, bool automatic) {
  const Caps w = worst_caps(m, n, nnz, panels, panel_row_min, dense_row_min);
  Caps k;
  if (w.panels <= 0 || m == 0 || n == 0 || nnz == 0) return k;
  const int64_t T = panel_row_min;
  int64_t Ld = w.dense_rows == 0 ? 0 : dense_row_min;
  int64_t nL = 0, nD = 0, nnzS = 0, nnzL = 0, nnzD = 0;
  auto count = [&]() {
    nL = nD = nnzS = nnzL = nnzD = 0;
    for (int32_t i = 0; i < m; ++i) {
      const int64_t len = rp[i + 1] - rp[i];
      if (Ld > 0 && len >= Ld) {
        ++nD;
        nnzD += len;
      } else if (len > T) {
        ++nL;
        nnzL += len;
      } else {
        nnzS += len;
      }
    }
  };
  // the same threshold doubling as hlp_lp_create (build_panels)
  for (;;) {
    count();
    if (nD <= w.dense_limit || Ld == 0) break;
    Ld = Ld > n / 2 ? 0 : 2 * Ld;
  }
  if (nL + nD < 1 || nL + nD > w.rows || nD > w.dense_rows) return k;
  if (automatic && 2 * (nnz - nnzS) < nnz) return k;
  k.panels = w.panels;
  k.rows = nL + nD;
  k.long_rows = nL;
  k.dense_rows = nD;
  k.dense_limit = w.dense_limit;
  k.nnz_short = nnzS;
  k.nnz_long = nnzL;
  k.nnz_dense = nnzD;
  if (nD > 0 && 2 * nnzD >= nnz) {
    k.slices = (nD + kDenseWT - 1) / kDenseWT;
    k.nnz_rest = nnz - nnzD;
  }
  return k;
}

size_t carve(hlp_lp* lp, void* base, int32_t m, int32_t n, int64_t nnz, int32_t precision, const Caps& k) {
  Carver c{static_cast<char*>(base)};
  const bool mixed = precision == HLP_MIXED;
  const int64_t N = std::max<int64_t>(m, n);
  hlp_lp tmp;
  hlp_lp* L = lp ? lp : &tmp;
  const int32_t panels = k.rows > 0 ? k.panels : 0;
  const int64_t nLmax = panels > 0 ? k.rows : 0;     // long and dense rows
  const int64_t R = (int64_t)panels * (panels > 0 ? k.long_rows : 0);
  L->panels = panels;  // reserved count; hlp_lp_create may switch the layout off
  L->nL_cap = (int32_t)nLmax;
  // dense rows (at least dense_row_min nonzeros): narrow panels of kDenseW columns
  const int64_t nDmax = panels > 0 ? k.dense_rows : 0;
  const int64_t PD = nDmax > 0 ? ((int64_t)n + kDenseW - 1) / kDenseW : 0;
  const int64_t GD = (PD + kDenseGroup - 1) / kDenseGroup;
  const int64_t RD = PD * nDmax;
  const int64_t PT = nDmax > 0 ? k.slices : 0;
  const int64_t RT = PT * n;
  L->nD_cap = (int32_t)nDmax;
  L->nD_limit = (int32_t)(panels > 0 ? k.dense_limit : 0);
  L->dense_P = (int32_t)PD;
  L->dense_PT_cap = (int32_t)PT;
  const int64_t RB = std::max<int64_t>(std::max<int64_t>(N, R), std::max(RD, RT));
  L->rp = c.take<int32_t>((int64_t)m + 1);
  L->col = c.take<int32_t>(nnz);
  L->val0 = c.take<double>(nnz);
  L->val = c.take<double>(nnz);
  L->cp = c.take<int32_t>((int64_t)n + 1);
  L->row = c.take<int32_t>(nnz);
  L->tval0 = c.take<double>(nnz);
  L->tval = c.take<double>(nnz);
  L->val32 = mixed ? c.take<float>(nnz) : nullptr;
  L->tval32 = mixed ? c.take<float>(nnz) : nullptr;
  L->dr = c.take<double>(m);
  L->dc = c.take<double>(n);
  L->ct = c.take<double>(n);
  L->lvt = c.take<double>(n);
  L->uvt = c.take<double>(n);
  L->lct = c.take<double>(m);
  L->uct = c.take<double>(m);
  L->x = c.take<double>(n);
  L->xa = c.take<double>(n);
  L->xbar = c.take<double>(n);
  L->xh = c.take<double>(n);
  L->dxv = c.take<double>(n);
  L->rbuf = c.take<double>(n);
  // with column panels, y (and y32) carry a compact copy of the long rows'
  // entries after the m entries: y[m + l] = y[lrow[l]]
  const int64_t ycopy = panels > 0 ? nLmax : 0;
  L->y = c.take<double>(m + ycopy);
  L->ya = c.take<double>(m);
  L->yh = c.take<double>(m + ycopy);  // with the same compact copy (column-side KKT over the split transpose)
  if (mixed) {
    L->x32 = c.take<float>(n);
    L->xa32 = c.take<float>(n);
    L->xbar32 = c.take<float>(n);
    L->xh32 = c.take<float>(n);
    L->dx32 = c.take<float>(n);
    L->c32 = c.take<float>(n);
    L->lv32 = c.take<float>(n);
    L->uv32 = c.take<float>(n);
    L->y32 = c.take<float>(m + ycopy);
    L->ya32 = c.take<float>(m);
    L->yh32 = c.take<float>(m);
    L->lc32 = c.take<float>(m);
    L->uc32 = c.take<float>(m);
    L->b32 = c.take<float>(m);
  }
  // FP64 centre and residual vectors (mixed); the adjoint also uses them.
  L->xcen = c.take<double>(n);
  L->ycen = c.take<double>(m);
  L->axc = c.take<double>(m);
  L->atyc = c.take<double>(n);
  // row blocks and the step scalars
  L->rbA = c.take<int32_t>((int64_t)m + 2);
  L->rbT = c.take<int32_t>((int64_t)n + 2);
  L->rbxA = c.take<int32_t>(4 * ((int64_t)m + 1));
  L->rbxT = c.take<int32_t>(4 * ((int64_t)n + 1));
  L->rbtmp = c.take<int32_t>(2 * (RB + 1));
  L->rbtmp_rows = RB;
  L->step = c.take<StepDev>(1);
  // reductions: 4 regions of partial_blocks x 8 doubles (at most one block per
  // row, plus the long/dense-row blocks of the panel kernels)
  L->partial_blocks = N + N / 128 + 8;
  L->partials = c.take<double>(4 * L->partial_blocks * 8);
  L->results = c.take<double>(NSLOT * NQ);
  L->fin_scratch = c.take<double>(4 * 256 * 8);
  L->pstate = c.take<PowerState>(1);
  L->flags = c.take<int32_t>(8);
  // transpose scratch
  L->kA = c.take<int32_t>(nnz);
  L->kB = c.take<int32_t>(std::max<int64_t>(nnz, (int64_t)n + 1));
  L->vA = c.take<int32_t>(nnz);
  L->vB = c.take<int32_t>(nnz);
  L->rowof = c.take<int32_t>(nnz);
  const int64_t nbr = (nnz + 4095) / 4096;
  L->hist_len = 256 * std::max<int64_t>(nbr, 1);
  L->hist = c.take<int32_t>(L->hist_len);
  L->scan_tmp_len = std::max<int64_t>(L->hist_len, RB + 1) / 1024 + 2;
  L->scan_tmp = c.take<int32_t>(L->scan_tmp_len);
  if (panels > 0) {
    L->rsum = c.take<double>(3 * nLmax);
    L->lrow = c.take<int32_t>(nLmax);
    L->plid = c.take<int32_t>((int64_t)m + 1);
    L->lbits = c.take<uint32_t>(((int64_t)m + 31) / 32);
    L->sp = c.take<int32_t>((int64_t)m + 1);
    L->scol = c.take<int32_t>(k.nnz_short);
    L->sval = c.take<double>(k.nnz_short);
    L->sval32 = mixed ? c.take<float>(k.nnz_short) : nullptr;
    L->pp = c.take<int32_t>(R + 1);
    L->pcol = c.take<int32_t>(k.nnz_long);
    L->pval = c.take<double>(k.nnz_long);
    L->pval32 = mixed ? c.take<float>(k.nnz_long) : nullptr;
    L->ppart = c.take<double>(R);
    L->rbS = c.take<int32_t>((int64_t)m + 2);
    L->rbxS = c.take<int32_t>(4 * ((int64_t)m + 1));
    L->rbP = c.take<int32_t>(R + 2);
    L->rbxP = c.take<int32_t>(4 * (R + 1));
    L->tabP = c.take<int32_t>(4 * (R + 1));
    L->rowc = c.take<int32_t>(nnz);
    L->pscrA = c.take<int32_t>(RB + 1);
    L->pscrB = c.take<int32_t>(RB + 1);
    L->pscrC = c.take<int32_t>((int64_t)m + 1);
    L->dlid = c.take<int32_t>((int64_t)m + 1);
  }
  if (nDmax > 0) {
    L->ppD = c.take<int32_t>(RD + 1);
    L->pcolD = c.take<uint16_t>(k.nnz_dense);
    L->pvalD = c.take<double>(k.nnz_dense);
    L->pval32D = mixed ? c.take<float>(k.nnz_dense) : nullptr;
    L->partD = c.take<double>(RD);
    L->part2D = c.take<double>(GD * nDmax);
    const int64_t bD = std::min<int64_t>(RD, row_block_bound(RD, k.nnz_dense, PD));
    L->rbD = c.take<int32_t>(RD + 2);
    L->capD_blocks = bD + 1;
    L->rbxD = c.take<int32_t>(4 * (bD + 1));
    L->tilesD = c.take<int32_t>(4 * (bD + 1));
  }
  if (PT > 0) {
    L->cpR = c.take<int32_t>((int64_t)n + 1);
    L->rowR = c.take<int32_t>(k.nnz_rest);
    L->tvalR = c.take<double>(k.nnz_rest);
    L->tval32R = mixed ? c.take<float>(k.nnz_rest) : nullptr;
    L->ppT = c.take<int32_t>(RT + 1);
    L->rowT = c.take<uint16_t>(k.nnz_dense);
    L->tvalT = c.take<double>(k.nnz_dense);
    L->tval32T = mixed ? c.take<float>(k.nnz_dense) : nullptr;
    L->partT = c.take<double>(RT);
    const int64_t bT = std::min<int64_t>(RT, row_block_bound(RT, k.nnz_dense, PT));
    L->rbR = c.take<int32_t>((int64_t)n + 2);
    L->rbxR = c.take<int32_t>(4 * ((int64_t)n + 1));
    L->rbT2 = c.take<int32_t>(RT + 2);
    L->capT_blocks = bT + 1;
    L->rbxT2 = c.take<int32_t>(4 * (bT + 1));
    L->tilesT = c.take<int32_t>(4 * (bT + 1));
  }
  // power iteration vectors alias iteration buffers (setup only)
  L->pv = L->rbuf;
  L->pw = L->atyc;
  L->pu = panels > 0 ? L->y : L->axc;  // with panels: room for the compact copy
  return c.off;
}

}  // namespace hlp

using namespace hlp;

extern "C" {

const char* hlp_last_error(void) { return g_err.c_str(); }

hlp_err hlp_params_default(hlp_params* p) {
  if (!p) {
    set_error("hlp_params_default: NULL");
    return HLP_EINVAL;
  }
  std::memset(p, 0, sizeof(*p));
  p->tol = 1e-8;
  p->max_iter = 10000000;
  p->time_limit_s = 3600.0;
  p->eval_freq = 64;
  p->precision = HLP_FP64;
  p->gamma = 1.0;
  p->beta_sufficient = 0.2;
  p->beta_necessary = 0.8;
  p->beta_artificial = 0.36;
  p->kp = 0.99;
  p->ki = 0.01;
  p->kd = 0.0;
  p->omega0 = 1.0;
  p->eta_override = 0.0;
  p->ruiz_iters = 10;
  p->pock_chambolle = 1;
  p->power_max_iter = 5000;
  p->restart_to_current = 0;
  p->power_tol = 1e-8;
  p->pid_min_norm = 1e-10;
  p->trace_iters = 0;
  p->debug_poison_iter = 0;
  p->graphs = 1;
  p->stream_matrix = -1;
  p->column_panels = -1;
  p->panel_row_min = 16;
  p->dense_row_min = 2048;
  return HLP_OK;
}

static hlp_err check_sizes(int32_t m, int32_t n, int64_t nnz) {
  if (m < 0 || n < 0 || nnz < 0) {
    set_error("m, n and nnz must be nonnegative");
    return HLP_EINVAL;
  }
  if (nnz >= (int64_t(1) << 31) || m >= INT32_MAX - 1 || n >= INT32_MAX - 1) {
    set_error("nnz >= 2^31 or a dimension near 2^31 is not supported (int32 device indexing)");
    return HLP_EUNSUPPORTED;
  }
  return HLP_OK;
}

hlp_err hlp_workspace_bytes(int32_t m, int32_t n, int64_t nnz, const hlp_params* p, size_t* bytes) {
  if (!bytes) {
    set_error("hlp_workspace_bytes: NULL output");
    return HLP_EINVAL;
  }
  HLP_TRY(check_sizes(m, n, nnz));
  hlp_params d;
  hlp_params_default(&d);
  if (!p) p = &d;
  *bytes = carve(nullptr, nullptr, m, n, nnz, p->precision,
                 worst_caps(m, n, nnz, panel_count(n, p), p->panel_row_min, p->dense_row_min));
  return HLP_OK;
}

static hlp_err check_row_ptr_host(int32_t m, int64_t nnz, const int64_t* rp) {
  if (rp[0] != 0 || rp[m] != nnz) {
    set_error("row_ptr must start at 0 and end at nnz");
    return HLP_EINVAL;
  }
  for (int32_t i = 0; i < m; ++i)
    if (rp[i] > rp[i + 1]) {
      set_error("row_ptr must be nondecreasing");
      return HLP_EINVAL;
    }
  return HLP_OK;
}

hlp_err hlp_workspace_bytes_csr(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const hlp_params* p,
                                size_t* bytes) {
  if (!bytes || !row_ptr) {
    set_error("hlp_workspace_bytes_csr: NULL row_ptr or output");
    return HLP_EINVAL;
  }
  HLP_TRY(check_sizes(m, n, nnz));
  hlp_params d;
  hlp_params_default(&d);
  if (!p) p = &d;
  HLP_TRY(check_row_ptr_host(m, nnz, row_ptr));
  *bytes = carve(nullptr, nullptr, m, n, nnz, p->precision,
                 exact_caps(m, n, nnz, row_ptr, panel_count(n, p), p->panel_row_min, p->dense_row_min,
                            p->column_panels == -1));
  return HLP_OK;
}

static hlp_err read_flags(hlp_lp* lp, int* out) {
  HLP_HIP(hipMemcpyAsync(out, lp->flags, sizeof(int), hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  return HLP_OK;
}

// First row block of each panel (panels start blocks), read back to the host.
static hlp_err panel_starts(hlp_lp* lp, const int32_t* rbx, int32_t nb, int32_t rows_per_panel, int32_t P,
                            std::vector<int32_t>& pstart) {
  pstart.assign((size_t)P + 1, -1);
  HLP_HIP(launch_panel_starts(rbx, nb, rows_per_panel, lp->pscrA, lp->stream));
  HLP_HIP(hipMemcpyAsync(pstart.data(), lp->pscrA, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  pstart[P] = nb;
  for (int32_t q = 0; q < P; ++q)
    if (pstart[q] < 0 || pstart[q + 1] <= pstart[q]) {
      set_error("column panels: inconsistent block table");
      return HLP_EUNSUPPORTED;
    }
  return HLP_OK;
}

// Column-panel layout of the long and dense rows (see hlp_params::column_panels
// and dense_row_min); P is the reserved panel count.  Leaves lp->panels = 0
// when the layout is not used.
static hlp_err build_panels(hlp_lp* lp, int32_t P, int32_t T, int32_t Ld, bool automatic) {
  lp->panels = 0;
  lp->nL = lp->nD = 0;
  if (P <= 0 || lp->m == 0 || lp->n == 0 || lp->nnz == 0) return HLP_OK;
  if (lp->nD_cap == 0) Ld = 0;  // no room reserved for dense rows
  int32_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // More dense rows than reserved: double the threshold until they fit (a
  // threshold above n leaves no dense row, so this ends).
  for (;;) {
    HLP_HIP(launch_panel_split(lp, T, Ld, lp->flags));
    HLP_HIP(hipMemcpyAsync(cnt, lp->flags, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipStreamSynchronize(lp->stream));
    if (cnt[2] <= lp->nD_limit || Ld == 0) break;
    Ld = Ld > lp->n / 2 ? 0 : 2 * Ld;
  }
  lp->dense_min = Ld;
  const int32_t nL = cnt[0], nD = cnt[2];
  const int64_t nnz_split = lp->nnz - cnt[1];
  if (nL + nD < 1 || nL + nD > lp->nL_cap || nD > lp->nD_cap) return HLP_OK;
  if (automatic && 2 * nnz_split < lp->nnz) return HLP_OK;
  // a layout sized for this matrix's rows (hlp_workspace_bytes_csr) must see
  // the rows it was sized for
  if (lp->exact_layout && (nL + nD != lp->nL_cap || nD != lp->nD_cap || cnt[1] != lp->cap_nnz_short)) {
    set_error("column panels: the rows differ from those the workspace layout was sized for");
    return HLP_EUNSUPPORTED;
  }
  lp->panels = P;
  lp->nL = nL;
  lp->nD = nD;
  lp->panel_w = (int32_t)(((int64_t)lp->n + P - 1) / P);
  lp->dense_w = kDenseW;
  lp->dense_wT = kDenseWT;
  HLP_HIP(launch_panel_layout(lp, lp->flags));
  HLP_HIP(hipMemcpyAsync(cnt, lp->flags, 6 * sizeof(int32_t), hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  lp->nbS = cnt[3];
  lp->nbP = nL > 0 ? cnt[4] : 0;
  lp->nbD = nD > 0 ? cnt[5] : 0;
  if (lp->nbD > lp->capD_blocks) {
    set_error("dense panels: more row blocks than reserved");
    return HLP_EUNSUPPORTED;
  }
  HLP_HIP(launch_panel_remap(lp));
  std::vector<int32_t> pstart;
  lp->nbPgrid = 0;
  for (int k = 0; k < 9; ++k) lp->poff[k] = 0;
  if (nL > 0) {
    // blocks of panel q: [pstart[q], pstart[q+1]); dealt to XCD q mod 8 in panel order
    HLP_TRY(panel_starts(lp, lp->rbxP, lp->nbP, nL, P, pstart));
    int32_t off = 0, widest = 0;
    for (int x = 0; x < 8; ++x) {
      lp->poff[x] = off;
      for (int q = x; q < P; q += 8) {
        const int32_t len = pstart[q + 1] - pstart[q];
        HLP_HIP(hipMemcpyAsync(lp->tabP + 4 * (int64_t)off, lp->rbxP + 4 * (int64_t)pstart[q],
                               16 * (size_t)len, hipMemcpyDeviceToDevice, lp->stream));
        off += len;
      }
      widest = std::max(widest, off - lp->poff[x]);
    }
    lp->poff[8] = off;
    if (off != lp->nbP) {
      set_error("column panels: inconsistent block table");
      return HLP_EUNSUPPORTED;
    }
    lp->nbPgrid = 8 * widest;
  }
  lp->nbC = (nL + 255) / 256;
  lp->ntilesD = lp->ntilesT = 0;
  lp->dense_PT = 0;
  lp->nbCD = (nD + 255) / 256;
  if (nD > 0) {
    // tiles: up to kTileBlocks consecutive row blocks of one narrow panel
    HLP_TRY(panel_starts(lp, lp->rbxD, lp->nbD, nD, lp->dense_P, pstart));
    std::vector<int32_t> tiles;
    for (int32_t q = 0; q < lp->dense_P; ++q)
      for (int32_t b = pstart[q]; b < pstart[q + 1]; b += kTileBlocks) {
        tiles.push_back(b);
        tiles.push_back(std::min(pstart[q + 1], b + kTileBlocks));
        tiles.push_back(q);
        tiles.push_back(0);
      }
    lp->ntilesD = (int32_t)(tiles.size() / 4);
    if ((int64_t)lp->ntilesD > lp->capD_blocks) {
      set_error("dense panels: tile table overflow");
      return HLP_EUNSUPPORTED;
    }
    HLP_HIP(hipMemcpyAsync(lp->tilesD, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           lp->stream));
    // the primal side (ATR and ATD, tiles of ATD), when the dense rows hold at
    // least half of the nonzeros (below that, the split costs more than the
    // LDS slices save)
    int32_t nnzD = 0;
    HLP_HIP(hipMemcpyAsync(&nnzD, lp->ppD + (int64_t)lp->dense_P * nD, sizeof(int32_t), hipMemcpyDeviceToHost,
                           lp->stream));
    HLP_HIP(hipStreamSynchronize(lp->stream));
    if (2 * (int64_t)nnzD < lp->nnz) {
      HLP_HIP(hipStreamSynchronize(lp->stream));
      return HLP_OK;
    }
    if (lp->dense_PT_cap == 0 || (lp->exact_layout && nnzD != lp->cap_nnz_dense)) {
      set_error("dense rows: the primal split was not reserved for these rows");
      return HLP_EUNSUPPORTED;
    }
    lp->dense_PT = (nD + lp->dense_wT - 1) / lp->dense_wT;
    HLP_HIP(launch_dense_transpose(lp, lp->flags));
    HLP_HIP(hipMemcpyAsync(cnt, lp->flags, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipStreamSynchronize(lp->stream));
    lp->nbR = cnt[6];
    lp->nbT2 = cnt[7];
    if (lp->nbT2 > lp->capT_blocks) {
      set_error("dense panels: more row blocks than reserved");
      return HLP_EUNSUPPORTED;
    }
    HLP_TRY(panel_starts(lp, lp->rbxT2, lp->nbT2, lp->n, lp->dense_PT, pstart));
    tiles.clear();
    for (int32_t r = 0; r < lp->dense_PT; ++r)
      for (int32_t b = pstart[r]; b < pstart[r + 1]; b += kTileBlocks) {
        tiles.push_back(b);
        tiles.push_back(std::min(pstart[r + 1], b + kTileBlocks));
        tiles.push_back(r);
        tiles.push_back(0);
      }
    lp->ntilesT = (int32_t)(tiles.size() / 4);
    if ((int64_t)lp->ntilesT > lp->capT_blocks) {
      set_error("dense panels: tile table overflow");
      return HLP_EUNSUPPORTED;
    }
    HLP_HIP(hipMemcpyAsync(lp->tilesT, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           lp->stream));
  }
  HLP_HIP(hipStreamSynchronize(lp->stream));
  return HLP_OK;
}

static hlp_err validate_and_scale_vectors(hlp_lp* lp, const double* c, const double* lc,
                                          const double* uc, const double* lv, const double* uv) {
  if ((lp->n && (!c || !lv || !uv)) || (lp->m && (!lc || !uc))) {
    set_error("NULL objective or bound vector");
    return HLP_EINVAL;
  }
  HLP_HIP(launch_fill(reinterpret_cast<double*>(lp->flags), 0.0, 1, lp->stream));
  HLP_HIP(launch_validate_vectors(c, lc, uc, lv, uv, lp->m, lp->n, lp->flags, lp->stream));
  int f = 0;
  HLP_TRY(read_flags(lp, &f));
  if (f) {
    set_error(flag_message(f));
    return HLP_EINVAL;
  }
  HLP_HIP(launch_scale_vectors(lp, c, lc, uc, lv, uv));
  double q[2] = {0.0, 0.0};
  HLP_HIP(hipMemcpyAsync(q, lp->results + SLOT_TMP * NQ, sizeof(q), hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  lp->norm_c = std::sqrt(q[0]);
  lp->norm_b = std::sqrt(q[1]);
  return HLP_OK;
}

}  // extern "C"

namespace hlp {

// Setup of hlp_lp_create into a handle object the caller provides (a fresh
// hlp_lp): argument checks, workspace layout, validation, copy, transpose,
// rescaling, panel layout, scaled vectors and the stepsize.  On error the
// object may hold pointers into the workspace and must be discarded.
// size_to_rows: a workspace below hlp_workspace_bytes may still hold a panel
// layout sized for the matrix's rows (read back from row_ptr on the host).
hlp_err setup_into(hlp_lp* lp, int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                   const double* val, const double* c, const double* lc, const double* uc, const double* lv,
                   const double* uv, const hlp_params* p, void* workspace, size_t workspace_bytes,
                   void* hip_stream, bool size_to_rows) {
  HLP_TRY(check_sizes(m, n, nnz));
  if (!row_ptr || (nnz > 0 && (!col_idx || !val)) || !workspace) {
    set_error("hlp_lp_create: NULL input pointer");
    return HLP_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) {
    set_error("workspace must be 256-byte aligned");
    return HLP_EINVAL;
  }
  hlp_params d;
  hlp_params_default(&d);
  if (!p) p = &d;
  if (p->precision != HLP_FP64 && p->precision != HLP_MIXED) {
    set_error("unknown precision");
    return HLP_EINVAL;
  }
  if (p->ruiz_iters < 0 || p->power_max_iter < 1 || !(p->power_tol >= 0.0) ||
      !(p->eta_override >= 0.0) || !std::isfinite(p->eta_override)) {
    set_error("bad setup parameters (ruiz_iters >= 0, power_max_iter >= 1, power_tol >= 0, finite eta_override >= 0)");
    return HLP_EINVAL;
  }
  if (p->column_panels < -1 || p->panel_row_min < 1 ||
      (p->dense_row_min != 0 && p->dense_row_min <= p->panel_row_min)) {
    set_error("bad setup parameters (column_panels >= -1, panel_row_min >= 1, dense_row_min 0 or > panel_row_min)");
    return HLP_EINVAL;
  }
  const int32_t P = panel_count(n, p);
  Caps caps = worst_caps(m, n, nnz, P, p->panel_row_min, p->dense_row_min);
  size_t need = carve(nullptr, nullptr, m, n, nnz, p->precision, caps);
  bool exact = false;
  if (workspace_bytes < need && size_to_rows && caps.panels > 0) {
    // smaller than the worst case: size the panel layout for this matrix's
    // rows (what hlp_workspace_bytes_csr reports)
    std::vector<int64_t> rp((size_t)m + 1);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    HLP_HIP(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int64_t) * ((size_t)m + 1), hipMemcpyDeviceToHost, st));
    HLP_HIP(hipStreamSynchronize(st));
    HLP_TRY(check_row_ptr_host(m, nnz, rp.data()));
    caps = exact_caps(m, n, nnz, rp.data(), P, p->panel_row_min, p->dense_row_min, p->column_panels == -1);
    need = carve(nullptr, nullptr, m, n, nnz, p->precision, caps);
    exact = true;
  }
  if (workspace_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return HLP_ENOMEM;
  }
  const double t0 = now_s();
  lp->m = m;
  lp->n = n;
  lp->nnz = nnz;
  lp->stream = reinterpret_cast<hipStream_t>(hip_stream);
  lp->precision = p->precision;
  carve(lp, workspace, m, n, nnz, p->precision, caps);
  lp->exact_layout = exact;
  lp->cap_nnz_short = caps.nnz_short;
  lp->cap_nnz_dense = caps.nnz_dense;
  auto fail = [](hlp_err e) { return e; };
  // 1. row pointers, then the rows themselves
  if (hipError_t e = launch_fill(reinterpret_cast<double*>(lp->flags), 0.0, 1, lp->stream); e != hipSuccess)
    return fail(hip_fail(e, "fill"));
  if (hipError_t e = launch_validate_rowptr(row_ptr, m, nnz, lp->flags, lp->stream); e != hipSuccess)
    return fail(hip_fail(e, "validate_rowptr"));
  int f = 0;
  if (hlp_err e = read_flags(lp, &f); e != HLP_OK) return fail(e);
  if (f) {
    set_error(flag_message(f));
    return fail(HLP_EINVAL);
  }
  if (hipError_t e = launch_validate_rows(row_ptr, col_idx, val, m, n, lp->flags, lp->stream); e != hipSuccess)
    return fail(hip_fail(e, "validate_rows"));
  if (hlp_err e = read_flags(lp, &f); e != HLP_OK) return fail(e);
  if (f) {
    set_error(flag_message(f));
    return fail(HLP_EINVAL);
  }
  // 2. copy, transpose
  if (hipError_t e = launch_copy_csr(row_ptr, col_idx, val, m, nnz, lp->rp, lp->col, lp->val0, lp->stream);
      e != hipSuccess)
    return fail(hip_fail(e, "copy_csr"));
  lp->Lr = lanes_for(m ? (double)nnz / m : 1.0);
  lp->Lc = lanes_for(n ? (double)nnz / n : 1.0);
  if (hipError_t e = launch_transpose(lp); e != hipSuccess) return fail(hip_fail(e, "transpose"));
  // row blocks of A~ and A~^T for the hot SpMVs
  if (hipError_t e = launch_build_row_blocks(lp, lp->rp, m, lp->rbA, lp->rbxA, lp->flags + 1); e != hipSuccess)
    return fail(hip_fail(e, "row blocks"));
  if (hipError_t e = launch_build_row_blocks(lp, lp->cp, n, lp->rbT, lp->rbxT, lp->flags + 2); e != hipSuccess)
    return fail(hip_fail(e, "row blocks"));
  {
    int32_t cnt[3] = {0, 0, 0};
    if (hipError_t e = hipMemcpyAsync(cnt, lp->flags, sizeof(cnt), hipMemcpyDeviceToHost, lp->stream); e != hipSuccess)
      return fail(hip_fail(e, "row block count"));
    if (hipError_t e = hipStreamSynchronize(lp->stream); e != hipSuccess) return fail(hip_fail(e, "sync"));
    lp->nbA = m ? cnt[1] : 0;
    lp->nbT = n ? cnt[2] : 0;
  }
  lp->nt = p->stream_matrix > 0 || (p->stream_matrix < 0 && 2.0 * 12.0 * (double)nnz > 128e6);
  // 3. rescaling of A, then the vectors
  if (hipError_t e = launch_rescale(lp, p->ruiz_iters, p->pock_chambolle); e != hipSuccess)
    return fail(hip_fail(e, "rescale"));
  if (hlp_err e = build_panels(lp, lp->panels, p->panel_row_min, p->dense_row_min, p->column_panels == -1);
      e != HLP_OK)
    return fail(e);
  if (hlp_err e = validate_and_scale_vectors(lp, c, lc, uc, lv, uv); e != HLP_OK) return fail(e);
  // 4. stepsize
  if (p->eta_override > 0.0) {
    lp->eta = p->eta_override;
    lp->power_iters = 0;
  } else if (m == 0 || n == 0 || nnz == 0) {
    lp->eta = 1.0;
    lp->power_iters = 0;
  } else {
    PowerState ps{};
    int first = 1;
    while (true) {
      if (hipError_t e = launch_power(lp, 16, first, p->power_max_iter, p->power_tol); e != hipSuccess)
        return fail(hip_fail(e, "power"));
      first = 0;
      if (hipError_t e = hipMemcpyAsync(&ps, lp->pstate, sizeof(ps), hipMemcpyDeviceToHost, lp->stream);
          e != hipSuccess)
        return fail(hip_fail(e, "power readback"));
      if (hipError_t e = hipStreamSynchronize(lp->stream); e != hipSuccess) return fail(hip_fail(e, "sync"));
      if (ps.done) break;
    }
    lp->power_iters = ps.it;
    lp->eta = ps.estimate > 0.0 ? 0.998 / ps.estimate : 1.0;
  }
  if (hipError_t e = hipStreamSynchronize(lp->stream); e != hipSuccess) return fail(hip_fail(e, "sync"));
  lp->setup_s = now_s() - t0;
  return HLP_OK;
}

}  // namespace hlp

extern "C" {

hlp_err hlp_lp_create(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      const double* val, const double* c, const double* lc, const double* uc,
                      const double* lv, const double* uv, const hlp_params* p, void* workspace,
                      size_t workspace_bytes, void* hip_stream, hlp_lp** out) {
  if (!out) {
    set_error("hlp_lp_create: NULL out");
    return HLP_EINVAL;
  }
  *out = nullptr;
  hlp_lp* lp = new (std::nothrow) hlp_lp();
  if (!lp) {
    set_error("out of host memory");
    return HLP_ENOMEM;
  }
  const hlp_err e = setup_into(lp, m, n, nnz, row_ptr, col_idx, val, c, lc, uc, lv, uv, p, workspace,
                               workspace_bytes, hip_stream, true);
  if (e != HLP_OK) {
    delete lp;
    return e;
  }
  *out = lp;
  return HLP_OK;
}

hlp_err hlp_lp_update_vectors(hlp_lp* lp, const double* c, const double* lc, const double* uc,
                              const double* lv, const double* uv) {
  if (!lp) {
    set_error("NULL handle");
    return HLP_EINVAL;
  }
  return validate_and_scale_vectors(lp, c, lc, uc, lv, uv);
}

hlp_err hlp_lp_scaling(const hlp_lp* lp, double* d_r, double* d_c, double* eta, int32_t* power_iters) {
  if (!lp) {
    set_error("NULL handle");
    return HLP_EINVAL;
  }
  if (d_r && lp->m) HLP_HIP(hipMemcpyAsync(d_r, lp->dr, sizeof(double) * lp->m, hipMemcpyDeviceToDevice, lp->stream));
  if (d_c && lp->n) HLP_HIP(hipMemcpyAsync(d_c, lp->dc, sizeof(double) * lp->n, hipMemcpyDeviceToDevice, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  if (eta) *eta = lp->eta;
  if (power_iters) *power_iters = lp->power_iters;
  return HLP_OK;
}

hlp_err hlp_lp_transpose(const hlp_lp* lp, int32_t* col_ptr, int32_t* row_idx, double* val) {
  if (!lp) {
    set_error("NULL handle");
    return HLP_EINVAL;
  }
  if (col_ptr)
    HLP_HIP(hipMemcpyAsync(col_ptr, lp->cp, sizeof(int32_t) * ((size_t)lp->n + 1), hipMemcpyDeviceToDevice, lp->stream));
  if (row_idx && lp->nnz)
    HLP_HIP(hipMemcpyAsync(row_idx, lp->row, sizeof(int32_t) * lp->nnz, hipMemcpyDeviceToDevice, lp->stream));
  if (val && lp->nnz)
    HLP_HIP(hipMemcpyAsync(val, lp->tval, sizeof(double) * lp->nnz, hipMemcpyDeviceToDevice, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  return HLP_OK;
}

hlp_err hlp_lp_panels(const hlp_lp* lp, int32_t* panels, int32_t* long_rows, int32_t* dense_panels,
                      int32_t* dense_rows) {
  if (!lp) {
    set_error("NULL handle");
    return HLP_EINVAL;
  }
  const bool on = lp->panels > 0;
  if (panels) *panels = lp->panels;
  if (long_rows) *long_rows = on ? lp->nL : 0;
  if (dense_panels) *dense_panels = on && lp->nD > 0 ? lp->dense_P : 0;
  if (dense_rows) *dense_rows = on ? lp->nD : 0;
  return HLP_OK;
}

void hlp_lp_destroy(hlp_lp* lp) {
  if (!lp) return;
  for (void*& g : lp->graph_exec)
    if (g) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(g));
  if (lp->capture_stream) (void)hipStreamDestroy(lp->capture_stream);
  delete lp;
}

}  // extern "C"
