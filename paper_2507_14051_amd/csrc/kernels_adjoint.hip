// Reverse mode of one unrolled iteration with the controller frozen (an
// extension of the method, not in the paper).  The forward iteration is
//   v = x - tau (c~ - A~^T y),  xhat = clamp(v, lv~, uv~),  xbar = 2 xhat - x,
//   w = A~ xbar - y / sigma,    yhat = sigma (clamp(w, lc~, uc~) - w),
//   then z' = a((1+gamma) zhat - gamma z) + (1-a) z0, or z' = z0' = zhat at a
//   restart; the output of the last iteration is zhat.
// Given the adjoint of the iteration's output, the reverse step is:
//   prep (rows):  yhat_bar from the next state / anchor adjoints; the row
//                 bound gradients from the clamp code of w; w_bar.
//   cols (A~^T):  xbar_bar = A~^T w_bar; xhat_bar; the column bound gradients
//                 from the clamp code of v; c~_bar -= tau v_bar; u = tau v_bar.
//   rows (A~):    y_bar = (prep part) + A~ u, fused with the prep of the
//                 previous iteration.
// Only the clamp codes of the forward pass are needed (the map is piecewise
// linear).  Ties count as active, the lower bound first.
#include "device.h"
#include "hlp_internal.h"

namespace hlp {

namespace {

inline int nblocks(int64_t threads) { return (int)((threads + kBlock - 1) / kBlock); }

enum { MODE_HALPERN = 0, MODE_RESTART = 1, MODE_LAST = 2 };

struct PrepArgs {
  const double* dr; const double* Gy; const uint8_t* code;
  double* gyn; double* gya; double* glc; double* guc; double* gw; double* py;
  int32_t m; int32_t mode; double a, gamma, sigma;
};

// yhat_bar of one iteration from the adjoint of its output; row side.
__device__ __forceinline__ void prep_row(const PrepArgs& p, int64_t i, double gyn_i) {
  double gyh, part = 0.0;
  if (p.mode == MODE_LAST) {
    gyh = p.Gy ? p.dr[i] * p.Gy[i] : 0.0;
  } else if (p.mode == MODE_RESTART) {
    gyh = gyn_i + p.gya[i];
    p.gya[i] = 0.0;
  } else {
    gyh = p.a * (1.0 + p.gamma) * gyn_i;
    part = -p.a * p.gamma * gyn_i;
    p.gya[i] += (1.0 - p.a) * gyn_i;
  }
  const uint8_t c = p.code[i];
  if (c == 1) p.glc[i] += p.sigma * gyh;
  if (c == 2) p.guc[i] += p.sigma * gyh;
  const double gw = c == 0 ? 0.0 : -p.sigma * gyh;
  p.gw[i] = gw;
  p.py[i] = part - gw / p.sigma;
}

__global__ void k_bwd_prep(PrepArgs p) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < p.m) prep_row(p, i, p.gyn[i]);
}

struct ColArgs {
  const int32_t* cp; const int32_t* row; const double* tval;
  const double* gw; const double* dc; const double* Gx; const uint8_t* code;
  double* gxn; double* gxa; double* gct; double* glv; double* guv; double* u;
  int32_t n; int32_t mode; double a, gamma, tau;
};

template <int L>
__global__ __launch_bounds__(kBlock) void k_bwd_cols(ColArgs p) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t j = t / L;
  const int lane = threadIdx.x & (L - 1);
  double acc = 0.0;
  if (j < p.n) {
    const int s = p.cp[j], e = p.cp[j + 1];
    for (int q = s + lane; q < e; q += L) acc += p.tval[q] * p.gw[p.row[q]];
  }
  acc = group_sum<L>(acc);
  if (j >= p.n || lane != 0) return;
  double gxh, gin = 0.0;
  if (p.mode == MODE_LAST) {
    gxh = p.Gx ? p.dc[j] * p.Gx[j] : 0.0;
  } else if (p.mode == MODE_RESTART) {
    gxh = p.gxn[j] + p.gxa[j];
    p.gxa[j] = 0.0;
  } else {
    const double g = p.gxn[j];
    gxh = p.a * (1.0 + p.gamma) * g;
    gin = -p.a * p.gamma * g;
    p.gxa[j] += (1.0 - p.a) * g;
  }
  gxh = gxh + 2.0 * acc;
  gin -= acc;
  const uint8_t c = p.code[j];
  if (c == 1) p.glv[j] += gxh;
  if (c == 2) p.guv[j] += gxh;
  const double gv = c == 0 ? gxh : 0.0;
  gin += gv;
  p.gct[j] -= p.tau * gv;
  p.u[j] = p.tau * gv;
  p.gxn[j] = gin;
}

struct RowArgs {
  const int32_t* rp; const int32_t* col; const double* val; const double* u;
  PrepArgs prev;
  int32_t do_prev;
};

template <int L>
__global__ __launch_bounds__(kBlock) void k_bwd_rows(RowArgs p) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = t / L;
  const int lane = threadIdx.x & (L - 1);
  const int32_t m = p.prev.m;
  double acc = 0.0;
  if (i < m) {
    const int s = p.rp[i], e = p.rp[i + 1];
    for (int q = s + lane; q < e; q += L) acc += p.val[q] * p.u[p.col[q]];
  }
  acc = group_sum<L>(acc);
  if (i >= m || lane != 0) return;
  const double gyin = p.prev.py[i] + acc;
  p.prev.gyn[i] = gyin;
  if (p.do_prev) prep_row(p.prev, i, gyin);
}

__global__ void k_bwd_out(const double* dr, const double* dc, const double* gct, const double* glv,
                          const double* guv, const double* glc, const double* guc, double* gc, double* olv,
                          double* ouv, double* olc, double* ouc, int32_t n, int32_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    if (gc) gc[i] = dc[i] * gct[i];
    if (olv) olv[i] = glv[i] / dc[i];
    if (ouv) ouv[i] = guv[i] / dc[i];
  }
  if (i < m) {
    if (olc) olc[i] = dr[i] * glc[i];
    if (ouc) ouc[i] = dr[i] * guc[i];
  }
}

__global__ void k_zero_adj(AdjVecs v, int32_t n, int32_t m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    v.gxn[i] = 0.0; v.gxa[i] = 0.0; v.gct[i] = 0.0; v.glv[i] = 0.0; v.guv[i] = 0.0; v.u[i] = 0.0;
  }
  if (i < m) {
    v.gyn[i] = 0.0; v.gya[i] = 0.0; v.glc[i] = 0.0; v.guc[i] = 0.0; v.gw[i] = 0.0; v.py[i] = 0.0;
  }
}

template <int L>
struct ColsL {
  static hipError_t run(const ColArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_bwd_cols<L>), dim3(nb), dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
};
template <int L>
struct RowsL {
  static hipError_t run(const RowArgs& a, int nb, hipStream_t s) {
    hipLaunchKernelGGL((k_bwd_rows<L>), dim3(nb), dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
};

template <template <int> class F, typename... Args>
hipError_t dispatch_L(int L, Args... args) {
  switch (L) {
    case 1: return F<1>::run(args...);
    case 2: return F<2>::run(args...);
    case 4: return F<4>::run(args...);
    case 8: return F<8>::run(args...);
    case 16: return F<16>::run(args...);
    case 32: return F<32>::run(args...);
    default: return F<64>::run(args...);
  }
}

PrepArgs prep_args(hlp_lp* lp, const AdjVecs& v, const AdjIter& it, const uint8_t* my, const double* Gy) {
  return PrepArgs{lp->dr, Gy, my, v.gyn, v.gya, v.glc, v.guc, v.gw, v.py, lp->m, it.mode, it.a, it.gamma,
                  it.sigma};
}

}  // namespace

hipError_t launch_bwd_prep(hlp_lp* lp, const AdjVecs& v, const AdjIter& it, const uint8_t* my, const double* Gy) {
  if (lp->m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_prep, dim3(nblocks(lp->m)), dim3(kBlock), 0, lp->stream, prep_args(lp, v, it, my, Gy));
  return hipGetLastError();
}

hipError_t launch_bwd_cols(hlp_lp* lp, const AdjVecs& v, const AdjIter& it, const uint8_t* mx, const double* Gx) {
  if (lp->n == 0) return hipSuccess;
  ColArgs a{lp->cp, lp->row, lp->tval, v.gw, lp->dc, Gx, mx, v.gxn, v.gxa, v.gct, v.glv, v.guv, v.u,
            lp->n, it.mode, it.a, it.gamma, it.tau};
  return dispatch_L<ColsL>(lp->Lc, a, nblocks((int64_t)lp->n * lp->Lc), lp->stream);
}

hipError_t launch_bwd_rows(hlp_lp* lp, const AdjVecs& v, int32_t do_prev, const AdjIter& prev,
                           const uint8_t* my_prev, const double* Gy) {
  if (lp->m == 0) return hipSuccess;
  RowArgs a{lp->rp, lp->col, lp->val, v.u, prep_args(lp, v, prev, my_prev, Gy), do_prev};
  return dispatch_L<RowsL>(lp->Lr, a, nblocks((int64_t)lp->m * lp->Lr), lp->stream);
}

hipError_t launch_bwd_out(hlp_lp* lp, const AdjVecs& v, double* gc, double* glc, double* guc, double* glv,
                          double* guv) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_out, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, lp->dr, lp->dc, v.gct, v.glv,
                     v.guv, v.glc, v.guc, gc, glv, guv, glc, guc, lp->n, lp->m);
  return hipGetLastError();
}

hipError_t launch_zero_adj(hlp_lp* lp, const AdjVecs& v) {
  int64_t N = lp->m > lp->n ? lp->m : lp->n;
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_adj, dim3(nblocks(N)), dim3(kBlock), 0, lp->stream, v, lp->n, lp->m);
  return hipGetLastError();
}

}  // namespace hlp
