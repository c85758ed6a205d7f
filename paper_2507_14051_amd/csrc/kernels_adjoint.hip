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
  const int32_t* rb; const int32_t* cp; const int32_t* row; const double* tval;
  const double* gw; const double* dc; const double* Gx; const uint8_t* code;
  double* gxn; double* gxa; double* gct; double* glv; double* guv; double* u;
  int32_t mode; double a, gamma, tau;
};

// Transpose side over the row blocks of A~^T: xbar_bar = A~^T w_bar, then the
// column epilogue.
__global__ __launch_bounds__(kBlock) void k_bwd_cols(ColArgs p) {
  __shared__ double lds[kRbLds];
  const int s = p.rb[blockIdx.x], e = p.rb[blockIdx.x + 1];
  const int j = s + threadIdx.x;
  const bool own = j < e;
  int a0 = 0, a1 = 0;
  double gn = 0.0, ga = 0.0;
  uint8_t c = 0;
  if (own) {
    a0 = p.cp[j]; a1 = p.cp[j + 1];
    gn = p.gxn[j]; ga = p.gxa[j]; c = p.code[j];
  }
  const double acc = rb_dot<double>(p.row, p.tval, p.gw, p.cp[s], p.cp[e], a0, a1, own, e - s, lds);
  if (!own) return;
  double gxh, gin = 0.0;
  if (p.mode == MODE_LAST) {
    gxh = p.Gx ? p.dc[j] * p.Gx[j] : 0.0;
  } else if (p.mode == MODE_RESTART) {
    gxh = gn + ga;
    p.gxa[j] = 0.0;
  } else {
    gxh = p.a * (1.0 + p.gamma) * gn;
    gin = -p.a * p.gamma * gn;
    p.gxa[j] = ga + (1.0 - p.a) * gn;
  }
  gxh = gxh + 2.0 * acc;
  gin -= acc;
  if (c == 1) p.glv[j] += gxh;
  if (c == 2) p.guv[j] += gxh;
  const double gv = c == 0 ? gxh : 0.0;
  gin += gv;
  p.gct[j] -= p.tau * gv;
  p.u[j] = p.tau * gv;
  p.gxn[j] = gin;
}

struct RowArgs {
  const int32_t* rb; const int32_t* rp; const int32_t* col; const double* val; const double* u;
  PrepArgs prev;
  int32_t do_prev;
};

// Matrix side over the row blocks of A~: y_bar = (prep part) + A~ u, fused
// with the row preparation of the previous iteration.
__global__ __launch_bounds__(kBlock) void k_bwd_rows(RowArgs p) {
  __shared__ double lds[kRbLds];
  const int s = p.rb[blockIdx.x], e = p.rb[blockIdx.x + 1];
  const int i = s + threadIdx.x;
  const bool own = i < e;
  int a0 = 0, a1 = 0;
  double pyi = 0.0;
  if (own) {
    a0 = p.rp[i]; a1 = p.rp[i + 1];
    pyi = p.prev.py[i];
  }
  const double acc = rb_dot<double>(p.col, p.val, p.u, p.rp[s], p.rp[e], a0, a1, own, e - s, lds);
  if (!own) return;
  const double gyin = pyi + acc;
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
  ColArgs a{lp->rbT, lp->cp, lp->row, lp->tval, v.gw, lp->dc, Gx, mx, v.gxn, v.gxa, v.gct, v.glv, v.guv, v.u,
            it.mode, it.a, it.gamma, it.tau};
  if (lp->nbT == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_cols, dim3(lp->nbT), dim3(kBlock), 0, lp->stream, a);
  return hipGetLastError();
}

hipError_t launch_bwd_rows(hlp_lp* lp, const AdjVecs& v, int32_t do_prev, const AdjIter& prev,
                           const uint8_t* my_prev, const double* Gy) {
  if (lp->m == 0) return hipSuccess;
  RowArgs a{lp->rbA, lp->rp, lp->col, lp->val, v.u, prep_args(lp, v, prev, my_prev, Gy), do_prev};
  if (lp->nbA == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_rows, dim3(lp->nbA), dim3(kBlock), 0, lp->stream, a);
  return hipGetLastError();
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
