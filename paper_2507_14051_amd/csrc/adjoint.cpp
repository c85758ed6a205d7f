// Unrolled iterations with a tape, and their reverse mode (an extension of the
// method: the derivative of the frozen K-step map, not part of the paper).
//
// Tape (caller's device buffer):
//   header | omega[K] (FP64) | k[K] (int32) | restart[K] (uint8)
//   | checkpoints: nseg x (x[n], y[m], x0[n], y0[m]) FP64, one every ckpt_every iterations
//   | clamp codes of one segment: ckpt_every x (n + m) uint8 (recomputed per segment)
//   | reverse-mode vectors: 6 x n + 6 x m FP64
// The forward pass records the controller (omega, the Halpern index k, the
// restart iterations) and the checkpoints; the backward pass recomputes each
// segment from its checkpoint to get the clamp codes, then runs the reverse
// iterations from the last to the first.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "hlp_internal.h"

namespace hlp {

namespace {

constexpr uint64_t kMagic = 0x68'6c'70'74'61'70'65'31ull;  // "hlptape1"
constexpr double kInf = std::numeric_limits<double>::infinity();

struct TapeHeader {
  uint64_t magic;
  int32_t K, ckpt, nseg, n, m, pad;
  double eta, gamma;
};

inline size_t up(size_t v) { return (v + 255) / 256 * 256; }

struct TapeLayout {
  size_t header, omega, kidx, rst, ckpts, masks, adj, total;
  int32_t nseg;
};

TapeLayout layout(int32_t K, int32_t ckpt, int32_t n, int32_t m) {
  TapeLayout L{};
  L.nseg = (K + ckpt - 1) / ckpt;
  size_t off = 0;
  L.header = off; off += up(sizeof(TapeHeader));
  L.omega = off; off += up(sizeof(double) * (size_t)K);
  L.kidx = off; off += up(sizeof(int32_t) * (size_t)K);
  L.rst = off; off += up((size_t)K);
  L.ckpts = off; off += up(sizeof(double) * (size_t)L.nseg * (2 * (size_t)n + 2 * (size_t)m));
  L.masks = off; off += up((size_t)ckpt * ((size_t)n + (size_t)m));
  L.adj = off; off += up(sizeof(double) * (6 * (size_t)n + 6 * (size_t)m));
  L.total = off;
  return L;
}

AdjVecs adj_vecs(char* base, const TapeLayout& L, int32_t n, int32_t m) {
  double* p = reinterpret_cast<double*>(base + L.adj);
  AdjVecs v;
  v.gxn = p; p += n; v.gxa = p; p += n; v.gct = p; p += n; v.glv = p; p += n; v.guv = p; p += n; v.u = p; p += n;
  v.gyn = p; p += m; v.gya = p; p += m; v.glc = p; p += m; v.guc = p; p += m; v.gw = p; p += m; v.py = p;
  return v;
}

hlp_err state_copy(hlp_lp* lp, double* dst, bool save) {
  const size_t n = lp->n, m = lp->m;
  double* segs[4] = {lp->x, lp->y, lp->xa, lp->ya};
  const size_t len[4] = {n, m, n, m};
  size_t off = 0;
  for (int k = 0; k < 4; ++k) {
    if (len[k]) {
      if (save)
        HLP_HIP(hipMemcpyAsync(dst + off, segs[k], sizeof(double) * len[k], hipMemcpyDeviceToDevice, lp->stream));
      else
        HLP_HIP(hipMemcpyAsync(segs[k], dst + off, sizeof(double) * len[k], hipMemcpyDeviceToDevice, lp->stream));
    }
    off += len[k];
  }
  return HLP_OK;
}

// Sets the device step scalars only when a new epoch or primal weight begins:
// within an epoch the Halpern index grows by one per iteration, so each launch
// just carries its offset j from the epoch's first iteration.
struct StepTracker {
  double eta;
  int64_t base_t = -1, base_k = 0;
  double base_om = 0.0;
  hlp_err at(hlp_lp* lp, int64_t t, double om, int64_t k, double gamma) {
    if (base_t < 0 || om != base_om || k - base_k != t - base_t) {
      HLP_HIP(launch_set_step(lp, eta / om, eta * om, gamma, k));
      base_t = t;
      base_k = k;
      base_om = om;
    }
    return HLP_OK;
  }
  int32_t j(int64_t t) const { return (int32_t)(t - base_t); }
};

double fixed_point_residual(const double* R, double eta, double omega) {
  double q = (omega / eta) * R[Q_DX2] + 2.0 * R[Q_DYADX] + R[Q_DY2] / (eta * omega);
  return std::sqrt(std::max(q, 0.0));
}

// The reverse mode recomputes each segment with the unsplit dual half-step;
// the forward pass uses the same kernels, so the column-panel layout is
// switched off while either runs (its summation order differs).
struct PanelsOff {
  hlp_lp* lp;
  int32_t saved;
  explicit PanelsOff(hlp_lp* l) : lp(l), saved(l->panels) { l->panels = 0; }
  ~PanelsOff() { lp->panels = saved; }
};

}  // namespace

}  // namespace hlp

using namespace hlp;

extern "C" {

hlp_err hlp_tape_bytes(const hlp_lp* lp, int32_t K, int32_t ckpt_every, size_t* bytes) {
  if (!lp || !bytes || K < 1 || ckpt_every < 1) {
    set_error("hlp_tape_bytes: NULL handle/output, K < 1 or ckpt_every < 1");
    return HLP_EINVAL;
  }
  *bytes = layout(K, ckpt_every, lp->n, lp->m).total;
  return HLP_OK;
}

hlp_err hlp_unrolled_forward(hlp_lp* lp, const hlp_params* pp, int32_t K, int32_t ckpt, int32_t replay,
                             const double* x0, const double* y0, double* x, double* y, void* tape,
                             size_t tape_bytes) {
  if (!lp || !tape || K < 1 || ckpt < 1) {
    set_error("hlp_unrolled_forward: NULL handle/tape, K < 1 or ckpt_every < 1");
    return HLP_EINVAL;
  }
  hlp_params p;
  hlp_params_default(&p);
  if (pp) p = *pp;
  if (p.precision != HLP_FP64 || lp->precision != HLP_FP64 || p.restart_to_current) {
    set_error("hlp_unrolled_forward: FP64 handles and restart_to_current = 0 only");
    return HLP_EUNSUPPORTED;
  }
  if (p.eval_freq < 1 || !(p.omega0 > 0.0) || !(p.gamma >= 0.0 && p.gamma <= 1.0)) {
    set_error("hlp_unrolled_forward: bad parameters");
    return HLP_EINVAL;
  }
  const TapeLayout L = layout(K, ckpt, lp->n, lp->m);
  if (tape_bytes < L.total) {
    set_error("tape too small: need " + std::to_string(L.total) + " bytes");
    return HLP_ENOMEM;
  }
  char* base = static_cast<char*>(tape);
  const int32_t n = lp->n, m = lp->m;
  std::vector<double> omega(K);
  std::vector<int32_t> kidx(K);
  std::vector<uint8_t> rst(K, 0);
  TapeHeader h{};
  if (replay) {
    HLP_HIP(hipMemcpyAsync(&h, base + L.header, sizeof(h), hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipMemcpyAsync(omega.data(), base + L.omega, sizeof(double) * K, hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipMemcpyAsync(kidx.data(), base + L.kidx, sizeof(int32_t) * K, hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipMemcpyAsync(rst.data(), base + L.rst, (size_t)K, hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipStreamSynchronize(lp->stream));
    if (h.magic != kMagic || h.K != K || h.ckpt != ckpt || h.n != n || h.m != m) {
      set_error("hlp_unrolled_forward: the tape was not recorded for this K / ckpt_every / problem");
      return HLP_EINVAL;
    }
  }
  const double eta = lp->eta;
  StepTracker steps{eta};
  PanelsOff unsplit(lp);
  HLP_HIP(launch_warm_start(lp, x0, y0));
  double om = p.omega0;
  int64_t k = 0;
  double r0 = kInf, r_prev = kInf;
  bool r0_pending = false;
  double pid_sum = 0.0, e_prev = 0.0;
  bool has_prev = false;
  double R[NSLOT * NQ];
  const size_t cstride = 2 * (size_t)n + 2 * (size_t)m;
  double* ck = reinterpret_cast<double*>(base + L.ckpts);
  for (int32_t t = 0; t < K; ++t) {
    if (t % ckpt == 0) HLP_TRY(state_copy(lp, ck + (size_t)(t / ckpt) * cstride, true));
    if (replay) {
      om = omega[t];
      k = kidx[t];
    } else {
      omega[t] = om;
      kidx[t] = (int32_t)k;
    }
    const bool check = !replay && ((t + 1) % p.eval_freq == 0);
    const bool need_r = !replay && (k == 0 || check);
    const bool last = t == K - 1;
    const bool res = need_r || last || (replay && rst[t]);
    HLP_TRY(steps.at(lp, t, om, k, p.gamma));
    StepArgs s;
    s.j = steps.j(t);
    s.residual = res ? 1 : 0;
    HLP_HIP(launch_primal(lp, s));
    HLP_HIP(launch_dual(lp, s));
    if (need_r) {
      HLP_HIP(launch_finalize(lp, 1 | 2, check ? SLOT_CHECK : SLOT_R0));
      if (!check) r0_pending = true;
    }
    const bool epoch_start = k == 0;
    ++k;
    bool restart = replay ? rst[t] != 0 : false;
    if (check) {
      HLP_HIP(hipMemcpyAsync(R, lp->results, sizeof(R), hipMemcpyDeviceToHost, lp->stream));
      HLP_HIP(hipStreamSynchronize(lp->stream));
      const double* RC = R + SLOT_CHECK * NQ;
      const double r = fixed_point_residual(RC, eta, om);
      if (epoch_start) r0 = r;
      else if (r0_pending) r0 = fixed_point_residual(R + SLOT_R0 * NQ, eta, om);
      r0_pending = false;
      restart = (r <= p.beta_sufficient * r0) || (r <= p.beta_necessary * r0 && r > r_prev) ||
                ((double)k >= p.beta_artificial * (double)(t + 1));
      if (restart) {
        const double dxn = std::sqrt(RC[Q_XA2]), dyn = std::sqrt(RC[Q_YA2]);
        if (dxn > p.pid_min_norm && dyn > p.pid_min_norm) {
          const double e = std::log(om * dxn / dyn);
          pid_sum += e;
          const double de = has_prev ? e - e_prev : 0.0;
          e_prev = e;
          has_prev = true;
          om = std::exp(std::log(om) - (p.kp * e + p.ki * pid_sum + p.kd * de));
        }
        r_prev = kInf;
      } else {
        r_prev = r;
      }
      rst[t] = restart ? 1 : 0;
    }
    if (restart && !last) {
      HLP_HIP(launch_restart_copy(lp, 0));
      k = 0;
    }
  }
  HLP_HIP(launch_unscale(lp, x, y));
  if (!replay) {
    h.magic = kMagic;
    h.K = K;
    h.ckpt = ckpt;
    h.nseg = L.nseg;
    h.n = n;
    h.m = m;
    h.eta = eta;
    h.gamma = p.gamma;
    HLP_HIP(hipMemcpyAsync(base + L.header, &h, sizeof(h), hipMemcpyHostToDevice, lp->stream));
    HLP_HIP(hipMemcpyAsync(base + L.omega, omega.data(), sizeof(double) * K, hipMemcpyHostToDevice, lp->stream));
    HLP_HIP(hipMemcpyAsync(base + L.kidx, kidx.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, lp->stream));
    HLP_HIP(hipMemcpyAsync(base + L.rst, rst.data(), (size_t)K, hipMemcpyHostToDevice, lp->stream));
  }
  HLP_HIP(hipStreamSynchronize(lp->stream));
  return HLP_OK;
}

hlp_err hlp_unrolled_backward(hlp_lp* lp, const void* tape, size_t tape_bytes, const double* gx,
                              const double* gy, double* gc, double* glc, double* guc, double* glv,
                              double* guv) {
  if (!lp || !tape) {
    set_error("hlp_unrolled_backward: NULL handle or tape");
    return HLP_EINVAL;
  }
  char* base = const_cast<char*>(static_cast<const char*>(tape));
  TapeHeader h{};
  if (tape_bytes < sizeof(h)) {
    set_error("tape too small");
    return HLP_ENOMEM;
  }
  HLP_HIP(hipMemcpyAsync(&h, base, sizeof(h), hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  if (h.magic != kMagic || h.n != lp->n || h.m != lp->m || h.K < 1 || h.ckpt < 1) {
    set_error("hlp_unrolled_backward: the tape holds no forward pass of this problem");
    return HLP_EINVAL;
  }
  const int32_t K = h.K, ckpt = h.ckpt, n = lp->n, m = lp->m;
  const TapeLayout L = layout(K, ckpt, n, m);
  if (tape_bytes < L.total) {
    set_error("tape too small: need " + std::to_string(L.total) + " bytes");
    return HLP_ENOMEM;
  }
  std::vector<double> omega(K);
  std::vector<int32_t> kidx(K);
  std::vector<uint8_t> rst(K);
  HLP_HIP(hipMemcpyAsync(omega.data(), base + L.omega, sizeof(double) * K, hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipMemcpyAsync(kidx.data(), base + L.kidx, sizeof(int32_t) * K, hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipMemcpyAsync(rst.data(), base + L.rst, (size_t)K, hipMemcpyDeviceToHost, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  const double eta = h.eta, gamma = h.gamma;
  StepTracker steps{eta};
  PanelsOff unsplit(lp);
  const AdjVecs v = adj_vecs(base, L, n, m);
  HLP_HIP(launch_zero_adj(lp, v));
  uint8_t* masks = reinterpret_cast<uint8_t*>(base + L.masks);
  const size_t mstride = (size_t)n + (size_t)m;
  const size_t cstride = 2 * (size_t)n + 2 * (size_t)m;
  double* ck = reinterpret_cast<double*>(base + L.ckpts);
  auto iter = [&](int32_t t) {
    const double om = omega[t];
    const int32_t mode = t == K - 1 ? 2 : (rst[t] ? 1 : 0);
    return AdjIter{eta / om, eta * om, (double)(kidx[t] + 1) / (double)(kidx[t] + 2), gamma, mode};
  };
  for (int32_t seg = L.nseg - 1; seg >= 0; --seg) {
    const int32_t t0 = seg * ckpt, t1 = std::min(K, t0 + ckpt);
    // recompute the segment's clamp codes from its checkpoint
    steps.base_t = -1;
    HLP_TRY(state_copy(lp, ck + (size_t)seg * cstride, false));
    for (int32_t t = t0; t < t1; ++t) {
      const double om = omega[t];
      HLP_TRY(steps.at(lp, t, om, kidx[t], gamma));
      StepArgs s;
      s.j = steps.j(t);
      s.mask_x = masks + (size_t)(t - t0) * mstride;
      s.mask_y = s.mask_x + n;
      HLP_HIP(launch_primal(lp, s));
      HLP_HIP(launch_dual(lp, s));
      if (rst[t] && t != K - 1) HLP_HIP(launch_restart_copy(lp, 0));
    }
    // reverse iterations
    for (int32_t t = t1 - 1; t >= t0; --t) {
      const uint8_t* mx = masks + (size_t)(t - t0) * mstride;
      const uint8_t* my = mx + n;
      const AdjIter it = iter(t);
      if (t == t1 - 1) HLP_HIP(launch_bwd_prep(lp, v, it, my, gy));
      HLP_HIP(launch_bwd_cols(lp, v, it, mx, gx));
      const bool has_prev = t - 1 >= t0;
      const AdjIter prev = has_prev ? iter(t - 1) : it;
      HLP_HIP(launch_bwd_rows(lp, v, has_prev ? 1 : 0, prev, has_prev ? my - mstride : my, gy));
    }
  }
  HLP_HIP(launch_bwd_out(lp, v, gc, glc, guc, glv, guv));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  return HLP_OK;
}

}  // extern "C"
