// Host controller: the iteration loop of restarted reflected Halpern PDHG
// (paper Secs. 2.2 and 3) with the relative KKT termination test (Sec. 4), in
// FP64 or in FP32 with iterative refinement.  All vector work runs in the HIP
// kernels; the host only keeps the scalar state (omega, PID memory, k, T,
// r0, r_prev) and reads ~13 reduced FP64 scalars once per check.
//
// The iterations between two checks form a "run": the step scalars are set
// once on the device, then the run's launches (two half-steps per iteration,
// residual variants at the first iteration of an epoch and at the check, the
// check's KKT kernel and the finalize kernels) are issued either directly or
// by replaying a HIP graph captured once per handle and run shape.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <vector>

#include "hlp_internal.h"

namespace hlp {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

constexpr double kInf = std::numeric_limits<double>::infinity();

// Controller state (Sec. 3): inner index k, total T, restart memory, PID memory.
struct Ctl {
  double omega = 1.0;
  int64_t k = 0, t = 0, restarts = 0, checks = 0;
  double r0 = kInf, r_prev = kInf;
  double pid_sum = 0.0, e_prev = 0.0;
  bool has_prev = false;
};

// r(z) = ||z - PDHG(z)||_P with P = [[omega/eta I, A^T], [A, 1/(eta omega) I]]
double fixed_point_residual(const double* R, double eta, double omega) {
  double q = (omega / eta) * R[Q_DX2] + 2.0 * R[Q_DYADX] + R[Q_DY2] / (eta * omega);
  return std::sqrt(std::max(q, 0.0));
}

// Sec. 3, adaptive restart: sufficient decay, necessary decay + no local
// progress, artificial restart (k and T after the increment).
bool restart_test(double r, double r0, double r_prev, int64_t k, int64_t t, const hlp_params& p) {
  return (r <= p.beta_sufficient * r0) || (r <= p.beta_necessary * r0 && r > r_prev) ||
         ((double)k >= p.beta_artificial * (double)t);
}

// Sec. 3, primal weight update: PID control of log omega with the error
// e = log(omega ||dx|| / ||dy||).
double pid_update(double omega, double dxn, double dyn, Ctl& c, const hlp_params& p) {
  if (!(dxn > p.pid_min_norm && dyn > p.pid_min_norm)) return omega;
  const double e = std::log(omega * dxn / dyn);
  c.pid_sum += e;
  const double de = c.has_prev ? e - c.e_prev : 0.0;
  c.e_prev = e;
  c.has_prev = true;
  return std::exp(std::log(omega) - (p.kp * e + p.ki * c.pid_sum + p.kd * de));
}

// Power of two for the refinement scale: 2^floor(log2(1/delta)) within [1, min(2^12 prev, 2^40)].
double pow2_scale(double delta, double prev) {
  const double cap = std::min(prev * 4096.0, std::ldexp(1.0, 40));
  if (!(delta > 0.0) || !std::isfinite(delta)) return cap;
  const double s = std::ldexp(1.0, (int)std::floor(std::log2(1.0 / delta)));
  return std::min(std::max(s, 1.0), cap);
}

struct Kkt {
  double pobj, dobj, rel_gap, rel_p, rel_d, rel;
  bool finite;
};

Kkt kkt_from(const double* R, const hlp_lp* lp) {
  Kkt k{};
  k.pobj = R[Q_POBJ];
  k.dobj = R[Q_DOBJ_R] + R[Q_DOBJ_C];
  const double rho_p = std::sqrt(std::max(R[Q_RP2], 0.0));
  const double rho_d = std::sqrt(std::max(R[Q_RD2], 0.0));
  k.rel_gap = std::fabs(k.pobj - k.dobj) / (1.0 + std::fabs(k.pobj) + std::fabs(k.dobj));
  k.rel_p = rho_p / (1.0 + lp->norm_b);
  k.rel_d = rho_d / (1.0 + lp->norm_c);
  k.rel = std::max(k.rel_gap, std::max(k.rel_p, k.rel_d));
  k.finite = std::isfinite(k.pobj) && std::isfinite(k.dobj) && std::isfinite(rho_p) && std::isfinite(rho_d);
  return k;
}

hlp_err check_params(const hlp_params* p) {
  if (!p) return HLP_OK;
  if (p->max_iter < 1 || p->eval_freq < 1 || !(p->tol >= 0.0) || !(p->gamma >= 0.0 && p->gamma <= 1.0) ||
      !(p->omega0 > 0.0) || !std::isfinite(p->omega0) || p->trace_iters < 0 || !(p->time_limit_s >= 0.0)) {
    set_error("bad parameters: need max_iter >= 1, eval_freq >= 1, tol >= 0, gamma in [0,1], omega0 > 0, "
              "trace_iters >= 0, time_limit_s >= 0");
    return HLP_EINVAL;
  }
  return HLP_OK;
}

#define HLP_K(call)                                   \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

// One run of `len` iterations ending at a check.  first_res: the first
// iteration starts an epoch (its residual goes to the R0 slot unless it is
// also the check).  trace_at(j) / poison_at(j): per-iteration extras (direct
// launches only).
struct RunShape {
  int32_t len;
  bool first_res;
  bool mixed;
};

hlp_err issue_run(hlp_lp* lp, const RunShape& rs, double* trace_base, int64_t trace_first, int64_t trace_n,
                  int64_t trace_stride, int32_t poison_j) {
  for (int32_t j = 0; j < rs.len; ++j) {
    const bool first = j == 0 && rs.first_res;
    const bool last = j == rs.len - 1;
    const int64_t tj = trace_first + j;
    const bool traced = trace_base && tj >= 0 && tj < trace_n;
    StepArgs s;
    s.j = j;
    s.residual = (first || last || traced) ? 1 : 0;
    if (rs.mixed) {
      HLP_K(launch_primal32(lp, s));
      HLP_K(launch_dual32(lp, s));
    } else {
      HLP_K(launch_primal(lp, s));
      HLP_K(launch_dual(lp, s));
    }
    const int f32 = rs.mixed ? 16 : 0;
    if (first && !last) HLP_K(launch_finalize(lp, 1 | 2 | f32, SLOT_R0));
    if (last) HLP_K(launch_finalize(lp, 1 | 2 | f32, SLOT_CHECK));
    if (traced) {
      if (rs.mixed) HLP_K(launch_trace32(lp, trace_base + tj * trace_stride));
      else HLP_K(launch_trace(lp, trace_base + tj * trace_stride));
    }
    if (poison_j == j) HLP_K(launch_poison(lp));
  }
  if (rs.mixed) {
    HLP_K(launch_combine(lp));
    HLP_K(launch_kkt_rows(lp));
    HLP_K(launch_kkt_cols(lp, lp->rbuf));
    HLP_K(launch_finalize(lp, 4 | 8, SLOT_CHECK));
  } else {
    HLP_K(launch_kkt_cols(lp, lp->rbuf));
    HLP_K(launch_finalize(lp, 4, SLOT_CHECK));
  }
  return HLP_OK;
}

// Capture a run of eval_freq iterations into a graph (once per handle and shape).
hlp_err graph_for(hlp_lp* lp, const RunShape& rs, hipGraphExec_t* out) {
  const int idx = (rs.mixed ? 2 : 0) + (rs.first_res ? 1 : 0);
  if (lp->graph_len != rs.len) {
    for (void*& g : lp->graph_exec)
      if (g) {
        HLP_HIP(hipGraphExecDestroy(static_cast<hipGraphExec_t>(g)));
        g = nullptr;
      }
    lp->graph_len = rs.len;
  }
  if (!lp->graph_exec[idx]) {
    if (!lp->capture_stream) HLP_HIP(hipStreamCreateWithFlags(&lp->capture_stream, hipStreamNonBlocking));
    hipStream_t user = lp->stream;
    lp->stream = lp->capture_stream;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(lp->capture_stream, hipStreamCaptureModeThreadLocal);
    hlp_err r = HLP_OK;
    if (e == hipSuccess) r = issue_run(lp, rs, nullptr, 0, 0, 0, -1);
    hipError_t e2 = hipStreamEndCapture(lp->capture_stream, &g);
    lp->stream = user;
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    if (r != HLP_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    lp->graph_exec[idx] = ex;
  }
  *out = static_cast<hipGraphExec_t>(lp->graph_exec[idx]);
  return HLP_OK;
}

// ------------------------------------------------------------------ the loop (both precisions)
hlp_err run_loop(hlp_lp* lp, const hlp_params& p, const double* x0, const double* y0, double* trace, Ctl& c,
                 Kkt& kk, int32_t& status) {
  const bool mixed = p.precision == HLP_MIXED;
  const double eta = lp->eta;
  const int64_t tstride = 2 * (int64_t)lp->n + 2 * (int64_t)lp->m;
  HLP_K(launch_warm_start(lp, x0, y0));
  double P = 1.0, D = 1.0;
  if (mixed) {
    // the first centre is the start point, with P = D = 1
    if (lp->n) HLP_HIP(hipMemcpyAsync(lp->xh, lp->x, sizeof(double) * lp->n, hipMemcpyDeviceToDevice, lp->stream));
    if (lp->m) HLP_HIP(hipMemcpyAsync(lp->yh, lp->y, sizeof(double) * lp->m, hipMemcpyDeviceToDevice, lp->stream));
    HLP_K(launch_kkt_rows(lp));
    HLP_K(launch_kkt_cols(lp, nullptr));
    HLP_K(launch_recentre(lp, P, D));
  }
  c.omega = p.omega0;  // in the FP32 path, omega in original units; the step uses omega D / P
  double R[NSLOT * NQ];
  const double t_start = now_s();
  while (true) {
    const int64_t next = std::min<int64_t>((c.t / p.eval_freq + 1) * p.eval_freq, p.max_iter);
    RunShape rs{(int32_t)(next - c.t), c.k == 0, mixed};
    const double om = mixed ? c.omega * D / P : c.omega;
    HLP_K(launch_set_step(lp, eta / om, eta * om, p.gamma, c.k, P, D));
    const int32_t poison_j =
        (p.debug_poison_iter > c.t && p.debug_poison_iter <= next) ? (int32_t)(p.debug_poison_iter - c.t - 1) : -1;
    const bool traced = trace && c.t < p.trace_iters;
    if (p.graphs && rs.len == p.eval_freq && rs.len > 1 && !traced && poison_j < 0) {
      hipGraphExec_t ex = nullptr;
      HLP_TRY(graph_for(lp, rs, &ex));
      HLP_HIP(hipGraphLaunch(ex, lp->stream));
    } else {
      HLP_TRY(issue_run(lp, rs, trace, c.t, trace ? p.trace_iters : 0, tstride, poison_j));
    }
    HLP_HIP(hipMemcpyAsync(R, lp->results, sizeof(R), hipMemcpyDeviceToHost, lp->stream));
    HLP_HIP(hipStreamSynchronize(lp->stream));
    c.t = next;
    c.k += rs.len;
    ++c.checks;
    const double* RC = R + SLOT_CHECK * NQ;
    const double r = fixed_point_residual(RC, eta, om);
    if (rs.first_res) c.r0 = rs.len == 1 ? r : fixed_point_residual(R + SLOT_R0 * NQ, eta, om);
    kk = kkt_from(RC, lp);
    hlp_check rec{};
    rec.iter = c.t;
    rec.k = c.k;
    rec.r = r;
    rec.r0 = c.r0;
    rec.rel_kkt = kk.rel;
    rec.rel_gap = kk.rel_gap;
    rec.rel_primal = kk.rel_p;
    rec.rel_dual = kk.rel_d;
    rec.omega = c.omega;
    rec.seconds = now_s() - t_start;
    if (lp->keep_log) lp->check_log.push_back(rec);
    status = -1;
    if (!kk.finite || !std::isfinite(r)) status = HLP_NUMERICAL;
    else if (kk.rel <= p.tol) status = HLP_OPTIMAL;
    else if (c.t >= p.max_iter) status = HLP_ITER_LIMIT;
    else if (now_s() - t_start >= p.time_limit_s) status = HLP_TIME_LIMIT;
    if (status >= 0) return HLP_OK;
    if (restart_test(r, c.r0, c.r_prev, c.k, c.t, p)) {
      if (lp->keep_log) lp->check_log.back().restart = 1;
      ++c.restarts;
      const double om_new = pid_update(om, std::sqrt(RC[Q_XA2]), std::sqrt(RC[Q_YA2]), c, p);
      if (mixed) {
        c.omega = om_new * P / D;
        // refinement: re-centre at zhat and rescale from the FP64 violations there
        P = pow2_scale(std::max(RC[Q_VP], RC[Q_VX]), P);
        D = pow2_scale(RC[Q_VD], D);
        HLP_K(launch_recentre(lp, P, D));
      } else {
        c.omega = om_new;
        HLP_K(launch_restart_copy(lp, p.restart_to_current));
      }
      c.k = 0;
      c.r_prev = kInf;
    } else {
      c.r_prev = r;
    }
  }
}

}  // namespace

}  // namespace hlp

using namespace hlp;

extern "C" {

hlp_err hlp_solve(hlp_lp* lp, const hlp_params* pp, const double* x0, const double* y0, double* x,
                  double* y, double* r, hlp_info* info, double* trace) {
  if (!lp) {
    set_error("hlp_solve: NULL handle");
    return HLP_EINVAL;
  }
  hlp_params p;
  hlp_params_default(&p);
  if (pp) p = *pp;
  HLP_TRY(check_params(&p));
  if (p.precision != lp->precision) {
    set_error("hlp_solve: precision differs from the one the handle was created with");
    return HLP_EUNSUPPORTED;
  }
  if (p.precision == HLP_MIXED && p.restart_to_current) {
    set_error("hlp_solve: the FP32 path re-centres at zhat; restart_to_current must be 0");
    return HLP_EUNSUPPORTED;
  }
  const double t0 = now_s();
  lp->check_log.clear();
  Ctl c;
  Kkt kk{};
  int32_t status = -1;
  HLP_TRY(run_loop(lp, p, x0, y0, trace, c, kk, status));
  HLP_HIP(launch_unscale(lp, x, y));
  if (r && lp->n)
    HLP_HIP(hipMemcpyAsync(r, lp->rbuf, sizeof(double) * lp->n, hipMemcpyDeviceToDevice, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  if (info) {
    info->status = status;
    info->power_iters = lp->power_iters;
    info->iters = c.t;
    info->restarts = c.restarts;
    info->checks = c.checks;
    info->rel_kkt = kk.rel;
    info->rel_gap = kk.rel_gap;
    info->rel_primal = kk.rel_p;
    info->rel_dual = kk.rel_d;
    info->pobj = kk.pobj;
    info->dobj = kk.dobj;
    info->omega = c.omega;
    info->eta = lp->eta;
    info->setup_s = lp->setup_s;
    info->solve_s = now_s() - t0;
  }
  return HLP_OK;
}

hlp_err hlp_check_log(const hlp_lp* lp, hlp_check* out, int64_t cap, int64_t* count) {
  if (!lp || !count || cap < 0 || (!out && cap > 0)) {
    set_error("hlp_check_log: NULL handle or count, cap < 0, or NULL out with cap > 0");
    return HLP_EINVAL;
  }
  const int64_t total = (int64_t)lp->check_log.size();
  *count = total;
  const int64_t k = std::min(cap, total);
  for (int64_t i = 0; i < k; ++i) out[i] = lp->check_log[(size_t)i];
  return HLP_OK;
}

hlp_err hlp_profile_iterations(hlp_lp* lp, const hlp_params* pp, int32_t iters, double* ms_out) {
  if (!lp || !ms_out || iters < 1) {
    set_error("hlp_profile_iterations: NULL handle/output or iters < 1");
    return HLP_EINVAL;
  }
  hlp_params p;
  hlp_params_default(&p);
  if (pp) p = *pp;
  const bool mixed = p.precision == HLP_MIXED;
  if (mixed && lp->precision != HLP_MIXED) {
    set_error("hlp_profile_iterations: the handle holds no FP32 mirror");
    return HLP_EUNSUPPORTED;
  }
  HLP_HIP(launch_warm_start(lp, nullptr, nullptr));
  if (mixed) {
    if (lp->n) HLP_HIP(hipMemcpyAsync(lp->xh, lp->x, sizeof(double) * lp->n, hipMemcpyDeviceToDevice, lp->stream));
    if (lp->m) HLP_HIP(hipMemcpyAsync(lp->yh, lp->y, sizeof(double) * lp->m, hipMemcpyDeviceToDevice, lp->stream));
    HLP_HIP(launch_kkt_rows(lp));
    HLP_HIP(launch_kkt_cols(lp, nullptr));
    HLP_HIP(launch_recentre(lp, 1.0, 1.0));
  }
  const double eta = lp->eta, om = p.omega0;
  HLP_HIP(launch_set_step(lp, eta / om, eta * om, p.gamma, 0, 1.0, 1.0));
  // Each half-step is launched with start/stop events that take the kernel's
  // own begin and end timestamps; two plain events bracket the whole run.
  std::vector<hipEvent_t> ev(4 * (size_t)iters + 2);
  for (auto& e : ev) HLP_HIP(hipEventCreate(&e));
  hipEvent_t t_begin = ev[4 * (size_t)iters], t_end = ev[4 * (size_t)iters + 1];
  HLP_HIP(hipEventRecord(t_begin, lp->stream));
  for (int32_t i = 0; i < iters; ++i) {
    StepArgs s;
    s.j = i;
    s.ev_start = ev[4 * i];
    s.ev_stop = ev[4 * i + 1];
    HLP_HIP(mixed ? launch_primal32(lp, s) : launch_primal(lp, s));
    s.ev_start = ev[4 * i + 2];
    s.ev_stop = ev[4 * i + 3];
    HLP_HIP(mixed ? launch_dual32(lp, s) : launch_dual(lp, s));
  }
  HLP_HIP(hipEventRecord(t_end, lp->stream));
  HLP_HIP(hipStreamSynchronize(lp->stream));
  double tp = 0.0, td = 0.0;
  for (int32_t i = 0; i < iters; ++i) {
    float a = 0.f, b = 0.f;
    HLP_HIP(hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]));
    HLP_HIP(hipEventElapsedTime(&b, ev[4 * i + 2], ev[4 * i + 3]));
    tp += a;
    td += b;
  }
  float all = 0.f;
  HLP_HIP(hipEventElapsedTime(&all, t_begin, t_end));
  for (auto& e : ev) (void)hipEventDestroy(e);
  ms_out[0] = tp / iters;
  ms_out[1] = td / iters;
  ms_out[2] = (double)all / iters;
  ms_out[3] = iters;
  return HLP_OK;
}

}  // extern "C"
