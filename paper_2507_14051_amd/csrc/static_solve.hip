// hlp_solve_static: setup and solve in one call with the library's own static
// device scratch as the workspace, for callers that cannot allocate device
// memory.  Same kernels and host controller as hlp_lp_create + hlp_solve; the
// workspace is the file-scope array below instead of a caller buffer.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "hlp_internal.h"

namespace {

constexpr size_t kStaticBytes = HLP_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// Each GPU the library runs on holds its own copy of this array until the
// process ends.  Host code never uses its name as an address: the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up on the first call on
// that device (with that device current) and kept.
hlp_err scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hlp::hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    hlp::set_error("hlp_solve_static: device ordinal beyond the supported range");
    return HLP_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hlp::hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) {
      hlp::set_error("hlp_solve_static: no device address for the static scratch");
      return HLP_EHIP;
    }
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return HLP_OK;
}

}  // namespace

extern "C" {

hlp_err hlp_solve_static(int32_t m, int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                         const double* val, const double* c, const double* lc, const double* uc,
                         const double* lv, const double* uv, const hlp_params* p, void* hip_stream, double* x,
                         double* y, double* r, hlp_info* info) {
  hlp_params q;
  hlp_params_default(&q);
  if (p) q = *p;
  q.graphs = 0;  // graph instantiation would allocate
  q.trace_iters = 0;
  size_t need = 0;
  HLP_TRY(hlp_workspace_bytes(m, n, nnz, &q, &need));
  if (need > kStaticBytes) {
    hlp::set_error("hlp_solve_static: the LP needs a workspace of " + std::to_string(need) +
                   " bytes; the static scratch holds " + std::to_string(kStaticBytes));
    return HLP_ENOMEM;
  }
  void* ws = nullptr;
  HLP_TRY(scratch_address(&ws));
  hlp_lp lp;
  lp.keep_log = false;
  HLP_TRY(hlp::setup_into(&lp, m, n, nnz, row_ptr, col_idx, val, c, lc, uc, lv, uv, &q, ws, kStaticBytes,
                          hip_stream, false));
  return hlp_solve(&lp, &q, nullptr, nullptr, x, y, r, info, nullptr);
}

}  // extern "C"
