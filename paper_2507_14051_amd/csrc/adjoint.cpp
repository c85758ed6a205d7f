// Reverse mode of K unrolled iterations (placeholder until the tape format lands).
#include "hlp_internal.h"

using namespace hlp;

extern "C" {

hlp_err hlp_tape_bytes(const hlp_lp* lp, int32_t K, int32_t ckpt_every, size_t* bytes) {
  (void)lp; (void)K; (void)ckpt_every; (void)bytes;
  set_error("not built yet");
  return HLP_EUNSUPPORTED;
}

hlp_err hlp_unrolled_forward(hlp_lp* lp, const hlp_params* p, int32_t K, int32_t ckpt_every, int32_t replay,
                             const double* x0, const double* y0, double* x, double* y, void* tape,
                             size_t tape_bytes) {
  (void)lp; (void)p; (void)K; (void)ckpt_every; (void)replay; (void)x0; (void)y0; (void)x; (void)y;
  (void)tape; (void)tape_bytes;
  set_error("not built yet");
  return HLP_EUNSUPPORTED;
}

hlp_err hlp_unrolled_backward(hlp_lp* lp, const void* tape, size_t tape_bytes, const double* gx,
                              const double* gy, double* gc, double* glc, double* guc, double* glv,
                              double* guv) {
  (void)lp; (void)tape; (void)tape_bytes; (void)gx; (void)gy; (void)gc; (void)glc; (void)guc; (void)glv;
  (void)guv;
  set_error("not built yet");
  return HLP_EUNSUPPORTED;
}

}  // extern "C"
