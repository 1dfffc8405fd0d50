// FP8 (OCP E4M3) form of the row sketch: placeholder until the FP8 MFMA
// kernel lands; reports the combination as unsupported.
#include "rpid_internal.hpp"

namespace rpid {

size_t sketch_fp8_workspace(int64_t m, int64_t n, int64_t l) {
  (void)m;
  (void)n;
  (void)l;
  return 256;
}

int sketch_fp8(rpid_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda, const float* Om,
               int64_t l, int64_t ldo, float* X, int64_t ldx, size_t ws_off) {
  (void)ctx; (void)A; (void)m; (void)n; (void)lda; (void)Om; (void)l; (void)ldo; (void)X;
  (void)ldx; (void)ws_off;
  return RPID_ERR_UNSUPPORTED;
}

}  // namespace rpid
