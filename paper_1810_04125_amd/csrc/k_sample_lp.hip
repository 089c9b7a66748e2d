// Reduced-precision sampling (FP32 and split BF16x3); see launch_sample.
#include "gen.h"

namespace hss {

void launch_sample_f32(const GenDev& g, int32_t transpose, int32_t bf16x3, const double* R,
                       int64_t ldr, double* S, int64_t lds, int32_t ncols, double* partial,
                       hipStream_t s) {
  (void)g; (void)transpose; (void)bf16x3; (void)R; (void)ldr; (void)S; (void)lds; (void)ncols;
  (void)partial; (void)s;
  throw Error(HSS_ERR_INVALID_ARG, "reduced-precision sampling is not available in this build");
}

}  // namespace hss
