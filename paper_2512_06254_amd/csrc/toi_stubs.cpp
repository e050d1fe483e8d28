// Entry points whose device path is not built yet: they report
// TOI_EUNSUPPORTED instead of computing anything.
#include "toi_internal.h"

namespace toi {

hipError_t launch_detect(toi_ctx*, const float*, int, int32_t*, int, int32_t*) { return hipErrorNotSupported; }

}  // namespace toi

extern "C" toi_status toi_image_batch(toi_ctx* c, const toi_snapshot*, int32_t, float*, float*) {
    return toi::fail(c, TOI_EUNSUPPORTED, "toi_image_batch: not implemented in this build");
}
