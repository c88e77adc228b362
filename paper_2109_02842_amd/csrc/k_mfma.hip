// Range compression as a dense contraction on the matrix cores (BF16 / FP16).
#include "device.hpp"

namespace pl {

int launch_range_compress_mfma(const HybridPlan&, const float2*, char*, float2*, hipStream_t) {
    return fail(PL_EUNSUPPORTED, "MFMA range compression is not built yet");
}

}  // namespace pl
