// Low-precision decode on the matrix cores (placeholder until the MFMA kernels land).
#include "latent_fetch.h"

namespace nam {

bool mfma_shape_supported(const MlpShape&) { return false; }

hipError_t launch_decode_mfma(const nam_material*, int64_t, const float*, const float*, const float*, const float*,
                              float*, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace nam
