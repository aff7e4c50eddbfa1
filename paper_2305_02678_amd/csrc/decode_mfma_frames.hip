// The matrix-core decode kernels with the learned-shading-frame transform in the fetch waves
// (Sec. 4.2), instantiated in a translation unit of their own so that the two halves of the
// kernel family compile in parallel.
#include "decode_mfma.h"

namespace nam {

hipError_t dispatch_mfma_frames(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s) {
    if (l1f16 && !hf8) return dispatch_filter<true, false, true>(m, L, cu, s);
    if (l1f16 && hf8) return dispatch_filter<true, true, true>(m, L, cu, s);
    if (!l1f16 && hf8) return dispatch_filter<false, true, true>(m, L, cu, s);
    return hipErrorInvalidValue;
}

}  // namespace nam
