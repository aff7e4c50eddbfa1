// The matrix-core decode kernels with both the learned-shading-frame transform (Sec. 4.2) and
// the albedo head (Sec. 6.4), instantiated in a translation unit of their own so that the
// kernel families compile in parallel.
#include "decode_mfma.h"

namespace nam {

hipError_t dispatch_mfma_frames_albedo(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu,
                                       hipStream_t s) {
    return dispatch_precision<true, true>(l1f16, hf8, m, L, cu, s);
}

}  // namespace nam
