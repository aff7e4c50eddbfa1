// The matrix-core decode kernels of decoders with the albedo head (Sec. 6.4: a second RGB
// output, the directional albedo of Eq. albedo) and no learned frames, instantiated in a
// translation unit of their own so that the kernel families compile in parallel.
#include "decode_mfma.h"

namespace nam {

hipError_t dispatch_mfma_albedo(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s) {
    return dispatch_precision<false, true>(l1f16, hf8, m, L, cu, s);
}

}  // namespace nam
