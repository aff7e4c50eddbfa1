// The matrix-core decode kernels with the learned-shading-frame transform in the fetch waves
// (Sec. 4.2) and a 3-output decoder, instantiated in a translation unit of their own so that
// the kernel families compile in parallel.
#include "decode_mfma.h"

namespace nam {

hipError_t dispatch_mfma_frames(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s) {
    return dispatch_precision<true, false>(l1f16, hf8, m, L, cu, s);
}

}  // namespace nam
