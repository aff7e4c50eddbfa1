// Host side of the matrix-core decode for materials without learned shading frames and with a
// 3-output decoder, and the entry point for every material (the kernels themselves are in
// decode_mfma.h; the variants with learned frames and with the albedo head are instantiated in
// decode_mfma_frames.hip, decode_mfma_albedo.hip and decode_mfma_frames_albedo.hip).
#include <algorithm>

#include "decode_mfma.h"

namespace nam {

bool mfma_shape_supported(const MlpShape& sh) {
    return (sh.C == 8 || sh.C == 16) && (sh.H == 16 || sh.H == 32 || sh.H == 64) && sh.NH >= 1 && sh.NH <= 4;
}

// Materials without learned frames run kernels with no frame code at all, and 3-output
// decoders kernels with no albedo code.
static hipError_t dispatch_launch(const nam_material* m, MfmaLaunch& L, hipStream_t s) {
    const int cu = m->ctx->cu_count;
    const bool l1f16 = m->wprec == NAM_F16 || m->first_layer_f16, hf8 = m->wprec != NAM_F16;
    const bool fr = L.item[0].nf != 0, al = m->shape.NO == 6;
    if (fr) return al ? dispatch_mfma_frames_albedo(l1f16, hf8, m, L, cu, s) : dispatch_mfma_frames(l1f16, hf8, m, L, cu, s);
    return al ? dispatch_mfma_albedo(l1f16, hf8, m, L, cu, s) : dispatch_precision<false, false>(l1f16, hf8, m, L, cu, s);
}

hipError_t launch_decode_mfma(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                              const float* wi, const float* wo, float* rgb, hipStream_t s) {
    MfmaLaunch L{};
    L.item[0] = mfma_args(m, n, uv, lod, xi, wi, wo, rgb);
    L.count = 1;
    return dispatch_launch(m, L, s);
}

bool mfma_same_kernel(const nam_material* a, const nam_material* b) {
    return a->wprec == b->wprec && a->first_layer_f16 == b->first_layer_f16 && a->wprec != NAM_F32 &&
           a->shape.C == b->shape.C && a->shape.H == b->shape.H && a->shape.NH == b->shape.NH &&
           (a->shape.NF > 0) == (b->shape.NF > 0) && a->shape.NO == b->shape.NO && a->desc.address == b->desc.address;
}

hipError_t launch_decode_mfma_group(int count, const nam_material* const* m, const int64_t* n, const float* const* uv,
                                    const float* const* lod, const float* const* wi, const float* const* wo,
                                    float* const* rgb, hipStream_t s) {
    if (count < 1 || count > kMaxGroup) return hipErrorInvalidValue;
    // the largest batches first, so that they start on XCD boundaries
    int order[kMaxGroup];
    for (int i = 0; i < count; ++i) order[i] = i;
    std::sort(order, order + count, [&](int x, int y) { return n[x] > n[y]; });
    MfmaLaunch L{};
    for (int k = 0; k < count; ++k) {
        const int i = order[k];
        if (!mfma_same_kernel(m[order[0]], m[i]) || n[i] < 1 || n[i] >= (int64_t(1) << 30)) return hipErrorInvalidValue;
        L.item[k] = mfma_args(m[i], n[i], uv[i], lod[i], nullptr, wi[i], wo[i], rgb[i]);
    }
    L.count = count;
    return dispatch_launch(m[order[0]], L, s);
}

}  // namespace nam
