// Host side of the matrix-core decode for materials without learned shading frames, and the
// entry point for every material (the kernels themselves are in decode_mfma.h; the
// frame-transform variants are instantiated in decode_mfma_frames.hip).
#include <algorithm>

#include "decode_mfma.h"

namespace nam {

bool mfma_shape_supported(const MlpShape& sh) {
    return (sh.C == 8 || sh.C == 16) && (sh.H == 16 || sh.H == 32 || sh.H == 64) && sh.NH >= 1 && sh.NH <= 4;
}

hipError_t dispatch_mfma_frames(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s);

// materials without learned frames run kernels with no frame code at all
template <bool L1F16, bool HF8>
static hipError_t dispatch_mode(const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s) {
    return L.item[0].nf ? dispatch_mfma_frames(L1F16, HF8, m, L, cu, s) : dispatch_filter<L1F16, HF8, false>(m, L, cu, s);
}

static hipError_t dispatch_launch(const nam_material* m, MfmaLaunch& L, hipStream_t s) {
    const int cu = m->ctx->cu_count;
    if (m->wprec == NAM_F16) return dispatch_mode<true, false>(m, L, cu, s);
    if (m->first_layer_f16) return dispatch_mode<true, true>(m, L, cu, s);
    return dispatch_mode<false, true>(m, L, cu, s);
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
           (a->shape.NF > 0) == (b->shape.NF > 0) && a->desc.address == b->desc.address;
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
