// Host side of the matrix-core decode for materials without learned shading frames, and the
// entry point for every material (the kernels themselves are in decode_mfma.h; the
// frame-transform variants are instantiated in decode_mfma_frames.hip).
#include "decode_mfma.h"

namespace nam {

bool mfma_shape_supported(const MlpShape& sh) {
    return (sh.C == 8 || sh.C == 16) && (sh.H == 16 || sh.H == 32 || sh.H == 64) && sh.NH >= 1 && sh.NH <= 4;
}

hipError_t dispatch_mfma_frames(bool l1f16, bool hf8, const nam_material* m, const MfmaArgs& a, int cu, hipStream_t s);

// materials without learned frames run kernels with no frame code at all
template <bool L1F16, bool HF8>
static hipError_t dispatch_mode(const nam_material* m, const MfmaArgs& a, int cu, hipStream_t s) {
    return a.nf ? dispatch_mfma_frames(L1F16, HF8, m, a, cu, s) : dispatch_filter<L1F16, HF8, false>(m, a, cu, s);
}

hipError_t launch_decode_mfma(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                              const float* wi, const float* wo, float* rgb, hipStream_t s) {
    MfmaArgs a{};
    a.pyr = m->pyr();
    a.tex = m->texels16;
    a.w = static_cast<const uint4*>(m->wmfma);
    a.bias = reinterpret_cast<const floatx4*>(static_cast<const char*>(m->wmfma) + m->wmfma_bias_offset);
    // E4M3 scales are powers of two, so 448 / s and 1 / s are exact
    a.in_hi = 448.0f / m->in_scale;
    a.in_inv = 1.0f / m->in_scale;
    for (int k = 0; k < kMaxLayers; ++k) {
        a.mid_hi[k] = 448.0f / m->mid_scale[k];
        a.mid_inv[k] = 1.0f / m->mid_scale[k];
    }
    a.out_scale = m->out_scale;
    a.n = (int)n;
    a.nchunks = (int)((n + kChunk - 1) / kChunk);
    a.uv = reinterpret_cast<const float2*>(uv);
    a.lod = lod;
    a.xi = xi;
    a.wi = wi;
    a.wo = wo;
    a.rgb = rgb;
    a.frames = m->frames32;
    a.nf = m->shape.NF;
    const int cu = m->ctx->cu_count;
    if (m->wprec == NAM_F16) return dispatch_mode<true, false>(m, a, cu, s);
    if (m->first_layer_f16) return dispatch_mode<true, true>(m, a, cu, s);
    return dispatch_mode<false, true>(m, a, cu, s);
}

}  // namespace nam
