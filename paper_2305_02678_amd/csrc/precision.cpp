// Post-training quantisation of a loaded material (Sec. 5.2, "Precision": FP32 master
// parameters converted to a lower precision at load time).  Texels are converted on the
// device (FP16, round to nearest even); the decoder is quantised and packed into the operand
// order of the matrix-core kernel on the host, where it is a few kilobytes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "mfma_pack.h"
#include "nam_internal.h"

namespace nam {

static uint32_t f32_bits(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    return u;
}

// OCP E4M3FN encoding (bias 7, 3 fraction bits, no infinity, S.1111.111 = NaN), round to
// nearest even on the bit pattern, saturating at +-448.
static uint8_t e4m3_encode(float x) {
    const uint32_t u = f32_bits(x);
    const uint8_t sign = (uint8_t)((u >> 24) & 0x80);
    const uint32_t a = u & 0x7fffffffu;
    if (a > 0x7f800000u) return sign | 0x7f;                 // NaN
    if (a >= f32_bits(448.0f)) return sign | 0x7e;           // saturate (incl. infinity)
    const int e = (int)(a >> 23) - 127;
    if (e < -6) {
        // subnormal range: multiples of 2^-9; |x| * 512 is exact, round it to an even integer
        const float v = std::fabs(x) * 512.0f;
        float r = std::floor(v);
        const float d = v - r;
        if (d > 0.5f || (d == 0.5f && std::fmod(r, 2.0f) != 0.0f)) r += 1.0f;
        return sign | (uint8_t)r;                            // r == 8 encodes 2^-6 (exponent 1)
    }
    const uint32_t mant = a & 0x7fffffu;
    const uint32_t keep = mant >> 20, rest = mant & 0xfffffu;
    uint32_t code = ((uint32_t)(e + 7) << 3) | keep;
    if (rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) code += 1;   // carries into the exponent
    if (code > 0x7e) code = 0x7e;
    return sign | (uint8_t)code;
}

static uint16_t f16_bits(float x) {
    const _Float16 h = (_Float16)x;   // round to nearest even
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}

static float layer_absmax(const std::vector<int>& dims, const std::vector<float>& p, int L) {
    size_t o = 0;
    for (int k = 0; k < L; ++k) o += (size_t)dims[k] * dims[k + 1] + dims[k + 1];
    float m = 0.0f;
    for (size_t i = 0; i < (size_t)dims[L] * dims[L + 1]; ++i) m = std::fmax(m, std::fabs(p[o + i]));
    return m;
}

// Per-layer E4M3 scale: the largest power of two s with absmax * s <= 448 (1 when absmax is 0 or
// not finite).  A power of two makes every rescaling in the decode exact, so the kernel applies
// it inside the hardware conversion.
static float scale_for(float absmax) {
    if (!(absmax > 0.0f) || !std::isfinite(absmax)) return 1.0f;
    int e = 0;
    (void)std::frexp(448.0f / absmax, &e);      // 448 / absmax = f 2^e, f in [0.5, 1)
    return std::ldexp(1.0f, e - 1);
}

// The decoder (dims, FP32 params packed as W_1, b_1, W_2, ...) in the operand order of the
// matrix-core kernels (mfma_pack.h): the A blocks, then the bias blocks.  Layer L's weights are
// rounded to E4M3 after scaling by sw[L] where fp8(L), else to FP16; its biases are kept in FP32
// and scaled by S[L] (the scale of its accumulator).  *a_bytes receives the offset of the bias
// blocks.
template <typename Fp8>
static std::vector<uint8_t> pack_mfma(const MfmaLayout& lay, const std::vector<int>& dims, const std::vector<float>& params,
                                      Fp8 fp8, const float* sw, const float* S, size_t* a_bytes) {
    const int NH = lay.NH;
    const int nA = lay.a_blocks(), nB = lay.b_blocks();
    *a_bytes = (size_t)nA * 64 * 16;
    const size_t b_bytes = (size_t)nB * 64 * 16;
    std::vector<uint8_t> host(*a_bytes + b_bytes, 0);
    size_t off = 0;
    std::vector<size_t> layer_off(NH + 2, 0);
    for (int L = 0; L <= NH; ++L) {
        layer_off[L] = off;
        off += (size_t)dims[L] * dims[L + 1] + dims[L + 1];
    }
    for (int L = 0; L <= NH; ++L) {
        const int fi = dims[L], fo = dims[L + 1];
        const float* W = params.data() + layer_off[L];
        const float* b = W + (size_t)fi * fo;
        const int rts = L < NH ? lay.RT : 1, kss = L == 0 ? 1 : lay.KS;
        for (int j = 0; j < rts; ++j) {
            for (int s = 0; s < kss; ++s) {
                uint8_t* blk = host.data() + (size_t)lay.a_index(L, j, s) * 64 * 16;
                for (int lane = 0; lane < 64; ++lane) {
                    const int g = lane / 16, r = lane % 16, row = 16 * j + r;
                    for (int e = 0; e < 8; ++e) {
                        const int in = MfmaLayout::k_source(L, s, g, e);
                        const float v = (row < fo && in < fi) ? W[(size_t)row * fi + in] : 0.0f;
                        if (fp8(L)) {
                            blk[lane * 16 + e] = e4m3_encode(v * sw[L]);
                        } else {
                            const uint16_t h = f16_bits(v);
                            std::memcpy(blk + lane * 16 + 2 * e, &h, 2);
                        }
                    }
                }
            }
            float* bb = reinterpret_cast<float*>(host.data() + *a_bytes + (size_t)lay.b_index(L, j) * 64 * 16);
            for (int lane = 0; lane < 64; ++lane) {
                const int g = lane / 16;
                for (int i = 0; i < 4; ++i) {
                    const int neuron = 16 * j + 4 * g + i;
                    bb[lane * 4 + i] = neuron < fo ? b[neuron] * S[L] : 0.0f;
                }
            }
        }
    }
    return host;
}

// A sampling decoder (dims, FP32 params) in FP16 for the matrix-core sampler of a quantised
// material (Sec. 5.2 "Precision": the sampler's parameters are converted to FP16 at load like
// the decoder's), uploaded to a new device buffer *out; *bias_offset receives the offset of its
// bias blocks.
nam_status pack_sampler_mfma(nam_ctx* ctx, const std::vector<int>& dims, const std::vector<float>& params, void** out,
                             size_t* bias_offset) {
    const int C = dims.front() - 3, H = dims[1], NH = (int)dims.size() - 2;
    if (!mfma_shape_supported(MlpShape{C, H, NH, 0}))
        return set_error(NAM_E_UNSUPPORTED, "sampling decoder shape not supported on MFMA");
    const MfmaLayout lay = mfma_layout(C, H, NH, true, false);
    float one[kMaxLayers];
    for (float& x : one) x = 1.0f;
    const std::vector<uint8_t> host = pack_mfma(lay, dims, params, [](int) { return false; }, one, one, bias_offset);
    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(NAM_E_HIP, "hipSetDevice failed");
    void* dev = nullptr;
    NAM_HIP(hipMalloc(&dev, host.size()));
    const hipError_t e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_error(e, "hipMemcpy(packed sampler)");
    }
    *out = dev;
    return NAM_OK;
}

}  // namespace nam

using namespace nam;

extern "C" nam_status nam_material_set_precision(nam_ctx* ctx, nam_material* m, nam_dtype weights, nam_dtype texels,
                                                 const float* act_absmax, int first_layer_f16) {
    if (!ctx || !m) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    if (weights != NAM_F32 && weights != NAM_F16 && weights != NAM_FP8_E4M3)
        return set_error(NAM_E_INVALID_ARG, "unknown weight type");
    if (texels != NAM_F32 && texels != NAM_F16 && texels != NAM_FP8_E4M3)
        return set_error(NAM_E_INVALID_ARG, "unknown texel type");
    if (m->server_refs > 0) return set_error(NAM_E_BUSY, "material is held by a server");
    if (weights == NAM_F32) {
        if (texels != NAM_F32) return set_error(NAM_E_UNSUPPORTED, "FP32 weights need FP32 texels");
        hipSetDevice(ctx->device);
        (void)hipFree(m->texels16);
        (void)hipFree(m->wmfma);
        (void)hipFree(m->smfma);
        m->texels16 = nullptr;
        m->wmfma = nullptr;
        m->smfma = nullptr;
        m->wmfma_bytes = 0;
        m->wprec = m->tprec = NAM_F32;
        return NAM_OK;
    }
    if (texels != NAM_F16) return set_error(NAM_E_UNSUPPORTED, "matrix-core decode needs FP16 texels");
    if (!mfma_shape_supported(m->shape)) return set_error(NAM_E_UNSUPPORTED, "decoder shape not supported on MFMA");
    if ((uint64_t)m->texel_count * m->desc.channels * 2 >= (uint64_t(1) << 32))
        return set_error(NAM_E_UNSUPPORTED, "matrix-core decode needs the FP16 pyramid below 4 GiB");
    const bool fp8 = weights == NAM_FP8_E4M3;
    if (fp8 && !act_absmax) return set_error(NAM_E_INVALID_ARG, "E4M3 weights need per-layer activation absmax");

    const int NH = m->shape.NH, H = m->shape.H;
    const MfmaLayout lay = mfma_layout(m->shape.C, H, NH, !fp8 || first_layer_f16, fp8);
    const bool l1f16 = !fp8 || first_layer_f16;
    auto layer_fp8 = [&](int L) { return fp8 && (L > 0 || !l1f16); };

    // scales: S_L = s_w * s_in for an E4M3 layer, 1 for an FP16 layer
    float sw[kMaxLayers], sa[kMaxLayers], S[kMaxLayers];
    for (int L = 0; L <= NH; ++L) {
        sw[L] = layer_fp8(L) ? scale_for(layer_absmax(m->dims, m->host_params, L)) : 1.0f;
        sa[L] = layer_fp8(L) ? scale_for(act_absmax[L]) : 1.0f;
        S[L] = sw[L] * sa[L];
    }

    size_t a_bytes = 0;
    const std::vector<uint8_t> host = pack_mfma(lay, m->dims, m->host_params, layer_fp8, sw, S, &a_bytes);

    if (hipSetDevice(ctx->device) != hipSuccess) return set_error(NAM_E_HIP, "hipSetDevice failed");
    void* wdev = nullptr;
    NAM_HIP(hipMalloc(&wdev, host.size()));
    hipError_t e = hipMemcpy(wdev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(wdev);
        return hip_error(e, "hipMemcpy(packed decoder)");
    }
    if (!m->texels16) {
        const size_t count = (size_t)m->texel_count * m->desc.channels;
        e = hipMalloc(&m->texels16, count * sizeof(__half));
        if (e != hipSuccess) {
            (void)hipFree(wdev);
            m->texels16 = nullptr;
            return hip_error(e, "hipMalloc(fp16 texels)");
        }
        e = launch_texels_to_f16(m->texels32, m->texels16, (int64_t)count, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            (void)hipFree(wdev);
            return hip_error(e, "texel conversion");
        }
    }
    void* sdev = nullptr;                 // the sampling decoder follows the material into FP16
    size_t sbias = 0;
    if (m->swt32) {
        const nam_status st = pack_sampler_mfma(ctx, m->sdims, m->host_sparams, &sdev, &sbias);
        if (st != NAM_OK) {
            (void)hipFree(wdev);
            return st;
        }
    }
    (void)hipFree(m->smfma);
    m->smfma = sdev;
    m->smfma_bias_offset = sbias;
    (void)hipFree(m->wmfma);
    m->wmfma = wdev;
    m->wmfma_bytes = host.size();
    m->wmfma_bias_offset = a_bytes;
    m->wprec = weights;
    m->tprec = NAM_F16;
    m->first_layer_f16 = fp8 && first_layer_f16;
    m->in_scale = sa[0];
    for (int L = 0; L < kMaxLayers; ++L) m->mid_scale[L] = 1.0f;
    for (int L = 0; L < NH; ++L) m->mid_scale[L] = sa[L + 1] / S[L];
    m->out_scale = 1.0f / S[NH];
    for (int L = 0; L <= NH; ++L) {
        m->w_scale[L] = sw[L];
        m->a_scale[L] = sa[L];
    }
    return NAM_OK;
}
