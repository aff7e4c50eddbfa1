// Latent fetch kernels: the filtered lookup alone, the distinct-texel footprint of a batch,
// and the FP32 -> FP16 texel conversion used by post-training quantisation.
#include "latent_fetch.h"

namespace nam {

template <int C, bool F16>
__global__ void __launch_bounds__(256) fetch_kernel(PyrArgs p, const float* __restrict__ tex32,
                                                    const __half* __restrict__ tex16, int n,
                                                    const float2* __restrict__ uv,
                                                    const float* __restrict__ lod, float* __restrict__ z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 q = uv[i];
    Taps t;
    query_taps(p, q.x, q.y, lod[i], t);
    float acc[C];
    if constexpr (F16) gather_f16<C>(tex16, t, acc);
    else gather_f32<C>(tex32, t, acc);
    float4* out = reinterpret_cast<float4*>(z + (int64_t)i * C);
    #pragma unroll
    for (int c4 = 0; c4 < C / 4; ++c4)
        out[c4] = make_float4(acc[4 * c4], acc[4 * c4 + 1], acc[4 * c4 + 2], acc[4 * c4 + 3]);
}

// Marks every texel that one of the taps addresses (weight irrelevant) in a bitmap: the 8
// trilinear taps, or with draws xi the 4 taps of the level chosen by Russian roulette.
__global__ void __launch_bounds__(256) footprint_kernel(PyrArgs p, int n, const float2* __restrict__ uv,
                                                        const float* __restrict__ lod,
                                                        const float* __restrict__ xi,
                                                        uint32_t* __restrict__ bitmap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 q = uv[i];
    Taps t;
    if (xi) {
        query_taps_rr(p, q.x, q.y, lod[i], xi[i], t);
        #pragma unroll
        for (int k = 0; k < 4; ++k) atomicOr(bitmap + (t.idx[k] >> 5), 1u << (t.idx[k] & 31));
    } else {
        query_taps(p, q.x, q.y, lod[i], t);
        #pragma unroll
        for (int k = 0; k < 8; ++k) atomicOr(bitmap + (t.idx[k] >> 5), 1u << (t.idx[k] & 31));
    }
}

__global__ void __launch_bounds__(256) popcount_kernel(const uint32_t* __restrict__ bitmap, int64_t words,
                                                       unsigned long long* __restrict__ count) {
    unsigned long long local = 0;
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words;
         w += (int64_t)gridDim.x * blockDim.x)
        local += __popc(bitmap[w]);
    // wave reduction, one atomic per wave
    for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(count, local);
}

__global__ void __launch_bounds__(256) f32_to_f16_kernel(const float4* __restrict__ src, __half2* __restrict__ dst,
                                                         int64_t count4) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = src[i];
        dst[2 * i] = __floats2half2_rn(v.x, v.y);
        dst[2 * i + 1] = __floats2half2_rn(v.z, v.w);
    }
}

static int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

hipError_t launch_fetch(const nam_material* m, int64_t n, const float* uv, const float* lod, float* z,
                        hipStream_t s) {
    const bool f16 = m->tprec == NAM_F16;
    const dim3 grid(blocks_for(n, 256)), block(256);
    const float2* uv2 = reinterpret_cast<const float2*>(uv);
    clear_stale_hip_error();
    if (m->desc.channels == 8) {
        if (f16) fetch_kernel<8, true><<<grid, block, 0, s>>>(m->pyr(), nullptr, m->texels16, (int)n, uv2, lod, z);
        else fetch_kernel<8, false><<<grid, block, 0, s>>>(m->pyr(), m->texels32, nullptr, (int)n, uv2, lod, z);
    } else {
        if (f16) fetch_kernel<16, true><<<grid, block, 0, s>>>(m->pyr(), nullptr, m->texels16, (int)n, uv2, lod, z);
        else fetch_kernel<16, false><<<grid, block, 0, s>>>(m->pyr(), m->texels32, nullptr, (int)n, uv2, lod, z);
    }
    return hipGetLastError();
}

hipError_t launch_footprint(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                            uint32_t* bitmap, hipStream_t s) {
    clear_stale_hip_error();
    footprint_kernel<<<blocks_for(n, 256), 256, 0, s>>>(m->pyr(), (int)n, reinterpret_cast<const float2*>(uv),
                                                       lod, xi, bitmap);
    return hipGetLastError();
}

hipError_t launch_popcount(const uint32_t* bitmap, int64_t words, unsigned long long* count, hipStream_t s) {
    clear_stale_hip_error();
    popcount_kernel<<<1024, 256, 0, s>>>(bitmap, words, count);
    return hipGetLastError();
}

hipError_t launch_texels_to_f16(const float* src, __half* dst, int64_t count, hipStream_t s) {
    // count is a multiple of 8 (C in {8, 16})
    clear_stale_hip_error();
    f32_to_f16_kernel<<<2048, 256, 0, s>>>(reinterpret_cast<const float4*>(src), reinterpret_cast<__half2*>(dst),
                                           count / 4);
    return hipGetLastError();
}

}  // namespace nam
