// FP32 decode on the vector ALU: one query per lane, fetch and every decoder layer fused in
// one kernel (Eq. neural-brdf; the shading-frame transform T is the material's learned
// frames when it has them, else the identity).
//
// Data flow per lane: the 8 trilinear taps are blended in registers, the network input
// [z, T wi, T wo] goes to the lane's own column of LDS, and each layer accumulates its outputs in
// registers while streaming its inputs back from that column; a lane only ever touches its
// own column, so no barrier is needed.  Weights are read with wave-uniform (scalar) loads
// from a per-layer transposed copy [in][out] followed by the bias, so that one input's
// weights for all outputs are contiguous.
#include "frames.h"
#include "latent_fetch.h"

namespace nam {

constexpr int kF32Threads = 128;

__device__ __forceinline__ float softplus_f32(float q) {
    // max(q, 0) + log(1 + exp(-|q|)), exact for every q without a threshold
    return fmaxf(q, 0.0f) + log1pf(expf(-fabsf(q)));
}

// out[o] = sum_j Wt[j][o] * col[j] + bias[o], j < IN, o < OUT; Wt and bias wave-uniform.
template <int IN, int OUT>
__device__ __forceinline__ void dense_from_lds(const float* __restrict__ Wt, const float* col, float* out) {
    const float* bias = Wt + IN * OUT;
    #pragma unroll
    for (int o = 0; o < OUT; ++o) out[o] = bias[o];
    #pragma unroll 2
    for (int j = 0; j < IN; ++j) {
        const float aj = col[j * kF32Threads];
        const float* wj = Wt + j * OUT;
        #pragma unroll
        for (int o = 0; o < OUT; ++o) out[o] = fmaf(wj[o], aj, out[o]);
    }
}

// NW: 3-vectors per direction in the network input (1 without frames or with one frame, 2
// with two frames); nf: the material's frame count (0: T is the identity); NO: decoder
// outputs, 3 (RGB) or 6 (RGB, then the albedo triplet), stored as rgb[i][NO].
template <int C, int H, int NH, int NW, int NO, bool F16TEX, bool CALIB>
__global__ void __launch_bounds__(kF32Threads)
decode_f32_kernel(PyrArgs p, const float* __restrict__ tex32, const __half* __restrict__ tex16,
                  const float* __restrict__ wt, const float* __restrict__ frames, int nf, int n, const float2* __restrict__ uv,
                  const float* __restrict__ lod, const float* __restrict__ xi, const float* __restrict__ wi,
                  const float* __restrict__ wo, float* __restrict__ rgb, unsigned int* __restrict__ absmax_bits) {
    __shared__ float act[kMaxWidth * kF32Threads];
    const int i = blockIdx.x * kF32Threads + threadIdx.x;
    const bool live = i < n;
    const int qi = live ? i : n - 1;        // tail lanes recompute the last query, store nothing
    float* col = act + threadIdx.x;

    // fetch and input assembly
    bool finite;
    {
        const float2 q = uv[qi];
        finite = query_ok(q.x, q.y, lod[qi]);
        Taps t;
        float z[C];
        if (xi) {                             // level by Russian roulette: 4 taps
            query_taps_rr(p, q.x, q.y, lod[qi], xi[qi], t);
            if constexpr (F16TEX) gather_f16<C, 4>(tex16, t, z);
            else gather_f32<C, 4>(tex32, t, z);
        } else {                              // trilinear: 8 taps
            query_taps(p, q.x, q.y, lod[qi], t);
            if constexpr (F16TEX) gather_f16<C>(tex16, t, z);
            else gather_f32<C>(tex32, t, z);
        }
        #pragma unroll
        for (int c = 0; c < C; ++c) col[c * kF32Threads] = z[c];
        float dwi[3], dwo[3], dirs[6 * NW];
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
            dwi[c] = wi[3 * qi + c];
            dwo[c] = wo[3 * qi + c];
        }
        if constexpr (NW == 2) {
            frame_inputs<C, 2>(as_constant(frames), z, dwi, dwo, dirs);
        } else if (nf == 1) {
            frame_inputs<C, 1>(as_constant(frames), z, dwi, dwo, dirs);
        } else {
            #pragma unroll
            for (int c = 0; c < 3; ++c) {
                dirs[c] = dwi[c];
                dirs[3 + c] = dwo[c];
            }
        }
        #pragma unroll
        for (int c = 0; c < 6 * NW; ++c) col[(C + c) * kF32Threads] = dirs[c];
    }

    float m_in[NH + 1];
    if constexpr (CALIB) {
        float m = 0.0f;
        #pragma unroll
        for (int j = 0; j < C + 6 * NW; ++j) m = fmaxf(m, fabsf(col[j * kF32Threads]));
        m_in[0] = live ? m : 0.0f;
    }

    // hidden layers (ReLU)
    const float* W = wt;
    {
        float h[H];
        dense_from_lds<C + 6 * NW, H>(W, col, h);
        float m = 0.0f;
        #pragma unroll
        for (int o = 0; o < H; ++o) { h[o] = fmaxf(h[o], 0.0f); col[o * kF32Threads] = h[o]; m = fmaxf(m, h[o]); }
        if constexpr (CALIB) m_in[1] = live ? m : 0.0f;
        W += (C + 6 * NW) * H + H;
    }
    #pragma unroll
    for (int k = 1; k < NH; ++k) {
        float h[H];
        dense_from_lds<H, H>(W, col, h);
        float m = 0.0f;
        #pragma unroll
        for (int o = 0; o < H; ++o) { h[o] = fmaxf(h[o], 0.0f); col[o * kF32Threads] = h[o]; m = fmaxf(m, h[o]); }
        if constexpr (CALIB) m_in[k + 1] = live ? m : 0.0f;
        W += H * H + H;
    }
    // output layer (softplus)
    float qv[NO];
    dense_from_lds<H, NO>(W, col, qv);
    if constexpr (CALIB) {
        #pragma unroll
        for (int k = 0; k <= NH; ++k) {
            float m = m_in[k];
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
            if ((threadIdx.x & 63) == 0) atomicMax(absmax_bits + k, __float_as_uint(m));
        }
    } else if (live) {
        // a non-finite uv or lod has no defined result: report NaN rather than what the ReLUs
        // make of NaN inputs
        #pragma unroll
        for (int c = 0; c < NO; ++c) rgb[NO * (int64_t)i + c] = finite ? softplus_f32(qv[c]) : __builtin_nanf("");
    }
}

template <int C, int H, int NH, int NW, int NO, bool CALIB>
static hipError_t launch_f32_shape(const nam_material* m, int n, const float* uv, const float* lod, const float* xi,
                                   const float* wi, const float* wo, float* rgb, unsigned int* absmax,
                                   hipStream_t s) {
    const dim3 grid((n + kF32Threads - 1) / kF32Threads), block(kF32Threads);
    const float2* uv2 = reinterpret_cast<const float2*>(uv);
    clear_stale_hip_error();
    if (m->tprec == NAM_F16 && !CALIB)
        decode_f32_kernel<C, H, NH, NW, NO, true, CALIB><<<grid, block, 0, s>>>(
            m->pyr(), nullptr, m->texels16, m->wt32, m->frames32, m->shape.NF, n, uv2, lod, xi, wi, wo, rgb, absmax);
    else
        decode_f32_kernel<C, H, NH, NW, NO, false, CALIB><<<grid, block, 0, s>>>(
            m->pyr(), m->texels32, nullptr, m->wt32, m->frames32, m->shape.NF, n, uv2, lod, xi, wi, wo, rgb, absmax);
    return hipGetLastError();
}

// Calibration records no output-layer activation, so it runs the 3-output kernel whatever the
// decoder's width (the hidden layers' weights are laid out alike).
template <bool CALIB, int NO>
static hipError_t dispatch_f32(const nam_material* m, int n, const float* uv, const float* lod, const float* xi,
                               const float* wi, const float* wo, float* rgb, unsigned int* absmax, hipStream_t s) {
    const MlpShape sh = m->shape;
#define NAM_F32_CASE(C_, H_, NH_)                                                                                  \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_)                                                                  \
        return sh.dir_groups() == 2 ? launch_f32_shape<C_, H_, NH_, 2, NO, CALIB>(m, n, uv, lod, xi, wi, wo, rgb, absmax, s) \
                                    : launch_f32_shape<C_, H_, NH_, 1, NO, CALIB>(m, n, uv, lod, xi, wi, wo, rgb, absmax, s);
#define NAM_F32_H(C_, H_) NAM_F32_CASE(C_, H_, 1) NAM_F32_CASE(C_, H_, 2) NAM_F32_CASE(C_, H_, 3) NAM_F32_CASE(C_, H_, 4)
    NAM_F32_H(8, 16) NAM_F32_H(8, 32) NAM_F32_H(8, 64)
    NAM_F32_H(16, 16) NAM_F32_H(16, 32) NAM_F32_H(16, 64)
#undef NAM_F32_H
#undef NAM_F32_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_decode_f32(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                             const float* wi, const float* wo, float* rgb, hipStream_t s) {
    return m->shape.NO == 6 ? dispatch_f32<false, 6>(m, (int)n, uv, lod, xi, wi, wo, rgb, nullptr, s)
                            : dispatch_f32<false, 3>(m, (int)n, uv, lod, xi, wi, wo, rgb, nullptr, s);
}

hipError_t launch_calibrate_f32(const nam_material* m, int64_t n, const float* uv, const float* lod,
                                const float* wi, const float* wo, unsigned int* absmax_bits, hipStream_t s) {
    return dispatch_f32<true, 3>(m, (int)n, uv, lod, nullptr, wi, wo, nullptr, absmax_bits, s);
}

}  // namespace nam
