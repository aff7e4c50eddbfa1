// Low-precision decode on the gfx950 matrix cores: one fused, persistent kernel per material
// precision (FP16 weights and activations; OCP E4M3 weights and activations with one scale per
// layer; E4M3 with the first layer kept in FP16).  Accumulation is FP32 throughout, the bias is
// added in FP32 (as the accumulator's initial value) and softplus is evaluated in FP32.
//
// Work decomposition.  A workgroup of 256 lanes handles chunks of 256 consecutive queries:
//   phase A  each lane fetches one query: 8 trilinear taps of FP16 texels (16-byte loads),
//            blended in FP32, and writes the network input [z, wi, wo, 0...] (32 slots) to LDS
//            in the lane order the matrix-core B operand expects;
//   phase B  each wave evaluates the decoder for 4 tiles of 16 queries: a layer is
//            Y^T = W Y_prev^T with the weights as the A operand (one 16-neuron row tile per
//            instruction, v_mfma_f32_16x16x32_{f16,fp8}) and one query per column.
// The accumulator of a row tile leaves lane (g, q) = (lane / 16, lane % 16) holding neurons
// 4g..4g+3 of query q; the next layer's B operand needs 8 consecutive K slots per lane, so
// the K order of every hidden layer's weights is permuted at load time to slot
// (s, g, e) <-> neuron 16 (2s + e / 4) + 4g + e % 4: two accumulator tiles, ReLU'd and
// converted, are exactly the next B operand, with no shuffle or LDS round trip.
// All weights and biases of the decoder stay in registers for the whole kernel.  LDS is double
// buffered so one barrier per chunk separates phase A of the next chunk from phase B.
// The grid is persistent; chunks are split into one contiguous range per XCD (workgroups are
// dispatched round-robin over the 8 XCDs), so neighbouring screen tiles, which share texels,
// are decoded under the same L2.
#include "latent_fetch.h"
#include "mfma_pack.h"

namespace nam {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kChunkQ = 256;          // queries per chunk = lanes per workgroup
constexpr int kTilesPerChunk = kChunkQ / 16;

struct MfmaArgs {
    PyrArgs pyr;
    const __half* tex;        // FP16 texels
    const uint4* w;           // packed A operands, see mfma_pack.h
    const floatx4* bias;      // per (layer, row tile, lane): 4 biases (pre-scaled for E4M3)
    float in_scale;           // E4M3 scale of the network input (1 when layer 1 is FP16)
    float mid_scale[kMaxLayers];   // multiplier from layer k's accumulator to layer k+1's input
    float out_scale;          // from the output accumulator to q
    int n;
    int nchunks;
    int groups;               // XCD groups: min(8, grid); the grid is a multiple of it
    const float2* uv;
    const float* lod;
    const float* wi;
    const float* wo;
    float* rgb;
};

__device__ __forceinline__ float softplus_f32(float q) {
    return fmaxf(q, 0.0f) + log1pf(expf(-fabsf(q)));
}

__device__ __forceinline__ floatx4 mfma_f16(const half8 a, const half8 b, const floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma_fp8(const long a, const long b, const floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

// Four non-negative floats -> 4 E4M3 bytes (round to nearest even; saturate at 448 first, the
// conversion instruction itself would produce NaN past the largest finite value).
__device__ __forceinline__ uint32_t pack_fp8x4(float a, float b, float c, float d) {
    a = fminf(fmaxf(a, -448.0f), 448.0f);
    b = fminf(fmaxf(b, -448.0f), 448.0f);
    c = fminf(fmaxf(c, -448.0f), 448.0f);
    d = fminf(fmaxf(d, -448.0f), 448.0f);
    int v = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    v = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, v, true);
    return (uint32_t)v;
}

template <int C, int H, int NH, bool L1F16, bool HF8>
__global__ void __launch_bounds__(kChunkQ, 2) decode_mfma_kernel(const MfmaArgs a) {
    constexpr int RT = H / 16;                 // row tiles of a hidden layer
    constexpr int KS = (H + 31) / 32;          // K steps over a hidden layer's outputs
    constexpr int L1_BYTES = L1F16 ? 16 : 8;   // B operand bytes per lane for layer 1
    __shared__ __attribute__((aligned(16))) uint8_t xbuf[2][kTilesPerChunk * 64 * L1_BYTES];
    __shared__ uint8_t okbuf[2][kChunkQ];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    // ---- decoder parameters -> registers (A operands in lane order, biases per lane)
    MfmaLayout lay = mfma_layout(C, H, NH, L1F16, HF8);
    uint4 w1[RT];
    uint4 wh[NH > 1 ? NH - 1 : 1][RT][KS];
    uint4 wout[KS];
    floatx4 b1[RT], bh[NH > 1 ? NH - 1 : 1][RT], bout;
    {
        const uint4* w = a.w;
        #pragma unroll
        for (int j = 0; j < RT; ++j) w1[j] = w[lay.a_index(0, j, 0) * 64 + lane];
        #pragma unroll
        for (int k = 0; k < NH - 1; ++k)
            #pragma unroll
            for (int j = 0; j < RT; ++j)
                #pragma unroll
                for (int s = 0; s < KS; ++s) wh[k][j][s] = w[lay.a_index(k + 1, j, s) * 64 + lane];
        #pragma unroll
        for (int s = 0; s < KS; ++s) wout[s] = w[lay.a_index(NH, 0, s) * 64 + lane];
        #pragma unroll
        for (int j = 0; j < RT; ++j) b1[j] = a.bias[lay.b_index(0, j) * 64 + lane];
        #pragma unroll
        for (int k = 0; k < NH - 1; ++k)
            #pragma unroll
            for (int j = 0; j < RT; ++j) bh[k][j] = a.bias[lay.b_index(k + 1, j) * 64 + lane];
        bout = a.bias[lay.b_index(NH, 0) * 64 + lane];
    }

    // ---- chunk range of this workgroup: one contiguous range per group of workgroups that
    // share an XCD (the grid is a multiple of the group count, so every range has workgroups)
    const int X = a.groups;
    const int xcd = blockIdx.x % X, slot = blockIdx.x / X;
    const int per_xcd = gridDim.x / X;
    const int c_begin = (int)((int64_t)a.nchunks * xcd / X);
    const int c_end = (int)((int64_t)a.nchunks * (xcd + 1) / X);

    int buf = 0;
    for (int c = c_begin + slot; c < c_end; c += per_xcd, buf ^= 1) {
        // ---------------- phase A: fetch one query per lane into LDS
        {
            const int i = c * kChunkQ + threadIdx.x;
            float x[32];
            #pragma unroll
            for (int k = 0; k < 32; ++k) x[k] = 0.0f;
            bool ok = false;
            if (i < a.n) {
                const float2 q = a.uv[i];
                const float l = a.lod[i];
                ok = query_ok(q.x, q.y, l);
                Taps t;
                query_taps(a.pyr, q.x, q.y, l, t);
                gather_f16<C>(a.tex, t, x);
                #pragma unroll
                for (int d = 0; d < 3; ++d) {
                    x[C + d] = a.wi[3 * i + d];
                    x[C + 3 + d] = a.wo[3 * i + d];
                }
            }
            okbuf[buf][threadIdx.x] = ok;
            const int tile = threadIdx.x >> 4, q = threadIdx.x & 15;
            if constexpr (L1F16) {
                #pragma unroll
                for (int g = 0; g < 4; ++g) {
                    half8 h;
                    #pragma unroll
                    for (int e = 0; e < 8; ++e) h[e] = (_Float16)x[8 * g + e];
                    *reinterpret_cast<half8*>(&xbuf[buf][((tile * 4 + g) * 16 + q) * 16]) = h;
                }
            } else {
                #pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const float s = a.in_scale;
                    uint2 v;
                    v.x = pack_fp8x4(x[8 * g] * s, x[8 * g + 1] * s, x[8 * g + 2] * s, x[8 * g + 3] * s);
                    v.y = pack_fp8x4(x[8 * g + 4] * s, x[8 * g + 5] * s, x[8 * g + 6] * s, x[8 * g + 7] * s);
                    *reinterpret_cast<uint2*>(&xbuf[buf][((tile * 4 + g) * 16 + q) * 8]) = v;
                }
            }
        }
        __syncthreads();

        // ---------------- phase B: decoder on 4 tiles of 16 queries per wave
        for (int tt = 0; tt < kTilesPerChunk / 4; ++tt) {
            const int tile = wave * (kTilesPerChunk / 4) + tt;
            floatx4 acc[RT];
            if constexpr (L1F16) {
                const half8 bx = *reinterpret_cast<const half8*>(&xbuf[buf][(tile * 64 + lane) * 16]);
                #pragma unroll
                for (int j = 0; j < RT; ++j) acc[j] = mfma_f16(__builtin_bit_cast(half8, w1[j]), bx, b1[j]);
            } else {
                const long bx = *reinterpret_cast<const long*>(&xbuf[buf][(tile * 64 + lane) * 8]);
                #pragma unroll
                for (int j = 0; j < RT; ++j) {
                    const long wa = (long)w1[j].x | ((long)w1[j].y << 32);
                    acc[j] = mfma_fp8(wa, bx, b1[j]);
                }
            }
            // hidden layers 2..NH, then the output layer
            #pragma unroll
            for (int k = 0; k < NH; ++k) {
                const bool last = (k == NH - 1);
                floatx4 nacc[RT];
                const float m = a.mid_scale[k];
                if constexpr (!HF8) {
                    half8 bk[KS];
                    #pragma unroll
                    for (int s = 0; s < KS; ++s)
                        #pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int j = 2 * s + e / 4;
                            bk[s][e] = (j < RT) ? (_Float16)fmaxf(acc[j][e % 4], 0.0f) : (_Float16)0.0f;
                        }
                    if (!last) {
                        #pragma unroll
                        for (int j = 0; j < RT; ++j) {
                            nacc[j] = bh[k][j];
                            #pragma unroll
                            for (int s = 0; s < KS; ++s) nacc[j] = mfma_f16(__builtin_bit_cast(half8, wh[k][j][s]), bk[s], nacc[j]);
                        }
                    } else {
                        nacc[0] = bout;
                        #pragma unroll
                        for (int s = 0; s < KS; ++s) nacc[0] = mfma_f16(__builtin_bit_cast(half8, wout[s]), bk[s], nacc[0]);
                    }
                } else {
                    long bk[KS];
                    #pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const int j0 = 2 * s, j1 = 2 * s + 1;
                        const uint32_t lo = pack_fp8x4(fmaxf(acc[j0][0], 0.0f) * m, fmaxf(acc[j0][1], 0.0f) * m,
                                                       fmaxf(acc[j0][2], 0.0f) * m, fmaxf(acc[j0][3], 0.0f) * m);
                        uint32_t hi = 0;
                        if (j1 < RT)
                            hi = pack_fp8x4(fmaxf(acc[j1][0], 0.0f) * m, fmaxf(acc[j1][1], 0.0f) * m,
                                            fmaxf(acc[j1][2], 0.0f) * m, fmaxf(acc[j1][3], 0.0f) * m);
                        bk[s] = (long)lo | ((long)hi << 32);
                    }
                    if (!last) {
                        #pragma unroll
                        for (int j = 0; j < RT; ++j) {
                            nacc[j] = bh[k][j];
                            #pragma unroll
                            for (int s = 0; s < KS; ++s) {
                                const long wa = (long)wh[k][j][s].x | ((long)wh[k][j][s].y << 32);
                                nacc[j] = mfma_fp8(wa, bk[s], nacc[j]);
                            }
                        }
                    } else {
                        nacc[0] = bout;
                        #pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            const long wa = (long)wout[s].x | ((long)wout[s].y << 32);
                            nacc[0] = mfma_fp8(wa, bk[s], nacc[0]);
                        }
                    }
                }
                #pragma unroll
                for (int j = 0; j < RT; ++j) acc[j] = nacc[j];
            }
            // lanes 0..15 hold rows 0..3 of the output tile for query (tile, lane)
            if (lane < 16) {
                const int i = c * kChunkQ + tile * 16 + lane;
                if (i < a.n) {
                    const bool ok = okbuf[buf][tile * 16 + lane];
                    #pragma unroll
                    for (int d = 0; d < 3; ++d)
                        a.rgb[3 * (int64_t)i + d] = ok ? softplus_f32(acc[0][d] * a.out_scale) : __builtin_nanf("");
                }
            }
        }
    }
}

bool mfma_shape_supported(const MlpShape& sh) {
    return (sh.C == 8 || sh.C == 16) && (sh.H == 16 || sh.H == 32 || sh.H == 64) && sh.NH >= 1 && sh.NH <= 4;
}

template <int C, int H, int NH, bool L1F16, bool HF8>
static hipError_t launch_shape(const MfmaArgs& args, int cu_count, hipStream_t s) {
    static int blocks_per_cu = 0;
    if (blocks_per_cu == 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, decode_mfma_kernel<C, H, NH, L1F16, HF8>, kChunkQ, 0) !=
                hipSuccess || b < 1)
            b = 1;
        blocks_per_cu = b;
    }
    int grid = cu_count * blocks_per_cu;
    if (grid > args.nchunks) grid = args.nchunks;
    if (grid >= 8) grid -= grid % 8;
    if (grid < 1) grid = 1;
    MfmaArgs a = args;
    a.groups = grid < 8 ? grid : 8;
    decode_mfma_kernel<C, H, NH, L1F16, HF8><<<grid, kChunkQ, 0, s>>>(a);
    return hipGetLastError();
}

template <bool L1F16, bool HF8>
static hipError_t dispatch(const MlpShape& sh, const MfmaArgs& args, int cu, hipStream_t s) {
#define NAM_M_CASE(C_, H_, NH_) \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_) return launch_shape<C_, H_, NH_, L1F16, HF8>(args, cu, s);
#define NAM_M_H(C_, H_) NAM_M_CASE(C_, H_, 1) NAM_M_CASE(C_, H_, 2) NAM_M_CASE(C_, H_, 3) NAM_M_CASE(C_, H_, 4)
    NAM_M_H(8, 16) NAM_M_H(8, 32) NAM_M_H(8, 64)
    NAM_M_H(16, 16) NAM_M_H(16, 32) NAM_M_H(16, 64)
#undef NAM_M_H
#undef NAM_M_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_decode_mfma(const nam_material* m, int64_t n, const float* uv, const float* lod,
                              const float* wi, const float* wo, float* rgb, hipStream_t s) {
    MfmaArgs a{};
    a.pyr = m->pyr();
    a.tex = m->texels16;
    a.w = static_cast<const uint4*>(m->wmfma);
    a.bias = reinterpret_cast<const floatx4*>(static_cast<const char*>(m->wmfma) + m->wmfma_bias_offset);
    a.in_scale = m->in_scale;
    for (int k = 0; k < kMaxLayers; ++k) a.mid_scale[k] = m->mid_scale[k];
    a.out_scale = m->out_scale;
    a.n = (int)n;
    a.nchunks = (int)((n + kChunkQ - 1) / kChunkQ);
    a.uv = reinterpret_cast<const float2*>(uv);
    a.lod = lod;
    a.wi = wi;
    a.wo = wo;
    a.rgb = rgb;
    const int cu = m->ctx->cu_count;
    if (m->wprec == NAM_F16) return dispatch<true, false>(m->shape, a, cu, s);
    if (m->first_layer_f16) return dispatch<true, true>(m->shape, a, cu, s);
    return dispatch<false, true>(m->shape, a, cu, s);
}

}  // namespace nam
