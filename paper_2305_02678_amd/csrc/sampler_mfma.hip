// The importance-sampling decoder on the matrix cores (Sec. 4.3; App. A) for quantised
// materials.  Sec. 5.2 ("Precision") trains the sampler's master parameters in FP32 beside the
// BRDF decoder's and converts the parameters to FP16 at load time; here the sampling decoder
// runs in FP16 (weights and layer inputs) with FP32 accumulation, and the output activations
// and the proxy stay in FP32 (proxy.h, shared with the FP32 kernel).
//
// The work decomposition is the matrix-core decode's: a persistent grid of 16-wave
// workgroups, each wave taking chunks of 64 consecutive queries on its own, with the chunks
// split into one contiguous range per XCD.  Per chunk a wave
//   fetches   the latent code of its 64 queries (fetch_latents: FP16 taps, FP16 filter) and
//             writes the network input [z, wi, 0 ...] (32 K slots) to its LDS region in the
//             B-operand layout;
//   decodes   the chunk's 4 tiles of 16 queries: layer k is Y^T = W_k Y_{k-1}^T on
//             v_mfma_f32_16x16x32_f16 with the weights (in LDS for the whole kernel) as the A
//             operand and the accumulators of one layer, ReLU'd and rounded, as the next B
//             operand (the K order of the packed weights makes them line up, mfma_pack.h); the
//             output layer is one 16-row tile per query tile, rows 0..8 used, so lane (g, q)
//             of tile t holds raw outputs 4 g .. 4 g + 3 of query 16 t + q;
//   gathers   the 9 raw outputs of each query through its LDS region to the query's own lane,
//             which applies the output activations and, per mode, stores the 9 proxy
//             parameters, the PDF of a given direction, or a sample with its PDF.
#include <algorithm>

#include "decode_mfma.h"
#include "proxy.h"

namespace nam {

struct SamplerMfmaArgs {
    PyrArgs pyr;
    const __half* tex;        // FP16 texels
    const uint4* w;           // the sampling decoder's packed A operands (mfma_pack.h)
    const floatx4* bias;      // per (layer, row tile, lane): 4 FP32 biases
    int n;
    int nchunks;
    int groups;               // XCD groups: min(8, grid); the grid is a multiple of it
    int mode;                 // SamplerMode
    const float2* uv;
    const float* lod;
    const float* wi;
    const float* wo_in;       // kModePdf
    const float* u;           // kModeSample
    float* params_out;        // kModeParams: [n][9]
    float* wo_out;            // kModeSample: [n][3]
    float* pdf_out;           // kModePdf, kModeSample: [n]
};

// ReLU'd accumulators of a layer's RT row tiles as the next layer's KS B operands (the K order
// of the packed weights puts row tiles 2 s and 2 s + 1 in step s).
template <int RT, int KS>
__device__ __forceinline__ void relu_operands(const floatx4 (&acc)[4][RT], half8 (&bk)[4][KS]) {
    #pragma unroll
    for (int t = 0; t < 4; ++t)
        #pragma unroll
        for (int s = 0; s < KS; ++s)
            #pragma unroll
            for (int e = 0; e < 8; e += 2) {
                const int j = 2 * s + e / 4;
                const half2_t h = (j < RT) ? relu_pack_f16(acc[t][j][e % 4], acc[t][j][e % 4 + 1])
                                           : half2_t{(_Float16)0.0f, (_Float16)0.0f};
                bk[t][s][e] = h[0];
                bk[t][s][e + 1] = h[1];
            }
}

template <int C, int H, int NH, int ADDR>
__global__ void __launch_bounds__(kBlock, 1) sampler_mfma_kernel(const SamplerMfmaArgs a) {
    constexpr int NT = 8;                      // trilinear taps per query
    constexpr int RT = H / 16;                 // row tiles of a hidden layer
    constexpr int KS = (H + 31) / 32;          // K steps over a hidden layer's outputs
    constexpr int NHB = (NH - 1) * RT * KS;    // hidden A blocks; the output layer's KS follow
    // the decoder first: every weight and bias read is a lane offset plus an immediate below
    // 64 KiB; each wave's 4 KiB region holds the tap table, then the network input, then the
    // raw outputs of its chunk
    struct alignas(16) Smem {
        uint8_t A0[RT][64 * 16];
        uint8_t AH[NHB + KS][64 * 16];
        floatx4 bias[NH * RT + 1][4];
        LevelRowL rows[kMaxLevels];
        uint8_t wreg[kWaves][4096];
    };
    static_assert(offsetof(Smem, rows) + sizeof(LevelRowL) * kMaxLevels <= 65536, "decoder beyond 64 KiB of LDS");
    __shared__ Smem sm;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: chunk indices in scalar registers
    const int g = lane >> 4;
    const MfmaLayout lay = mfma_layout(C, H, NH, true, false);
    {
        const uint4* w = a.w;
        for (int i = threadIdx.x; i < RT * 64; i += kBlock)
            *reinterpret_cast<uint4*>(&sm.A0[i >> 6][(i & 63) * 16]) = w[lay.a_index(0, i >> 6, 0) * 64 + (i & 63)];
        for (int i = threadIdx.x; i < (NHB + KS) * 64; i += kBlock) {
            const int b = i >> 6, ln = i & 63;
            const int blk = b < NHB ? lay.a_index(b / (RT * KS) + 1, (b / KS) % RT, b % KS) : lay.a_index(NH, 0, b - NHB);
            *reinterpret_cast<uint4*>(&sm.AH[b][ln * 16]) = w[blk * 64 + ln];
        }
        for (int i = threadIdx.x; i < (NH * RT + 1) * 4; i += kBlock) sm.bias[i >> 2][i & 3] = a.bias[(i >> 2) * 64 + 16 * (i & 3)];
        if (threadIdx.x < a.pyr.M) {
            const LevelRow r = a.pyr.rows[threadIdx.x];
            sm.rows[threadIdx.x] = LevelRowL{(float)r.w, (float)r.h, r.w - 1, r.h - 1, (uint32_t)(r.off * C * 2),
                                             (uint32_t)(r.w * C * 2), 0, 0};
        }
    }
    __syncthreads();

    const int X = a.groups;
    const int grp = (int)blockIdx.x % X;
    const int stride = ((int)gridDim.x / X) * kWaves;
    int c = (int)((int64_t)a.nchunks * grp / X) + ((int)blockIdx.x / X) * kWaves + wave;
    const int c_end = (int)((int64_t)a.nchunks * (grp + 1) / X);
    if (c >= c_end) return;
    const int n = a.n;
    const int mode = a.mode;
    uint8_t* const reg = sm.wreg[wave];
    const int t_own = lane >> 4, q_own = lane & 15;            // this lane's query in the B layout

    float2 uv = *chunk_elem<1>(a.uv, n, c * kChunk, lane);
    float lod = *chunk_elem<1>(a.lod, n, c * kChunk, lane);
    for (; c < c_end; c += stride) {
        const int first = c * kChunk;                              // uniform
        // ---- fetch.  Lane = query: taps, wi and the mode's direction or draws, then the texels
        const bool use = query_ok(uv.x, uv.y, lod);
        uint32_t off[NT];
        float w[NT];
        tap_stencil<C, ADDR, false>(a.pyr.M, sm.rows, use, uv.x, uv.y, lod, 0.0f, off, w);
        float wi[3], e3[3] = {0.0f, 0.0f, 0.0f};
        {
            const float* p = chunk_elem<3>(a.wi, n, first, lane);
            #pragma unroll
            for (int d = 0; d < 3; ++d) wi[d] = p[d];
            if (mode != kModeParams) {
                const float* q = chunk_elem<3>(mode == kModePdf ? a.wo_in : a.u, n, first, lane);
                #pragma unroll
                for (int d = 0; d < 3; ++d) e3[d] = q[d];
            }
        }
        half2_t zown[C / 2];
        fetch_latents<C, NT, true, false>(reinterpret_cast<const uint8_t*>(a.tex), off, w, reg, reg, lane, 0.0f, 1.0f,
                                          zown, [&] {
            const int nf = (c + stride) * kChunk;                  // next chunk: clamped, valid queries
            uv = *chunk_elem<1>(a.uv, n, nf, lane);
            lod = *chunk_elem<1>(a.lod, n, nf, lane);
        });
        {
            // wi after z, zeros up to slot 32
            float x[24];
            #pragma unroll
            for (int k = 0; k < 24; ++k) x[k] = 0.0f;
            #pragma unroll
            for (int d = 0; d < 3; ++d) x[d] = wi[d];
            #pragma unroll
            for (int gg = C / 8; gg < 4; ++gg) store_slots_f<true>(reg, t_own, gg, q_own, x + 8 * (gg - C / 8), 0.0f, 1.0f);
        }
        lds_wave_sync();

        // ---- decode the chunk's 4 tiles at the higher issue priority (as in the decode)
        __builtin_amdgcn_s_setprio(1);
        floatx4 acc[4][RT];
        #pragma unroll
        for (int j = 0; j < RT; ++j) {
            const floatx4 b = sm.bias[lay.b_index(0, j)][g];
            const half8 wa = *reinterpret_cast<const half8*>(&sm.A0[j][lane * 16]);
            #pragma unroll
            for (int t = 0; t < 4; ++t) acc[t][j] = mfma_f16(wa, *reinterpret_cast<const half8*>(reg + (t * 64 + lane) * 16), b);
        }
        lds_wave_sync();                                           // the input is consumed
        #pragma unroll
        for (int kk = 1; kk < NH; ++kk) {
            half8 bk[4][KS];
            relu_operands<RT, KS>(acc, bk);
            #pragma unroll
            for (int j = 0; j < RT; ++j) {
                const floatx4 b = sm.bias[lay.b_index(kk, j)][g];
                half8 wa[KS];
                #pragma unroll
                for (int s = 0; s < KS; ++s) wa[s] = *reinterpret_cast<const half8*>(&sm.AH[(kk - 1) * RT * KS + j * KS + s][lane * 16]);
                #pragma unroll
                for (int t = 0; t < 4; ++t) {
                    floatx4 v = b;
                    #pragma unroll
                    for (int s = 0; s < KS; ++s) v = mfma_f16(wa[s], bk[t][s], v);
                    acc[t][j] = v;
                }
            }
        }
        floatx4 out[4];
        {
            half8 bk[4][KS];
            relu_operands<RT, KS>(acc, bk);
            const floatx4 b = sm.bias[lay.b_index(NH, 0)][g];
            #pragma unroll
            for (int t = 0; t < 4; ++t) out[t] = b;
            #pragma unroll
            for (int s = 0; s < KS; ++s) {
                const half8 wa = *reinterpret_cast<const half8*>(&sm.AH[NHB + s][lane * 16]);
                #pragma unroll
                for (int t = 0; t < 4; ++t) out[t] = mfma_f16(wa, bk[t][s], out[t]);
            }
        }
        __builtin_amdgcn_s_setprio(0);

        // ---- gather: query Q's 16 accumulator rows at bytes [64 Q, 64 Q + 64) of the region
        #pragma unroll
        for (int t = 0; t < 4; ++t) *reinterpret_cast<floatx4*>(reg + ((16 * t + q_own) * 16 + 4 * g) * 4) = out[t];
        lds_wave_sync();
        float raw[9];
        {
            const floatx4 r0 = *reinterpret_cast<const floatx4*>(reg + lane * 64);
            const floatx4 r1 = *reinterpret_cast<const floatx4*>(reg + lane * 64 + 16);
            const float r2 = *reinterpret_cast<const float*>(reg + lane * 64 + 32);
            #pragma unroll
            for (int k = 0; k < 4; ++k) {
                raw[k] = r0[k];
                raw[4 + k] = r1[k];
            }
            raw[8] = r2;
        }
        lds_wave_sync();                                           // the region is free for the next chunk

        // ---- activations and the mode's output for this lane's query
        if (first + lane < n) {
            float pr[9];
            proxy_activate(raw, pr);
            const float nan = __builtin_nanf("");
            const int64_t i = (int64_t)first + lane;
            if (mode == kModeParams) {
                #pragma unroll
                for (int k = 0; k < 9; ++k) a.params_out[9 * i + k] = use ? pr[k] : nan;
            } else if (mode == kModePdf) {
                a.pdf_out[i] = use ? proxy_pdf(pr, wi, e3) : nan;
            } else {
                float wo[3];
                const float pd = proxy_sample(pr, wi, e3, wo);
                #pragma unroll
                for (int d = 0; d < 3; ++d) a.wo_out[3 * i + d] = use ? wo[d] : nan;
                a.pdf_out[i] = use ? pd : nan;
            }
        }
    }
}

template <int C, int H, int NH, int ADDR>
static hipError_t launch_sampler_mfma_shape(SamplerMfmaArgs& a, int cu_count, hipStream_t s) {
    static const int blocks_per_cu = [] {   // thread-safe one-time query
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, sampler_mfma_kernel<C, H, NH, ADDR>, kBlock, 0) != hipSuccess ||
            b < 1)
            b = 1;
        return b;
    }();
    // the persistent grid, no larger than a chunk per wave, a multiple of the XCD groups
    int grid = std::min(cu_count * blocks_per_cu, (a.nchunks + kWaves - 1) / kWaves);
    if (grid >= 8) grid -= grid % 8;
    grid = std::max(grid, 1);
    a.groups = std::min(grid, 8);
    clear_stale_hip_error();
    sampler_mfma_kernel<C, H, NH, ADDR><<<grid, kBlock, 0, s>>>(a);
    return hipGetLastError();
}

template <int ADDR>
static hipError_t dispatch_sampler_mfma(const MlpShape& sh, SamplerMfmaArgs& a, int cu, hipStream_t s) {
#define NAM_SM_CASE(C_, H_, NH_) \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_) return launch_sampler_mfma_shape<C_, H_, NH_, ADDR>(a, cu, s);
#define NAM_SM_H(C_, H_) NAM_SM_CASE(C_, H_, 1) NAM_SM_CASE(C_, H_, 2) NAM_SM_CASE(C_, H_, 3) NAM_SM_CASE(C_, H_, 4)
    NAM_SM_H(8, 16) NAM_SM_H(8, 32) NAM_SM_H(8, 64)
    NAM_SM_H(16, 16) NAM_SM_H(16, 32) NAM_SM_H(16, 64)
#undef NAM_SM_H
#undef NAM_SM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sampler_mfma(const nam_material* m, int64_t n, int mode, const float* uv, const float* lod,
                               const float* wi, const float* wo_in, const float* u, float* params_out, float* wo_out,
                               float* pdf_out, hipStream_t s) {
    SamplerMfmaArgs a{};
    a.pyr = m->pyr();
    a.tex = m->texels16;
    a.w = static_cast<const uint4*>(m->smfma);
    a.bias = reinterpret_cast<const floatx4*>(static_cast<const char*>(m->smfma) + m->smfma_bias_offset);
    a.n = (int)n;
    a.nchunks = (int)((n + kChunk - 1) / kChunk);
    a.mode = mode;
    a.uv = reinterpret_cast<const float2*>(uv);
    a.lod = lod;
    a.wi = wi;
    a.wo_in = wo_in;
    a.u = u;
    a.params_out = params_out;
    a.wo_out = wo_out;
    a.pdf_out = pdf_out;
    return m->desc.address == NAM_WRAP ? dispatch_sampler_mfma<NAM_WRAP>(m->sshape, a, m->ctx->cu_count, s)
                                       : dispatch_sampler_mfma<NAM_CLAMP>(m->sshape, a, m->ctx->cu_count, s);
}

}  // namespace nam
