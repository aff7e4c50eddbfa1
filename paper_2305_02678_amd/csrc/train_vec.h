// The FP32 vector-ALU training kernel (one sample per lane; see train.hip), shared by the
// plain and the learned-shading-frame instantiations.
#pragma once

#include "frames.h"
#include "latent_fetch.h"
#include "train_internal.h"

namespace nam {

constexpr int kTW = 64;                 // lanes per workgroup (one wave)
constexpr int kRS = kTW + 1;            // LDS row stride (floats): consecutive rows one bank apart

__device__ __forceinline__ float softplus_acc(float q) { return fmaxf(q, 0.0f) + log1pf(expf(-fabsf(q))); }
__device__ __forceinline__ float logistic(float q) { return 1.0f / (1.0f + expf(-q)); }

// Rows of the LDS activation table: a0 (C + 6 inputs, padded to a multiple of 8), then the
// NH hidden layers (H rows each), then the output deltas (8 rows, NO = 3 or 6 used).  The
// forward-only mode (FWD) keeps no layer for a backward pass, so its hidden layers alternate
// between two blocks: a smaller table, hence more waves per CU.
// With NF learned shading frames the input is [z, T wi, T wo] (C + 6 NF rows), and 6 NF more
// rows after the output deltas hold the gradients of the frame layer's raw outputs.
template <int C, int H, int NH, bool FWD, int NF = 0>
struct TrainRows {
    static constexpr int IN = C + 6 * (NF > 1 ? NF : 1);
    static constexpr int IN_PAD = (IN + 7) / 8 * 8;
    static constexpr int BLOCKS = FWD ? (NH > 1 ? 2 : 1) : NH;
    static constexpr int hid(int k) { return IN_PAD + (FWD ? (k & 1) : k) * H; }   // hidden layer k (0-based)
    static constexpr int OUT = IN_PAD + BLOCKS * H;
    static constexpr int FR = OUT + 8;
    static constexpr int TOTAL = FR + (NF > 0 && !FWD ? (6 * NF + 7) / 8 * 8 : 0);
};

// out[o] = bias[o] + sum_j Wt[j][o] * col[j]   (Wt = per-layer transposed weights, uniform)
template <int IN, int OUT>
__device__ __forceinline__ void dense_t(const float* __restrict__ Wt, const float* __restrict__ bias,
                                        const float* col, float* out) {
    #pragma unroll
    for (int o = 0; o < OUT; ++o) out[o] = bias[o];
    #pragma unroll 2
    for (int j = 0; j < IN; ++j) {
        const float aj = col[j * kRS];
        const float* wj = Wt + j * OUT;
        #pragma unroll
        for (int o = 0; o < OUT; ++o) out[o] = fmaf(wj[o], aj, out[o]);
    }
}

// d_in[j] = sum_o W[o][j] * dcol[o]  (W = original [out][in] layout, rows uniform)
template <int IN, int OUT>
__device__ __forceinline__ void dense_back(const float* __restrict__ W, const float* dcol, float* d_in) {
    #pragma unroll
    for (int j = 0; j < IN; ++j) d_in[j] = 0.0f;
    #pragma unroll 2
    for (int o = 0; o < OUT; ++o) {
        const float d = dcol[o * kRS];
        const float* wo = W + o * IN;
        #pragma unroll
        for (int j = 0; j < IN; ++j) d_in[j] = fmaf(wo[j], d, d_in[j]);
    }
}

typedef float lg_f32x4 __attribute__((ext_vector_type(4)));

// Weight and bias gradient of one layer over the wave's 64 samples, added into the
// workgroup's partial slice: gW[o][j] += sum_s delta[o][s] * act[j][s], gb[o] += sum_s delta[o][s].
// delta rows start at `drow`, activation rows at `arow`.  The weight part runs on the FP32
// matrix cores: 16 x 16 tiles of (output, input) with the 64 samples as the K dimension (16
// steps of 4); in step k lane (g, r) = (lane / 16, lane % 16) supplies delta[16 t + r] and
// act[16 u + r] of sample 4 k + g and ends with outputs 16 t + 4 g .. 16 t + 4 g + 3 of input
// 16 u + r.
template <int FI, int FO>
__device__ __forceinline__ void layer_grad(const float* lds, int drow, int arow, float* __restrict__ gW,
                                           float* __restrict__ gb, int lane) {
    constexpr int RO = (FO + 15) / 16, CJ = (FI + 15) / 16;
    const int g = lane >> 4, r = lane & 15;
    #pragma unroll
    for (int t = 0; t < RO; ++t) {
        lg_f32x4 acc[CJ];
        #pragma unroll
        for (int u = 0; u < CJ; ++u) acc[u] = lg_f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const int o = 16 * t + r;
        #pragma unroll 4
        for (int k = 0; k < kTW / 4; ++k) {
            const int smp = 4 * k + g;
            const float dv = o < FO ? lds[(drow + o) * kRS + smp] : 0.0f;
            #pragma unroll
            for (int u = 0; u < CJ; ++u) {
                const int jj = 16 * u + r;
                const float av = jj < FI ? lds[(arow + jj) * kRS + smp] : 0.0f;
                acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(dv, av, acc[u], 0, 0, 0);
            }
        }
        #pragma unroll
        for (int u = 0; u < CJ; ++u) {
            const int jj = 16 * u + r;
            #pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int oo = 16 * t + 4 * g + e;
                if (oo < FO && jj < FI) gW[oo * FI + jj] += acc[u][e];
            }
        }
    }
    if (lane < FO) {
        float s = 0.0f;
        for (int q = 0; q < kTW; ++q) s += lds[(drow + lane) * kRS + q];
        gb[lane] += s;
    }
}

// NO: decoder outputs, 3 (RGB) or 6 (RGB, then the albedo triplet); outputs, targets and
// output gradients are [n][NO].
// NF: learned shading frames (0: T is the identity); the frame layer W_F[6 NF][C], b_F[6 NF]
// is a.fparams and its gradient the first 6 NF (C + 1) floats of a workgroup's partial slice,
// the decoder's gradient following.
template <int C, int H, int NH, int NO, int MODE, int NF = 0>
__global__ void __launch_bounds__(kTW) fwdbwd_kernel(const TrainArgs a) {
    using R = TrainRows<C, H, NH, MODE == kModeForward, NF>;
    constexpr int IN = R::IN;
    constexpr int NFP = 6 * NF * C + 6 * NF;       // frame-layer parameters
    __shared__ __attribute__((aligned(16))) float lds[R::TOTAL * kRS];
    __shared__ LevelRow lrows[kMaxLevels];
    const int lane = threadIdx.x;
    if (lane < a.M) lrows[lane] = a.rows[lane];
    float* col = lds + lane;

    // this workgroup's partial gradient slice (zeroed here, accumulated over its chunks)
    float* fpart = a.partial ? a.partial + (size_t)blockIdx.x * a.np : nullptr;
    float* part = fpart ? fpart + NFP : nullptr;
    if (MODE != kModeForward) {
        for (int p = lane; p < a.np; p += kTW) fpart[p] = 0.0f;
    }
    float loss_acc = 0.0f;
    lds_sync_wave();

    // parameter offsets of layer k (packed W, b) and of its transposed copy
    int off[NH + 2];
    {
        int o = 0;
        #pragma unroll
        for (int k = 0; k <= NH; ++k) {
            off[k] = o;
            const int fi = k == 0 ? IN : H, fo = k == NH ? NO : H;
            o += fi * fo + fo;
        }
        off[NH + 1] = o;
    }

    const int nchunks = (a.n + kTW - 1) / kTW;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int i = c * kTW + lane;
        const bool in_range = i < a.n;
        const int ic = in_range ? i : a.n - 1;

        // ---- fetch (a non-finite query decodes to NaN and contributes no gradient), or the
        // given code of the sample
        Taps t;
        bool finite = true;
        float z[C];
        if (a.z_in) {
            #pragma unroll
            for (int cc = 0; cc < C; ++cc) {
                z[cc] = a.z_in[(int64_t)ic * C + cc];
                finite = finite && __builtin_isfinite(z[cc]);
            }
        } else {
            const float2 q = reinterpret_cast<const float2*>(a.uv)[ic];
            finite = query_ok(q.x, q.y, a.lod[ic]);
            query_taps_rows(lrows, a.M, a.address, q.x, q.y, a.lod[ic], t);
            gather_f32<C>(a.tex, t, z);
        }
        const bool live = in_range && finite;
        {
            #pragma unroll
            for (int cc = 0; cc < C; ++cc) {
                z[cc] = finite ? z[cc] : 0.0f;
                col[cc * kRS] = z[cc];
            }
            if (NF > 0) {
                const float wi[3] = {a.wi[3 * ic], a.wi[3 * ic + 1], a.wi[3 * ic + 2]};
                const float wo[3] = {a.wo[3 * ic], a.wo[3 * ic + 1], a.wo[3 * ic + 2]};
                float tw[6 * (NF > 0 ? NF : 1)];
                frame_inputs<C, NF>(as_constant(a.fparams), z, wi, wo, tw);
                #pragma unroll
                for (int d = 0; d < 6 * NF; ++d) col[(C + d) * kRS] = tw[d];
            } else {
                #pragma unroll
                for (int d = 0; d < 3; ++d) {
                    col[(C + d) * kRS] = a.wi[3 * ic + d];
                    col[(C + 3 + d) * kRS] = a.wo[3 * ic + d];
                }
            }
            #pragma unroll
            for (int r = IN; r < R::IN_PAD; ++r) col[r * kRS] = 0.0f;
        }

        // ---- forward, keeping every layer's activations
        {
            float h[H];
            dense_t<IN, H>(a.wt + off[0], a.params + off[0] + IN * H, col, h);
            #pragma unroll
            for (int o = 0; o < H; ++o) col[(R::hid(0) + o) * kRS] = fmaxf(h[o], 0.0f);
        }
        #pragma unroll
        for (int k = 1; k < NH; ++k) {
            float h[H];
            dense_t<H, H>(a.wt + off[k], a.params + off[k] + H * H, col + R::hid(k - 1) * kRS, h);
            #pragma unroll
            for (int o = 0; o < H; ++o) col[(R::hid(k) + o) * kRS] = fmaxf(h[o], 0.0f);
        }
        float qv[NO];
        dense_t<H, NO>(a.wt + off[NH], a.params + off[NH] + H * NO, col + R::hid(NH - 1) * kRS, qv);

        if (MODE == kModeForward) {
            if (in_range) {
                #pragma unroll
                for (int d = 0; d < NO; ++d)
                    a.rgb[NO * (int64_t)i + d] = finite ? softplus_acc(qv[d]) : __builtin_nanf("");
            }
            continue;
        }

        // ---- output deltas: dL/dq = dL/drgb * logistic(q)
        {
            #pragma unroll
            for (int d = 0; d < NO; ++d) {
                float g;
                if (MODE == kModeLoss) {
                    const float e = live ? softplus_acc(qv[d]) - a.target[NO * ic + d] : 0.0f;
                    loss_acc = fmaf(e, e, loss_acc);
                    g = 2.0f * e * a.inv_count;
                } else {
                    g = a.d_rgb[NO * ic + d];
                }
                col[(R::OUT + d) * kRS] = live ? g * logistic(qv[d]) : 0.0f;
            }
            #pragma unroll
            for (int d = NO; d < 8; ++d) col[(R::OUT + d) * kRS] = 0.0f;
        }
        lds_sync_wave();

        // ---- output layer: deltas of the last hidden layer, then its gradient
        {
            float dh[H];
            dense_back<H, NO>(a.params + off[NH], col + R::OUT * kRS, dh);
            #pragma unroll
            for (int j = 0; j < H; ++j) dh[j] = col[(R::hid(NH - 1) + j) * kRS] > 0.0f ? dh[j] : 0.0f;
            layer_grad<H, NO>(lds, R::OUT, R::hid(NH - 1), part + off[NH], part + off[NH] + H * NO, lane);
            lds_sync_wave();
            #pragma unroll
            for (int j = 0; j < H; ++j) col[(R::hid(NH - 1) + j) * kRS] = dh[j];
            lds_sync_wave();
        }
        // ---- hidden layers NH-1 .. 1 (0-based k: layer k+1 maps hidden k-1 -> hidden k)
        #pragma unroll
        for (int k = NH - 1; k >= 1; --k) {
            float dh[H];
            dense_back<H, H>(a.params + off[k], col + R::hid(k) * kRS, dh);
            #pragma unroll
            for (int j = 0; j < H; ++j) dh[j] = col[(R::hid(k - 1) + j) * kRS] > 0.0f ? dh[j] : 0.0f;
            layer_grad<H, H>(lds, R::hid(k), R::hid(k - 1), part + off[k], part + off[k] + H * H, lane);
            lds_sync_wave();
            #pragma unroll
            for (int j = 0; j < H; ++j) col[(R::hid(k - 1) + j) * kRS] = dh[j];
            lds_sync_wave();
        }
        // ---- input layer: the latent-code gradient and the first layer's gradient
        {
            float dx[IN];
            dense_back<IN, H>(a.params + off[0], col + R::hid(0) * kRS, dx);
            layer_grad<IN, H>(lds, R::hid(0), 0, part + off[0], part + off[0] + IN * H, lane);
            if (NF > 0) {
                // through the frame transform into the frame layer and the latent code
                float z[C], draw[6 * (NF > 0 ? NF : 1)];
                #pragma unroll
                for (int cc = 0; cc < C; ++cc) z[cc] = col[cc * kRS];
                const float wi[3] = {a.wi[3 * ic], a.wi[3 * ic + 1], a.wi[3 * ic + 2]};
                const float wo[3] = {a.wo[3 * ic], a.wo[3 * ic + 1], a.wo[3 * ic + 2]};
                const_f32_ptr F = as_constant(a.fparams);
                frame_backward<C, NF>(F, z, wi, wo, dx + C, draw);
                #pragma unroll
                for (int r = 0; r < 6 * NF; ++r) {
                    col[(R::FR + r) * kRS] = draw[r];
                    #pragma unroll
                    for (int cc = 0; cc < C; ++cc) dx[cc] = fmaf(F[r * C + cc], draw[r], dx[cc]);
                }
                lds_sync_wave();
                layer_grad<C, 6 * (NF > 0 ? NF : 1)>(lds, R::FR, 0, fpart, fpart + 6 * NF * C, lane);
            }
            if (a.dz) {
                float m = 0.0f;
                if (in_range) {
                    #pragma unroll
                    for (int cc = 0; cc < C; ++cc) a.dz[(int64_t)i * C + cc] = live ? dx[cc] : 0.0f;
                }
                if (live) {
                    #pragma unroll
                    for (int cc = 0; cc < C; ++cc) m = fmaxf(m, fabsf(dx[cc]));
                    if (!__builtin_isfinite(m)) m = __builtin_inff();
                }
                for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
                if (lane == 0 && m > 0.0f && a.dz_absmax) atomicMax(a.dz_absmax, __float_as_uint(m));
            } else {
                // the code's gradient into the texels, C lanes per sample: in round r, lane
                // (u, c) = (lane / C, lane % C) adds channel c of sample r (64 / C) + u, so one
                // atomic instruction covers 64 / C whole texels (one memory request each)
                // instead of one word of each of 64 texels.  The gradients (rows 0 .. C - 1, a
                // column per sample) and the taps (16 words per sample after them: texel
                // indices, -1 where nothing is added, then the weights) go through LDS rows
                // whose contents are spent.
                static_assert((R::TOTAL - C) * kRS >= 16 * kTW, "scatter exchange rows");
                lds_sync_wave();
                #pragma unroll
                for (int cc = 0; cc < C; ++cc) col[cc * kRS] = dx[cc];
                float* tap = lds + C * kRS + 16 * lane;
                #pragma unroll
                for (int k = 0; k < 8; ++k) {
                    tap[k] = __int_as_float(live && t.w[k] != 0.0f ? (int)t.idx[k] : -1);
                    tap[8 + k] = t.w[k];
                }
                lds_sync_wave();
                constexpr int SPR = 64 / C;
                const int u = lane / C, c = lane % C;
                for (int r = 0; r < C; ++r) {
                    const int q = r * SPR + u;
                    const float d = lds[c * kRS + q];
                    const float* tq = lds + C * kRS + 16 * q;
                    #pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int o = __float_as_int(tq[k]);
                        if (o >= 0) unsafeAtomicAdd(a.d_tex + (int64_t)o * C + c, tq[8 + k] * d);
                    }
                }
            }
            lds_sync_wave();
        }
    }
    if (MODE == kModeLoss) {
        for (int o = 32; o > 0; o >>= 1) loss_acc += __shfl_xor(loss_acc, o, 64);
        if (lane == 0) a.loss_partial[blockIdx.x] = loss_acc;
    }
}

}  // namespace nam
