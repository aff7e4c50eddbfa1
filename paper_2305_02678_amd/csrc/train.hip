// Differentiation of the decode (training by backpropagation into the decoder and directly
// into the latent texels, Sec. 5 and the direct-optimisation alternative of Sec. 2 "Obtaining
// latent textures"), plus Adam.
//
// Layout: the pyramid is one FP32 buffer, levels concatenated (level 0 first), [texel][C];
// parameters are packed W_1[d_1][d_0], b_1, W_2, b_2, ...; gradients use the same layouts.
//
// fwdbwd_kernel: one wave per workgroup, one sample per lane.  The forward pass keeps every
// layer's activations in the lane's own LDS column.  The backward pass walks the layers down:
// the deltas of the layer below are accumulated in registers from wave-uniform weight rows,
// the weight gradient of the layer is the in-LDS product of the wave's 64 deltas and 64
// activations (8 x 8 register tiles per lane), added into the workgroup's own slice of a
// partial-gradient buffer (no atomics; reduced over workgroups in a fixed order afterwards,
// so parameter gradients are deterministic), and the deltas then overwrite the activations
// they no longer need.  The gradient of the latent code is scattered into the 8 trilinear
// taps with FP32 atomic adds.
#include "latent_fetch.h"
#include "train_internal.h"

namespace nam {

constexpr int kTW = 64;                 // lanes per workgroup (one wave)

__device__ __forceinline__ float softplus_acc(float q) { return fmaxf(q, 0.0f) + log1pf(expf(-fabsf(q))); }
__device__ __forceinline__ float logistic(float q) { return 1.0f / (1.0f + expf(-q)); }

// Rows of the LDS activation table: a0 (C + 6 inputs, padded to a multiple of 8), then the
// NH hidden layers (H rows each), then the output deltas (8 rows, NO = 3 or 6 used).  The
// forward-only mode (FWD) keeps no layer for a backward pass, so its hidden layers alternate
// between two blocks: a smaller table, hence more waves per CU.
template <int C, int H, int NH, bool FWD>
struct TrainRows {
    static constexpr int IN = C + 6;
    static constexpr int IN_PAD = (IN + 7) / 8 * 8;
    static constexpr int BLOCKS = FWD ? (NH > 1 ? 2 : 1) : NH;
    static constexpr int hid(int k) { return IN_PAD + (FWD ? (k & 1) : k) * H; }   // hidden layer k (0-based)
    static constexpr int OUT = IN_PAD + BLOCKS * H;
    static constexpr int TOTAL = OUT + 8;
};

// out[o] = bias[o] + sum_j Wt[j][o] * col[j]   (Wt = per-layer transposed weights, uniform)
template <int IN, int OUT>
__device__ __forceinline__ void dense_t(const float* __restrict__ Wt, const float* __restrict__ bias,
                                        const float* col, float* out) {
    #pragma unroll
    for (int o = 0; o < OUT; ++o) out[o] = bias[o];
    #pragma unroll 2
    for (int j = 0; j < IN; ++j) {
        const float aj = col[j * kTW];
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
        const float d = dcol[o * kTW];
        const float* wo = W + o * IN;
        #pragma unroll
        for (int j = 0; j < IN; ++j) d_in[j] = fmaf(wo[j], d, d_in[j]);
    }
}

// Weight and bias gradient of one layer over the wave's 64 samples, added into the
// workgroup's partial slice: gW[o][j] += sum_s delta[o][s] * act[j][s], gb[o] += sum_s delta[o][s].
// delta rows start at `drow`, activation rows at `arow` (FO_PAD x 64 and FI_PAD x 64 floats).
template <int FI, int FO>
__device__ __forceinline__ void layer_grad(const float* lds, int drow, int arow, float* __restrict__ gW,
                                           float* __restrict__ gb, int lane) {
    constexpr int FI_PAD = (FI + 7) / 8 * 8, FO_PAD = (FO + 7) / 8 * 8;
    constexpr int TJ = FI_PAD / 8, TILES = (FO_PAD / 8) * TJ;
    static_assert(TILES <= kTW, "one 8x8 tile per lane");
    if (lane < TILES) {
        const int to = lane / TJ, tj = lane % TJ;
        float acc[8][8];
        #pragma unroll
        for (int a = 0; a < 8; ++a)
            #pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = 0.0f;
        for (int s = 0; s < kTW; ++s) {
            float dv[8], av[8];
            #pragma unroll
            for (int a = 0; a < 8; ++a) dv[a] = lds[(drow + to * 8 + a) * kTW + s];
            #pragma unroll
            for (int b = 0; b < 8; ++b) av[b] = lds[(arow + tj * 8 + b) * kTW + s];
            #pragma unroll
            for (int a = 0; a < 8; ++a)
                #pragma unroll
                for (int b = 0; b < 8; ++b) acc[a][b] = fmaf(dv[a], av[b], acc[a][b]);
        }
        #pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int o = to * 8 + a;
            #pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int j = tj * 8 + b;
                if (o < FO && j < FI) gW[o * FI + j] += acc[a][b];
            }
        }
    }
    if (lane < FO) {
        float s = 0.0f;
        for (int t = 0; t < kTW; ++t) s += lds[(drow + lane) * kTW + t];
        gb[lane] += s;
    }
}

// NO: decoder outputs, 3 (RGB) or 6 (RGB, then the albedo triplet); outputs, targets and
// output gradients are [n][NO].
template <int C, int H, int NH, int NO, int MODE>
__global__ void __launch_bounds__(kTW) fwdbwd_kernel(const TrainArgs a) {
    using R = TrainRows<C, H, NH, MODE == kModeForward>;
    constexpr int IN = R::IN;
    __shared__ float lds[R::TOTAL * kTW];
    __shared__ LevelRow lrows[kMaxLevels];
    const int lane = threadIdx.x;
    if (lane < a.M) lrows[lane] = a.rows[lane];
    float* col = lds + lane;

    // this workgroup's partial gradient slice (zeroed here, accumulated over its chunks)
    float* part = a.partial ? a.partial + (size_t)blockIdx.x * a.np : nullptr;
    if (MODE != kModeForward) {
        for (int p = lane; p < a.np; p += kTW) part[p] = 0.0f;
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

        // ---- fetch (a non-finite query decodes to NaN and contributes no gradient)
        Taps t;
        const float2 q = reinterpret_cast<const float2*>(a.uv)[ic];
        const bool finite = query_ok(q.x, q.y, a.lod[ic]);
        const bool live = in_range && finite;
        query_taps_rows(lrows, a.M, a.address, q.x, q.y, a.lod[ic], t);
        {
            float z[C];
            gather_f32<C>(a.tex, t, z);
            #pragma unroll
            for (int cc = 0; cc < C; ++cc) col[cc * kTW] = finite ? z[cc] : 0.0f;
            #pragma unroll
            for (int d = 0; d < 3; ++d) {
                col[(C + d) * kTW] = a.wi[3 * ic + d];
                col[(C + 3 + d) * kTW] = a.wo[3 * ic + d];
            }
            #pragma unroll
            for (int r = IN; r < R::IN_PAD; ++r) col[r * kTW] = 0.0f;
        }

        // ---- forward, keeping every layer's activations
        {
            float h[H];
            dense_t<IN, H>(a.wt + off[0], a.params + off[0] + IN * H, col, h);
            #pragma unroll
            for (int o = 0; o < H; ++o) col[(R::hid(0) + o) * kTW] = fmaxf(h[o], 0.0f);
        }
        #pragma unroll
        for (int k = 1; k < NH; ++k) {
            float h[H];
            dense_t<H, H>(a.wt + off[k], a.params + off[k] + H * H, col + R::hid(k - 1) * kTW, h);
            #pragma unroll
            for (int o = 0; o < H; ++o) col[(R::hid(k) + o) * kTW] = fmaxf(h[o], 0.0f);
        }
        float qv[NO];
        dense_t<H, NO>(a.wt + off[NH], a.params + off[NH] + H * NO, col + R::hid(NH - 1) * kTW, qv);

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
                col[(R::OUT + d) * kTW] = live ? g * logistic(qv[d]) : 0.0f;
            }
            #pragma unroll
            for (int d = NO; d < 8; ++d) col[(R::OUT + d) * kTW] = 0.0f;
        }
        lds_sync_wave();

        // ---- output layer: deltas of the last hidden layer, then its gradient
        {
            float dh[H];
            dense_back<H, NO>(a.params + off[NH], col + R::OUT * kTW, dh);
            #pragma unroll
            for (int j = 0; j < H; ++j) dh[j] = col[(R::hid(NH - 1) + j) * kTW] > 0.0f ? dh[j] : 0.0f;
            layer_grad<H, NO>(lds, R::OUT, R::hid(NH - 1), part + off[NH], part + off[NH] + H * NO, lane);
            lds_sync_wave();
            #pragma unroll
            for (int j = 0; j < H; ++j) col[(R::hid(NH - 1) + j) * kTW] = dh[j];
            lds_sync_wave();
        }
        // ---- hidden layers NH-1 .. 1 (0-based k: layer k+1 maps hidden k-1 -> hidden k)
        #pragma unroll
        for (int k = NH - 1; k >= 1; --k) {
            float dh[H];
            dense_back<H, H>(a.params + off[k], col + R::hid(k) * kTW, dh);
            #pragma unroll
            for (int j = 0; j < H; ++j) dh[j] = col[(R::hid(k - 1) + j) * kTW] > 0.0f ? dh[j] : 0.0f;
            layer_grad<H, H>(lds, R::hid(k), R::hid(k - 1), part + off[k], part + off[k] + H * H, lane);
            lds_sync_wave();
            #pragma unroll
            for (int j = 0; j < H; ++j) col[(R::hid(k - 1) + j) * kTW] = dh[j];
            lds_sync_wave();
        }
        // ---- input layer: the latent-code gradient and the first layer's gradient
        {
            float dx[IN];
            dense_back<IN, H>(a.params + off[0], col + R::hid(0) * kTW, dx);
            layer_grad<IN, H>(lds, R::hid(0), 0, part + off[0], part + off[0] + IN * H, lane);
            if (live) {
                #pragma unroll
                for (int k = 0; k < 8; ++k) {
                    float* g = a.d_tex + t.idx[k] * C;
                    const float w = t.w[k];
                    if (w != 0.0f) {
                        #pragma unroll
                        for (int cc = 0; cc < C; ++cc) unsafeAtomicAdd(g + cc, w * dx[cc]);
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

// d_params[p] = sum over workgroups of partial[b][p], in workgroup order (deterministic).
__global__ void __launch_bounds__(256) reduce_partials_kernel(const float* __restrict__ partial, int blocks, int np,
                                                              float* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float s = 0.0f;
    for (int b = 0; b < blocks; ++b) s += partial[(size_t)b * np + p];
    out[p] = s;
}

// loss = inv_count * sum of the per-workgroup squared-error sums (one wave, fixed order).
__global__ void __launch_bounds__(64) reduce_loss_kernel(const float* __restrict__ part, int blocks, float inv_count,
                                                         float* __restrict__ loss) {
    float s = 0.0f;
    for (int b = threadIdx.x; b < blocks; b += 64) s += part[b];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) *loss = s * inv_count;
}

// Per layer W^T [in][out] followed by the bias, for the wave-uniform forward reads.
__global__ void __launch_bounds__(256) transpose_params_kernel(const float* __restrict__ p, float* __restrict__ wt,
                                                               LayerDims L) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L.total) return;
    int k = 0;
    while (k + 1 < L.n_layers && idx >= L.off[k + 1]) ++k;
    const int local = idx - L.off[k];
    const int fi = L.in[k], fo = L.out[k];
    if (local < fi * fo) {
        const int o = local / fi, j = local % fi;      // source W[o][j]
        wt[L.off[k] + j * fo + o] = p[idx];
    } else {
        wt[idx] = p[idx];                              // bias
    }
}

// Adam (step counted from 1), element-wise; c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void __launch_bounds__(256) adam_kernel(int64_t count, float* __restrict__ p, float* __restrict__ m,
                                                   float* __restrict__ v, const float* __restrict__ g, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

template <int C, int H, int NH, int MODE>
static hipError_t launch_fb_shape(const MlpShape& sh, const TrainArgs& a, int grid, hipStream_t s) {
    clear_stale_hip_error();
    if (sh.NO == 6) fwdbwd_kernel<C, H, NH, 6, MODE><<<grid, kTW, 0, s>>>(a);
    else fwdbwd_kernel<C, H, NH, 3, MODE><<<grid, kTW, 0, s>>>(a);
    return hipGetLastError();
}

template <int MODE>
static hipError_t dispatch_fb(const MlpShape& sh, const TrainArgs& a, int grid, hipStream_t s) {
#define NAM_T_CASE(C_, H_, NH_) \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_) return launch_fb_shape<C_, H_, NH_, MODE>(sh, a, grid, s);
#define NAM_T_H(C_, H_) NAM_T_CASE(C_, H_, 1) NAM_T_CASE(C_, H_, 2) NAM_T_CASE(C_, H_, 3) NAM_T_CASE(C_, H_, 4)
    NAM_T_H(8, 16) NAM_T_H(8, 32) NAM_T_H(8, 64)
    NAM_T_H(16, 16) NAM_T_H(16, 32) NAM_T_H(16, 64)
#undef NAM_T_H
#undef NAM_T_CASE
    return hipErrorInvalidValue;
}

template <int MODE>
static int occupancy_fb(const MlpShape& sh) {
    int b = 0;
#define NAM_O_CASE(C_, H_, NH_) \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_)                                                            \
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                  \
            &b, sh.NO == 6 ? (const void*)fwdbwd_kernel<C_, H_, NH_, 6, MODE> : (const void*)fwdbwd_kernel<C_, H_, NH_, 3, MODE>, \
            kTW, 0);
#define NAM_O_H(C_, H_) NAM_O_CASE(C_, H_, 1) NAM_O_CASE(C_, H_, 2) NAM_O_CASE(C_, H_, 3) NAM_O_CASE(C_, H_, 4)
    NAM_O_H(8, 16) NAM_O_H(8, 32) NAM_O_H(8, 64)
    NAM_O_H(16, 16) NAM_O_H(16, 32) NAM_O_H(16, 64)
#undef NAM_O_H
#undef NAM_O_CASE
    return b < 1 ? 1 : b;
}

int fwdbwd_blocks_per_cu(const MlpShape& sh, int mode) {
    if (mode == kModeForward) return occupancy_fb<kModeForward>(sh);
    if (mode == kModeLoss) return occupancy_fb<kModeLoss>(sh);
    return occupancy_fb<kModeGrad>(sh);
}

hipError_t launch_fwdbwd(const MlpShape& sh, int mode, const TrainArgs& a, int grid, hipStream_t s) {
    if (mode == kModeForward) return dispatch_fb<kModeForward>(sh, a, grid, s);
    if (mode == kModeLoss) return dispatch_fb<kModeLoss>(sh, a, grid, s);
    return dispatch_fb<kModeGrad>(sh, a, grid, s);
}

hipError_t launch_reduce_partials(const float* partial, int blocks, int np, float* out, hipStream_t s) {
    clear_stale_hip_error();
    reduce_partials_kernel<<<(np + 255) / 256, 256, 0, s>>>(partial, blocks, np, out);
    return hipGetLastError();
}

hipError_t launch_reduce_loss(const float* part, int blocks, float inv_count, float* loss, hipStream_t s) {
    clear_stale_hip_error();
    reduce_loss_kernel<<<1, 64, 0, s>>>(part, blocks, inv_count, loss);
    return hipGetLastError();
}

hipError_t launch_transpose_params(const float* p, float* wt, const LayerDims& L, hipStream_t s) {
    clear_stale_hip_error();
    transpose_params_kernel<<<(L.total + 255) / 256, 256, 0, s>>>(p, wt, L);
    return hipGetLastError();
}

hipError_t launch_adam(int64_t count, float* p, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    clear_stale_hip_error();
    adam_kernel<<<(int)blocks, 256, 0, s>>>(count, p, m, v, g, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace nam
