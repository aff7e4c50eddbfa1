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
#include "train_vec.h"

namespace nam {

__global__ void __launch_bounds__(256) zero_kernel(uint4* __restrict__ p, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

// Fixed-point scale of the deterministic scatter: every sample's taps carry weights summing to
// at most 1, so a texel's gradient is bounded by n * max|dz| < 2^e; contributions are scaled by
// 2^(62 - e), rounded to integers and summed in 64-bit two's complement, which is associative,
// so the sum is the same in any order.  Returns false when there is nothing to add (max 0) and
// sets *exact = false when the gradients are not finite (then plain float atomics are used).
__device__ __forceinline__ bool det_shift(const unsigned int* absmax, int n, int* shift, bool* exact) {
    const float m = __uint_as_float(*absmax);
    *exact = __builtin_isfinite(m);
    if (!(m > 0.0f)) return false;
    if (!*exact) return true;
    int e;
    (void)frexp((double)m * (double)n, &e);
    *shift = 62 - e;
    return true;
}

// C threads per sample: thread (i, c) adds channel c of sample i at its 8 taps, so one atomic
// instruction of a wave covers 64 / C whole texels (one memory request each).
template <int C>
__global__ void __launch_bounds__(256) det_scatter_kernel(const LevelRow* __restrict__ rows, int M, int address, int n,
                                                          const float* __restrict__ uv, const float* __restrict__ lod,
                                                          const float* __restrict__ dz,
                                                          const unsigned int* __restrict__ absmax,
                                                          long long* __restrict__ acc, float* __restrict__ d_tex) {
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i = gt / C;
    const int c = (int)(gt % C);
    if (i >= n) return;
    int shift = 0;
    bool exact = true;
    if (!det_shift(absmax, n, &shift, &exact)) return;
    const float2 q = reinterpret_cast<const float2*>(uv)[i];
    const float l = lod[i];
    if (!query_ok(q.x, q.y, l)) return;
    Taps t;
    query_taps_rows(rows, M, address, q.x, q.y, l, t);
    const float d = dz[i * C + c];
    #pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float w = t.w[k];
        if (w == 0.0f) continue;
        if (exact) {
            // the product of two floats is exact in double; scaling by 2^shift is exact too
            const long long v = __double2ll_rn(ldexp((double)w * (double)d, shift));
            atomicAdd(reinterpret_cast<unsigned long long*>(acc + t.idx[k] * C + c), (unsigned long long)v);
        } else {
            unsafeAtomicAdd(d_tex + t.idx[k] * C + c, w * d);
        }
    }
}

__global__ void __launch_bounds__(256) det_finish_kernel(int64_t count, const long long* __restrict__ acc,
                                                         const unsigned int* __restrict__ absmax, int n,
                                                         float* __restrict__ d_tex) {
    int shift = 0;
    bool exact = true;
    if (!det_shift(absmax, n, &shift, &exact) || !exact) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        d_tex[i] += (float)ldexp((double)acc[i], -shift);
}

// d_params[p] = sum over slices of partial[b][p] as a fixed two-level tree (deterministic):
// the first pass sums each group of kReduceGroup consecutive slices in slice order and leaves
// the result in place of the group's first slice (one thread owns a (group, parameter) pair);
// the second sums the groups in group order.
constexpr int kReduceGroup = 16;

__global__ void __launch_bounds__(256) reduce_groups_kernel(float* __restrict__ partial, int blocks, int np) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int b0 = blockIdx.y * kReduceGroup;
    const int b1 = min(b0 + kReduceGroup, blocks);
    float v[kReduceGroup];
    #pragma unroll
    for (int i = 0; i < kReduceGroup; ++i) v[i] = b0 + i < b1 ? partial[(size_t)(b0 + i) * np + p] : 0.0f;
    float s = v[0];
    #pragma unroll
    for (int i = 1; i < kReduceGroup; ++i) s += v[i];
    partial[(size_t)b0 * np + p] = s;
}

__global__ void __launch_bounds__(256) reduce_partials_kernel(const float* __restrict__ partial, int blocks, int np,
                                                              float* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float s = 0.0f;
    for (int b = 0; b < blocks; b += kReduceGroup) s += partial[(size_t)b * np + p];
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
    if (sh.NF > 0) return fwdbwd_frames_blocks_per_cu(sh, mode);
    if (mode == kModeForward) return occupancy_fb<kModeForward>(sh);
    if (mode == kModeLoss) return occupancy_fb<kModeLoss>(sh);
    return occupancy_fb<kModeGrad>(sh);
}

hipError_t launch_fwdbwd(const MlpShape& sh, int mode, const TrainArgs& a, int grid, hipStream_t s) {
    if (sh.NF > 0) return launch_fwdbwd_frames(sh, mode, a, grid, s);
    if (mode == kModeForward) return dispatch_fb<kModeForward>(sh, a, grid, s);
    if (mode == kModeLoss) return dispatch_fb<kModeLoss>(sh, a, grid, s);
    return dispatch_fb<kModeGrad>(sh, a, grid, s);
}

__global__ void __launch_bounds__(256) fill_f32_kernel(float* __restrict__ p, int64_t count, float v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Row l: the level's width and height (max(1, side >> l)) and its first texel in the
// concatenated pyramid.
__global__ void __launch_bounds__(64) level_rows_kernel(int W, int H, int M, LevelRow* __restrict__ rows) {
    const int l = threadIdx.x;
    if (l >= M) return;
    int64_t off = 0;
    for (int k = 0; k < l; ++k) off += (int64_t)max(1, W >> k) * max(1, H >> k);
    rows[l] = LevelRow{max(1, W >> l), max(1, H >> l), off};
}

hipError_t launch_fill_f32(float* p, int64_t count, float v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    clear_stale_hip_error();
    fill_f32_kernel<<<(int)blocks, 256, 0, s>>>(p, count, v);
    return hipGetLastError();
}

hipError_t launch_level_rows(int width, int height, int levels, LevelRow* rows, hipStream_t s) {
    clear_stale_hip_error();
    level_rows_kernel<<<1, 64, 0, s>>>(width, height, levels, rows);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t count = (int64_t)(bytes / 16);
    if (count == 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    clear_stale_hip_error();
    zero_kernel<<<(int)blocks, 256, 0, s>>>(static_cast<uint4*>(p), count);
    return hipGetLastError();
}

hipError_t launch_det_scatter(const LevelRow* rows, int M, int address, int C, int n, const float* uv, const float* lod,
                              const float* dz, const unsigned int* absmax, long long* acc, float* d_tex, hipStream_t s) {
    const int blocks = (int)(((int64_t)n * C + 255) / 256);     // C threads per sample
    if (blocks == 0) return hipSuccess;
    clear_stale_hip_error();
    if (C == 8) det_scatter_kernel<8><<<blocks, 256, 0, s>>>(rows, M, address, n, uv, lod, dz, absmax, acc, d_tex);
    else if (C == 16) det_scatter_kernel<16><<<blocks, 256, 0, s>>>(rows, M, address, n, uv, lod, dz, absmax, acc, d_tex);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_det_finish(int64_t count, const long long* acc, const unsigned int* absmax, int n, float* d_tex,
                             hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) return hipSuccess;
    clear_stale_hip_error();
    det_finish_kernel<<<(int)blocks, 256, 0, s>>>(count, acc, absmax, n, d_tex);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(float* partial, int blocks, int np, float* out, hipStream_t s) {
    if (np < 1 || blocks < 1) return hipSuccess;
    clear_stale_hip_error();
    const int groups = (blocks + kReduceGroup - 1) / kReduceGroup;
    reduce_groups_kernel<<<dim3((np + 255) / 256, groups), 256, 0, s>>>(partial, blocks, np);
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
