// Low-precision decode on the gfx950 matrix cores: one fused, persistent kernel per material
// precision (FP16 weights and activations; OCP E4M3 weights and activations with one scale per
// layer; E4M3 with the first layer kept in FP16).  Accumulation is FP32 throughout, the bias is
// added in FP32 (as the accumulator's initial value) and softplus is evaluated in FP32.
//
// Work decomposition.  A workgroup of 8 waves handles chunks of 256 consecutive queries, with
// two roles that meet at one barrier per chunk through a double-buffered LDS input block:
//   fetch waves (0-3)    each lane fetches one query: 8 trilinear taps of FP16 texels (16-byte
//                        loads), blended in FP32, applies the learned shading frames if the
//                        material has them (FP32), and writes the network input
//                        [z, T wi, T wo, 0...] (32 slots) to LDS in the lane order of the
//                        matrix-core B operand;
//   decoder waves (4-7)  each evaluates the decoder for 4 tiles of 16 queries: a layer is
//                        Y^T = W Y_prev^T with the weights as the A operand (one 16-neuron row
//                        tile per instruction, v_mfma_f32_16x16x32_{f16,fp8}) and one query per
//                        column.
// The accumulator of a row tile leaves lane (g, q) = (lane / 16, lane % 16) holding neurons
// 4g..4g+3 of query q; the next layer's B operand needs 8 consecutive K slots per lane, so
// the K order of every hidden layer's weights is permuted at load time to slot
// (s, g, e) <-> neuron 16 (2s + e / 4) + 4g + e % 4: two accumulator tiles, ReLU'd and
// converted, are exactly the next B operand, with no shuffle or LDS round trip.  The output
// layer of tile t uses a copy of its weights moved to rows 4t..4t+2, and the wave's 4 tiles
// accumulate into one tile: lane (g, q) ends with the RGB of query 16 g + q of the wave, which
// it stores directly (12 contiguous bytes per lane).  A decoder with the albedo head (6
// outputs: RGB, then the directional albedo of Eq. albedo, Sec. 6.5) instead puts a tile's six
// rows at rows 0..5 or 8..13 of the accumulator of its tile pair, so the output layer costs the
// same number of matrix-core instructions; two lanes then store a query's 24 bytes.
// All weights and biases of the decoder stay in registers for the whole kernel.  The grid is
// persistent; chunks are split into one contiguous range per XCD (workgroups are dispatched
// round-robin over the 8 XCDs), so neighbouring screen tiles, which share texels, are decoded
// under the same L2.
#pragma once

#include <algorithm>

#include "latent_fetch.h"
#include "frames.h"
#include "mfma_pack.h"

namespace nam {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 512;           // lanes per workgroup: 4 fetch waves + 4 decoder waves
constexpr int kChunk = 256;           // queries per chunk (one per fetch lane)

struct MfmaArgs {
    PyrArgs pyr;
    const __half* tex;        // FP16 texels
    const uint4* w;           // packed A operands, see mfma_pack.h
    const floatx4* bias;      // per (layer, row tile, lane): 4 biases (pre-scaled for E4M3)
    float in_hi, in_inv;      // E4M3 network input: clamp bound 448 / s and 1 / s for its scale s
    float mid_hi[kMaxLayers];      // from layer k's accumulator to layer k+1's E4M3 input (a power
    float mid_inv[kMaxLayers];     // of two m): clamp bound 448 / m and 1 / m
    float out_scale;          // from the output accumulator to q
    int n;
    int nchunks;
    int groups;               // XCD groups: min(8, grid); the grid is a multiple of it
    const float2* uv;
    const float* lod;
    const float* xi;          // per-query draws of the Russian-roulette level choice (RR kernels)
    const float* wi;
    const float* wo;
    float* rgb;
    const uint32_t* frames16; // learned shading frames: W_F[6 nf][C / 2] as FP16 pairs, then b_F[6 nf] (FP32)
    int nf;                   // number of frames (0: T is the identity)
};

// softplus(q) = max(q, 0) + log1p(exp(-|q|)) in FP32 on the hardware exp2/log2: log1p(e) is
// taken as log(1 + e) * e / ((1 + e) - 1), Kahan's correction of the rounding of 1 + e (exact
// to a few ulp for every e in (0, 1]; e itself when 1 + e rounds to 1).  exp(-|q|) underflows
// to 0 for |q| > 87, where softplus(q) = max(q, 0) in FP32 anyway.
__device__ __forceinline__ float softplus_fast(float q) {
    const float e = __builtin_amdgcn_exp2f(-fabsf(q) * 1.44269504088896341f);
    const float u = 1.0f + e;
    const float d = u - 1.0f;
    const float l = d == 0.0f ? e : (__builtin_amdgcn_logf(u) * 0.693147180559945309f) * (e * __builtin_amdgcn_rcpf(d));
    return fmaxf(q, 0.0f) + l;
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// ReLU of two FP32 accumulators, rounded to FP16 (convert, then a packed max: rounding keeps
// the sign, so the order does not matter).
__device__ __forceinline__ half2_t relu_pack_f16(float a, float b) {
    half2_t h = {(_Float16)a, (_Float16)b};
    const half2_t z = {(_Float16)0.0f, (_Float16)0.0f};
    return __builtin_elementwise_max(h, z);
}

__device__ __forceinline__ floatx4 mfma_f16(const half8 a, const half8 b, const floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ floatx4 mfma_fp8(const long a, const long b, const floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
}

typedef short short2_t __attribute__((ext_vector_type(2)));

// E4M3 bytes of x * m for four values, m a power of two given as inv = 1 / m and the clamp
// bounds [lo, hi] in units of x (hi = 448 / m; lo = 0 gives the ReLU, lo = -hi a symmetric
// clamp).  The clamp comes first because the conversion turns values past 448 into NaN; the
// conversion then scales by the exponent of inv and rounds to nearest even, which for a power
// of two is exactly E4M3(clamp(x, lo, hi) * m).
__device__ __forceinline__ uint32_t scaled_fp8x4(float a, float b, float c, float d, float lo, float hi, float inv) {
    a = __builtin_amdgcn_fmed3f(a, lo, hi);
    b = __builtin_amdgcn_fmed3f(b, lo, hi);
    c = __builtin_amdgcn_fmed3f(c, lo, hi);
    d = __builtin_amdgcn_fmed3f(d, lo, hi);
    // the first conversion fills the low half-word and the second the high one, so the initial
    // contents of the word do not matter
    const short2_t any = __builtin_nondeterministic_value(short2_t{});
    short2_t r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(any, a, b, inv, false);
    r = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(r, c, d, inv, true);
    return __builtin_bit_cast(uint32_t, r);
}

// Texel words of one query's NT taps in flight (C / 8 16-byte words per tap) and the tap weights:
// 8 taps for trilinear filtering, 4 with the level chosen by Russian roulette.
template <int C, int NT>
struct TapLoads {
    uint4 v[NT][C / 8];
    float w[NT];
};

// One pyramid level in LDS for the matrix-core decode.  The FP16 pyramid is below 4 GiB (checked
// when the precision is set), so texel addresses are 32-bit byte offsets from the pyramid base.
struct LevelRowL {
    float wf, hf;        // texels along x and y
    int32_t wm, hm;      // the same minus one: wrap mask, or clamp bound
    uint32_t offb;       // byte offset of the level's first texel
    uint32_t pitchb;     // bytes per row
    int32_t pad0, pad1;
};

// Taps along one axis, the same arithmetic as the generic filter (fraction taken from the
// exact p = c W, half-texel shift applied to the fraction).  Under wrap addressing c has
// already dropped whole periods when |c| >= 256.
template <int ADDR>
__device__ __forceinline__ void axis32(float c, float W, int wm, int& x0, int& x1, float& a) {
    float p;
    if constexpr (ADDR == NAM_WRAP) p = c * W;
    else p = fminf(fmaxf(c * W, -1.5f), W + 1.5f);
    const float fp = floorf(p);
    const float fr = p - fp;
    const bool hi = fr >= 0.5f;
    a = fr + (hi ? -0.5f : 0.5f);
    const int i = (int)fp - (hi ? 0 : 1);
    if constexpr (ADDR == NAM_WRAP) {
        x0 = i & wm;
        x1 = (i + 1) & wm;
    } else {
        x0 = min(max(i, 0), wm);
        x1 = min(max(i + 1, 0), wm);
    }
}

// Bilinear stencil of one level as byte offsets of the 4 texels (C FP16 channels each); weights
// scaled by the level weight.
template <int C, int ADDR>
__device__ __forceinline__ void level_stencil32(const LevelRowL& row, float u, float v, uint32_t* off, float* w,
                                                float scale) {
    constexpr int kShift = C == 16 ? 5 : 4;      // log2 of the texel size in bytes
    int x0, x1, y0, y1;
    float ax, by;
    axis32<ADDR>(u, row.wf, row.wm, x0, x1, ax);
    axis32<ADDR>(v, row.hf, row.hm, y0, y1, by);
    const uint32_t r0 = row.offb + __umul24((uint32_t)y0, row.pitchb);   // y < 2^15, pitch < 2^20
    const uint32_t r1 = row.offb + __umul24((uint32_t)y1, row.pitchb);
    const uint32_t c0 = (uint32_t)x0 << kShift, c1 = (uint32_t)x1 << kShift;
    off[0] = r0 + c0;
    off[1] = r0 + c1;
    off[2] = r1 + c0;
    off[3] = r1 + c1;
    const float wa0 = (1.0f - ax) * scale, wa1 = ax * scale;
    w[0] = wa0 * (1.0f - by);
    w[1] = wa1 * (1.0f - by);
    w[2] = wa0 * by;
    w[3] = wa1 * by;
}

// Addresses and loads of one query's taps (issued, not awaited).  Trilinear: both levels, 8
// taps.  RR: the coarser level iff the draw xi < t (t the fractional part of the clamped level,
// exact in FP32; a NaN draw takes the finer level), 4 bilinear taps at full weight (Sec. 4.1).
// A non-finite query filters at (0, 0, 0), so every load stays inside the pyramid; its result
// is replaced by NaN (non-finite) or dropped (past the end of the batch) through the per-query
// flag, so the weights need no special value.
template <int C, int ADDR, bool RR>
__device__ __forceinline__ void issue_taps(const MfmaArgs& a, const LevelRowL* rows, bool use, float u, float v,
                                           float l, float xi, TapLoads<C, RR ? 4 : 8>& tl) {
    constexpr int NT = RR ? 4 : 8;
    u = use ? u : 0.0f;
    v = use ? v : 0.0f;
    l = use ? l : 0.0f;
    if constexpr (ADDR == NAM_WRAP) {      // drop whole periods once for both levels
        u = fabsf(u) < 256.0f ? u : u - floorf(u);
        v = fabsf(v) < 256.0f ? v : v - floorf(v);
    }
    const float lam = __builtin_amdgcn_fmed3f(l, 0.0f, (float)(a.pyr.M - 1));   // l is finite here
    const int l0 = (int)lam;
    const int l1 = min(l0 + 1, a.pyr.M - 1);
    const float tt = lam - (float)l0;
    uint32_t off[NT];
    if constexpr (RR) {
        level_stencil32<C, ADDR>(rows[xi < tt ? l1 : l0], u, v, off, tl.w, 1.0f);
    } else {
        level_stencil32<C, ADDR>(rows[l0], u, v, off, tl.w, 1.0f - tt);
        level_stencil32<C, ADDR>(rows[l1], u, v, off + 4, tl.w + 4, tt);
    }
    const uint8_t* tex = reinterpret_cast<const uint8_t*>(a.tex);
    #pragma unroll
    for (int k = 0; k < NT; ++k) {
        const uint4* p = reinterpret_cast<const uint4*>(tex + off[k]);
        #pragma unroll
        for (int c8 = 0; c8 < C / 8; ++c8) tl.v[k][c8] = p[c8];
    }
}

// z = sum_k w_k T_k with FP16 texels widened to FP32 (one mixed-precision FMA per channel).
template <int C, int NT>
__device__ __forceinline__ void blend_taps(const TapLoads<C, NT>& tl, float* z) {
    #pragma unroll
    for (int c = 0; c < C; ++c) z[c] = 0.0f;
    #pragma unroll
    for (int k = 0; k < NT; ++k)
        #pragma unroll
        for (int c8 = 0; c8 < C / 8; ++c8) {
            const uint32_t words[4] = {tl.v[k][c8].x, tl.v[k][c8].y, tl.v[k][c8].z, tl.v[k][c8].w};
            #pragma unroll
            for (int h = 0; h < 4; ++h) {
                const half2_t pair = __builtin_bit_cast(half2_t, words[h]);
                z[8 * c8 + 2 * h] = fmaf(tl.w[k], (float)pair[0], z[8 * c8 + 2 * h]);
                z[8 * c8 + 2 * h + 1] = fmaf(tl.w[k], (float)pair[1], z[8 * c8 + 2 * h + 1]);
            }
        }
}

// Network input of one query in the B-operand layout of layer 0: slot 8 g + e of query q of a
// 16-query tile goes to lane (g, q).  FP16: 16 bytes per lane; E4M3: 8 bytes per lane.
template <int C, bool L1F16>
__device__ __forceinline__ void write_input(uint8_t* xb, int qi, const float* x, float in_hi, float in_inv) {
    const int tile = qi >> 4, q = qi & 15;
    if constexpr (L1F16) {
        #pragma unroll
        for (int g = 0; g < 4; ++g) {
            half8 h;
            #pragma unroll
            for (int e = 0; e < 8; e += 2) {
                const half2_t p = {(_Float16)x[8 * g + e], (_Float16)x[8 * g + e + 1]};
                h[e] = p[0];
                h[e + 1] = p[1];
            }
            *reinterpret_cast<half8*>(xb + ((tile * 4 + g) * 16 + q) * 16) = h;
        }
    } else {
        #pragma unroll
        for (int g = 0; g < 4; ++g) {
            uint2 v;
            v.x = scaled_fp8x4(x[8 * g], x[8 * g + 1], x[8 * g + 2], x[8 * g + 3], -in_hi, in_hi, in_inv);
            v.y = scaled_fp8x4(x[8 * g + 4], x[8 * g + 5], x[8 * g + 6], x[8 * g + 7], -in_hi, in_hi, in_inv);
            *reinterpret_cast<uint2*>(xb + ((tile * 4 + g) * 16 + q) * 8) = v;
        }
    }
}

// One query of the fetch pipeline: its taps in flight, its directions and whether it is finite.
template <int C, bool RR>
struct FetchSlot {
    TapLoads<C, RR ? 4 : 8> tl;
    float dir[6];
    bool ok;
};

// Element of query qi of chunk c of a per-query array, clamped to the last query of the batch
// (loads past the end read valid memory and are never used).  The chunk base is uniform and
// the lane offset 32-bit, so the address is a scalar base plus a vector offset.
template <int W, typename T>
__device__ __forceinline__ const T* chunk_elem(const T* arr, int n, int c, int qi) {
    const int first = min(c * kChunk, n - 1);              // uniform; n < 2^31 and c * 256 < 2^31
    const int last = min(n - 1 - first, kChunk - 1);       // uniform
    const uint32_t off = __umul24((uint32_t)min(qi, last), (uint32_t)(W * sizeof(T)));
    return reinterpret_cast<const T*>(reinterpret_cast<const uint8_t*>(arr + (int64_t)W * first) + off);
}

// Issues chunk cn's loads for query qi of the chunk (taps and directions) from its uv / lod.
template <int C, int ADDR, bool RR>
__device__ __forceinline__ void fetch_issue(const MfmaArgs& a, const LevelRowL* rows, int cn, int qi, float2 uv,
                                            float lod, float xi, FetchSlot<C, RR>& fs) {
    const int room = min(max(a.n - cn * kChunk, 0), kChunk);   // uniform
    const bool live = qi < room;
    const bool ok = query_ok(uv.x, uv.y, lod);
    fs.ok = live && ok;
    issue_taps<C, ADDR, RR>(a, rows, ok, uv.x, uv.y, lod, xi, fs.tl);
    const float* wi = chunk_elem<3>(a.wi, a.n, cn, qi);
    const float* wo = chunk_elem<3>(a.wo, a.n, cn, qi);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
        fs.dir[d] = wi[d];
        fs.dir[3 + d] = wo[d];
    }
}

template <int C, bool L1F16, bool RR, bool FR>
__device__ __forceinline__ void fetch_finish(const MfmaArgs& a, const FetchSlot<C, RR>& fs, uint8_t* xb, uint8_t* okb,
                                             int qi) {
    float x[32];
    #pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = 0.0f;
    blend_taps<C, RR ? 4 : 8>(fs.tl, x);
    // the frame transform (weights wave-uniform) writes [T wi, T wo] after z
    if constexpr (FR) {
        const_u32_ptr wh = as_constant_u32(a.frames16);
        const_f32_ptr fb = as_constant(reinterpret_cast<const float*>(a.frames16 + 3 * a.nf * C));
        if (a.nf == 2) frame_inputs_f16<C, 2>(wh, fb, x, fs.dir, fs.dir + 3, x + C);
        else frame_inputs_f16<C, 1>(wh, fb, x, fs.dir, fs.dir + 3, x + C);
    } else {
        #pragma unroll
        for (int d = 0; d < 6; ++d) x[C + d] = fs.dir[d];
    }
    okb[qi] = fs.ok;
    write_input<C, L1F16>(xb, qi, x, a.in_hi, a.in_inv);
}

// One chunk of a fetch wave: issues the taps of chunk c + stride into `next`, then blends the
// taps of chunk c (already in flight in `done`) into the LDS input block.  The memory counter
// retires loads in issue order, so a wait for one load also waits for everything issued before
// it; hence uv / lod run two chunks ahead and are issued before the taps of the chunk after c
// (waiting for them never waits for texels), and the issue is unconditional (past the end of
// the range it reads clamped, valid queries whose results are never used): a load issued on
// only one side of a branch would make the compiler's waits at the join assume the other side
// and drain the counter.
template <int C, bool L1F16, int ADDR, bool RR, bool FR>
__device__ __forceinline__ void fetch_step(const MfmaArgs& a, const LevelRowL* rows, int qi, int c, int stride,
                                           float2& uv_n, float& lod_n, float& xi_n, const FetchSlot<C, RR>& done,
                                           FetchSlot<C, RR>& next, uint8_t* xb, uint8_t* okb) {
    const int cn = c + stride;
    const float2 uv_c = uv_n;
    const float lod_c = lod_n;
    const float xi_c = xi_n;
    uv_n = *chunk_elem<1>(a.uv, a.n, cn + stride, qi);
    lod_n = *chunk_elem<1>(a.lod, a.n, cn + stride, qi);
    if constexpr (RR) xi_n = *chunk_elem<1>(a.xi, a.n, cn + stride, qi);
    __builtin_amdgcn_sched_barrier(0);
    fetch_issue<C, ADDR, RR>(a, rows, cn, qi, uv_c, lod_c, xi_c, next);
    __builtin_amdgcn_sched_barrier(0);
    fetch_finish<C, L1F16, RR, FR>(a, done, xb, okb, qi);
}

// Output-layer weights for tile t: the stored copy, or copy 0 moved down 4t rows (lane
// (g, r) takes lane (g, r - 4t) of its 16-lane row, zero above) with a DPP row shift.
template <int NC, int KS>
__device__ __forceinline__ uint4 out_weights(const uint4* w0, const uint4 (*copies)[KS], int t, int s) {
    if constexpr (NC == 4) {
        return copies[t][s];
    } else {
        if (t == 0) return w0[s];
        const uint4 v = w0[s];
        uint4 r;
        #define NAM_ROW_SHR(field, n) (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v.field, 0x110 + (n), 0xF, 0xF, false)
        if (t == 1) r = make_uint4(NAM_ROW_SHR(x, 4), NAM_ROW_SHR(y, 4), NAM_ROW_SHR(z, 4), NAM_ROW_SHR(w, 4));
        else if (t == 2) r = make_uint4(NAM_ROW_SHR(x, 8), NAM_ROW_SHR(y, 8), NAM_ROW_SHR(z, 8), NAM_ROW_SHR(w, 8));
        else r = make_uint4(NAM_ROW_SHR(x, 12), NAM_ROW_SHR(y, 12), NAM_ROW_SHR(z, 12), NAM_ROW_SHR(w, 12));
        #undef NAM_ROW_SHR
        return r;
    }
}

// Workgroup of 8 waves on 256-query chunks.  Waves 0-3 fetch (one query per lane): the texel
// loads of the next chunk are issued before the current chunk is blended, from two register
// sets used alternately, and uv / lod run one chunk further ahead (issued first).  Waves 4-7 hold the whole
// decoder in registers and evaluate it on the matrix cores, 64 queries (4 tiles) each.  The
// two roles meet at one barrier per chunk through a double-buffered LDS input block, so the
// fetch of chunk k + 1 overlaps the decode of chunk k; each SIMD runs one wave of each role.
// One launch decodes up to kMaxGroup batches of materials that share this kernel (the server's
// grouped launch): workgroups [first[i], first[i+1]) serve batch i.  A plain decode is a group
// of one.
constexpr int kMaxGroup = 8;
struct MfmaLaunch {
    MfmaArgs item[kMaxGroup];
    int first[kMaxGroup + 1];
    int count;
};

template <int C, int H, int NH, bool L1F16, bool HF8, int ADDR, bool RR, bool FR, bool AL>
__global__ void __launch_bounds__(kBlock, 1) decode_mfma_kernel(const MfmaLaunch L) {
    int item = 0;                              // uniform
    #pragma unroll
    for (int k = 1; k < kMaxGroup; ++k) item += (k < L.count && (int)blockIdx.x >= L.first[k]) ? 1 : 0;
    const MfmaArgs& a = L.item[item];
    const int block = (int)blockIdx.x - L.first[item];
    const int nblocks = L.first[item + 1] - L.first[item];
    constexpr int RT = H / 16;                 // row tiles of a hidden layer
    constexpr int KS = (H + 31) / 32;          // K steps over a hidden layer's outputs
    constexpr int L1_BYTES = L1F16 ? 16 : 8;   // B operand bytes per lane for layer 1
    __shared__ __attribute__((aligned(16))) uint8_t xbuf[2][kChunk * 4 * L1_BYTES];   // 4 lane groups per query
    __shared__ uint8_t okbuf[2][kChunk];
    __shared__ LevelRowL lrows[kMaxLevels];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (threadIdx.x < a.pyr.M) {
        const LevelRow r = a.pyr.rows[threadIdx.x];
        lrows[threadIdx.x] = LevelRowL{(float)r.w, (float)r.h, r.w - 1, r.h - 1, (uint32_t)(r.off * C * 2),
                                       (uint32_t)(r.w * C * 2), 0, 0};
    }
    __syncthreads();

    // chunk range of this workgroup: one contiguous range per group of workgroups sharing an
    // XCD (the grid is a multiple of the group count, so every range has workgroups)
    const int X = a.groups;
    const int grp = block % X;
    const int slot = block / X;
    const int stride = nblocks / X;
    const int c_begin = (int)((int64_t)a.nchunks * grp / X) + slot;
    const int c_end = (int)((int64_t)a.nchunks * (grp + 1) / X);
    const int n = a.n;

    if (wave < 4) {
        // ======================= fetch waves
        const int qi = wave * 64 + lane;          // query of this lane inside a chunk
        FetchSlot<C, RR> s0, s1;
        float2 uv_n = make_float2(0.0f, 0.0f);
        float lod_n = 0.0f;
        float xi_n = 0.0f;
        int c = c_begin;
        int k = 0;
        if (c >= c_end) return;
        {
            const float2 uv0 = *chunk_elem<1>(a.uv, n, c, qi);
            const float lod0 = *chunk_elem<1>(a.lod, n, c, qi);
            const float xi0 = RR ? *chunk_elem<1>(a.xi, n, c, qi) : 0.0f;
            uv_n = *chunk_elem<1>(a.uv, n, c + stride, qi);
            lod_n = *chunk_elem<1>(a.lod, n, c + stride, qi);
            if constexpr (RR) xi_n = *chunk_elem<1>(a.xi, n, c + stride, qi);
            __builtin_amdgcn_sched_barrier(0);
            fetch_issue<C, ADDR, RR>(a, lrows, c, qi, uv0, lod0, xi0, s0);
        }
        // two chunks per trip so that the register sets alternate statically, and a counted loop:
        // an exit between the two halves would give the loop head a second predecessor in which
        // the half-finished register set is still loading, and the compiler's waits would drain
        // the memory counter on every trip
        const int nc = (c_end - c + stride - 1) / stride;   // chunks of this workgroup (>= 1)
        for (int pair = 0; pair < nc / 2; ++pair) {
            fetch_step<C, L1F16, ADDR, RR, FR>(a, lrows, qi, c, stride, uv_n, lod_n, xi_n, s0, s1, xbuf[k & 1],
                                           okbuf[k & 1]);
            __syncthreads();
            fetch_step<C, L1F16, ADDR, RR, FR>(a, lrows, qi, c + stride, stride, uv_n, lod_n, xi_n, s1, s0,
                                           xbuf[(k + 1) & 1], okbuf[(k + 1) & 1]);
            __syncthreads();
            c += 2 * stride;
            k += 2;
        }
        if (nc & 1) {
            fetch_finish<C, L1F16, RR, FR>(a, s0, xbuf[k & 1], okbuf[k & 1], qi);
            __syncthreads();
        }
        return;
    }

    // ======================= decoder waves
    // The decoder is the critical path of a chunk (its matrix-core chains wait on its own
    // conversions); a higher issue priority lets the fetch wave on the same SIMD fill the gaps
    // instead of delaying those conversions.
    __builtin_amdgcn_s_setprio(1);
    const int mw = wave - 4;
    const MfmaLayout lay = mfma_layout(C, H, NH, L1F16, HF8);
    uint4 w1[RT];
    uint4 wh[NH > 1 ? NH - 1 : 1][RT][KS];
    // output layer, one copy per tile of the wave (rows 4t..4t+2); the largest decoder keeps
    // only copy 0 and shifts it on use, to stay within the register budget.  With the albedo
    // head (AL) the six outputs of a tile take rows 0..5 (even tile) or 8..13 (odd tile) of the
    // accumulator of its tile pair: two copies, no shifts, and no more MFMAs than RGB alone.
    constexpr int kOutCopies = AL ? 2 : ((H == 64 && NH == 4) ? 1 : 4);
    uint4 wout[kOutCopies][KS];
    floatx4 b1[RT], bh[NH > 1 ? NH - 1 : 1][RT], bout;
    {
        const uint4* w = a.w;
        #pragma unroll
        for (int j = 0; j < RT; ++j) w1[j] = w[lay.a_index(0, j, 0) * 64 + lane];
        #pragma unroll
        for (int kk = 0; kk < NH - 1; ++kk)
            #pragma unroll
            for (int j = 0; j < RT; ++j)
                #pragma unroll
                for (int s = 0; s < KS; ++s) wh[kk][j][s] = w[lay.a_index(kk + 1, j, s) * 64 + lane];
        // the packed output block holds the RGB rows at rows 0..2 (and the albedo rows at 3..5);
        // copy t moves rows 0..2 to rows 4t..4t+2 (lane (g, r) takes lane (g, r - 4t)) and
        // clears the rest, so the four tiles of the wave accumulate into disjoint row groups of
        // one accumulator.  With the albedo head copy p moves rows 0..5 to rows 8p..8p+5.
        constexpr int kRows = AL ? 6 : 3, kStride = AL ? 8 : 4;
        #pragma unroll
        for (int t = 0; t < kOutCopies; ++t)
            #pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int d = (lane & 15) - kStride * t;
                wout[t][s] = (d >= 0 && d < kRows) ? w[lay.a_index(NH, 0, s) * 64 + lane - kStride * t]
                                                   : make_uint4(0, 0, 0, 0);
            }
        #pragma unroll
        for (int j = 0; j < RT; ++j) b1[j] = a.bias[lay.b_index(0, j) * 64 + lane];
        #pragma unroll
        for (int kk = 0; kk < NH - 1; ++kk)
            #pragma unroll
            for (int j = 0; j < RT; ++j) bh[kk][j] = a.bias[lay.b_index(kk + 1, j) * 64 + lane];
        if constexpr (AL) {
            // row group g holds outputs 4 (g & 1) .. 4 (g & 1) + 3 of its tile: b0..b3, or b4 b5 0 0
            // (the packer leaves neurons past the output width at zero)
            bout = a.bias[lay.b_index(NH, 0) * 64 + 16 * ((lane >> 4) & 1)];
        } else {
            bout = a.bias[lay.b_index(NH, 0) * 64 + (lane & 15)];   // b0 b1 b2 0 in every row group
        }
    }

    int k = 0;
    for (int c = c_begin; c < c_end; c += stride, ++k) {
        __syncthreads();                          // chunk c is in xbuf[k & 1]
        const uint8_t* xb = xbuf[k & 1];
        // output accumulator of the wave's 64 queries: lane (g, q) ends with the RGB
        // pre-activations of query q of tile g at its rows 4g..4g+2, i.e. of query `lane`
        floatx4 out = bout;
        floatx4 out2 = bout;       // albedo head: the accumulator of tiles 2 and 3
        // two tiles at a time: their matrix-core chains are independent, so the conversion of
        // one tile's accumulators overlaps the other tile's MFMAs
        #pragma unroll
        for (int tp = 0; tp < 4; tp += 2) {
            floatx4 acc[2][RT];
            #pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int tile = mw * 4 + tp + u;
                if constexpr (L1F16) {
                    const half8 bx = *reinterpret_cast<const half8*>(xb + (tile * 64 + lane) * 16);
                    #pragma unroll
                    for (int j = 0; j < RT; ++j) acc[u][j] = mfma_f16(__builtin_bit_cast(half8, w1[j]), bx, b1[j]);
                } else {
                    const long bx = *reinterpret_cast<const long*>(xb + (tile * 64 + lane) * 8);
                    #pragma unroll
                    for (int j = 0; j < RT; ++j) {
                        const long wa = (long)w1[j].x | ((long)w1[j].y << 32);
                        acc[u][j] = mfma_fp8(wa, bx, b1[j]);
                    }
                }
            }
            // hidden layers 2..NH, then the output layer
            #pragma unroll
            for (int kk = 0; kk < NH; ++kk) {
                const bool last = (kk == NH - 1);
                floatx4 nacc[2][RT];
                if constexpr (!HF8) {
                    half8 bk[2][KS];
                    #pragma unroll
                    for (int u = 0; u < 2; ++u)
                        #pragma unroll
                        for (int s = 0; s < KS; ++s)
                            #pragma unroll
                            for (int e = 0; e < 8; e += 2) {
                                const int j = 2 * s + e / 4;
                                const half2_t h = (j < RT) ? relu_pack_f16(acc[u][j][e % 4], acc[u][j][e % 4 + 1])
                                                           : half2_t{(_Float16)0.0f, (_Float16)0.0f};
                                bk[u][s][e] = h[0];
                                bk[u][s][e + 1] = h[1];
                            }
                    if (!last) {
                        #pragma unroll
                        for (int j = 0; j < RT; ++j)
                            #pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                nacc[u][j] = bh[kk][j];
                                #pragma unroll
                                for (int s = 0; s < KS; ++s)
                                    nacc[u][j] = mfma_f16(__builtin_bit_cast(half8, wh[kk][j][s]), bk[u][s], nacc[u][j]);
                            }
                    } else {
                        #pragma unroll
                        for (int u = 0; u < 2; ++u)
                            #pragma unroll
                            for (int s = 0; s < KS; ++s) {
                                if constexpr (AL) {
                                    floatx4& o = tp == 0 ? out : out2;
                                    o = mfma_f16(__builtin_bit_cast(half8, wout[u][s]), bk[u][s], o);
                                } else {
                                    out = mfma_f16(__builtin_bit_cast(half8, out_weights<kOutCopies>(wout[0], wout, tp + u, s)),
                                                   bk[u][s], out);
                                }
                            }
                    }
                } else {
                    const float hi = a.mid_hi[kk], inv = a.mid_inv[kk];
                    long bk[2][KS];
                    #pragma unroll
                    for (int u = 0; u < 2; ++u)
                        #pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            const int j0 = 2 * s, j1 = 2 * s + 1;
                            const uint32_t w0 = scaled_fp8x4(acc[u][j0][0], acc[u][j0][1], acc[u][j0][2], acc[u][j0][3],
                                                             0.0f, hi, inv);
                            uint32_t w1 = 0;
                            if (j1 < RT)
                                w1 = scaled_fp8x4(acc[u][j1][0], acc[u][j1][1], acc[u][j1][2], acc[u][j1][3], 0.0f, hi, inv);
                            bk[u][s] = (long)w0 | ((long)w1 << 32);
                        }
                    if (!last) {
                        #pragma unroll
                        for (int j = 0; j < RT; ++j)
                            #pragma unroll
                            for (int u = 0; u < 2; ++u) {
                                nacc[u][j] = bh[kk][j];
                                #pragma unroll
                                for (int s = 0; s < KS; ++s) {
                                    const long wa = (long)wh[kk][j][s].x | ((long)wh[kk][j][s].y << 32);
                                    nacc[u][j] = mfma_fp8(wa, bk[u][s], nacc[u][j]);
                                }
                            }
                    } else {
                        #pragma unroll
                        for (int u = 0; u < 2; ++u)
                            #pragma unroll
                            for (int s = 0; s < KS; ++s) {
                                if constexpr (AL) {
                                    floatx4& o = tp == 0 ? out : out2;
                                    o = mfma_fp8((long)wout[u][s].x | ((long)wout[u][s].y << 32), bk[u][s], o);
                                } else {
                                    const uint4 wt = out_weights<kOutCopies>(wout[0], wout, tp + u, s);
                                    const long wa = (long)wt.x | ((long)wt.y << 32);
                                    out = mfma_fp8(wa, bk[u][s], out);
                                }
                            }
                    }
                }
                if (!last) {
                    #pragma unroll
                    for (int u = 0; u < 2; ++u)
                        #pragma unroll
                        for (int j = 0; j < RT; ++j) acc[u][j] = nacc[u][j];
                }
            }
        }
        // softplus and store: 3 contiguous floats per lane, 768 contiguous bytes per wave.  With
        // the albedo head, lane (g, q) holds outputs 4 (g & 1) .. (4 or 2 of them) of query q of
        // tile g >> 1 (first accumulator) and of tile 2 + (g >> 1) (second): two lanes write a
        // query's 24 bytes, and each half-wave writes 384 contiguous bytes per accumulator.
        if constexpr (AL) {
            const int first = c * kChunk + mw * 64;                  // uniform
            const int g = lane >> 4, half_sel = g & 1;
            float* dst = a.rgb + 6 * (int64_t)first;
            #pragma unroll
            for (int h = 0; h < 2; ++h) {
                const floatx4 o = h == 0 ? out : out2;
                const int qi = (2 * h + (g >> 1)) * 16 + (lane & 15);    // query within the wave
                const bool okq = okbuf[k & 1][mw * 64 + qi];
                if (first + qi < n) {
                    #pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (i < 2 || !half_sel) {
                            const float qv = HF8 ? o[i] * a.out_scale : o[i];
                            dst[6 * qi + 4 * half_sel + i] = okq ? softplus_fast(qv) : __builtin_nanf("");
                        }
                    }
                }
            }
        } else {
            const int first = c * kChunk + mw * 64;                  // uniform
            const bool okq = okbuf[k & 1][mw * 64 + lane];
            float* dst = a.rgb + 3 * (int64_t)first;
            if (first + lane < n) {
                #pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const float qv = HF8 ? out[i] * a.out_scale : out[i];
                    dst[3 * lane + i] = okq ? softplus_fast(qv) : __builtin_nanf("");
                }
            }
        }
    }
}

// Workgroups of a launch over `count` batches: the persistent grid (one workgroup per CU times
// the occupancy) is shared in proportion to the batches' chunks, each batch's share a multiple
// of 8 where it can be (whole XCD groups) and at least one workgroup; batches are given in
// decreasing size so that the large ones start on XCD boundaries.
inline void split_grid(MfmaLaunch* L, int grid) {
    int64_t total = 0;
    for (int i = 0; i < L->count; ++i) total += L->item[i].nchunks;
    int start = 0;
    for (int i = 0; i < L->count; ++i) {
        MfmaArgs& a = L->item[i];
        int w = (int)std::max<int64_t>(1, (int64_t)grid * a.nchunks / std::max<int64_t>(total, 1));
        if (w > a.nchunks) w = a.nchunks;
        if (w >= 8) w -= w % 8;
        if (w < 1) w = 1;
        a.groups = w < 8 ? w : 8;
        L->first[i] = start;
        start += w;
    }
    L->first[L->count] = start;
}

template <int C, int H, int NH, bool L1F16, bool HF8, int ADDR, bool RR, bool FR, bool AL>
static hipError_t launch_shape(MfmaLaunch& L, int cu_count, hipStream_t s) {
    static const int blocks_per_cu = [] {   // thread-safe one-time query
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, decode_mfma_kernel<C, H, NH, L1F16, HF8, ADDR, RR, FR, AL>, kBlock, 0) !=
                hipSuccess || b < 1)
            b = 1;
        return b;
    }();
    split_grid(&L, cu_count * blocks_per_cu);
    clear_stale_hip_error();
    decode_mfma_kernel<C, H, NH, L1F16, HF8, ADDR, RR, FR, AL><<<L.first[L.count], kBlock, 0, s>>>(L);
    return hipGetLastError();
}

template <bool L1F16, bool HF8, int ADDR, bool RR, bool FR, bool AL>
static hipError_t dispatch(const MlpShape& sh, MfmaLaunch& args, int cu, hipStream_t s) {
#define NAM_M_CASE(C_, H_, NH_) \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_) return launch_shape<C_, H_, NH_, L1F16, HF8, ADDR, RR, FR, AL>(args, cu, s);
#define NAM_M_H(C_, H_) NAM_M_CASE(C_, H_, 1) NAM_M_CASE(C_, H_, 2) NAM_M_CASE(C_, H_, 3) NAM_M_CASE(C_, H_, 4)
    NAM_M_H(8, 16) NAM_M_H(8, 32) NAM_M_H(8, 64)
    NAM_M_H(16, 16) NAM_M_H(16, 32) NAM_M_H(16, 64)
#undef NAM_M_H
#undef NAM_M_CASE
    return hipErrorInvalidValue;
}

// Every batch of a launch uses a material of the same shape (output width included),
// precision, address mode and frame presence, and the same filter (checked by the callers).
template <bool L1F16, bool HF8, bool FR, bool AL>
static hipError_t dispatch_filter(const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s) {
    const bool wrap = m->desc.address == NAM_WRAP;
    if (L.item[0].xi)
        return wrap ? dispatch<L1F16, HF8, NAM_WRAP, true, FR, AL>(m->shape, L, cu, s)
                    : dispatch<L1F16, HF8, NAM_CLAMP, true, FR, AL>(m->shape, L, cu, s);
    return wrap ? dispatch<L1F16, HF8, NAM_WRAP, false, FR, AL>(m->shape, L, cu, s)
                : dispatch<L1F16, HF8, NAM_CLAMP, false, FR, AL>(m->shape, L, cu, s);
}

// The four kernel families (frames or not, albedo head or not), each instantiated in a
// translation unit of its own so that they compile in parallel.
hipError_t dispatch_mfma_frames(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s);
hipError_t dispatch_mfma_albedo(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu, hipStream_t s);
hipError_t dispatch_mfma_frames_albedo(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu,
                                       hipStream_t s);

// The precision switch of one family.
template <bool FR, bool AL>
static hipError_t dispatch_precision(bool l1f16, bool hf8, const nam_material* m, MfmaLaunch& L, int cu,
                                     hipStream_t s) {
    if (l1f16 && !hf8) return dispatch_filter<true, false, FR, AL>(m, L, cu, s);
    if (l1f16 && hf8) return dispatch_filter<true, true, FR, AL>(m, L, cu, s);
    if (!l1f16 && hf8) return dispatch_filter<false, true, FR, AL>(m, L, cu, s);
    return hipErrorInvalidValue;
}

// The kernel arguments of one batch.
inline MfmaArgs mfma_args(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                          const float* wi, const float* wo, float* rgb) {
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
    a.frames16 = m->frames16;
    a.nf = m->shape.NF;
    return a;
}

}  // namespace nam
