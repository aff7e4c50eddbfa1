// Low-precision decode on the gfx950 matrix cores: one fused, persistent kernel per material
// precision (FP16 weights and activations; OCP E4M3 weights and activations with one scale per
// layer; E4M3 with the first layer kept in FP16).  Accumulation is FP32 throughout, the bias is
// added in FP32 (as the accumulator's initial value) and softplus is evaluated in FP32.
//
// Work decomposition.  Every wave of a workgroup (16 waves, four per SIMD) decodes chunks of
// 64 consecutive queries from start to end, with no barrier between waves:
//   fetch    each lane fetches one query: 8 trilinear taps of FP16 texels (16-byte loads),
//            blended in FP32, applies the learned shading frames if the material has
//            them, and writes the network input [z, T wi, T wo, 0...] (32 slots) to the wave's
//            LDS slot in the lane order of the matrix-core B operand;
//   decode   the chunk's 4 tiles of 16 queries go through the decoder: a layer is
//            Y^T = W Y_prev^T with the weights as the A operand (one 16-neuron row tile per
//            instruction, v_mfma_f32_16x16x32_{f16,fp8}, read from LDS once for the 4 tiles)
//            and one query per column.
// Four waves per SIMD interleave there: while one waits for its texels, the others issue
// their blends and matrix-core chains.
// The accumulator of a row tile leaves lane (g, q) = (lane / 16, lane % 16) holding neurons
// 4g..4g+3 of query q; the next layer's B operand needs 8 consecutive K slots per lane, so
// the K order of every hidden layer's weights is permuted at load time to slot
// (s, g, e) <-> neuron 16 (2s + e / 4) + 4g + e % 4: two accumulator tiles, ReLU'd and
// converted, are exactly the next B operand, with no shuffle or LDS round trip.  The output
// layer of tile t uses a copy of its weights moved to rows 4t..4t+2, and the chunk's 4 tiles
// accumulate into one tile: lane (g, q) ends with the RGB of query 16 g + q of the chunk, which
// it stores directly (12 contiguous bytes per lane).  A decoder with the albedo head (6
// outputs: RGB, then the directional albedo of Eq. albedo, Sec. 6.4) instead puts a tile's six
// rows at rows 0..5 or 8..13 of the accumulator of its tile pair, so the output layer costs the
// same number of matrix-core instructions; two lanes then store a query's 24 bytes.
// The weights and biases sit in LDS for the whole kernel.  The grid is persistent; chunks are
// split into one contiguous range per XCD (workgroups are dispatched round-robin over the 8
// XCDs), so neighbouring screen tiles, which share texels, are decoded under the same L2.
#pragma once

#include <algorithm>
#include <cstddef>

#include "latent_fetch.h"
#include "frames.h"
#include "mfma_pack.h"

namespace nam {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 16;            // waves per workgroup: four per SIMD
constexpr int kBlock = kWaves * 64;   // lanes per workgroup
constexpr int kChunk = 64;            // queries per wave chunk (one per lane while fetching)

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

// One query's decoded RGB as it lies in the output array (12 bytes, 4-byte aligned).
struct Rgb {
    float r, g, b;
};

// Orders a wave's LDS writes before its later LDS reads by other lanes of the same wave: the
// wave's LDS operations complete in order once the counter drains, and the wave barrier keeps
// the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f);      // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}

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

// One pyramid level in LDS for the matrix-core decode.  The FP16 pyramid is below 4 GiB (checked
// when the precision is set), so texel addresses are 32-bit byte offsets from the pyramid base.
struct LevelRowL {
    float wf, hf;        // texels along x and y
    int32_t wm, hm;      // the same minus one: wrap mask, or clamp bound
    uint32_t offb;       // byte offset of the level's first texel
    uint32_t pitchb;     // bytes per row
    int32_t pad0, pad1;
};

// Taps along one axis, the same arithmetic as the generic filter (axis_taps: fraction taken
// from the exact p = c W, half-texel shift applied to the fraction, p bounded to +-2^24 under
// clamp addressing).  Under wrap addressing c has already dropped whole periods when
// |c| >= 256.
template <int ADDR>
__device__ __forceinline__ void axis32(float c, float W, int wm, int& x0, int& x1, float& a) {
    float p;
    if constexpr (ADDR == NAM_WRAP) p = c * W;
    else p = fminf(fmaxf(c * W, -16777216.0f), 16777216.0f);
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

// Tap byte offsets and weights of one query (no loads).  Trilinear: both levels, 8 taps in
// stencil order (level l0, then l1; (x0,y0), (x1,y0), (x0,y1), (x1,y1)).  RR: the coarser level
// iff the draw xi < t (t the fractional part of the clamped level, exact in FP32; a NaN draw
// takes the finer level), 4 bilinear taps at full weight (Sec. 4.1).  A non-finite query
// filters at (0, 0, 0), so every load stays inside the pyramid; its result is replaced by NaN
// (non-finite) or dropped (past the end of the batch) through the per-query flag.
template <int C, int ADDR, bool RR>
__device__ __forceinline__ void tap_stencil(int M, const LevelRowL* rows, bool use, float u, float v, float l,
                                            float xi, uint32_t* off, float* w) {
    u = use ? u : 0.0f;
    v = use ? v : 0.0f;
    l = use ? l : 0.0f;
    if constexpr (ADDR == NAM_WRAP) {      // drop whole periods once for both levels
        u = fabsf(u) < 256.0f ? u : u - floorf(u);
        v = fabsf(v) < 256.0f ? v : v - floorf(v);
    }
    const float lam = __builtin_amdgcn_fmed3f(l, 0.0f, (float)(M - 1));   // l is finite here
    const int l0 = (int)lam;
    const int l1 = min(l0 + 1, M - 1);
    const float tt = lam - (float)l0;
    if constexpr (RR) {
        level_stencil32<C, ADDR>(rows[xi < tt ? l1 : l0], u, v, off, w, 1.0f);
    } else {
        level_stencil32<C, ADDR>(rows[l0], u, v, off, w, 1.0f - tt);
        level_stencil32<C, ADDR>(rows[l1], u, v, off + 4, w + 4, tt);
    }
}

__device__ __forceinline__ uint32_t half2_bits(half2_t h) { return __builtin_bit_cast(uint32_t, h); }
__device__ __forceinline__ half2_t bits_half2(uint32_t u) { return __builtin_bit_cast(half2_t, u); }

// z += w T on four FP16 channel pairs (one packed multiply-add each, rounded once; the first tap
// a rounded product): the filter of the matrix-core decoders, in FP16 with FP16 weights.
__device__ __forceinline__ void blend4(half2_t* z, half2_t w2, const uint4& t, bool first) {
    const uint32_t words[4] = {t.x, t.y, t.z, t.w};
    #pragma unroll
    for (int h = 0; h < 4; ++h) {
        const half2_t v = bits_half2(words[h]);
        z[h] = first ? w2 * v : __builtin_elementwise_fma(w2, v, z[h]);
    }
}

// Eight B-operand slots (8 FP16 values as four pairs) stored for layer 1: FP16 as they are,
// E4M3 scaled and rounded (8 bytes).
template <bool L1F16>
__device__ __forceinline__ void store_slots_h(uint8_t* xb, int t, int g, int q, const half2_t* p, float in_hi,
                                              float in_inv) {
    if constexpr (L1F16) {
        *reinterpret_cast<uint4*>(xb + ((t * 4 + g) * 16 + q) * 16) =
            make_uint4(half2_bits(p[0]), half2_bits(p[1]), half2_bits(p[2]), half2_bits(p[3]));
    } else {
        uint2 v;
        v.x = scaled_fp8x4((float)p[0][0], (float)p[0][1], (float)p[1][0], (float)p[1][1], -in_hi, in_hi, in_inv);
        v.y = scaled_fp8x4((float)p[2][0], (float)p[2][1], (float)p[3][0], (float)p[3][1], -in_hi, in_hi, in_inv);
        *reinterpret_cast<uint2*>(xb + ((t * 4 + g) * 16 + q) * 8) = v;
    }
}

// The same for eight FP32 values (directions, frame transforms), rounded to FP16 or E4M3.
template <bool L1F16>
__device__ __forceinline__ void store_slots_f(uint8_t* xb, int t, int g, int q, const float* x, float in_hi,
                                              float in_inv) {
    if constexpr (L1F16) {
        half2_t p[4];
        #pragma unroll
        for (int e = 0; e < 4; ++e) p[e] = half2_t{(_Float16)x[2 * e], (_Float16)x[2 * e + 1]};
        store_slots_h<true>(xb, t, g, q, p, in_hi, in_inv);
    } else {
        uint2 v;
        v.x = scaled_fp8x4(x[0], x[1], x[2], x[3], -in_hi, in_hi, in_inv);
        v.y = scaled_fp8x4(x[4], x[5], x[6], x[7], -in_hi, in_hi, in_inv);
        *reinterpret_cast<uint2*>(xb + ((t * 4 + g) * 16 + q) * 8) = v;
    }
}

// Element of query q (0 <= q < 64) of the wave chunk starting at query `first` of a per-query
// array, clamped to the last query of the batch (loads past the end read valid memory and are
// never used).  The chunk base is uniform and the lane offset 32-bit, so the address is a
// scalar base plus a vector offset.
template <int W, typename T>
__device__ __forceinline__ const T* chunk_elem(const T* arr, int n, int first, int q) {
    const int base = min(first, n - 1);                    // uniform; n < 2^31
    const int last = n - 1 - base;                         // uniform
    const uint32_t off = __umul24((uint32_t)min(q, last), (uint32_t)(W * sizeof(T)));
    return reinterpret_cast<const T*>(reinterpret_cast<const uint8_t*>(arr + (int64_t)W * base) + off);
}

// The texel fetch of one wave chunk for the matrix-core kernels, from the tap offsets and
// weights of the lane's query (tap_stencil): loads the taps, filters them in FP16 (blend4) and
// writes z to the B-operand slots of the chunk's input at xb (K slots 0 .. C - 1 of each
// query).  C = 16: two lanes share each texel (one 16-byte half each), so a load instruction
// covers the whole texels of 32 queries; the tap offsets and FP16 weights reach the sharing
// lanes through a per-wave table at tb (offsets and weights of taps 4 kg..4 kg+3 of query Q at
// rows kg and NT / 4 + kg, 16 bytes per query: conflict-free reads), which is spent before the
// input is written (tb may equal xb).  C = 8: one 16-byte load per tap, one query per lane.
// `next` runs once the texel loads are issued (the caller loads its next chunk's queries
// there).  C = 8: zown receives the lane's own z in FP16 pairs (its blend).  FR with E4M3
// input slots: an FP16 copy of z goes to tb (which lies below xb then), 32 bytes per query,
// for the frame layer (frame_raw_mfma).
template <int C, int NT, bool L1F16, bool FR, typename Next>
__device__ __forceinline__ void fetch_latents(const uint8_t* tex, const uint32_t* off, const float* w, uint8_t* tb,
                                              uint8_t* xb, int lane, float in_hi, float in_inv, half2_t* zown,
                                              Next&& next) {
    const int t_own = lane >> 4, q_own = lane & 15;            // this lane's query in the B layout
    if constexpr (C == 16) {
        // table row of this lane's query
        #pragma unroll
        for (int k = 0; k < NT; k += 4) {
            uint32_t h4[4];
            #pragma unroll
            for (int e = 0; e < 4; ++e) {
                const _Float16 wh = (_Float16)w[k + e];
                h4[e] = half2_bits(half2_t{wh, wh});
            }
            *reinterpret_cast<uint4*>(tb + ((k / 4) * 64 + lane) * 16) = make_uint4(off[k], off[k + 1], off[k + 2], off[k + 3]);
            *reinterpret_cast<uint4*>(tb + ((NT / 4 + k / 4) * 64 + lane) * 16) = make_uint4(h4[0], h4[1], h4[2], h4[3]);
        }
        lds_wave_sync();
        // lane (q, hf): texel half hf of queries q and 32 + q
        const int q = lane & 31, hf = lane >> 5;
        uint32_t toff[2][NT], tw[2][NT];
        #pragma unroll
        for (int qh = 0; qh < 2; ++qh) {
            const int Q = 32 * qh + q;
            #pragma unroll
            for (int k = 0; k < NT; k += 4) {
                const uint4 o = *reinterpret_cast<const uint4*>(tb + ((k / 4) * 64 + Q) * 16);
                toff[qh][k] = o.x; toff[qh][k + 1] = o.y; toff[qh][k + 2] = o.z; toff[qh][k + 3] = o.w;
            }
        }
        uint4 tl[2][NT];
        #pragma unroll
        for (int qh = 0; qh < 2; ++qh)
            #pragma unroll
            for (int k = 0; k < NT; ++k) {
                const uint32_t o = toff[qh][k] + 16u * (uint32_t)hf;     // 32-bit offset from the uniform base
                tl[qh][k] = *reinterpret_cast<const uint4*>(tex + o);
            }
        next();
        // the weights only now: fewer registers held while the texels are in flight
        __builtin_amdgcn_sched_barrier(0);
        #pragma unroll
        for (int qh = 0; qh < 2; ++qh) {
            const int Q = 32 * qh + q;
            #pragma unroll
            for (int k = 0; k < NT; k += 4) {
                const uint4 ww = *reinterpret_cast<const uint4*>(tb + ((NT / 4 + k / 4) * 64 + Q) * 16);
                tw[qh][k] = ww.x; tw[qh][k + 1] = ww.y; tw[qh][k + 2] = ww.z; tw[qh][k + 3] = ww.w;
            }
        }
        lds_wave_sync();                                   // the table is spent: the region takes the input
        #pragma unroll
        for (int qh = 0; qh < 2; ++qh) {
            half2_t zq[4];
            #pragma unroll
            for (int k = 0; k < NT; ++k) blend4(zq, bits_half2(tw[qh][k]), tl[qh][k], k == 0);
            const int Q = 32 * qh + q;
            store_slots_h<L1F16>(xb, Q >> 4, hf, Q & 15, zq, in_hi, in_inv);
            if constexpr (FR && !L1F16)                        // z in FP16 for the frame layer
                *reinterpret_cast<uint4*>(tb + Q * 32 + hf * 16) =
                    make_uint4(half2_bits(zq[0]), half2_bits(zq[1]), half2_bits(zq[2]), half2_bits(zq[3]));
        }
    } else {
        // C = 8: one 16-byte load per tap, one query per lane
        uint4 tl[NT];
        #pragma unroll
        for (int k = 0; k < NT; ++k) tl[k] = *reinterpret_cast<const uint4*>(tex + off[k]);
        next();
        #pragma unroll
        for (int k = 0; k < NT; ++k) {
            const _Float16 wh = (_Float16)w[k];
            blend4(zown, half2_t{wh, wh}, tl[k], k == 0);
        }
        store_slots_h<L1F16>(xb, t_own, 0, q_own, zown, in_hi, in_inv);
        if constexpr (FR && !L1F16)                            // z in FP16 for the frame layer
            *reinterpret_cast<uint4*>(tb + lane * 32) =
                make_uint4(half2_bits(zown[0]), half2_bits(zown[1]), half2_bits(zown[2]), half2_bits(zown[3]));
    }
}

typedef _Float16 half4 __attribute__((ext_vector_type(4)));

// Raw outputs of the learned-frame layer (Sec. 4.2, Eq. frame-rotation) for a chunk's 64
// queries on the matrix cores: one v_mfma_f32_16x16x16_f16 per tile of 16 queries, A = W_F
// (lane (g, r): row r, channels 4g..4g+3, FP16; rows past 6 NF zero), B = the tile's z in
// FP16 read from the input slots (E4M3 input slots: from the FP16 copy at tb), the bias b_F as
// the accumulator's initial value; FP16 products, FP32 accumulation, as the frame layer's
// arithmetic is defined for the matrix-core precisions.  The accumulators leave lane (g, q)
// with outputs 4g..4g+3 of query 16 t + q; they pass through fs (3 KiB) so that each lane ends
// with the outputs of its own query (v[0 .. 6 NF)).
template <int C, bool L1F16>
__device__ __forceinline__ void frame_raw_mfma(half4 afr, floatx4 bfr, const uint8_t* xb, const uint8_t* tb,
                                               uint8_t* fs, int lane, float* v) {
    const int g = lane >> 4, q = lane & 15;
    lds_wave_sync();                                         // the z slots (or the copy) are written
    #pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint2 zb = make_uint2(0u, 0u);
        if (C == 16 || g < 2) {
            const uint8_t* src = L1F16 ? xb + ((t * 4 + (g >> 1)) * 16 + q) * 16 + (g & 1) * 8
                                       : tb + (16 * t + q) * 32 + g * 8;
            zb = *reinterpret_cast<const uint2*>(src);
        }
        const floatx4 o = __builtin_amdgcn_mfma_f32_16x16x16f16(afr, __builtin_bit_cast(half4, zb), bfr, 0, 0, 0);
        if (g < 3) *reinterpret_cast<floatx4*>(fs + ((t * 3 + g) * 16 + q) * 16) = o;
    }
    lds_wave_sync();
    const int t = lane >> 4;                                 // this lane's own query 16 t + q
    #pragma unroll
    for (int gg = 0; gg < 3; ++gg) {
        const floatx4 o = *reinterpret_cast<const floatx4*>(fs + ((t * 3 + gg) * 16 + q) * 16);
        v[4 * gg] = o[0];
        v[4 * gg + 1] = o[1];
        v[4 * gg + 2] = o[2];
        v[4 * gg + 3] = o[3];
    }
}

constexpr int kMaxGroup = 8;

// One launch decodes up to kMaxGroup batches of materials that share this kernel (the server's
// grouped launch): workgroups [first[i], first[i+1]) serve batch i.  A plain decode is a group
// of one.
struct MfmaLaunch {
    MfmaArgs item[kMaxGroup];
    int first[kMaxGroup + 1];
    int count;
};

// Workgroup of kWaves waves, each of which decodes chunks of 64 consecutive queries on its
// own: it fetches and blends the taps of its chunk (one query per lane), writes the network
// input to its LDS slot in the B-operand layout, then runs the chunk's 4 tiles of 16 queries
// through the decoder on the matrix cores, each A operand read from LDS once for the 4 tiles.
// The weights and biases are copied to LDS once per workgroup.  Four waves share each SIMD and
// interleave there (one waits for texels while another runs its matrix-core chain), so no
// barrier separates the fetch from the decode.  The uv / lod (and draw) of a wave's next chunk
// are loaded before the current chunk's texels are awaited.
template <int C, int H, int NH, bool L1F16, bool HF8, int ADDR, bool RR, bool FR, bool AL>
__global__ void __launch_bounds__(kBlock, 1) decode_mfma_kernel(const MfmaLaunch L) {
    int item = 0;                              // uniform
    #pragma unroll
    for (int k = 1; k < kMaxGroup; ++k) item += (k < L.count && (int)blockIdx.x >= L.first[k]) ? 1 : 0;
    const MfmaArgs& a = L.item[item];
    const int block = (int)blockIdx.x - L.first[item];
    const int nblocks = L.first[item + 1] - L.first[item];
    constexpr int NT = RR ? 4 : 8;             // taps per query
    constexpr int RT = H / 16;                 // row tiles of a hidden layer
    constexpr int KS = (H + 31) / 32;          // K steps over a hidden layer's outputs
    constexpr int L1_BYTES = L1F16 ? 16 : 8;   // A / B operand bytes per lane for layer 1
    constexpr int HB = HF8 ? 8 : 16;           // A operand bytes per lane for the later layers
    constexpr int kOutCopies = AL ? 2 : 4;     // output blocks: one per tile (RGB), per tile parity (albedo)
    constexpr int NHB = (NH - 1) * RT * KS;    // hidden A blocks
    // Each wave's LDS region first holds the tap table of its chunk (fetch_latents), then the
    // network input in the B-operand layout (E4M3: in its upper half, the lower half keeping z
    // in FP16 for the frame layer).
    // one LDS block with the decoder first: every weight and bias read is a lane offset plus
    // an immediate below 64 KiB
    struct alignas(16) Smem {
        uint8_t A0[RT][64 * L1_BYTES];
        uint8_t AH[NHB + kOutCopies * KS][64 * HB];
        floatx4 bias[NH * RT + 1][4];
        LevelRowL rows[kMaxLevels];
        uint8_t wreg[kWaves][4096];
        uint8_t fscr[FR ? kWaves : 1][FR ? 3072 : 16];    // FR: the frame layer's outputs per wave
    };
    static_assert(offsetof(Smem, rows) + sizeof(LevelRowL) * kMaxLevels <= 65536, "decoder beyond 64 KiB of LDS");
    __shared__ Smem sm;
    auto& sA0 = sm.A0;
    auto& sAH = sm.AH;
    auto& sBias = sm.bias;
    LevelRowL* lrows = sm.rows;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: chunk indices in scalar registers
    const int g = lane >> 4;                   // lane group of the matrix-core layouts
    const MfmaLayout lay = mfma_layout(C, H, NH, L1F16, HF8);
    {
        // decoder blocks to LDS: layer 1, the hidden layers, the output copies (copy t moves
        // the output rows 0..2 to rows 4t..4t+2, or rows 0..5 to rows 8t..8t+5 with the albedo
        // head: lane (g, r) takes lane (g, r - stride t) of the packed block, zero elsewhere),
        // the biases (the 16 lanes of a group hold the same four), the level table, and zeros
        // in the input slots that are never written
        const uint4* w = a.w;
        for (int i = threadIdx.x; i < RT * 64; i += kBlock) {
            const uint4 v = w[lay.a_index(0, i >> 6, 0) * 64 + (i & 63)];
            if constexpr (L1F16) *reinterpret_cast<uint4*>(&sA0[i >> 6][(i & 63) * 16]) = v;
            else *reinterpret_cast<uint2*>(&sA0[i >> 6][(i & 63) * 8]) = make_uint2(v.x, v.y);
        }
        for (int i = threadIdx.x; i < NHB * 64; i += kBlock) {
            const int b = i >> 6, ln = i & 63;
            const int kk = b / (RT * KS), j = (b / KS) % RT, s = b % KS;
            const uint4 v = w[lay.a_index(kk + 1, j, s) * 64 + ln];
            if constexpr (HF8) *reinterpret_cast<uint2*>(&sAH[b][ln * 8]) = make_uint2(v.x, v.y);
            else *reinterpret_cast<uint4*>(&sAH[b][ln * 16]) = v;
        }
        constexpr int kRows = AL ? 6 : 3, kStride = AL ? 8 : 4;
        for (int i = threadIdx.x; i < kOutCopies * KS * 64; i += kBlock) {
            const int t = i / (KS * 64), s = (i >> 6) % KS, ln = i & 63;
            const int d = (ln & 15) - kStride * t;
            const uint4 v = (d >= 0 && d < kRows) ? w[lay.a_index(NH, 0, s) * 64 + ln - kStride * t]
                                                  : make_uint4(0, 0, 0, 0);
            uint8_t* dst = &sAH[NHB + t * KS + s][0];
            if constexpr (HF8) *reinterpret_cast<uint2*>(dst + ln * 8) = make_uint2(v.x, v.y);
            else *reinterpret_cast<uint4*>(dst + ln * 16) = v;
        }
        for (int i = threadIdx.x; i < (NH * RT + 1) * 4; i += kBlock) sBias[i >> 2][i & 3] = a.bias[(i >> 2) * 64 + 16 * (i & 3)];
        if (threadIdx.x < a.pyr.M) {
            const LevelRow r = a.pyr.rows[threadIdx.x];
            lrows[threadIdx.x] = LevelRowL{(float)r.w, (float)r.h, r.w - 1, r.h - 1, (uint32_t)(r.off * C * 2),
                                           (uint32_t)(r.w * C * 2), 0, 0};
        }
    }
    __syncthreads();

    // chunks of this wave: one contiguous range per group of workgroups sharing an XCD (the
    // grid is a multiple of the group count, so every range has workgroups); inside it the
    // waves of a workgroup take consecutive chunks, so a CU covers neighbouring queries
    const int X = a.groups;
    const int grp = block % X;
    const int stride = (nblocks / X) * kWaves;
    int c = (int)((int64_t)a.nchunks * grp / X) + (block / X) * kWaves + wave;
    const int c_end = (int)((int64_t)a.nchunks * (grp + 1) / X);
    if (c >= c_end) return;
    const int n = a.n;
    uint8_t* const tb = sm.wreg[wave];                    // tap table, spent before the input is written
    uint8_t* const xb = tb + (L1F16 ? 0 : 2048);          // network input, B-operand layout

    // FR: this lane's share of the frame layer as the A operand and accumulator of its
    // matrix-core form (frame_raw_mfma); W_F is stored as FP16 channel pairs [6 NF][C / 2]
    half4 afr = {};
    floatx4 bfr = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (FR) {
        const int r = lane & 15;
        if (r < 6 * a.nf && 4 * g < C)
            afr = __builtin_bit_cast(half4, make_uint2(a.frames16[r * (C / 2) + 2 * g], a.frames16[r * (C / 2) + 2 * g + 1]));
        const float* fbias = reinterpret_cast<const float*>(a.frames16 + 3 * a.nf * C);
        #pragma unroll
        for (int i = 0; i < 4; ++i) bfr[i] = (4 * g + i < 6 * a.nf) ? fbias[4 * g + i] : 0.0f;
    }
    float2 uv = *chunk_elem<1>(a.uv, n, c * kChunk, lane);
    float lod = *chunk_elem<1>(a.lod, n, c * kChunk, lane);
    float xi = RR ? *chunk_elem<1>(a.xi, n, c * kChunk, lane) : 0.0f;
    for (; c < c_end; c += stride) {
        const int first = c * kChunk;                              // uniform
        // ---- fetch.  Lane = query: taps, directions, flag; then the texels and the blend
        const bool use = query_ok(uv.x, uv.y, lod);
        const bool okc = (first + lane < n) && use;
        const uint64_t okm = __ballot(okc);
        uint32_t off[NT];
        float w[NT];
        tap_stencil<C, ADDR, RR>(a.pyr.M, lrows, use, uv.x, uv.y, lod, xi, off, w);
        float dir[6];
        {
            const float* wi = chunk_elem<3>(a.wi, n, first, lane);
            const float* wo = chunk_elem<3>(a.wo, n, first, lane);
            #pragma unroll
            for (int d = 0; d < 3; ++d) {
                dir[d] = wi[d];
                dir[3 + d] = wo[d];
            }
        }
        const int t_own = lane >> 4, q_own = lane & 15;            // this lane's query in the B layout
        half2_t zown[C / 2];                                       // C = 8: this lane's own z
        fetch_latents<C, NT, L1F16, FR>(reinterpret_cast<const uint8_t*>(a.tex), off, w, tb, xb, lane, a.in_hi,
                                        a.in_inv, zown, [&] {
            const int nf = (c + stride) * kChunk;                  // next chunk: clamped, valid queries
            uv = *chunk_elem<1>(a.uv, n, nf, lane);
            lod = *chunk_elem<1>(a.lod, n, nf, lane);
            if constexpr (RR) xi = *chunk_elem<1>(a.xi, n, nf, lane);
        });
        // directions (or their frame transforms) after z, zeros up to slot 32, in this lane's
        // own query
        {
            float x[24];
            #pragma unroll
            for (int k = 0; k < 24; ++k) x[k] = 0.0f;
            if constexpr (FR) {
                float v[12];
                frame_raw_mfma<C, L1F16>(afr, bfr, xb, tb, sm.fscr[wave], lane, v);
                if (a.nf == 2) {
                    frame_apply<2>(0, v, dir, dir + 3, x);
                    frame_apply<2>(1, v + 6, dir, dir + 3, x);
                } else {
                    frame_apply<1>(0, v, dir, dir + 3, x);
                }
            } else {
                #pragma unroll
                for (int d = 0; d < 6; ++d) x[d] = dir[d];
            }
            #pragma unroll
            for (int gg = C / 8; gg < 4; ++gg)
                store_slots_f<L1F16>(xb, t_own, gg, q_own, x + 8 * (gg - C / 8), a.in_hi, a.in_inv);
        }
        lds_wave_sync();

        // ---- decode the chunk's 4 tiles: a layer is Y^T = W Y_prev^T, weights as the A operand.
        // A wave decoding runs at a higher issue priority, so its matrix-core chain goes first
        // and the fetching waves on the SIMD fill the gaps with their vector work.
        __builtin_amdgcn_s_setprio(1);
        floatx4 acc[4][RT];
        {
            #pragma unroll
            for (int j = 0; j < RT; ++j) {
                const floatx4 b = sBias[lay.b_index(0, j)][g];
                if constexpr (L1F16) {
                    const half8 wa = *reinterpret_cast<const half8*>(&sA0[j][lane * 16]);
                    #pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[t][j] = mfma_f16(wa, *reinterpret_cast<const half8*>(xb + (t * 64 + lane) * 16), b);
                } else {
                    const long wa = *reinterpret_cast<const long*>(&sA0[j][lane * 8]);
                    #pragma unroll
                    for (int t = 0; t < 4; ++t)
                        acc[t][j] = mfma_fp8(wa, *reinterpret_cast<const long*>(xb + (t * 64 + lane) * 8), b);
                }
            }
        }
        lds_wave_sync();                          // the slot is free for the next chunk
        // output accumulator: tile t's rows sit at rows 4t..4t+2, so lane (g, q) ends with the
        // RGB pre-activations of query 16 g + q = lane (albedo head: rows 8 (t & 1) ..
        // 8 (t & 1) + 5 of the accumulator of tiles 0-1 or 2-3)
        const floatx4 bout = AL ? sBias[lay.b_index(NH, 0)][g & 1] : sBias[lay.b_index(NH, 0)][0];
        // (RGB: tiles 2 and 3 accumulate into a second tile, halving the dependent chain; their
        // rows sit in lane groups 2 and 3, which take their values from it)
        floatx4 out = bout, out2 = bout;
        #pragma unroll
        for (int kk = 0; kk < NH; ++kk) {
            const bool last = (kk == NH - 1);
            if constexpr (!HF8) {
                half8 bk[4][KS];
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
                if (!last) {
                    #pragma unroll
                    for (int j = 0; j < RT; ++j) {
                        const floatx4 b = sBias[lay.b_index(kk + 1, j)][g];
                        half8 wa[KS];
                        #pragma unroll
                        for (int s = 0; s < KS; ++s)
                            wa[s] = *reinterpret_cast<const half8*>(&sAH[kk * RT * KS + j * KS + s][lane * 16]);
                        #pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            floatx4 v = b;
                            #pragma unroll
                            for (int s = 0; s < KS; ++s) v = mfma_f16(wa[s], bk[t][s], v);
                            acc[t][j] = v;
                        }
                    }
                } else {
                    #pragma unroll
                    for (int t = 0; t < 4; ++t)
                        #pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            const int cp = AL ? (t & 1) : t;
                            const half8 wa = *reinterpret_cast<const half8*>(&sAH[NHB + cp * KS + s][lane * 16]);
                            if (AL && t >= 2) out2 = mfma_f16(wa, bk[t][s], out2);
                            else if (t >= 2) out2 = mfma_f16(wa, bk[t][s], out2);
                            else out = mfma_f16(wa, bk[t][s], out);
                        }
                }
            } else {
                const float hi = a.mid_hi[kk], inv = a.mid_inv[kk];
                long bk[4][KS];
                #pragma unroll
                for (int t = 0; t < 4; ++t)
                    #pragma unroll
                    for (int s = 0; s < KS; ++s) {
                        const int j0 = 2 * s, j1 = 2 * s + 1;
                        const uint32_t w0 = scaled_fp8x4(acc[t][j0][0], acc[t][j0][1], acc[t][j0][2], acc[t][j0][3],
                                                         0.0f, hi, inv);
                        uint32_t w1 = 0;
                        if (j1 < RT)
                            w1 = scaled_fp8x4(acc[t][j1][0], acc[t][j1][1], acc[t][j1][2], acc[t][j1][3], 0.0f, hi, inv);
                        bk[t][s] = (long)w0 | ((long)w1 << 32);
                    }
                if (!last) {
                    #pragma unroll
                    for (int j = 0; j < RT; ++j) {
                        const floatx4 b = sBias[lay.b_index(kk + 1, j)][g];
                        long wa[KS];
                        #pragma unroll
                        for (int s = 0; s < KS; ++s)
                            wa[s] = *reinterpret_cast<const long*>(&sAH[kk * RT * KS + j * KS + s][lane * 8]);
                        #pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            floatx4 v = b;
                            #pragma unroll
                            for (int s = 0; s < KS; ++s) v = mfma_fp8(wa[s], bk[t][s], v);
                            acc[t][j] = v;
                        }
                    }
                } else {
                    #pragma unroll
                    for (int t = 0; t < 4; ++t)
                        #pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            const int cp = AL ? (t & 1) : t;
                            const long wa = *reinterpret_cast<const long*>(&sAH[NHB + cp * KS + s][lane * 8]);
                            if (AL && t >= 2) out2 = mfma_fp8(wa, bk[t][s], out2);
                            else if (t >= 2) out2 = mfma_fp8(wa, bk[t][s], out2);
                            else out = mfma_fp8(wa, bk[t][s], out);
                        }
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
        // softplus and store.  RGB: 3 contiguous floats per lane, 768 contiguous bytes per
        // wave.  Albedo head: lane (g, q) holds outputs 4 (g & 1) .. (4 or 2 of them) of query q
        // of tile g >> 1 (first accumulator) and of tile 2 + (g >> 1) (second), so two lanes
        // write a query's 24 bytes and each half-wave 384 contiguous bytes per accumulator.
        if constexpr (AL) {
            const int half_sel = g & 1;
            float* dst = a.rgb + 6 * (int64_t)first;
            #pragma unroll
            for (int h = 0; h < 2; ++h) {
                const floatx4 o = h == 0 ? out : out2;
                const int qi = (2 * h + (g >> 1)) * 16 + (lane & 15);    // query within the chunk
                const bool okq = (okm >> qi) & 1;
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
            // softplus on every lane, then a select: no branch around it, one 12-byte store
            Rgb v;
            float* vp = &v.r;
            #pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float o = g < 2 ? out[i] : out2[i];
                const float sp = softplus_fast(HF8 ? o * a.out_scale : o);
                vp[i] = okc ? sp : __builtin_nanf("");
            }
            if (first + lane < n) reinterpret_cast<Rgb*>(a.rgb + 3 * (int64_t)first)[lane] = v;
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
        const int need = (a.nchunks + kWaves - 1) / kWaves;     // workgroups with a chunk for every wave
        if (w > need) w = need;
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
