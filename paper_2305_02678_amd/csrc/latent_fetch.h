// Device-side latent texture addressing and filtering (the hierarchical latent texture of
// Sec. 4.1, "Latent texture", read with trilinear filtering: bilinear inside the two levels
// nearest to the fractional mip level, linear across them).
//
// Conventions: texel x of a level of width W is centred at u = (x + 1/2) / W; x <-> u,
// y <-> v, row-major [y][x][C]; the mip level is clamped to [0, M-1]; wrap addressing is
// periodic in u and v, clamp addressing replicates the edge texels.  Sizes are powers of two,
// so the wrap modulus is a bit mask, also correct for negative tap positions.
#pragma once

#include "nam_internal.h"

namespace nam {

// The 8 taps of one query: flat texel index into the concatenated pyramid and weight.
struct Taps {
    int64_t idx[8];
    float w[8];
};

__device__ __forceinline__ bool query_ok(float u, float v, float lod) {
    return __builtin_isfinite(u) && __builtin_isfinite(v) && __builtin_isfinite(lod);
}

// Taps along one axis of a level of size W: sample position s = c W - 1/2, taps floor(s) and
// floor(s) + 1, fraction a = s - floor(s).  Forming s itself can round (c W - 1/2 crosses a
// power of two: -1023.65 - 0.5 loses the last bit) and so can the fractional part of a small
// negative c (1 - 0.077), so the split is taken from p = c W, which is exact: its fractional
// part fr is exact for |p| >= 1, and the half-texel shift is applied to fr (fr - 1/2 or
// fr + 1/2, both exact there).  Under wrap addressing |c| >= 256 first drops whole periods
// (exact for |c| >= 1) so that p stays below 2^23.  Under clamp addressing p is bounded to
// +-2^24, past which it is a whole number anyway (for a power-of-two level it is from 2^23 on,
// exactly), so the two taps keep the weights of the exact position also where both are the
// edge texel: the sum is the same in exact arithmetic, and a filter that rounds each product
// (the FP16 filter of the matrix-core kernels) rounds the same products as the exact weights
// give.
__device__ __forceinline__ void axis_taps(float c, int W, int address, int& x0, int& x1, float& a) {
    float p;
    if (address == NAM_WRAP) {
        const float cc = fabsf(c) < 256.0f ? c : c - floorf(c);
        p = cc * (float)W;
    } else {
        p = fminf(fmaxf(c * (float)W, -16777216.0f), 16777216.0f);
    }
    const float fp = floorf(p);
    const float fr = p - fp;
    int i = (int)fp;
    if (fr >= 0.5f) {
        a = fr - 0.5f;
    } else {
        a = fr + 0.5f;
        i -= 1;
    }
    if (address == NAM_WRAP) {
        x0 = i & (W - 1);
        x1 = (i + 1) & (W - 1);
    } else {
        x0 = min(max(i, 0), W - 1);
        x1 = min(max(i + 1, 0), W - 1);
    }
}

// Bilinear stencil in one level (u, v finite); weights scaled by the level's blend weight.
__device__ __forceinline__ void level_stencil(const LevelRow row, int address, float u, float v,
                                              int64_t* idx, float* w, float scale) {
    int x0, x1, y0, y1;
    float a, b;
    axis_taps(u, row.w, address, x0, x1, a);
    axis_taps(v, row.h, address, y0, y1, b);
    const int64_t base = row.off;
    const int64_t W = row.w;
    idx[0] = base + y0 * W + x0;
    idx[1] = base + y0 * W + x1;
    idx[2] = base + y1 * W + x0;
    idx[3] = base + y1 * W + x1;
    const float wa0 = (1.0f - a) * scale, wa1 = a * scale;
    w[0] = wa0 * (1.0f - b);
    w[1] = wa1 * (1.0f - b);
    w[2] = wa0 * b;
    w[3] = wa1 * b;
}

// Fills the 8 taps (level l0 first) from a level table `rows` (global or LDS).  A non-finite
// query is redirected to texel 0 with NaN weights so that every load stays inside the pyramid
// and the result is NaN.
template <typename Rows>
__device__ __forceinline__ void query_taps_rows(Rows rows, int M, int address, float u, float v, float lod,
                                                Taps& t) {
    const bool ok = query_ok(u, v, lod);
    if (!ok) { u = 0.0f; v = 0.0f; lod = 0.0f; }
    const float top = (float)(M - 1);
    const float lam = fminf(fmaxf(lod, 0.0f), top);
    const int l0 = (int)lam;                       // lam >= 0: truncation is floor
    const int l1 = min(l0 + 1, M - 1);
    const float tt = lam - (float)l0;
    level_stencil(rows[l0], address, u, v, t.idx, t.w, 1.0f - tt);
    level_stencil(rows[l1], address, u, v, t.idx + 4, t.w + 4, tt);
    if (!ok) {
        #pragma unroll
        for (int k = 0; k < 8; ++k) t.w[k] = __builtin_nanf("");
    }
}

__device__ __forceinline__ void query_taps(const PyrArgs p, float u, float v, float lod, Taps& t) {
    query_taps_rows(p.rows, p.M, p.address, u, v, lod, t);
}

// Taps with the level chosen by Russian roulette (Sec. 4.1, "Latent texture": one of the two
// nearest levels is picked at random and filtered bilinearly): with t the fractional part of the
// clamped level, the coarser level l1 is used iff the caller's draw xi < t (a NaN draw uses l0),
// at full weight.  Only taps 0..3 are filled.  t = lam - floor(lam) is exact in FP32, so the
// choice does not depend on the precision it is made in.  Non-finite queries as above.
__device__ __forceinline__ void query_taps_rr(const PyrArgs p, float u, float v, float lod, float xi, Taps& t) {
    const bool ok = query_ok(u, v, lod);
    if (!ok) { u = 0.0f; v = 0.0f; lod = 0.0f; }
    const float top = (float)(p.M - 1);
    const float lam = fminf(fmaxf(lod, 0.0f), top);
    const int l0 = (int)lam;
    const int l1 = min(l0 + 1, p.M - 1);
    const float tt = lam - (float)l0;
    level_stencil(p.rows[xi < tt ? l1 : l0], p.address, u, v, t.idx, t.w, 1.0f);
    if (!ok) {
        #pragma unroll
        for (int k = 0; k < 4; ++k) t.w[k] = __builtin_nanf("");
    }
}

// z[c] = sum_k w_k * T[idx_k][c] over the first NT taps, FP32 texels; C a multiple of 4.
template <int C, int NT = 8>
__device__ __forceinline__ void gather_f32(const float* __restrict__ tex, const Taps& t, float* z) {
    #pragma unroll
    for (int c = 0; c < C; ++c) z[c] = 0.0f;
    #pragma unroll
    for (int k = 0; k < NT; ++k) {
        const float4* p = reinterpret_cast<const float4*>(tex + t.idx[k] * C);
        #pragma unroll
        for (int c4 = 0; c4 < C / 4; ++c4) {
            const float4 v = p[c4];
            z[4 * c4 + 0] = fmaf(t.w[k], v.x, z[4 * c4 + 0]);
            z[4 * c4 + 1] = fmaf(t.w[k], v.y, z[4 * c4 + 1]);
            z[4 * c4 + 2] = fmaf(t.w[k], v.z, z[4 * c4 + 2]);
            z[4 * c4 + 3] = fmaf(t.w[k], v.w, z[4 * c4 + 3]);
        }
    }
}

// Same for FP16 texels (widened to FP32 before the blend); C a multiple of 8.
template <int C, int NT = 8>
__device__ __forceinline__ void gather_f16(const __half* __restrict__ tex, const Taps& t, float* z) {
    #pragma unroll
    for (int c = 0; c < C; ++c) z[c] = 0.0f;
    #pragma unroll
    for (int k = 0; k < NT; ++k) {
        const uint4* p = reinterpret_cast<const uint4*>(tex + t.idx[k] * C);
        #pragma unroll
        for (int c8 = 0; c8 < C / 8; ++c8) {
            const uint4 v = p[c8];
            const uint32_t words[4] = {v.x, v.y, v.z, v.w};
            #pragma unroll
            for (int h = 0; h < 4; ++h) {
                const __half2 pair = *reinterpret_cast<const __half2*>(&words[h]);
                const float2 f = __half22float2(pair);
                z[8 * c8 + 2 * h + 0] = fmaf(t.w[k], f.x, z[8 * c8 + 2 * h + 0]);
                z[8 * c8 + 2 * h + 1] = fmaf(t.w[k], f.y, z[8 * c8 + 2 * h + 1]);
            }
        }
    }
}

}  // namespace nam
