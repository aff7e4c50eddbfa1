// Learned shading frames on the vector ALU, FP32, one query per lane (Sec. 4.2,
// "Transformation to learned shading frames", Eq. frame-rotation; the bitangent as stated
// under "Alternative geometric priors" in Sec. 9).
//
// One linear layer (W_F[6N][C], b_F[6N]) maps the latent code z to a normal n_f and a
// tangent t_f per frame (output 6f + r: n_f for r < 3, t_f for r >= 3).  Each is normalised
// on its own; the bitangent is the normalised cross product n^_f x t^_f.  T stacks the rows
// t_f, b_f, n_f of every frame, and the decoder input after z is [T wi, T wo].  A vector v is
// normalised as v / sqrt(max(v.v, 1e-12)), so a zero vector stays zero.
#pragma once

#include <hip/hip_runtime.h>

namespace nam {

__device__ __forceinline__ void unit3(float& x, float& y, float& z) {
    const float r = rsqrtf(fmaxf(fmaf(x, x, fmaf(y, y, z * z)), 1e-12f));
    x *= r;
    y *= r;
    z *= r;
}

// Frame f from its raw normal and tangent v[0..2], v[3..5]: normalise both, form the bitangent
// and write the rows t, b, n applied to wi (out[3 f ..]) and to wo (out[3 NF + 3 f ..]).
template <int NF>
__device__ __forceinline__ void frame_apply(int f, const float* v, const float* wi, const float* wo, float* out) {
    float nx = v[0], ny = v[1], nz = v[2], tx = v[3], ty = v[4], tz = v[5];
    unit3(nx, ny, nz);
    unit3(tx, ty, tz);
    float bx = ny * tz - nz * ty, by = nz * tx - nx * tz, bz = nx * ty - ny * tx;
    unit3(bx, by, bz);
    const float rows[3][3] = {{tx, ty, tz}, {bx, by, bz}, {nx, ny, nz}};
    #pragma unroll
    for (int r = 0; r < 3; ++r) {
        out[3 * f + r] = fmaf(rows[r][0], wi[0], fmaf(rows[r][1], wi[1], rows[r][2] * wi[2]));
        out[3 * NF + 3 * f + r] = fmaf(rows[r][0], wo[0], fmaf(rows[r][1], wo[1], rows[r][2] * wo[2]));
    }
}

// The frame layer is read through the constant address space: its addresses are
// wave-uniform and it does not change during a kernel, so the reads become scalar loads that
// cost no vector-memory issue and no vector registers.
typedef const __attribute__((address_space(4))) float* const_f32_ptr;

__device__ __forceinline__ const_f32_ptr as_constant(const float* p) { return (const_f32_ptr)p; }

// out[3 f + r] = (row r of frame f) . wi and out[3 NF + 3 f + r] = (row r of frame f) . wo,
// rows ordered t, b, n.  F (wave-uniform) holds W_F[6 NF][C] then b_F[6 NF].
template <int C, int NF>
__device__ __forceinline__ void frame_inputs(const_f32_ptr F, const float* z, const float* wi, const float* wo,
                                             float* out) {
    #pragma unroll
    for (int f = 0; f < NF; ++f) {
        float v[6];
        #pragma unroll
        for (int r = 0; r < 6; ++r) {
            const_f32_ptr w = F + (6 * f + r) * C;
            float s = F[6 * NF * C + 6 * f + r];
            #pragma unroll
            for (int c = 0; c < C; ++c) s = fmaf(w[c], z[c], s);
            v[r] = s;
        }
        frame_apply<NF>(f, v, wi, wo, out);
    }
}

// Reverse of unit3 for one vector: given the raw v, its normalised u and the gradient gu of
// a loss with respect to u, the gradient with respect to v: (gu - u (u . gu)) / |v| above the
// 1e-12 floor of v.v, gu * 1e6 (the linear map v / 1e-6) below it.
__device__ __forceinline__ void unit3_back(const float* v, const float* u, const float* gu, float* gv) {
    const float ss = fmaf(v[0], v[0], fmaf(v[1], v[1], v[2] * v[2]));
    const float r = rsqrtf(fmaxf(ss, 1e-12f));
    const float ug = ss > 1e-12f ? fmaf(u[0], gu[0], fmaf(u[1], gu[1], u[2] * gu[2])) : 0.0f;
    #pragma unroll
    for (int c = 0; c < 3; ++c) gv[c] = (gu[c] - u[c] * ug) * r;
}

// Gradient through the frame layer for training (Sec. 4.2 with the decoder and the latents
// trained together, Sec. 5).  G[0 .. 6 NF) is the gradient of the loss with respect to the
// decoder inputs [T wi, T wo] (the layout frame_inputs writes); draw[6 NF] receives the
// gradient with respect to the raw layer outputs (n_f, t_f per frame).  Per frame: the
// gradient of each row of T is G_i[row] wi + G_o[row] wo; the bitangent b = c / |c| with
// c = n^ x t^ passes its gradient gc to n^ (t^ x gc) and t^ (gc x n^); n^ and t^ pass theirs
// through their normalisations.  The raw outputs are recomputed from z.
template <int C, int NF>
__device__ __forceinline__ void frame_backward(const_f32_ptr F, const float* z, const float* wi, const float* wo,
                                               const float* G, float* draw) {
    #pragma unroll
    for (int f = 0; f < NF; ++f) {
        float v[6];
        #pragma unroll
        for (int r = 0; r < 6; ++r) {
            const_f32_ptr w = F + (6 * f + r) * C;
            float s = F[6 * NF * C + 6 * f + r];
            #pragma unroll
            for (int c = 0; c < C; ++c) s = fmaf(w[c], z[c], s);
            v[r] = s;
        }
        float n[3] = {v[0], v[1], v[2]}, t[3] = {v[3], v[4], v[5]};
        unit3(n[0], n[1], n[2]);
        unit3(t[0], t[1], t[2]);
        float c[3] = {n[1] * t[2] - n[2] * t[1], n[2] * t[0] - n[0] * t[2], n[0] * t[1] - n[1] * t[0]};
        float b[3] = {c[0], c[1], c[2]};
        unit3(b[0], b[1], b[2]);
        float gt[3], gb[3], gn[3], gc[3];
        #pragma unroll
        for (int k = 0; k < 3; ++k) {
            gt[k] = fmaf(G[3 * f + 0], wi[k], G[3 * NF + 3 * f + 0] * wo[k]);
            gb[k] = fmaf(G[3 * f + 1], wi[k], G[3 * NF + 3 * f + 1] * wo[k]);
            gn[k] = fmaf(G[3 * f + 2], wi[k], G[3 * NF + 3 * f + 2] * wo[k]);
        }
        unit3_back(c, b, gb, gc);
        gn[0] += t[1] * gc[2] - t[2] * gc[1];
        gn[1] += t[2] * gc[0] - t[0] * gc[2];
        gn[2] += t[0] * gc[1] - t[1] * gc[0];
        gt[0] += gc[1] * n[2] - gc[2] * n[1];
        gt[1] += gc[2] * n[0] - gc[0] * n[2];
        gt[2] += gc[0] * n[1] - gc[1] * n[0];
        unit3_back(v, n, gn, draw + 6 * f);
        unit3_back(v + 3, t, gt, draw + 6 * f + 3);
    }
}

typedef const __attribute__((address_space(4))) uint32_t* const_u32_ptr;
typedef _Float16 frame_half2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ const_u32_ptr as_constant_u32(const uint32_t* p) { return (const_u32_ptr)p; }

// The same transform for the matrix-core decoders, whose layers read FP16 activations and
// weights and accumulate in FP32: the frame layer takes z and W_F rounded to FP16 (packed in
// pairs of channels, Wh[6 NF][C / 2]) and accumulates two channels per dot-product
// instruction in FP32; the normalisations and the transform stay in FP32.  bias: b_F[6 NF].
// zh: z in FP16 channel pairs.
template <int C, int NF>
__device__ __forceinline__ void frame_inputs_h(const_u32_ptr Wh, const_f32_ptr bias, const frame_half2* zh,
                                               const float* wi, const float* wo, float* out) {
    #pragma unroll
    for (int f = 0; f < NF; ++f) {
        float v[6];
        #pragma unroll
        for (int r = 0; r < 6; ++r) {
            const_u32_ptr w = Wh + (6 * f + r) * (C / 2);
            float s = bias[6 * f + r];
            #pragma unroll
            for (int c = 0; c < C / 2; ++c) s = __builtin_amdgcn_fdot2(zh[c], __builtin_bit_cast(frame_half2, w[c]), s, false);
            v[r] = s;
        }
        frame_apply<NF>(f, v, wi, wo, out);
    }
}

}  // namespace nam
