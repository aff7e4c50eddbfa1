// The analytic importance-sampling proxy (Sec. 4.3; App. A, Eq. pdf_full, Eq. pdf_spec) in
// FP32, one query per lane: output activations of the sampling decoder, the PDF of a
// direction and the sample transform.
//
// Parameters p[9] = {w_d, mu_dx, mu_dy, w_s, alpha_x, alpha_y, rho, mu_sx, mu_sy}.
// Activations (the paper names quadratic approximations of tanh and sinh and a softmax, not
// their formulas): qtanh(x) = x (1 - |x| / 4) for |x| < 2 and sign(x) beyond; qsinh(x) =
// x (1 + |x| / 2); (w_d, w_s) = softmax; mu = qsinh; alpha = 1e-3 + (1 - 1e-3)(1 + qtanh) / 2;
// rho = 0.999 qtanh (M stays invertible).
// PDF over the sphere: w_d max(0, wo . n_d) / pi + w_s D_std(h') det(M^-1) / |M^-1 h|^3 /
// (4 |wo . h|), with n_d = normalise(-mu_dx, -mu_dy, 1), h = normalise(wi + wo) folded to the
// upper hemisphere, h' = M^-1 h / |M^-1 h| and D_std(h') = max(h'_z, 0) / pi, the density of
// the alpha = 1 GGX normal sampler.
// Sampling with u in [0,1)^3: diffuse if u_0 < w_d (a cosine sample turned by the minimal
// rotation from +z to n_d), else h = normalise(M h_std) with h_std a cosine sample and
// wo = 2 (wi . h) h - wi.
#pragma once

#include <hip/hip_runtime.h>

namespace nam {

constexpr float kInvPi = 0.318309886183790672f;

// What a fused sampler launch stores: the 9 proxy parameters, the PDF of given directions, or
// samples and their PDFs.
enum SamplerMode { kModeParams = 0, kModePdf = 1, kModeSample = 2 };

// Single-instruction forms of the transcendental steps: every operand below is a normal,
// well-conditioned number (a softmax sum in [1, 2], anisotropies >= 1e-3, sqrt(1 - rho^2) >=
// 0.044, u in [0, 1)), where the hardware reciprocal and square root err by about 1 ulp and the
// exponential and sine by a few ulp of their argument, far inside the proxy's tolerance.
__device__ __forceinline__ float rcp_f(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_f(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float exp_f(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

__device__ __forceinline__ float qtanh_f(float x) {
    const float a = fabsf(x);
    return a < 2.0f ? x * (1.0f - 0.25f * a) : copysignf(1.0f, x);
}

__device__ __forceinline__ float qsinh_f(float x) { return x * (1.0f + 0.5f * fabsf(x)); }

__device__ __forceinline__ void proxy_activate(const float* raw, float* p) {
    const float m = fmaxf(raw[0], raw[3]);
    const float ed = exp_f(raw[0] - m), es = exp_f(raw[3] - m);
    const float inv = rcp_f(ed + es);
    p[0] = ed * inv;
    p[3] = es * inv;
    p[1] = qsinh_f(raw[1]);
    p[2] = qsinh_f(raw[2]);
    p[4] = 1e-3f + (1.0f - 1e-3f) * 0.5f * (1.0f + qtanh_f(raw[4]));
    p[5] = 1e-3f + (1.0f - 1e-3f) * 0.5f * (1.0f + qtanh_f(raw[5]));
    p[6] = 0.999f * qtanh_f(raw[6]);
    p[7] = qsinh_f(raw[7]);
    p[8] = qsinh_f(raw[8]);
}

__device__ __forceinline__ float dot3f(const float* a, const float* b) {
    return fmaf(a[0], b[0], fmaf(a[1], b[1], a[2] * b[2]));
}

__device__ __forceinline__ float proxy_pdf(const float* p, const float* wi, const float* wo) {
    const float nx = -p[1], ny = -p[2];
    const float rn = rsqrtf(fmaf(nx, nx, fmaf(ny, ny, 1.0f)));
    const float cd = fmaf(wo[0], nx, fmaf(wo[1], ny, wo[2])) * rn;
    const float pd = cd > 0.0f ? cd * kInvPi : 0.0f;
    float h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    const float hh = dot3f(h, h);
    float ps = 0.0f;
    if (hh > 0.0f) {
        const float s = copysignf(rsqrtf(hh), h[2]);   // normalise and fold to h_z >= 0
        h[0] *= s;
        h[1] *= s;
        h[2] *= s;
        // M^-1 h: M^-1 = [[1/ax, 0, mx/ax], [i10, i11, i10 mx + i11 my], [0, 0, 1]]
        const float ax = p[4], ay = p[5], rho = p[6], mx = p[7], my = p[8];
        const float sr = sqrt_f(1.0f - rho * rho);
        const float i00 = rcp_f(ax), i11 = rcp_f(ay * sr), i10 = -rho * i00 * rcp_f(sr);
        const float hx = h[0] + mx * h[2], hy = h[1] + my * h[2];   // (A^-1 applied after the shift)
        const float q0 = i00 * hx, q1 = fmaf(i10, hx, i11 * hy), q2 = h[2];
        const float lp2 = fmaf(q0, q0, fmaf(q1, q1, q2 * q2));
        const float rl = rsqrtf(lp2);
        const float dstd = q2 > 0.0f ? q2 * rl * kInvPi : 0.0f;
        const float oh = fabsf(dot3f(wo, h));
        const float det_mi = i00 * i11;
        ps = oh > 0.0f ? dstd * det_mi * (rl * rl * rl) * rcp_f(4.0f * oh) : 0.0f;
    }
    return fmaf(p[0], pd, p[3] * ps);
}

__device__ __forceinline__ float proxy_sample(const float* p, const float* wi, const float* u, float* wo) {
    // the hardware sine and cosine take their argument in revolutions: sin(2 pi u_2)
    const float sn = __builtin_amdgcn_sinf(u[2]), cs = __builtin_amdgcn_cosf(u[2]);
    const float r = sqrt_f(u[1]);
    const float v0 = r * cs, v1 = r * sn, v2 = sqrt_f(1.0f - u[1]);
    if (u[0] < p[0]) {
        const float nx0 = -p[1], ny0 = -p[2];
        const float rn = rsqrtf(fmaf(nx0, nx0, fmaf(ny0, ny0, 1.0f)));
        const float nx = nx0 * rn, ny = ny0 * rn, nz = rn;
        const float a = rcp_f(1.0f + nz);
        // minimal rotation taking e_z to n: columns (1 - a nx^2, -a nx ny, -nx), (-a nx ny, 1 - a ny^2, -ny), n
        wo[0] = fmaf(v0, 1.0f - a * nx * nx, fmaf(v1, -a * nx * ny, v2 * nx));
        wo[1] = fmaf(v0, -a * nx * ny, fmaf(v1, 1.0f - a * ny * ny, v2 * ny));
        wo[2] = fmaf(v0, -nx, fmaf(v1, -ny, v2 * nz));
    } else {
        const float ax = p[4], ay = p[5], rho = p[6], mx = p[7], my = p[8];
        const float sr = sqrt_f(1.0f - rho * rho);
        float h[3] = {fmaf(ax, v0, -mx * v2), fmaf(ay * rho, v0, fmaf(ay * sr, v1, -my * v2)), v2};
        const float rl = rsqrtf(dot3f(h, h));
        h[0] *= rl;
        h[1] *= rl;
        h[2] *= rl;
        const float d = 2.0f * dot3f(wi, h);
        wo[0] = fmaf(d, h[0], -wi[0]);
        wo[1] = fmaf(d, h[1], -wi[1]);
        wo[2] = fmaf(d, h[2], -wi[2]);
    }
    return proxy_pdf(p, wi, wo);
}

}  // namespace nam
