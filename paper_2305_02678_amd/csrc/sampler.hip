// The importance-sampling decoder (Sec. 4.3; App. A): one fused FP32 kernel per sampler shape
// fetches the latent code (trilinear), evaluates the sampling decoder on [z, wi] (ReLU hidden
// layers, 9 linear outputs), applies the output activations and then, per mode, stores the
// 9 proxy parameters, the PDF of a given wo, or a sample wo with its PDF.  A second, network
// free kernel evaluates PDFs or draws samples from cached proxy parameters (the paper queries
// the sampling network once per hit and reuses its parameters for sampling and for PDFs).
//
// Layout per lane as in the FP32 decode: the network input goes to the lane's own LDS column
// and each layer streams it back; weights are wave-uniform, transposed per layer [in][out]
// followed by the bias.
#include "latent_fetch.h"
#include "proxy.h"

namespace nam {

constexpr int kSmpThreads = 128;

template <int IN, int OUT>
__device__ __forceinline__ void dense_col(const float* __restrict__ Wt, const float* col, float* out) {
    const float* bias = Wt + IN * OUT;
    #pragma unroll
    for (int o = 0; o < OUT; ++o) out[o] = bias[o];
    #pragma unroll 2
    for (int j = 0; j < IN; ++j) {
        const float aj = col[j * kSmpThreads];
        const float* wj = Wt + j * OUT;
        #pragma unroll
        for (int o = 0; o < OUT; ++o) out[o] = fmaf(wj[o], aj, out[o]);
    }
}

template <int C, int H, int NH>
__global__ void __launch_bounds__(kSmpThreads)
sampler_kernel(PyrArgs p, const float* __restrict__ tex32, const float* __restrict__ swt, int n, int mode,
               const float2* __restrict__ uv, const float* __restrict__ lod, const float* __restrict__ wi,
               const float* __restrict__ wo_in, const float* __restrict__ u, float* __restrict__ params_out,
               float* __restrict__ wo_out, float* __restrict__ pdf_out) {
    __shared__ float act[kMaxWidth * kSmpThreads];
    const int i = blockIdx.x * kSmpThreads + threadIdx.x;
    const bool live = i < n;
    const int qi = live ? i : n - 1;
    float* col = act + threadIdx.x;
    float w_in[3];
    bool finite;
    {
        const float2 q = uv[qi];
        finite = query_ok(q.x, q.y, lod[qi]);
        Taps t;
        float z[C];
        query_taps(p, q.x, q.y, lod[qi], t);
        gather_f32<C>(tex32, t, z);
        #pragma unroll
        for (int c = 0; c < C; ++c) col[c * kSmpThreads] = z[c];
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
            w_in[c] = wi[3 * qi + c];
            col[(C + c) * kSmpThreads] = w_in[c];
        }
    }
    const float* W = swt;
    {
        float h[H];
        dense_col<C + 3, H>(W, col, h);
        #pragma unroll
        for (int o = 0; o < H; ++o) col[o * kSmpThreads] = fmaxf(h[o], 0.0f);
        W += (C + 3) * H + H;
    }
    #pragma unroll
    for (int k = 1; k < NH; ++k) {
        float h[H];
        dense_col<H, H>(W, col, h);
        #pragma unroll
        for (int o = 0; o < H; ++o) col[o * kSmpThreads] = fmaxf(h[o], 0.0f);
        W += H * H + H;
    }
    float raw[9], pr[9];
    dense_col<H, 9>(W, col, raw);
    proxy_activate(raw, pr);
    if (!live) return;
    const float nan = __builtin_nanf("");
    if (mode == kModeParams) {
        #pragma unroll
        for (int k = 0; k < 9; ++k) params_out[9 * (int64_t)i + k] = finite ? pr[k] : nan;
    } else if (mode == kModePdf) {
        const float w[3] = {wo_in[3 * (int64_t)i], wo_in[3 * (int64_t)i + 1], wo_in[3 * (int64_t)i + 2]};
        pdf_out[i] = finite ? proxy_pdf(pr, w_in, w) : nan;
    } else {
        const float uu[3] = {u[3 * (int64_t)i], u[3 * (int64_t)i + 1], u[3 * (int64_t)i + 2]};
        float w[3];
        const float pd = proxy_sample(pr, w_in, uu, w);
        #pragma unroll
        for (int c = 0; c < 3; ++c) wo_out[3 * (int64_t)i + c] = finite ? w[c] : nan;
        pdf_out[i] = finite ? pd : nan;
    }
}

// PDFs (u == nullptr) or samples from cached proxy parameters params[n][9].
__global__ void __launch_bounds__(256)
proxy_kernel(int n, const float* __restrict__ params, const float* __restrict__ wi,
             const float* __restrict__ wo_in, const float* __restrict__ u, float* __restrict__ wo_out,
             float* __restrict__ pdf_out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float pr[9], w_in[3];
    #pragma unroll
    for (int k = 0; k < 9; ++k) pr[k] = params[9 * (int64_t)i + k];
    #pragma unroll
    for (int c = 0; c < 3; ++c) w_in[c] = wi[3 * (int64_t)i + c];
    if (u) {
        const float uu[3] = {u[3 * (int64_t)i], u[3 * (int64_t)i + 1], u[3 * (int64_t)i + 2]};
        float w[3];
        pdf_out[i] = proxy_sample(pr, w_in, uu, w);
        #pragma unroll
        for (int c = 0; c < 3; ++c) wo_out[3 * (int64_t)i + c] = w[c];
    } else {
        const float w[3] = {wo_in[3 * (int64_t)i], wo_in[3 * (int64_t)i + 1], wo_in[3 * (int64_t)i + 2]};
        pdf_out[i] = proxy_pdf(pr, w_in, w);
    }
}

template <int C, int H, int NH>
static hipError_t launch_sampler_shape(const nam_material* m, int n, int mode, const float* uv, const float* lod,
                                       const float* wi, const float* wo_in, const float* u, float* params_out,
                                       float* wo_out, float* pdf_out, hipStream_t s) {
    const dim3 grid((n + kSmpThreads - 1) / kSmpThreads), block(kSmpThreads);
    clear_stale_hip_error();
    sampler_kernel<C, H, NH><<<grid, block, 0, s>>>(m->pyr(), m->texels32, m->swt32, n, mode,
                                                    reinterpret_cast<const float2*>(uv), lod, wi, wo_in, u,
                                                    params_out, wo_out, pdf_out);
    return hipGetLastError();
}

hipError_t launch_sampler(const nam_material* m, int64_t n, int mode, const float* uv, const float* lod,
                          const float* wi, const float* wo_in, const float* u, float* params_out, float* wo_out,
                          float* pdf_out, hipStream_t s) {
    const MlpShape sh = m->sshape;
#define NAM_S_CASE(C_, H_, NH_)                                                                               \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_)                                                             \
        return launch_sampler_shape<C_, H_, NH_>(m, (int)n, mode, uv, lod, wi, wo_in, u, params_out, wo_out, \
                                                 pdf_out, s);
#define NAM_S_H(C_, H_) NAM_S_CASE(C_, H_, 1) NAM_S_CASE(C_, H_, 2) NAM_S_CASE(C_, H_, 3) NAM_S_CASE(C_, H_, 4)
    NAM_S_H(8, 16) NAM_S_H(8, 32) NAM_S_H(8, 64)
    NAM_S_H(16, 16) NAM_S_H(16, 32) NAM_S_H(16, 64)
#undef NAM_S_H
#undef NAM_S_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_proxy(int64_t n, const float* params, const float* wi, const float* wo_in, const float* u,
                        float* wo_out, float* pdf_out, hipStream_t s) {
    clear_stale_hip_error();
    proxy_kernel<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>((int)n, params, wi, wo_in, u, wo_out,
                                                                         pdf_out);
    return hipGetLastError();
}

}  // namespace nam
