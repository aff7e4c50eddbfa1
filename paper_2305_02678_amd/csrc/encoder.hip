// The encoder of Sec. 5.1 on the vector ALU, FP32: an MLP from the parameters of the original
// material at a location (A attributes: albedo, roughness, ...) to the latent code (C
// channels), ReLU hidden layers and a linear output layer.  Its weights are packed as the
// decoder's (W_1[HE][A], b_1, ..., W_out[C][HE], b_out).
//
// encoder_forward_kernel: one item per lane.  For queries the parameters are first filtered
// at (uv, lod) with the latent fetch's trilinear taps over a pyramid of the parameters (levels
// concatenated, [texel][A]); the bake instead takes parameter rows as given (every texel of
// every level: the latent texture's initialisation).  The weights are wave-uniform reads.
//
// encoder_backward_kernel: the encoder's share of the first training phase, the gradient of
// sum_i dz_i . E(filtered parameters at query i).  As the decoder's vector training kernel:
// one wave per workgroup, one sample per lane, every layer's activations in the lane's LDS
// column; the layers are walked down, each layer's weight gradient is the in-LDS product of
// the wave's 64 deltas and 64 inputs (layer_grad), added into the workgroup's own partial
// slice, which is reduced over workgroups in a fixed order afterwards.
#include "train_vec.h"

namespace nam {

typedef const __attribute__((address_space(4))) float* cf32;

// y[o] = b[o] + sum_j W[o][j] x[j] (W packed [FO][FI], b after it; wave-uniform)
template <int FI, int FO, bool RELU>
__device__ __forceinline__ void enc_dense(cf32 W, const float* x, float* y) {
    cf32 b = W + FI * FO;
    #pragma unroll
    for (int o = 0; o < FO; ++o) {
        float s = b[o];
        #pragma unroll
        for (int j = 0; j < FI; ++j) s = fmaf(W[o * FI + j], x[j], s);
        y[o] = RELU ? fmaxf(s, 0.0f) : s;
    }
}

// The parameters of item i: a parameter row, or the trilinear filter of the pyramid at the
// query; false for a query with a non-finite uv or lod.
template <int A, bool QUERIES>
__device__ __forceinline__ bool enc_input(const EncoderArgs& a, const LevelRow* rows, int i, float* x) {
    if (!QUERIES) {
        #pragma unroll
        for (int j = 0; j < A; ++j) x[j] = a.attrs[(int64_t)i * A + j];
        return true;
    }
    const float2 q = reinterpret_cast<const float2*>(a.uv)[i];
    const float l = a.lod[i];
    Taps t;
    query_taps_rows(rows, a.M, a.address, q.x, q.y, l, t);
    #pragma unroll
    for (int j = 0; j < A; ++j) x[j] = 0.0f;
    #pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float* T = a.attrs + t.idx[k] * A;
        #pragma unroll
        for (int j = 0; j < A; ++j) x[j] = fmaf(t.w[k], T[j], x[j]);
    }
    return query_ok(q.x, q.y, l);
}

template <int A, int C, int HE, int NHE, bool QUERIES>
__global__ void __launch_bounds__(256) encoder_forward_kernel(const EncoderArgs a) {
    __shared__ LevelRow rows[kMaxLevels];
    if (QUERIES && threadIdx.x < a.M) rows[threadIdx.x] = a.rows[threadIdx.x];
    if (QUERIES) __syncthreads();
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    float x[A];
    const bool ok = enc_input<A, QUERIES>(a, rows, i, x);
    cf32 P = (cf32)a.params;
    float h[HE], h2[HE], out[C];
    enc_dense<A, HE, true>(P, x, h);
    P += A * HE + HE;
    #pragma unroll
    for (int k = 1; k < NHE; ++k) {
        enc_dense<HE, HE, true>(P, h, h2);
        #pragma unroll
        for (int o = 0; o < HE; ++o) h[o] = h2[o];
        P += HE * HE + HE;
    }
    enc_dense<HE, C, false>(P, h, out);
    #pragma unroll
    for (int c = 0; c < C; ++c) a.z[(int64_t)i * C + c] = ok ? out[c] : __builtin_nanf("");
}

// LDS rows of the backward table: the input (A padded to 8), the NHE hidden layers (their
// activations, then their deltas), the output deltas.
template <int A, int C, int HE, int NHE>
struct EncRows {
    static constexpr int X = 0;
    static constexpr int A_PAD = (A + 7) / 8 * 8;
    static constexpr int hid(int k) { return A_PAD + k * HE; }
    static constexpr int D = A_PAD + NHE * HE;
    static constexpr int TOTAL = D + C;
};

template <int A, int C, int HE, int NHE>
__global__ void __launch_bounds__(kTW) encoder_backward_kernel(const EncoderArgs a) {
    using R = EncRows<A, C, HE, NHE>;
    __shared__ float lds[R::TOTAL * kTW];
    __shared__ LevelRow rows[kMaxLevels];
    const int lane = threadIdx.x;
    if (lane < a.M) rows[lane] = a.rows[lane];
    float* col = lds + lane;
    float* part = a.partial + (size_t)blockIdx.x * a.np;
    for (int p = lane; p < a.np; p += kTW) part[p] = 0.0f;
    lds_sync_wave();

    int off[NHE + 1];                          // packed offsets of the layers
    {
        int o = 0;
        #pragma unroll
        for (int k = 0; k <= NHE; ++k) {
            off[k] = o;
            const int fi = k == 0 ? A : HE, fo = k == NHE ? C : HE;
            o += fi * fo + fo;
        }
    }
    cf32 P = (cf32)a.params;
    const int nchunks = (a.n + kTW - 1) / kTW;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int i = c * kTW + lane;
        const bool in_range = i < a.n;
        const int ic = in_range ? i : a.n - 1;
        // ---- input and forward (a sample that contributes nothing has zero input and delta)
        float x[A];
        const bool live = enc_input<A, true>(a, rows, ic, x) && in_range;
        #pragma unroll
        for (int j = 0; j < A; ++j) col[(R::X + j) * kTW] = live ? x[j] : 0.0f;
        #pragma unroll
        for (int j = A; j < R::A_PAD; ++j) col[(R::X + j) * kTW] = 0.0f;
        {
            float xin[A], h[HE];
            #pragma unroll
            for (int j = 0; j < A; ++j) xin[j] = live ? x[j] : 0.0f;
            enc_dense<A, HE, true>(P + off[0], xin, h);
            #pragma unroll
            for (int o = 0; o < HE; ++o) col[(R::hid(0) + o) * kTW] = h[o];
            #pragma unroll
            for (int k = 1; k < NHE; ++k) {
                float h2[HE];
                enc_dense<HE, HE, true>(P + off[k], h, h2);
                #pragma unroll
                for (int o = 0; o < HE; ++o) {
                    h[o] = h2[o];
                    col[(R::hid(k) + o) * kTW] = h2[o];
                }
            }
        }
        // ---- output deltas: the given code gradient (the output layer is linear)
        #pragma unroll
        for (int cc = 0; cc < C; ++cc) col[(R::D + cc) * kTW] = live ? a.dz[(int64_t)ic * C + cc] : 0.0f;
        lds_sync_wave();
        // ---- layers from the output down: weight gradient, then the deltas of the layer below
        int drow = R::D;
        #pragma unroll
        for (int k = NHE; k >= 0; --k) {
            const int arow = k == 0 ? R::X : R::hid(k - 1);
            if (k == NHE) {
                if (k == 0) layer_grad<A, C>(lds, drow, arow, part + off[k], part + off[k] + A * C, lane);
                else layer_grad<HE, C>(lds, drow, arow, part + off[k], part + off[k] + HE * C, lane);
            } else {
                if (k == 0) layer_grad<A, HE>(lds, drow, arow, part + off[k], part + off[k] + A * HE, lane);
                else layer_grad<HE, HE>(lds, drow, arow, part + off[k], part + off[k] + HE * HE, lane);
            }
            if (k == 0) break;
            // delta of hidden layer k - 1: (W_k^T delta_k) masked by its ReLU
            float dprev[HE];
            {
                const int FO = k == NHE ? C : HE;
                cf32 W = P + off[k];
                #pragma unroll
                for (int j = 0; j < HE; ++j) dprev[j] = 0.0f;
                for (int o = 0; o < FO; ++o) {
                    const float d = col[(drow + o) * kTW];
                    #pragma unroll
                    for (int j = 0; j < HE; ++j) dprev[j] = fmaf(W[o * HE + j], d, dprev[j]);
                }
                #pragma unroll
                for (int j = 0; j < HE; ++j) dprev[j] = col[(arow + j) * kTW] > 0.0f ? dprev[j] : 0.0f;
            }
            lds_sync_wave();                       // layer_grad has read the activations
            #pragma unroll
            for (int j = 0; j < HE; ++j) col[(arow + j) * kTW] = dprev[j];
            lds_sync_wave();
            drow = arow;
        }
        lds_sync_wave();
    }
}

template <int A, int C, int HE, int NHE>
static hipError_t launch_encoder_shape(int mode, const EncoderArgs& a, int grid, hipStream_t s) {
    clear_stale_hip_error();
    const unsigned blocks = (unsigned)((a.n + 255) / 256);
    if (mode == 0) encoder_forward_kernel<A, C, HE, NHE, false><<<blocks, 256, 0, s>>>(a);
    else if (mode == 1) encoder_forward_kernel<A, C, HE, NHE, true><<<blocks, 256, 0, s>>>(a);
    else encoder_backward_kernel<A, C, HE, NHE><<<grid, kTW, 0, s>>>(a);
    return hipGetLastError();
}

bool encoder_shape_supported(int A, int C, int HE, int NHE) {
    return (A == 4 || A == 8 || A == 16) && (C == 8 || C == 16) && (HE == 16 || HE == 32 || HE == 64) &&
           (NHE == 1 || NHE == 2);
}

// mode 0: bake (rows), 1: query codes, 2: backward into a.partial (grid workgroups)
hipError_t launch_encoder(int A, int C, int HE, int NHE, int mode, const EncoderArgs& a, int grid, hipStream_t s) {
#define NAM_E_CASE(A_, C_, HE_, NHE_) \
    if (A == A_ && C == C_ && HE == HE_ && NHE == NHE_) return launch_encoder_shape<A_, C_, HE_, NHE_>(mode, a, grid, s);
#define NAM_E_H(A_, C_) NAM_E_CASE(A_, C_, 16, 1) NAM_E_CASE(A_, C_, 16, 2) NAM_E_CASE(A_, C_, 32, 1) \
    NAM_E_CASE(A_, C_, 32, 2) NAM_E_CASE(A_, C_, 64, 1) NAM_E_CASE(A_, C_, 64, 2)
    NAM_E_H(4, 8) NAM_E_H(4, 16) NAM_E_H(8, 8) NAM_E_H(8, 16) NAM_E_H(16, 8) NAM_E_H(16, 16)
#undef NAM_E_H
#undef NAM_E_CASE
    return hipErrorInvalidValue;
}

}  // namespace nam
