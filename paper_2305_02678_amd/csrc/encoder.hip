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
// sum_i dz_i . E(filtered parameters at query i).  One wave per workgroup, one sample per lane
// for the forward and the deltas, every layer's activations in the lane's LDS column; the layers
// are walked down, and each layer's weight gradient, a contraction over the samples, runs on the
// FP32 matrix cores from those columns (grad_mfma), accumulated in registers over all of the
// wave's chunks and written once into the workgroup's own partial slice, which is reduced over
// workgroups in a fixed order afterwards.
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

// The same with the weights in LDS (read at wave-uniform addresses): inside a loop over chunks
// the scalar form would keep every weight in scalar registers, more than there are.
template <int FI, int FO, bool RELU>
__device__ __forceinline__ void enc_dense_lds(const float* W, const float* x, float* y) {
    const float* b = W + FI * FO;
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

// LDS rows of the backward table (row stride kES floats, odd, so that the 16 rows a matrix-core
// operand reads lie in different banks): the input (A values), the NHE hidden layers (their
// activations, then their deltas), the output deltas.
constexpr int kES = kTW + 1;

template <int A, int C, int HE, int NHE>
struct EncRows {
    static constexpr int X = 0;
    static constexpr int hid(int k) { return A + k * HE; }
    static constexpr int D = A + NHE * HE;
    static constexpr int TOTAL = D + C;
};

typedef float f32x4e __attribute__((ext_vector_type(4)));

// Weight gradient of one layer on the FP32 matrix cores, accumulated over the wave's samples:
// G[o][j] += sum_s delta[o][s] x[j][s] for o < FO, j <= FI, with x[FI][s] = 1 so that column FI
// is the bias gradient.  v_mfma_f32_16x16x4f32 tiles of 16 rows x 16 columns, K = 4 samples
// per instruction, 16 K steps per 64 samples: lane l takes delta[16 r + l % 16][4 k + l / 16]
// as the A operand and x[16 c + l % 16][4 k + l / 16] as the B operand, straight from the
// lanes' LDS columns.  The accumulator of tile (r, c) leaves lane l holding rows
// 16 r + 4 (l / 16) .. + 3 of column 16 c + l % 16.
template <int FI, int FO>
struct GradTiles {
    static constexpr int RO = (FO + 15) / 16;
    static constexpr int CJ = (FI + 1 + 15) / 16;
    f32x4e acc[RO][CJ];
};

template <int FI, int FO>
__device__ __forceinline__ void grad_mfma(const float* lds, int drow, int arow, int lane, GradTiles<FI, FO>& G) {
    const int i = lane & 15, q = lane >> 4;
    #pragma unroll 1
    for (int k = 0; k < kTW / 4; ++k) {
        const int smp = 4 * k + q;
        float av[GradTiles<FI, FO>::RO], bv[GradTiles<FI, FO>::CJ];
        #pragma unroll
        for (int r = 0; r < GradTiles<FI, FO>::RO; ++r) {
            const int o = 16 * r + i;
            av[r] = o < FO ? lds[(drow + o) * kES + smp] : 0.0f;
        }
        #pragma unroll
        for (int c = 0; c < GradTiles<FI, FO>::CJ; ++c) {
            const int j = 16 * c + i;
            bv[c] = j < FI ? lds[(arow + j) * kES + smp] : (j == FI ? 1.0f : 0.0f);
        }
        #pragma unroll
        for (int r = 0; r < GradTiles<FI, FO>::RO; ++r)
            #pragma unroll
            for (int c = 0; c < GradTiles<FI, FO>::CJ; ++c)
                G.acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r], bv[c], G.acc[r][c], 0, 0, 0);
    }
}

// The layer's gradient into the packed slice (W[FO][FI], then b[FO]), every entry written once.
template <int FI, int FO>
__device__ __forceinline__ void grad_store(const GradTiles<FI, FO>& G, float* part, int lane) {
    const int col = lane & 15, g = lane >> 4;
    #pragma unroll
    for (int r = 0; r < GradTiles<FI, FO>::RO; ++r)
        #pragma unroll
        for (int c = 0; c < GradTiles<FI, FO>::CJ; ++c)
            #pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = 16 * r + 4 * g + e, j = 16 * c + col;
                if (o < FO && j < FI) part[o * FI + j] = G.acc[r][c][e];
                else if (o < FO && j == FI) part[FI * FO + o] = G.acc[r][c][e];
            }
}

template <int FI, int FO>
__device__ __forceinline__ void grad_zero(GradTiles<FI, FO>& G) {
    #pragma unroll
    for (int r = 0; r < GradTiles<FI, FO>::RO; ++r)
        #pragma unroll
        for (int c = 0; c < GradTiles<FI, FO>::CJ; ++c) G.acc[r][c] = f32x4e{0.0f, 0.0f, 0.0f, 0.0f};
}

template <int A, int C, int HE, int NHE>
__global__ void __launch_bounds__(kTW) encoder_backward_kernel(const EncoderArgs a) {
    using R = EncRows<A, C, HE, NHE>;
    constexpr int NP = A * HE + HE + (NHE - 1) * (HE * HE + HE) + HE * C + C;
    __shared__ float lds[R::TOTAL * kES];
    __shared__ float wl[NP];                   // the encoder's parameters
    __shared__ LevelRow rows[kMaxLevels];
    const int lane = threadIdx.x;
    if (lane < a.M) rows[lane] = a.rows[lane];
    for (int p = lane; p < NP; p += kTW) wl[p] = a.params[p];
    float* col = lds + lane;
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
    // the wave's gradients, accumulated over all its chunks in matrix-core accumulators
    GradTiles<A, HE> g0;
    GradTiles<HE, HE> gh;                      // the hidden-to-hidden layer (NHE = 2)
    GradTiles<HE, C> go;
    grad_zero(g0);
    grad_zero(gh);
    grad_zero(go);
    const int nchunks = (a.n + kTW - 1) / kTW;
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int i = c * kTW + lane;
        const bool in_range = i < a.n;
        const int ic = in_range ? i : a.n - 1;
        // ---- input and forward (a sample that contributes nothing has zero input and delta)
        float x[A];
        const bool live = enc_input<A, true>(a, rows, ic, x) && in_range;
        #pragma unroll
        for (int j = 0; j < A; ++j) {
            x[j] = live ? x[j] : 0.0f;
            col[(R::X + j) * kES] = x[j];
        }
        {
            float h[HE];
            enc_dense_lds<A, HE, true>(wl + off[0], x, h);
            #pragma unroll
            for (int o = 0; o < HE; ++o) col[(R::hid(0) + o) * kES] = h[o];
            if (NHE == 2) {
                float h2[HE];
                enc_dense_lds<HE, HE, true>(wl + off[1], h, h2);
                #pragma unroll
                for (int o = 0; o < HE; ++o) col[(R::hid(1) + o) * kES] = h2[o];
            }
        }
        // ---- output deltas: the given code gradient (the output layer is linear)
        #pragma unroll
        for (int cc = 0; cc < C; ++cc) col[(R::D + cc) * kES] = live ? a.dz[(int64_t)ic * C + cc] : 0.0f;
        lds_sync_wave();
        // ---- layers from the output down: weight gradient, then the deltas of the layer below
        int drow = R::D;
        #pragma unroll
        for (int k = NHE; k >= 0; --k) {
            const int arow = k == 0 ? R::X : R::hid(k - 1);
            if (k == NHE) grad_mfma<HE, C>(lds, drow, arow, lane, go);
            else if (k == 0) grad_mfma<A, HE>(lds, drow, arow, lane, g0);
            else grad_mfma<HE, HE>(lds, drow, arow, lane, gh);
            if (k == 0) break;
            // delta of hidden layer k - 1: (W_k^T delta_k) masked by its ReLU
            float dprev[HE];
            {
                const int FO = k == NHE ? C : HE;
                const float* W = wl + off[k];
                #pragma unroll
                for (int j = 0; j < HE; ++j) dprev[j] = 0.0f;
                for (int o = 0; o < FO; ++o) {
                    const float d = col[(drow + o) * kES];
                    #pragma unroll
                    for (int j = 0; j < HE; ++j) dprev[j] = fmaf(W[o * HE + j], d, dprev[j]);
                }
                #pragma unroll
                for (int j = 0; j < HE; ++j) dprev[j] = col[(arow + j) * kES] > 0.0f ? dprev[j] : 0.0f;
            }
            lds_sync_wave();                       // the gradient has read the activations
            #pragma unroll
            for (int j = 0; j < HE; ++j) col[(arow + j) * kES] = dprev[j];
            lds_sync_wave();
            drow = arow;
        }
        lds_sync_wave();                           // the table is free for the next chunk
    }
    float* part = a.partial + (size_t)blockIdx.x * a.np;
    grad_store(g0, part + off[0], lane);
    if (NHE == 2) grad_store(gh, part + off[1], lane);
    grad_store(go, part + off[NHE], lane);
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
