// Matrix-core training kernels (layouts and the scheme are described in train_mfma.h).
#include "train_mfma.h"

namespace nam {

constexpr int kTMWaves = 4;
constexpr int kTMThreads = 64 * kTMWaves;

// softplus and its derivative, the logistic function, in FP32 on the hardware exp2, log2 and
// reciprocal (a few ulp).  Both start from e = exp(-|q|), which the compiler shares between them;
// log1p(e) = log(1 + e) e / ((1 + e) - 1) is Kahan's correction of the rounding of 1 + e (e itself
// where 1 + e rounds to 1), and logistic(q) = 1 / (1 + e) for q >= 0 and e / (1 + e) below.
__device__ __forceinline__ float tm_exp_neg_abs(float q) { return __builtin_amdgcn_exp2f(-fabsf(q) * 1.44269504088896341f); }
__device__ __forceinline__ float tm_softplus(float q) {
    const float e = tm_exp_neg_abs(q);
    const float u = 1.0f + e, d = u - 1.0f;
    const float l = d == 0.0f ? e : (__builtin_amdgcn_logf(u) * 0.693147180559945309f) * (e * __builtin_amdgcn_rcpf(d));
    return fmaxf(q, 0.0f) + l;
}
__device__ __forceinline__ float tm_logistic(float q) {
    const float e = tm_exp_neg_abs(q);
    const float r = __builtin_amdgcn_rcpf(1.0f + e);
    return q >= 0.0f ? r : e * r;
}

__device__ __forceinline__ f32x4 ld4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }
__device__ __forceinline__ void st4(float* p, f32x4 v) { *reinterpret_cast<f32x4*>(p) = v; }

// Builds the operand blocks of TrainLayout from packed parameters, one thread per float.
template <int C, int H, int NH>
__global__ void __launch_bounds__(256) pack_train_kernel(const float* __restrict__ p, int NO, float* __restrict__ blob) {
    using L = TrainLayout<C, H, NH>;
    constexpr int IN = C + 6, HT = L::HT;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= L::BLOB) return;
    const int oo = param_off<C, H>(NH + 1);
    float v = 0.0f;
    if (e < L::FWH) {
        const int x = e - L::FW1, qq = x & 3, lane = (x >> 2) & 63, blk = x >> 8;
        const int grp = blk % L::G1, tp = blk / L::G1, g = lane >> 4, o = 16 * tp + (lane & 15);
        const int q = 4 * grp + qq;
        if (q < L::Q1) {
            const int in = slot_input<C>(q, g);
            if (in >= 0 && in < IN) v = p[o * IN + in];
            else if (in == C + 6) v = p[IN * H + o];
        }
    } else if (e < L::FWO) {
        const int k = 2 + (e - L::FWH) / L::WH_SZ, x = (e - L::FWH) % L::WH_SZ;
        const int r = x & 3, lane = (x >> 2) & 63, blk = x >> 8, t = blk % HT, tp = blk / HT;
        v = p[param_off<C, H>(k) + (16 * tp + (lane & 15)) * H + 16 * t + 4 * (lane >> 4) + r];
    } else if (e < L::BWO) {
        const int x = e - L::FWO, r = x & 3, lane = (x >> 2) & 63, t = x >> 8, i = lane & 15;
        if (i < NO) v = p[oo + i * H + 16 * t + 4 * (lane >> 4) + r];
    } else if (e < L::BWH) {
        const int x = e - L::BWO, lane = x & 63, blk = x >> 6, q = blk % L::NKO, tp = blk / L::NKO;
        const int o = 4 * q + (lane >> 4);
        if (o < NO) v = p[oo + o * H + 16 * tp + (lane & 15)];
    } else if (e < L::BW1) {
        const int k = 2 + (e - L::BWH) / L::WH_SZ, x = (e - L::BWH) % L::WH_SZ;
        const int r = x & 3, lane = (x >> 2) & 63, blk = x >> 8, t = blk % HT, tp = blk / HT;
        v = p[param_off<C, H>(k) + (16 * t + 4 * (lane >> 4) + r) * H + 16 * tp + (lane & 15)];
    } else if (e < L::BIAS) {
        const int x = e - L::BW1, r = x & 3, lane = (x >> 2) & 63, t = x >> 8, i = lane & 15;
        if (i < C) v = p[(16 * t + 4 * (lane >> 4) + r) * IN + i];
    } else {
        const int x = e - L::BIAS, li = x / (HT * 16), y = x % (HT * 16), o = y;   // o = 16t + 4g + r
        if (li < NH - 1) v = p[param_off<C, H>(li + 2) + H * H + o];
        else if (o < NO) v = p[oo + NO * H + o];
    }
    blob[e] = v;
}

// One lane's share of a sample: the texel offsets and weights of its 8 taps (its 4 channels),
// the loaded texel words, and the direction values of its layer-1 slots.
struct TmFetch {
    int off[8];
    float w[8];
    f32x4 v[8];
    f32x4 dv;
    bool finite;
};

template <int C>
__device__ __forceinline__ void tm_issue(const TrainArgs& a, const LevelRow* lrows, int tile, int g, int s,
                                         TmFetch& f) {
    const int i = tile * 16 + s;
    const int ic = i < a.n ? i : a.n - 1;
    const bool fetching = C == 16 || g < 2;
    const int cg = fetching ? 4 * g : 0;
    if (a.z_in) {
        // the sample's given code: channels 4g..4g+3 as a single tap of weight 1; the code is
        // finite only if all C channels are (the other lanes of the sample hold the rest)
        f.v[0] = ld4(a.z_in + (int64_t)ic * C + cg);
        f.w[0] = 1.0f;
        #pragma unroll
        for (int k = 1; k < 8; ++k) {
            f.v[k] = f32x4{0, 0, 0, 0};
            f.w[k] = 0.0f;
            f.off[k] = 0;
        }
        f.off[0] = 0;
        int ok = !fetching || (__builtin_isfinite(f.v[0][0]) && __builtin_isfinite(f.v[0][1]) &&
                               __builtin_isfinite(f.v[0][2]) && __builtin_isfinite(f.v[0][3]));
        ok &= __shfl_xor(ok, 16, 64);
        ok &= __shfl_xor(ok, 32, 64);
        f.finite = ok != 0;
    } else {
        const float2 q = reinterpret_cast<const float2*>(a.uv)[ic];
        const float l = a.lod[ic];
        f.finite = query_ok(q.x, q.y, l);
        Taps t;
        query_taps_rows(lrows, a.M, a.address, q.x, q.y, l, t);
        #pragma unroll
        for (int k = 0; k < 8; ++k) {
            f.off[k] = (int)t.idx[k] * C + cg;
            f.w[k] = t.w[k];
        }
        if (fetching) {
            #pragma unroll
            for (int k = 0; k < 8; ++k) f.v[k] = ld4(a.tex + f.off[k]);
        }
    }
    auto dir = [&](int d) { return d < 3 ? a.wi[3 * ic + d] : a.wo[3 * ic + d - 3]; };
    if (C == 16) {
        f.dv[0] = dir(g);
        f.dv[1] = g < 2 ? dir(4 + g) : (g == 2 ? 1.0f : 0.0f);
        f.dv[2] = 0.0f;
        f.dv[3] = 0.0f;
    } else if (g == 2) {
        f.dv = f32x4{dir(0), dir(1), dir(2), dir(3)};
    } else if (g == 3) {
        f.dv = f32x4{dir(4), dir(5), 1.0f, 0.0f};
    }
}

// Row sums over the 16 lanes of a lane group (lanes 16g..16g+15).
__device__ __forceinline__ float sum16(float v) {
    #pragma unroll
    for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int C, int H, int NH, bool TRAIN>
__global__ void __launch_bounds__(kTMThreads, 1) train_mfma_kernel(const TrainArgs a) {
    using L = TrainLayout<C, H, NH>;
    constexpr int HT = L::HT, Q1 = L::Q1, G1 = L::G1, NCT1 = L::NCT1, NKO = L::NKO;
    constexpr int FX = L::FX, FA = L::FA, FD = L::FD;
    __shared__ __attribute__((aligned(16))) float smem[L::LDS_FLOATS];
    __shared__ LevelRow lrows[kMaxLevels];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, s = lane & 15;
    const float* blob = smem;
    float* sw = smem + L::BLOB + wave * L::SCR;
    float* X0 = sw;
    float* MA = sw + L::SA;            // a_k at MA + (k - 1) * 16 * FA
    float* MD = sw + L::SD;            // output deltas
    const int NO = a.NO;

    // decoder blocks to LDS; the scratch's never-written padding columns of X0 to zero
    for (int e = tid; e < L::BLOB / 4; e += kTMThreads)
        st4(smem + 4 * e, ld4(a.blob + 4 * e));
    for (int e = tid; e < kTMWaves * 16 * FX; e += kTMThreads) {
        const int w = e / (16 * FX), x = e % (16 * FX);
        smem[L::BLOB + w * L::SCR + x] = 0.0f;
    }
    if (tid < a.M) lrows[tid] = a.rows[tid];
    __syncthreads();

    f32x4 dW1[HT][NCT1], dWh[NH > 1 ? NH - 1 : 1][HT][HT], dWo[HT];
    float dbh[NH > 1 ? NH - 1 : 1][HT][4], dbo[4];
    if (TRAIN) {
        #pragma unroll
        for (int t = 0; t < HT; ++t) {
            #pragma unroll
            for (int c = 0; c < NCT1; ++c) dW1[t][c] = f32x4{0, 0, 0, 0};
            dWo[t] = f32x4{0, 0, 0, 0};
            #pragma unroll
            for (int k = 0; k < NH - 1; ++k) {
                #pragma unroll
                for (int c = 0; c < HT; ++c) dWh[k][t][c] = f32x4{0, 0, 0, 0};
                #pragma unroll
                for (int r = 0; r < 4; ++r) dbh[k][t][r] = 0.0f;
            }
        }
        #pragma unroll
        for (int r = 0; r < 4; ++r) dbo[r] = 0.0f;
    }
    float loss_acc = 0.0f;
    float absmax = 0.0f;

    const int tiles = (a.n + 15) / 16;
    const int waves = gridDim.x * kTMWaves;
    const int wid = blockIdx.x * kTMWaves + wave;
    const bool fetching = C == 16 || g < 2;

    TmFetch cur, nxt;
    if (wid < tiles) tm_issue<C>(a, lrows, wid, g, s, cur);
    for (int tile = wid; tile < tiles; tile += waves) {
        if (tile + waves < tiles) tm_issue<C>(a, lrows, tile + waves, g, s, nxt);
        const int i = tile * 16 + s;
        const bool in_range = i < a.n;
        const bool live = in_range && cur.finite;

        // ---- blend and the layer-1 input (zero for samples that contribute nothing)
        float x0[Q1];
        {
            f32x4 z = f32x4{0, 0, 0, 0};
            if (fetching) {
                #pragma unroll
                for (int k = 0; k < 8; ++k) z += cur.w[k] * cur.v[k];
            }
            if constexpr (C == 16) {
                #pragma unroll
                for (int q = 0; q < 4; ++q) x0[q] = z[q];
                x0[4] = cur.dv[0];
                x0[5] = cur.dv[1];
            } else {
                #pragma unroll
                for (int q = 0; q < 4; ++q) x0[q] = fetching ? z[q] : cur.dv[q];
            }
            #pragma unroll
            for (int q = 0; q < Q1; ++q) x0[q] = live ? x0[q] : 0.0f;
            if (TRAIN) {
                if constexpr (C == 16) {
                    st4(X0 + s * FX + 4 * g, f32x4{x0[0], x0[1], x0[2], x0[3]});
                    X0[s * FX + C + g] = x0[4];
                    X0[s * FX + C + 4 + g] = x0[5];
                } else {
                    st4(X0 + s * FX + 4 * g, f32x4{x0[0], x0[1], x0[2], x0[3]});
                }
            }
        }

        // ---- forward
        f32x4 act[HT];
        {
            f32x4 acc[HT];
            #pragma unroll
            for (int t = 0; t < HT; ++t) acc[t] = f32x4{0, 0, 0, 0};
            #pragma unroll
            for (int grp = 0; grp < G1; ++grp) {
                #pragma unroll
                for (int t = 0; t < HT; ++t) {
                    const f32x4 A = ld4(blob + L::FW1 + ((t * G1 + grp) * 64 + lane) * 4);
                    #pragma unroll
                    for (int qq = 0; qq < 4; ++qq)
                        if (4 * grp + qq < Q1) acc[t] = mfma_f32(A[qq], x0[4 * grp + qq], acc[t]);
                }
            }
            #pragma unroll
            for (int t = 0; t < HT; ++t) {
                #pragma unroll
                for (int r = 0; r < 4; ++r) act[t][r] = fmaxf(acc[t][r], 0.0f);
                if (TRAIN) st4(MA + s * FA + 16 * t + 4 * g, act[t]);
            }
        }
        #pragma unroll
        for (int k = 2; k <= NH; ++k) {
            f32x4 acc[HT];
            #pragma unroll
            for (int t = 0; t < HT; ++t) acc[t] = ld4(blob + L::BIAS + ((k - 2) * HT + t) * 16 + 4 * g);
            #pragma unroll
            for (int t = 0; t < HT; ++t) {
                #pragma unroll
                for (int tp = 0; tp < HT; ++tp) {
                    const f32x4 A = ld4(blob + L::FWH + (k - 2) * L::WH_SZ + ((tp * HT + t) * 64 + lane) * 4);
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) acc[tp] = mfma_f32(A[r], act[t][r], acc[tp]);
                }
            }
            #pragma unroll
            for (int t = 0; t < HT; ++t) {
                #pragma unroll
                for (int r = 0; r < 4; ++r) act[t][r] = fmaxf(acc[t][r], 0.0f);
                if (TRAIN) st4(MA + (k - 1) * 16 * FA + s * FA + 16 * t + 4 * g, act[t]);
            }
        }
        f32x4 qo = ld4(blob + L::BIAS + (NH - 1) * HT * 16 + 4 * g);
        #pragma unroll
        for (int t = 0; t < HT; ++t) {
            const f32x4 A = ld4(blob + L::FWO + (t * 64 + lane) * 4);
            #pragma unroll
            for (int r = 0; r < 4; ++r) qo = mfma_f32(A[r], act[t][r], qo);
        }

        if (!TRAIN) {
            if (in_range) {
                #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 4 * g + r;
                    if (row < NO) a.rgb[(int64_t)NO * i + row] = cur.finite ? tm_softplus(qo[r]) : __builtin_nanf("");
                }
            }
        } else {
            // ---- output deltas: dL/dq = dL/dy * logistic(q)
            f32x4 dq = f32x4{0, 0, 0, 0};
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 4 * g + r;
                if (row < NO && live) {
                    float gy;
                    if (a.target) {
                        const float e = tm_softplus(qo[r]) - a.target[(int64_t)NO * i + row];
                        loss_acc = fmaf(e, e, loss_acc);
                        gy = 2.0f * e * a.inv_count;
                    } else {
                        gy = a.d_rgb[(int64_t)NO * i + row];
                    }
                    dq[r] = gy * tm_logistic(qo[r]);
                }
                dbo[r] += dq[r];
            }
            st4(MD + s * FD + 4 * g, dq);
            lds_sync_wave();
            float* An = MA + (NH - 1) * 16 * FA;       // a_NH
            // dW_out += delta_out a_NH^T (samples on K)
            {
                float Ad[4];
                #pragma unroll
                for (int r = 0; r < 4; ++r) Ad[r] = MD[(4 * g + r) * FD + s];
                #pragma unroll
                for (int c = 0; c < HT; ++c) {
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) dWo[c] = mfma_f32(Ad[r], An[(4 * g + r) * FA + 16 * c + s], dWo[c]);
                }
            }
            // delta_NH = W_out^T delta_out, masked by a_NH > 0
            f32x4 dl[HT];
            {
                float B[NKO];
                #pragma unroll
                for (int q = 0; q < NKO; ++q) B[q] = MD[s * FD + 4 * q + g];
                #pragma unroll
                for (int tp = 0; tp < HT; ++tp) {
                    f32x4 acc = f32x4{0, 0, 0, 0};
                    #pragma unroll
                    for (int q = 0; q < NKO; ++q) acc = mfma_f32(blob[L::BWO + (tp * NKO + q) * 64 + lane], B[q], acc);
                    const f32x4 m = ld4(An + s * FA + 16 * tp + 4 * g);
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) dl[tp][r] = m[r] > 0.0f ? acc[r] : 0.0f;
                }
            }
            // hidden layers k = NH .. 2: dW_k, then delta_{k-1}
            #pragma unroll
            for (int k = NH; k >= 2; --k) {
                float* Ak = MA + (k - 1) * 16 * FA;     // a_k, overwritten by delta_k
                float* Ap = MA + (k - 2) * 16 * FA;     // a_{k-1}
                #pragma unroll
                for (int t = 0; t < HT; ++t) {
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) dbh[k - 2][t][r] += dl[t][r];
                    st4(Ak + s * FA + 16 * t + 4 * g, dl[t]);
                }
                lds_sync_wave();
                {
                    float Ad[HT][4], Bv[HT][4];
                    #pragma unroll
                    for (int c = 0; c < HT; ++c) {
                        #pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            Ad[c][r] = Ak[(4 * g + r) * FA + 16 * c + s];
                            Bv[c][r] = Ap[(4 * g + r) * FA + 16 * c + s];
                        }
                    }
                    #pragma unroll
                    for (int co = 0; co < HT; ++co) {
                        #pragma unroll
                        for (int cj = 0; cj < HT; ++cj) {
                            #pragma unroll
                            for (int r = 0; r < 4; ++r) dWh[k - 2][co][cj] = mfma_f32(Ad[co][r], Bv[cj][r], dWh[k - 2][co][cj]);
                        }
                    }
                }
                f32x4 acc[HT];
                #pragma unroll
                for (int tp = 0; tp < HT; ++tp) acc[tp] = f32x4{0, 0, 0, 0};
                #pragma unroll
                for (int t = 0; t < HT; ++t) {
                    #pragma unroll
                    for (int tp = 0; tp < HT; ++tp) {
                        const f32x4 A = ld4(blob + L::BWH + (k - 2) * L::WH_SZ + ((tp * HT + t) * 64 + lane) * 4);
                        #pragma unroll
                        for (int r = 0; r < 4; ++r) acc[tp] = mfma_f32(A[r], dl[t][r], acc[tp]);
                    }
                }
                #pragma unroll
                for (int tp = 0; tp < HT; ++tp) {
                    const f32x4 m = ld4(Ap + s * FA + 16 * tp + 4 * g);
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) dl[tp][r] = m[r] > 0.0f ? acc[tp][r] : 0.0f;
                }
            }
            // delta_1 -> dW_1 (with the bias column), then the gradient of the latent code
            #pragma unroll
            for (int t = 0; t < HT; ++t) st4(MA + s * FA + 16 * t + 4 * g, dl[t]);
            lds_sync_wave();
            {
                float Ad[HT][4], Bx[NCT1][4];
                #pragma unroll
                for (int r = 0; r < 4; ++r) {
                    #pragma unroll
                    for (int c = 0; c < HT; ++c) Ad[c][r] = MA[(4 * g + r) * FA + 16 * c + s];
                    #pragma unroll
                    for (int c = 0; c < NCT1; ++c) Bx[c][r] = X0[(4 * g + r) * FX + 16 * c + s];
                }
                #pragma unroll
                for (int co = 0; co < HT; ++co) {
                    #pragma unroll
                    for (int cj = 0; cj < NCT1; ++cj) {
                        #pragma unroll
                        for (int r = 0; r < 4; ++r) dW1[co][cj] = mfma_f32(Ad[co][r], Bx[cj][r], dW1[co][cj]);
                    }
                }
            }
            f32x4 dz = f32x4{0, 0, 0, 0};
            #pragma unroll
            for (int t = 0; t < HT; ++t) {
                const f32x4 A = ld4(blob + L::BW1 + (t * 64 + lane) * 4);
                #pragma unroll
                for (int r = 0; r < 4; ++r) dz = mfma_f32(A[r], dl[t][r], dz);
            }
            // lane (g, s) holds channels 4g..4g+3 of sample s (C = 8: lanes g < 2)
            if (a.dz) {
                if (in_range && fetching) {
                    const f32x4 v = live ? dz : f32x4{0, 0, 0, 0};
                    st4(a.dz + (int64_t)i * C + 4 * g, v);
                    #pragma unroll
                    for (int r = 0; r < 4; ++r) absmax = fmaxf(absmax, __builtin_isfinite(v[r]) ? fabsf(v[r]) : __builtin_inff());
                }
            } else {
                // scatter into the texels, C lanes per sample: in round r, lane (u, c) =
                // (lane / C, lane % C) adds channel c of sample r (64 / C) + u, so one atomic
                // instruction covers 64 / C whole texels and the memory side takes each texel as
                // one request (with the lanes of the accumulator layout it took a quarter of a
                // texel per request).  Channel c of sample q is component c % 4 of lane
                // 16 (c / 4) + q; the taps of sample q are in lane q, whose offsets point at
                // channel 0.  Every lane runs the exchanges; only live samples add.
                constexpr int SPR = 64 / C;
                const int u = lane / C, c = lane % C;
                #pragma unroll
                for (int r = 0; r < 16 / SPR; ++r) {
                    const int q = r * SPR + u;
                    const int src = 16 * (c >> 2) + q;
                    const float d0 = __shfl(dz[0], src), d1 = __shfl(dz[1], src);
                    const float d2 = __shfl(dz[2], src), d3 = __shfl(dz[3], src);
                    const int cc = c & 3;
                    const float d = cc == 0 ? d0 : (cc == 1 ? d1 : (cc == 2 ? d2 : d3));
                    const bool lq = __shfl((int)live, q) != 0;
                    #pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int o = __shfl(cur.off[k], q);
                        const float w = __shfl(cur.w[k], q);
                        if (lq) unsafeAtomicAdd(a.d_tex + o + c, w * d);
                    }
                }
            }
        }
        cur = nxt;
    }

    if (!TRAIN) return;
    // ---- this wave's gradients into its own partial slice (every parameter written once)
    float* part = a.partial + (size_t)wid * a.np;
    constexpr int IN = C + 6;
    #pragma unroll
    for (int co = 0; co < HT; ++co) {
        #pragma unroll
        for (int cj = 0; cj < NCT1; ++cj) {
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * co + 4 * g + r, j = 16 * cj + s;
                if (j < IN) part[o * IN + j] = dW1[co][cj][r];
                else if (j == IN) part[IN * H + o] = dW1[co][cj][r];
            }
        }
    }
    #pragma unroll
    for (int k = 2; k <= NH; ++k) {
        const int off = param_off<C, H>(k);
        #pragma unroll
        for (int co = 0; co < HT; ++co) {
            #pragma unroll
            for (int cj = 0; cj < HT; ++cj) {
                #pragma unroll
                for (int r = 0; r < 4; ++r) part[off + (16 * co + 4 * g + r) * H + 16 * cj + s] = dWh[k - 2][co][cj][r];
            }
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float b = sum16(dbh[k - 2][co][r]);
                if (s == 0) part[off + H * H + 16 * co + 4 * g + r] = b;
            }
        }
    }
    {
        const int off = param_off<C, H>(NH + 1);
        #pragma unroll
        for (int c = 0; c < HT; ++c) {
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 4 * g + r;
                if (o < NO) part[off + o * H + 16 * c + s] = dWo[c][r];
            }
        }
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float b = sum16(dbo[r]);
            const int o = 4 * g + r;
            if (s == 0 && o < NO) part[off + NO * H + o] = b;
        }
    }
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        loss_acc += __shfl_xor(loss_acc, o, 64);
        absmax = fmaxf(absmax, __shfl_xor(absmax, o, 64));
    }
    if (lane == 0) {
        a.loss_partial[wid] = loss_acc;
        if (a.dz && a.dz_absmax && absmax > 0.0f) atomicMax(a.dz_absmax, __float_as_uint(absmax));
    }
}

// pack: pack the decoder from params into blob; run: launch the kernel on the packed blob
template <int C, int H, int NH>
static hipError_t launch_tm_shape(bool pack, bool run, bool train, const float* params, int NO, float* blob,
                                  const TrainArgs& a, int grid, hipStream_t st) {
    using L = TrainLayout<C, H, NH>;
    clear_stale_hip_error();
    if (pack) {
        pack_train_kernel<C, H, NH><<<(L::BLOB + 255) / 256, 256, 0, st>>>(params, NO, blob);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || !run) return e;
    }
    if (train) train_mfma_kernel<C, H, NH, true><<<grid, kTMThreads, 0, st>>>(a);
    else train_mfma_kernel<C, H, NH, false><<<grid, kTMThreads, 0, st>>>(a);
    return hipGetLastError();
}

bool train_mfma_supported(const MlpShape& sh) {
    return (sh.C == 8 || sh.C == 16) && (sh.H == 32 || sh.H == 64) && (sh.NH == 2 || sh.NH == 3) &&
           (sh.NO == 3 || sh.NO == 6) && sh.NF == 0;
}

int train_mfma_blob_floats(const MlpShape& sh) {
#define NAM_TM_SZ(C_, H_, NH_) if (sh.C == C_ && sh.H == H_ && sh.NH == NH_) return TrainLayout<C_, H_, NH_>::BLOB;
    NAM_TM_SZ(8, 32, 2) NAM_TM_SZ(8, 32, 3) NAM_TM_SZ(8, 64, 2) NAM_TM_SZ(8, 64, 3)
    NAM_TM_SZ(16, 32, 2) NAM_TM_SZ(16, 32, 3) NAM_TM_SZ(16, 64, 2) NAM_TM_SZ(16, 64, 3)
#undef NAM_TM_SZ
    return 0;
}

static hipError_t dispatch_tm(const MlpShape& sh, bool pack, bool run, bool train, const float* params, float* blob,
                              const TrainArgs& a, int grid, hipStream_t st) {
#define NAM_TM_CASE(C_, H_, NH_) \
    if (sh.C == C_ && sh.H == H_ && sh.NH == NH_) \
        return launch_tm_shape<C_, H_, NH_>(pack, run, train, params, sh.NO, blob, a, grid, st);
    NAM_TM_CASE(8, 32, 2) NAM_TM_CASE(8, 32, 3) NAM_TM_CASE(8, 64, 2) NAM_TM_CASE(8, 64, 3)
    NAM_TM_CASE(16, 32, 2) NAM_TM_CASE(16, 32, 3) NAM_TM_CASE(16, 64, 2) NAM_TM_CASE(16, 64, 3)
#undef NAM_TM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_train_mfma(const MlpShape& sh, bool train, const float* params, float* blob, const TrainArgs& a,
                             int grid, hipStream_t st) {
    return dispatch_tm(sh, true, true, train, params, blob, a, grid, st);
}

// ---- plain FP32 decodes on the FP32 matrix cores: the forward kernel on a blob packed once
// per material, followed by one loss slot per wave (the kernel writes them; nothing reads them)
static bool decode_f32_mfma_supported(const nam_material* m) {
    return train_mfma_supported(m->shape) && m->texel_count * m->desc.channels < (int64_t(1) << 31);
}

hipError_t prepare_decode_f32_mfma(nam_material* m) {
    if (!decode_f32_mfma_supported(m)) return hipSuccess;
    const size_t floats = (size_t)train_mfma_blob_floats(m->shape) + (size_t)4 * m->ctx->cu_count;
    float* blob = nullptr;
    hipError_t e = hipMalloc(&blob, floats * sizeof(float));
    if (e != hipSuccess) return e;
    e = dispatch_tm(m->shape, true, false, false, m->params32, blob, TrainArgs{}, 0, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(blob);
        return e;
    }
    m->fblob = blob;
    m->fblob_bytes = floats * sizeof(float);
    return hipSuccess;
}

hipError_t launch_decode_f32_mfma(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* wi,
                                  const float* wo, float* rgb, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (!m->fblob || n > INT32_MAX) return hipErrorInvalidValue;
    // persistent: one workgroup of 4 waves per CU at most, 16 queries per tile
    const int64_t tiles = (n + 15) / 16;
    int64_t waves = (int64_t)m->ctx->cu_count * 4;
    if (waves > tiles) waves = tiles;
    const int grid = (int)((waves + 3) / 4);
    TrainArgs a{};
    a.rows = m->rows;
    a.M = m->desc.levels;
    a.address = (int)m->desc.address;
    a.tex = m->texels32;
    a.params = m->params32;
    a.wt = m->fblob;
    a.blob = m->fblob;
    a.n = (int)n;
    a.uv = uv;
    a.lod = lod;
    a.wi = wi;
    a.wo = wo;
    a.rgb = rgb;
    a.NO = m->shape.NO;
    a.loss_partial = m->fblob + train_mfma_blob_floats(m->shape);
    return dispatch_tm(m->shape, false, true, false, nullptr, m->fblob, a, grid, st);
}

}  // namespace nam
