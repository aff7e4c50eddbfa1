// Achievable matrix-core rate and issue cost of vector work beside it, on one gfx950 GPU.
//
// Build and run (one MI355X):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         paper_2305_02678_amd/probes/issue_cost.hip -o /tmp/issue_cost && /tmp/issue_cost
//
// Every launch runs one 16-wave workgroup per compute unit (four waves per SIMD).  Each wave
// loops over a fixed body of matrix-core instructions (FP16 inputs, FP32 accumulation;
// independent accumulators, so no result waits) and V packed-FP16 maximum operations on
// independent registers.  The time per loop body, per SIMD, in cycles of the 2.4 GHz clock,
// gives:
//   * the achievable dense FP16 rate (V = 0), against the 2.5 PFLOP/s datasheet figure;
//   * how many issue cycles one matrix-core instruction takes from the SIMD's vector issue
//     port once vector work fills the gaps: the intercept of time against V at large V, where
//     each added vector instruction costs its own 4 cycles.
// The decoders are bound by that port: their per-chunk cost is about
// (matrix-core instructions) x (intercept per instruction) + 4 x (other vector instructions).
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

constexpr int kBlock = 1024;   // 16 waves: four per SIMD
constexpr int kIters = 2000;

// BIG = 0: eight v_mfma_f32_16x16x32_f16 per body; BIG = 1: four v_mfma_f32_32x32x16_f16 (the
// same FLOPs).  V packed maxima per matrix-core instruction, rotating over 8 registers.
template <int BIG, int V>
__global__ void __launch_bounds__(kBlock) issue_body(float* out, int iters, float seed) {
    half8 a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (_Float16)(seed * (float)(threadIdx.x + i));
        b[i] = (_Float16)(seed - (float)i);
    }
    constexpr int N = BIG ? 4 : 8;
    floatx16 big[N];
    floatx4 small[N];
    for (int c = 0; c < N; ++c) {
        for (int i = 0; i < 16; ++i) big[c][i] = (float)(c + i);
        small[c] = floatx4{0.0f, (float)c, 0.0f, 0.0f};
    }
    half2_t h[8];
    for (int i = 0; i < 8; ++i) h[i] = half2_t{(_Float16)(seed * (float)(i + threadIdx.x)), (_Float16)(seed * (float)i)};
    for (int it = 0; it < iters; ++it) {   // a run-time count: the body is not unrolled
        #pragma unroll
        for (int c = 0; c < N; ++c) {
            if constexpr (BIG) big[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, big[c], 0, 0, 0);
            else small[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, small[c], 0, 0, 0);
            #pragma unroll
            for (int v = 0; v < V; ++v) {
                const int k = (c * V + v) & 7;
                h[k] = __builtin_elementwise_max(h[k], h[(k + 1) & 7]);
            }
        }
    }
    float s = 0.0f;
    for (int c = 0; c < N; ++c) {
        if constexpr (BIG) {
            for (int i = 0; i < 16; ++i) s += big[c][i];
        } else {
            s += small[c][0] + small[c][1] + small[c][2] + small[c][3];
        }
    }
    for (int i = 0; i < 8; ++i) s += (float)h[i][0] + (float)h[i][1];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// SIMD cycles (at 2.4 GHz) per loop body of one wave: the launch time over the bodies each SIMD runs.
template <int BIG, int V>
static double cycles_per_body(float* out, int cus) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    for (int w = 0; w < 20; ++w) issue_body<BIG, V><<<cus, kBlock>>>(out, kIters, 0.001f);
    CHECK(hipGetLastError());
    const int reps = 20;
    CHECK(hipEventRecord(e0));
    for (int r = 0; r < reps; ++r) issue_body<BIG, V><<<cus, kBlock>>>(out, kIters, 0.001f);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    const double bodies_per_simd = (kBlock / 64) / 4.0 * kIters;
    return (ms * 1e-3 / reps) * 2.4e9 / bodies_per_simd;
}

int main() {
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int cus = p.multiProcessorCount;
    float* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * (size_t)cus * kBlock));
    std::printf("device %s, %d CUs; cycles at 2.4 GHz per loop body per SIMD (4 waves per SIMD)\n", p.gcnArchName, cus);
    // the clock ramps up over the first few hundred launches of a sustained load
    for (int w = 0; w < 400; ++w) issue_body<0, 0><<<cus, kBlock>>>(out, kIters, 0.001f);
    CHECK(hipDeviceSynchronize());

    // per wave and body: 8 x 16x16x32 = 4 x 32x32x16 products = 131,072 FLOP
    const double flop_per_body = 8.0 * 16 * 16 * 32 * 2;
    const double c0 = cycles_per_body<0, 0>(out, cus);
    const double b0 = cycles_per_body<1, 0>(out, cus);
    // 4 SIMDs per CU, one body per SIMD per `c` cycles
    const double tf16 = flop_per_body * 4.0 * cus * 2.4e9 / c0 / 1e12;
    const double tf32 = flop_per_body * 4.0 * cus * 2.4e9 / b0 / 1e12;
    std::printf("16x16x32 f16, no vector work: %.1f cycles per body (%.2f per instruction): %.0f TFLOP/s, %.1f%% of 2516.6\n",
                c0, c0 / 8, tf16, 100.0 * tf16 / 2516.6);
    std::printf("32x32x16 f16, no vector work: %.1f cycles per body (%.2f per instruction): %.0f TFLOP/s, %.1f%% of 2516.6\n",
                b0, b0 / 4, tf32, 100.0 * tf32 / 2516.6);

    // vector instructions per body, as read from the assembly of each variant: 24, 40 and 56 packed
    // maxima for the 16x16x32 body with V = 2, 4, 6 and for the 32x32x16 body with V = 4, 8, 12 (the
    // rotation over 8 registers adds 8 to the nominal count)
    const double s1 = cycles_per_body<0, 2>(out, cus), s2 = cycles_per_body<0, 4>(out, cus), s3 = cycles_per_body<0, 6>(out, cus);
    const double g1 = cycles_per_body<1, 4>(out, cus), g2 = cycles_per_body<1, 8>(out, cus), g3 = cycles_per_body<1, 12>(out, cus);
    std::printf("16x16x32 x 8 with 24 / 40 / 56 packed maxima: %.1f / %.1f / %.1f cycles\n", s1, s2, s3);
    std::printf("32x32x16 x 4 with 24 / 40 / 56 packed maxima: %.1f / %.1f / %.1f cycles\n", g1, g2, g3);
    const double slope16 = (s3 - s2) / 16.0, slope32 = (g3 - g2) / 16.0;
    std::printf("cycles per added vector instruction (port-bound range): 16x16x32 body %.2f, 32x32x16 body %.2f\n", slope16, slope32);
    std::printf("issue cycles per matrix-core instruction (intercept at 56 maxima, 4 cycles each): 16x16x32 %.2f, 32x32x16 %.2f\n",
                (s3 - 56 * 4.0) / 8.0, (g3 - 56 * 4.0) / 4.0);
    CHECK(hipFree(out));
    return 0;
}
