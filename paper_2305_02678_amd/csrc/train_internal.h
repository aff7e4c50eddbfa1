// Shared declarations of the differentiation kernels and their host launchers.
#pragma once

#include "nam_internal.h"

namespace nam {

constexpr int kModeForward = 0;   // rgb only
constexpr int kModeLoss = 1;      // mean squared error against targets, gradients of it
constexpr int kModeGrad = 2;      // gradients of sum(d_rgb * rgb) for a given d_rgb

struct TrainArgs {
    const LevelRow* rows;         // device level table
    int M;                        // levels
    int address;                  // NAM_WRAP / NAM_CLAMP
    const float* tex;             // [texels][C]
    float* d_tex;                 // [texels][C], accumulated (+=)
    const float* params;          // packed W_k [out][in], b_k
    const float* wt;              // per layer W_k^T [in][out], b_k
    float* partial;               // [grid][np] per-workgroup parameter gradients
    int np;
    int n;
    const float* uv;
    const float* lod;
    const float* wi;
    const float* wo;
    const float* target;          // kModeLoss
    const float* d_rgb;           // kModeGrad
    float* rgb;                   // kModeForward
    float inv_count;              // 1 / (3 n)
    float* loss_partial;          // [grid]
};

struct LayerDims {
    int n_layers;
    int off[kMaxLayers + 1];
    int in[kMaxLayers];
    int out[kMaxLayers];
    int total;
};

// Orders a wave's LDS writes before its later LDS reads by other lanes (waits for the LDS
// counter only) and keeps the compiler from moving memory operations across.
__device__ __forceinline__ void lds_sync_wave() {
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
}

hipError_t launch_fwdbwd(const MlpShape& sh, int mode, const TrainArgs& a, int grid, hipStream_t s);
hipError_t launch_reduce_partials(const float* partial, int blocks, int np, float* out, hipStream_t s);
hipError_t launch_reduce_loss(const float* part, int blocks, float inv_count, float* loss, hipStream_t s);
hipError_t launch_transpose_params(const float* p, float* wt, const LayerDims& L, hipStream_t s);
hipError_t launch_adam(int64_t count, float* p, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
int fwdbwd_blocks_per_cu(const MlpShape& sh, int mode);

}  // namespace nam
