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
    // deterministic mode: the latent-code gradient of every sample is written to dz [n][C]
    // (zero for skipped samples) instead of being scattered with float atomics, and the largest
    // |dz| is folded into *dz_absmax (float bits; a max does not depend on the order)
    float* dz;
    unsigned int* dz_absmax;
    // latent codes given per sample ([n][C], the encoder's first training phase): used in
    // place of the texel fetch (uv, lod, tex and d_tex unused); dz receives their gradient,
    // and a sample whose code has a non-finite component contributes nothing
    const float* z_in;
    // matrix-core kernels: the decoder's packed operand blocks and the number of outputs
    const float* blob;
    int NO;
    // learned shading frames (vector kernel): W_F[6 NF][C] then b_F[6 NF]; params is then the
    // decoder that follows them, and np counts both
    const float* fparams;
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
// The vector kernel with learned shading frames (sh.NF in {1, 2}; C in {8, 16}, H in {32, 64},
// 2 or 3 hidden layers, 3 outputs); hipErrorInvalidValue for other shapes.
bool train_frames_supported(const MlpShape& sh);
hipError_t launch_fwdbwd_frames(const MlpShape& sh, int mode, const TrainArgs& a, int grid, hipStream_t s);
int fwdbwd_frames_blocks_per_cu(const MlpShape& sh, int mode);
// Overwrites partial (the per-slice sums are reduced in place).
hipError_t launch_reduce_partials(float* partial, int blocks, int np, float* out, hipStream_t s);
hipError_t launch_reduce_loss(const float* part, int blocks, float inv_count, float* loss, hipStream_t s);
hipError_t launch_transpose_params(const float* p, float* wt, const LayerDims& L, hipStream_t s);
hipError_t launch_adam(int64_t count, float* p, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
int fwdbwd_blocks_per_cu(const MlpShape& sh, int mode);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t count, float v, hipStream_t s);
// The level table of a pyramid computed on the device (no host copy): rows[l] for l < levels.
hipError_t launch_level_rows(int width, int height, int levels, LevelRow* rows, hipStream_t s);
// Matrix-core training path (decoders C in {8, 16}, H in {32, 64}, 2 or 3 hidden layers, no
// frames): packs the decoder into blob (train_mfma_blob_floats(sh) floats), then runs the
// forward (train = false) or the forward-backward kernel, grid workgroups of 4 waves; partial
// and loss_partial hold one slice per wave.
bool train_mfma_supported(const MlpShape& sh);
int train_mfma_blob_floats(const MlpShape& sh);
hipError_t launch_train_mfma(const MlpShape& sh, bool train, const float* params, float* blob, const TrainArgs& a,
                             int grid, hipStream_t st);
// Deterministic scatter of dz into the texels: fixed-point 64-bit integer atomics (exactly
// associative) into acc [texels][C], then d_tex += acc scaled back.
hipError_t launch_det_scatter(const LevelRow* rows, int M, int address, int C, int n, const float* uv, const float* lod,
                              const float* dz, const unsigned int* absmax, long long* acc, float* d_tex, hipStream_t s);
// The encoder of Sec. 5.1 (encoder.hip): its weights packed as a decoder's.
struct EncoderArgs {
    const LevelRow* rows;     // the parameter pyramid's level table (queries)
    int M;
    int address;
    const float* attrs;       // queries: the parameter pyramid [texels][A]; bake: rows [n][A]
    const float* params;      // packed encoder
    int n;
    const float* uv;          // queries
    const float* lod;
    float* z;                 // forward: [n][C]
    const float* dz;          // backward: [n][C]
    float* partial;           // backward: [grid][np]
    int np;
};

bool encoder_shape_supported(int A, int C, int HE, int NHE);
// mode 0: the encoder on parameter rows; 1: on the parameters filtered at queries; 2: the
// gradient of its parameters into a.partial (grid workgroups, one slice each)
hipError_t launch_encoder(int A, int C, int HE, int NHE, int mode, const EncoderArgs& a, int grid, hipStream_t s);
hipError_t launch_det_finish(int64_t count, const long long* acc, const unsigned int* absmax, int n, float* d_tex,
                             hipStream_t s);

}  // namespace nam
