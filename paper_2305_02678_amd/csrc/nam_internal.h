// Internal declarations of libnam shared by the host API and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <string>
#include <vector>

#include "nam.h"

namespace nam {

constexpr int kMaxLevels = 16;
constexpr int kMaxLayers = 5;      // up to 4 hidden layers + output layer
constexpr int kMaxWidth = 64;

// One row per pyramid level, resident on the device next to the texels.  Kernels index it
// with a per-lane level number (16 bytes per row, one load per level per query).
struct LevelRow {
    int32_t w, h;       // texels along x and y
    int64_t off;        // first texel of the level in the concatenated pyramid
};

// Everything a fetch needs, passed to kernels by value.
struct PyrArgs {
    const LevelRow* rows;   // device, [M]
    int M;                  // number of levels
    int address;            // NAM_WRAP / NAM_CLAMP
};

// Decoder shape supported by the kernels: C + 6 inputs, NH hidden layers of width H, 3 outputs.
struct MlpShape {
    int C, H, NH;
    int NF = 0;                               // learned shading frames (0: T is the identity)
    int NO = 3;                               // decoder outputs: 3 (RGB) or 6 (RGB, then albedo)
    int n_layers() const { return NH + 1; }
    int dir_groups() const { return NF > 1 ? NF : 1; }   // 3-vectors per direction in the input
    int in_dim() const { return C + 6 * dir_groups(); }
};

// Looks up the current device's copy of the static region used by nam_loss_backward_noalloc
// (once per device; *out = NULL if the lookup failed).
void bind_fixed_scratch(int device, void** out);

}  // namespace nam

struct nam_row_table {
    int width, height, levels;
    nam::LevelRow* dev;
};

struct nam_ctx {
    int device = 0;
    int cu_count = 0;
    // scratch for nam_texel_footprint (bitmap) and nam_calibrate (absmax)
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    // training: transposed weights + per-workgroup partial gradients + loss partials
    void* train_ws = nullptr;
    size_t train_ws_bytes = 0;
    // nam_train_step: gradient buffers of texels and parameters
    void* grad_ws = nullptr;
    size_t grad_ws_bytes = 0;
    // deterministic training mode (nam_set_deterministic): per-sample latent-code gradients,
    // their largest magnitude and the 64-bit fixed-point texel accumulators
    int deterministic = 0;
    void* det_ws = nullptr;
    size_t det_ws_bytes = 0;
    std::vector<nam_row_table> row_tables;   // device level tables of pyramid shapes seen
    // this device's copy of the library's static region (nam_loss_backward_noalloc); not owned
    void* fixed_scratch = nullptr;
};

struct nam_material {
    nam_ctx* ctx = nullptr;
    nam_pyramid_desc desc{};
    nam::MlpShape shape{};
    std::vector<int> dims;
    std::vector<float> host_params;           // FP32 master copy of the decoder
    std::vector<nam::LevelRow> host_rows;
    int64_t texel_count = 0;                  // over all levels

    nam::LevelRow* rows = nullptr;            // device
    float* texels32 = nullptr;                // device, [texel_count][C]
    __half* texels16 = nullptr;               // device, [texel_count][C] when quantised
    float* params32 = nullptr;                // device, packed as given
    float* wt32 = nullptr;                    // device, FP32 weights transposed per layer [in][out]
    float* frames32 = nullptr;                // device, FP32 frame layer W_F[6N][C] then b_F[6N]
    uint32_t* frames16 = nullptr;             // device, W_F[6N][C/2] as FP16 pairs, then b_F[6N] FP32
    std::vector<float> host_frames;
    // importance-sampling decoder on [z, wi] (9 outputs), FP32, transposed per layer [in][out]
    float* swt32 = nullptr;
    std::vector<int> sdims;
    std::vector<float> host_sparams;
    nam::MlpShape sshape{};
    void* smfma = nullptr;                    // device, the sampling decoder packed for the matrix cores
    size_t smfma_bias_offset = 0;             // (FP16; quantised materials only), bytes to its biases
    float* fblob = nullptr;                   // device, the FP32 decoder packed for the FP32 matrix cores
                                              // (plain FP32 decodes; decoders the training kernel takes)
    size_t fblob_bytes = 0;
    void* wmfma = nullptr;                    // device, MFMA-packed low-precision decoder
    size_t wmfma_bytes = 0;
    size_t wmfma_bias_offset = 0;             // bytes from wmfma to the bias blocks

    nam_dtype wprec = NAM_F32;
    nam_dtype tprec = NAM_F32;
    int first_layer_f16 = 0;
    // E4M3 scaling: layer L's accumulator holds its pre-activation times S_L (S_L = weight
    // scale * input scale for an E4M3 layer, 1 for an FP16 layer)
    float in_scale = 1.0f;                    // input scale of layer 0 (1 if FP16)
    float mid_scale[nam::kMaxLayers] = {1, 1, 1, 1, 1};  // s_in(L+1) / S_L
    float out_scale = 1.0f;                   // 1 / S_NH
    float w_scale[nam::kMaxLayers] = {};      // per layer weight scale (E4M3 layers)
    float a_scale[nam::kMaxLayers] = {};      // per layer input scale (E4M3 layers)
    int server_refs = 0;

    nam::PyrArgs pyr() const { return nam::PyrArgs{rows, desc.levels, (int)desc.address}; }
};

// ---------------------------------------------------------------------------- errors
namespace nam {
nam_status set_error(nam_status s, const std::string& msg);
nam_status hip_error(hipError_t e, const char* what);
}  // namespace nam

#define NAM_HIP(call)                                                  \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return nam::hip_error(_e, #call);        \
    } while (0)

// --------------------------------------------------------------------- kernel launchers
// Each returns hipSuccess or the launch error; arguments are validated by the caller.
namespace nam {
// A launch's error is read back with hipGetLastError, which would also return an error left
// on this thread by an earlier runtime call of another library; clear it right before.
inline void clear_stale_hip_error() { (void)hipGetLastError(); }

hipError_t launch_fetch(const nam_material* m, int64_t n, const float* uv, const float* lod, float* z,
                        hipStream_t s);
hipError_t launch_footprint(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                            uint32_t* bitmap, hipStream_t s);
hipError_t launch_popcount(const uint32_t* bitmap, int64_t words, unsigned long long* count, hipStream_t s);
// xi: per-query draws for the Russian-roulette level choice, or nullptr for trilinear filtering
hipError_t launch_decode_f32(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                             const float* wi, const float* wo, float* rgb, hipStream_t s);
// Plain trilinear FP32 decodes on the FP32 matrix cores (the training kernel's forward), for the
// decoders that kernel takes (C in {8, 16}, H in {32, 64}, 2 or 3 hidden layers, 3 or 6
// outputs, no frames; 32-bit texel offsets): prepare packs the decoder into m->fblob once and
// leaves it null where unsupported; the launch needs it (n below 2^31).
hipError_t prepare_decode_f32_mfma(nam_material* m);
hipError_t launch_decode_f32_mfma(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* wi,
                                  const float* wo, float* rgb, hipStream_t s);
hipError_t launch_calibrate_f32(const nam_material* m, int64_t n, const float* uv, const float* lod,
                                const float* wi, const float* wo, unsigned int* absmax_bits, hipStream_t s);
// One matrix-core launch over up to 8 batches (n[i] queries of material m[i], each below
// 2^30) whose materials share a kernel (mfma_same_kernel); trilinear filter.
bool mfma_same_kernel(const nam_material* a, const nam_material* b);
hipError_t launch_decode_mfma_group(int count, const nam_material* const* m, const int64_t* n, const float* const* uv,
                                    const float* const* lod, const float* const* wi, const float* const* wo,
                                    float* const* rgb, hipStream_t s);
hipError_t launch_sampler(const nam_material* m, int64_t n, int mode, const float* uv, const float* lod,
                          const float* wi, const float* wo_in, const float* u, float* params_out, float* wo_out,
                          float* pdf_out, hipStream_t s);
// The sampler of a quantised material on the matrix cores (FP16 sampling decoder, m->smfma).
hipError_t launch_sampler_mfma(const nam_material* m, int64_t n, int mode, const float* uv, const float* lod,
                               const float* wi, const float* wo_in, const float* u, float* params_out, float* wo_out,
                               float* pdf_out, hipStream_t s);
hipError_t launch_proxy(int64_t n, const float* params, const float* wi, const float* wo_in, const float* u,
                        float* wo_out, float* pdf_out, hipStream_t s);
hipError_t launch_texels_to_f16(const float* src, __half* dst, int64_t count, hipStream_t s);
hipError_t launch_decode_mfma(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                              const float* wi, const float* wo, float* rgb, hipStream_t s);
bool mfma_shape_supported(const MlpShape& sh);
// A sampling decoder (dims C + 3, H, ..., 9; FP32 params) packed in FP16 for the matrix-core
// sampler into a new device buffer *out (bias blocks at *bias_offset bytes).
nam_status pack_sampler_mfma(nam_ctx* ctx, const std::vector<int>& dims, const std::vector<float>& params, void** out,
                             size_t* bias_offset);
}  // namespace nam
