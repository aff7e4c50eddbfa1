// Host side of the differentiation entry points: argument checks, workspace, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "train_internal.h"

namespace nam {

nam_status check_pyramid(const nam_pyramid_desc* d);
nam_status check_decoder_frames(const nam_mlp_desc* mlp, int C, int nf, MlpShape* out);
std::vector<LevelRow> pyramid_rows(const nam_pyramid_desc& d, int64_t* total);

// Device region of nam_loss_backward_noalloc: the level table, the decoder's operand blocks
// (or transposed weights), the per-wave partial gradients and the loss partials live here
// instead of in context-owned allocations.  Every GPU the library runs on holds its own copy
// until the process ends.  In host code the array's name is not a device address: kernels and
// copies take the address hipGetSymbolAddress returned for the current device.
constexpr size_t kFixedScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
std::string g_scratch_error[kMaxDevices];
}  // namespace

// Called by nam_create with `device` current: looks up this device's copy of the region once.
// A failed lookup is remembered and reported by nam_loss_backward_noalloc; nothing else needs it.
void bind_fixed_scratch(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device] && g_scratch_error[device].empty()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            g_scratch_error[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        } else {
            g_scratch_ptr[device] = p;
        }
    }
    *out = g_scratch_ptr[device];
}

const char* fixed_scratch_error(int device) {
    if (device < 0 || device >= kMaxDevices) return "device index beyond the library's table";
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_error[device].empty() ? "static scratch not bound" : g_scratch_error[device].c_str();
}

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Model {
    MlpShape shape;
    LayerDims dims;                   // the decoder
    int nfp = 0;                      // frame-layer parameters ahead of the decoder (6 NF (C + 1))
    int np() const { return nfp + dims.total; }
    int64_t texels = 0;
    const LevelRow* rows = nullptr;   // device table (owned by the context cache)
};

// Device copy of a pyramid's level table, cached per pyramid shape in the context.
nam_status level_table(nam_ctx* ctx, const nam_pyramid_desc& d, const LevelRow** out, int64_t* total) {
    const std::vector<LevelRow> rows = pyramid_rows(d, total);
    for (auto& e : ctx->row_tables) {
        if (e.levels == d.levels && e.width == d.width && e.height == d.height) {
            *out = e.dev;
            return NAM_OK;
        }
    }
    LevelRow* dev = nullptr;
    NAM_HIP(hipMalloc(&dev, sizeof(LevelRow) * kMaxLevels));
    hipError_t e = hipMemcpy(dev, rows.data(), sizeof(LevelRow) * rows.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_error(e, "hipMemcpy(level table)");
    }
    ctx->row_tables.push_back({d.width, d.height, d.levels, dev});
    *out = dev;
    return NAM_OK;
}

// Shape of a model from its descriptor (no device work, no allocation); texels counted on
// the host.
nam_status model_shape(const nam_model_desc* md, Model* m) {
    if (!md) return set_error(NAM_E_INVALID_ARG, "model descriptor is NULL");
    nam_status s = check_pyramid(&md->pyramid);
    if (s != NAM_OK) return s;
    if (md->n_frames < 0 || md->n_frames > 2) return set_error(NAM_E_UNSUPPORTED, "n_frames must be 0, 1 or 2");
    s = check_decoder_frames(&md->mlp, md->pyramid.channels, md->n_frames, &m->shape);
    if (s != NAM_OK) return s;
    if (md->n_frames > 0 && !train_frames_supported(m->shape))
        return set_error(NAM_E_UNSUPPORTED, "training with learned shading frames supports C in {8, 16}, hidden "
                                            "widths 32 or 64, 2 or 3 hidden layers and 3 outputs");
    m->nfp = 6 * md->n_frames * md->pyramid.channels + 6 * md->n_frames;
    const int K = md->mlp.n_layers;
    int o = 0;
    m->dims.n_layers = K;
    for (int k = 0; k < K; ++k) {
        m->dims.off[k] = o;
        m->dims.in[k] = md->mlp.dims[k];
        m->dims.out[k] = md->mlp.dims[k + 1];
        o += md->mlp.dims[k] * md->mlp.dims[k + 1] + md->mlp.dims[k + 1];
    }
    m->dims.off[K] = o;
    m->dims.total = o;
    int64_t texels = 0;
    for (int l = 0; l < md->pyramid.levels; ++l) {
        const int64_t w = md->pyramid.width >> l > 0 ? md->pyramid.width >> l : 1;
        const int64_t h = md->pyramid.height >> l > 0 ? md->pyramid.height >> l : 1;
        texels += w * h;
    }
    m->texels = texels;
    return NAM_OK;
}

nam_status make_model(nam_ctx* ctx, const nam_model_desc* md, Model* m) {
    nam_status s = model_shape(md, m);
    if (s != NAM_OK) return s;
    return level_table(ctx, md->pyramid, &m->rows, &m->texels);
}

nam_status grow(void** buf, size_t* have, size_t need) {
    if (*have >= need) return NAM_OK;
    (void)hipFree(*buf);
    *buf = nullptr;
    *have = 0;
    NAM_HIP(hipMalloc(buf, need));
    *have = need;
    return NAM_OK;
}

nam_status check_batch(int64_t n, const float* uv, const float* lod, const float* wi, const float* wo) {
    if (n < 0) return set_error(NAM_E_INVALID_ARG, "n must be >= 0");
    if (n > (int64_t(1) << 31) - 64) return set_error(NAM_E_UNSUPPORTED, "at most 2^31 - 64 samples per call");
    if (n > 0 && (!uv || !lod || !wi || !wo)) return set_error(NAM_E_INVALID_ARG, "sample pointer is NULL");
    if (n > 0 && ((reinterpret_cast<uintptr_t>(uv) & 7) != 0)) return set_error(NAM_E_INVALID_ARG, "uv must be 8-byte aligned");
    return NAM_OK;
}

// A fixed device region that replaces the context's allocations (the no-allocation entry
// point): the level table at its start, then the training workspace.
struct FixedWs {
    char* base;
    size_t bytes;
};
constexpr size_t kRowsBytes = 256;      // kMaxLevels rows of 16 bytes

// Shared body of forward / backward / loss-backward.
// Codes mode (z_in non-null, the encoder's first training phase): the latent codes are given
// per sample instead of fetched; uv, lod and the texels are not read, dz_out receives the codes'
// gradient, and the deterministic mode changes nothing (no scatter).
nam_status run(nam_ctx* ctx, const nam_model_desc* md, int mode, const float* texels, const float* params,
               int64_t n, const float* uv, const float* lod, const float* wi, const float* wo, const float* target,
               const float* d_rgb, float* rgb, float* d_texels, float* d_params, float* loss, hipStream_t st,
               const FixedWs* fws = nullptr, const float* z_in = nullptr, float* dz_out = nullptr) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    const bool codes = z_in != nullptr;
    nam_status s = codes ? check_batch(n, z_in, z_in, wi, wo) : check_batch(n, uv, lod, wi, wo);
    if (s != NAM_OK) return s;
    if ((!codes && !texels) || !params) return set_error(NAM_E_INVALID_ARG, "texels or params is NULL");
    if (fws && ctx->deterministic && mode != kModeForward)
        return set_error(NAM_E_UNSUPPORTED, "the deterministic mode needs per-call device memory; use nam_loss_backward");
    DeviceGuard g(ctx->device);
    Model m;
    s = fws ? model_shape(md, &m) : make_model(ctx, md, &m);
    if (s != NAM_OK) return s;
    const int np = m.np();
    // the matrix-core kernels address texel channels with 32-bit offsets
    const bool mfma = train_mfma_supported(m.shape) && m.texels * md->pyramid.channels < (int64_t(1) << 31);
    int grid, slices;
    if (mfma) {
        // one workgroup of 4 waves per CU (the decoder's blocks fill most of the LDS); one
        // partial slice per wave, 16 samples per tile
        const int64_t tiles = (n + 15) / 16;
        int64_t waves = (int64_t)ctx->cu_count * 4;
        if (waves > tiles) waves = tiles;
        grid = (int)((waves + 3) / 4);
        if (grid < 1) grid = 1;
        slices = grid * 4;
    } else {
        const int64_t nchunks = (n + 63) / 64;
        grid = ctx->cu_count * fwdbwd_blocks_per_cu(m.shape, mode);
        if (grid > nchunks) grid = (int)nchunks;
        if (grid < 1) grid = 1;
        slices = grid;
    }

    // workspace: transposed weights (or the matrix-core operand blocks), per-workgroup (per-wave)
    // partial gradients, per-workgroup (per-wave) loss sums
    const size_t wt_floats = mfma ? (size_t)train_mfma_blob_floats(m.shape) : (size_t)np;
    const size_t wt_bytes = (wt_floats * 4 + 255) / 256 * 256;
    char* ws;
    if (fws) {
        // as many partial slices as the region holds (whole workgroups); fewer slices only
        // mean fewer workgroups over the same samples
        const size_t fixed_bytes = kRowsBytes + wt_bytes + 256 * 2;
        const size_t per_slice = (size_t)np * 4 + 4;
        int64_t max_slices = fws->bytes > fixed_bytes ? (int64_t)((fws->bytes - fixed_bytes) / per_slice) : 0;
        if (mfma) max_slices -= max_slices % 4;
        if (max_slices < (mfma ? 4 : 1))
            return set_error(NAM_E_UNSUPPORTED,
                             "the decoder's gradients do not fit the library's static scratch (" +
                                 std::to_string(fws->bytes >> 20) + " MiB; " + std::to_string(np) + " parameters)");
        if (slices > max_slices) {
            slices = (int)max_slices;
            grid = mfma ? slices / 4 : slices;
        }
        LevelRow* rows = reinterpret_cast<LevelRow*>(fws->base);
        NAM_HIP(launch_level_rows(md->pyramid.width, md->pyramid.height, md->pyramid.levels, rows, st));
        m.rows = rows;
        ws = fws->base + kRowsBytes;
    }
    const size_t part_bytes = mode == kModeForward ? 0 : ((size_t)slices * np * 4 + 255) / 256 * 256;
    const size_t loss_bytes = (size_t)slices * 4;
    if (!fws) {
        s = grow(&ctx->train_ws, &ctx->train_ws_bytes, wt_bytes + part_bytes + loss_bytes);
        if (s != NAM_OK) return s;
        ws = static_cast<char*>(ctx->train_ws);
    }
    float* wt = reinterpret_cast<float*>(ws);
    float* partial = mode == kModeForward ? nullptr : reinterpret_cast<float*>(ws + wt_bytes);
    float* loss_part = reinterpret_cast<float*>(ws + wt_bytes + part_bytes);

    const float* dec = params + m.nfp;       // the decoder after the frame layer
    if (!mfma) NAM_HIP(launch_transpose_params(dec, wt, m.dims, st));
    if (n == 0) {
        if (d_params) NAM_HIP(launch_fill_f32(d_params, np, 0.0f, st));
        if (loss) NAM_HIP(launch_fill_f32(loss, 1, 0.0f, st));
        return NAM_OK;
    }
    TrainArgs a{};
    a.rows = m.rows;
    a.M = md->pyramid.levels;
    a.address = (int)md->pyramid.address;
    a.tex = texels;
    a.d_tex = d_texels;
    a.params = dec;
    a.fparams = m.nfp ? params : nullptr;
    a.wt = wt;
    a.partial = partial;
    a.np = np;
    a.n = (int)n;
    a.uv = uv;
    a.lod = lod;
    a.wi = wi;
    a.wo = wo;
    a.target = target;
    a.d_rgb = d_rgb;
    a.rgb = rgb;
    a.inv_count = (float)(1.0 / (3.0 * (double)n));
    a.loss_partial = loss_part;
    long long* det_acc = nullptr;
    a.z_in = z_in;
    if (codes) {
        a.dz = dz_out;
        a.dz_absmax = nullptr;
    } else if (ctx->deterministic && mode != kModeForward) {
        // [dz: n x C floats][absmax: 256 B][acc: texels x C int64]
        const size_t C = (size_t)md->pyramid.channels;
        const size_t dz_bytes = ((size_t)n * C * 4 + 255) / 256 * 256;
        const size_t acc_bytes = (size_t)m.texels * C * 8;
        s = grow(&ctx->det_ws, &ctx->det_ws_bytes, dz_bytes + 256 + acc_bytes);
        if (s != NAM_OK) return s;
        char* dw = static_cast<char*>(ctx->det_ws);
        a.dz = reinterpret_cast<float*>(dw);
        a.dz_absmax = reinterpret_cast<unsigned int*>(dw + dz_bytes);
        det_acc = reinterpret_cast<long long*>(dw + dz_bytes + 256);
        NAM_HIP(launch_zero(dw + dz_bytes, 256 + acc_bytes, st));
    }
    a.blob = wt;
    a.NO = m.shape.NO;
    if (mfma) NAM_HIP(launch_train_mfma(m.shape, mode != kModeForward, dec, wt, a, grid, st));
    else NAM_HIP(launch_fwdbwd(m.shape, mode, a, grid, st));
    if (det_acc) {
        NAM_HIP(launch_det_scatter(m.rows, a.M, a.address, md->pyramid.channels, a.n, uv, lod, a.dz, a.dz_absmax,
                                   det_acc, d_texels, st));
        NAM_HIP(launch_det_finish(m.texels * md->pyramid.channels, det_acc, a.dz_absmax, a.n, d_texels, st));
    }
    if (mode != kModeForward) NAM_HIP(launch_reduce_partials(partial, slices, np, d_params, st));
    if (mode == kModeLoss && loss) NAM_HIP(launch_reduce_loss(loss_part, slices, a.inv_count, loss, st));
    return NAM_OK;
}

// Encoder shape (A parameters -> hidden layers of one width -> C) from its descriptor.
nam_status encoder_shape(const nam_mlp_desc* e, int* A, int* C, int* HE, int* NHE, int* np) {
    if (!e || !e->dims) return set_error(NAM_E_INVALID_ARG, "encoder descriptor is NULL");
    const int K = e->n_layers;
    if (K < 2 || K > 3) return set_error(NAM_E_UNSUPPORTED, "the encoder must have 1 or 2 hidden layers");
    *A = e->dims[0];
    *C = e->dims[K];
    *HE = e->dims[1];
    *NHE = K - 1;
    for (int k = 1; k < K; ++k)
        if (e->dims[k] != *HE) return set_error(NAM_E_UNSUPPORTED, "the encoder's hidden widths must be equal");
    if (!encoder_shape_supported(*A, *C, *HE, *NHE))
        return set_error(NAM_E_UNSUPPORTED, "encoder: 4, 8 or 16 parameters, hidden width 16, 32 or 64, 8 or 16 outputs");
    int64_t p = 0;
    for (int k = 0; k < K; ++k) p += (int64_t)e->dims[k] * e->dims[k + 1] + e->dims[k + 1];
    *np = (int)p;
    return NAM_OK;
}

// The parameter pyramid of the encoder's queries: a latent-pyramid geometry with A channels.
nam_status encoder_pyramid(nam_ctx* ctx, const nam_pyramid_desc* d, int A, const LevelRow** rows) {
    if (!d) return set_error(NAM_E_INVALID_ARG, "parameter pyramid descriptor is NULL");
    if (d->channels != A) return set_error(NAM_E_SHAPE, "the parameter pyramid's channels must equal the encoder's inputs");
    nam_pyramid_desc g = *d;
    g.channels = 8;                   // the geometry checks of a latent pyramid
    nam_status s = check_pyramid(&g);
    if (s != NAM_OK) return s;
    int64_t total = 0;
    return level_table(ctx, g, rows, &total);
}

nam_status adam_args(const nam_adam_cfg* cfg, float* c1, float* c2) {
    if (!cfg) return set_error(NAM_E_INVALID_ARG, "Adam configuration is NULL");
    if (cfg->step < 1) return set_error(NAM_E_INVALID_ARG, "Adam step counts from 1");
    if (!(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f && cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f && cfg->eps > 0.0f))
        return set_error(NAM_E_INVALID_ARG, "Adam needs 0 <= beta < 1 and eps > 0");
    *c1 = (float)(1.0 - std::pow((double)cfg->beta1, (double)cfg->step));
    *c2 = (float)(1.0 - std::pow((double)cfg->beta2, (double)cfg->step));
    return NAM_OK;
}

}  // namespace

}  // namespace nam

using namespace nam;

extern "C" {

nam_status nam_forward(nam_ctx* ctx, const nam_model_desc* md, const float* texels, const float* params, int64_t n,
                       const float* uv, const float* lod, const float* wi, const float* wo, float* rgb, void* stream) {
    if (n > 0 && !rgb) return set_error(NAM_E_INVALID_ARG, "rgb is NULL");
    return run(ctx, md, kModeForward, texels, params, n, uv, lod, wi, wo, nullptr, nullptr, rgb, nullptr, nullptr,
               nullptr, (hipStream_t)stream);
}

nam_status nam_backward(nam_ctx* ctx, const nam_model_desc* md, const float* texels, const float* params, int64_t n,
                        const float* uv, const float* lod, const float* wi, const float* wo, const float* d_rgb,
                        float* d_texels, float* d_params, void* stream) {
    if (!d_params || (n > 0 && (!d_rgb || !d_texels))) return set_error(NAM_E_INVALID_ARG, "gradient pointer is NULL");
    return run(ctx, md, kModeGrad, texels, params, n, uv, lod, wi, wo, nullptr, d_rgb, nullptr, d_texels, d_params,
               nullptr, (hipStream_t)stream);
}

nam_status nam_loss_backward(nam_ctx* ctx, const nam_model_desc* md, const float* texels, const float* params,
                             int64_t n, const float* uv, const float* lod, const float* wi, const float* wo,
                             const float* target, float* d_texels, float* d_params, float* loss, void* stream) {
    if (!d_params || (n > 0 && (!target || !d_texels))) return set_error(NAM_E_INVALID_ARG, "gradient pointer is NULL");
    return run(ctx, md, kModeLoss, texels, params, n, uv, lod, wi, wo, target, nullptr, nullptr, d_texels, d_params,
               loss, (hipStream_t)stream);
}

nam_status nam_loss_backward_noalloc(nam_ctx* ctx, const nam_model_desc* md, const float* texels,
                                     const float* params, int64_t n, const float* uv, const float* lod, const float* wi,
                                     const float* wo, const float* target, float* d_texels, float* d_params, float* loss,
                                     void* stream) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    if (!d_params || (n > 0 && (!target || !d_texels))) return set_error(NAM_E_INVALID_ARG, "gradient pointer is NULL");
    if (!ctx->fixed_scratch) return set_error(NAM_E_HIP, fixed_scratch_error(ctx->device));
    const FixedWs fws{static_cast<char*>(ctx->fixed_scratch), kFixedScratchBytes};
    return run(ctx, md, kModeLoss, texels, params, n, uv, lod, wi, wo, target, nullptr, nullptr, d_texels, d_params,
               loss, (hipStream_t)stream, &fws);
}

nam_status nam_set_deterministic(nam_ctx* ctx, int on) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    if (on != 0 && on != 1) return set_error(NAM_E_INVALID_ARG, "deterministic must be 0 or 1");
    ctx->deterministic = on;
    return NAM_OK;
}

nam_status nam_adam_update(nam_ctx* ctx, int64_t count, float* p, float* m, float* v, const float* g,
                           const nam_adam_cfg* cfg, void* stream) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    if (count < 0) return set_error(NAM_E_INVALID_ARG, "count must be >= 0");
    if (count > 0 && (!p || !m || !v || !g)) return set_error(NAM_E_INVALID_ARG, "Adam pointer is NULL");
    float c1, c2;
    nam_status s = adam_args(cfg, &c1, &c2);
    if (s != NAM_OK) return s;
    if (count == 0) return NAM_OK;
    DeviceGuard gd(ctx->device);
    NAM_HIP(launch_adam(count, p, m, v, g, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2, (hipStream_t)stream));
    return NAM_OK;
}

nam_status nam_train_step(nam_ctx* ctx, const nam_model_desc* md, float* texels, float* params, float* m_texels,
                          float* v_texels, float* m_params, float* v_params, int64_t n, const float* uv,
                          const float* lod, const float* wi, const float* wo, const float* target,
                          const nam_adam_cfg* cfg, float* loss, void* stream) {
    if (!ctx || !md) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    if (!texels || !params || !m_texels || !v_texels || !m_params || !v_params)
        return set_error(NAM_E_INVALID_ARG, "parameter or optimiser-state pointer is NULL");
    if (n > 0 && !target) return set_error(NAM_E_INVALID_ARG, "target is NULL");
    float c1, c2;
    nam_status s = adam_args(cfg, &c1, &c2);
    if (s != NAM_OK) return s;
    DeviceGuard g(ctx->device);
    Model m;
    s = make_model(ctx, md, &m);
    if (s != NAM_OK) return s;
    const int64_t tex_count = m.texels * md->pyramid.channels;
    const int np = m.np();
    const size_t gtex_bytes = ((size_t)tex_count * 4 + 255) / 256 * 256;
    s = grow(&ctx->grad_ws, &ctx->grad_ws_bytes, gtex_bytes + (size_t)np * 4);
    if (s != NAM_OK) return s;
    float* g_tex = static_cast<float*>(ctx->grad_ws);
    float* g_par = reinterpret_cast<float*>(static_cast<char*>(ctx->grad_ws) + gtex_bytes);
    hipStream_t st = (hipStream_t)stream;
    NAM_HIP(hipMemsetAsync(g_tex, 0, (size_t)tex_count * 4, st));
    s = run(ctx, md, kModeLoss, texels, params, n, uv, lod, wi, wo, target, nullptr, nullptr, g_tex, g_par, loss, st);
    if (s != NAM_OK) return s;
    NAM_HIP(launch_adam(np, params, m_params, v_params, g_par, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2, st));
    NAM_HIP(launch_adam(tex_count, texels, m_texels, v_texels, g_tex, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2,
                        st));
    return NAM_OK;
}

nam_status nam_loss_backward_codes(nam_ctx* ctx, const nam_model_desc* md, const float* params, int64_t n,
                                   const float* z, const float* wi, const float* wo, const float* target, float* dz,
                                   float* d_params, float* loss, void* stream) {
    if (!d_params || (n > 0 && (!target || !dz || !z))) return set_error(NAM_E_INVALID_ARG, "NULL pointer");
    return run(ctx, md, kModeLoss, nullptr, params, n, nullptr, nullptr, wi, wo, target, nullptr, nullptr, nullptr,
               d_params, loss, (hipStream_t)stream, nullptr, z, dz);
}

static nam_status encoder_run(nam_ctx* ctx, const nam_mlp_desc* enc, const float* eparams, int mode,
                              const nam_pyramid_desc* pyr, const float* attrs, int64_t n, const float* uv,
                              const float* lod, float* z, const float* dz, float* d_eparams, void* stream) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    int A, C, HE, NHE, np;
    nam_status s = encoder_shape(enc, &A, &C, &HE, &NHE, &np);
    if (s != NAM_OK) return s;
    if (n < 0) return set_error(NAM_E_INVALID_ARG, "n must be >= 0");
    if (n > (int64_t(1) << 31) - 256) return set_error(NAM_E_UNSUPPORTED, "at most 2^31 - 256 items per call");
    if (!eparams || (mode == 2 && !d_eparams)) return set_error(NAM_E_INVALID_ARG, "parameter pointer is NULL");
    if (n > 0 && (!attrs || (mode < 2 ? !z : !dz) || (mode >= 1 && (!uv || !lod))))
        return set_error(NAM_E_INVALID_ARG, "input or output pointer is NULL");
    if (mode >= 1 && n > 0 && (reinterpret_cast<uintptr_t>(uv) & 7) != 0)
        return set_error(NAM_E_INVALID_ARG, "uv must be 8-byte aligned");
    DeviceGuard g(ctx->device);
    EncoderArgs a{};
    if (mode >= 1) {
        s = encoder_pyramid(ctx, pyr, A, &a.rows);
        if (s != NAM_OK) return s;
        a.M = pyr->levels;
        a.address = (int)pyr->address;
    }
    a.attrs = attrs;
    a.params = eparams;
    a.n = (int)n;
    a.uv = uv;
    a.lod = lod;
    a.z = z;
    a.dz = dz;
    a.np = np;
    hipStream_t st = (hipStream_t)stream;
    if (mode < 2) {
        if (n == 0) return NAM_OK;
        NAM_HIP(launch_encoder(A, C, HE, NHE, mode, a, 0, st));
        return NAM_OK;
    }
    if (n == 0) {
        NAM_HIP(launch_fill_f32(d_eparams, np, 0.0f, st));
        return NAM_OK;
    }
    // one wave per workgroup; a partial slice per workgroup, reduced in a fixed order
    const int64_t nchunks = (n + 63) / 64;
    int grid = ctx->cu_count * 4;
    if (grid > nchunks) grid = (int)nchunks;
    s = grow(&ctx->train_ws, &ctx->train_ws_bytes, (size_t)grid * np * 4);
    if (s != NAM_OK) return s;
    a.partial = static_cast<float*>(ctx->train_ws);
    NAM_HIP(launch_encoder(A, C, HE, NHE, 2, a, grid, st));
    NAM_HIP(launch_reduce_partials(a.partial, grid, np, d_eparams, st));
    return NAM_OK;
}

nam_status nam_encode_texels(nam_ctx* ctx, const nam_mlp_desc* encoder, const float* eparams, int64_t n,
                             const float* attrs, float* z, void* stream) {
    return encoder_run(ctx, encoder, eparams, 0, nullptr, attrs, n, nullptr, nullptr, z, nullptr, nullptr, stream);
}

nam_status nam_encode_queries(nam_ctx* ctx, const nam_mlp_desc* encoder, const float* eparams,
                              const nam_pyramid_desc* params_pyramid, const float* attrs, int64_t n, const float* uv,
                              const float* lod, float* z, void* stream) {
    return encoder_run(ctx, encoder, eparams, 1, params_pyramid, attrs, n, uv, lod, z, nullptr, nullptr, stream);
}

nam_status nam_encoder_backward(nam_ctx* ctx, const nam_mlp_desc* encoder, const float* eparams,
                                const nam_pyramid_desc* params_pyramid, const float* attrs, int64_t n,
                                const float* uv, const float* lod, const float* dz, float* d_eparams, void* stream) {
    return encoder_run(ctx, encoder, eparams, 2, params_pyramid, attrs, n, uv, lod, nullptr, dz, d_eparams, stream);
}

}  // extern "C"
