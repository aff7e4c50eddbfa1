// Host side of the differentiation entry points: argument checks, workspace, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "train_internal.h"

namespace nam {

nam_status check_pyramid(const nam_pyramid_desc* d);
nam_status check_decoder(const nam_mlp_desc* mlp, int C, MlpShape* out);
std::vector<LevelRow> pyramid_rows(const nam_pyramid_desc& d, int64_t* total);

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
    LayerDims dims;
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

nam_status make_model(nam_ctx* ctx, const nam_model_desc* md, Model* m) {
    if (!md) return set_error(NAM_E_INVALID_ARG, "model descriptor is NULL");
    nam_status s = check_pyramid(&md->pyramid);
    if (s != NAM_OK) return s;
    s = check_decoder(&md->mlp, md->pyramid.channels, &m->shape);
    if (s != NAM_OK) return s;
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

// Shared body of forward / backward / loss-backward.
nam_status run(nam_ctx* ctx, const nam_model_desc* md, int mode, const float* texels, const float* params,
               int64_t n, const float* uv, const float* lod, const float* wi, const float* wo, const float* target,
               const float* d_rgb, float* rgb, float* d_texels, float* d_params, float* loss, hipStream_t st) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    nam_status s = check_batch(n, uv, lod, wi, wo);
    if (s != NAM_OK) return s;
    if (!texels || !params) return set_error(NAM_E_INVALID_ARG, "texels or params is NULL");
    DeviceGuard g(ctx->device);
    Model m;
    s = make_model(ctx, md, &m);
    if (s != NAM_OK) return s;
    const int np = m.dims.total;
    const int64_t nchunks = (n + 63) / 64;
    int grid = ctx->cu_count * fwdbwd_blocks_per_cu(m.shape, mode);
    if (grid > nchunks) grid = (int)nchunks;
    if (grid < 1) grid = 1;

    // workspace: transposed weights, per-workgroup partials, per-workgroup loss sums
    const size_t wt_bytes = ((size_t)np * 4 + 255) / 256 * 256;
    const size_t part_bytes = mode == kModeForward ? 0 : ((size_t)grid * np * 4 + 255) / 256 * 256;
    const size_t loss_bytes = (size_t)grid * 4;
    s = grow(&ctx->train_ws, &ctx->train_ws_bytes, wt_bytes + part_bytes + loss_bytes);
    if (s != NAM_OK) return s;
    char* ws = static_cast<char*>(ctx->train_ws);
    float* wt = reinterpret_cast<float*>(ws);
    float* partial = mode == kModeForward ? nullptr : reinterpret_cast<float*>(ws + wt_bytes);
    float* loss_part = reinterpret_cast<float*>(ws + wt_bytes + part_bytes);

    NAM_HIP(launch_transpose_params(params, wt, m.dims, st));
    if (n == 0) {
        if (d_params) NAM_HIP(hipMemsetAsync(d_params, 0, (size_t)np * 4, st));
        if (loss) NAM_HIP(hipMemsetAsync(loss, 0, 4, st));
        return NAM_OK;
    }
    TrainArgs a{};
    a.rows = m.rows;
    a.M = md->pyramid.levels;
    a.address = (int)md->pyramid.address;
    a.tex = texels;
    a.d_tex = d_texels;
    a.params = params;
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
    NAM_HIP(launch_fwdbwd(m.shape, mode, a, grid, st));
    if (mode != kModeForward) NAM_HIP(launch_reduce_partials(partial, grid, np, d_params, st));
    if (mode == kModeLoss && loss) NAM_HIP(launch_reduce_loss(loss_part, grid, a.inv_count, loss, st));
    return NAM_OK;
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
    const int np = m.dims.total;
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

}  // extern "C"
