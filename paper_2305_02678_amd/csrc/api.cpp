// Host side of the libnam C ABI: argument checks, handles, device copies, kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "mfma_pack.h"
#include "nam_internal.h"

namespace nam {

static thread_local std::string g_last_error;

nam_status set_error(nam_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

nam_status hip_error(hipError_t e, const char* what) {
    if (e == hipErrorOutOfMemory) return set_error(NAM_E_OOM, std::string("out of device memory in ") + what);
    return set_error(NAM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Makes the context's device current for the scope of a call and restores the caller's.
class DeviceGuard {
public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev_ >= 0) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

private:
    int prev_ = -1;
    bool ok_ = true;
};

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static int ilog2(int v) {
    int r = 0;
    while ((1 << (r + 1)) <= v) ++r;
    return r;
}

nam_status check_pyramid(const nam_pyramid_desc* d);
nam_status check_decoder(const nam_mlp_desc* mlp, int C, MlpShape* out);
nam_status check_decoder_frames(const nam_mlp_desc* mlp, int C, int nf, MlpShape* out);
std::vector<LevelRow> pyramid_rows(const nam_pyramid_desc& d, int64_t* total);

static nam_status check_desc(const nam_pyramid_desc* d) {
    if (!d) return set_error(NAM_E_INVALID_ARG, "pyramid descriptor is NULL");
    if (d->address != NAM_WRAP && d->address != NAM_CLAMP)
        return set_error(NAM_E_INVALID_ARG, "address mode must be NAM_WRAP or NAM_CLAMP");
    if (!is_pow2(d->width) || !is_pow2(d->height))
        return set_error(NAM_E_SHAPE, "texture width and height must be powers of two");
    if (d->width > 32768 || d->height > 32768)
        return set_error(NAM_E_UNSUPPORTED, "texture sides above 32768 are not supported");
    const int full = ilog2(d->width > d->height ? d->width : d->height) + 1;
    if (d->levels < 1 || d->levels > full || d->levels > kMaxLevels)
        return set_error(NAM_E_SHAPE, "levels must be in [1, log2(max side) + 1] (and at most 16)");
    if (d->channels != 8 && d->channels != 16)
        return set_error(NAM_E_UNSUPPORTED, "latent channels must be 8 or 16");
    return NAM_OK;
}

static std::vector<LevelRow> level_rows(const nam_pyramid_desc& d, int64_t* total) {
    std::vector<LevelRow> rows(d.levels);
    int64_t off = 0;
    for (int l = 0; l < d.levels; ++l) {
        rows[l].w = d.width >> l > 0 ? d.width >> l : 1;
        rows[l].h = d.height >> l > 0 ? d.height >> l : 1;
        rows[l].off = off;
        off += (int64_t)rows[l].w * rows[l].h;
    }
    *total = off;
    return rows;
}

static nam_status check_mlp(const nam_mlp_desc* mlp, int C, int nf, MlpShape* out) {
    if (!mlp || !mlp->dims) return set_error(NAM_E_INVALID_ARG, "decoder descriptor is NULL");
    const int K = mlp->n_layers;
    if (K < 2 || K > kMaxLayers)
        return set_error(NAM_E_UNSUPPORTED, "decoder must have 1 to 4 hidden layers");
    MlpShape sh{C, 0, K - 1, nf};
    if (mlp->dims[0] != sh.in_dim())
        return set_error(NAM_E_SHAPE, nf > 1 ? "dims[0] must equal channels + 6 * n_frames"
                                             : "dims[0] must equal channels + 6");
    if (mlp->dims[K] != 3 && mlp->dims[K] != 6)
        return set_error(NAM_E_SHAPE, "the last decoder width must be 3 (RGB) or 6 (RGB and albedo)");
    sh.NO = mlp->dims[K];
    const int H = mlp->dims[1];
    for (int k = 1; k < K; ++k)
        if (mlp->dims[k] != H) return set_error(NAM_E_UNSUPPORTED, "hidden widths must all be equal");
    if (H != 16 && H != 32 && H != 64) return set_error(NAM_E_UNSUPPORTED, "hidden width must be 16, 32 or 64");
    sh.H = H;
    *out = sh;
    return NAM_OK;
}

nam_status check_pyramid(const nam_pyramid_desc* d) { return check_desc(d); }
nam_status check_decoder(const nam_mlp_desc* mlp, int C, MlpShape* out) { return check_mlp(mlp, C, 0, out); }
nam_status check_decoder_frames(const nam_mlp_desc* mlp, int C, int nf, MlpShape* out) {
    return check_mlp(mlp, C, nf, out);
}
std::vector<LevelRow> pyramid_rows(const nam_pyramid_desc& d, int64_t* total) { return level_rows(d, total); }

static int64_t param_count(const std::vector<int>& dims) {
    int64_t n = 0;
    for (size_t k = 1; k < dims.size(); ++k) n += (int64_t)dims[k - 1] * dims[k] + dims[k];
    return n;
}

// Per layer: W^T [in][out] followed by the bias, for wave-uniform weight reads.
static std::vector<float> transpose_layers(const std::vector<int>& dims, const std::vector<float>& p) {
    std::vector<float> out(p.size());
    size_t o = 0;
    for (size_t k = 1; k < dims.size(); ++k) {
        const int fi = dims[k - 1], fo = dims[k];
        for (int r = 0; r < fo; ++r)
            for (int j = 0; j < fi; ++j) out[o + (size_t)j * fo + r] = p[o + (size_t)r * fi + j];
        for (int r = 0; r < fo; ++r) out[o + (size_t)fi * fo + r] = p[o + (size_t)fi * fo + r];
        o += (size_t)fi * fo + fo;
    }
    return out;
}

static void free_material_device(nam_material* m) {
    (void)hipFree(m->rows);
    (void)hipFree(m->texels32);
    (void)hipFree(m->texels16);
    (void)hipFree(m->params32);
    (void)hipFree(m->wt32);
    (void)hipFree(m->wmfma);
    (void)hipFree(m->fblob);
    m->fblob = nullptr;
    m->fblob_bytes = 0;
    (void)hipFree(m->frames32);
    (void)hipFree(m->frames16);
    (void)hipFree(m->swt32);
    (void)hipFree(m->smfma);
    m->swt32 = nullptr;
    m->smfma = nullptr;
    m->frames16 = nullptr;
    m->rows = nullptr; m->texels32 = nullptr; m->texels16 = nullptr;
    m->params32 = nullptr; m->wt32 = nullptr; m->wmfma = nullptr; m->frames32 = nullptr;
}

static nam_status check_queries(int64_t n, const void* a, const void* b) {
    if (n < 0) return set_error(NAM_E_INVALID_ARG, "n must be >= 0");
    if (n > 0 && (!a || !b)) return set_error(NAM_E_INVALID_ARG, "query pointer is NULL");
    return NAM_OK;
}

static bool aligned4(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 3) == 0; }

// Largest number of queries per launch (kernels index queries with 32-bit integers).
constexpr int64_t kChunk = int64_t(1) << 30;

static nam_status grow_scratch(nam_ctx* ctx, size_t bytes) {
    if (ctx->scratch_bytes >= bytes) return NAM_OK;
    (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    NAM_HIP(hipMalloc(&ctx->scratch, bytes));
    ctx->scratch_bytes = bytes;
    return NAM_OK;
}

}  // namespace nam

using namespace nam;

extern "C" {

const char* nam_last_error(void) { return g_last_error.c_str(); }

int nam_version(void) { return 100; }

nam_status nam_create(int device, nam_ctx** out) {
    if (!out) return set_error(NAM_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    NAM_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return set_error(NAM_E_INVALID_ARG, "no such HIP device");
    DeviceGuard g(device);
    if (!g.ok()) return set_error(NAM_E_HIP, "hipSetDevice failed");
    hipDeviceProp_t prop;
    NAM_HIP(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(NAM_E_UNSUPPORTED, std::string("libnam is built for gfx950, device is ") + prop.gcnArchName);
    nam_ctx* c = new (std::nothrow) nam_ctx();
    if (!c) return set_error(NAM_E_OOM, "host allocation failed");
    c->device = device;
    c->cu_count = prop.multiProcessorCount;
    bind_fixed_scratch(device, &c->fixed_scratch);
    *out = c;
    return NAM_OK;
}

nam_status nam_destroy(nam_ctx* ctx) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "ctx is NULL");
    DeviceGuard g(ctx->device);
    (void)hipFree(ctx->scratch);
    (void)hipFree(ctx->train_ws);
    (void)hipFree(ctx->grad_ws);
    (void)hipFree(ctx->det_ws);
    for (auto& t : ctx->row_tables) (void)hipFree(t.dev);
    delete ctx;
    return NAM_OK;
}

nam_status nam_pyramid_bytes(const nam_pyramid_desc* desc, nam_dtype texel_type, size_t* bytes) {
    if (!bytes) return set_error(NAM_E_INVALID_ARG, "bytes is NULL");
    nam_status s = check_desc(desc);
    if (s != NAM_OK) return s;
    size_t es;
    switch (texel_type) {
        case NAM_F32: es = 4; break;
        case NAM_F16: es = 2; break;
        case NAM_FP8_E4M3: es = 1; break;
        default: return set_error(NAM_E_INVALID_ARG, "unknown texel type");
    }
    int64_t total = 0;
    level_rows(*desc, &total);
    *bytes = (size_t)total * desc->channels * es;
    return NAM_OK;
}

nam_status nam_material_load(nam_ctx* ctx, const nam_pyramid_desc* desc, const float* const* levels,
                             const nam_mlp_desc* mlp, const float* params, nam_material** out) {
    return nam_material_load_framed(ctx, desc, levels, mlp, params, 0, nullptr, out);
}

nam_status nam_material_load_framed(nam_ctx* ctx, const nam_pyramid_desc* desc, const float* const* levels,
                                    const nam_mlp_desc* mlp, const float* params, int n_frames,
                                    const float* frame_params, nam_material** out) {
    if (!ctx || !levels || !params || !out) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (n_frames < 0 || n_frames > 2) return set_error(NAM_E_UNSUPPORTED, "n_frames must be 0, 1 or 2");
    if (n_frames > 0 && !frame_params) return set_error(NAM_E_INVALID_ARG, "frame_params is NULL");
    nam_status s = check_desc(desc);
    if (s != NAM_OK) return s;
    MlpShape shape;
    s = check_mlp(mlp, desc->channels, n_frames, &shape);
    if (s != NAM_OK) return s;
    for (int l = 0; l < desc->levels; ++l)
        if (!levels[l]) return set_error(NAM_E_INVALID_ARG, "a level pointer is NULL");

    DeviceGuard g(ctx->device);
    if (!g.ok()) return set_error(NAM_E_HIP, "hipSetDevice failed");
    nam_material* m = new (std::nothrow) nam_material();
    if (!m) return set_error(NAM_E_OOM, "host allocation failed");
    m->ctx = ctx;
    m->desc = *desc;
    m->shape = shape;
    m->dims.assign(mlp->dims, mlp->dims + mlp->n_layers + 1);
    const int64_t np = param_count(m->dims);
    m->host_params.assign(params, params + np);
    m->host_rows = level_rows(*desc, &m->texel_count);
    const int C = desc->channels;

    auto fail = [&](nam_status st) { free_material_device(m); delete m; return st; };
    hipError_t e;
    if ((e = hipMalloc(&m->rows, sizeof(LevelRow) * desc->levels)) != hipSuccess) return fail(hip_error(e, "hipMalloc(rows)"));
    if ((e = hipMalloc(&m->texels32, sizeof(float) * m->texel_count * C)) != hipSuccess) return fail(hip_error(e, "hipMalloc(texels)"));
    if ((e = hipMalloc(&m->params32, sizeof(float) * np)) != hipSuccess) return fail(hip_error(e, "hipMalloc(params)"));
    if ((e = hipMalloc(&m->wt32, sizeof(float) * np)) != hipSuccess) return fail(hip_error(e, "hipMalloc(weights)"));
    if ((e = hipMemcpy(m->rows, m->host_rows.data(), sizeof(LevelRow) * desc->levels, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_error(e, "hipMemcpy(rows)"));
    for (int l = 0; l < desc->levels; ++l) {
        const LevelRow& r = m->host_rows[l];
        if ((e = hipMemcpy(m->texels32 + r.off * C, levels[l], sizeof(float) * (size_t)r.w * r.h * C,
                           hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_error(e, "hipMemcpy(level)"));
    }
    if ((e = hipMemcpy(m->params32, params, sizeof(float) * np, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_error(e, "hipMemcpy(params)"));
    const std::vector<float> wt = transpose_layers(m->dims, m->host_params);
    if ((e = hipMemcpy(m->wt32, wt.data(), sizeof(float) * np, hipMemcpyHostToDevice)) != hipSuccess)
        return fail(hip_error(e, "hipMemcpy(weights)"));
    if (n_frames == 0 && (e = prepare_decode_f32_mfma(m)) != hipSuccess)
        return fail(hip_error(e, "packing the FP32 matrix-core decoder"));
    if (n_frames > 0) {
        const size_t nfp = (size_t)6 * n_frames * (C + 1);
        m->host_frames.assign(frame_params, frame_params + nfp);
        if ((e = hipMalloc(&m->frames32, sizeof(float) * nfp)) != hipSuccess) return fail(hip_error(e, "hipMalloc(frames)"));
        if ((e = hipMemcpy(m->frames32, frame_params, sizeof(float) * nfp, hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_error(e, "hipMemcpy(frames)"));
        // the matrix-core decoders' copy: weights as FP16 pairs (round to nearest even), FP32 biases
        const int rows = 6 * n_frames;
        std::vector<uint32_t> h16((size_t)rows * (C / 2) + rows);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < C / 2; ++c) {
                const _Float16 lo = (_Float16)frame_params[r * C + 2 * c], hi = (_Float16)frame_params[r * C + 2 * c + 1];
                uint16_t bl, bh;
                std::memcpy(&bl, &lo, 2);
                std::memcpy(&bh, &hi, 2);
                h16[(size_t)r * (C / 2) + c] = (uint32_t)bl | ((uint32_t)bh << 16);
            }
        std::memcpy(h16.data() + (size_t)rows * (C / 2), frame_params + (size_t)rows * C, sizeof(float) * rows);
        if ((e = hipMalloc(&m->frames16, sizeof(uint32_t) * h16.size())) != hipSuccess)
            return fail(hip_error(e, "hipMalloc(frames16)"));
        if ((e = hipMemcpy(m->frames16, h16.data(), sizeof(uint32_t) * h16.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return fail(hip_error(e, "hipMemcpy(frames16)"));
    }
    *out = m;
    return NAM_OK;
}

nam_status nam_material_footprint(const nam_material* m, size_t* bytes) {
    if (!m || !bytes) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    const size_t np = m->host_params.size();
    size_t b = sizeof(LevelRow) * m->desc.levels + 2 * sizeof(float) * np + m->wmfma_bytes + m->fblob_bytes +
               sizeof(float) * (m->host_frames.size() + m->host_sparams.size()) +
               (m->frames16 ? sizeof(uint32_t) * (size_t)6 * m->shape.NF * (m->desc.channels / 2 + 1) : 0);
    if (m->texels32) b += sizeof(float) * (size_t)m->texel_count * m->desc.channels;
    if (m->texels16) b += sizeof(__half) * (size_t)m->texel_count * m->desc.channels;
    if (m->smfma) {
        const MfmaLayout lay = mfma_layout(m->sshape.C, m->sshape.H, m->sshape.NH, true, false);
        b += (size_t)(lay.a_blocks() + lay.b_blocks()) * 64 * 16;
    }
    *bytes = b;
    return NAM_OK;
}

nam_status nam_material_free(nam_material* m) {
    if (!m) return set_error(NAM_E_INVALID_ARG, "material is NULL");
    if (m->server_refs > 0) return set_error(NAM_E_BUSY, "material is held by a server");
    DeviceGuard g(m->ctx->device);
    free_material_device(m);
    delete m;
    return NAM_OK;
}

nam_status nam_fetch(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod, float* z,
                     void* stream) {
    if (!ctx || !m) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    nam_status s = check_queries(n, uv, lod);
    if (s != NAM_OK) return s;
    if (n > 0 && !z) return set_error(NAM_E_INVALID_ARG, "z is NULL");
    if (n == 0) return NAM_OK;
    if (!aligned4(uv) || !aligned4(lod) || !aligned4(z)) return set_error(NAM_E_INVALID_ARG, "pointers must be 4-byte aligned");
    if (((uintptr_t)uv & 7) != 0) return set_error(NAM_E_INVALID_ARG, "uv must be 8-byte aligned");
    if (((uintptr_t)z & 15) != 0) return set_error(NAM_E_INVALID_ARG, "z must be 16-byte aligned");
    DeviceGuard g(ctx->device);
    const int C = m->desc.channels;
    for (int64_t o = 0; o < n; o += kChunk) {
        const int64_t c = n - o < kChunk ? n - o : kChunk;
        NAM_HIP(launch_fetch(m, c, uv + 2 * o, lod + o, z + o * C, (hipStream_t)stream));
    }
    return NAM_OK;
}

}  // extern "C"

// Distinct texels addressed by the taps of n queries (trilinear, or Russian roulette with xi).
static nam_status texel_footprint(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                                  const float* xi, uint64_t* distinct, void* stream) {
    if (!ctx || !m || !distinct) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    nam_status s = check_queries(n, uv, lod);
    if (s != NAM_OK) return s;
    *distinct = 0;
    if (n == 0) return NAM_OK;
    if (((uintptr_t)uv & 7) != 0 || !aligned4(lod)) return set_error(NAM_E_INVALID_ARG, "misaligned query pointer");
    DeviceGuard g(ctx->device);
    const int64_t words = (m->texel_count + 31) / 32;
    s = grow_scratch(ctx, sizeof(uint32_t) * words + 256);
    if (s != NAM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    uint32_t* bitmap = reinterpret_cast<uint32_t*>(static_cast<char*>(ctx->scratch) + 256);
    unsigned long long* count = reinterpret_cast<unsigned long long*>(ctx->scratch);
    NAM_HIP(hipMemsetAsync(ctx->scratch, 0, sizeof(uint32_t) * words + 256, st));
    for (int64_t o = 0; o < n; o += kChunk) {
        const int64_t c = n - o < kChunk ? n - o : kChunk;
        NAM_HIP(launch_footprint(m, c, uv + 2 * o, lod + o, xi ? xi + o : nullptr, bitmap, st));
    }
    NAM_HIP(launch_popcount(bitmap, words, count, st));
    unsigned long long h = 0;
    NAM_HIP(hipMemcpyAsync(&h, count, sizeof(h), hipMemcpyDeviceToHost, st));
    NAM_HIP(hipStreamSynchronize(st));
    *distinct = h;
    return NAM_OK;
}

extern "C" {

nam_status nam_texel_footprint(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                               uint64_t* distinct, void* stream) {
    return texel_footprint(ctx, m, n, uv, lod, nullptr, distinct, stream);
}

nam_status nam_texel_footprint_stochastic(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv,
                                          const float* lod, const float* xi, uint64_t* distinct, void* stream) {
    if (n > 0 && !xi) return set_error(NAM_E_INVALID_ARG, "NULL draws");
    if (n > 0 && !aligned4(xi)) return set_error(NAM_E_INVALID_ARG, "misaligned draws");
    return texel_footprint(ctx, m, n, uv, lod, xi, distinct, stream);
}

}  // extern "C"

namespace nam {
// One material's decode of n queries on a stream (arguments already checked), in launches of
// at most 2^30 queries.  xi: per-query draws for the Russian-roulette level choice, or nullptr
// for trilinear filtering.
hipError_t decode_launch(const nam_material* m, int64_t n, const float* uv, const float* lod, const float* xi,
                         const float* wi, const float* wo, float* rgb, hipStream_t st) {
    for (int64_t o = 0; o < n; o += kChunk) {
        const int64_t c = n - o < kChunk ? n - o : kChunk;
        const float* x = xi ? xi + o : nullptr;
        // FP32: trilinear decodes on the FP32 matrix cores where the decoder allows, the rest on
        // the vector ALU
        const hipError_t e =
            m->wprec != NAM_F32
                ? launch_decode_mfma(m, c, uv + 2 * o, lod + o, x, wi + 3 * o, wo + 3 * o, rgb + m->shape.NO * o, st)
            : (m->fblob && !x)
                ? launch_decode_f32_mfma(m, c, uv + 2 * o, lod + o, wi + 3 * o, wo + 3 * o, rgb + m->shape.NO * o, st)
                : launch_decode_f32(m, c, uv + 2 * o, lod + o, x, wi + 3 * o, wo + 3 * o, rgb + m->shape.NO * o, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace nam

extern "C" {

nam_status nam_decode(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                      const float* wi, const float* wo, float* rgb, void* stream) {
    if (!ctx || !m) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    nam_status s = check_queries(n, uv, lod);
    if (s != NAM_OK) return s;
    if (n > 0 && (!wi || !wo || !rgb)) return set_error(NAM_E_INVALID_ARG, "query pointer is NULL");
    if (n == 0) return NAM_OK;
    if (((uintptr_t)uv & 7) != 0 || !aligned4(lod) || !aligned4(wi) || !aligned4(wo) || !aligned4(rgb))
        return set_error(NAM_E_INVALID_ARG, "misaligned pointer (uv needs 8 bytes, the rest 4)");
    DeviceGuard g(ctx->device);
    NAM_HIP(decode_launch(m, n, uv, lod, nullptr, wi, wo, rgb, (hipStream_t)stream));
    return NAM_OK;
}

nam_status nam_decode_stochastic(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                                 const float* xi, const float* wi, const float* wo, float* rgb, void* stream) {
    if (!ctx || !m) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    nam_status s = check_queries(n, uv, lod);
    if (s != NAM_OK) return s;
    if (n > 0 && (!xi || !wi || !wo || !rgb)) return set_error(NAM_E_INVALID_ARG, "query pointer is NULL");
    if (n == 0) return NAM_OK;
    if (((uintptr_t)uv & 7) != 0 || !aligned4(lod) || !aligned4(xi) || !aligned4(wi) || !aligned4(wo) ||
        !aligned4(rgb))
        return set_error(NAM_E_INVALID_ARG, "misaligned pointer (uv needs 8 bytes, the rest 4)");
    DeviceGuard g(ctx->device);
    NAM_HIP(decode_launch(m, n, uv, lod, xi, wi, wo, rgb, (hipStream_t)stream));
    return NAM_OK;
}

nam_status nam_calibrate(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                         const float* wi, const float* wo, float* absmax_out, void* stream) {
    if (!ctx || !m || !absmax_out) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    nam_status s = check_queries(n, uv, lod);
    if (s != NAM_OK) return s;
    if (n == 0) return set_error(NAM_E_INVALID_ARG, "calibration needs at least one query");
    if (!wi || !wo) return set_error(NAM_E_INVALID_ARG, "query pointer is NULL");
    if (((uintptr_t)uv & 7) != 0 || !aligned4(lod) || !aligned4(wi) || !aligned4(wo))
        return set_error(NAM_E_INVALID_ARG, "misaligned pointer");
    DeviceGuard g(ctx->device);
    s = grow_scratch(ctx, 256);
    if (s != NAM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    unsigned int* bits = static_cast<unsigned int*>(ctx->scratch);
    NAM_HIP(hipMemsetAsync(bits, 0, sizeof(unsigned int) * kMaxLayers, st));
    for (int64_t o = 0; o < n; o += kChunk) {
        const int64_t c = n - o < kChunk ? n - o : kChunk;
        NAM_HIP(launch_calibrate_f32(m, c, uv + 2 * o, lod + o, wi + 3 * o, wo + 3 * o, bits, st));
    }
    unsigned int h[kMaxLayers];
    NAM_HIP(hipMemcpyAsync(h, bits, sizeof(h), hipMemcpyDeviceToHost, st));
    NAM_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < m->shape.n_layers(); ++k) std::memcpy(&absmax_out[k], &h[k], sizeof(float));
    return NAM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- importance sampling

static nam_status sampler_run(nam_ctx* ctx, const nam_material* m, int64_t n, int mode, const float* uv,
                              const float* lod, const float* wi, const float* wo_in, const float* u,
                              float* params_out, float* wo_out, float* pdf_out, void* stream) {
    if (!ctx || !m) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    if (!m->swt32) return set_error(NAM_E_INVALID_ARG, "the material has no sampling decoder (nam_material_set_sampler)");
    nam_status s = check_queries(n, uv, lod);
    if (s != NAM_OK) return s;
    const void* need[] = {wi, mode == 0 ? (const void*)params_out : (const void*)pdf_out,
                          mode == 1 ? (const void*)wo_in : mode == 2 ? (const void*)u : (const void*)wi,
                          mode == 2 ? (const void*)wo_out : (const void*)wi};
    for (const void* q : need)
        if (n > 0 && !q) return set_error(NAM_E_INVALID_ARG, "query pointer is NULL");
    if (n == 0) return NAM_OK;
    for (const void* q : {(const void*)lod, (const void*)wi, (const void*)wo_in, (const void*)u, (const void*)params_out,
                          (const void*)wo_out, (const void*)pdf_out})
        if (q && !aligned4(q)) return set_error(NAM_E_INVALID_ARG, "misaligned pointer (uv needs 8 bytes, the rest 4)");
    if (((uintptr_t)uv & 7) != 0) return set_error(NAM_E_INVALID_ARG, "misaligned pointer (uv needs 8 bytes, the rest 4)");
    DeviceGuard g(ctx->device);
    const int64_t step = int64_t(1) << 30;
    for (int64_t o = 0; o < n; o += step) {
        const int64_t k = std::min(step, n - o);
        auto launch = m->smfma ? launch_sampler_mfma : launch_sampler;
        NAM_HIP(launch(m, k, mode, uv + 2 * o, lod + o, wi + 3 * o, wo_in ? wo_in + 3 * o : nullptr, u ? u + 3 * o : nullptr,
                       params_out ? params_out + 9 * o : nullptr, wo_out ? wo_out + 3 * o : nullptr,
                       pdf_out ? pdf_out + o : nullptr, (hipStream_t)stream));
    }
    return NAM_OK;
}

static nam_status proxy_run(nam_ctx* ctx, int64_t n, const float* params, const float* wi, const float* wo_in,
                            const float* u, float* wo_out, float* pdf_out, void* stream) {
    if (!ctx) return set_error(NAM_E_INVALID_ARG, "NULL handle");
    if (n < 0) return set_error(NAM_E_INVALID_ARG, "n must be >= 0");
    if (n == 0) return NAM_OK;
    if (!params || !wi || !pdf_out || (u ? !wo_out : !wo_in)) return set_error(NAM_E_INVALID_ARG, "NULL pointer");
    for (const void* q : {(const void*)params, (const void*)wi, (const void*)wo_in, (const void*)u, (const void*)wo_out,
                          (const void*)pdf_out})
        if (q && !aligned4(q)) return set_error(NAM_E_INVALID_ARG, "pointers must be 4-byte aligned");
    DeviceGuard g(ctx->device);
    const int64_t step = int64_t(1) << 30;
    for (int64_t o = 0; o < n; o += step) {
        const int64_t k = std::min(step, n - o);
        NAM_HIP(launch_proxy(k, params + 9 * o, wi + 3 * o, wo_in ? wo_in + 3 * o : nullptr, u ? u + 3 * o : nullptr,
                             wo_out ? wo_out + 3 * o : nullptr, pdf_out + o, (hipStream_t)stream));
    }
    return NAM_OK;
}

extern "C" {

nam_status nam_material_set_sampler(nam_ctx* ctx, nam_material* m, const nam_mlp_desc* mlp, const float* params) {
    if (!ctx || !m || !mlp || !mlp->dims || !params) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    const int K = mlp->n_layers, C = m->desc.channels;
    if (K < 2 || K > kMaxLayers) return set_error(NAM_E_UNSUPPORTED, "sampling decoder must have 1 to 4 hidden layers");
    if (mlp->dims[0] != C + 3) return set_error(NAM_E_SHAPE, "sampling decoder: dims[0] must equal channels + 3");
    if (mlp->dims[K] != 9) return set_error(NAM_E_SHAPE, "sampling decoder: the last width must be 9");
    const int H = mlp->dims[1];
    for (int k = 1; k < K; ++k)
        if (mlp->dims[k] != H) return set_error(NAM_E_UNSUPPORTED, "sampling decoder: hidden widths must all be equal");
    if (H != 16 && H != 32 && H != 64)
        return set_error(NAM_E_UNSUPPORTED, "sampling decoder: hidden width must be 16, 32 or 64");
    std::vector<int> dims(mlp->dims, mlp->dims + K + 1);
    const int64_t np = param_count(dims);
    std::vector<float> host(params, params + np);
    const std::vector<float> wt = transpose_layers(dims, host);
    DeviceGuard g(ctx->device);
    if (!g.ok()) return set_error(NAM_E_HIP, "hipSetDevice failed");
    void* sdev = nullptr;                  // a quantised material samples in FP16
    size_t sbias = 0;
    if (m->wprec != NAM_F32) {
        const nam_status st = pack_sampler_mfma(ctx, dims, host, &sdev, &sbias);
        if (st != NAM_OK) return st;
    }
    float* dev = nullptr;
    hipError_t e = hipMalloc(&dev, sizeof(float) * np);
    if (e == hipSuccess) e = hipMemcpy(dev, wt.data(), sizeof(float) * np, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        (void)hipFree(sdev);
        return hip_error(e, "hipMemcpy(sampler)");
    }
    (void)hipFree(m->swt32);
    (void)hipFree(m->smfma);
    m->swt32 = dev;
    m->smfma = sdev;
    m->smfma_bias_offset = sbias;
    m->sdims = std::move(dims);
    m->host_sparams = std::move(host);
    m->sshape = MlpShape{C, H, K - 1, 0};
    return NAM_OK;
}

nam_status nam_sampler_params(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                              const float* wi, float* params, void* stream) {
    return sampler_run(ctx, m, n, 0, uv, lod, wi, nullptr, nullptr, params, nullptr, nullptr, stream);
}

nam_status nam_sampler_pdf(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                           const float* wi, const float* wo, float* pdf, void* stream) {
    return sampler_run(ctx, m, n, 1, uv, lod, wi, wo, nullptr, nullptr, nullptr, pdf, stream);
}

nam_status nam_sampler_sample(nam_ctx* ctx, const nam_material* m, int64_t n, const float* uv, const float* lod,
                              const float* wi, const float* u, float* wo, float* pdf, void* stream) {
    return sampler_run(ctx, m, n, 2, uv, lod, wi, nullptr, u, nullptr, wo, pdf, stream);
}

nam_status nam_proxy_pdf(nam_ctx* ctx, int64_t n, const float* params, const float* wi, const float* wo, float* pdf,
                         void* stream) {
    return proxy_run(ctx, n, params, wi, wo, nullptr, nullptr, pdf, stream);
}

nam_status nam_proxy_sample(nam_ctx* ctx, int64_t n, const float* params, const float* wi, const float* u, float* wo,
                            float* pdf, void* stream) {
    return proxy_run(ctx, n, params, wi, nullptr, u, wo, pdf, stream);
}

}  // extern "C"
