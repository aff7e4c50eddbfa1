// Material files: the exported model of Sec. 7.1 (the final model, latent mips plus decoder
// weights, written after training and loaded by the renderer), which is what makes materials
// interchangeable by exchanging latent textures and a small weight table (Sec. 10).
//
// Format, little-endian:
//   char[8]  magic "NAMMAT01"
//   int32    width, height, channels, levels, address, n_layers, dims[n_layers + 1], n_frames,
//            s_layers (0: no sampling decoder), sdims[s_layers + 1] when s_layers > 0
//   float32  level 0 .. levels-1 ([H_l][W_l][C] each), decoder parameters (packed W_1, b_1, ...),
//            frame layer (W_F[6N][C], b_F[6N]) when n_frames > 0, sampling-decoder parameters
//   uint64   FNV-1a hash of every byte before it
// The FP32 master copy is stored; the precision is not (a loaded material starts in FP32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "nam_internal.h"

using namespace nam;

namespace {

constexpr char kMagic[8] = {'N', 'A', 'M', 'M', 'A', 'T', '0', '1'};
constexpr int32_t kMaxFileLevels = 32;

struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n) {
        const uint8_t* b = static_cast<const uint8_t*>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
};

struct FileCloser {
    void operator()(FILE* f) const { if (f) std::fclose(f); }
};
using File = std::unique_ptr<FILE, FileCloser>;

struct Writer {
    FILE* f;
    Fnv hash;
    bool ok = true;
    void put(const void* p, size_t n) {
        if (!ok || n == 0) return;
        ok = std::fwrite(p, 1, n, f) == n;
        hash.add(p, n);
    }
    void i32(int32_t v) { put(&v, 4); }
};

struct Reader {
    FILE* f;
    Fnv hash;
    bool ok = true;
    bool get(void* p, size_t n) {
        if (!ok) return false;
        if (n && std::fread(p, 1, n, f) != n) ok = false;
        if (ok) hash.add(p, n);
        return ok;
    }
    bool i32(int32_t* v) { return get(v, 4); }
};

}  // namespace

extern "C" {

nam_status nam_material_save(const nam_material* m, const char* path) {
    if (!m || !path) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    const int C = m->desc.channels;
    std::vector<float> tex((size_t)m->texel_count * C);
    if (hipSetDevice(m->ctx->device) != hipSuccess) return set_error(NAM_E_HIP, "hipSetDevice failed");
    NAM_HIP(hipMemcpy(tex.data(), m->texels32, sizeof(float) * tex.size(), hipMemcpyDeviceToHost));
    File f(std::fopen(path, "wb"));
    if (!f) return set_error(NAM_E_IO, std::string("cannot open for writing: ") + path);
    Writer w{f.get()};
    w.put(kMagic, sizeof(kMagic));
    const nam_pyramid_desc& d = m->desc;
    for (int32_t v : {d.width, d.height, d.channels, d.levels, (int32_t)d.address}) w.i32(v);
    w.i32((int32_t)m->dims.size() - 1);
    for (int v : m->dims) w.i32(v);
    w.i32(m->shape.NF);
    w.i32(m->sdims.empty() ? 0 : (int32_t)m->sdims.size() - 1);
    for (int v : m->sdims) w.i32(v);
    w.put(tex.data(), sizeof(float) * tex.size());
    w.put(m->host_params.data(), sizeof(float) * m->host_params.size());
    w.put(m->host_frames.data(), sizeof(float) * m->host_frames.size());
    w.put(m->host_sparams.data(), sizeof(float) * m->host_sparams.size());
    const uint64_t h = w.hash.h;
    w.put(&h, sizeof(h));
    if (!w.ok || std::fflush(f.get()) != 0) return set_error(NAM_E_IO, std::string("write failed: ") + path);
    return NAM_OK;
}

nam_status nam_material_load_file(nam_ctx* ctx, const char* path, nam_material** out) {
    if (!ctx || !path || !out) return set_error(NAM_E_INVALID_ARG, "NULL argument");
    *out = nullptr;
    File f(std::fopen(path, "rb"));
    if (!f) return set_error(NAM_E_IO, std::string("cannot open for reading: ") + path);
    Reader r{f.get()};
    char magic[8];
    if (!r.get(magic, sizeof(magic)) || std::memcmp(magic, kMagic, sizeof(kMagic)) != 0)
        return set_error(NAM_E_IO, "not a material file (magic)");
    int32_t hdr[5], n_layers = 0;
    for (int32_t& v : hdr) r.i32(&v);
    if (!r.i32(&n_layers)) return set_error(NAM_E_IO, "truncated header");
    if (n_layers < 1 || n_layers > kMaxLayers) return set_error(NAM_E_IO, "malformed header (layer count)");
    std::vector<int> dims(n_layers + 1);
    for (int& v : dims) {
        int32_t x = 0;
        r.i32(&x);
        v = x;
    }
    int32_t nf = 0, s_layers = 0;
    if (!r.i32(&nf) || !r.i32(&s_layers)) return set_error(NAM_E_IO, "truncated header");
    if (s_layers < 0 || s_layers > kMaxLayers) return set_error(NAM_E_IO, "malformed header (sampler layers)");
    std::vector<int> sdims(s_layers ? s_layers + 1 : 0);
    for (int& v : sdims) {
        int32_t x = 0;
        r.i32(&x);
        v = x;
        if (v < 1 || v > 4096) return set_error(NAM_E_IO, "malformed header (sampler widths)");
    }
    if (!r.ok) return set_error(NAM_E_IO, "truncated header");
    nam_pyramid_desc d{hdr[0], hdr[1], hdr[2], hdr[3], (nam_address)hdr[4]};
    // sizes are checked before anything is allocated from them
    if (d.levels < 1 || d.levels > kMaxFileLevels || d.width < 1 || d.height < 1 || d.width > (1 << 16) ||
        d.height > (1 << 16) || d.channels < 1 || d.channels > 64 || nf < 0 || nf > 2)
        return set_error(NAM_E_IO, "malformed header (sizes)");
    for (int v : dims)
        if (v < 1 || v > 4096) return set_error(NAM_E_IO, "malformed header (decoder widths)");
    size_t texels = 0, np = 0;
    for (int l = 0; l < d.levels; ++l) texels += (size_t)std::max(1, d.width >> l) * std::max(1, d.height >> l);
    for (int k = 1; k <= n_layers; ++k) np += (size_t)dims[k - 1] * dims[k] + dims[k];
    const size_t nfp = (size_t)6 * nf * (d.channels + 1);
    size_t nsp = 0;
    for (int k = 1; k <= s_layers; ++k) nsp += (size_t)sdims[k - 1] * sdims[k] + sdims[k];
    // the rest of the file must hold exactly the arrays and the hash: a damaged header is
    // reported before any allocation is sized from it
    const long here = std::ftell(f.get());
    if (here < 0 || std::fseek(f.get(), 0, SEEK_END) != 0) return set_error(NAM_E_IO, "cannot seek");
    const long end = std::ftell(f.get());
    if (end < 0 || std::fseek(f.get(), here, SEEK_SET) != 0) return set_error(NAM_E_IO, "cannot seek");
    const size_t expect = sizeof(float) * (texels * d.channels + np + nfp + nsp) + sizeof(uint64_t);
    if ((size_t)(end - here) != expect) return set_error(NAM_E_IO, "file size does not match its header");
    std::vector<std::vector<float>> levels(d.levels);
    std::vector<const float*> ptrs(d.levels);
    std::vector<float> params, frames, sparams;
    try {
        for (int l = 0; l < d.levels; ++l) {
            levels[l].resize((size_t)std::max(1, d.width >> l) * std::max(1, d.height >> l) * d.channels);
            ptrs[l] = levels[l].data();
        }
        params.resize(np);
        frames.resize(nfp);
        sparams.resize(nsp);
    } catch (const std::bad_alloc&) {
        return set_error(NAM_E_OOM, "host allocation failed");
    }
    for (int l = 0; l < d.levels; ++l) r.get(levels[l].data(), sizeof(float) * levels[l].size());
    r.get(params.data(), sizeof(float) * np);
    r.get(frames.data(), sizeof(float) * frames.size());
    r.get(sparams.data(), sizeof(float) * sparams.size());
    const uint64_t h = r.hash.h;
    uint64_t stored = 0;
    if (!r.get(&stored, sizeof(stored))) return set_error(NAM_E_IO, "truncated file");
    if (stored != h) return set_error(NAM_E_IO, "checksum mismatch");
    nam_mlp_desc mlp{n_layers, dims.data()};
    nam_status st = nam_material_load_framed(ctx, &d, ptrs.data(), &mlp, params.data(), nf, nf ? frames.data() : nullptr,
                                             out);
    if (st != NAM_OK || !s_layers) return st;
    nam_mlp_desc smlp{s_layers, sdims.data()};
    st = nam_material_set_sampler(ctx, *out, &smlp, sparams.data());
    if (st != NAM_OK) {
        const std::string msg = nam_last_error();
        nam_material_free(*out);
        *out = nullptr;
        return set_error(st, msg);
    }
    return NAM_OK;
}

}  // extern "C"
