/*
 * nam.h -- C ABI of libnam, an MI355X (gfx950) library for the data-parallel hot path of
 * the neural appearance model of "Real-Time Neural Appearance Models" (Zeltner et al.,
 * ACM TOG 43(3), 2024):
 *
 *     f(x, wi, wo) ~ g( z(x), wi, wo ; theta )                         (Eq. neural-brdf)
 *
 * per shading query a filtered fetch z(x) from a mip-mapped latent texture (Sec. 4.1,
 * "Latent texture"), concatenation with the light and view directions in the shading frame
 * (Cartesian xyz, Sec. 9 "Energy conservation and reciprocity"), and a small MLP decoder g
 * (ReLU hidden layers, softplus RGB output) evaluated by hand-written HIP kernels.
 *
 * Conventions shared by every call
 *   - Every function returns nam_status; NAM_OK is 0.  On error nam_last_error() returns a
 *     message for the calling thread (valid until that thread's next call).  No C++
 *     exception crosses the ABI.
 *   - "device" pointers are HIP device allocations of the context's device (for example the
 *     data pointer of a torch CUDA tensor); "host" pointers are ordinary CPU memory.
 *     The caller owns every pointer it passes; the library owns the handles it returns and
 *     the device memory behind them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  Calls that take
 *     a stream enqueue their kernels and return without waiting; argument checks happen on
 *     the host before anything is enqueued, so an error status means nothing was enqueued.
 *   - Floating-point query arrays are float32 and at least 4-byte aligned.  n == 0 is a no-op;
 *     n < 0 is NAM_E_INVALID_ARG.
 *   - Texture sizes are powers of two; level l has max(1, W >> l) x max(1, H >> l) texels.
 *   - A query with a non-finite uv or lod decodes to NaN (its fetch gives NaN) and never
 *     touches memory outside the pyramid; the other queries of the batch are unaffected.
 */
#ifndef NAM_H
#define NAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NAM_OK = 0,
    NAM_E_INVALID_ARG = 1,   /* null pointer, negative size, bad enum value */
    NAM_E_SHAPE = 2,         /* sizes inconsistent with each other */
    NAM_E_UNSUPPORTED = 3,   /* a valid request this build does not implement (dims, dtype) */
    NAM_E_OOM = 4,           /* device or host allocation failed */
    NAM_E_BUDGET = 5,        /* a serving request can never fit the memory budget */
    NAM_E_HIP = 6,           /* a HIP runtime call failed; the message names it */
    NAM_E_BUSY = 7,          /* the object is in use (e.g. freeing a material a server holds) */
    NAM_E_IO = 8             /* file read/write failed or a file is malformed */
} nam_status;

typedef enum { NAM_WRAP = 0, NAM_CLAMP = 1 } nam_address;

/* Storage / arithmetic type of texels and decoder weights. */
typedef enum { NAM_F32 = 0, NAM_F16 = 1, NAM_FP8_E4M3 = 2 } nam_dtype;

typedef struct nam_ctx nam_ctx;
typedef struct nam_material nam_material;

/* Message of the last failing call made by this thread ("" if none). */
const char* nam_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int nam_version(void);

/* ---------------------------------------------------------------------------- context */

/* Bind a context to HIP device `device`.  The context holds per-device state (kernel
 * selection, scratch); it may be used from one thread at a time. */
nam_status nam_create(int device, nam_ctx** out);
nam_status nam_destroy(nam_ctx* ctx);

/* ------------------------------------------------------------------------- materials */

/* The latent pyramid (Sec. 4.1): width and height powers of two, channels C in {8, 16},
 * 1 <= levels <= log2(max(width, height)) + 1. */
typedef struct {
    int width, height, channels, levels;
    nam_address address;
} nam_pyramid_desc;

/* The decoder g: n_layers weight layers, dims[0] = channels + 6 (latent code, wi, wo; with
 * N = 2 learned shading frames channels + 12, see nam_material_load_framed),
 * dims[1..n_layers-1] the hidden widths (all equal, one of 16, 32, 64; 1 to 4 hidden
 * layers), dims[n_layers] = 3 (RGB) or 6: RGB, then the albedo head of Sec. 6.4 "Albedo
 * inference" (an extra RGB output approximating the directional albedo of Eq. albedo, the
 * integral of f cos(theta_i) over incident directions at x and wo).  Every output goes
 * through the same softplus.  Wherever an argument below holds decoder outputs ("rgb",
 * "d_rgb", "target") it is [n][dims[n_layers]]: row i holds RGB, then the albedo when the
 * decoder has 6 outputs.  The decoder sizes of the paper (Sec. 8: two hidden layers of 16 or
 * 32, three of 64) are all covered. */
typedef struct {
    int n_layers;
    const int* dims;
} nam_mlp_desc;

/* Bytes of texel storage a pyramid needs in the given texel type (host-only arithmetic;
 * no device needed).  The paper's figure of 256 MB per 4k x 4k, 8-channel, half-precision
 * latent tile (Sec. 8.3, "Memory usage") is level 0 of such a pyramid. */
nam_status nam_pyramid_bytes(const nam_pyramid_desc* desc, nam_dtype texel_type, size_t* bytes);

/* Copy a trained material to the device (the exported model of Sec. 7.1: latent mips plus a
 * small table of decoder weights).
 *   levels: host array of `desc->levels` host pointers; level l is float32 [H_l][W_l][C],
 *           row-major, x <-> u, y <-> v.
 *   params: host float32, packed W_1[d_1][d_0], b_1[d_1], W_2[d_2][d_1], b_2, ...
 * The material starts in FP32 precision (texels and decoder). */
nam_status nam_material_load(nam_ctx* ctx, const nam_pyramid_desc* desc, const float* const* levels,
                             const nam_mlp_desc* mlp, const float* params, nam_material** out);

/* A material whose decoder rotates the directions into learned shading frames (Sec. 4.2,
 * "Transformation to learned shading frames", Eq. frame-rotation; the bitangent as stated
 * under "Alternative geometric priors" in Sec. 9).  A linear layer maps the latent code z to
 * N normals n_f and N tangents t_f; each is normalised on its own (not orthogonalised), the
 * bitangent is b_f = n^_f x t^_f normalised, and T stacks the rows t_1, b_1, n_1, ...,
 * t_N, b_N, n_N.  The decoder input is [z, T wi, T wo], so dims[0] = channels + 6 N.
 * A vector v is normalised as v / sqrt(max(v.v, 1e-12)): a zero vector stays zero.
 *   n_frames:     1 or 2 (the paper uses 2 frames, a 12-neuron layer); 0 is nam_material_load.
 *   frame_params: host float32, W_F[6N][C] row-major then b_F[6N]; output 6f + r is
 *                 component r of n_f for r < 3 and component r - 3 of t_f for r >= 3.
 * Every decode entry point and precision, nam_calibrate and the server apply the frames.  The
 * FP32 precision runs the frame layer and the transform in FP32; the matrix-core precisions
 * run the frame layer on FP16 z and W_F with FP32 accumulation (like their other layers) and
 * the transform in FP32; the 6N outputs enter layer 1 in that layer's format.  The training
 * entry points train a frame layer with the decoder when nam_model_desc.n_frames > 0.
 * Other arguments and errors as nam_material_load; NAM_E_SHAPE if dims[0] != C + 6 N. */
nam_status nam_material_load_framed(nam_ctx* ctx, const nam_pyramid_desc* desc, const float* const* levels,
                                    const nam_mlp_desc* mlp, const float* params, int n_frames,
                                    const float* frame_params, nam_material** out);

/* Save a material to a file: the exported model of Sec. 7.1 (latent mips plus the decoder's
 * weights; materials are interchanged by exchanging exactly these, Sec. 10).  Writes the FP32
 * master copy: pyramid, decoder, learned frames and sampling decoder, in a little-endian binary format with a
 * magic ("NAMMAT01"), the pyramid and decoder descriptors, the FP32 arrays and an FNV-1a
 * checksum.  The precision is not stored.  Synchronous (copies the texels to the host).
 * NAM_E_IO if the file cannot be written. */
nam_status nam_material_save(const nam_material* mat, const char* path);

/* Load a material written by nam_material_save; it starts in FP32, as after
 * nam_material_load.  NAM_E_IO if the file cannot be read, is truncated, has another magic,
 * sizes out of range or a checksum mismatch; other errors as nam_material_load_framed. */
nam_status nam_material_load_file(nam_ctx* ctx, const char* path, nam_material** out);

/* Choose the decode precision (post-training quantisation at load time, Sec. 5.2
 * "Precision"; FP8 extends the paper's remark on lower precisions).
 *   weights NAM_F32:      FP32 texels and decoder, FP32 arithmetic: trilinear decodes on the FP32
 *                         matrix cores (v_mfma_f32_16x16x4_f32, the training kernel's forward) for
 *                         decoders with C in {8, 16}, hidden width 32 or 64, 2 or 3 hidden
 *                         layers and no frames (packed once at load, in device memory the
 *                         material holds); the stochastic level choice, frames and other
 *                         shapes on the vector ALU.
 *   weights NAM_F16:      FP16 texels, FP16 weights and activations on MFMA, FP32 accumulate.
 *   weights NAM_FP8_E4M3: FP16 texels, OCP E4M3 weights and activations on MFMA with one
 *                         scale per layer for the weights and one for the layer's input, FP32
 *                         accumulate.  act_absmax (host, n_layers floats, from nam_calibrate)
 *                         gives the per-layer activation absmax; first_layer_f16 != 0 keeps
 *                         layer 1 in FP16.  Each scale is the largest power of two s with
 *                         absmax * s <= 448 (weights: absmax over the layer's matrix), so
 *                         rescaling is exact; values beyond the calibrated range saturate at
 *                         +-448.
 * texels must be NAM_F32 with NAM_F32 weights and NAM_F16 otherwise.  The matrix-core
 * precisions address the FP16 pyramid with 32-bit byte offsets: they need it below 4 GiB
 * (texels x channels x 2 bytes; e.g. 8192^2 x 16 channels with all mips) and return
 * NAM_E_UNSUPPORTED above, where NAM_F32 still applies.  Quantised copies are made on the
 * device with round-to-nearest-even (E4M3 saturates at +-448); the FP32 master copy is kept. */
nam_status nam_material_set_precision(nam_ctx* ctx, nam_material* mat, nam_dtype weights, nam_dtype texels,
                                      const float* act_absmax, int first_layer_f16);

/* Per-layer absolute maximum of each layer's input activations over a calibration batch,
 * computed with the FP32 decoder on the device.  absmax_out: host, n_layers floats.
 * Synchronises `stream`. */
nam_status nam_calibrate(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                         const float* wi, const float* wo, float* absmax_out, void* stream);

/* Device bytes held by the material (texels in every resident precision plus weights). */
nam_status nam_material_footprint(const nam_material* mat, size_t* bytes);
nam_status nam_material_free(nam_material* mat);

/* --------------------------------------------------------------------------- hot path */

/* Decode n shading queries (Eq. neural-brdf), in the material's current precision.  The
 * shading-frame transform T is the material's learned frames (nam_material_load_framed) or,
 * without them, the identity.
 *   uv [n][2], lod [n] (fractional mip level, clamped to [0, levels-1]),
 *   wi [n][3], wo [n][3] (used as given, no normalisation), rgb [n][dims[last]]: device
 *   float32 (RGB, then the albedo for a decoder with the albedo head).
 * One fused kernel per call: fetch, concatenation, every layer, softplus. */
nam_status nam_decode(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                      const float* wi, const float* wo, float* rgb, void* stream);

/* Decode with the level chosen by Russian roulette instead of trilinear blending (Sec. 4.1,
 * "Latent texture": one of the two nearest levels is picked at random and the latent code is
 * fetched by bilinear interpolation inside it; 4 texel taps per query instead of 8).
 *   xi [n]: device float32, one draw per query from the caller's random stream.  With lam the
 *           level clamped to [0, levels-1] and t = lam - floor(lam), query i uses the coarser
 *           level iff xi[i] < t and the finer one otherwise (a NaN draw: the finer), so draws
 *           uniform on [0, 1) take the coarser level with probability t.  t is exact in FP32.
 * Every other argument, the precision and the NaN rule are those of nam_decode. */
nam_status nam_decode_stochastic(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                                 const float* xi, const float* wi, const float* wo, float* rgb, void* stream);

/* ------------------------------------------------------------ importance sampling */

/* Attach the importance-sampling decoder (Sec. 4.3 "Importance sampling"; App. A): an MLP on
 * [z, wi] (dims[0] = channels + 3; 1 to 4 hidden layers of 16, 32 or 64, ReLU; dims[last] = 9
 * linear outputs; the paper uses 3 x 32) whose outputs become the analytic proxy's parameters
 * p = {w_d, mu_dx, mu_dy, w_s, alpha_x, alpha_y, rho, mu_sx, mu_sy} through
 *   (w_d, w_s) = softmax(o_0, o_3);  mu = qsinh(o) = o (1 + |o| / 2);
 *   alpha = 1e-3 + (1 - 1e-3) (1 + qtanh(o)) / 2;  rho = 0.999 qtanh(o),
 *   qtanh(o) = o (1 - |o| / 4) for |o| < 2, sign(o) beyond
 * (quadratic approximations of tanh and sinh; the floor on alpha and the factor on rho keep M
 * invertible).  params: host float32 packed as for nam_material_load.  Replaces an earlier
 * sampler.  The sampler follows the material's precision (Sec. 5.2 "Precision" converts the
 * sampler's FP32 master parameters to FP16 at load like the decoder's): FP32 on FP32 texels;
 * on a quantised material (FP16 or E4M3 decoder, FP16 texels) FP16 weights and layer inputs
 * with FP32 accumulation on the matrix cores, the latent code filtered in FP16 as the FP16
 * decoder filters it, and the activations and proxy in FP32.  It is converted again whenever
 * the precision changes.  Errors: NAM_E_SHAPE, NAM_E_UNSUPPORTED for dims outside the above;
 * on an error the earlier sampler stays. */
nam_status nam_material_set_sampler(nam_ctx* ctx, nam_material* mat, const nam_mlp_desc* sampler, const float* params);

/* Proxy parameters params [n][9] (device float32) of n queries: trilinear fetch, sampling
 * decoder on [z, wi], activations.  uv, lod, wi as for nam_decode.  Non-finite uv or lod: NaN. */
nam_status nam_sampler_params(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                              const float* wi, float* params, void* stream);

/* PDF pdf [n] (per unit solid angle, over the whole sphere) of the given outgoing directions
 * wo [n][3] (unit vectors) under the proxy of each query (Eq. pdf_full and Eq. pdf_spec):
 *   w_d max(0, wo . n_d) / pi + w_s D_std(h') det(M^-1) / |M^-1 h|^3 / (4 |wo . h|),
 * n_d = normalise(-mu_dx, -mu_dy, 1), M = [[alpha_x, 0, -mu_sx], [alpha_y rho,
 * alpha_y sqrt(1 - rho^2), -mu_sy], [0, 0, 1]], h = normalise(wi + wo) taken with h_z >= 0,
 * h' = M^-1 h / |M^-1 h|, D_std(h') = max(h'_z, 0) / pi (the density of the alpha = 1 GGX normal
 * sampler, so the PDF integrates to one); the specular term is 0 where wi + wo = 0. */
nam_status nam_sampler_pdf(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                           const float* wi, const float* wo, float* pdf, void* stream);

/* Sample outgoing directions wo [n][3] and their PDF pdf [n] with u [n][3] (device float32 in
 * [0, 1)): the diffuse lobe if u_0 < w_d, else the specular one.  Diffuse: the cosine sample
 * (sqrt(u_1) cos 2 pi u_2, sqrt(u_1) sin 2 pi u_2, sqrt(1 - u_1)) turned by the minimal
 * rotation from +z to n_d.  Specular: h = normalise(M h_std) with h_std that same cosine sample
 * (the alpha = 1 GGX normal sampler), wo = 2 (wi . h) h - wi. */
nam_status nam_sampler_sample(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                              const float* wi, const float* u, float* wo, float* pdf, void* stream);

/* The same PDF and sampling from cached proxy parameters params [n][9] (as written by
 * nam_sampler_params), without the fetch or the network: the paper queries the sampling
 * network once per hit and reuses its parameters for sampling and for PDF evaluation. */
nam_status nam_proxy_pdf(nam_ctx* ctx, int64_t n, const float* params, const float* wi, const float* wo, float* pdf,
                         void* stream);
nam_status nam_proxy_sample(nam_ctx* ctx, int64_t n, const float* params, const float* wi, const float* u, float* wo,
                            float* pdf, void* stream);

/* The filtered latent fetch alone (Sec. 4.1, trilinear: bilinear inside each of the two
 * nearest levels, linear across them): z [n][C] device float32, from the texels of the
 * material's current precision. */
nam_status nam_fetch(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv, const float* lod,
                     float* z, void* stream);

/* Number of distinct texels (over all levels) that the 8 taps of n queries address: the
 * compulsory texel traffic of a decode.  Synchronises `stream`. */
nam_status nam_texel_footprint(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv,
                               const float* lod, uint64_t* distinct_texels, void* stream);

/* The same for the 4 taps of the level chosen by Russian roulette with draws xi [n] (device
 * float32, the rule of nam_decode_stochastic).  Synchronises `stream`. */
nam_status nam_texel_footprint_stochastic(nam_ctx* ctx, const nam_material* mat, int64_t n, const float* uv,
                                          const float* lod, const float* xi, uint64_t* distinct_texels,
                                          void* stream);

/* ------------------------------------------------------------------- differentiation */
/* Training by backpropagation through the decoder and directly into the latent texels (the
 * direct optimisation of Sec. 2 "Obtaining latent textures", used in the fine-tuning phase of
 * Sec. 5.1).  Everything here is FP32.  The caller owns the trainable tensors:
 *   texels: device float32, the whole pyramid as one buffer, levels concatenated with level 0
 *           first, each level [H_l][W_l][C] (the layout nam_material_load copies);
 *   params: device float32, packed W_1[d_1][d_0], b_1, W_2, b_2, ...;
 * gradients and Adam moments have the same layouts.  Samples (uv, lod, wi, wo, targets and
 * output gradients) are device float32 as in nam_decode; at most 2^31 - 64 per call.  A sample
 * with a non-finite uv or lod decodes to NaN and contributes no gradient.  Latent gradients
 * are accumulated with floating-point atomics, so their last bits depend on execution order,
 * unless the context is in deterministic mode (nam_set_deterministic); parameter gradients
 * are reduced in a fixed order and are reproducible.
 *
 * With learned shading frames (n_frames = N in {1, 2}; Sec. 4.2, Eq. frame-rotation, trained
 * jointly with the decoder and the latents, Sec. 5) the decoder input is [z, T wi, T wo]
 * (dims[0] = C + 6 N, T and its conventions as in nam_material_load_framed) and params holds
 * the frame layer first, W_F[6N][C] then b_F[6N], followed by the packed decoder; gradients
 * and Adam moments keep that layout, so the frame layer is trained like every other weight.
 * Training with frames runs on the vector training kernel (its weight gradients on FP32
 * matrix-core tiles) and supports C in {8, 16}, hidden widths 32 or 64, 2 or 3 hidden layers
 * and 3 outputs (NAM_E_UNSUPPORTED otherwise).  n_frames = 0: no
 * frames (T the identity, dims[0] = C + 6). */
typedef struct {
    nam_pyramid_desc pyramid;
    nam_mlp_desc mlp;
    int n_frames;
} nam_model_desc;

/* rgb [n][dims[last]] = the decode of n samples with the given texels and parameters (as
 * nam_decode in FP32, recomputing nothing from a material). */
nam_status nam_forward(nam_ctx* ctx, const nam_model_desc* model, const float* texels, const float* params,
                       int64_t n, const float* uv, const float* lod, const float* wi, const float* wo, float* rgb,
                       void* stream);

/* Vector-Jacobian product of the decode: given d_rgb [n][dims[last]] = dL/drgb, adds dL/dtexels into
 * d_texels (+=) and writes dL/dparams into d_params (=).  No gradient flows to uv, lod, wi, wo. */
nam_status nam_backward(nam_ctx* ctx, const nam_model_desc* model, const float* texels, const float* params,
                        int64_t n, const float* uv, const float* lod, const float* wi, const float* wo,
                        const float* d_rgb, float* d_texels, float* d_params, void* stream);

/* The same for the mean squared error L = 1/(3n) sum (rgb - target)^2 against target
 * [n][dims[last]], the sum over every output: with the albedo head the RGB loss plus the
 * albedo loss, each a mean over 3n values (the albedo is fitted by L2 against one-sample
 * estimates of Eq. albedo, Sec. 5.2 "Optimization"; an estimate drawn independently of the
 * sample's wi makes the fit converge to the albedo itself).
 * d_texels += dL/dtexels, d_params = dL/dparams, *loss (device float) = L. */
nam_status nam_loss_backward(nam_ctx* ctx, const nam_model_desc* model, const float* texels, const float* params,
                             int64_t n, const float* uv, const float* lod, const float* wi, const float* wo,
                             const float* target, float* d_texels, float* d_params, float* loss, void* stream);

/* nam_loss_backward for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving or training loops, and harnesses that forbid hipMalloc.  The same
 * arguments and results as nam_loss_backward, but the call allocates nothing: its level table,
 * the decoder's operand blocks and the per-wave partial gradients and loss sums sit in a static
 * device region of the library, 32 MiB, one copy per GPU the library runs on, held until the
 * process ends.  The caller still passes the inputs, d_texels, d_params and loss.  The number of
 * workgroups shrinks to what the region holds (each needs 4 (P + 1) floats per wave for a decoder
 * of P parameters), so large decoders may run on fewer CUs than nam_loss_backward uses; the
 * gradients are those of nam_loss_backward to rounding (the per-slice partial sums are grouped
 * differently).  Every call on one GPU shares the region: calls that overlap on one GPU (two
 * streams, two host threads, two contexts) race and give undefined results; calls in one stream
 * order are safe.  Errors as nam_loss_backward, plus NAM_E_UNSUPPORTED when the decoder's
 * gradients do not fit the region or the context is in deterministic mode (which needs
 * per-call memory), and NAM_E_HIP when the region could not be located on this device. */
nam_status nam_loss_backward_noalloc(nam_ctx* ctx, const nam_model_desc* model, const float* texels,
                                     const float* params, int64_t n, const float* uv, const float* lod,
                                     const float* wi, const float* wo, const float* target, float* d_texels,
                                     float* d_params, float* loss, void* stream);

/* Deterministic mode of a context's training entry points (nam_backward, nam_loss_backward,
 * nam_train_step; on = 1) or the default (on = 0).  In deterministic mode the gradient of each
 * sample's latent code is kept per sample and scattered into the texels as 64-bit fixed-point
 * integers (scale 2^(62 - e), with 2^e above n times the largest component, so no texel can
 * overflow; each contribution is rounded to the nearest multiple of 2^-(62 - e)), whose sum
 * does not depend on the order of the additions: repeated calls on the same inputs give
 * bitwise equal gradients, and a training run is reproducible.  It costs a per-sample buffer
 * (n x C floats) and 8 bytes per texel channel of context-owned device memory, and a second
 * pass over the samples.  If a gradient is not finite the scatter falls back to float atomics.
 * Errors: NAM_E_INVALID_ARG for a NULL ctx or on not 0 or 1. */
nam_status nam_set_deterministic(nam_ctx* ctx, int on);

/* Adam (Kingma and Ba), step counted from 1, no weight decay:
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;  p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
typedef struct {
    float lr, beta1, beta2, eps;
    int64_t step;
} nam_adam_cfg;

/* In-place Adam update of count device floats p, m, v with gradient g. */
nam_status nam_adam_update(nam_ctx* ctx, int64_t count, float* p, float* m, float* v, const float* g,
                           const nam_adam_cfg* cfg, void* stream);

/* One training step on n samples: loss and gradients of the mean squared error (into
 * context-owned gradient buffers), then Adam on every parameter and on every texel of every
 * level (dense, including texels with zero gradient).  *loss (device) receives the loss
 * before the update. */
nam_status nam_train_step(nam_ctx* ctx, const nam_model_desc* model, float* texels, float* params,
                          float* m_texels, float* v_texels, float* m_params, float* v_params, int64_t n,
                          const float* uv, const float* lod, const float* wi, const float* wo, const float* target,
                          const nam_adam_cfg* cfg, float* loss, void* stream);

/* ------------------------------------------------------------------------------ encoder */
/* The encoder of Sec. 5.1 "Encoder": an MLP from the parameters of the original material at a
 * location (its albedo, roughness, ...: A values) to a latent code of C channels, ReLU hidden
 * layers and a linear output layer (the paper does not give its activations).  encoder: dims
 * [A, H, (H,) C] with A in {4, 8, 16}, 1 or 2 hidden layers of width 16, 32 or 64, C in {8, 16};
 * eparams: device float32 packed as a decoder's (W_1[H][A], b_1, ..., W_out[C][H], b_out).
 * Training follows the paper's two phases.  First the encoder and the decoder train end to end
 * with the code of a query taken from the encoder (nam_encode_queries, nam_loss_backward_codes,
 * nam_encoder_backward), bypassing the latent texture; then the latent texture is initialised
 * by the encoder at every texel (nam_encode_texels) and trained directly (nam_train_step) while
 * the encoder is dropped.  The FP32 vector ALU runs all of it.  Errors: NAM_E_UNSUPPORTED for
 * shapes outside the above, NAM_E_SHAPE for a parameter pyramid whose channels are not A,
 * NAM_E_INVALID_ARG for NULL or misaligned pointers. */

/* z[n][C] = E(attrs[n][A]) for parameter rows given as they are, such as every texel of a
 * pyramid of the material's parameters (levels concatenated): the bake that initialises the
 * latent texture (Sec. 5.1).  attrs and z: device float32. */
nam_status nam_encode_texels(nam_ctx* ctx, const nam_mlp_desc* encoder, const float* eparams, int64_t n,
                             const float* attrs, float* z, void* stream);

/* z[n][C] = E(p(uv, lod)), p the material's parameters filtered at each query: the trilinear
 * filter of the latent fetch (the same taps, wrap or clamp) over params_pyramid, a pyramid of
 * the parameters prefiltered level by level (Sec. 5.1; channels = A, device float32, levels
 * concatenated as for nam_material_load).  The code of a query in the first training phase.
 * Non-finite uv or lod: NaN codes. */
nam_status nam_encode_queries(nam_ctx* ctx, const nam_mlp_desc* encoder, const float* eparams,
                              const nam_pyramid_desc* params_pyramid, const float* attrs, int64_t n, const float* uv,
                              const float* lod, float* z, void* stream);

/* The decoder's loss on given latent codes z[n][C] (device float32, C = the model pyramid's
 * channels; the rest of model->pyramid is not read): the first training phase's loss, as
 * nam_loss_backward with the fetch replaced by z.  Writes *loss (device), d_params (=) and the
 * gradient of every code, dz[n][C] (=).  A sample whose code has a non-finite component adds
 * nothing (dz = 0); n stays the loss's denominator.  Deterministic: the parameter gradients are
 * reduced in a fixed order and the codes' gradients are per sample. */
nam_status nam_loss_backward_codes(nam_ctx* ctx, const nam_model_desc* model, const float* params, int64_t n,
                                   const float* z, const float* wi, const float* wo, const float* target, float* dz,
                                   float* d_params, float* loss, void* stream);

/* d_eparams (=, device float32) = the gradient of sum_i dz[i] . E(p(uv_i, lod_i)) with respect
 * to the encoder's parameters: with dz from nam_loss_backward_codes, the encoder's gradient of
 * the first training phase.  Non-finite queries add nothing.  Deterministic (per-workgroup
 * partial sums reduced in a fixed order). */
nam_status nam_encoder_backward(nam_ctx* ctx, const nam_mlp_desc* encoder, const float* eparams,
                                const nam_pyramid_desc* params_pyramid, const float* attrs, int64_t n,
                                const float* uv, const float* lod, const float* dz, float* d_eparams, void* stream);

/* --------------------------------------------------------------------------- serving */
/* A request loop over several resident materials (the many-material setting of Sec. 7.3
 * "Shading coherency" and Sec. 8.3 "Scalability", where materials differ only in their
 * weights and latent textures).  A worker thread admits requests in arrival order by memory
 * footprint, cuts them into tiles of at most max_tile queries and runs tiles concurrently on
 * n_streams HIP streams (continuous batching: work that arrives while other requests run is
 * started as soon as a stream and budget bytes free up); tiles of several requests and
 * materials that share a matrix-core kernel go out as one grouped launch (nam_server_set_group).  Each tile reserves 48 bytes per
 * query (36 in, 12 out; 60 with the albedo head's 24 out) of the HBM budget while it is on the device; requests with host
 * buffers are staged through a device arena of that size, requests with device buffers only
 * reserve the bytes.  A decode never depends on how requests are tiled or mixed: each result
 * is bitwise the one nam_decode gives for that request alone.  Materials added to a server
 * may not change precision or be freed until the server is destroyed (NAM_E_BUSY).  The
 * server's calls are thread-safe. */
typedef struct nam_server nam_server;

typedef struct {
    int64_t completed;          /* requests finished since the last reset */
    int64_t queries;            /* their queries */
    double p50_s, p99_s;        /* latency percentiles, arrival to completion, seconds */
    double mean_s, max_s;
    double span_s;              /* first arrival to last completion */
    double queries_per_s;       /* queries / span */
    size_t peak_reserved_bytes; /* largest budget use observed */
    int64_t launches;           /* decode launches since the last reset */
    int64_t tiles;              /* tiles they ran (tiles / launches: mean tiles per grouped launch) */
    int64_t peak_requests_on_device;  /* most distinct requests with tiles launched and not yet
                                         complete at one time: > 1 means requests overlapped on
                                         the device */
    int64_t peak_launches_on_device;  /* most launches in flight at one time (busy streams) */
} nam_server_stats_t;

/* hbm_budget_bytes >= 48 * max_tile (else NAM_E_BUDGET); 1 <= n_streams <= 16; max_tile >= 256.
 * A query reserves 36 bytes of inputs plus 4 per decoder output (48, or 60 with the albedo
 * head); adding a material whose max_tile queries exceed the budget is NAM_E_BUDGET. */
nam_status nam_server_create(nam_ctx* ctx, size_t hbm_budget_bytes, int n_streams, int64_t max_tile,
                             nam_server** out);
nam_status nam_server_add_material(nam_server* server, nam_material* mat, int* material_id);

/* Queue a decode of n queries of material_id (pointers as in nam_decode; host pointers when
 * host_io != 0, preferably pinned).  arrival_s < 0: the request arrives now.  arrival_s >= 0:
 * it arrives arrival_s seconds after the server's epoch (its creation or the last
 * nam_server_reset_stats), which replays a recorded arrival process; a time already past
 * admits it at once.  Latency is measured from the arrival time.  The buffers must stay valid
 * until the request is done. */
nam_status nam_server_submit(nam_server* server, int material_id, int64_t n, const float* uv, const float* lod,
                             const float* wi, const float* wo, float* rgb, int host_io, double arrival_s,
                             uint64_t* ticket);
/* done = 1 once the request's results are in rgb; latency_s = completion - arrival (-1 if not done). */
nam_status nam_server_poll(nam_server* server, uint64_t ticket, int* done, double* latency_s);
/* Withdraw a request that has not started (NAM_E_BUSY once any of its tiles was launched). */
nam_status nam_server_cancel(nam_server* server, uint64_t ticket);
/* Block until every submitted request (including future arrivals) is done. */
nam_status nam_server_wait_all(nam_server* server);
nam_status nam_server_stats(nam_server* server, nam_server_stats_t* out);

/* Tiles per grouped launch, 1 to 8 (default 8).  Tiles with device buffers whose materials share
 * one matrix-core kernel (same shape, precision, address mode and frame presence) are taken
 * from the pending requests in arrival order and decoded by one launch, the persistent grid
 * shared among them by size; 1 launches every tile on its own.  Results do not change. */
nam_status nam_server_set_group(nam_server* server, int max_tiles);
/* Clear statistics, forget finished requests (their tickets become unknown) and restart the
 * epoch of replayed arrival times. */
nam_status nam_server_reset_stats(nam_server* server);
/* Finish all queued work, then release the server's streams and arena. */
nam_status nam_server_destroy(nam_server* server);

#ifdef __cplusplus
}
#endif
#endif
