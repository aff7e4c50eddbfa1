/*
 * FP64 CPU oracle for the neural appearance decode path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP library
 * is checked against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or constant with the HIP library.
 *
 * Every quantity is computed in double precision from the stored input values.  Each
 * function states the passage of "Real-Time Neural Appearance Models" (Zeltner et al.,
 * TOG 43(3), 2024) it follows.  Where the paper is silent the adopted reading is stated
 * inline (texel centres at (x + 1/2) / W, wrap addressing by default, lod clamped to the
 * pyramid, trilinear blend between the two nearest levels).
 *
 * Layouts (all row-major, caller-owned):
 *   level l of the latent pyramid: [H_l][W_l][C], H_l = max(1, H >> l), W_l = max(1, W >> l)
 *   decoder parameters, packed:    W_1[d_1][d_0], b_1[d_1], W_2[d_2][d_1], b_2, ...
 *   queries: uv[n][2], lod[n], wi[n][3], wo[n][3]
 *   outputs: out[n][KO], KO = dims[K] = 3 (RGB reflectance) or 6 (RGB reflectance, then the
 *            directional albedo of Eq. albedo as the extra RGB output of Sec. 6.4 "Albedo
 *            inference"; every output goes through the same softplus)
 *   learned shading frames:        W_F[6N][C], b_F[6N] (N frames; see frame_transform)
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <fenv.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_WRAP 0
#define ORC_CLAMP 1

typedef struct {
    int width, height, channels, n_levels, address;
} orc_pyramid;

static int lvl_w(const orc_pyramid* p, int l) { int w = p->width >> l; return w < 1 ? 1 : w; }
static int lvl_h(const orc_pyramid* p, int l) { int h = p->height >> l; return h < 1 ? 1 : h; }

static long pos_mod(long a, long m) { long r = a % m; return r < 0 ? r + m : r; }
static long clampl(long a, long lo, long hi) { return a < lo ? lo : (a > hi ? hi : a); }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following parallel regions (timing of the single-thread baseline). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Level choice for a fractional level index (Sec. 4.1, "Latent texture": the level comes
 * from the footprint area and may lie between two pyramid levels).  Reading: clamp to
 * [0, M-1], blend the two nearest levels linearly (trilinear filtering). */
static void resolve_levels(const orc_pyramid* p, double lod, int* l0, int* l1, double* t) {
    double top = (double)(p->n_levels - 1);
    double lam = lod < 0.0 ? 0.0 : (lod > top ? top : lod);
    int a = (int)floor(lam);
    if (a > p->n_levels - 1) a = p->n_levels - 1;
    *l0 = a;
    *l1 = a + 1 < p->n_levels ? a + 1 : p->n_levels - 1;
    *t = lam - (double)a;
}

/* Bilinear stencil inside one level (Sec. 4.1: bilinear interpolation within a level).
 * Texel x has its centre at (x + 1/2) / W_l.  Outputs the 4 texel indices (within the
 * level, y * W_l + x) and their weights, ordered (x0,y0), (x1,y0), (x0,y1), (x1,y1). */
static void bilinear_stencil(const orc_pyramid* p, int l, double u, double v, long idx[4], double w[4]) {
    long W = lvl_w(p, l), H = lvl_h(p, l);
    if (p->address == ORC_WRAP) {
        u = u - floor(u);
        v = v - floor(v);
    }
    double s = u * (double)W - 0.5, r = v * (double)H - 0.5;
    double fx = floor(s), fy = floor(r);
    double a = s - fx, b = r - fy;
    long x0 = (long)fx, y0 = (long)fy, x1 = x0 + 1, y1 = y0 + 1;
    if (p->address == ORC_WRAP) {
        x0 = pos_mod(x0, W); x1 = pos_mod(x1, W);
        y0 = pos_mod(y0, H); y1 = pos_mod(y1, H);
    } else {
        x0 = clampl(x0, 0, W - 1); x1 = clampl(x1, 0, W - 1);
        y0 = clampl(y0, 0, H - 1); y1 = clampl(y1, 0, H - 1);
    }
    idx[0] = y0 * W + x0; w[0] = (1.0 - a) * (1.0 - b);
    idx[1] = y0 * W + x1; w[1] = a * (1.0 - b);
    idx[2] = y1 * W + x0; w[2] = (1.0 - a) * b;
    idx[3] = y1 * W + x1; w[3] = a * b;
}

/* The 8 taps of one query: level, index inside the level, and full trilinear weight. */
static void query_taps(const orc_pyramid* p, double u, double v, double lod,
                       int lv[8], long idx[8], double w[8]) {
    int l0, l1; double t;
    resolve_levels(p, lod, &l0, &l1, &t);
    double w0[4], w1[4];
    bilinear_stencil(p, l0, u, v, idx, w0);
    bilinear_stencil(p, l1, u, v, idx + 4, w1);
    for (int k = 0; k < 4; ++k) {
        lv[k] = l0; w[k] = (1.0 - t) * w0[k];
        lv[4 + k] = l1; w[4 + k] = t * w1[k];
    }
}

/* Latent code z(x) of Eq. (neural-brdf) for one query: the filtered fetch from the
 * hierarchical latent texture, z = sum over the 8 taps of weight * texel.  Non-finite uv or
 * lod give NaN. */
static void fetch_one(const orc_pyramid* p, const double* const* levels,
                      const double* uv, const double* lod, double* z) {
    const int C = p->channels;
    if (!(isfinite(uv[0]) && isfinite(uv[1]) && isfinite(lod[0]))) {
        for (int c = 0; c < C; ++c) z[c] = NAN;
        return;
    }
    int lv[8]; long idx[8]; double w[8];
    query_taps(p, uv[0], uv[1], lod[0], lv, idx, w);
    for (int c = 0; c < C; ++c) z[c] = 0.0;
    for (int k = 0; k < 8; ++k) {
        const double* T = levels[lv[k]] + idx[k] * C;
        for (int c = 0; c < C; ++c) z[c] += w[k] * T[c];
    }
}

/* Latent code with the level chosen by Russian roulette (Sec. 4.1, "Latent texture": a
 * fractional level index selects one of the two nearest levels at random, and the code is
 * fetched by bilinear interpolation within that level).  Reading: with t the fractional
 * part of the clamped level, the coarser level l1 is taken with probability t, the finer l0
 * with probability 1 - t; the caller supplies the uniform draw xi and the choice is l1 iff
 * xi < t (a NaN draw gives l0).  The expectation over xi of any function of the code is
 * (1 - t) times its value at the l0 code plus t times its value at the l1 code. */
static void fetch_one_rr(const orc_pyramid* p, const double* const* levels,
                         const double* uv, const double* lod, double xi, double* z) {
    const int C = p->channels;
    if (!(isfinite(uv[0]) && isfinite(uv[1]) && isfinite(lod[0]))) {
        for (int c = 0; c < C; ++c) z[c] = NAN;
        return;
    }
    int l0, l1; double t;
    resolve_levels(p, lod[0], &l0, &l1, &t);
    const int l = xi < t ? l1 : l0;
    long idx[4]; double w[4];
    bilinear_stencil(p, l, uv[0], uv[1], idx, w);
    for (int c = 0; c < C; ++c) z[c] = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double* T = levels[l] + idx[k] * C;
        for (int c = 0; c < C; ++c) z[c] += w[k] * T[c];
    }
}

/* z[n][C] for a batch of queries. */
int orc_fetch(const orc_pyramid* p, const double* const* levels, long n,
              const double* uv, const double* lod, double* z) {
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) fetch_one(p, levels, uv + 2 * i, lod + i, z + i * p->channels);
    return 0;
}

/* Texel addresses of the 8 taps of every query as flat indices into the level-concatenated
 * pyramid (level 0 first).  out[n][8]. */
int orc_taps(const orc_pyramid* p, long n, const double* uv, const double* lod, long* out) {
    long base[64];
    if (p->n_levels < 1 || p->n_levels > 64) return -1;
    long acc = 0;
    for (int l = 0; l < p->n_levels; ++l) { base[l] = acc; acc += (long)lvl_w(p, l) * lvl_h(p, l); }
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        int lv[8]; long idx[8]; double w[8];
        query_taps(p, uv[2 * i], uv[2 * i + 1], lod[i], lv, idx, w);
        for (int k = 0; k < 8; ++k) out[8 * i + k] = base[lv[k]] + idx[k];
    }
    return 0;
}

static double softplus(double q) { return fmax(q, 0.0) + log1p(exp(-fabs(q))); }
static double logistic(double q) { return 1.0 / (1.0 + exp(-q)); }

/* Decoder network g of Eq. (neural-brdf) with the shading-frame transform T taken as the
 * identity: input [z, wi, wo] (Cartesian directions, Sec. 9 "Energy conservation and
 * reciprocity"), ReLU hidden layers, softplus output.  Stores the activations of every
 * layer in act (act[0] = input, act[k] = output of layer k after ReLU, act[K] = q before
 * softplus) when act is not NULL.  Writes softplus of all dims[K] outputs. */
static void mlp_eval(int K, const int* dims, const double* params, const double* x,
                     double* rgb, double* const* act, double* scratch_a, double* scratch_b) {
    const double* in = x;
    double* out = scratch_a;
    const double* P = params;
    for (int k = 1; k <= K; ++k) {
        int fi = dims[k - 1], fo = dims[k];
        const double* W = P;
        const double* b = P + (long)fi * fo;
        for (int o = 0; o < fo; ++o) {
            double s = b[o];
            for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * in[j];
            out[o] = (k < K) ? (s > 0.0 ? s : 0.0) : s;
        }
        if (act) memcpy(act[k], out, sizeof(double) * fo);
        P += (long)fi * fo + fo;
        in = out;
        out = (out == scratch_a) ? scratch_b : scratch_a;
    }
    for (int c = 0; c < dims[K]; ++c) rgb[c] = softplus(in[c]);
}

/* Output widths of the decoder: RGB, or RGB followed by the albedo triplet. */
static int out_width_ok(int ko) { return ko == 3 || ko == 6; }

static int max_width(int K, const int* dims) {
    int m = 0;
    for (int k = 0; k <= K; ++k) if (dims[k] > m) m = dims[k];
    return m;
}

/* Full decode f(x, wi, wo) ~ g(z(x), wi, wo; theta): fetch, concatenation, decoder.  When
 * q_out is not NULL it receives the output-layer pre-activations q[n][KO]. */
int orc_decode(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
               const double* params, long n, const double* uv, const double* lod,
               const double* wi, const double* wo, double* rgb, double* q_out) {
    const int C = p->channels;
    if (K < 1 || K > 16 || dims[0] != C + 6 || !out_width_ok(dims[K])) return -1;
    const int KO = dims[K];
    const int MW = max_width(K, dims);
    #pragma omp parallel
    {
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * (MW + 6));
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            double* x = act[0];
            fetch_one(p, levels, uv + 2 * i, lod + i, x);
            for (int c = 0; c < 3; ++c) { x[C + c] = wi[3 * i + c]; x[C + 3 + c] = wo[3 * i + c]; }
            mlp_eval(K, dims, params, x, rgb + (long)KO * i, act, sa, sb);
            if (q_out) for (int c = 0; c < KO; ++c) q_out[(long)KO * i + c] = act[K][c];
            /* the paper defines no result for a non-finite position or level: NaN */
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i])))
                for (int c = 0; c < KO; ++c) rgb[(long)KO * i + c] = NAN;
        }
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(sa); free(sb);
    }
    return 0;
}

/* Decode with the level chosen by Russian roulette (fetch_one_rr), one draw xi[i] per
 * query; otherwise identical to orc_decode. */
int orc_decode_rr(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                  const double* params, long n, const double* uv, const double* lod, const double* xi,
                  const double* wi, const double* wo, double* rgb) {
    const int C = p->channels;
    if (K < 1 || K > 16 || dims[0] != C + 6 || !out_width_ok(dims[K])) return -1;
    const int KO = dims[K];
    const int MW = max_width(K, dims);
    #pragma omp parallel
    {
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * (MW + 6));
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            double* x = act[0];
            fetch_one_rr(p, levels, uv + 2 * i, lod + i, xi[i], x);
            for (int c = 0; c < 3; ++c) { x[C + c] = wi[3 * i + c]; x[C + 3 + c] = wo[3 * i + c]; }
            mlp_eval(K, dims, params, x, rgb + (long)KO * i, act, sa, sb);
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i])))
                for (int c = 0; c < KO; ++c) rgb[(long)KO * i + c] = NAN;
        }
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(sa); free(sb);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Learned shading frames (Sec. 4.2 "Transformation to learned shading frames", Eq.
 * frame-rotation; the bitangent as stated under "Alternative geometric priors" in Sec. 9).
 * One linear layer maps the latent code z to N normals n_f and N tangents t_f.  Each is
 * normalised on its own (the pair is not orthogonalised) and the bitangent is the
 * normalised cross product b_f = n_f x t_f / |n_f x t_f|.  T stacks the rows
 * t_1, b_1, n_1, ..., t_N, b_N, n_N (3N x 3), and the decoder input is [z, T wi, T wo].
 * Readings (the paper leaves them open): the layer has a bias; its 6N outputs are ordered
 * frame by frame as n (x, y, z) then t (x, y, z); a vector v is normalised as
 * v / sqrt(max(v.v, 1e-12)), so a zero vector stays zero; the cross product is taken of the
 * normalised n and t (the same direction as of the raw pair).
 * fparams: W_F[6N][C] row-major, then b_F[6N]. */
static void normalise3(const double* v, double* u) {
    double s = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double r = 1.0 / sqrt(s > 1e-12 ? s : 1e-12);
    for (int c = 0; c < 3; ++c) u[c] = v[c] * r;
}

/* out[0 .. 3N) = T wi, out[3N .. 6N) = T wo for one latent code z. */
static void frame_transform(int nf, int C, const double* fparams, const double* z,
                            const double* wi, const double* wo, double* out) {
    const double* W = fparams;
    const double* bias = fparams + 6L * nf * C;
    for (int f = 0; f < nf; ++f) {
        double raw[6], nrm[3], tan[3], crs[3], bit[3];
        for (int r = 0; r < 6; ++r) {
            double s = bias[6 * f + r];
            for (int c = 0; c < C; ++c) s += W[(6L * f + r) * C + c] * z[c];
            raw[r] = s;
        }
        normalise3(raw, nrm);
        normalise3(raw + 3, tan);
        crs[0] = nrm[1] * tan[2] - nrm[2] * tan[1];
        crs[1] = nrm[2] * tan[0] - nrm[0] * tan[2];
        crs[2] = nrm[0] * tan[1] - nrm[1] * tan[0];
        normalise3(crs, bit);
        const double* row[3] = {tan, bit, nrm};
        for (int r = 0; r < 3; ++r) {
            out[3 * f + r] = row[r][0] * wi[0] + row[r][1] * wi[1] + row[r][2] * wi[2];
            out[3 * nf + 3 * f + r] = row[r][0] * wo[0] + row[r][1] * wo[1] + row[r][2] * wo[2];
        }
    }
}

/* [T wi, T wo] (n x 6N) of n latent codes z[n][C]; exposed for the frame pins. */
int orc_frames(int nf, int C, const double* fparams, long n, const double* z,
               const double* wi, const double* wo, double* out) {
    if (nf < 1 || nf > 8 || C < 1) return -1;
    for (long i = 0; i < n; ++i)
        frame_transform(nf, C, fparams, z + (long)C * i, wi + 3 * i, wo + 3 * i, out + 6L * nf * i);
    return 0;
}

/* Full decode with learned shading frames: fetch (trilinear, or one level by Russian
 * roulette when xi is not NULL), frame transform, decoder on [z, T wi, T wo]
 * (dims[0] = C + 6N). */
int orc_decode_frames(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                      const double* params, int nf, const double* fparams, long n, const double* uv,
                      const double* lod, const double* xi, const double* wi, const double* wo,
                      double* rgb) {
    const int C = p->channels;
    if (nf < 1 || nf > 8 || K < 1 || K > 16 || dims[0] != C + 6 * nf || !out_width_ok(dims[K])) return -1;
    const int KO = dims[K];
    const int MW = max_width(K, dims);
    #pragma omp parallel
    {
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * (MW + 6 * nf));
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            double* x = act[0];
            if (xi) fetch_one_rr(p, levels, uv + 2 * i, lod + i, xi[i], x);
            else fetch_one(p, levels, uv + 2 * i, lod + i, x);
            frame_transform(nf, C, fparams, x, wi + 3 * i, wo + 3 * i, x + C);
            mlp_eval(K, dims, params, x, rgb + (long)KO * i, act, sa, sb);
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i])))
                for (int c = 0; c < KO; ++c) rgb[(long)KO * i + c] = NAN;
        }
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(sa); free(sb);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Importance sampling with the analytic proxy (Sec. 4.3 "Importance sampling"; App. A
 * "Importance sampling details", Eq. pdf_full and Eq. pdf_spec).
 *
 * A second decoder maps [z, wi] to 9 raw outputs, turned into the proxy parameters
 * p = {w_d, mu_dx, mu_dy, w_s, alpha_x, alpha_y, rho, mu_sx, mu_sy} by output activations
 * built on quadratic approximations of tanh and sinh, and a softmax for (w_d, w_s).
 * Readings (the paper names the activations and ranges but not their formulas):
 *   qtanh(x) = x (1 - |x| / 4) for |x| < 2, sign(x) beyond (C1, slope 1 at 0, flat at +-2);
 *   qsinh(x) = x (1 + |x| / 2) (odd, C1, slope 1 at 0, quadratic growth);
 *   (w_d, w_s) = softmax(raw_0, raw_3); mu = qsinh(raw);
 *   alpha = 1e-3 + (1 - 1e-3) (1 + qtanh(raw)) / 2 and rho = 0.999 qtanh(raw): the floor and
 *   the factor keep M invertible (the paper gives the closed ranges [0, 1] and [-1, 1]).
 * PDF over the whole sphere of wo:  p = w_d p_d + w_s p_s.
 *   p_d: cosine lobe about n_d = normalise(-mu_dx, -mu_dy, 1): max(0, wo . n_d) / pi.
 *   p_s: with h = normalise(wi + wo), taken in the upper hemisphere (h and -h reflect wi to the
 *        same wo; the sampler only produces h_z > 0), h' = M^-1 h / |M^-1 h|,
 *        p_s = D_std(h') det(M^-1) / |M^-1 h|^3 / (4 |wo . h|), where D_std is the density of
 *        the alpha = 1 GGX normal sampler, max(h'_z, 0) / pi (the NDF times the cosine: the
 *        density that sampler draws, so p_s integrates to one); p_s = 0 where wi + wo = 0.
 * Sampling with u in [0,1)^3: the diffuse lobe if u_0 < w_d, else the specular one.
 *   diffuse: Malley's cosine sample (sqrt(u_1) cos 2 pi u_2, sqrt(u_1) sin 2 pi u_2,
 *            sqrt(1 - u_1)), turned by the minimal rotation that takes +z to n_d;
 *   specular: h_std the same cosine sample (the alpha = 1 GGX normal sampler),
 *             h = normalise(M h_std), wo = 2 (wi . h) h - wi. */
static double qtanh(double x) { return fabs(x) < 2.0 ? x * (1.0 - 0.25 * fabs(x)) : (x > 0 ? 1.0 : -1.0); }
static double qsinh(double x) { return x * (1.0 + 0.5 * fabs(x)); }

void orc_proxy_activate(const double* raw, double* p) {
    const double m = raw[0] > raw[3] ? raw[0] : raw[3];
    const double ed = exp(raw[0] - m), es = exp(raw[3] - m);
    p[0] = ed / (ed + es);
    p[3] = es / (ed + es);
    p[1] = qsinh(raw[1]);
    p[2] = qsinh(raw[2]);
    p[4] = 1e-3 + (1.0 - 1e-3) * 0.5 * (1.0 + qtanh(raw[4]));
    p[5] = 1e-3 + (1.0 - 1e-3) * 0.5 * (1.0 + qtanh(raw[5]));
    p[6] = 0.999 * qtanh(raw[6]);
    p[7] = qsinh(raw[7]);
    p[8] = qsinh(raw[8]);
}

/* M of App. A, row-major 3x3, and its inverse (M is upper block triangular with last row e_z). */
static void proxy_m(const double* p, double M[9], double Mi[9], double* det_mi) {
    const double ax = p[4], ay = p[5], rho = p[6], mx = p[7], my = p[8];
    const double sr = sqrt(1.0 - rho * rho);
    M[0] = ax;       M[1] = 0.0;     M[2] = -mx;
    M[3] = ay * rho; M[4] = ay * sr; M[5] = -my;
    M[6] = 0.0;      M[7] = 0.0;     M[8] = 1.0;
    /* inverse of A = [[ax, 0], [ay rho, ay sr]] and of the translation column */
    const double i00 = 1.0 / ax, i10 = -rho / (ax * sr), i11 = 1.0 / (ay * sr);
    Mi[0] = i00; Mi[1] = 0.0; Mi[2] = i00 * mx;
    Mi[3] = i10; Mi[4] = i11; Mi[5] = i10 * mx + i11 * my;
    Mi[6] = 0.0; Mi[7] = 0.0; Mi[8] = 1.0;
    *det_mi = 1.0 / (ax * ay * sr);
}

static void mat3v(const double* A, const double* v, double* o) {
    for (int r = 0; r < 3; ++r) o[r] = A[3 * r] * v[0] + A[3 * r + 1] * v[1] + A[3 * r + 2] * v[2];
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

double orc_proxy_pdf(const double* p, const double* wi, const double* wo) {
    const double inv_pi = 1.0 / 3.14159265358979323846;
    double nd[3] = {-p[1], -p[2], 1.0};
    const double ln = sqrt(dot3(nd, nd));
    for (int c = 0; c < 3; ++c) nd[c] /= ln;
    const double cd = dot3(wo, nd);
    const double pd = cd > 0.0 ? cd * inv_pi : 0.0;
    double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
    const double lh = sqrt(dot3(h, h));
    double ps = 0.0;
    if (lh > 0.0) {
        const double sg = h[2] < 0.0 ? -1.0 : 1.0;
        for (int c = 0; c < 3; ++c) h[c] *= sg / lh;
        double M[9], Mi[9], det_mi, hp[3];
        proxy_m(p, M, Mi, &det_mi);
        mat3v(Mi, h, hp);
        const double lp = sqrt(dot3(hp, hp));
        const double dstd = hp[2] > 0.0 ? (hp[2] / lp) * inv_pi : 0.0;
        const double oh = fabs(dot3(wo, h));
        ps = oh > 0.0 ? dstd * det_mi / (lp * lp * lp) / (4.0 * oh) : 0.0;
    }
    return p[0] * pd + p[3] * ps;
}

static void cosine_sample(double u1, double u2, double* v) {
    const double r = sqrt(u1), phi = 2.0 * 3.14159265358979323846 * u2;
    v[0] = r * cos(phi);
    v[1] = r * sin(phi);
    v[2] = sqrt(1.0 - u1);
}

double orc_proxy_sample(const double* p, const double* wi, const double* u, double* wo) {
    double v[3];
    cosine_sample(u[1], u[2], v);
    if (u[0] < p[0]) {
        double n[3] = {-p[1], -p[2], 1.0};
        const double ln = sqrt(dot3(n, n));
        for (int c = 0; c < 3; ++c) n[c] /= ln;
        /* minimal rotation taking e_z to n (n_z > 0): columns R e_x, R e_y, R e_z = n */
        const double a = 1.0 / (1.0 + n[2]);
        const double ex[3] = {1.0 - a * n[0] * n[0], -a * n[0] * n[1], -n[0]};
        const double ey[3] = {-a * n[0] * n[1], 1.0 - a * n[1] * n[1], -n[1]};
        for (int c = 0; c < 3; ++c) wo[c] = v[0] * ex[c] + v[1] * ey[c] + v[2] * n[c];
    } else {
        double M[9], Mi[9], det_mi, h[3];
        proxy_m(p, M, Mi, &det_mi);
        mat3v(M, v, h);
        const double lh = sqrt(dot3(h, h));
        for (int c = 0; c < 3; ++c) h[c] /= lh;
        const double d = dot3(wi, h);
        for (int c = 0; c < 3; ++c) wo[c] = 2.0 * d * h[c] - wi[c];
    }
    return orc_proxy_pdf(p, wi, wo);
}

/* Proxy parameters of n queries: fetch (trilinear), sampling decoder on [z, wi] (ReLU hidden
 * layers, 9 linear outputs), activations.  sdims[0] = C + 3, sdims[K] = 9.  out[n][9]. */
int orc_sampler_params(const orc_pyramid* p, const double* const* levels, int K, const int* sdims,
                       const double* sparams, long n, const double* uv, const double* lod, const double* wi,
                       double* out) {
    const int C = p->channels;
    if (K < 1 || K > 16 || sdims[0] != C + 3 || sdims[K] != 9) return -1;
    const int MW = max_width(K, sdims);
    #pragma omp parallel
    {
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * (MW + 3));
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        double unused[9];   /* the raw outputs are taken from act[K], not through softplus */
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            double* x = act[0];
            fetch_one(p, levels, uv + 2 * i, lod + i, x);
            for (int c = 0; c < 3; ++c) x[C + c] = wi[3 * i + c];
            mlp_eval(K, sdims, sparams, x, unused, act, sa, sb);
            orc_proxy_activate(act[K], out + 9 * i);
        }
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(sa); free(sb);
    }
    return 0;
}

/* PDF of given wo (pdf_out[n]) or samples from u[n][3] (wo_out[n][3] and their pdf) for proxy
 * parameters params[n][9]. */
int orc_proxy_batch(long n, const double* params, const double* wi, const double* wo_in, const double* u,
                    double* wo_out, double* pdf_out) {
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        if (u) pdf_out[i] = orc_proxy_sample(params + 9 * i, wi + 3 * i, u + 3 * i, wo_out + 3 * i);
        else pdf_out[i] = orc_proxy_pdf(params + 9 * i, wi + 3 * i, wo_in + 3 * i);
    }
    return 0;
}

/* Mean squared error of the decoded outputs against targets [n][KO], L = 1/(3n) sum over the
 * KO = 3 or 6 outputs of (out - target)^2: the RGB loss, plus for KO = 6 the albedo loss, each a
 * mean over 3n values, added with equal weight (Sec. 5.2 "Optimization": the albedo output is
 * fitted with an L2 loss against one-sample estimates of Eq. albedo),
 * and its exact gradient with respect to every decoder parameter and every texel (direct
 * optimisation of the latent texture by backpropagation, Sec. 5 and Sec. 2 "Obtaining latent
 * textures").  ReLU'(0) = 0, softplus' = logistic.  dparams is overwritten; dlevels[l] (same
 * layout as levels[l]) is overwritten.  Gradients of uv, lod and directions are not formed.
 * Samples whose uv or lod is not finite add nothing to the loss or the gradients; n (all
 * samples) stays the denominator. */
int orc_loss_grad(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                  const double* params, long n, const double* uv, const double* lod,
                  const double* wi, const double* wo, const double* target,
                  double* loss, double* dparams, double* const* dlevels) {
    const int C = p->channels;
    if (K < 1 || K > 16 || dims[0] != C + 6 || !out_width_ok(dims[K])) return -1;
    const int KO = dims[K];
    long np = 0;
    for (int k = 1; k <= K; ++k) np += (long)dims[k - 1] * dims[k] + dims[k];
    for (int l = 0; l < p->n_levels; ++l)
        memset(dlevels[l], 0, sizeof(double) * (size_t)lvl_w(p, l) * lvl_h(p, l) * C);
    memset(dparams, 0, sizeof(double) * np);
    const int MW = max_width(K, dims);
    double total = 0.0;
    #pragma omp parallel reduction(+:total)
    {
        double* g = (double*)calloc(np, sizeof(double));
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * (MW + 6));
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        double* d = (double*)malloc(sizeof(double) * (MW + 6));
        double* dprev = (double*)malloc(sizeof(double) * (MW + 6));
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            /* a sample with a non-finite position or level has no defined output (the paper
             * defines none); it is skipped: no loss term, no gradient, while the mean still
             * divides by 3n over the whole batch */
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i]))) continue;
            int lv[8]; long idx[8]; double w[8];
            query_taps(p, uv[2 * i], uv[2 * i + 1], lod[i], lv, idx, w);
            double* x = act[0];
            for (int c = 0; c < C; ++c) x[c] = 0.0;
            for (int k = 0; k < 8; ++k) {
                const double* T = levels[lv[k]] + idx[k] * C;
                for (int c = 0; c < C; ++c) x[c] += w[k] * T[c];
            }
            for (int c = 0; c < 3; ++c) { x[C + c] = wi[3 * i + c]; x[C + 3 + c] = wo[3 * i + c]; }
            double y[6];
            mlp_eval(K, dims, params, x, y, act, sa, sb);
            /* output layer: dL/dq = 2 (out - target) / (3n) * logistic(q) */
            for (int c = 0; c < KO; ++c) {
                double e = y[c] - target[(long)KO * i + c];
                total += e * e;
                d[c] = 2.0 * e / (3.0 * (double)n) * logistic(act[K][c]);
            }
            /* walk layers backwards; parameter block offsets */
            long off[17]; long o = 0;
            for (int k = 1; k <= K; ++k) { off[k] = o; o += (long)dims[k - 1] * dims[k] + dims[k]; }
            for (int k = K; k >= 1; --k) {
                int fi = dims[k - 1], fo = dims[k];
                const double* W = params + off[k];
                double* gW = g + off[k];
                double* gb = gW + (long)fi * fo;
                const double* a_in = act[k - 1];
                for (int r = 0; r < fo; ++r) {
                    gb[r] += d[r];
                    for (int j = 0; j < fi; ++j) gW[(long)r * fi + j] += d[r] * a_in[j];
                }
                for (int j = 0; j < fi; ++j) {
                    double s = 0.0;
                    for (int r = 0; r < fo; ++r) s += W[(long)r * fi + j] * d[r];
                    /* ReLU derivative of the layer below (its stored output is post-ReLU) */
                    if (k > 1) s = (a_in[j] > 0.0) ? s : 0.0;
                    dprev[j] = s;
                }
                memcpy(d, dprev, sizeof(double) * fi);
            }
            /* d now holds dL/dx; scatter dL/dz into the 8 taps */
            for (int k = 0; k < 8; ++k) {
                double* G = dlevels[lv[k]] + idx[k] * C;
                for (int c = 0; c < C; ++c) {
                    double add = w[k] * d[c];
                    #pragma omp atomic
                    G[c] += add;
                }
            }
        }
        #pragma omp critical
        for (long j = 0; j < np; ++j) dparams[j] += g[j];
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(g); free(sa); free(sb); free(d); free(dprev);
    }
    *loss = total / (3.0 * (double)n);
    return 0;
}

/* Reverse of normalise3: given u = v / sqrt(max(v.v, 1e-12)) and the gradient gu of a loss
 * with respect to u, the gradient with respect to v.  Where v.v > 1e-12 the map is
 * v / |v| with Jacobian (I - u u^T) / |v|; below the floor it is linear, v / 1e-6. */
static void normalise3_back(const double* v, const double* u, const double* gu, double* gv) {
    double s = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    if (s > 1e-12) {
        double r = 1.0 / sqrt(s);
        double ug = u[0] * gu[0] + u[1] * gu[1] + u[2] * gu[2];
        for (int c = 0; c < 3; ++c) gv[c] = (gu[c] - u[c] * ug) * r;
    } else {
        for (int c = 0; c < 3; ++c) gv[c] = gu[c] * 1e6;
    }
}

static void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Mean squared error of the decode with learned shading frames (Sec. 4.2 "Transformation to
 * learned shading frames", Eq. frame-rotation; the frame layer is trained jointly with the
 * decoder and the latents, Sec. 5) and its exact gradient with respect to the decoder
 * parameters, the frame layer (W_F, b_F) and every texel.  Trilinear fetch; input
 * [z, T wi, T wo] with T and its conventions as in frame_transform.  The chain rule, per frame,
 * from the gradient G of the decoder input block T w (rows t, b, n of T):
 *   dL/d row = G_i[row] wi + G_o[row] wo for row in (t^, b^, n^);
 *   b^ = c / |c| with c = n^ x t^:  dc from the normalisation, then dn^ += t^ x dc and
 *   dt^ += dc x n^ (d(a x b) . dc = da . (b x dc) + db . (dc x a));
 *   n^, t^ normalise the raw layer outputs n, t: dn, dt from the normalisation;
 *   the raw outputs are W_F z + b_F: dW_F += [dn, dt] z^T, db_F += [dn, dt], and the latent
 *   code receives W_F^T [dn, dt] on top of the decoder's own input gradient.
 * dparams, dfparams are overwritten; dlevels[l] is overwritten.  Non-finite samples are skipped
 * as in orc_loss_grad; the mean divides by 3n. */
int orc_loss_grad_frames(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                         const double* params, int nf, const double* fparams, long n, const double* uv,
                         const double* lod, const double* wi, const double* wo, const double* target,
                         double* loss, double* dparams, double* dfparams, double* const* dlevels) {
    const int C = p->channels;
    if (nf < 1 || nf > 8 || K < 1 || K > 16 || dims[0] != C + 6 * nf || !out_width_ok(dims[K])) return -1;
    const int KO = dims[K];
    long np = 0;
    for (int k = 1; k <= K; ++k) np += (long)dims[k - 1] * dims[k] + dims[k];
    const long nfp = 6L * nf * C + 6L * nf;
    for (int l = 0; l < p->n_levels; ++l)
        memset(dlevels[l], 0, sizeof(double) * (size_t)lvl_w(p, l) * lvl_h(p, l) * C);
    memset(dparams, 0, sizeof(double) * np);
    memset(dfparams, 0, sizeof(double) * nfp);
    const int MW = max_width(K, dims) + 6 * nf;
    const double* WF = fparams;
    const double* bF = fparams + 6L * nf * C;
    double total = 0.0;
    #pragma omp parallel reduction(+:total)
    {
        double* g = (double*)calloc(np, sizeof(double));
        double* gf = (double*)calloc(nfp, sizeof(double));
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * MW);
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        double* d = (double*)malloc(sizeof(double) * MW);
        double* dprev = (double*)malloc(sizeof(double) * MW);
        double* z = (double*)malloc(sizeof(double) * C);
        double* dz = (double*)malloc(sizeof(double) * C);
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i]))) continue;
            int lv[8]; long idx[8]; double w[8];
            query_taps(p, uv[2 * i], uv[2 * i + 1], lod[i], lv, idx, w);
            for (int c = 0; c < C; ++c) z[c] = 0.0;
            for (int k = 0; k < 8; ++k) {
                const double* T = levels[lv[k]] + idx[k] * C;
                for (int c = 0; c < C; ++c) z[c] += w[k] * T[c];
            }
            const double* wiv = wi + 3 * i;
            const double* wov = wo + 3 * i;
            double* x = act[0];
            for (int c = 0; c < C; ++c) x[c] = z[c];
            frame_transform(nf, C, fparams, z, wiv, wov, x + C);
            double y[6];
            mlp_eval(K, dims, params, x, y, act, sa, sb);
            for (int c = 0; c < KO; ++c) {
                double e = y[c] - target[(long)KO * i + c];
                total += e * e;
                d[c] = 2.0 * e / (3.0 * (double)n) * logistic(act[K][c]);
            }
            long off[17]; long o = 0;
            for (int k = 1; k <= K; ++k) { off[k] = o; o += (long)dims[k - 1] * dims[k] + dims[k]; }
            for (int k = K; k >= 1; --k) {
                int fi = dims[k - 1], fo = dims[k];
                const double* W = params + off[k];
                double* gW = g + off[k];
                double* gb = gW + (long)fi * fo;
                const double* a_in = act[k - 1];
                for (int r = 0; r < fo; ++r) {
                    gb[r] += d[r];
                    for (int j = 0; j < fi; ++j) gW[(long)r * fi + j] += d[r] * a_in[j];
                }
                for (int j = 0; j < fi; ++j) {
                    double sum = 0.0;
                    for (int r = 0; r < fo; ++r) sum += W[(long)r * fi + j] * d[r];
                    if (k > 1) sum = (a_in[j] > 0.0) ? sum : 0.0;
                    dprev[j] = sum;
                }
                memcpy(d, dprev, sizeof(double) * fi);
            }
            /* d = dL/d[z, T wi, T wo]; the latent code's own part, then each frame */
            for (int c = 0; c < C; ++c) dz[c] = d[c];
            const double* Gi = d + C;
            const double* Go = d + C + 3 * nf;
            for (int f = 0; f < nf; ++f) {
                double raw[6], nrm[3], tan[3], crs[3], bit[3];
                for (int r = 0; r < 6; ++r) {
                    double sum = bF[6 * f + r];
                    for (int c = 0; c < C; ++c) sum += WF[(6L * f + r) * C + c] * z[c];
                    raw[r] = sum;
                }
                normalise3(raw, nrm);
                normalise3(raw + 3, tan);
                cross3(nrm, tan, crs);
                normalise3(crs, bit);
                double gt[3], gbv[3], gn[3], gc[3], t1[3], t2[3], draw[6];
                for (int c = 0; c < 3; ++c) {
                    gt[c] = Gi[3 * f + 0] * wiv[c] + Go[3 * f + 0] * wov[c];
                    gbv[c] = Gi[3 * f + 1] * wiv[c] + Go[3 * f + 1] * wov[c];
                    gn[c] = Gi[3 * f + 2] * wiv[c] + Go[3 * f + 2] * wov[c];
                }
                normalise3_back(crs, bit, gbv, gc);
                cross3(tan, gc, t1);
                cross3(gc, nrm, t2);
                for (int c = 0; c < 3; ++c) { gn[c] += t1[c]; gt[c] += t2[c]; }
                normalise3_back(raw, nrm, gn, draw);
                normalise3_back(raw + 3, tan, gt, draw + 3);
                for (int r = 0; r < 6; ++r) {
                    gf[6L * nf * C + 6 * f + r] += draw[r];
                    for (int c = 0; c < C; ++c) {
                        gf[(6L * f + r) * C + c] += draw[r] * z[c];
                        dz[c] += WF[(6L * f + r) * C + c] * draw[r];
                    }
                }
            }
            for (int k = 0; k < 8; ++k) {
                double* G = dlevels[lv[k]] + idx[k] * C;
                for (int c = 0; c < C; ++c) {
                    double add = w[k] * dz[c];
                    #pragma omp atomic
                    G[c] += add;
                }
            }
        }
        #pragma omp critical
        {
            for (long j = 0; j < np; ++j) dparams[j] += g[j];
            for (long j = 0; j < nfp; ++j) dfparams[j] += gf[j];
        }
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(g); free(gf); free(sa); free(sb); free(d); free(dprev); free(z); free(dz);
    }
    *loss = total / (3.0 * (double)n);
    return 0;
}

/* One Adam update (Kingma & Ba; the training of Sec. 5 optimises decoder and latents with
 * it), step counted from 1, no weight decay:
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 *   p <- p - lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps). */
void orc_adam(long n, double* p, double* m, double* v, const double* g,
              double lr, double b1, double b2, double eps, long step) {
    double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (long i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* ------------------------------------------------------------------------------------
 * Reduced-precision storage (Sec. 5 "Precision": FP16 post-training quantisation at load;
 * lower precisions are named as future work).  Round-to-nearest-even onto a binary format
 * with `mant` fraction bits and minimum normal exponent `emin`; values past `maxv` either
 * saturate (E4M3FN has no infinity) or become infinite (IEEE half). */
static double round_format(double x, int mant, int emin, double maxv, int saturate) {
    if (isnan(x)) return x;
    double ax = fabs(x);
    if (ax == 0.0) return x;
    int e;
    frexp(ax, &e);            /* ax = f * 2^e, f in [0.5, 1) -> leading exponent e - 1 */
    int lead = e - 1;
    if (lead < emin) lead = emin;
    double quantum = ldexp(1.0, lead - mant);
    int old = fegetround();
    fesetround(FE_TONEAREST);
    double r = nearbyint(ax / quantum) * quantum;
    fesetround(old);
    if (r > maxv) r = saturate ? maxv : INFINITY;
    return copysign(r, x);
}

/* IEEE binary16: 10 fraction bits, min normal 2^-14, max 65504, overflow to infinity
 * (a value at or past 65520 rounds to infinity). */
double orc_round_fp16(double x) {
    double ax = fabs(x);
    if (ax >= 65520.0) return copysign(INFINITY, x);
    return round_format(x, 10, -14, 65504.0, 0);
}

/* OCP 8-bit E4M3FN: 3 fraction bits, min normal 2^-6, max 448, saturating. */
double orc_round_e4m3(double x) { return round_format(x, 3, -6, 448.0, 1); }

void orc_round_array(long n, const double* x, double* y, int fmt) {
    for (long i = 0; i < n; ++i) y[i] = fmt == 0 ? orc_round_fp16(x[i]) : orc_round_e4m3(x[i]);
}

/* Decode with reduced-precision decoder arithmetic, to separate the error of the number
 * formats from the error of the summation order (a diagnostic, not a reference):
 *   the network input [z, wi, wo] and every hidden activation are rounded to `afmt`
 *   after multiplication by the layer's activation scale sa[k]; the weights of layer k are
 *   given already rounded and multiplied by sw[k]; products accumulate exactly (double);
 *   the sum is divided by sw[k] * sa[k] before the (unrounded) bias.  fmt: 0 = FP16, 1 = E4M3,
 *   2 = no rounding.  The texels are used as given. */
/* Latent code with the filter arithmetic of the FP16 decoders (reading R15b: the latents are
 * 16-bit images, Sec. 7.1 "Neural material shaders", and the paper leaves the arithmetic of
 * their interpolation open).  The eight trilinear weights of query_taps are rounded to FP16;
 * the sum over the taps, in their stencil order (level l0, then l1; (x0,y0), (x1,y0),
 * (x0,y1), (x1,y1)), is kept in FP16: the first tap's product rounded once, then every
 * multiply-add rounded once.  Non-finite uv or lod give NaN. */
static void fetch_one_fp16(const orc_pyramid* p, const double* const* levels,
                           const double* uv, const double* lod, double* z) {
    const int C = p->channels;
    if (!(isfinite(uv[0]) && isfinite(uv[1]) && isfinite(lod[0]))) {
        for (int c = 0; c < C; ++c) z[c] = NAN;
        return;
    }
    int lv[8]; long idx[8]; double w[8];
    query_taps(p, uv[0], uv[1], lod[0], lv, idx, w);
    for (int k = 0; k < 8; ++k) {
        const double wk = orc_round_fp16(w[k]);
        const double* T = levels[lv[k]] + idx[k] * C;
        for (int c = 0; c < C; ++c) z[c] = orc_round_fp16(k == 0 ? wk * T[c] : wk * T[c] + z[c]);
    }
}

/* z[n][C] for a batch of queries, filtered as in fetch_one_fp16. */
int orc_fetch_fp16(const orc_pyramid* p, const double* const* levels, long n,
                   const double* uv, const double* lod, double* z) {
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) fetch_one_fp16(p, levels, uv + 2 * i, lod + i, z + i * p->channels);
    return 0;
}

/* orc_decode_quant with the latent code filtered as the FP16 decoders filter it
 * (fetch_one_fp16) when blend_fp16 is 1, exactly when it is 0. */
int orc_decode_quant_blend(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                           const double* qparams, const double* sw, const double* sa, const int* afmt,
                           long n, const double* uv, const double* lod, const double* wi, const double* wo,
                           double* rgb, int blend_fp16);

int orc_decode_quant(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                     const double* qparams, const double* sw, const double* sa, const int* afmt,
                     long n, const double* uv, const double* lod, const double* wi, const double* wo,
                     double* rgb) {
    return orc_decode_quant_blend(p, levels, K, dims, qparams, sw, sa, afmt, n, uv, lod, wi, wo, rgb, 0);
}

int orc_decode_quant_blend(const orc_pyramid* p, const double* const* levels, int K, const int* dims,
                           const double* qparams, const double* sw, const double* sa, const int* afmt,
                           long n, const double* uv, const double* lod, const double* wi, const double* wo,
                           double* rgb, int blend_fp16) {
    const int C = p->channels;
    if (K < 1 || K > 16 || dims[0] != C + 6 || !out_width_ok(dims[K])) return -1;
    const int KO = dims[K];
    const int MW = max_width(K, dims);
    #pragma omp parallel
    {
        double* a = (double*)malloc(sizeof(double) * (MW + 6));
        double* b = (double*)malloc(sizeof(double) * (MW + 6));
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            if (blend_fp16) fetch_one_fp16(p, levels, uv + 2 * i, lod + i, a);
            else fetch_one(p, levels, uv + 2 * i, lod + i, a);
            for (int c = 0; c < 3; ++c) { a[C + c] = wi[3 * i + c]; a[C + 3 + c] = wo[3 * i + c]; }
            const double* P = qparams;
            for (int k = 1; k <= K; ++k) {
                int fi = dims[k - 1], fo = dims[k];
                for (int j = 0; j < fi; ++j) {
                    double s = a[j] * sa[k - 1];
                    a[j] = afmt[k - 1] == 2 ? s : (afmt[k - 1] == 0 ? orc_round_fp16(s) : orc_round_e4m3(s));
                }
                const double* W = P;
                const double* bias = P + (long)fi * fo;
                for (int o = 0; o < fo; ++o) {
                    double s = 0.0;
                    for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * a[j];
                    s = s / (sw[k - 1] * sa[k - 1]) + bias[o];
                    b[o] = (k < K) ? (s > 0.0 ? s : 0.0) : s;
                }
                P += (long)fi * fo + fo;
                double* t = a; a = b; b = t;
            }
            for (int c = 0; c < KO; ++c) rgb[(long)KO * i + c] = softplus(a[c]);
        }
        free(a); free(b);
    }
    return 0;
}

/* Proxy parameters with the reduced-precision arithmetic of the matrix-core sampling decoder
 * (Sec. 5.2 "Precision": the sampler's master parameters converted to FP16 at load, as the
 * BRDF decoder's), a diagnostic as orc_decode_quant is: the latent code is filtered as in
 * fetch_one_fp16 when blend_fp16 is 1 (exactly when 0); every layer's input (the network input
 * [z, wi], then each ReLU'd hidden activation) is rounded to FP16 when fmt is 0 (kept when 2);
 * the weights are given already rounded; products accumulate exactly; the bias is added
 * unrounded; the raw outputs pass through orc_proxy_activate.  sdims[0] = C + 3,
 * sdims[K] = 9.  out[n][9]; non-finite uv or lod give NaN parameters. */
int orc_sampler_params_quant(const orc_pyramid* p, const double* const* levels, int K, const int* sdims,
                             const double* qparams, int fmt, long n, const double* uv, const double* lod,
                             const double* wi, double* out, int blend_fp16) {
    const int C = p->channels;
    if (K < 1 || K > 16 || sdims[0] != C + 3 || sdims[K] != 9 || (fmt != 0 && fmt != 2)) return -1;
    const int MW = max_width(K, sdims);
    #pragma omp parallel
    {
        double* a = (double*)malloc(sizeof(double) * (MW + 3));
        double* b = (double*)malloc(sizeof(double) * (MW + 3));
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            double* x = a;
            double* y = b;
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i]))) {
                for (int c = 0; c < 9; ++c) out[9 * i + c] = NAN;
                continue;
            }
            if (blend_fp16) fetch_one_fp16(p, levels, uv + 2 * i, lod + i, x);
            else fetch_one(p, levels, uv + 2 * i, lod + i, x);
            for (int c = 0; c < 3; ++c) x[C + c] = wi[3 * i + c];
            const double* P = qparams;
            for (int k = 1; k <= K; ++k) {
                const int fi = sdims[k - 1], fo = sdims[k];
                if (fmt == 0)
                    for (int j = 0; j < fi; ++j) x[j] = orc_round_fp16(x[j]);
                const double* W = P;
                const double* bias = P + (long)fi * fo;
                for (int o = 0; o < fo; ++o) {
                    double s = 0.0;
                    for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * x[j];
                    s += bias[o];
                    y[o] = (k < K) ? (s > 0.0 ? s : 0.0) : s;
                }
                P += (long)fi * fo + fo;
                double* t = x; x = y; y = t;
            }
            orc_proxy_activate(x, out + 9 * i);
        }
        free(a); free(b);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Encoder (Sec. 5.1 "Encoder"): an MLP E from the parameters of the original material at a
 * location (albedo, roughness, ...: A attributes) to its latent code.  Reading: ReLU hidden
 * layers, a linear output layer of C units; edims = [A, H_1, ..., C] with KE layers, packed as
 * the decoder is (W_1[edims[1]][A], b_1, W_2, b_2, ...).  In the first training phase the
 * latent code of a query is E applied to the material parameters filtered at the query (the
 * trilinear filter of query_taps over a pyramid of the parameters, prefiltered level by
 * level) and goes to the decoder directly; the latent texture is then initialised with E of
 * every texel of that pyramid (orc_encode). */

static long mlp_param_count(int K, const int* dims) {
    long np = 0;
    for (int k = 1; k <= K; ++k) np += (long)dims[k - 1] * dims[k] + dims[k];
    return np;
}

/* act[0] = x; act[k] = layer k's output, ReLU'd below the last layer, linear at the last. */
static void enc_forward(int KE, const int* edims, const double* ep, const double* x, double* const* act) {
    memcpy(act[0], x, sizeof(double) * edims[0]);
    const double* P = ep;
    for (int k = 1; k <= KE; ++k) {
        const int fi = edims[k - 1], fo = edims[k];
        const double* W = P;
        const double* b = P + (long)fi * fo;
        for (int o = 0; o < fo; ++o) {
            double s = b[o];
            for (int j = 0; j < fi; ++j) s += W[(long)o * fi + j] * act[k - 1][j];
            act[k][o] = (k < KE) ? (s > 0.0 ? s : 0.0) : s;
        }
        P += (long)fi * fo + fo;
    }
}

static int enc_dims_ok(int KE, const int* edims) {
    if (KE < 1 || KE > 16) return 0;
    for (int k = 0; k <= KE; ++k) if (edims[k] < 1) return 0;
    return 1;
}

/* z[n][C] = E(attrs[n][A]): the encoder on given parameter rows (texels). */
int orc_encode(int KE, const int* edims, const double* eparams, long n, const double* attrs, double* z) {
    if (!enc_dims_ok(KE, edims)) return -1;
    const int A = edims[0], C = edims[KE];
    const int MW = max_width(KE, edims);
    #pragma omp parallel
    {
        double* act[17];
        for (int k = 0; k <= KE; ++k) act[k] = (double*)malloc(sizeof(double) * MW);
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            enc_forward(KE, edims, eparams, attrs + (long)A * i, act);
            memcpy(z + (long)C * i, act[KE], sizeof(double) * C);
        }
        for (int k = 0; k <= KE; ++k) free(act[k]);
    }
    return 0;
}

/* z[n][C] = E(filtered parameters at (uv, lod)); p describes the parameter pyramid
 * (p->channels = A).  Non-finite uv or lod give NaN codes. */
int orc_encode_queries(const orc_pyramid* p, const double* const* levels, int KE, const int* edims,
                       const double* eparams, long n, const double* uv, const double* lod, double* z) {
    if (!enc_dims_ok(KE, edims) || edims[0] != p->channels) return -1;
    const int C = edims[KE];
    const int MW = max_width(KE, edims);
    #pragma omp parallel
    {
        double* act[17];
        for (int k = 0; k <= KE; ++k) act[k] = (double*)malloc(sizeof(double) * MW);
        double* a = (double*)malloc(sizeof(double) * MW);
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i]))) {
                for (int c = 0; c < C; ++c) z[(long)C * i + c] = NAN;
                continue;
            }
            fetch_one(p, levels, uv + 2 * i, lod + i, a);
            enc_forward(KE, edims, eparams, a, act);
            memcpy(z + (long)C * i, act[KE], sizeof(double) * C);
        }
        for (int k = 0; k <= KE; ++k) free(act[k]);
        free(a);
    }
    return 0;
}

/* The decoder's mean squared error on given latent codes z[n][C] (C = dims[0] - 6), the
 * first training phase's loss: as orc_loss_grad with the fetch replaced by z, so
 * L = 1/(3n) sum over the KO outputs of (out - target)^2.  Writes the loss, dparams and the
 * gradient of every sample's code dz[n][C].  A sample whose code has a non-finite component
 * (its query was not finite) is skipped: no loss term, dz = 0, n stays the denominator. */
int orc_loss_grad_codes(int K, const int* dims, const double* params, long n, const double* z,
                        const double* wi, const double* wo, const double* target,
                        double* loss, double* dparams, double* dz) {
    if (K < 1 || K > 16 || dims[0] < 7 || !out_width_ok(dims[K])) return -1;
    const int C = dims[0] - 6, KO = dims[K];
    const long np = mlp_param_count(K, dims);
    memset(dparams, 0, sizeof(double) * np);
    const int MW = max_width(K, dims);
    double total = 0.0;
    #pragma omp parallel reduction(+:total)
    {
        double* g = (double*)calloc(np, sizeof(double));
        double* act[17];
        for (int k = 0; k <= K; ++k) act[k] = (double*)malloc(sizeof(double) * (MW + 6));
        double* sa = (double*)malloc(sizeof(double) * MW);
        double* sb = (double*)malloc(sizeof(double) * MW);
        double* d = (double*)malloc(sizeof(double) * (MW + 6));
        double* dprev = (double*)malloc(sizeof(double) * (MW + 6));
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            int finite = 1;
            for (int c = 0; c < C; ++c) finite &= isfinite(z[(long)C * i + c]) ? 1 : 0;
            for (int c = 0; c < C; ++c) dz[(long)C * i + c] = 0.0;
            if (!finite) continue;
            double* x = act[0];
            for (int c = 0; c < C; ++c) x[c] = z[(long)C * i + c];
            for (int c = 0; c < 3; ++c) { x[C + c] = wi[3 * i + c]; x[C + 3 + c] = wo[3 * i + c]; }
            double y[6];
            mlp_eval(K, dims, params, x, y, act, sa, sb);
            for (int c = 0; c < KO; ++c) {
                const double e = y[c] - target[(long)KO * i + c];
                total += e * e;
                d[c] = 2.0 * e / (3.0 * (double)n) * logistic(act[K][c]);
            }
            long off[17]; long o = 0;
            for (int k = 1; k <= K; ++k) { off[k] = o; o += (long)dims[k - 1] * dims[k] + dims[k]; }
            for (int k = K; k >= 1; --k) {
                const int fi = dims[k - 1], fo = dims[k];
                const double* W = params + off[k];
                double* gW = g + off[k];
                double* gb = gW + (long)fi * fo;
                const double* a_in = act[k - 1];
                for (int r = 0; r < fo; ++r) {
                    gb[r] += d[r];
                    for (int j = 0; j < fi; ++j) gW[(long)r * fi + j] += d[r] * a_in[j];
                }
                for (int j = 0; j < fi; ++j) {
                    double s = 0.0;
                    for (int r = 0; r < fo; ++r) s += W[(long)r * fi + j] * d[r];
                    if (k > 1) s = (a_in[j] > 0.0) ? s : 0.0;
                    dprev[j] = s;
                }
                memcpy(d, dprev, sizeof(double) * fi);
            }
            for (int c = 0; c < C; ++c) dz[(long)C * i + c] = d[c];
        }
        #pragma omp critical
        for (long j = 0; j < np; ++j) dparams[j] += g[j];
        for (int k = 0; k <= K; ++k) free(act[k]);
        free(g); free(sa); free(sb); free(d); free(dprev);
    }
    *loss = total / (3.0 * (double)n);
    return 0;
}

/* Gradient of sum_i dz[i] . E(filtered parameters at query i) with respect to the encoder's
 * parameters (the encoder's share of the first training phase, with dz from
 * orc_loss_grad_codes): d_eparams is overwritten.  Non-finite queries contribute nothing. */
int orc_encoder_backward(const orc_pyramid* p, const double* const* levels, int KE, const int* edims,
                         const double* eparams, long n, const double* uv, const double* lod, const double* dz,
                         double* d_eparams) {
    if (!enc_dims_ok(KE, edims) || edims[0] != p->channels) return -1;
    const int C = edims[KE];
    const long np = mlp_param_count(KE, edims);
    memset(d_eparams, 0, sizeof(double) * np);
    const int MW = max_width(KE, edims);
    #pragma omp parallel
    {
        double* g = (double*)calloc(np, sizeof(double));
        double* act[17];
        for (int k = 0; k <= KE; ++k) act[k] = (double*)malloc(sizeof(double) * MW);
        double* a = (double*)malloc(sizeof(double) * MW);
        double* d = (double*)malloc(sizeof(double) * MW);
        double* dprev = (double*)malloc(sizeof(double) * MW);
        long off[17]; long o = 0;
        for (int k = 1; k <= KE; ++k) { off[k] = o; o += (long)edims[k - 1] * edims[k] + edims[k]; }
        #pragma omp for schedule(static)
        for (long i = 0; i < n; ++i) {
            if (!(isfinite(uv[2 * i]) && isfinite(uv[2 * i + 1]) && isfinite(lod[i]))) continue;
            fetch_one(p, levels, uv + 2 * i, lod + i, a);
            enc_forward(KE, edims, eparams, a, act);
            for (int c = 0; c < C; ++c) d[c] = dz[(long)C * i + c];       /* the output layer is linear */
            for (int k = KE; k >= 1; --k) {
                const int fi = edims[k - 1], fo = edims[k];
                const double* W = eparams + off[k];
                double* gW = g + off[k];
                double* gb = gW + (long)fi * fo;
                const double* a_in = act[k - 1];
                for (int r = 0; r < fo; ++r) {
                    gb[r] += d[r];
                    for (int j = 0; j < fi; ++j) gW[(long)r * fi + j] += d[r] * a_in[j];
                }
                if (k == 1) break;
                for (int j = 0; j < fi; ++j) {
                    double s = 0.0;
                    for (int r = 0; r < fo; ++r) s += W[(long)r * fi + j] * d[r];
                    dprev[j] = (a_in[j] > 0.0) ? s : 0.0;
                }
                memcpy(d, dprev, sizeof(double) * fi);
            }
        }
        #pragma omp critical
        for (long j = 0; j < np; ++j) d_eparams[j] += g[j];
        for (int k = 0; k <= KE; ++k) free(act[k]);
        free(g); free(a); free(d); free(dprev);
    }
    return 0;
}
