"""Seeded synthetic workloads for the neural appearance decode path.

This module only draws inputs: latent pyramids, decoder weights, shading queries,
training targets and serving request streams.  It holds none of the decode
arithmetic (no texel addressing, no interpolation, no network evaluation), so the
FP64 oracle and the HIP library can both consume its arrays without sharing any
method code.

Conventions (the paper leaves them open):
  * RNG: ``numpy.random.Generator(PCG64(SeedSequence(seed)))``; five children are
    spawned in the fixed order [latents, weights, queries, targets, requests].
  * Texels: level 0 i.i.d. N(0, 1) drawn in row-major (y, x, channel) order; the
    coarser levels are 2x2 box averages computed in float64 and rounded once to
    float32 (the latent pyramid of the paper's Sec. 4.1 "Latent texture").
    Level sizes are max(1, W >> l) by max(1, H >> l).
  * Decoder weights: Xavier-uniform U(-a, a), a = sqrt(6 / (fan_in + fan_out)),
    drawn layer by layer in row-major [out][in] order; biases zero.  Packed as
    W1, b1, W2, b2, ... (the network of Eq. neural-brdf).
  * Directions: cosine-weighted upper hemisphere by Malley's method, in the
    shading frame (z up), unit length.
  * Learned shading frames (optional, drawn after the decoder weights): W_F[6N][C]
    Xavier-uniform scaled by 1/4, biases placing every normal at +z and every tangent
    at +x, so the frames are perturbations of the geometric frame that the latent code
    steers (a stand-in for a trained, normal-mapped frame layer; no frame is near zero
    length).
Every float array handed out is float32 (the stored type); the oracle reads those
exact values promoted to float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

CHILD_LATENTS, CHILD_WEIGHTS, CHILD_QUERIES, CHILD_TARGETS, CHILD_REQUESTS = range(5)

WRAP, CLAMP = 0, 1


def rngs(seed: int) -> List[np.random.Generator]:
    """The five child generators of one workload seed, in the fixed order."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(5)]


def level_dims(width: int, height: int, levels: int):
    return [(max(1, height >> l), max(1, width >> l)) for l in range(levels)]


def full_chain(width: int, height: int) -> int:
    return int(math.log2(max(width, height))) + 1


def box_pyramid(level0: np.ndarray, levels: int, work_dtype=np.float64) -> List[np.ndarray]:
    """2x2 box-filtered chain, computed in work_dtype (float64 unless a large serving texture
    asks for float32) and rounded to float32 at the end.

    level0 is [H][W][C].  Along an axis already at size 1 the filter averages only along the
    other axis.
    """
    out = [np.asarray(level0, dtype=work_dtype)]
    for _ in range(1, levels):
        p = out[-1]
        h, w, c = p.shape
        if h > 1:
            p = 0.5 * (p[0::2] + p[1::2])
        if w > 1:
            p = 0.5 * (p[:, 0::2] + p[:, 1::2])
        out.append(p)
    return [np.ascontiguousarray(x, dtype=np.float32) for x in out]


def gaussian_pyramid_level0(rng, width, height, channels, dtype=np.float64):
    return rng.standard_normal((height, width, channels), dtype=dtype)


def xavier_mlp(rng, dims: Sequence[int]) -> np.ndarray:
    """Packed float32 parameters W1[out][in], b1[out], W2, b2, ... ; biases zero."""
    chunks = []
    for k in range(len(dims) - 1):
        fi, fo = dims[k], dims[k + 1]
        a = math.sqrt(6.0 / (fi + fo))
        chunks.append(rng.uniform(-a, a, size=(fo, fi)).reshape(-1))
        chunks.append(np.zeros(fo))
    return np.concatenate(chunks).astype(np.float32)


def n_params(dims: Sequence[int]) -> int:
    return sum(dims[k] * dims[k + 1] + dims[k + 1] for k in range(len(dims) - 1))


def unpack_params(params: np.ndarray, dims: Sequence[int]):
    """Views [(W_k [out][in], b_k [out]), ...] into a packed parameter vector."""
    out, o = [], 0
    for k in range(len(dims) - 1):
        fi, fo = dims[k], dims[k + 1]
        W = params[o:o + fi * fo].reshape(fo, fi)
        o += fi * fo
        b = params[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def cosine_hemisphere(rng, n: int) -> np.ndarray:
    """Malley's method: r = sqrt(xi1), phi = 2 pi xi2, (r cos phi, r sin phi, sqrt(1 - xi1))."""
    xi = rng.random((n, 2))
    r = np.sqrt(xi[:, 0])
    phi = 2.0 * np.pi * xi[:, 1]
    w = np.stack([r * np.cos(phi), r * np.sin(phi), np.sqrt(1.0 - xi[:, 0])], axis=1)
    return w.astype(np.float32)


@dataclasses.dataclass
class Material:
    width: int
    height: int
    channels: int
    levels: List[np.ndarray]          # [H_l][W_l][C] float32 each
    dims: List[int]                   # decoder widths, dims[0] = C + 6 max(1, n_frames), dims[-1] = 3 or 6 (albedo)
    params: np.ndarray                # packed float32
    address: int = WRAP
    n_frames: int = 0                 # learned shading frames (0: none)
    frame_params: Optional[np.ndarray] = None   # W_F[6N][C] then b_F[6N], float32

    @property
    def n_levels(self) -> int:
        return len(self.levels)

    def texel_count(self) -> int:
        return sum(l.shape[0] * l.shape[1] for l in self.levels)


@dataclasses.dataclass
class Queries:
    uv: np.ndarray    # [N][2] float32
    lod: np.ndarray   # [N] float32
    wi: np.ndarray    # [N][3] float32
    wo: np.ndarray    # [N][3] float32

    def __len__(self):
        return self.lod.shape[0]

    def subset(self, idx) -> "Queries":
        return Queries(self.uv[idx], self.lod[idx], self.wi[idx], self.wo[idx])


def frame_layer(rng, n_frames: int, channels: int) -> np.ndarray:
    """W_F[6N][C] (Xavier-uniform / 4) then b_F[6N] (every normal +z, every tangent +x)."""
    a = math.sqrt(6.0 / (channels + 6 * n_frames))
    W = 0.25 * rng.uniform(-a, a, size=(6 * n_frames, channels))
    b = np.tile([0.0, 0.0, 1.0, 1.0, 0.0, 0.0], n_frames)
    return np.concatenate([W.reshape(-1), b]).astype(np.float32)


def decoder_for(rng_w, channels: int, hidden, n_frames: int = 0, albedo: bool = False):
    """(dims, packed decoder parameters, frame layer or None), drawn in that order.  With
    albedo the decoder has 6 outputs: RGB reflectance, then the directional-albedo triplet."""
    dims = [channels + 6 * max(1, n_frames)] + list(hidden) + [6 if albedo else 3]
    params = xavier_mlp(rng_w, dims)
    frames = frame_layer(rng_w, n_frames, channels) if n_frames else None
    return dims, params, frames


def sampler_decoder(rng, channels: int, hidden=(32, 32, 32)):
    """(sdims, packed parameters) of an importance-sampling decoder on [z, wi] with 9 outputs
    (the paper's sampler is 3 x 32): Xavier-uniform weights, zero biases."""
    sdims = [channels + 3] + list(hidden) + [9]
    return sdims, xavier_mlp(rng, sdims)


def make_material(rng_lat, rng_w, width, height, channels, levels, hidden, address=WRAP, dtype=np.float64,
                  n_frames: int = 0, albedo: bool = False):
    lv0 = gaussian_pyramid_level0(rng_lat, width, height, channels, dtype)
    pyr = box_pyramid(lv0, levels, dtype)
    dims, params, frames = decoder_for(rng_w, channels, hidden, n_frames, albedo)
    return Material(width, height, channels, pyr, dims, params, address, n_frames, frames)


def uniform_queries(rng, n, lod_lo, lod_hi) -> Queries:
    uv = rng.random((n, 2)).astype(np.float32)
    lod = rng.uniform(lod_lo, lod_hi, size=n).astype(np.float32)
    wi = cosine_hemisphere(rng, n)
    wo = cosine_hemisphere(rng, n)
    return Queries(uv, lod, wi, wo)


# ----------------------------------------------------------------------------------------
# Frame-scale screen-space queries (a stand-in for the paper's rendered views: per pixel a
# uv from a smooth screen-to-uv map and a mip level from the footprint area, Sec. 4.1).


@dataclasses.dataclass
class ScreenMap:
    theta: float
    shear: float
    kx: float
    ky: float
    c: np.ndarray            # [2]
    f: np.ndarray            # [2] integer warp frequencies
    phi: np.ndarray          # [2] warp phases
    tex_w: int
    tex_h: int
    screen_w: int
    screen_h: int
    warp_amp: float = 0.02

    def matrix(self) -> np.ndarray:
        ct, st = math.cos(self.theta), math.sin(self.theta)
        R = np.array([[ct, -st], [st, ct]])
        D = np.diag([self.kx / self.tex_w, self.ky / self.tex_h])
        S = np.array([[1.0, self.shear], [0.0, 1.0]])
        return R @ D @ S

    def uv_and_lod(self, px: np.ndarray, py: np.ndarray):
        """uv and footprint level for pixel centres (px + 1/2, py + 1/2).

        lod = 1/2 log2(|det J| W H), J = d(u, v)/d(pixel x, pixel y) in closed form.
        """
        A = self.matrix()
        x = px.astype(np.float64) + 0.5
        y = py.astype(np.float64) + 0.5
        au = 2 * np.pi * self.f[0] / self.screen_w
        av = 2 * np.pi * self.f[1] / self.screen_h
        u = A[0, 0] * x + A[0, 1] * y + self.c[0] + self.warp_amp * np.sin(au * x + self.phi[0])
        v = A[1, 0] * x + A[1, 1] * y + self.c[1] + self.warp_amp * np.sin(av * y + self.phi[1])
        j00 = A[0, 0] + self.warp_amp * au * np.cos(au * x + self.phi[0])
        j11 = A[1, 1] + self.warp_amp * av * np.cos(av * y + self.phi[1])
        det = j00 * j11 - A[0, 1] * A[1, 0]
        area = np.maximum(np.abs(det) * self.tex_w * self.tex_h, 1e-30)
        lod = 0.5 * np.log2(area)
        return np.stack([u, v], axis=1), lod


def random_screen_map(rng, tex_w, tex_h, screen_w, screen_h, k_lo=0.7, k_hi=12.0) -> ScreenMap:
    theta = rng.uniform(0.0, 2 * np.pi)
    shear = rng.uniform(-0.2, 0.2)
    kx = math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))
    ky = math.exp(rng.uniform(math.log(k_lo), math.log(k_hi)))
    c = rng.random(2)
    f = rng.integers(1, 4, size=2)
    phi = rng.uniform(0.0, 2 * np.pi, size=2)
    return ScreenMap(theta, shear, kx, ky, c, f.astype(np.float64), phi, tex_w, tex_h, screen_w, screen_h)


def tile_order(screen_w: int, screen_h: int, tile: int = 16):
    """Pixel coordinates in 16x16 screen-tile order (tile rows, tile columns, then rows within a
    tile); tiles on the right and bottom edges are ragged."""
    ty, tx, iy, ix = np.meshgrid(np.arange((screen_h + tile - 1) // tile),
                                 np.arange((screen_w + tile - 1) // tile),
                                 np.arange(tile), np.arange(tile), indexing="ij")
    px = (tx * tile + ix).reshape(-1)
    py = (ty * tile + iy).reshape(-1)
    keep = (px < screen_w) & (py < screen_h)
    return px[keep], py[keep]


def screen_queries(rng, smap: ScreenMap, n: Optional[int] = None) -> Queries:
    px, py = tile_order(smap.screen_w, smap.screen_h)
    if n is not None:
        px, py = px[:n], py[:n]
    uv, lod = smap.uv_and_lod(px, py)
    m = len(px)
    return Queries(uv.astype(np.float32), lod.astype(np.float32),
                   cosine_hemisphere(rng, m), cosine_hemisphere(rng, m))


# ----------------------------------------------------------------------------------------
# Analytic training targets: Lambert + GGX microfacet reflectance with spatially varying,
# uv-periodic albedo and roughness (stands in for the paper's layered reference materials).


@dataclasses.dataclass
class NoiseField:
    amp: np.ndarray     # [K][4]
    fu: np.ndarray      # [K][4] integer
    fv: np.ndarray      # [K][4] integer
    phase: np.ndarray   # [K][4]

    def __call__(self, uv: np.ndarray) -> np.ndarray:
        u = uv[:, 0:1, None].astype(np.float64)
        v = uv[:, 1:2, None].astype(np.float64)
        s = self.amp[None] * np.sin(2 * np.pi * (self.fu[None] * u + self.fv[None] * v) + self.phase[None])
        return s.sum(axis=2)   # [N][K]


def make_noise(rng, k: int) -> NoiseField:
    return NoiseField(rng.uniform(0.5, 1.5, size=(k, 4)),
                      rng.integers(1, 5, size=(k, 4)).astype(np.float64),
                      rng.integers(1, 5, size=(k, 4)).astype(np.float64),
                      rng.uniform(0, 2 * np.pi, size=(k, 4)))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


@dataclasses.dataclass
class AnalyticMaterial:
    albedo_noise: NoiseField      # 3 channels
    rough_noise: NoiseField       # 1 channel
    f0: float = 0.04

    def albedo(self, uv):
        return 0.05 + 0.9 * _sigmoid(self.albedo_noise(uv))

    def roughness(self, uv):
        return 0.3 + 0.6 * _sigmoid(self.rough_noise(uv))[:, 0]

    def brdf(self, uv, wi, wo) -> np.ndarray:
        """f = rho / pi + F D G / (4 cos_i cos_o) in float64; GGX D with alpha = r^2,
        separable Smith G, Schlick F with achromatic F0."""
        wi = wi.astype(np.float64)
        wo = wo.astype(np.float64)
        rho = self.albedo(uv)
        a = self.roughness(uv) ** 2
        a2 = a * a
        h = wi + wo
        h /= np.linalg.norm(h, axis=1, keepdims=True)
        ci, co, ch = wi[:, 2], wo[:, 2], h[:, 2]
        D = a2 / (np.pi * (ch * ch * (a2 - 1.0) + 1.0) ** 2)

        def g1(c):
            return 2.0 * c / (c + np.sqrt(a2 + (1.0 - a2) * c * c))

        G = g1(ci) * g1(co)
        F = self.f0 + (1.0 - self.f0) * (1.0 - np.clip(np.sum(wi * h, axis=1), 0.0, 1.0)) ** 5
        spec = F * D * G / (4.0 * ci * co)
        return rho / np.pi + spec[:, None]

    def visible_normals(self, rng, uv, wo) -> np.ndarray:
        """Microfacet normals h drawn from the GGX distribution of normals visible from wo,
        G1(wo) max(0, wo.h) D(h) / cos(theta_o) (Heitz 2018, "Sampling the GGX distribution of
        visible normals"): stretch wo by alpha, sample the projected disk of the unit
        hemisphere seen from it, unstretch.  [len(uv)][3] float64, h_z >= 0."""
        a = self.roughness(uv) ** 2
        wo = wo.astype(np.float64)
        v = np.stack([a * wo[:, 0], a * wo[:, 1], wo[:, 2]], 1)
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        lensq = v[:, 0] ** 2 + v[:, 1] ** 2
        safe = lensq > 0
        inv = np.where(safe, 1.0 / np.sqrt(np.where(safe, lensq, 1.0)), 0.0)
        t1 = np.stack([np.where(safe, -v[:, 1] * inv, 1.0), np.where(safe, v[:, 0] * inv, 0.0),
                       np.zeros(len(v))], 1)
        t2 = np.cross(v, t1)
        xi = rng.random((len(uv), 2))
        r = np.sqrt(xi[:, 0])
        phi = 2.0 * np.pi * xi[:, 1]
        p1, p2 = r * np.cos(phi), r * np.sin(phi)
        s = 0.5 * (1.0 + v[:, 2])
        p2 = (1.0 - s) * np.sqrt(np.maximum(0.0, 1.0 - p1 * p1)) + s * p2
        p3 = np.sqrt(np.maximum(0.0, 1.0 - p1 * p1 - p2 * p2))
        nh = p1[:, None] * t1 + p2[:, None] * t2 + p3[:, None] * v
        h = np.stack([a * nh[:, 0], a * nh[:, 1], np.maximum(0.0, nh[:, 2])], 1)
        return h / np.linalg.norm(h, axis=1, keepdims=True)

    def albedo_estimates(self, rng, uv, wo) -> np.ndarray:
        """One-sample estimates of the directional albedo (Eq. albedo) at (uv, wo), one sample
        per lobe, each drawn from that lobe's own density, as a material's sampling routine
        would: the Lambertian lobe sampled by the cosine density weighs rho exactly, whatever
        the draw; the GGX lobe sampled through its visible normals (wi the reflection of wo
        about h) weighs f_spec cos(theta_i) / pdf(wi) = F(wo.h) G1(wi), or 0 below the
        horizon.  Unbiased, and bounded by rho + 1.  The draws are independent of any wi the
        decoder sees, so an L2 fit converges to the albedo itself.  [len(uv)][3] float64."""
        rho = self.albedo(uv)
        a2 = self.roughness(uv) ** 4
        wo = wo.astype(np.float64)
        h = self.visible_normals(rng, uv, wo)
        oh = np.sum(wo * h, axis=1)
        wi = 2.0 * oh[:, None] * h - wo
        ci = wi[:, 2]
        g1 = np.where(ci > 0, 2.0 * ci / (ci + np.sqrt(a2 + (1.0 - a2) * ci * ci)), 0.0)
        F = self.f0 + (1.0 - self.f0) * (1.0 - np.clip(oh, 0.0, 1.0)) ** 5
        return rho + (F * g1)[:, None]

    def directional_albedo(self, uv, wo, grid: int = 256) -> np.ndarray:
        """Eq. albedo by quadrature: under the cosine-hemisphere map of the unit square the
        integral of f cos(theta_i) over the hemisphere is pi times the mean of f over the
        square, taken here at the grid x grid cell midpoints.  [len(uv)][3] float64."""
        k = (np.arange(grid) + 0.5) / grid
        u1, u2 = np.meshgrid(k, k, indexing="ij")
        r = np.sqrt(u1.reshape(-1))
        phi = 2.0 * np.pi * u2.reshape(-1)
        wi = np.stack([r * np.cos(phi), r * np.sin(phi), np.sqrt(1.0 - u1.reshape(-1))], 1)
        out = np.empty((len(uv), 3))
        for i in range(len(uv)):
            m = wi.shape[0]
            f = self.brdf(np.repeat(uv[i:i + 1], m, 0), wi, np.repeat(wo[i:i + 1].astype(np.float64), m, 0))
            out[i] = np.pi * f.mean(0)
        return out


def material_parameters(am: "AnalyticMaterial", tex: int, levels: int) -> List[np.ndarray]:
    """The parameters of the analytic material as a texture pyramid, the encoder's input
    (Sec. 5.1): level 0 holds [albedo r, g, b, roughness] at the texel centres of a tex x tex
    grid, the coarser levels its 2x2 box averages (the material has no normal map, so the
    prefiltering needs nothing beyond the average).  [levels] arrays of [H][W][4] float32."""
    x = (np.arange(tex) + 0.5) / tex
    U, V = np.meshgrid(x, x, indexing="xy")
    uv = np.stack([U.ravel(), V.ravel()], 1)
    level0 = np.concatenate([am.albedo(uv), am.roughness(uv)[:, None]], 1).reshape(tex, tex, 4)
    return box_pyramid(level0, levels)


def encoder_params(rng, attributes: int, channels: int, hidden=(32, 32)):
    """(dims, packed parameters) of an encoder from the material's parameters to the latent
    code: Xavier-uniform weights, zero biases."""
    dims = [attributes] + list(hidden) + [channels]
    return dims, xavier_mlp(rng, dims)


def make_analytic_material(rng) -> AnalyticMaterial:
    return AnalyticMaterial(make_noise(rng, 3), make_noise(rng, 1))


def truncated_exponential(rng, n, mean, hi) -> np.ndarray:
    """Exp(mean) restricted to [0, hi] by inverting its CDF."""
    xi = rng.random(n)
    return -mean * np.log1p(-xi * (1.0 - math.exp(-hi / mean)))


# ----------------------------------------------------------------------------------------
# The five workloads.


@dataclasses.dataclass
class Workload:
    name: str
    material: Material
    queries: Queries
    targets: Optional[np.ndarray] = None        # [N][3] float32 (training)
    analytic: Optional[AnalyticMaterial] = None
    screen: Optional[ScreenMap] = None


def tiny(seed: int = 1001, n: int = 4096) -> Workload:
    """One 64x64 x 8-channel float32 material with 3 box levels, 4096 random queries with
    lod in [0, 2], decoder 14 -> 32 -> 32 -> 3."""
    r = rngs(seed)
    mat = make_material(r[CHILD_LATENTS], r[CHILD_WEIGHTS], 64, 64, 8, 3, [32, 32])
    q = uniform_queries(r[CHILD_QUERIES], n, 0.0, 2.0)
    return Workload("tiny 64x64x8, 3 levels, 4096 queries, MLP 14-32-32-3", mat, q)


FRAME_W, FRAME_H = 1920, 1080


def frame(seed: int = 1002, tex: int = 2048, channels: int = 16, screen=(FRAME_W, FRAME_H),
          hidden=(64, 64, 64), n: Optional[int] = None, n_frames: int = 0, albedo: bool = False) -> Workload:
    """Frame-scale decode: a tex x tex x C float32 material with the full mip chain, one query
    per pixel of a 1920x1080 frame in 16x16 screen-tile order, decoder 22 -> 64 -> 64 -> 64 -> 3
    (28 -> ... with two learned shading frames; ... -> 6 with the albedo head)."""
    r = rngs(seed)
    mat = make_material(r[CHILD_LATENTS], r[CHILD_WEIGHTS], tex, tex, channels, full_chain(tex, tex), hidden,
                        n_frames=n_frames, albedo=albedo)
    smap = random_screen_map(r[CHILD_QUERIES], tex, tex, screen[0], screen[1])
    q = screen_queries(r[CHILD_QUERIES], smap, n)
    fr = f", {n_frames} learned shading frames" if n_frames else ""
    return Workload(f"frame {screen[0]}x{screen[1]}, latent {tex}^2 x {channels}, full chain, "
                    f"MLP {'-'.join(str(d) for d in mat.dims)}{fr}", mat, q, screen=smap)


def training(seed: int = 1004, tex: int = 1024, channels: int = 16, n: int = 1 << 20,
             hidden=(64, 64, 64), levels: Optional[int] = None, albedo: bool = False) -> Workload:
    """Training batch: uv uniform, lod ~ Exp(mean 1) truncated to [0, M-1], cosine
    directions, targets from the analytic Lambert + GGX material.  With albedo the decoder
    has 6 outputs and each target row is [f(x, wi, wo), one-sample estimate of the albedo at
    (x, wo)] (the estimates drawn after everything else, from the targets' stream)."""
    r = rngs(seed)
    M = levels if levels is not None else full_chain(tex, tex)
    mat = make_material(r[CHILD_LATENTS], r[CHILD_WEIGHTS], tex, tex, channels, M, hidden, albedo=albedo)
    rq = r[CHILD_QUERIES]
    uv = rq.random((n, 2)).astype(np.float32)
    lod = truncated_exponential(rq, n, 1.0, M - 1).astype(np.float32)
    q = Queries(uv, lod, cosine_hemisphere(rq, n), cosine_hemisphere(rq, n))
    am = make_analytic_material(r[CHILD_TARGETS])
    tgt = am.brdf(q.uv, q.wi, q.wo)
    if albedo:
        tgt = np.concatenate([tgt, am.albedo_estimates(r[CHILD_TARGETS], q.uv, q.wo)], 1)
    return Workload(f"train {n} samples, latent {tex}^2 x {channels}, {M} levels, "
                    f"MLP {'-'.join(str(d) for d in mat.dims)}", mat, q, tgt.astype(np.float32), am)


def training_samples(am: AnalyticMaterial, rng, n: int, n_levels: int, albedo: bool = False):
    """A fresh batch from the same analytic material (held-out sets, later steps); with
    albedo the targets carry the one-sample albedo estimates as columns 3-5."""
    uv = rng.random((n, 2)).astype(np.float32)
    lod = truncated_exponential(rng, n, 1.0, n_levels - 1).astype(np.float32)
    q = Queries(uv, lod, cosine_hemisphere(rng, n), cosine_hemisphere(rng, n))
    tgt = am.brdf(q.uv, q.wi, q.wo)
    if albedo:
        tgt = np.concatenate([tgt, am.albedo_estimates(rng, q.uv, q.wo)], 1)
    return q, tgt.astype(np.float32)


@dataclasses.dataclass
class Request:
    arrival_s: float
    material: int
    queries: Queries


def serving_materials(seed: int = 1005, count: int = 8, sides=(512, 1024, 2048, 4096),
                      channels=(8, 16), hidden=(64, 64, 64)) -> List[Material]:
    """Resident materials: side 2^k with k uniform over the given powers of two, C uniform over
    {8, 16}, full chains, independent seeds.  Texels are drawn and box-filtered in float32 (up
    to 4096^2 x 16 per material; no parity test reads them in float64)."""
    r = rngs(seed)
    mats = []
    for i in range(count):
        side = int(r[CHILD_LATENTS].choice(sides))
        ch = int(r[CHILD_LATENTS].choice(channels))
        sub = rngs(seed * 1000 + i)
        mats.append(make_material(sub[CHILD_LATENTS], sub[CHILD_WEIGHTS], side, side, ch,
                                  full_chain(side, side), hidden, dtype=np.float32))
    return mats


def request_sizes(rng, count, lo=4096, hi=8294400) -> np.ndarray:
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=count)).astype(np.int64)


def request_stream(seed: int, materials: Sequence[Material], count: int, rate_per_s: float,
                   lo=4096, hi=8294400, max_queries: Optional[int] = None) -> List[Request]:
    """Poisson arrivals at rate_per_s; each request names one material and carries a screen
    tile of the frame generator (16:9 aspect, up to 3840x2160) of log-uniform size."""
    r = rngs(seed)[CHILD_REQUESTS]
    sizes = request_sizes(r, count, lo, hi)
    if max_queries is not None:
        sizes = np.minimum(sizes, max_queries)
    gaps = r.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        m = int(r.integers(0, len(materials)))
        mat = materials[m]
        n = int(sizes[i])
        sw = int(math.ceil(math.sqrt(n * 16.0 / 9.0)))
        sh = int(math.ceil(n / sw))
        smap = random_screen_map(r, mat.width, mat.height, sw, sh)
        out.append(Request(float(t[i]), m, screen_queries(r, smap, n)))
    return out
