"""Pins of the oracle's importance-sampling proxy (Sec. 4.3; App. A, Eq. pdf_full, Eq. pdf_spec)
and of its sampling decoder, against closed forms, an independent slope-space derivation of
the anisotropic, non-centred GGX density, numerical integration over the sphere and the
histogram of the oracle's own samples.

Targets: a wrong Jacobian (determinant or cube), M used where M^-1 belongs or transposed, the
half vector not folded to the upper hemisphere, a wrong reflection, the lobe choice inverted,
the diffuse lobe not tilted by n_d, the activations or the output order wrong.
"""
import numpy as np
import pytest

import oracle
from paper_2305_02678_amd import workloads as wl


def _params(w_d, mu_d, alpha, rho, mu_s):
    return np.array([w_d, mu_d[0], mu_d[1], 1.0 - w_d, alpha[0], alpha[1], rho, mu_s[0], mu_s[1]])


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _sphere_grid(nz, nphi):
    z = -1.0 + (np.arange(nz) + 0.5) * 2.0 / nz
    phi = (np.arange(nphi) + 0.5) * 2.0 * np.pi / nphi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    r = np.sqrt(1.0 - Z ** 2)
    w = np.stack([r * np.cos(P), r * np.sin(P), Z], -1).reshape(-1, 3)
    return w, (2.0 / nz) * (2.0 * np.pi / nphi)


SETS = [
    ((0.3, -0.2), (0.5, 0.8), 0.0, (0.0, 0.0)),
    ((-0.4, 0.1), (0.3, 0.6), 0.5, (0.2, -0.3)),
    ((0.0, 0.0), (0.9, 0.25), -0.7, (-0.5, 0.4)),
]


def test_activations_closed_form():
    raw = np.array([0.3, 1.0, -1.0, -0.2, 0.0, 3.0, 1.0, 2.0, -0.5])
    p = oracle.proxy_activate(raw)[0]
    e = np.exp(0.5)
    expect = [e / (1 + e), 1.5, -1.5, 1 / (1 + e), 1e-3 + 0.999 * 0.5, 1.0, 0.999 * 0.75, 4.0, -0.625]
    np.testing.assert_allclose(p, expect, rtol=1e-15, atol=1e-16)
    r = np.random.default_rng(1).normal(0, 4, (2000, 9))
    P = oracle.proxy_activate(r)
    assert np.allclose(P[:, 0] + P[:, 3], 1.0) and (P[:, [0, 3]] > 0).all()
    assert (P[:, 4:6] >= 1e-3).all() and (P[:, 4:6] <= 1.0).all() and (np.abs(P[:, 6]) <= 0.999).all()
    assert np.all(np.diff(oracle.proxy_activate(np.outer(np.linspace(-5, 5, 101), np.ones(9)))[:, [1, 4, 6]], axis=0) >= 0)


@pytest.mark.parametrize("mu_d,alpha,rho,mu_s", SETS)
def test_pdf_integrates_to_one_over_the_sphere(mu_d, alpha, rho, mu_s):
    """Midpoint rule over (cos theta, phi); each lobe alone and the mixture."""
    wo, dA = _sphere_grid(1200, 2400)
    wi = np.tile(_unit(np.array([0.3, -0.4, 0.8])), (len(wo), 1))
    for w_d in (1.0, 0.0, 0.35):
        P = np.tile(_params(w_d, mu_d, alpha, rho, mu_s), (len(wo), 1))
        total = oracle.proxy_pdf(P, wi, wo).sum() * dA
        assert abs(total - 1.0) < 2e-3, (w_d, total)


@pytest.mark.parametrize("mu_d,alpha,rho,mu_s", SETS)
def test_specular_lobe_is_the_slope_space_ggx(mu_d, alpha, rho, mu_s):
    """With w_s = 1 the density of wo times 4 |wo . h| is the density of h; in slope space the
    sampled slopes are A s_std - mu_s with s_std ~ 1 / (pi (1 + |s|^2)^2) and
    A = [[ax, 0], [ay rho, ay sqrt(1 - rho^2)]], so p(h) = P_std(A^-1 (slope(h) + mu_s)) / (det A h_z^3)."""
    rng = np.random.default_rng(7)
    n = 4000
    wi = _unit(rng.normal(size=(n, 3)) + [0, 0, 1.5])
    wo = _unit(rng.normal(size=(n, 3)))
    h = _unit(wi + wo)
    h = h * np.sign(h[:, 2:3])
    P = np.tile(_params(0.0, mu_d, alpha, rho, mu_s), (n, 1))
    got = oracle.proxy_pdf(P, wi, wo) * 4.0 * np.abs(np.sum(wo * h, 1))
    A = np.array([[alpha[0], 0.0], [alpha[1] * rho, alpha[1] * np.sqrt(1 - rho ** 2)]])
    slope = h[:, :2] / h[:, 2:3]
    s_std = np.linalg.solve(A, (slope + np.array(mu_s)).T).T
    ref = 1.0 / (np.pi * (1.0 + np.sum(s_std ** 2, 1)) ** 2) / (np.linalg.det(A) * h[:, 2] ** 3)
    np.testing.assert_allclose(got, ref, rtol=1e-10)


def test_diffuse_samples_are_cosine_about_the_tilted_normal():
    """w_d = 1: the cosine to n_d = normalise(-mu_d, 1) of the samples has a uniform square (the
    cosine-weighted hemisphere), for a tilted and an untilted normal."""
    n = 100000
    u = (np.stack(np.meshgrid(np.arange(1), np.arange(n), indexing="ij"), -1).reshape(-1, 2)[:, 1:] + 0.5) / n
    rng = np.random.default_rng(3)
    for mu in ((0.0, 0.0), (0.6, -0.3)):
        U = np.concatenate([np.zeros((n, 1)), u, rng.random((n, 1))], 1)
        P = np.tile(_params(1.0, mu, (0.5, 0.5), 0.0, (0, 0)), (n, 1))
        wo, pdf = oracle.proxy_sample(P, np.tile([0, 0, 1.0], (n, 1)), U)
        nd = _unit(np.array([-mu[0], -mu[1], 1.0]))
        c = wo @ nd
        np.testing.assert_allclose(np.sort(c ** 2), (np.arange(n) + 0.5) / n, atol=2e-5)
        np.testing.assert_allclose(pdf, c / np.pi, rtol=1e-12)


@pytest.mark.parametrize("mu_d,alpha,rho,mu_s", SETS)
def test_samples_follow_the_pdf(mu_d, alpha, rho, mu_s):
    """Histogram of 400,000 stratified samples over 8 x 16 (cos theta, phi) bins against the
    PDF integrated per bin; the returned pdf is the PDF of the returned direction."""
    rng = np.random.default_rng(11)
    n = 400000
    k = np.arange(n)
    U = np.stack([(k + rng.random(n)) / n, rng.random(n), rng.random(n)], 1)
    wi = np.tile(_unit(np.array([-0.5, 0.2, 0.7])), (n, 1))
    P = np.tile(_params(0.4, mu_d, alpha, rho, mu_s), (n, 1))
    wo, pdf = oracle.proxy_sample(P, wi, U)
    np.testing.assert_allclose(np.linalg.norm(wo, axis=1), 1.0, rtol=1e-12)
    np.testing.assert_allclose(pdf, oracle.proxy_pdf(P, wi, wo), rtol=1e-12)
    nz, nphi = 8, 16
    bz = np.minimum(((wo[:, 2] + 1.0) / 2.0 * nz).astype(int), nz - 1)
    bp = np.minimum((np.mod(np.arctan2(wo[:, 1], wo[:, 0]), 2 * np.pi) / (2 * np.pi) * nphi).astype(int), nphi - 1)
    hist = np.bincount(bz * nphi + bp, minlength=nz * nphi) / n
    g, dA = _sphere_grid(nz * 150, nphi * 150)
    Pg = np.tile(P[0], (len(g), 1))
    dens = oracle.proxy_pdf(Pg, np.tile(wi[0], (len(g), 1)), g).reshape(nz, 150, nphi, 150).sum((1, 3)) * dA
    expect = dens.reshape(-1)
    big = expect > 0.01
    assert abs(expect.sum() - 1.0) < 3e-3
    np.testing.assert_allclose(hist[big], expect[big], rtol=0.05)
    assert np.abs(hist - expect).max() < 4e-3


def test_sampler_decoder_closed_forms():
    """Zero weights: every query gets activate(b_K).  A decoder that passes z_0..z_8 through
    (identity hidden layers on ReLU'd inputs shifted by +10 and back) gives activate(z[:9])."""
    rng = np.random.default_rng(5)
    C, M = 16, 3
    levels = [rng.standard_normal((16 >> l, 16 >> l, C)) for l in range(M)]
    q = wl.uniform_queries(rng, 300, 0, M - 1)
    dims = [C + 3, 32, 32, 9]
    bK = rng.normal(size=9)
    zero = np.concatenate([np.zeros(19 * 32 + 32 + 32 * 32 + 32 + 9 * 32), bK])
    out = oracle.sampler_params(levels, dims, zero, q.uv, q.lod, q.wi)
    np.testing.assert_allclose(out, np.tile(oracle.proxy_activate(bK), (300, 1)), rtol=1e-15)
    W1 = np.zeros((32, 19))
    W1[:9, :9] = np.eye(9)
    b1 = np.zeros(32)
    b1[:9] = 10.0
    W2, b2 = np.eye(32), np.zeros(32)
    W3 = np.zeros((9, 32))
    W3[:, :9] = np.eye(9)
    b3 = np.full(9, -10.0)
    packed = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    z = oracle.fetch(levels, q.uv, q.lod)
    assert np.abs(z[:, :9]).max() < 10
    out = oracle.sampler_params(levels, dims, packed, q.uv, q.lod, q.wi)
    np.testing.assert_allclose(out, oracle.proxy_activate(z[:, :9]), rtol=1e-12, atol=1e-12)


def _sampler_problem(C, hidden, n, seed):
    rng = np.random.default_rng(seed)
    M = 4
    levels = [rng.standard_normal((32 >> l, 32 >> l, C)) for l in range(M)]
    q = wl.uniform_queries(rng, n, -0.5, M - 0.5)
    dims, sp = wl.sampler_decoder(rng, C, hidden)
    return levels, q, dims, sp.astype(np.float64)


def test_quantised_sampler_without_rounding_equals_sampler_params():
    """With the rounding switched off (exact filter, layer inputs kept), the reduced-precision
    sampler is the sampling decoder itself; non-finite queries give NaN parameters."""
    levels, q, dims, sp = _sampler_problem(16, (32, 32, 32), 500, 9)
    q.uv[7, 0] = np.nan
    q.lod[11] = np.inf
    got = oracle.sampler_params_quant(levels, dims, sp, q.uv, q.lod, q.wi, fmt=oracle.FMT_NONE, blend_fp16=False)
    ref = oracle.sampler_params(levels, dims, sp, q.uv, q.lod, q.wi)
    ok = np.ones(len(q.lod), bool)
    ok[[7, 11]] = False
    np.testing.assert_allclose(got[ok], ref[ok], rtol=1e-12, atol=1e-14)
    assert np.isnan(got[~ok]).all()


def test_quantised_sampler_rounds_every_layer_input_and_nothing_else():
    """A one-hidden-layer sampler that carries h = z_0 + wi_x to two outputs, hand-computed with
    IEEE half rounding at the two places the arithmetic rounds (the network input, the hidden
    activation): raw_1 = 3 r(h) (not itself an FP16 value, so rounding the output would show),
    raw_7 = r(h) + 0.1 (the bias added unrounded).  The texel 0.3 sits under a texel-centre query
    at an integer level, so the FP16 filter gives r(0.3) and the exact one 0.3."""
    C, H = 8, 16
    levels = [np.full((8 >> l, 8 >> l, C), 0.3) for l in range(3)]
    uv = np.array([[2.5 / 8, 5.5 / 8]])
    lod = np.array([0.0])
    wi = np.array([[0.1, -0.2, 0.97]])
    W1 = np.zeros((H, C + 3))
    W1[0, 0] = 1.0
    W1[0, C] = 1.0
    W2 = np.zeros((9, H))
    W2[1, 0] = 3.0
    W2[7, 0] = 1.0
    b2 = np.zeros(9)
    b2[7] = 0.1
    packed = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), b2])
    dims = [C + 3, H, 9]
    r = lambda x: float(np.float16(x))
    qs = lambda x: x * (1.0 + 0.5 * abs(x))
    h = r(r(0.3) + r(0.1))                 # the input rounded, its exact sum rounded again
    got = oracle.sampler_params_quant(levels, dims, packed, uv, lod, wi)[0]
    assert got[1] == pytest.approx(qs(3.0 * h), rel=1e-15)
    assert got[7] == pytest.approx(qs(h + 0.1), rel=1e-15)
    assert got[0] == got[3] == 0.5
    exact = oracle.sampler_params_quant(levels, dims, packed, uv, lod, wi, fmt=oracle.FMT_NONE, blend_fp16=False)[0]
    assert exact[1] == pytest.approx(qs(3.0 * 0.4), rel=1e-15)
    assert abs(got[1] - exact[1]) > 1e-4 and abs(r(3.0 * h) - 3.0 * h) > 0
    # the FP16 filter alone: input rounding off, so only z_0 = r(0.3) enters unrounded wi
    f = oracle.sampler_params_quant(levels, dims, packed, uv, lod, wi, fmt=oracle.FMT_NONE, blend_fp16=True)[0]
    assert f[1] == pytest.approx(qs(3.0 * (r(0.3) + 0.1)), rel=1e-15)


def test_quantised_sampler_error_is_at_fp16_level():
    """The FP16 arithmetic moves the parameters of a random sampler by an FP16-sized amount,
    not more: within 2e-2 of the exact ones (relative to max(1, |p|)), and by more than 1e-6
    somewhere (the rounding is applied)."""
    levels, q, dims, sp = _sampler_problem(16, (32, 32, 32), 400, 10)
    ref = oracle.sampler_params(levels, dims, sp, q.uv, q.lod, q.wi)
    qp = np.concatenate([np.concatenate([W.astype(np.float16).astype(np.float64).ravel(), b])
                         for W, b in wl.unpack_params(sp, dims)])
    got = oracle.sampler_params_quant(levels, dims, qp, q.uv, q.lod, q.wi)
    e = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert 1e-6 < e.max() < 2e-2
