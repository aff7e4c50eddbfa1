"""The seeded input generators: determinism, distributions and structure."""
import math

import numpy as np
import pytest

from paper_2305_02678_amd import workloads as wl


def test_tiny_is_deterministic_and_shaped():
    a, b = wl.tiny(), wl.tiny()
    for x, y in zip(a.material.levels, b.material.levels):
        assert np.array_equal(x, y)
    assert np.array_equal(a.material.params, b.material.params)
    assert np.array_equal(a.queries.uv, b.queries.uv)
    c = wl.tiny(seed=1234)
    assert not np.array_equal(a.queries.uv, c.queries.uv)
    m = a.material
    assert [l.shape for l in m.levels] == [(64, 64, 8), (32, 32, 8), (16, 16, 8)]
    assert m.dims == [14, 32, 32, 3]
    assert m.params.dtype == np.float32 and m.params.size == wl.n_params(m.dims) == 14 * 32 + 32 + 32 * 32 + 32 + 32 * 3 + 3
    q = a.queries
    assert len(q) == 4096 and q.uv.dtype == np.float32
    assert q.uv.min() >= 0 and q.uv.max() < 1 and q.lod.min() >= 0 and q.lod.max() <= 2


def test_box_pyramid_levels_are_2x2_means():
    rng = np.random.default_rng(0)
    l0 = rng.standard_normal((16, 8, 3))
    pyr = wl.box_pyramid(l0, 5)
    assert [p.shape for p in pyr] == [(16, 8, 3), (8, 4, 3), (4, 2, 3), (2, 1, 3), (1, 1, 3)]
    np.testing.assert_allclose(pyr[1][2, 1], l0[4:6, 2:4].mean(axis=(0, 1)), rtol=1e-6)
    np.testing.assert_allclose(pyr[4][0, 0], l0.mean(axis=(0, 1)), rtol=1e-5, atol=1e-6)


def test_xavier_bounds_and_zero_biases():
    rng = np.random.default_rng(1)
    dims = [22, 64, 64, 64, 3]
    p = wl.xavier_mlp(rng, dims)
    for (W, b), fi, fo in zip(wl.unpack_params(p, dims), dims[:-1], dims[1:]):
        a = math.sqrt(6 / (fi + fo))
        assert W.shape == (fo, fi) and np.abs(W).max() <= a and np.abs(W).max() > 0.9 * a
        assert np.all(b == 0)


def test_cosine_hemisphere_moments():
    w = wl.cosine_hemisphere(np.random.default_rng(2), 200000).astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(w, axis=1), 1.0, atol=1e-6)
    assert w[:, 2].min() >= 0
    # pdf cos(theta)/pi: E[cos] = 2/3, E[cos^2] = 1/2, E[x] = E[y] = 0
    assert abs(w[:, 2].mean() - 2 / 3) < 3e-3
    assert abs((w[:, 2] ** 2).mean() - 0.5) < 3e-3
    assert abs(w[:, 0].mean()) < 5e-3 and abs(w[:, 1].mean()) < 5e-3


def test_tile_order_is_a_permutation_of_the_frame():
    px, py = wl.tile_order(40, 21)
    assert len(px) == 40 * 21
    assert len(set(zip(px.tolist(), py.tolist()))) == 40 * 21
    # the first 256 pixels form the top-left 16x16 tile
    assert px[:256].max() == 15 and py[:256].max() == 15


def test_screen_map_lod_matches_numerical_jacobian():
    rng = np.random.default_rng(3)
    smap = wl.random_screen_map(rng, 2048, 2048, 1920, 1080)
    px = rng.integers(0, 1920, 50)
    py = rng.integers(0, 1080, 50)
    uv, lod = smap.uv_and_lod(px, py)
    h = 1e-3

    def uv_at(x, y):
        A = smap.matrix()
        u = A[0, 0] * x + A[0, 1] * y + smap.c[0] + smap.warp_amp * np.sin(2 * np.pi * smap.f[0] / 1920 * x + smap.phi[0])
        v = A[1, 0] * x + A[1, 1] * y + smap.c[1] + smap.warp_amp * np.sin(2 * np.pi * smap.f[1] / 1080 * y + smap.phi[1])
        return np.stack([u, v], 1)

    x, y = px + 0.5, py + 0.5
    np.testing.assert_allclose(uv_at(x, y), uv, atol=1e-12)
    Jx = (uv_at(x + h, y) - uv_at(x - h, y)) / (2 * h)
    Jy = (uv_at(x, y + h) - uv_at(x, y - h)) / (2 * h)
    det = Jx[:, 0] * Jy[:, 1] - Jy[:, 0] * Jx[:, 1]
    np.testing.assert_allclose(lod, 0.5 * np.log2(np.abs(det) * 2048 * 2048), atol=1e-5)


def test_frame_workload_structure_small_texture():
    w = wl.frame(tex=256, channels=16, n=4096)
    assert len(w.queries) == 4096
    assert w.material.n_levels == 9 and w.material.dims == [22, 64, 64, 64, 3]
    assert np.isfinite(w.queries.lod).all()


def test_truncated_exponential_range_and_mean():
    x = wl.truncated_exponential(np.random.default_rng(4), 200000, 1.0, 10.0)
    assert x.min() >= 0 and x.max() <= 10.0
    # mean of Exp(1) truncated at 10: 1 - 10 e^-10 / (1 - e^-10)
    assert abs(x.mean() - (1 - 10 * math.exp(-10) / (1 - math.exp(-10)))) < 1e-2


def test_analytic_brdf_is_positive_reciprocal_and_energy_bounded():
    rng = np.random.default_rng(5)
    am = wl.make_analytic_material(rng)
    n = 4000
    uv = rng.random((n, 2))
    wi = wl.cosine_hemisphere(rng, n)
    wo = wl.cosine_hemisphere(rng, n)
    f = am.brdf(uv, wi, wo)
    assert (f > 0).all()
    # reciprocal up to the float32 rounding of the unit direction vectors (Schlick uses wi.h)
    np.testing.assert_allclose(am.brdf(uv, wo, wi), f, rtol=1e-5)
    rho = am.albedo(uv)
    assert rho.min() >= 0.05 and rho.max() <= 0.95
    r = am.roughness(uv)
    assert r.min() >= 0.3 and r.max() <= 0.9
    # periodic in uv (wrap-consistent)
    np.testing.assert_allclose(am.brdf(uv + 1.0, wi, wo), f, rtol=1e-9)
    # directional albedo int f cos dwi <= 1 (cosine sampling: estimator pi * f)
    m = 20000
    wim = wl.cosine_hemisphere(rng, m)
    for k in range(3):
        uvk = np.repeat(uv[k:k + 1], m, 0)
        wok = np.repeat(wo[k:k + 1], m, 0)
        alb = (np.pi * am.brdf(uvk, wim, wok)).mean(0)
        assert (alb < 1.0).all()


def test_training_workload_small():
    w = wl.training(tex=32, channels=8, n=1000, hidden=(32, 32))
    assert w.material.n_levels == 6 and w.targets.shape == (1000, 3)
    assert w.queries.lod.max() <= 5.0 and w.queries.lod.min() >= 0


def test_request_stream_sizes_and_order():
    mats = wl.serving_materials(count=3, sides=(64, 128))
    reqs = wl.request_stream(7, mats, 20, rate_per_s=100.0, lo=64, hi=5000)
    t = [r.arrival_s for r in reqs]
    assert t == sorted(t) and t[0] == 0.0
    for r in reqs:
        assert 64 <= len(r.queries) <= 5000 and 0 <= r.material < 3


def test_frame_layer_and_sampler_recipes():
    """Learned-frame layers: W_F Xavier-uniform scaled by 1/4, normals at +z and tangents at +x;
    the material's other draws do not move when frames are added (they are drawn last).
    Sampling decoders: [C + 3, hidden..., 9], Xavier weights, zero biases."""
    rng = np.random.default_rng(3)
    F = wl.frame_layer(rng, 2, 16)
    assert F.dtype == np.float32 and F.size == 12 * 16 + 12
    a = np.sqrt(6.0 / (16 + 12)) / 4
    assert np.abs(F[:192]).max() <= a and np.abs(F[:192]).max() > 0.9 * a
    np.testing.assert_array_equal(F[192:], np.tile([0, 0, 1, 1, 0, 0], 2))
    r1, r2 = wl.rngs(7), wl.rngs(7)
    plain = wl.make_material(r1[0], r1[1], 16, 16, 8, 3, [32, 32])
    framed = wl.make_material(r2[0], r2[1], 16, 16, 8, 3, [32, 32], n_frames=2)
    assert framed.dims == [20, 32, 32, 3] and plain.dims == [14, 32, 32, 3]
    for a_, b_ in zip(plain.levels, framed.levels):
        np.testing.assert_array_equal(a_, b_)
    sd, sp = wl.sampler_decoder(np.random.default_rng(4), 16)
    assert sd == [19, 32, 32, 32, 9] and sp.size == wl.n_params(sd)
    for W, b in wl.unpack_params(sp, sd):
        assert not b.any()


def test_directional_albedo_quadrature_and_one_sample_estimates():
    """Eq. albedo: the quadrature returns rho exactly for a Lambertian f = rho / pi, converges
    with the grid for the analytic material, and the mean of the one-sample estimates (rho for
    the Lambertian lobe, F G1 of one visible-normal sample for the GGX lobe) agrees with it
    within 4 standard errors; every estimate lies in [rho, rho + 1]."""
    rng = np.random.default_rng(77)
    am = wl.make_analytic_material(rng)

    class Lambert(wl.AnalyticMaterial):
        def brdf(self, uv, wi, wo):
            return np.repeat(self.albedo(uv)[:1], len(wi), 0) / np.pi

    uv = rng.random((3, 2))
    wo = wl.cosine_hemisphere(rng, 3)
    lam = Lambert(am.albedo_noise, am.rough_noise)
    for i in range(3):
        np.testing.assert_allclose(lam.directional_albedo(uv[i:i + 1], wo[i:i + 1], grid=16)[0],
                                   am.albedo(uv[i:i + 1])[0], rtol=1e-13)
    a256 = am.directional_albedo(uv, wo, grid=256)
    a512 = am.directional_albedo(uv, wo, grid=512)
    np.testing.assert_allclose(a256, a512, rtol=2e-3)
    n = 200000
    for i in range(3):
        est = am.albedo_estimates(rng, np.repeat(uv[i:i + 1], n, 0), np.repeat(wo[i:i + 1], n, 0))
        rho = am.albedo(uv[i:i + 1])[0]
        assert np.all(est >= rho) and np.all(est <= rho + 1.0)
        se = est.std(0) / math.sqrt(n)
        assert np.all(np.abs(est.mean(0) - a512[i]) < 4 * se + 1e-4), (i, est.mean(0), a512[i], se)


def test_albedo_training_workload_small():
    w = wl.training(seed=1004, tex=32, channels=8, n=4096, hidden=(32, 32), albedo=True)
    assert w.material.dims == [14, 32, 32, 6]
    assert w.targets.shape == (4096, 6) and w.targets.dtype == np.float32
    plain = wl.training(seed=1004, tex=32, channels=8, n=4096, hidden=(32, 32))
    np.testing.assert_array_equal(w.targets[:, :3], plain.targets)      # same samples, same RGB targets
    np.testing.assert_array_equal(w.material.levels[0], plain.material.levels[0])
    assert np.all(w.targets[:, 3:] > 0)
