"""GPU parity of the fetch and the FP32 decode against the FP64 oracle, through the C ABI.

Tolerances (FP32 path):
  * decoded RGB: max relative error <= 1e-5 per channel (y > 0 since softplus > 0);
  * fetch: |z - z_ref| <= 1e-5; the blend is 8 FP32 FMAs of weights <= 1 on N(0, 1) texels
    (|T| < 6), so the rounding error is below 8 * 2 * 2^-24 * 6 ~ 6e-6;
  * texel centres: bit-exact (every weight is exactly 0 or 1).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2305_02678_amd import workloads as wl

pytestmark = pytest.mark.gpu

RGB_RTOL_F32 = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def nam(torch):
    from paper_2305_02678_amd import nam as n
    n.lib()
    return n


@pytest.fixture(scope="module")
def ctx(nam):
    c = nam.Context(0)
    yield c


@pytest.fixture(scope="module")
def tiny():
    return wl.tiny()


def rel_err(got, ref):
    return np.abs(got - ref) / np.abs(ref)


def _say(*a):
    print(*a, flush=True)


def test_one_hip_runtime_in_process(nam, torch):
    torch.zeros(1, device="cuda")
    maps = open("/proc/self/maps").read()
    libs = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(libs) == 1, libs
    assert any("libnam.so" in line for line in maps.splitlines())


def test_fetch_texel_centres_bit_exact(nam, ctx, tiny, torch):
    m = tiny.material
    mat = nam.Material.from_workload(ctx, m)
    for l, T in enumerate(m.levels):
        H, W, C = T.shape
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        uv = np.stack([(xs.ravel() + 0.5) / W, (ys.ravel() + 0.5) / H], 1).astype(np.float32)
        lod = np.full(len(uv), l, np.float32)
        z = nam.fetch(mat, torch.from_numpy(uv).cuda(), torch.from_numpy(lod).cuda()).cpu().numpy()
        assert np.array_equal(z, T.reshape(-1, C)), l


@pytest.mark.parametrize("address", [wl.WRAP, wl.CLAMP])
def test_fetch_matches_oracle(nam, ctx, tiny, torch, address):
    m = tiny.material
    mat = nam.Material(ctx, m.levels, m.dims, m.params, address)
    q = tiny.queries
    rng = np.random.default_rng(0)
    uv = np.concatenate([q.uv, rng.uniform(-3, 4, (1000, 2)).astype(np.float32)])
    lod = np.concatenate([q.lod, rng.uniform(-2, 5, 1000).astype(np.float32)])
    z = nam.fetch(mat, torch.from_numpy(uv).cuda(), torch.from_numpy(lod).cuda()).cpu().numpy()
    zr = oracle.fetch(m.levels, uv, lod, address)
    assert np.abs(z - zr).max() <= 1e-5


def test_fetch_small_negative_uv_on_a_large_texture(nam, ctx, torch):
    """u in (-1/2, 0) on a 2048-wide level: the wrapped position must not go through a rounded
    fractional part of u (1 + u is inexact in FP32)."""
    r = wl.rngs(11)
    lv0 = r[0].standard_normal((2048, 2048, 8))
    levels = wl.box_pyramid(lv0, 2)
    dims = [14, 16, 3]
    mat = nam.Material(ctx, levels, dims, wl.xavier_mlp(r[1], dims))
    n = 20000
    uv = (-r[2].random((n, 2)) * 0.5 * 10.0 ** -r[2].integers(0, 6, (n, 1))).astype(np.float32)
    uv[::3] += r[2].integers(-300, 300, (len(uv[::3]), 2)).astype(np.float32)   # also |u| >= 256
    lod = r[2].uniform(0, 1, n).astype(np.float32)
    z = nam.fetch(mat, torch.from_numpy(uv).cuda(), torch.from_numpy(lod).cuda()).cpu().numpy()
    zr = oracle.fetch(levels, uv, lod)
    assert np.abs(z - zr).max() <= 1e-5


def test_decode_f32_tiny_parity(nam, ctx, tiny, torch):
    m, q = tiny.material, tiny.queries
    mat = nam.Material.from_workload(ctx, m)
    rgb = nam.decode(mat, *nam.to_device(q)).cpu().numpy().astype(np.float64)
    ref = oracle.decode(m.levels, m.dims, m.params, q.uv, q.lod, q.wi, q.wo)
    e = rel_err(rgb, ref)
    _say(f"tiny fp32: max rel {e.max():.3e} mean {e.mean():.3e}")
    assert e.max() <= RGB_RTOL_F32


@pytest.mark.parametrize("C", [8, 16])
@pytest.mark.parametrize("H,NH", [(16, 1), (16, 2), (32, 2), (32, 4), (64, 1), (64, 3), (64, 4)])
def test_decode_f32_shapes_ragged(nam, ctx, torch, C, H, NH):
    r = wl.rngs(100 + C + H + NH)
    mat_np = wl.make_material(r[0], r[1], 32, 16, C, 5, [H] * NH)
    mat_np.params = (mat_np.params + 0.05 * r[1].standard_normal(mat_np.params.size)).astype(np.float32)
    n = 1000 + 37
    q = wl.uniform_queries(r[2], n, -0.5, 5.5)
    q.uv[:100] += r[2].integers(-3, 4, (100, 2)).astype(np.float32)
    for address in (wl.WRAP, wl.CLAMP):
        mat = nam.Material(ctx, mat_np.levels, mat_np.dims, mat_np.params, address)
        rgb = nam.decode(mat, *nam.to_device(q)).cpu().numpy().astype(np.float64)
        ref = oracle.decode(mat_np.levels, mat_np.dims, mat_np.params, q.uv, q.lod, q.wi, q.wo, address)
        assert rel_err(rgb, ref).max() <= RGB_RTOL_F32


def test_decode_edge_inputs(nam, ctx, tiny, torch):
    m = tiny.material
    mat = nam.Material.from_workload(ctx, m)
    # n = 0 is a no-op
    empty = torch.empty((0, 2), device="cuda")
    out = nam.decode(mat, empty, torch.empty(0, device="cuda"), torch.empty((0, 3), device="cuda"),
                     torch.empty((0, 3), device="cuda"))
    assert out.shape == (0, 3)
    # n = 1, and non-finite inputs mixed with finite ones
    q = tiny.queries.subset(slice(0, 8))
    uv, lod = q.uv.copy(), q.lod.copy()
    uv[1, 0] = np.nan
    uv[2, 1] = np.inf
    lod[3] = -np.inf
    lod[4] = np.nan
    uv[5] = [1e30, -1e30]
    lod[6] = 1e30
    qq = wl.Queries(uv, lod, q.wi, q.wo)
    rgb = nam.decode(mat, *nam.to_device(qq)).cpu().numpy()
    assert np.isnan(rgb[1:5]).all()
    assert np.isfinite(rgb[[0, 5, 6, 7]]).all()
    ref = oracle.decode(m.levels, m.dims, m.params, uv[[0, 5, 6, 7]], lod[[0, 5, 6, 7]], q.wi[[0, 5, 6, 7]],
                        q.wo[[0, 5, 6, 7]])
    assert rel_err(rgb[[0, 5, 6, 7]], ref).max() <= RGB_RTOL_F32
    one = nam.decode(mat, *nam.to_device(q.subset(slice(0, 1)))).cpu().numpy()
    assert np.array_equal(one[0], nam.decode(mat, *nam.to_device(q)).cpu().numpy()[0])


def test_single_texel_pyramid(nam, ctx, torch):
    r = wl.rngs(5)
    m = wl.make_material(r[0], r[1], 1, 1, 8, 1, [32, 32])
    q = wl.uniform_queries(r[2], 300, -1, 3)
    mat = nam.Material.from_workload(ctx, m)
    rgb = nam.decode(mat, *nam.to_device(q)).cpu().numpy()
    ref = oracle.decode(m.levels, m.dims, m.params, q.uv, q.lod, q.wi, q.wo)
    assert rel_err(rgb, ref).max() <= RGB_RTOL_F32


def test_texel_footprint_matches_oracle_taps(nam, ctx, tiny, torch):
    m, q = tiny.material, tiny.queries
    mat = nam.Material.from_workload(ctx, m)
    for sl in (slice(0, 1), slice(0, 100), slice(0, 4096)):
        qq = q.subset(sl)
        u = nam.texel_footprint(mat, *nam.to_device(qq)[:2])
        assert u == len(np.unique(oracle.taps(m.levels, qq.uv, qq.lod)))


def test_calibrate_first_layer_absmax(nam, ctx, tiny, torch):
    m, q = tiny.material, tiny.queries
    mat = nam.Material.from_workload(ctx, m)
    am = mat.calibrate(*nam.to_device(q))
    z = oracle.fetch(m.levels, q.uv, q.lod)
    x = np.concatenate([z, q.wi, q.wo], 1)
    assert abs(am[0] - np.abs(x).max()) <= 1e-5 * np.abs(x).max()
    assert (am > 0).all() and len(am) == len(m.dims) - 1


def test_bad_arguments(nam, ctx, tiny, torch):
    m = tiny.material
    mat = nam.Material.from_workload(ctx, m)
    L = nam.lib()
    uv, lod, wi, wo = nam.to_device(tiny.queries)
    rgb = torch.empty((len(tiny.queries), 3), device="cuda")
    assert L.nam_decode(ctx.handle, mat.handle, -1, uv.data_ptr(), lod.data_ptr(), wi.data_ptr(), wo.data_ptr(),
                        rgb.data_ptr(), None) == nam.NAM_E_INVALID_ARG
    assert L.nam_decode(ctx.handle, mat.handle, 10, None, lod.data_ptr(), wi.data_ptr(), wo.data_ptr(),
                        rgb.data_ptr(), None) == nam.NAM_E_INVALID_ARG
    assert L.nam_decode(ctx.handle, mat.handle, 10, uv.data_ptr() + 4, lod.data_ptr(), wi.data_ptr(),
                        wo.data_ptr(), rgb.data_ptr(), None) == nam.NAM_E_INVALID_ARG
    with pytest.raises(nam.NamError) as e:
        nam.Material(ctx, m.levels, [14, 48, 3], np.zeros(14 * 48 + 48 + 48 * 3 + 3, np.float32))
    assert e.value.status == nam.NAM_E_UNSUPPORTED
    with pytest.raises(nam.NamError) as e:
        nam.Material(ctx, m.levels, [15, 32, 3], np.zeros(15 * 32 + 32 + 32 * 3 + 3, np.float32))
    assert e.value.status == nam.NAM_E_SHAPE
    assert mat.footprint() >= sum(l.nbytes for l in m.levels)


@pytest.fixture(scope="module")
def frame():
    return wl.frame()


def test_decode_f32_frame_full_size_sampled(nam, ctx, frame, torch):
    """The full 1920x1080 frame on the 2048^2 x 16 material in the benchmark's launch
    configuration; 32768 random pixels plus the ragged last 1000 are checked one by one."""
    m, q = frame.material, frame.queries
    mat = nam.Material.from_workload(ctx, m)
    rgb = nam.decode(mat, *nam.to_device(q)).cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(len(q), 32768, replace=False), np.arange(len(q) - 1000, len(q))])
    s = q.subset(idx)
    ref = oracle.decode(m.levels, m.dims, m.params, s.uv, s.lod, s.wi, s.wo)
    e = rel_err(rgb[idx], ref)
    _say(f"frame fp32: max rel {e.max():.3e} mean {e.mean():.3e}")
    assert e.max() <= RGB_RTOL_F32
