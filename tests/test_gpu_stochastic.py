"""Decode with the level chosen by Russian roulette (Sec. 4.1), through the C ABI, against the
FP64 oracle's orc_decode_rr on the same draws.

Tolerances are those of the trilinear decode: FP32 max relative RGB error <= 1e-5, FP16
<= 2e-3.  The level choice is an integer decision made from the draw and t = lam - floor(lam),
both exact in FP32 and FP64, so both sides take the same level for every query.
"""
import numpy as np
import pytest

import oracle
from paper_2305_02678_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def nam(torch):
    from paper_2305_02678_amd import nam as n
    n.lib()
    return n


@pytest.fixture(scope="module")
def ctx(nam):
    return nam.Context(0)


def _say(*a):
    print(*a, flush=True)


def rel_err(got, ref):
    return np.abs(got - ref) / np.abs(ref)


def draws(rng, n):
    """Seeded uniform draws on [0, 1) in FP32, with the edge values 0, the largest float below 1
    and NaN planted."""
    xi = rng.random(n).astype(np.float32)
    xi[:: 97] = 0.0
    xi[1:: 97] = np.nextafter(np.float32(1.0), np.float32(0.0))
    xi[2:: 211] = np.nan
    return xi


def small_problem(C, H, NH, address, seed=41, n=3000, tex=64, M=6):
    r = wl.rngs(seed)
    mat = wl.make_material(r[0], r[1], tex, tex, C, M, [H] * NH, address=address)
    q = wl.uniform_queries(r[2], n, -0.5, M - 0.5)
    q.lod[: n // 20] = np.round(q.lod[: n // 20])           # integer levels: t = 0
    q.uv[: n // 10] += r[2].integers(-3, 4, (n // 10, 2)).astype(np.float32)
    return mat, q, draws(r[4], n)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("address", [wl.WRAP, wl.CLAMP])
@pytest.mark.parametrize("C,H,NH", [(8, 32, 2), (16, 64, 3), (16, 16, 4), (8, 64, 1)])
def test_rr_matches_oracle_fp32_and_fp16(nam, ctx, torch, address, C, H, NH):
    m, q, xi = small_problem(C, H, NH, address)
    ref = oracle.decode_rr(m.levels, m.dims, m.params, q.uv, q.lod, xi, q.wi, q.wo, address)
    mat = nam.Material.from_workload(ctx, m)
    dq = nam.to_device(q)
    dxi = _dev(torch, xi)
    e32 = rel_err(nam.decode(mat, *dq, xi=dxi).cpu().numpy(), ref)
    mat.set_precision(nam.F16)
    e16 = rel_err(nam.decode(mat, *dq, xi=dxi).cpu().numpy(), ref)
    _say(f"rr C{C} H{H}x{NH} addr {address}: fp32 max {e32.max():.2e}, fp16 max {e16.max():.2e}")
    assert e32.max() <= 1e-5
    assert e16.max() <= 2e-3


def test_rr_frame(nam, ctx, torch):
    w = wl.frame()
    m, q = w.material, w.queries
    xi = draws(np.random.default_rng(12), len(q))
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(len(q), 12000, replace=False), np.arange(len(q) - 300, len(q))])
    s = q.subset(idx)
    ref = oracle.decode_rr(m.levels, m.dims, m.params, s.uv, s.lod, xi[idx], s.wi, s.wo)
    mat = nam.Material.from_workload(ctx, m)
    dq, dxi = nam.to_device(q), _dev(torch, xi)
    e32 = rel_err(nam.decode(mat, *dq, xi=dxi).cpu().numpy()[idx], ref)
    mat.set_precision(nam.F16)
    e16 = rel_err(nam.decode(mat, *dq, xi=dxi).cpu().numpy()[idx], ref)
    _say(f"rr frame: fp32 max {e32.max():.2e}, fp16 max {e16.max():.2e} mean {e16.mean():.2e}")
    assert e32.max() <= 1e-5
    assert e16.max() <= 2e-3


@pytest.mark.parametrize("prec", ["f32", "f16"])
def test_rr_draw_one_is_the_integer_level_decode(nam, ctx, torch, prec):
    """A draw of (almost) 1 never falls below t: every query takes level floor(lam), where the
    trilinear decode at that integer level adds only zero-weight taps, so the two agree bit
    for bit in FP16 (one kernel).  In FP32 the trilinear decode runs on the FP32 matrix cores
    and the stochastic one on the vector ALU, two FP32 summation orders: held to the FP32
    parity bound (1e-5 relative)."""
    m, q, _ = small_problem(16, 64, 3, wl.WRAP, n=2000)
    mat = nam.Material.from_workload(ctx, m)
    if prec == "f16":
        mat.set_precision(nam.F16)
    M = len(m.levels)
    l0 = np.floor(np.clip(q.lod, 0, M - 1)).astype(np.float32)
    one = np.full(len(q), np.nextafter(np.float32(1.0), np.float32(0.0)), np.float32)
    a = nam.decode(mat, *nam.to_device(q), xi=_dev(torch, one)).cpu().numpy()
    q0 = wl.Queries(q.uv, l0, q.wi, q.wo)
    b = nam.decode(mat, *nam.to_device(q0)).cpu().numpy()
    if prec == "f32":
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=0.0)
    else:
        np.testing.assert_array_equal(a, b)


def test_rr_mean_over_draws_is_the_level_mixture(nam, ctx, torch):
    m, q, _ = small_problem(8, 32, 2, wl.WRAP, n=1500)
    mat = nam.Material.from_workload(ctx, m)
    M = len(m.levels)
    lam = np.clip(q.lod.astype(np.float64), 0, M - 1)
    l0 = np.floor(lam)
    t = lam - l0
    l1 = np.minimum(l0 + 1, M - 1)
    K = 32
    dq = nam.to_device(q)
    mean = np.zeros((len(q), 3))
    for k in range(K):
        mean += nam.decode(mat, *dq, xi=_dev(torch, np.full(len(q), (k + 0.5) / K))).cpu().numpy()
    mean /= K
    g0 = nam.decode(mat, *nam.to_device(wl.Queries(q.uv, l0.astype(np.float32), q.wi, q.wo))).cpu().numpy()
    g1 = nam.decode(mat, *nam.to_device(wl.Queries(q.uv, l1.astype(np.float32), q.wi, q.wo))).cpu().numpy()
    mix = (1 - t)[:, None] * g0 + t[:, None] * g1
    assert (np.abs(mean - mix) <= np.abs(g1 - g0) / (2 * K) + 1e-5).all()


def test_rr_arguments_and_non_finite(nam, ctx, torch):
    w = wl.tiny()
    mat = nam.Material.from_workload(ctx, w.material)
    q = wl.Queries(w.queries.uv.copy(), w.queries.lod.copy(), w.queries.wi, w.queries.wo)
    q.uv[3] = [np.nan, 0.5]
    q.lod[7] = np.inf
    xi = np.random.default_rng(0).random(len(q)).astype(np.float32)
    for prec in (None, nam.F16):
        if prec is not None:
            mat.set_precision(prec)
        rgb = nam.decode(mat, *nam.to_device(q), xi=_dev(torch, xi)).cpu().numpy()
        assert np.isnan(rgb[[3, 7]]).all()
        assert np.isfinite(np.delete(rgb, [3, 7], axis=0)).all()
    lib = nam.lib()
    dq = nam.to_device(q)
    out = torch.empty((len(q), 3), device="cuda")
    st = lib.nam_decode_stochastic(ctx.handle, mat.handle, len(q), dq[0].data_ptr(), dq[1].data_ptr(), None,
                                   dq[2].data_ptr(), dq[3].data_ptr(), out.data_ptr(), None)
    assert st == nam.NAM_E_INVALID_ARG


def test_rr_footprint(nam, ctx, torch):
    """Distinct texels of the Russian-roulette taps: with draws of 1 they are the oracle's
    level-l0 taps (its first four at the integer level); they never exceed the trilinear
    footprint, and with uniform draws they lie between the footprints of the two levels."""
    m, q, xi = small_problem(16, 32, 2, wl.WRAP, n=5000)
    mat = nam.Material.from_workload(ctx, m)
    M = len(m.levels)
    l0 = np.floor(np.clip(q.lod, 0, M - 1)).astype(np.float32)
    l1 = np.minimum(l0 + 1, M - 1).astype(np.float32)
    one = np.full(len(q), np.nextafter(np.float32(1.0), np.float32(0.0)), np.float32)
    dq = nam.to_device(q)
    got = nam.texel_footprint(mat, dq[0], dq[1], xi=_dev(torch, one))
    assert got == len(np.unique(oracle.taps(m.levels, q.uv, l0)[:, :4]))
    zero = np.zeros(len(q), np.float32)
    mixed = nam.texel_footprint(mat, dq[0], dq[1], xi=_dev(torch, xi))
    tri = nam.texel_footprint(mat, dq[0], dq[1])
    u0 = len(np.unique(oracle.taps(m.levels, q.uv, l0)[:, :4]))
    u1 = len(np.unique(oracle.taps(m.levels, q.uv, l1)[:, :4]))
    assert nam.texel_footprint(mat, dq[0], dq[1], xi=_dev(torch, zero)) <= tri
    assert mixed <= tri and mixed <= u0 + u1
