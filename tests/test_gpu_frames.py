"""Decode with learned shading frames (Sec. 4.2, Eq. frame-rotation), through the C ABI,
against the FP64 oracle's orc_decode_frames on the same inputs.

Tolerances are those of the plain decode: FP32 max relative RGB error <= 1e-5, FP16 <= 2e-3.
The frame layer and the transform run in FP32 in every precision.  An identity frame layer
(N = 1) must reproduce the plain decode bit for bit in every precision and for both filters,
which ties the frame plumbing to the already-tested decode.
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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def small_problem(C, H, NH, nf, address, seed=43, n=3000, tex=64, M=6):
    r = wl.rngs(seed)
    mat = wl.make_material(r[0], r[1], tex, tex, C, M, [H] * NH, address=address, n_frames=nf)
    q = wl.uniform_queries(r[2], n, -0.5, M - 0.5)
    q.uv[: n // 10] += r[2].integers(-3, 4, (n // 10, 2)).astype(np.float32)
    q.lod[: n // 20] = np.round(q.lod[: n // 20])
    xi = r[4].random(n).astype(np.float32)
    return mat, q, xi


def _ref(m, q, xi=None, address=wl.WRAP):
    return oracle.decode_frames(m.levels, m.dims, m.params, m.n_frames, m.frame_params, q.uv, q.lod, q.wi, q.wo,
                                xi=xi, address=address)


@pytest.mark.parametrize("address", [wl.WRAP, wl.CLAMP])
@pytest.mark.parametrize("C,H,NH,nf", [(16, 64, 3, 2), (8, 32, 2, 2), (16, 16, 4, 1), (8, 64, 1, 2), (16, 32, 2, 1)])
def test_frames_match_oracle_fp32_and_fp16(nam, ctx, torch, address, C, H, NH, nf):
    m, q, xi = small_problem(C, H, NH, nf, address)
    assert m.dims[0] == C + 6 * max(1, nf)
    ref = _ref(m, q, address=address)
    ref_rr = _ref(m, q, xi, address)
    mat = nam.Material.from_workload(ctx, m)
    dq, dxi = nam.to_device(q), _dev(torch, xi)
    e32 = rel_err(nam.decode(mat, *dq).cpu().numpy(), ref)
    r32 = rel_err(nam.decode(mat, *dq, xi=dxi).cpu().numpy(), ref_rr)
    mat.set_precision(nam.F16)
    e16 = rel_err(nam.decode(mat, *dq).cpu().numpy(), ref)
    r16 = rel_err(nam.decode(mat, *dq, xi=dxi).cpu().numpy(), ref_rr)
    _say(f"frames C{C} H{H}x{NH} N{nf} addr {address}: fp32 {e32.max():.2e} (rr {r32.max():.2e}), "
         f"fp16 {e16.max():.2e} (rr {r16.max():.2e})")
    assert max(e32.max(), r32.max()) <= 1e-5
    assert max(e16.max(), r16.max()) <= 2e-3


def test_frames_frame_workload(nam, ctx, torch):
    """The 1080p frame with two frames (decoder 28-64-64-64-3) at full size, sampled queries
    plus the ragged last chunk."""
    w = wl.frame(n_frames=2)
    m, q = w.material, w.queries
    assert m.dims == [28, 64, 64, 64, 3]
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(len(q), 12000, replace=False), np.arange(len(q) - 300, len(q))])
    s = q.subset(idx)
    ref = _ref(m, s)
    mat = nam.Material.from_workload(ctx, m)
    dq = nam.to_device(q)
    e32 = rel_err(nam.decode(mat, *dq).cpu().numpy()[idx], ref)
    mat.set_precision(nam.F16)
    e16 = rel_err(nam.decode(mat, *dq).cpu().numpy()[idx], ref)
    _say(f"frames 1080p: fp32 max {e32.max():.2e}, fp16 max {e16.max():.2e} mean {e16.mean():.2e}")
    assert e32.max() <= 1e-5
    assert e16.max() <= 2e-3


def _identity_pair(nam, ctx, C=16, H=64, NH=3, seed=44):
    r = wl.rngs(seed)
    plain = wl.make_material(r[0], r[1], 64, 64, C, 6, [H] * NH)
    F = np.zeros(6 * C + 6, np.float32)
    F[6 * C:] = [0.0, 0.0, 2.0, 0.5, 0.0, 0.0]              # n = (0, 0, 2), t = (0.5, 0, 0)
    framed = wl.Material(plain.width, plain.height, C, plain.levels, plain.dims, plain.params, plain.address, 1, F)
    q = wl.uniform_queries(r[2], 5000, -0.5, 5.5)
    return nam.Material.from_workload(ctx, plain), nam.Material.from_workload(ctx, framed), q, r[4].random(5000)


def test_identity_frame_is_bit_exact_in_every_precision(nam, ctx, torch):
    """n along +z and t along +x with power-of-two lengths: T is exactly the identity in FP32,
    so the framed material decodes bit for bit as the plain one (FP32, FP16, E4M3, both
    filters), including calibration.  The one exception is the plain FP32 trilinear decode,
    which runs on the FP32 matrix cores while framed decodes run on the vector ALU: both are
    FP32 roundings summed in different orders, held to the FP32 parity bound (1e-5 relative)."""
    plain, framed, q, xi = _identity_pair(nam, ctx)
    dq, dxi = nam.to_device(q), _dev(torch, xi)
    calib = nam.to_device(wl.uniform_queries(np.random.default_rng(9), 20000, 0, 5))
    am_p, am_f = plain.calibrate(*calib), framed.calibrate(*calib)
    assert np.array_equal(am_p, am_f)
    for prec in (nam.F32, nam.F16, nam.FP8_E4M3):
        kw = {"act_absmax": am_p} if prec == nam.FP8_E4M3 else {}
        plain.set_precision(prec, **kw)
        framed.set_precision(prec, **kw)
        for x in (None, dxi):
            a = nam.decode(plain, *dq, xi=x)
            b = nam.decode(framed, *dq, xi=x)
            if prec == nam.F32 and x is None:
                torch.testing.assert_close(a, b, rtol=1e-5, atol=0.0)
            else:
                assert torch.equal(a, b), (prec, x is None)


def test_fp8_with_frames_stays_close(nam, ctx, torch):
    """E4M3 with two frames: calibrated on the framed FP32 decoder; the error against the FP64
    oracle stays in the range of the plain E4M3 decode (mean relative error <= 1e-2)."""
    m, q, _ = small_problem(16, 64, 3, 2, wl.WRAP, n=20000)
    mat = nam.Material.from_workload(ctx, m)
    am = mat.calibrate(*nam.to_device(q))
    assert am.shape == (4,) and np.all(am > 0)
    mat.set_precision(nam.FP8_E4M3, act_absmax=am)
    e8 = rel_err(nam.decode(mat, *nam.to_device(q)).cpu().numpy(), _ref(m, q))
    _say(f"frames e4m3: max {e8.max():.2e} mean {e8.mean():.2e}")
    assert np.isfinite(e8).all() and e8.mean() <= 1e-2


def test_server_applies_the_frames(nam, ctx, torch):
    m, q, _ = small_problem(16, 64, 3, 2, wl.WRAP, n=40000)
    mat = nam.Material.from_workload(ctx, m)
    mat.set_precision(nam.F16)
    srv = nam.Server(ctx, budget_bytes=64 << 20, n_streams=2, max_tile=8192)
    mid = srv.add_material(mat)
    dq = nam.to_device(q)
    out = torch.empty((len(q), 3), device="cuda")
    srv.submit(mid, *dq, out)
    srv.wait_all()
    alone = nam.decode(mat, *dq)
    torch.cuda.synchronize()
    assert torch.equal(out, alone)
    srv.close()


def test_frame_argument_checks(nam, ctx):
    m, _, _ = small_problem(8, 32, 2, 2, wl.WRAP, n=10)
    with pytest.raises(nam.NamError, match="NAM_E_UNSUPPORTED"):
        nam.Material(ctx, m.levels, m.dims, m.params, m.address, 3, np.zeros(3 * 6 * 9, np.float32))
    with pytest.raises(nam.NamError, match="NAM_E_SHAPE"):
        nam.Material(ctx, m.levels, m.dims, m.params, m.address, 1, m.frame_params[: 6 * 9])
    with pytest.raises(nam.NamError, match="NAM_E_SHAPE"):
        nam.Material(ctx, m.levels, [14] + m.dims[1:], m.params, m.address, 2, m.frame_params)


# ----------------------------------------------------- training through the frame layer


def _grad_close(g, ref, name):
    """The gradient tolerance of the training tests: per tensor norm-relative <= 1e-3, and
    element-wise |g - ref| <= 1e-3 max(|ref|, 1e-3 max|ref|)."""
    g, ref = np.asarray(g, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    norm_rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    bound = 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    bad = np.abs(g - ref) > bound
    _say(f"{name}: norm-relative error {norm_rel:.2e}, element-wise violations {bad.sum()} of {g.size}")
    assert norm_rel <= 1e-3, name
    assert not bad.any(), (name, np.flatnonzero(bad)[:5])


def _frame_train_problem(C, hidden, nf, n=700, seed=47, tex=16):
    r = wl.rngs(seed)
    M = wl.full_chain(tex, tex)
    mat = wl.make_material(r[0], r[1], tex, tex, C, M, list(hidden), n_frames=nf)
    mat.params = (mat.params + 0.1 * r[1].standard_normal(mat.params.size)).astype(np.float32)
    F = mat.frame_params.astype(np.float64)
    F[: 6 * nf * C] += 0.2 * r[1].standard_normal(6 * nf * C)      # frames that read z strongly
    mat.frame_params = F.astype(np.float32)
    q = wl.uniform_queries(r[2], n, -0.5, M - 0.5)
    q.uv[: n // 4] += r[2].integers(-2, 3, (n // 4, 2)).astype(np.float32)
    q.uv[3] = [np.nan, 0.5]
    q.lod[8] = np.inf
    am = wl.make_analytic_material(r[3])
    tgt = am.brdf(np.nan_to_num(q.uv), q.wi, q.wo).astype(np.float32)
    return mat, q, tgt


@pytest.mark.parametrize("C,hidden,nf", [(8, (32, 32), 1), (8, (32, 32), 2), (16, (64, 64, 64), 2)])
def test_frame_layer_gradients_match_oracle(nam, ctx, torch, C, hidden, nf):
    """Loss, decoder, frame-layer and texel gradients of a model with learned shading frames
    against the oracle's analytic gradients (pinned by central differences), non-finite
    samples present; the forward against the oracle's framed decode."""
    mat, q, tgt = _frame_train_problem(C, hidden, nf)
    model = nam.Model.from_workload(ctx, mat)
    assert model.n_frames == nf
    params = np.concatenate([mat.frame_params, mat.params])
    tex, par, tg = _dev(torch, nam.concat_levels(mat.levels)), _dev(torch, params), _dev(torch, tgt)
    dq = nam.to_device(q)
    rgb = model.forward(tex, par, *dq).cpu().numpy()
    ref = oracle.decode_frames(mat.levels, mat.dims, mat.params, nf, mat.frame_params, q.uv, q.lod, q.wi, q.wo)
    keep = np.isfinite(ref).all(axis=1)
    assert np.isnan(rgb[~keep]).all()
    assert rel_err(rgb[keep], ref[keep]).max() <= 1e-5
    loss, d_tex, d_par = model.loss_backward(tex, par, *dq, tg)
    L, dP, dF, dL = oracle.loss_grad_frames(mat.levels, mat.dims, mat.params, mat.frame_params, nf, q.uv, q.lod,
                                            q.wi, q.wo, tgt)
    assert abs(loss.item() - L) <= 1e-5 * L
    g = d_par.cpu().numpy()
    nfp = model.frame_param_count
    _grad_close(g[:nfp], dF, f"frame layer nf={nf}")
    _grad_close(g[nfp:], dP, f"decoder nf={nf}")
    _grad_close(d_tex.cpu().numpy(), nam.concat_levels(dL), f"texels nf={nf}")


def test_framed_material_trains_end_to_end(nam, ctx, torch):
    """A decoder 28-64-64-64-3 with two learned shading frames, its frame layer, decoder and
    latents trained together by nam_train_step (300 Adam steps on the analytic material); the
    loss falls, and the trained frame layer and decoder loaded as a framed material decode
    (nam_decode, FP32) what the training forward computes."""
    w = wl.training(seed=1004, tex=64, channels=16, n=1 << 16, hidden=(64, 64, 64))
    r = wl.rngs(77)
    m = w.material
    m.n_frames = 2
    dims = [16 + 12, 64, 64, 64, 3]
    dec = wl.xavier_mlp(r[1], dims).astype(np.float32)
    F = wl.frame_layer(r[1], 2, 16)
    m.dims, m.params, m.frame_params = dims, dec, F
    model = nam.Model.from_workload(ctx, m)
    tex = _dev(torch, nam.concat_levels(m.levels))
    par = _dev(torch, np.concatenate([F, dec]))
    tr = nam.Trainer(model, tex, par, lr=2e-3)
    dq = nam.to_device(w.queries)
    tg = _dev(torch, w.targets)
    losses = [tr.step(*dq, tg).item() for _ in range(300)]
    _say(f"framed training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.2 * losses[0]
    p = par.cpu().numpy()
    nfp = model.frame_param_count
    assert np.abs(p[:nfp] - F).max() > 1e-3            # the frame layer did move
    levels = nam.split_levels(tex.cpu().numpy(), m.width, m.height, m.n_levels)
    mat = nam.Material(ctx, levels, dims, p[nfp:], m.address, 2, p[:nfp])
    sub = w.queries.subset(np.arange(4096))
    got = nam.decode(mat, *nam.to_device(sub)).cpu().numpy()
    fwd = model.forward(tex, par, *nam.to_device(sub)).cpu().numpy()
    assert rel_err(got, fwd).max() <= 1e-5
