"""The encoder of Sec. 5.1 and the first training phase through the C ABI, against the FP64
oracle (orc_encode, orc_encode_queries, orc_loss_grad_codes, orc_encoder_backward).

Tolerances (FP32 kernels against FP64): codes within 1e-5 relative to max(1, |z|) (a few FP32
roundings through at most three layers); gradients norm-relative within 1e-5 per tensor (sums
over thousands of samples in a different order), as the decoder's own training tests.  The
two-phase run at the end checks the paper's procedure: the end-to-end phase lowers the loss,
the bake carries it into a latent texture, and training that texture directly lowers it
further.
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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _rel(a, b):
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def _norm_rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _attr_pyramid(rng, size, levels, A):
    return [rng.random((size >> l, size >> l, A)).astype(np.float32) for l in range(levels)]


def _queries(rng, n, M):
    q = wl.uniform_queries(rng, n, -0.5, M - 0.5)
    q.uv[: n // 10] += rng.integers(-3, 4, (n // 10, 2)).astype(np.float32)
    return q


SHAPES = [(4, 16, 32, 2), (4, 8, 16, 1), (8, 16, 64, 2), (16, 8, 32, 1), (16, 16, 64, 1)]


@pytest.mark.parametrize("A,C,HE,NHE", SHAPES)
@pytest.mark.parametrize("address", [wl.WRAP, wl.CLAMP])
def test_encoder_codes_match_oracle(nam, ctx, torch, A, C, HE, NHE, address):
    rng = np.random.default_rng(10 + A + C + HE + NHE)
    M, size, n = 5, 32, 3 * 1024 + 77
    attr = _attr_pyramid(rng, size, M, A)
    dims, ep = wl.encoder_params(rng, A, C, [HE] * NHE)
    ep = (ep + 0.05 * rng.standard_normal(ep.size)).astype(np.float32)
    enc = nam.Encoder(ctx, dims, size, size, M, address)
    flat = _dev(torch, np.concatenate([l.reshape(-1, A) for l in attr]))
    dep = _dev(torch, ep)
    q = _queries(rng, n, M)
    q.uv[5, 0] = np.nan
    q.lod[9] = np.inf
    z = enc.encode_queries(dep, flat, _dev(torch, q.uv), _dev(torch, q.lod)).cpu().numpy().astype(np.float64)
    ref = oracle.encode_queries(attr, dims, ep, q.uv, q.lod, address)
    ok = np.isfinite(ref).all(1)
    assert (~ok).sum() == 2 and np.isnan(z[~ok]).all()
    e = _rel(z[ok], ref[ok])
    baked = enc.encode_texels(dep, flat).cpu().numpy().astype(np.float64)
    eb = _rel(baked, oracle.encode(dims, ep, np.concatenate([l.reshape(-1, A) for l in attr])))
    _say(f"encoder A{A} C{C} H{HE}x{NHE}: query codes {e.max():.2e}, bake {eb.max():.2e}")
    assert e.max() <= 1e-5 and eb.max() <= 1e-5
    # at texel centres of integer levels the query code is the baked texel's, bit for bit
    for level in range(M):
        w = size >> level
        x, y = rng.integers(0, w, 64), rng.integers(0, w, 64)
        uv = np.stack([(x + 0.5) / w, (y + 0.5) / w], 1).astype(np.float32)
        zc = enc.encode_queries(dep, flat, _dev(torch, uv), _dev(torch, np.full(64, level, np.float32)))
        base = sum((size >> l) ** 2 for l in range(level))
        np.testing.assert_array_equal(zc.cpu().numpy(), baked[base + y * w + x].astype(np.float32))


@pytest.mark.parametrize("C,hidden", [(16, (64, 64, 64)), (8, (32, 32)), (8, (16,)), (16, (32, 32, 32, 32))])
def test_codes_loss_matches_oracle(nam, ctx, torch, C, hidden):
    """The decoder's loss on given codes: matrix-core (C 16, 3 x 64; C 8, 2 x 32) and vector
    (1 x 16, 4 x 32) training kernels; a non-finite code is skipped."""
    rng = np.random.default_rng(20 + C + len(hidden))
    n = 2 * 4096 + 37
    dims = [C + 6] + list(hidden) + [3]
    params = (wl.xavier_mlp(rng, dims) + 0.05 * rng.standard_normal(wl.n_params(dims))).astype(np.float32)
    z = rng.normal(0, 1, (n, C)).astype(np.float32)
    z[7, 3] = np.nan
    wi, wo = wl.cosine_hemisphere(rng, n), wl.cosine_hemisphere(rng, n)
    target = rng.random((n, 3)).astype(np.float32)
    model = nam.Model(ctx, 16, 16, C, 1, dims)
    loss, dz, dp = model.loss_backward_codes(_dev(torch, params), _dev(torch, z), _dev(torch, wi), _dev(torch, wo),
                                             _dev(torch, target))
    rl, rdp, rdz = oracle.loss_grad_codes(dims, params, z, wi, wo, target)
    dz, dp = dz.cpu().numpy().astype(np.float64), dp.cpu().numpy().astype(np.float64)
    el, ep_, ez = abs(float(loss.item()) - rl) / rl, _norm_rel(dp, rdp), _norm_rel(dz, rdz)
    _say(f"codes loss C{C} {hidden}: loss {el:.2e}, d_params {ep_:.2e}, dz {ez:.2e}")
    assert el <= 1e-5 and ep_ <= 1e-5 and ez <= 1e-5
    assert np.all(dz[7] == 0.0)


def test_codes_loss_equals_the_texture_loss_on_fetched_codes(nam, ctx, torch):
    """Codes fetched from a latent pyramid give the texture loss and its parameter gradients."""
    w = wl.training(seed=77, tex=64, channels=16, n=20000, hidden=(64, 64, 64), levels=5)
    m, q = w.material, w.queries
    model = nam.Model.from_workload(ctx, m)
    texels = _dev(torch, np.concatenate([l.reshape(-1, 16) for l in m.levels]))
    params = _dev(torch, m.params)
    dq = [_dev(torch, a) for a in (q.uv, q.lod, q.wi, q.wo, w.targets)]
    loss_t, _, dp_t = model.loss_backward(texels, params, *dq)
    mat = nam.Material.from_workload(ctx, m)
    z = nam.fetch(mat, dq[0], dq[1])
    loss_c, _, dp_c = model.loss_backward_codes(params, z, dq[2], dq[3], dq[4])
    assert abs(loss_c.item() - loss_t.item()) <= 1e-6 * loss_t.item()
    assert _norm_rel(dp_c.cpu().numpy(), dp_t.cpu().numpy()) <= 1e-5
    mat.free()


@pytest.mark.parametrize("A,C,HE,NHE", SHAPES)
@pytest.mark.parametrize("address", [wl.WRAP, wl.CLAMP])
def test_encoder_backward_matches_oracle(nam, ctx, torch, A, C, HE, NHE, address):
    """The encoder's parameter gradient (weight gradients on FP32 matrix-core tiles, the bias as
    a column of ones: a second 16-column tile when A = 16) against the oracle's, for every
    supported shape, both address modes, a ragged batch and a non-finite query."""
    rng = np.random.default_rng(30 + A + C + HE + NHE + 7 * address)
    M, size, n = 5, 32, 5 * 1024 + 33
    attr = _attr_pyramid(rng, size, M, A)
    dims, ep = wl.encoder_params(rng, A, C, [HE] * NHE)
    ep = (ep + 0.05 * rng.standard_normal(ep.size)).astype(np.float32)
    enc = nam.Encoder(ctx, dims, size, size, M, address)
    flat = _dev(torch, np.concatenate([l.reshape(-1, A) for l in attr]))
    q = _queries(rng, n, M)
    q.lod[11] = np.nan
    dz = rng.normal(0, 1e-3, (n, C)).astype(np.float32)
    g = enc.backward(_dev(torch, ep), flat, _dev(torch, q.uv), _dev(torch, q.lod), _dev(torch, dz)).cpu().numpy()
    ref = oracle.encoder_backward(attr, dims, ep, q.uv, q.lod, dz, address)
    e = _norm_rel(g.astype(np.float64), ref)
    _say(f"encoder backward A{A} C{C} H{HE}x{NHE} address {address}: {e:.2e}")
    assert e <= 1e-5
    g2 = enc.backward(_dev(torch, ep), flat, _dev(torch, q.uv), _dev(torch, q.lod), _dev(torch, dz)).cpu().numpy()
    assert np.array_equal(g, g2)                       # fixed-order reduction


def test_encoder_arguments(nam, ctx, torch):
    dims, ep = wl.encoder_params(np.random.default_rng(0), 4, 16, (32, 32))
    flat = _dev(torch, np.zeros((16 * 16 + 64 + 16 + 4 + 1, 4)))
    with pytest.raises(nam.NamError, match="NAM_E_UNSUPPORTED"):
        nam.Encoder(ctx, [5, 32, 16], 16, 16, 5).encode_texels(_dev(torch, np.zeros(5 * 32 + 32 + 32 * 16 + 16)),
                                                             _dev(torch, np.zeros((3, 5))))
    enc = nam.Encoder(ctx, dims, 16, 16, 5)
    enc.pyramid.channels = 8
    with pytest.raises(nam.NamError, match="NAM_E_SHAPE"):
        enc.encode_queries(_dev(torch, ep), flat, _dev(torch, np.zeros((4, 2))), _dev(torch, np.zeros(4)))
    enc = nam.Encoder(ctx, dims, 16, 16, 5)
    assert enc.encode_queries(_dev(torch, ep), flat, _dev(torch, np.zeros((0, 2))), _dev(torch, np.zeros(0))).shape == (0, 16)
    g = enc.backward(_dev(torch, ep), flat, _dev(torch, np.zeros((0, 2))), _dev(torch, np.zeros(0)),
                     _dev(torch, np.zeros((0, 16))))
    assert float(g.abs().max()) == 0.0


def test_two_phase_training(nam, ctx, torch):
    """Sec. 5.1's procedure on the analytic material: 128^2 parameters (albedo, roughness) with 8
    levels, encoder 4-32-32-16, decoder 22-64-64-3, samples from a pool of 2^22, Adam.
    Held-out errors on 65,536 samples: MSE, MSE below the 99th-percentile target (the full MSE
    is dominated by rare specular peaks) and mean relative error.  Asserted, with margins from
    the first measurement (shown in brackets):
      * the end-to-end phase (800 steps, lr 3e-3) lowers the held-out MSE below 0.05 of its
        start [0.0088];
      * the bake carries the end-to-end model into a latent pyramid: its decode's MSE is within
        1.1 of the end-to-end loss [1.00];
      * training that pyramid directly (800 steps, lr 3e-4) lowers the MSE below the 99th
        percentile and the mean relative error by a fifth or more [0.51, 0.60 of the bake];
      * the bake after 800 end-to-end steps beats 800 steps of direct optimisation from N(0, 1)
        texels (same decoder initialisation, lr 3e-3) by 1.3 or more on each metric [2.0, 2.7,
        1.44]: the encoder bootstraps the latent texture (the paper's motivation for it)."""
    tex, M, C, NP = 128, 8, 16, 1 << 22
    w = wl.training(seed=1004, tex=tex, channels=C, n=NP, hidden=(64, 64), levels=M)
    am, m = w.analytic, w.material
    attr = wl.material_parameters(am, tex, M)
    dims_e, ep = wl.encoder_params(wl.rngs(5)[0], 4, C, (32, 32))
    enc = nam.Encoder(ctx, dims_e, tex, tex, M)
    model = nam.Model.from_workload(ctx, m)
    flat = _dev(torch, np.concatenate([l.reshape(-1, 4) for l in attr]))
    eparams, params = _dev(torch, ep), _dev(torch, m.params)
    pool = [_dev(torch, a) for a in (w.queries.uv, w.queries.lod, w.queries.wi, w.queries.wo, w.targets)]
    hq, ht = wl.training_samples(am, wl.rngs(4242)[wl.CHILD_TARGETS], 65536, M)
    held = [_dev(torch, a) for a in (hq.uv, hq.lod, hq.wi, hq.wo, ht)]
    body = torch.from_numpy(ht.max(axis=1) <= np.percentile(ht.max(axis=1), 99.0)).cuda()

    def errors(texels, prm):
        rgb = model.forward(texels, prm, *held[:4])
        se = ((rgb - held[4]) ** 2).mean(dim=1)
        return np.array([float(se.mean()), float(se[body].mean()), float((torch.abs(rgb - held[4]) / held[4]).mean())])

    def codes_loss():
        z = enc.encode_queries(eparams, flat, held[0], held[1])
        return float(model.loss_backward_codes(params, z, held[2], held[3], held[4])[0].item())

    g = torch.Generator(device="cuda")
    g.manual_seed(0)

    def batch():
        idx = torch.randint(0, NP, (65536,), device="cuda", generator=g)
        return [p[idx].contiguous() for p in pool]

    start = codes_loss()
    state = [torch.zeros_like(t) for t in (eparams, eparams, params, params)]
    for step in range(1, 801):
        uv, lod, wi, wo, tgt = batch()
        z = enc.encode_queries(eparams, flat, uv, lod)
        _, dz, dp = model.loss_backward_codes(params, z, wi, wo, tgt)
        de = enc.backward(eparams, flat, uv, lod, dz)
        nam.adam_update(ctx, eparams, state[0], state[1], de, step, lr=3e-3)
        nam.adam_update(ctx, params, state[2], state[3], dp, step, lr=3e-3)
    end1 = codes_loss()
    texels = enc.encode_texels(eparams, flat)
    baked = errors(texels, params)
    fine_tex, fine_par = texels.clone(), params.clone()
    tr = nam.Trainer(model, fine_tex, fine_par, lr=3e-4)
    for _ in range(800):
        tr.step(*batch())
    fine = errors(fine_tex, fine_par)
    rand_tex = _dev(torch, np.concatenate([l.reshape(-1, C) for l in m.levels]))
    rand_par = _dev(torch, m.params)
    tr = nam.Trainer(model, rand_tex, rand_par, lr=3e-3)
    for _ in range(800):
        tr.step(*batch())
    direct = errors(rand_tex, rand_par)
    _say(f"two-phase training: end-to-end loss {start:.5f} -> {end1:.5f}; held-out MSE / MSE below the 99th "
         f"percentile / mean relative error: baked {baked[0]:.5f} / {baked[1]:.5f} / {baked[2]:.4f}, after "
         f"direct training {fine[0]:.5f} / {fine[1]:.5f} / {fine[2]:.4f}, direct from N(0, 1) texels "
         f"{direct[0]:.5f} / {direct[1]:.5f} / {direct[2]:.4f}")
    assert end1 < 0.05 * start
    assert baked[0] < 1.1 * end1
    assert fine[1] < 0.8 * baked[1] and fine[2] < 0.8 * baked[2]
    assert np.all(1.3 * baked < direct)
