"""Parity at the benchmarked sizes, with the launches bench.py times.

The training step of bench.py's training leg (1,048,576 samples, latent 1024^2 x 16 with 11
levels, decoder 22-64-64-64-3, MSE; Sec. 5 with the latents trained directly) and the encoder's
first training phase of its encoder leg (the same samples, a 1024^2 x 4 parameter pyramid,
encoder 4-32-32-16; Sec. 5.1) against the FP64 oracle over the whole batch: the oracle computes
the loss and every gradient of 2^20 samples in a few seconds on the host's cores.

Tolerances as in test_gpu_train.py: gradients within 1e-3 norm-relative and element-wise within
1e-3 of max(|g_ref|, 1e-3 max|g_ref|); the loss within 1e-5 relative; codes within 1e-5 of
max(1, |z_ref|) (test_gpu_encoder.py). Inputs that the tests choose (codes, their gradients) come from a seeded
generator, never from the GPU.

ReLU kinks. Among 2^20 samples x 192 hidden neurons some pre-activations lie within FP32 rounding
of zero; there the GPU (FP32) and the oracle (FP64) may take different sides of the ReLU, and the
whole backward pass of that sample differs (both are correct roundings of the method). A sample
is ambiguous when a hidden pre-activation a satisfies |a| <= 2^-16 (|W| |x| + |b|) for its layer
(an FP32 dot product of at most 64 terms, with inputs carried in FP32, errs by far less). The
per-sample outputs of ambiguous samples (their code gradients, and the texels their taps touch)
are left out of the element-wise bound and counted; the norm bound covers everything.
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


@pytest.fixture(scope="module")
def batch():
    return wl.training()


def _say(*a):
    print(*a, flush=True)


def _dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrs]


def _grad_close(g, ref, name, keep=None):
    """keep: rows (first axis) held to the element-wise bound (default all)."""
    g, ref = np.asarray(g, np.float64), np.asarray(ref, np.float64)
    norm_rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    bound = 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    bad = np.abs(g - ref) > bound
    if keep is not None:
        bad &= keep.reshape((-1,) + (1,) * (bad.ndim - 1))
    bad, g = bad.ravel(), g.ravel()
    _say(f"{name}: norm-relative error {norm_rel:.2e}, element-wise violations {bad.sum()} of {g.size}")
    assert norm_rel <= 1e-3, name
    assert not bad.any(), (name, np.flatnonzero(bad)[:5])
    return norm_rel


def _ambiguous(dims, params, x0, chunk=1 << 16):
    """Samples (rows of the decoder input x0) with a hidden pre-activation within 2^-16 of its
    accumulated magnitude, from an FP64 forward pass of the packed decoder."""
    params = np.asarray(params, np.float64)
    layers, o = [], 0
    for k in range(len(dims) - 2):                      # hidden layers only
        fi, fo = dims[k], dims[k + 1]
        layers.append((params[o:o + fi * fo].reshape(fo, fi), params[o + fi * fo:o + fi * fo + fo]))
        o += fi * fo + fo
    out = np.zeros(x0.shape[0], bool)
    for a in range(0, x0.shape[0], chunk):
        x = np.asarray(x0[a:a + chunk], np.float64)
        flag = np.zeros(x.shape[0], bool)
        for W, b in layers:
            pre = x @ W.T + b
            mag = np.abs(x) @ np.abs(W).T + np.abs(b)
            flag |= (np.abs(pre) <= 2.0 ** -16 * mag).any(1)
            x = np.maximum(pre, 0.0)
        out[a:a + chunk] = flag
    return out


@pytest.mark.parametrize("deterministic", [False, True])
def test_training_gradients_at_full_size(nam, ctx, torch, batch, deterministic):
    """Loss and the gradients of the decoder and of all 22.4 M texel channels for the 2^20-sample
    batch of the training step, against the oracle's exact gradients of the same batch; with
    float atomics and in the deterministic mode (fixed-point scatter)."""
    m, q = batch.material, batch.queries
    model = nam.Model.from_workload(ctx, m)
    tex, par = _dev(torch, nam.concat_levels(m.levels), m.params)
    dq = _dev(torch, q.uv, q.lod, q.wi, q.wo, batch.targets)
    ctx.set_deterministic(deterministic)
    try:
        loss, d_tex, d_par = model.loss_backward(tex, par, *dq)
    finally:
        ctx.set_deterministic(False)
    L, dP, dL = oracle.loss_grad([l.astype(np.float64) for l in m.levels], m.dims, m.params, q.uv, q.lod,
                                 q.wi, q.wo, batch.targets)
    _say(f"training at full size ({len(q)} samples, {oracle.threads()} oracle threads): "
         f"loss {loss.item():.8f} vs {L:.8f}")
    assert abs(loss.item() - L) <= 1e-5 * L
    _grad_close(d_par.cpu().numpy(), dP, "decoder parameters")
    lv64 = [l.astype(np.float64) for l in m.levels]
    amb = _ambiguous(m.dims, m.params, np.concatenate([oracle.fetch(lv64, q.uv, q.lod), q.wi, q.wo], 1))
    skip = np.zeros(nam.concat_levels(dL).shape[0], bool)
    skip[oracle.taps(lv64, q.uv[amb], q.lod[amb]).ravel()] = True
    _say(f"{amb.sum()} samples at a ReLU kink; {skip.sum()} of {skip.size} texels they touch left out of the "
         "element-wise bound")
    _grad_close(d_tex.cpu().numpy(), nam.concat_levels(dL), "texels", keep=~skip)


def test_encoder_phase_at_full_size(nam, ctx, torch, batch):
    """The encoder leg's three calls on the 2^20-sample batch: query codes (sampled queries), the
    decoder's loss and gradients on given codes, and the encoder's gradient for given code
    gradients, each against the oracle."""
    m, q, am = batch.material, batch.queries, batch.analytic
    n = len(q)
    attr = wl.material_parameters(am, m.width, m.n_levels)
    dims_e, ep = wl.encoder_params(wl.rngs(5)[0], 4, m.channels, (32, 32))
    ep = ep.astype(np.float32)
    enc = nam.Encoder(ctx, dims_e, m.width, m.height, m.n_levels)
    model = nam.Model.from_workload(ctx, m)
    flat, dep, par = _dev(torch, np.concatenate([l.reshape(-1, 4) for l in attr]), ep, m.params)
    uv, lod, wi, wo, tgt = _dev(torch, q.uv, q.lod, q.wi, q.wo, batch.targets)
    rng = np.random.default_rng(2305)

    # query codes, on 20,000 sampled queries
    z = enc.encode_queries(dep, flat, uv, lod).cpu().numpy().astype(np.float64)
    idx = np.sort(rng.choice(n, 20000, replace=False))
    zr = oracle.encode_queries(attr, dims_e, ep, q.uv[idx], q.lod[idx])
    ez = (np.abs(z[idx] - zr) / np.maximum(1.0, np.abs(zr))).max()       # the measure of test_gpu_encoder.py
    _say(f"encoder codes at full size: max relative error {ez:.2e} on {idx.size} sampled queries")
    assert ez <= 1e-5

    # the decoder's loss and gradients on given codes, over the whole batch
    zc = rng.normal(0.0, 1.0, (n, m.channels)).astype(np.float32)
    loss, dz, dp = model.loss_backward_codes(par, *_dev(torch, zc), wi, wo, tgt)
    L, dP, dZ = oracle.loss_grad_codes(m.dims, m.params, zc, q.wi, q.wo, batch.targets)
    _say(f"codes loss at full size: {loss.item():.8f} vs {L:.8f}")
    assert abs(loss.item() - L) <= 1e-5 * L
    _grad_close(dp.cpu().numpy(), dP, "decoder parameters on given codes")
    amb = _ambiguous(m.dims, m.params, np.concatenate([zc, q.wi, q.wo], 1))
    _say(f"{amb.sum()} samples at a ReLU kink: their code gradients left out of the element-wise bound")
    _grad_close(dz.cpu().numpy(), dZ, "code gradients", keep=~amb)

    # the encoder's gradient for given code gradients, over the whole batch.  The given gradients
    # have a mean (a loss's gradients are systematically signed; zero-mean ones would cancel to
    # about 1/1000 of their terms over 2^20 samples, below what an FP32 sum resolves), and are
    # zero for samples at a kink of the encoder's ReLUs, so that both sides see the same terms
    gz = rng.normal(1e-3, 1e-3, (n, m.channels)).astype(np.float32)
    amb_e = _ambiguous(dims_e, ep, oracle.fetch(attr, q.uv, q.lod))
    gz[amb_e] = 0.0
    _say(f"{amb_e.sum()} samples at a kink of the encoder: no code gradient given")
    ge = enc.backward(dep, flat, uv, lod, *_dev(torch, gz)).cpu().numpy()
    ref = oracle.encoder_backward(attr, dims_e, ep, q.uv, q.lod, gz)
    _grad_close(ge, ref, "encoder parameters")


def test_framed_training_gradients_at_full_size(nam, ctx, torch, batch):
    """The training leg's decoder with two learned shading frames (28-64-64-64-3, Sec. 4.2; the
    vector training kernel, each workgroup over many 64-sample chunks) on the 2^20-sample batch:
    loss and the gradients of the frame layer, the decoder and the texels against the oracle."""
    m, q = batch.material, batch.queries
    r = wl.rngs(77)
    dims = [m.channels + 12] + list(m.dims[1:])
    dec = wl.xavier_mlp(r[1], dims).astype(np.float32)
    F = wl.frame_layer(r[1], 2, m.channels).astype(np.float32)
    model = nam.Model(ctx, m.width, m.height, m.channels, m.n_levels, dims, m.address, n_frames=2)
    tex, par = _dev(torch, nam.concat_levels(m.levels), np.concatenate([F, dec]))
    dq = _dev(torch, q.uv, q.lod, q.wi, q.wo, batch.targets)
    loss, d_tex, d_par = model.loss_backward(tex, par, *dq)
    lv64 = [l.astype(np.float64) for l in m.levels]
    L, dP, dF, dL = oracle.loss_grad_frames(lv64, dims, dec, F, 2, q.uv, q.lod, q.wi, q.wo, batch.targets)
    _say(f"framed training at full size: loss {loss.item():.8f} vs {L:.8f}")
    assert abs(loss.item() - L) <= 1e-5 * L
    g = d_par.cpu().numpy()
    nfp = model.frame_param_count
    _grad_close(g[:nfp], dF, "frame layer")
    _grad_close(g[nfp:], dP, "decoder parameters")
    z = oracle.fetch(lv64, q.uv, q.lod)
    amb = _ambiguous(dims, dec, np.concatenate([z, oracle.frames(2, F, z, q.wi, q.wo)], 1))
    skip = np.zeros(nam.concat_levels(dL).shape[0], bool)
    skip[oracle.taps(lv64, q.uv[amb], q.lod[amb]).ravel()] = True
    _say(f"{amb.sum()} samples at a ReLU kink; {skip.sum()} of {skip.size} texels they touch left out of the "
         "element-wise bound")
    _grad_close(d_tex.cpu().numpy(), nam.concat_levels(dL), "texels", keep=~skip)
