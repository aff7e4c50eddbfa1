"""Pins of the oracle's decoder with the extra albedo output (Sec. 6.4 "Albedo inference": the
decoder gives a second RGB triplet, the directional albedo of Eq. albedo, fitted with an L2 loss
against one-sample estimates, Sec. 5.2 "Optimization").

The 6-output decoder is pinned by closed forms (zero weights, an identity network that routes
six chosen inputs to the six outputs), by its relation to two 3-output decoders that are pinned
on their own (the outputs do not interact: rows 0-2 and rows 3-5 of the last layer are two
separate RGB decoders over the same hidden layers), by the loss of a decoder whose albedo rows
repeat its RGB rows (exactly twice the RGB loss, gradients exactly twice), and by central
differences of the summed loss.

Targets: only three outputs written or passed through softplus, a wrong output stride, the
albedo rows read from the RGB rows, the albedo term left out of the loss or weighted
differently, the target stride of the loss wrong.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2305_02678_amd import workloads as wl


def _pack(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def _unpack(params, dims):
    return [(W.astype(np.float64), b.astype(np.float64)) for W, b in wl.unpack_params(params, dims)]


def _box_chain(level0, M):
    out = [level0]
    for _ in range(1, M):
        a = out[-1]
        out.append(0.25 * (a[0::2, 0::2] + a[1::2, 0::2] + a[0::2, 1::2] + a[1::2, 1::2]))
    return out


def _material(C=8, M=4, seed=21):
    rng = np.random.default_rng(seed)
    return _box_chain(rng.standard_normal((16, 16, C)), M), rng


def _softplus(q):
    return np.log1p(np.exp(q))


def test_zero_weights_give_softplus_of_all_six_biases():
    levels, rng = _material()
    dims = [14, 32, 6]
    bK = np.array([0.0, 1.0, -1.0, 2.5, -3.0, 0.25])
    p = _pack([(np.zeros((32, 14)), np.zeros(32)), (np.zeros((6, 32)), bK)])
    q = wl.uniform_queries(rng, 9, 0, 3)
    out = oracle.decode(levels, dims, p, q.uv, q.lod, q.wi, q.wo)
    assert out.shape == (9, 6)
    np.testing.assert_allclose(out, np.tile([math.log1p(math.exp(b)) for b in bK], (9, 1)), rtol=1e-15)
    assert abs(out[0, 0] - 0.6931471805599453) < 1e-16


def test_identity_network_routes_six_inputs_to_six_outputs():
    """W_1 = [I; 0], W_K picks inputs sel[0..5] (latent channels, wi and wo mixed, out of
    order): out_c = softplus(relu(x[sel[c]]))."""
    levels, rng = _material()
    dims = [14, 32, 32, 6]
    sel = np.array([7, 2, 9, 13, 0, 11])
    W1 = np.zeros((32, 14)); W1[:14, :14] = np.eye(14)
    W3 = np.zeros((6, 32)); W3[np.arange(6), sel] = 1.0
    p = _pack([(W1, np.zeros(32)), (np.eye(32), np.zeros(32)), (W3, np.zeros(6))])
    q = wl.uniform_queries(rng, 80, 0, 3)
    q.wo[:, :2] *= -1.0
    out = oracle.decode(levels, dims, p, q.uv, q.lod, q.wi, q.wo)
    x = np.concatenate([oracle.fetch(levels, q.uv, q.lod), q.wi.astype(np.float64), q.wo.astype(np.float64)], 1)
    np.testing.assert_allclose(out, _softplus(np.maximum(0.0, x[:, sel])), rtol=1e-14, atol=1e-15)


def _split(params, dims):
    """The two 3-output decoders hidden in a 6-output one: same hidden layers, last layer rows
    0-2 (RGB) and rows 3-5 (albedo)."""
    lay = _unpack(params, dims)
    W, b = lay[-1]
    d3 = list(dims[:-1]) + [3]
    return d3, _pack(lay[:-1] + [(W[:3], b[:3])]), _pack(lay[:-1] + [(W[3:], b[3:])])


@pytest.mark.parametrize("mode", ["trilinear", "roulette", "frames", "quant"])
def test_outputs_are_two_independent_rgb_decoders(mode):
    levels, rng = _material(C=8, M=4)
    C = 8
    nf = 2 if mode == "frames" else 0
    dims = [C + 6 * max(nf, 1), 32, 32, 6]
    params = wl.xavier_mlp(rng, dims).astype(np.float64)
    params += 0.1 * rng.standard_normal(params.size)
    q = wl.uniform_queries(rng, 300, -0.5, 3.5)
    d3, p_rgb, p_alb = _split(params, dims)
    if mode == "trilinear":
        f = lambda d, p: oracle.decode(levels, d, p, q.uv, q.lod, q.wi, q.wo)
    elif mode == "roulette":
        xi = rng.random(300)
        f = lambda d, p: oracle.decode_rr(levels, d, p, q.uv, q.lod, xi, q.wi, q.wo)
    elif mode == "frames":
        fp = rng.standard_normal(6 * nf * C + 6 * nf)
        f = lambda d, p: oracle.decode_frames(levels, d, p, nf, fp, q.uv, q.lod, q.wi, q.wo)
    else:
        K = len(dims) - 1
        f = lambda d, p: oracle.decode_quant(levels, d, oracle.round_fp16(p), np.ones(K), np.ones(K), [0] * K,
                                             q.uv, q.lod, q.wi, q.wo)
    out = f(dims, params)
    assert out.shape == (300, 6)
    np.testing.assert_array_equal(out[:, :3], f(d3, p_rgb))
    np.testing.assert_array_equal(out[:, 3:], f(d3, p_alb))
    assert np.abs(out[:, :3] - out[:, 3:]).min() > 0     # the two heads differ everywhere


def test_repeated_rows_double_the_rgb_loss_and_gradients():
    """Albedo rows equal to the RGB rows and albedo targets equal to the RGB targets: the loss
    of the 6-output decoder is twice that of the 3-output one, and so is every gradient (the
    output layer's rows 3-5 get the gradient of rows 0-2)."""
    levels, rng = _material(C=8, M=5)
    d3 = [14, 32, 32, 3]
    p3 = wl.xavier_mlp(rng, d3).astype(np.float64) + 0.05 * rng.standard_normal(wl.n_params(d3))
    lay = _unpack(p3, d3)
    W, b = lay[-1]
    d6 = [14, 32, 32, 6]
    p6 = _pack(lay[:-1] + [(np.concatenate([W, W]), np.concatenate([b, b]))])
    q = wl.uniform_queries(rng, 256, 0, 4)
    t3 = rng.uniform(0.1, 2.0, (256, 3))
    L3, g3, dl3 = oracle.loss_grad(levels, d3, p3, q.uv, q.lod, q.wi, q.wo, t3)
    L6, g6, dl6 = oracle.loss_grad(levels, d6, p6, q.uv, q.lod, q.wi, q.wo, np.concatenate([t3, t3], 1))
    assert abs(L6 - 2.0 * L3) <= 1e-15 * L3
    hid = sum(d3[k] * d3[k + 1] + d3[k + 1] for k in range(len(d3) - 2))
    np.testing.assert_allclose(g6[:hid], 2.0 * g3[:hid], rtol=1e-12, atol=1e-18)
    g6_out = _unpack(g6, d6)[-1]
    g3_out = _unpack(g3, d3)[-1]
    for half in (slice(0, 3), slice(3, 6)):
        np.testing.assert_allclose(g6_out[0][half], g3_out[0], rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(g6_out[1][half], g3_out[1], rtol=1e-12, atol=1e-18)
    for a, c in zip(dl6, dl3):
        np.testing.assert_allclose(a, 2.0 * c, rtol=1e-12, atol=1e-18)


def test_albedo_loss_gradients_match_central_differences():
    """L = mean over 3n of (rgb - t_rgb)^2 + mean over 3n of (albedo - t_albedo)^2."""
    levels, rng = _material(C=8, M=5, seed=23)
    dims = [14, 32, 32, 6]
    params = wl.xavier_mlp(rng, dims).astype(np.float64) + 0.05 * rng.standard_normal(wl.n_params(dims))
    n = 200
    q = wl.uniform_queries(rng, n, -0.5, 4.5)
    q.uv[: n // 4] += rng.integers(-2, 3, size=(n // 4, 2))
    tgt = rng.uniform(0.1, 2.0, (n, 6))

    def loss(lv, p):
        y = oracle.decode(lv, dims, p, q.uv, q.lod, q.wi, q.wo)
        return np.mean((y[:, :3] - tgt[:, :3]) ** 2) + np.mean((y[:, 3:] - tgt[:, 3:]) ** 2)

    L, dP, dL = oracle.loss_grad(levels, dims, params, q.uv, q.lod, q.wi, q.wo, tgt)
    assert abs(L - loss(levels, params)) < 1e-14
    out_rows = slice(params.size - (32 * 6 + 6), params.size)
    picks = np.concatenate([rng.choice(params.size - 198, 60, replace=False), np.arange(params.size)[out_rows][::4]])
    for j in picks:
        h = 1e-6 * max(1.0, abs(params[j]))
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        fd = (loss(levels, pp) - loss(levels, pm)) / (2 * h)
        assert abs(fd - dP[j]) <= 1e-6 * abs(dP[j]) + 2e-9, (j, fd, dP[j])
    for l in (0, 2, 4):
        flat = levels[l].reshape(-1)
        for j in rng.choice(flat.size, min(flat.size, 12), replace=False):
            lp = [x.copy() for x in levels]
            lm = [x.copy() for x in levels]
            lp[l].reshape(-1)[j] += 1e-6
            lm[l].reshape(-1)[j] -= 1e-6
            fd = (loss(lp, params) - loss(lm, params)) / 2e-6
            g = dL[l].reshape(-1)[j]
            assert abs(fd - g) <= 1e-6 * abs(g) + 2e-9, (l, j, fd, g)


def test_other_output_widths_are_rejected():
    levels, rng = _material()
    q = wl.uniform_queries(rng, 4, 0, 2)
    for ko in (4, 9):
        with pytest.raises(ValueError):
            oracle.decode(levels, [14, ko], np.zeros(14 * ko + ko), q.uv, q.lod, q.wi, q.wo)
