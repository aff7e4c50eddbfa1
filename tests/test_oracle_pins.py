"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test targets a mistake the oracle could plausibly contain: a wrong texel-centre
offset, swapped x/y, a dropped level blend, a transposed weight matrix, misplaced biases,
a wrong softplus, a missing ReLU, a wrong sign in a gradient, a wrong Adam bias correction,
a wrong rounding mode.  None of them retypes the oracle's own formula.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import twin
from paper_2305_02678_amd import workloads as wl


def _box_chain(level0, M):
    out = [np.asarray(level0, np.float64)]
    for _ in range(1, M):
        p = out[-1]
        if p.shape[0] > 1:
            p = 0.5 * (p[0::2] + p[1::2])
        if p.shape[1] > 1:
            p = 0.5 * (p[:, 0::2] + p[:, 1::2])
        out.append(p)
    return out


def _rand_levels(rng, w, h, c, M):
    """Independent random levels (not a box chain), so level mix-ups show."""
    return [rng.standard_normal((max(1, h >> l), max(1, w >> l), c)) for l in range(M)]


# ---------------------------------------------------------------------------------- fetch


@pytest.mark.parametrize("address", [oracle.WRAP, oracle.CLAMP])
def test_texel_centres_are_exact(address):
    """At integer lod l and uv on a texel centre of level l, the fetch returns that texel
    bit for bit (every weight is exactly 0 or 1)."""
    rng = np.random.default_rng(1)
    levels = _rand_levels(rng, 16, 8, 5, 4)
    for l, T in enumerate(levels):
        H, W, _ = T.shape
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        uv = np.stack([(xs.ravel() + 0.5) / W, (ys.ravel() + 0.5) / H], 1)
        z = oracle.fetch(levels, uv, np.full(len(uv), float(l)), address)
        assert np.array_equal(z, T.reshape(-1, T.shape[2]))


@pytest.mark.parametrize("address", [oracle.WRAP, oracle.CLAMP])
@pytest.mark.parametrize("shape", [(8, 8, 3, 4), (8, 4, 2, 4), (4, 8, 2, 4), (2, 1, 1, 2), (1, 1, 3, 1), (8, 2, 4, 3)])
def test_fetch_matches_brute_force_tent_sum(address, shape):
    """Against the numpy twin that weighs every texel (and every periodic image) by the
    tent kernel: no shared neighbour-finding logic."""
    w, h, c, M = shape
    rng = np.random.default_rng(hash((address,) + shape) % 2**32)
    levels = _rand_levels(rng, w, h, c, M)
    n = 300
    uv = rng.uniform(-2.3, 3.1, size=(n, 2))
    uv[:40] = rng.random((40, 2))
    lod = rng.uniform(-1.0, M + 0.5, size=n)
    lod[:10] = np.arange(10) % M  # integer levels
    z = oracle.fetch(levels, uv, lod, address)
    zt = twin.fetch(levels, uv, lod, address)
    np.testing.assert_allclose(z, zt, rtol=0, atol=1e-12)


def test_box_level_consistency():
    """With a 2x2 box chain, every lod in [l, l+1] sampled at a level-(l+1) texel centre
    gives that coarse texel: the four level-l taps each weigh 1/4."""
    rng = np.random.default_rng(2)
    levels = _box_chain(rng.standard_normal((16, 16, 4)), 5)
    for l in range(4):
        T = levels[l + 1]
        H, W, _ = T.shape
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        uv = np.stack([(xs.ravel() + 0.5) / W, (ys.ravel() + 0.5) / H], 1)
        for lam in (l, l + 0.25, l + 0.5, l + 0.999):
            z = oracle.fetch(levels, uv, np.full(len(uv), lam))
            np.testing.assert_allclose(z, T.reshape(-1, 4), atol=1e-13)


def test_lod_clamping_top_level_and_linearity_in_t():
    rng = np.random.default_rng(3)
    levels = _box_chain(rng.standard_normal((8, 8, 3)), 4)
    uv = rng.uniform(-1, 2, size=(50, 2))
    z0 = oracle.fetch(levels, uv, np.zeros(50))
    np.testing.assert_array_equal(oracle.fetch(levels, uv, np.full(50, -3.7)), z0)
    ztop = oracle.fetch(levels, uv, np.full(50, 3.0))
    np.testing.assert_array_equal(oracle.fetch(levels, uv, np.full(50, 17.0)), ztop)
    # full chain: the 1x1 top level is the mean of level 0, constant over uv
    np.testing.assert_allclose(ztop, np.broadcast_to(levels[0].mean(axis=(0, 1)), ztop.shape), atol=1e-13)
    # between two levels z is affine in the fractional level
    za = oracle.fetch(levels, uv, np.full(50, 1.0))
    zb = oracle.fetch(levels, uv, np.full(50, 2.0))
    for t in (0.1, 0.5, 0.85):
        np.testing.assert_allclose(oracle.fetch(levels, uv, np.full(50, 1.0 + t)), (1 - t) * za + t * zb, atol=1e-13)


def test_fetch_is_linear_in_texels_and_reproduces_constants():
    rng = np.random.default_rng(4)
    A = _rand_levels(rng, 8, 8, 2, 3)
    B = _rand_levels(rng, 8, 8, 2, 3)
    uv = rng.uniform(-1, 2, size=(64, 2))
    lod = rng.uniform(0, 2, size=64)
    a, b = 0.75, -2.5
    lin = oracle.fetch([a * x + b * y for x, y in zip(A, B)], uv, lod)
    np.testing.assert_allclose(lin, a * oracle.fetch(A, uv, lod) + b * oracle.fetch(B, uv, lod), atol=1e-12)
    const = [np.full_like(x, 3.25) for x in A]
    for address in (oracle.WRAP, oracle.CLAMP):
        np.testing.assert_allclose(oracle.fetch(const, uv, lod, address), 3.25, atol=1e-14)


def test_affine_texture_is_reproduced_in_the_interior_under_clamp():
    """T_l[y][x] = p x + q y + c is reproduced exactly by bilinear interpolation at sample
    position (s, r) = (u W - 1/2, v H - 1/2) away from the edges."""
    W = H = 16
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    p, q, c = 0.3, -1.7, 0.25
    T = (p * xs + q * ys + c)[..., None]
    rng = np.random.default_rng(5)
    uv = rng.uniform(1.0 / W, 1.0 - 1.0 / W, size=(200, 2))
    z = oracle.fetch([T], uv, np.zeros(200), oracle.CLAMP)[:, 0]
    s, r = uv[:, 0] * W - 0.5, uv[:, 1] * H - 0.5
    np.testing.assert_allclose(z, p * s + q * r + c, atol=1e-12)


def test_x_maps_to_u_and_y_to_v():
    """A texture that varies only along x responds only to u (row-major [y][x], x <-> u)."""
    T = np.zeros((4, 4, 1))
    T[:, 2, 0] = 1.0
    z = oracle.fetch([T], [[(2 + 0.5) / 4, 0.1]], [0.0])
    assert z[0, 0] == 1.0
    z = oracle.fetch([T], [[0.1, (2 + 0.5) / 4]], [0.0])
    assert z[0, 0] != 1.0


def test_tap_indices_cover_every_weighted_texel():
    rng = np.random.default_rng(6)
    levels = _rand_levels(rng, 8, 4, 1, 3)
    sizes = [l.shape[0] * l.shape[1] for l in levels]
    base = np.concatenate([[0], np.cumsum(sizes)])
    uv = rng.uniform(-1, 2, size=(100, 2))
    lod = rng.uniform(-0.5, 2.5, size=100)
    t = oracle.taps(levels, uv, lod)
    assert t.min() >= 0 and t.max() < base[-1]
    for i in range(100):
        # an impulse at each texel: nonzero fetch <=> texel among the taps
        for l in range(3):
            H, W, _ = levels[l].shape
            for idx in range(H * W):
                imp = [np.zeros_like(x) for x in levels]
                imp[l].reshape(-1)[idx] = 1.0
                if twin.fetch(imp, uv[i:i + 1], lod[i:i + 1])[0, 0] != 0.0:
                    assert base[l] + idx in t[i]
        if i > 10:
            break


# -------------------------------------------------------------------------------- decoder


def _pack(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def _tiny_material(C=8, M=3, seed=7):
    rng = np.random.default_rng(seed)
    return _box_chain(rng.standard_normal((16, 16, C)), M), rng


def _softplus(q):
    return np.log1p(np.exp(q))


def test_zero_weights_give_softplus_of_output_bias():
    levels, rng = _tiny_material()
    dims = [14, 32, 32, 3]
    bK = np.array([0.0, 1.0, -1.0])
    layers = [(np.zeros((32, 14)), np.zeros(32)), (np.zeros((32, 32)), np.zeros(32)), (np.zeros((3, 32)), bK)]
    q = wl.uniform_queries(rng, 20, 0, 2)
    rgb = oracle.decode(levels, dims, _pack(layers), q.uv, q.lod, q.wi, q.wo)
    np.testing.assert_allclose(rgb[0], [math.log(2.0), math.log1p(math.e), math.log1p(math.exp(-1.0))], rtol=1e-15)
    assert abs(rgb[0, 0] - 0.6931471805599453) < 1e-16


@pytest.mark.parametrize("offset", [0, 8, 11])   # z channels, wi, wo
def test_identity_network_passes_selected_inputs_through(offset):
    """W_1 = [I; 0], hidden W = I, W_K selects 3 inputs: rgb = softplus(relu(x_sel)).  The
    offset selects latent channels 0-2 (C = 8), wi (8..10) or wo (11..13), which fixes the
    concatenation order [z, wi, wo]."""
    levels, rng = _tiny_material()
    dims = [14, 32, 32, 3]
    W1 = np.zeros((32, 14)); W1[:14, :14] = np.eye(14)
    W2 = np.eye(32)
    W3 = np.zeros((3, 32)); W3[np.arange(3), offset + np.arange(3)] = 1.0
    layers = [(W1, np.zeros(32)), (W2, np.zeros(32)), (W3, np.zeros(3))]
    q = wl.uniform_queries(rng, 64, 0, 2)
    q.wi[:, :2] *= -1.0 * (rng.random((64, 1)) < 0.5)   # some negative direction components
    rgb = oracle.decode(levels, dims, _pack(layers), q.uv, q.lod, q.wi, q.wo)
    x = np.concatenate([oracle.fetch(levels, q.uv, q.lod), q.wi.astype(np.float64), q.wo.astype(np.float64)], 1)
    np.testing.assert_allclose(rgb, _softplus(np.maximum(0.0, x[:, offset:offset + 3])), rtol=1e-14, atol=1e-15)


def test_permutation_network_fixes_weight_orientation():
    """W_1 a non-symmetric permutation: neuron o reads input perm[o].  Reading W_1 transposed
    would route a different input to the output."""
    levels, rng = _tiny_material()
    dims = [14, 16, 3]
    perm = np.array([5, 0, 13, 2, 9, 1, 7, 12, 3, 11, 4, 6, 8, 10])
    W1 = np.zeros((16, 14)); W1[np.arange(14), perm] = 1.0
    W2 = np.zeros((3, 16)); W2[0, 0] = W2[1, 2] = W2[2, 4] = 1.0
    layers = [(W1, np.full(16, 5.0)), (W2, np.zeros(3))]  # bias 5 keeps ReLU linear
    q = wl.uniform_queries(rng, 32, 0, 2)
    rgb = oracle.decode(levels, dims, _pack(layers), q.uv, q.lod, q.wi, q.wo)
    x = np.concatenate([oracle.fetch(levels, q.uv, q.lod), q.wi.astype(np.float64), q.wo.astype(np.float64)], 1)
    np.testing.assert_allclose(rgb, _softplus(x[:, perm[[0, 2, 4]]] + 5.0), rtol=1e-14)


def test_constant_weight_network_closed_form():
    """W_k = w_k everywhere, b_k = beta_k: all units of a layer are equal, so
    h_1 = relu(w_1 sum(x) + beta_1), h_k = relu(w_k d_{k-1} h_{k-1} + beta_k)."""
    levels, rng = _tiny_material(C=16)
    dims = [22, 64, 64, 64, 3]
    w = [0.05, -0.03, 0.04, 0.02]
    beta = [0.1, 0.6, -0.2, -0.4]
    layers = [(np.full((dims[k + 1], dims[k]), w[k]), np.full(dims[k + 1], beta[k])) for k in range(4)]
    q = wl.uniform_queries(rng, 200, 0, 2)
    rgb = oracle.decode(levels, dims, _pack(layers), q.uv, q.lod, q.wi, q.wo)
    x = np.concatenate([oracle.fetch(levels, q.uv, q.lod), q.wi.astype(np.float64), q.wo.astype(np.float64)], 1)
    h = np.maximum(0.0, w[0] * x.sum(1) + beta[0])
    for k in (1, 2):
        h = np.maximum(0.0, w[k] * dims[k] * h + beta[k])
    out = w[3] * 64 * h + beta[3]
    assert (h == 0).any() and (h > 0).any()        # both ReLU branches exercised
    np.testing.assert_allclose(rgb, np.repeat(_softplus(out)[:, None], 3, 1), rtol=1e-13)


def test_softplus_identities_on_output():
    """softplus(q) - softplus(-q) = q and softplus(q) -> q for large q; exercised through
    the decoder with W_K = 0 and chosen output biases."""
    levels, rng = _tiny_material()
    dims = [14, 8, 3]
    q = wl.uniform_queries(rng, 1, 0, 2)
    for b in (0.3, 7.0, 40.0):
        lay_p = [(np.zeros((8, 14)), np.zeros(8)), (np.zeros((3, 8)), np.array([b, -b, 0.0]))]
        r = oracle.decode(levels, dims, _pack(lay_p), q.uv, q.lod, q.wi, q.wo)[0]
        assert abs((r[0] - r[1]) - b) < 1e-13
    lay = [(np.zeros((8, 14)), np.zeros(8)), (np.zeros((3, 8)), np.array([-745.0 + 1, 60.0, -30.0]))]
    r = oracle.decode(levels, dims, _pack(lay), q.uv, q.lod, q.wi, q.wo)[0]
    assert r[1] == 60.0 + math.exp(-60.0) or abs(r[1] - 60.0) < 1e-14
    assert abs(r[2] / math.exp(-30.0) - 1) < 1e-12


def test_decode_rejects_bad_dims():
    levels, rng = _tiny_material()
    q = wl.uniform_queries(rng, 4, 0, 2)
    with pytest.raises(ValueError):
        oracle.decode(levels, [13, 3], np.zeros(13 * 3 + 3), q.uv, q.lod, q.wi, q.wo)


# ------------------------------------------------------------------------------ gradients


def _fd_problem(seed=8, n=256):
    rng = np.random.default_rng(seed)
    C, M = 8, 5
    levels = _box_chain(rng.standard_normal((16, 16, C)), M)
    dims = [14, 32, 32, 3]
    params = wl.xavier_mlp(rng, dims).astype(np.float64)
    params[[i for i in range(params.size)]] += 0.05 * rng.standard_normal(params.size)  # nonzero biases
    q = wl.uniform_queries(rng, n, 0, M - 1)
    q.lod[: n // 8] = rng.uniform(-1, 0, n // 8)          # magnification
    q.lod[n // 8: n // 4] = M - 1                          # top level, t = 0
    q.uv[: n // 4] += rng.integers(-2, 3, size=(n // 4, 2))  # wrap images
    tgt = rng.uniform(0.1, 2.0, size=(n, 3))
    return levels, dims, params, q, tgt


def _loss(levels, dims, params, q, tgt):
    rgb = oracle.decode(levels, dims, params, q.uv, q.lod, q.wi, q.wo)
    return np.mean((rgb - tgt) ** 2)


def test_analytic_gradients_match_central_differences():
    levels, dims, params, q, tgt = _fd_problem()
    L, dP, dL = oracle.loss_grad(levels, dims, params, q.uv, q.lod, q.wi, q.wo, tgt)
    assert abs(L - _loss(levels, dims, params, q, tgt)) < 1e-14
    rng = np.random.default_rng(9)
    checked = 0
    for j in rng.choice(params.size, 160, replace=False):
        h = 1e-6 * max(1.0, abs(params[j]))
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        fd = (_loss(levels, dims, pp, q, tgt) - _loss(levels, dims, pm, q, tgt)) / (2 * h)
        # FD truncation ~h^2, cancellation ~ eps * L / h ~ 1e-10: relative 1e-6 plus a 2e-9 floor
        assert abs(fd - dP[j]) <= 1e-6 * abs(dP[j]) + 2e-9, (j, fd, dP[j])
        checked += 1
    for l in range(len(levels)):
        flat = levels[l].reshape(-1)
        for j in rng.choice(flat.size, min(flat.size, 40), replace=False):
            lp = [x.copy() for x in levels]
            lm = [x.copy() for x in levels]
            lp[l].reshape(-1)[j] += 1e-6
            lm[l].reshape(-1)[j] -= 1e-6
            fd = (_loss(lp, dims, params, q, tgt) - _loss(lm, dims, params, q, tgt)) / 2e-6
            g = dL[l].reshape(-1)[j]
            assert abs(fd - g) <= 1e-6 * abs(g) + 2e-9, (l, j, fd, g)
            checked += 1
    assert checked > 300


def _plant_non_finite(q):
    """Samples 3, 17, 40 and 41 get a NaN or infinite position or level (R13: skipped)."""
    q.uv[3, 0] = np.nan
    q.uv[17, 1] = -np.inf
    q.lod[40] = np.nan
    q.lod[41] = np.inf
    return np.array([3, 17, 40, 41])


def test_non_finite_samples_closed_form_with_zero_weights():
    """Zero weights make every output softplus(b_K), whatever the latent code, so the loss and
    the output-bias gradient have closed forms: L = (1/3n) sum over finite samples of
    (softplus(b) - t)^2, dL/db = (2/3n) sum over finite samples of (softplus(b) - t) logistic(b).
    A NaN sample that is not skipped makes both NaN; dividing by the finite count instead of
    the whole batch scales them by n / n_finite."""
    levels, rng = _tiny_material()
    dims = [14, 32, 32, 3]
    bK = np.array([0.3, -0.7, 1.1])
    layers = [(np.zeros((32, 14)), 0.1 * np.ones(32)), (np.zeros((32, 32)), np.zeros(32)),
              (np.zeros((3, 32)), bK)]
    params = _pack(layers)
    n = 64
    q = wl.uniform_queries(rng, n, 0, 2)
    bad = _plant_non_finite(q)
    tgt = rng.uniform(0.1, 2.0, size=(n, 3))
    L, dP, dL = oracle.loss_grad(levels, dims, params, q.uv, q.lod, q.wi, q.wo, tgt)
    keep = np.ones(n, bool)
    keep[bad] = False
    sp = np.log1p(np.exp(bK))
    sig = 1.0 / (1.0 + np.exp(-bK))
    L_ref = ((sp[None, :] - tgt[keep]) ** 2).sum() / (3 * n)
    db_ref = 2.0 * (sp[None, :] - tgt[keep]).sum(axis=0) * sig / (3 * n)
    assert abs(L - L_ref) <= 1e-14 * L_ref
    np.testing.assert_allclose(dP[-3:], db_ref, rtol=1e-13, atol=0)
    assert np.isfinite(dP).all()
    for g in dL:
        assert np.all(g == 0.0)      # W_1 = 0: no gradient reaches the code


def test_gradients_with_non_finite_samples_match_central_differences():
    """The loss with non-finite samples is (1/3n) times the squared error summed over the finite
    samples, each output taken from the decode; its central differences pin the analytic
    gradients of a batch that holds non-finite samples (n stays the denominator)."""
    levels, dims, params, q, tgt = _fd_problem(seed=12, n=128)
    _plant_non_finite(q)

    def loss(lv, pr):
        rgb = oracle.decode(lv, dims, pr, q.uv, q.lod, q.wi, q.wo)
        keep = np.isfinite(rgb).all(axis=1)
        return ((rgb[keep] - tgt[keep]) ** 2).sum() / (3 * len(q.lod))

    L, dP, dL = oracle.loss_grad(levels, dims, params, q.uv, q.lod, q.wi, q.wo, tgt)
    assert np.isfinite(L) and abs(L - loss(levels, params)) < 1e-14
    assert np.isfinite(dP).all() and all(np.isfinite(g).all() for g in dL)
    rng = np.random.default_rng(13)
    for j in rng.choice(params.size, 60, replace=False):
        h = 1e-6 * max(1.0, abs(params[j]))
        pp, pm = params.copy(), params.copy()
        pp[j] += h
        pm[j] -= h
        fd = (loss(levels, pp) - loss(levels, pm)) / (2 * h)
        assert abs(fd - dP[j]) <= 1e-6 * abs(dP[j]) + 2e-9, (j, fd, dP[j])
    for l in range(len(levels)):
        flat = levels[l].reshape(-1)
        for j in rng.choice(flat.size, min(flat.size, 12), replace=False):
            lp = [x.copy() for x in levels]
            lm = [x.copy() for x in levels]
            lp[l].reshape(-1)[j] += 1e-6
            lm[l].reshape(-1)[j] -= 1e-6
            fd = (loss(lp, params) - loss(lm, params)) / 2e-6
            g = dL[l].reshape(-1)[j]
            assert abs(fd - g) <= 1e-6 * abs(g) + 2e-9, (l, j, fd, g)


def test_latent_gradient_of_a_linear_probe_is_the_tap_weight():
    """With a network whose output q_0 = z_0 exactly (identity path, large positive bias
    so ReLU is linear), dq_0/dT[texel] is the trilinear weight of that texel; checked against
    the brute-force tent weights of the twin."""
    rng = np.random.default_rng(10)
    C, M = 2, 3
    levels = [rng.standard_normal((max(1, 8 >> l), max(1, 8 >> l), C)) for l in range(M)]
    dims = [8, 8, 3]
    W1 = np.zeros((8, 8)); W1[0, 0] = 1.0
    W2 = np.zeros((3, 8)); W2[0, 0] = 1.0
    params = _pack([(W1, np.full(8, 50.0)), (W2, np.array([-50.0, 0.0, 0.0]))])
    q = wl.uniform_queries(rng, 1, 0, M - 1)
    q.lod[:] = 0.6
    rgb, qq = oracle.decode(levels, dims, params, q.uv, q.lod, q.wi, q.wo, return_q=True)
    # choose the target so that dL/dq_0 = 1: L = (rgb0 - tgt)^2/3 -> dL/drgb0 = 2(rgb0 - tgt)/3
    sig = 1.0 / (1.0 + math.exp(-qq[0, 0]))
    tgt = rgb.copy()
    tgt[0, 0] = rgb[0, 0] - 1.5 / sig
    _, _, dL = oracle.loss_grad(levels, dims, params, q.uv, q.lod, q.wi, q.wo, tgt)
    for l in range(M):
        H, W, _ = levels[l].shape
        for idx in range(H * W):
            imp = [np.zeros_like(x) for x in levels]
            imp[l].reshape(-1, C)[idx, 0] = 1.0
            wgt = twin.fetch(imp, q.uv, q.lod)[0, 0]
            assert abs(dL[l].reshape(-1, C)[idx, 0] - wgt) < 1e-12
            assert dL[l].reshape(-1, C)[idx, 1] == 0.0


# ----------------------------------------------------------------------------------- Adam


def test_adam_first_step_is_signed_learning_rate():
    rng = np.random.default_rng(11)
    g = rng.standard_normal(1000)
    g[::10] = 0.0
    p0 = rng.standard_normal(1000)
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    oracle.adam(p, m, v, g, lr=1e-3, step=1)
    expect = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p, expect, rtol=0, atol=1e-15)
    assert np.array_equal(p[::10], p0[::10])


def test_adam_matches_torch_optim_over_several_steps():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    p0 = rng.standard_normal(257)
    grads = [rng.standard_normal(257) for _ in range(7)]
    t = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(257), np.zeros(257)
    for k, g in enumerate(grads, start=1):
        t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        oracle.adam(p, m, v, g, lr=3e-3, step=k)
    np.testing.assert_allclose(p, t.detach().numpy(), rtol=0, atol=1e-14)


# ------------------------------------------------------------------------------- rounding


def test_fp16_rounding_matches_ieee_half():
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-9, 6, 20000),
                        [0.0, -0.0, 65504.0, 65519.9, 65520.0, 1e6, -1e6, 2.0 ** -24, 2.0 ** -25,
                         3 * 2.0 ** -26, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11]])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(oracle.round_fp16(x), ref)


def _e4m3_table():
    """All finite OCP E4M3FN values from the bit layout: sign, 4 exponent bits (bias 7),
    3 fraction bits; exponent field 0 is subnormal; S.1111.111 is NaN."""
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue
            v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
            vals.append((v, m))
    return vals


def test_e4m3_rounding_is_nearest_even_and_saturating():
    table = _e4m3_table()
    vals = np.array([v for v, _ in table])
    assert vals.max() == 448.0 and sorted(vals)[1] == 2.0 ** -9
    rng = np.random.default_rng(14)
    x = np.concatenate([rng.uniform(0, 500, 3000), 2.0 ** rng.uniform(-12, 9, 3000),
                        (vals[1:] + vals[:-1]) / 2])  # every midpoint between neighbours
    got = oracle.round_e4m3(x)
    gotn = oracle.round_e4m3(-x)
    for xi, g, gn in zip(x, got, gotn):
        d = np.abs(vals - min(xi, 448.0))
        best = np.flatnonzero(d == d.min())
        if len(best) == 2:   # tie: the code with even fraction bits
            best = [b for b in best if table[b][1] % 2 == 0]
        assert g == vals[best[0]], (xi, g)
        assert gn == -g
    assert oracle.round_e4m3(np.array([1e9]))[0] == 448.0


def test_quantised_decode_without_rounding_equals_decode():
    levels, rng = _tiny_material(C=16)
    dims = [22, 64, 64, 64, 3]
    params = wl.xavier_mlp(rng, dims).astype(np.float64)
    params += 0.01 * rng.standard_normal(params.size)
    q = wl.uniform_queries(rng, 64, 0, 2)
    ref = oracle.decode(levels, dims, params, q.uv, q.lod, q.wi, q.wo)
    # unit scales, no rounding
    got = oracle.decode_quant(levels, dims, params, np.ones(4), np.ones(4), [oracle.FMT_NONE] * 4,
                              q.uv, q.lod, q.wi, q.wo)
    np.testing.assert_allclose(got, ref, rtol=1e-13)
    # power-of-two scales are exact and change nothing without rounding
    sw = np.array([4.0, 8.0, 0.5, 2.0])
    qp = []
    for k, (W, b) in enumerate(wl.unpack_params(params, dims)):
        qp += [W.reshape(-1) * sw[k], b]
    got = oracle.decode_quant(levels, dims, np.concatenate(qp), sw, np.array([2.0, 0.25, 1.0, 16.0]),
                              [oracle.FMT_NONE] * 4, q.uv, q.lod, q.wi, q.wo)
    np.testing.assert_allclose(got, ref, rtol=1e-13)


def _f16_levels(rng, w, h, c, M, scale=1.0):
    return [np.asarray(lv * scale, np.float16).astype(np.float64) for lv in _rand_levels(rng, w, h, c, M)]


@pytest.mark.parametrize("address", [oracle.WRAP, oracle.CLAMP])
def test_fp16_filter_within_the_rounding_error_bound(address):
    """The FP16 filter (8 products summed in FP16, weights rounded to FP16) stays inside the
    textbook bound of recursive summation: with u = 2^-11 the unit roundoff of FP16 and
    g_n = n u / (1 - n u), |z16 - z| <= (u (1 + g_8) + g_8) sum_k |w_k T_k|, where z is the exact
    trilinear code of the same FP16 texels; a dropped or misplaced tap breaks it by orders of
    magnitude.  Every z16 is an FP16 value, and the sum is really kept in FP16: it differs from
    the exact code rounded once to FP16 for a visible fraction of the channels."""
    rng = np.random.default_rng(160)
    levels = _f16_levels(rng, 32, 16, 8, 5, scale=3.0)
    q = wl.uniform_queries(rng, 4000, -0.5, 4.5)
    q.uv[:500] += rng.integers(-3, 4, (500, 2))
    z = oracle.fetch(levels, q.uv, q.lod, address)
    z16 = oracle.fetch_fp16(levels, q.uv, q.lod, address)
    u = 2.0 ** -11
    g8 = 8 * u / (1 - 8 * u)
    taps = oracle.taps(levels, q.uv, q.lod, address)
    flat = np.concatenate([lv.reshape(-1, lv.shape[2]) for lv in levels])
    # sum_k |w_k| |T_k| with the weights recovered from the tent sum (brute force) is bounded by
    # max_k |T_k| since the weights are non-negative and sum to 1
    bound = (u * (1 + g8) + g8) * np.abs(flat[taps]).max(axis=1)
    assert np.all(np.abs(z16 - z) <= bound + 1e-300)
    assert np.all(np.asarray(z16, np.float16).astype(np.float64) == z16)
    single = np.asarray(z, np.float16).astype(np.float64)
    frac = np.mean(z16 != single)
    assert 0.02 < frac < 0.9, frac


def test_fp16_filter_exact_at_texel_centres_and_single_tap_weights():
    """At a texel centre of an integer level the weights are 1 and 0, so the FP16 filter returns
    the FP16 texel itself; with the level weight t in (0, 1) at texel centres of both levels the
    code is fp16(fp16(1 - t) T_l0 + ...) computed by hand for one channel."""
    rng = np.random.default_rng(161)
    levels = _f16_levels(rng, 16, 16, 8, 5)
    for l in range(5):
        W = 16 >> l
        xs, ys = np.meshgrid(np.arange(W), np.arange(W))
        uv = np.stack([(xs.ravel() + 0.5) / W, (ys.ravel() + 0.5) / W], 1)
        z16 = oracle.fetch_fp16(levels, uv, np.full(len(uv), float(l)))
        np.testing.assert_array_equal(z16, levels[l][ys.ravel(), xs.ravel()])
    # lod 3.25 at (0.25, 0.25), the centre of texel (0, 0) of the 2x2 level 3: its taps weigh
    # 0.75, 0, 0, 0; on the 1x1 level 4 the stencil position is -1/4 on both axes, fraction 3/4,
    # so all four taps land on the one texel with weights 0.25 * (1/16, 3/16, 3/16, 9/16)
    z16 = oracle.fetch_fp16(levels, np.array([[0.25, 0.25]]), np.array([3.25]))[0]
    a, b = levels[3][0, 0], levels[4][0, 0]
    h = lambda x: float(np.float16(x))
    want = []
    for c in range(8):
        acc = h(0.75 * a[c])
        for k in range(3):
            acc = h(0.0 + acc)                  # the three zero-weight taps of level 3
        for wk in (1 / 64, 3 / 64, 3 / 64, 9 / 64):
            acc = h(wk * b[c] + acc)            # exact products, one rounding per step
        want.append(acc)
    np.testing.assert_array_equal(z16, want)


def test_quantised_decode_with_fp16_filter_uses_it():
    """decode_quant(blend_fp16=True) feeds the FP16-filtered code to the network: with the
    identity-routing network of P8 and no rounding elsewhere, rgb_c = softplus(max(0, z16_c))."""
    rng = np.random.default_rng(162)
    levels = _f16_levels(rng, 16, 16, 8, 5)
    C, H = 8, 32
    dims = [C + 6, H, H, 3]
    W1 = np.zeros((H, C + 6)); W1[:C + 6, :C + 6] = np.eye(C + 6)
    W2 = np.eye(H)
    W3 = np.zeros((3, H)); W3[:, :3] = np.eye(3)
    params = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(3)])
    q = wl.uniform_queries(rng, 300, 0, 4)
    got = oracle.decode_quant(levels, dims, params, np.ones(3), np.ones(3), [oracle.FMT_NONE] * 3,
                              q.uv, q.lod, q.wi, q.wo, blend_fp16=True)
    z16 = oracle.fetch_fp16(levels, q.uv, q.lod)
    np.testing.assert_allclose(got, np.logaddexp(0.0, np.maximum(z16[:, :3], 0.0)), rtol=1e-14)
    exact = oracle.decode_quant(levels, dims, params, np.ones(3), np.ones(3), [oracle.FMT_NONE] * 3,
                                q.uv, q.lod, q.wi, q.wo)
    assert np.any(got != exact)


def test_non_finite_queries_decode_to_nan():
    levels, rng = _tiny_material()
    dims = [14, 32, 32, 3]
    params = wl.xavier_mlp(rng, dims)
    q = wl.uniform_queries(rng, 4, 0, 2)
    q.uv[1, 0] = np.nan
    q.lod[2] = np.inf
    rgb = oracle.decode(levels, dims, params, q.uv, q.lod, q.wi, q.wo)
    assert np.isnan(rgb[1:3]).all() and np.isfinite(rgb[[0, 3]]).all()


# ------------------------------------------------- Russian-roulette level choice (Sec. 4.1)


def _rr_problem(seed=31, n=400, C=8, M=4):
    levels, rng = _tiny_material(C=C, M=M, seed=seed)
    dims = [C + 6, 32, 32, 3]
    params = wl.xavier_mlp(rng, dims)
    q = wl.uniform_queries(rng, n, -0.7, M - 0.3)      # levels below 0 and above the top too
    q.lod[: n // 10] = np.round(q.lod[: n // 10])       # integer levels: t = 0
    q.lod = q.lod.astype(np.float32)
    return levels, dims, params, q, M


def _levels_and_t(lod, M):
    lam = np.clip(lod.astype(np.float64), 0.0, M - 1.0)
    l0 = np.floor(lam)
    return l0, np.minimum(l0 + 1, M - 1), lam - l0


@pytest.mark.parametrize("address", [wl.WRAP, wl.CLAMP])
def test_rr_extreme_draws_pick_one_level(address):
    """A draw of 1 never goes below t, so every query takes the finer level: the decode at the
    integer level l0 (where the trilinear filter is the bilinear one); a draw of 0 takes the
    coarser level wherever t > 0."""
    levels, dims, params, q, M = _rr_problem()
    l0, l1, t = _levels_and_t(q.lod, M)
    ones, zeros = np.ones(len(q)), np.zeros(len(q))
    got0 = oracle.decode_rr(levels, dims, params, q.uv, q.lod, ones, q.wi, q.wo, address)
    ref0 = oracle.decode(levels, dims, params, q.uv, l0, q.wi, q.wo, address)
    np.testing.assert_allclose(got0, ref0, rtol=1e-13, atol=0)
    got1 = oracle.decode_rr(levels, dims, params, q.uv, q.lod, zeros, q.wi, q.wo, address)
    ref1 = oracle.decode(levels, dims, params, q.uv, np.where(t > 0, l1, l0), q.wi, q.wo, address)
    np.testing.assert_allclose(got1, ref1, rtol=1e-13, atol=0)
    assert (t > 0).sum() > 100 and (t == 0).sum() >= 40


def test_rr_expectation_is_the_level_mixture_not_the_trilinear_decode():
    """Over a stratified grid of K draws the mean decode is (1 - t) g(z_l0) + t g(z_l1) up to
    the grid's resolution (the share of draws below t is within 1 / (2K) of t); it is not the
    decode of the trilinear code."""
    levels, dims, params, q, M = _rr_problem(n=300)
    l0, l1, t = _levels_and_t(q.lod, M)
    K = 64
    mean = np.zeros((len(q), 3))
    for k in range(K):
        mean += oracle.decode_rr(levels, dims, params, q.uv, q.lod, np.full(len(q), (k + 0.5) / K), q.wi, q.wo)
    mean /= K
    g0 = oracle.decode(levels, dims, params, q.uv, l0, q.wi, q.wo)
    g1 = oracle.decode(levels, dims, params, q.uv, l1, q.wi, q.wo)
    mix = (1 - t)[:, None] * g0 + t[:, None] * g1
    bound = np.abs(g1 - g0) / (2 * K) + 1e-12
    assert (np.abs(mean - mix) <= bound).all()
    tri = oracle.decode(levels, dims, params, q.uv, q.lod, q.wi, q.wo)
    assert (np.abs(tri - mix) > 10 * bound).sum() > 50      # the network is not linear in z


def test_rr_non_finite_queries_and_draws():
    levels, dims, params, q, M = _rr_problem(n=8)
    q.uv[1, 0] = np.nan
    q.lod[2] = -np.inf
    xi = np.full(len(q), 0.5)
    xi[5] = np.nan                                        # a NaN draw takes the finer level
    rgb = oracle.decode_rr(levels, dims, params, q.uv, q.lod, xi, q.wi, q.wo)
    assert np.isnan(rgb[1:3]).all() and np.isfinite(rgb[[0, 3, 4, 5, 6, 7]]).all()
    l0, _, _ = _levels_and_t(q.lod[5:6], M)
    np.testing.assert_allclose(rgb[5], oracle.decode(levels, dims, params, q.uv[5:6], l0, q.wi[5:6], q.wo[5:6])[0],
                               rtol=1e-13)
