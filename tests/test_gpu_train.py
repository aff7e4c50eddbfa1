"""Differentiation on the GPU against the FP64 oracle and against finite differences.

Tolerances:
  * forward: max relative RGB error <= 1e-5 (FP32);
  * gradients vs the oracle's analytic gradients: per tensor ||g - g_ref|| / ||g_ref|| <= 1e-3,
    and element-wise |g - g_ref| <= 1e-3 * max(|g_ref|, 1e-3 * max|g_ref|);
  * gradients vs central finite differences of the FP64 loss: the same element-wise bound,
    coordinates within h of a ReLU kink skipped (counted);
  * Adam: relative 1e-5 against the FP64 update.
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


def fd_problem(seed=21, n=256, C=8, hidden=(32, 32), tex=16, nonzero_bias=True):
    """16x16 x 8 texture, full chain of 5 levels, MLP 14-32-32-3 (the finite-difference case)."""
    r = wl.rngs(seed)
    M = wl.full_chain(tex, tex)
    mat = wl.make_material(r[0], r[1], tex, tex, C, M, list(hidden))
    if nonzero_bias:
        mat.params = (mat.params + 0.1 * r[1].standard_normal(mat.params.size)).astype(np.float32)
    q = wl.uniform_queries(r[2], n, 0.0, M - 1.0)
    q.lod[: n // 8] = -0.5
    q.lod[n // 8: n // 4] = M - 1
    q.uv[: n // 4] += r[2].integers(-2, 3, (n // 4, 2)).astype(np.float32)
    am = wl.make_analytic_material(r[3])
    tgt = am.brdf(q.uv, q.wi, q.wo).astype(np.float32)
    return mat, q, tgt


def to_dev(torch, *arrs):
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrs]


def grad_close(g, ref, name):
    g, ref = np.asarray(g, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    norm_rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    scale = np.abs(ref).max()
    bound = 1e-3 * np.maximum(np.abs(ref), 1e-3 * scale)
    bad = np.abs(g - ref) > bound
    _say(f"{name}: norm-relative error {norm_rel:.2e}, element-wise violations {bad.sum()} of {g.size}")
    assert norm_rel <= 1e-3, name
    assert not bad.any(), (name, np.flatnonzero(bad)[:5])


def test_forward_matches_oracle(nam, ctx, torch):
    w = wl.tiny()
    m, q = w.material, w.queries
    model = nam.Model.from_workload(ctx, m)
    tex, par = to_dev(torch, nam.concat_levels(m.levels), m.params)
    rgb = model.forward(tex, par, *nam.to_device(q)).cpu().numpy()
    ref = oracle.decode(m.levels, m.dims, m.params, q.uv, q.lod, q.wi, q.wo)
    assert (np.abs(rgb - ref) / ref).max() <= 1e-5


@pytest.mark.parametrize("shape", [(8, (32, 32)), (16, (64, 64, 64)), (8, (16,)), (16, (32, 32, 32, 32))])
def test_loss_gradients_match_oracle(nam, ctx, torch, shape):
    C, hidden = shape
    mat, q, tgt = fd_problem(C=C, hidden=hidden, n=1000)
    model = nam.Model.from_workload(ctx, mat)
    tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
    loss, d_tex, d_par = model.loss_backward(tex, par, *nam.to_device(q), tg)
    L, dP, dL = oracle.loss_grad(mat.levels, mat.dims, mat.params, q.uv, q.lod, q.wi, q.wo, tgt)
    assert abs(loss.item() - L) <= 1e-5 * L
    grad_close(d_par.cpu().numpy(), dP, f"params {shape}")
    grad_close(d_tex.cpu().numpy(), nam.concat_levels(dL), f"texels {shape}")


def test_vjp_equals_loss_gradient(nam, ctx, torch):
    """nam_backward with d_rgb = 2 (rgb - target) / (3n) gives the loss gradient."""
    mat, q, tgt = fd_problem(n=777)
    model = nam.Model.from_workload(ctx, mat)
    tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
    dq = nam.to_device(q)
    rgb = model.forward(tex, par, *dq)
    d_rgb = (2.0 * (rgb - tg) / (3 * len(q))).contiguous()
    d_tex, d_par = model.backward(tex, par, *dq, d_rgb)
    _, d_tex2, d_par2 = model.loss_backward(tex, par, *dq, tg)
    np.testing.assert_allclose(d_par.cpu().numpy(), d_par2.cpu().numpy(), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(d_tex.cpu().numpy(), d_tex2.cpu().numpy(), rtol=1e-4, atol=1e-9)


def test_gradients_match_finite_differences(nam, ctx, torch):
    """GPU gradients against central differences of the FP64 loss (h = 1e-6 max(1, |p|))."""
    mat, q, tgt = fd_problem(n=256)
    model = nam.Model.from_workload(ctx, mat)
    tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
    _, d_tex, d_par = model.loss_backward(tex, par, *nam.to_device(q), tg)
    g_par, g_tex = d_par.cpu().numpy().astype(np.float64), d_tex.cpu().numpy().astype(np.float64)
    levels64 = [l.astype(np.float64) for l in mat.levels]
    P = mat.params.astype(np.float64)

    def loss(levels, params):
        rgb = oracle.decode(levels, mat.dims, params, q.uv, q.lod, q.wi, q.wo)
        return np.mean((rgb - tgt) ** 2)

    rng = np.random.default_rng(5)
    gscale = np.abs(g_par).max()
    checked = skipped = 0
    for j in rng.choice(P.size, 120, replace=False):
        h = 1e-6 * max(1.0, abs(P[j]))
        pp, pm = P.copy(), P.copy()
        pp[j] += h
        pm[j] -= h
        fd = (loss(levels64, pp) - loss(levels64, pm)) / (2 * h)
        fd2 = (loss(levels64, P + np.eye(1, P.size, j)[0] * 2 * h) - loss(levels64, P - np.eye(1, P.size, j)[0] * 2 * h)) / (4 * h)
        if abs(fd - fd2) > 1e-6 * max(abs(fd), 1e-9):     # a ReLU kink inside [p - 2h, p + 2h]
            skipped += 1
            continue
        assert abs(g_par[j] - fd) <= 1e-3 * max(abs(fd), 1e-3 * gscale) + 1e-9, (j, g_par[j], fd)
        checked += 1
    flat = nam.concat_levels(levels64).astype(np.float64)
    tscale = np.abs(g_tex).max()
    for j in rng.choice(flat.size, 120, replace=False):
        fp, fm = flat.copy(), flat.copy()
        fp.ravel()[j] += 1e-6
        fm.ravel()[j] -= 1e-6
        lp = nam.split_levels(fp, 16, 16, len(levels64))
        lm = nam.split_levels(fm, 16, 16, len(levels64))
        fd = (loss(lp, P) - loss(lm, P)) / 2e-6
        assert abs(g_tex.ravel()[j] - fd) <= 1e-3 * max(abs(fd), 1e-3 * tscale) + 1e-9, (j, g_tex.ravel()[j], fd)
        checked += 1
    _say(f"finite differences: {checked} coordinates checked, {skipped} skipped at ReLU kinks")
    assert checked >= 200


def test_adam_matches_oracle(nam, ctx, torch):
    rng = np.random.default_rng(9)
    n = 100003
    p0 = rng.standard_normal(n).astype(np.float32)
    p, m, v = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    tp, tm, tv = to_dev(torch, p0, np.zeros(n), np.zeros(n))
    for step in range(1, 5):
        g = rng.standard_normal(n).astype(np.float32)
        g[::7] = 0.0
        (tg,) = to_dev(torch, g)
        nam.adam_update(ctx, tp, tm, tv, tg, step, lr=1e-3)
        oracle.adam(p, m, v, g.astype(np.float64), lr=1e-3, step=step)
    np.testing.assert_allclose(tp.cpu().numpy(), p, rtol=1e-6, atol=1e-7)
    # m is a cancelling FP32 recurrence: absolute error ~1e-8 on values of order 0.1
    np.testing.assert_allclose(tm.cpu().numpy(), m, rtol=1e-5, atol=1e-7)


def test_train_step_is_loss_backward_then_adam(nam, ctx, torch):
    mat, q, tgt = fd_problem(n=3000)
    model = nam.Model.from_workload(ctx, mat)
    tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
    dq = nam.to_device(q)
    tex2, par2 = tex.clone(), par.clone()
    tr = nam.Trainer(model, tex, par, lr=1e-2)
    l1 = tr.step(*dq, tg).item()
    # by hand: gradients, then Adam step 1 on both tensors
    loss, d_tex, d_par = model.loss_backward(tex2, par2, *dq, tg)
    for p_, g_ in ((tex2, d_tex), (par2, d_par)):
        nam.adam_update(ctx, p_, torch.zeros_like(p_), torch.zeros_like(p_), g_, 1, lr=1e-2)
    assert abs(l1 - loss.item()) <= 1e-6 * loss.item()
    np.testing.assert_allclose(par.cpu().numpy(), par2.cpu().numpy(), rtol=0, atol=1e-6)
    np.testing.assert_allclose(tex.cpu().numpy(), tex2.cpu().numpy(), rtol=0, atol=1e-6)
    losses = [l1] + [tr.step(*dq, tg).item() for _ in range(30)]
    _say(f"train step losses: {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]


def test_autograd_function(nam, ctx, torch):
    mat, q, tgt = fd_problem(n=500)
    model = nam.Model.from_workload(ctx, mat)
    tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
    tex.requires_grad_(True)
    par.requires_grad_(True)
    dq = nam.to_device(q)
    rgb = nam.neural_material(tex, par, *dq, model)
    loss = ((rgb - tg) ** 2).mean()
    loss.backward()
    _, d_tex, d_par = model.loss_backward(tex.detach(), par.detach(), *dq, tg)
    np.testing.assert_allclose(par.grad.cpu().numpy(), d_par.cpu().numpy(), rtol=1e-4, atol=1e-8)
    np.testing.assert_allclose(tex.grad.cpu().numpy(), d_tex.cpu().numpy(), rtol=1e-4, atol=1e-8)


def test_non_finite_samples_contribute_nothing(nam, ctx, torch):
    """Samples with a NaN or infinite uv or lod are skipped by the loss and its gradients, with
    the whole batch (3n) as the denominator, on the GPU as in the oracle."""
    mat, q, tgt = fd_problem(n=300)
    model = nam.Model.from_workload(ctx, mat)
    tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
    q2 = wl.Queries(q.uv.copy(), q.lod.copy(), q.wi, q.wo)
    q2.uv[5] = [np.nan, 0.2]
    q2.uv[77] = [0.4, -np.inf]
    q2.lod[9] = np.inf
    q2.lod[200] = np.nan
    loss, d_tex, d_par = model.loss_backward(tex, par, *nam.to_device(q2), tg)
    assert np.isfinite(d_tex.cpu().numpy()).all() and np.isfinite(d_par.cpu().numpy()).all()
    L, dP, dL = oracle.loss_grad(mat.levels, mat.dims, mat.params, q2.uv, q2.lod, q2.wi, q2.wo, tgt)
    assert abs(loss.item() - L) <= 1e-5 * L
    grad_close(d_par.cpu().numpy(), dP, "params with non-finite samples")
    grad_close(d_tex.cpu().numpy(), nam.concat_levels(dL), "texels with non-finite samples")
    rgb = model.forward(tex, par, *nam.to_device(q2)).cpu().numpy()
    assert np.isnan(rgb[[5, 9, 77, 200]]).all()


def test_deterministic_mode_matches_oracle_and_repeats_bitwise(nam, torch):
    """Deterministic mode: latent gradients within the oracle tolerance and equal bit for bit
    over repeated calls, parameter gradients and loss bit for bit those of the default mode
    (the mode changes only the latent scatter), with non-finite samples present; then a dense
    case (20,000 samples on a 16x16 pyramid, so every coarse texel receives thousands of
    contributions) against the default mode's float atomics."""
    ctx = nam.Context(0)
    ctx_default = nam.Context(0)
    ctx.set_deterministic(True)
    for C, hidden, n in ((8, (32, 32), 1000), (16, (64, 64, 64), 1000), (16, (64, 64, 64), 20000)):
        mat, q, tgt = fd_problem(C=C, hidden=hidden, n=n)
        q.uv[7] = [np.nan, 0.1]
        q.lod[11] = np.inf
        model = nam.Model.from_workload(ctx, mat)
        model_default = nam.Model.from_workload(ctx_default, mat)
        tex, par, tg = to_dev(torch, nam.concat_levels(mat.levels), mat.params, tgt)
        dq = nam.to_device(q)
        runs = [model.loss_backward(tex, par, *dq, tg) for _ in range(3)]
        loss, d_tex, d_par = runs[0]
        for l2, t2, p2 in runs[1:]:
            assert torch.equal(t2, d_tex) and torch.equal(p2, d_par) and torch.equal(l2, loss)
        ref_loss, ref_tex, ref_par = model_default.loss_backward(tex, par, *dq, tg)
        assert torch.equal(ref_par, d_par) and torch.equal(ref_loss, loss)
        if n <= 1000:
            L, dP, dL = oracle.loss_grad(mat.levels, mat.dims, mat.params, q.uv, q.lod, q.wi, q.wo, tgt)
            assert abs(loss.item() - L) <= 1e-5 * L
            grad_close(d_par.cpu().numpy(), dP, f"deterministic params C={C}")
            grad_close(d_tex.cpu().numpy(), nam.concat_levels(dL), f"deterministic texels C={C}")
        else:
            grad_close(d_tex.cpu().numpy(), ref_tex.cpu().numpy(), f"deterministic vs atomic texels, n={n}")
        # the vector-Jacobian product in deterministic mode adds into d_texels like the default
        rgb = model.forward(tex, par, *dq)
        d_rgb = torch.nan_to_num(2.0 * (rgb - tg) / (3 * len(q))).contiguous()
        base = torch.full_like(tex, 0.25)
        d_tex2, d_par2 = model.backward(tex, par, *dq, d_rgb, d_texels=base.clone())
        np.testing.assert_allclose(d_tex2.cpu().numpy() - 0.25, d_tex.cpu().numpy(), rtol=0, atol=1e-7)


def test_deterministic_training_run_repeats_bitwise(nam, torch):
    """Two 40-step training runs from the same initial state in deterministic mode end with
    bitwise equal texels, decoder and loss."""
    ctx = nam.Context(0)
    ctx.set_deterministic(True)
    w = wl.training(seed=1004, tex=64, channels=16, n=1 << 15, hidden=(64, 64, 64))
    m = w.material
    model = nam.Model.from_workload(ctx, m)
    ends = []
    for _ in range(2):
        tex, par = to_dev(torch, nam.concat_levels(m.levels), m.params)
        tr = nam.Trainer(model, tex, par, lr=3e-3)
        dq = nam.to_device(w.queries)
        (tg,) = to_dev(torch, w.targets)
        for _ in range(40):
            loss = tr.step(*dq, tg)
        ends.append((tex.clone(), par.clone(), loss.clone()))
    assert torch.equal(ends[0][0], ends[1][0]) and torch.equal(ends[0][1], ends[1][1])
    assert torch.equal(ends[0][2], ends[1][2])
