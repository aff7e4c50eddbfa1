"""nam_loss_backward_noalloc (the variant that allocates nothing, for callers under graph
capture or otherwise unable to allocate) against nam_loss_backward and the FP64 oracle.

Two calls in a row on the same GPU, the second with a smaller batch, so the second runs on a
region that still holds the first call's partial sums.  The first batch is large enough that
the static region holds fewer per-wave slices than the ordinary call uses (the decoder
22-64-64-64-3 has 9,987 parameters: 32 MiB holds 838 slices, the ordinary call uses one per
wave of the grid).

Bars (as for the other training tests): loss within 1e-5 relative; gradients per tensor
||g - g_ref|| / ||g_ref|| <= 1e-3 and element-wise |g - g_ref| <= 1e-3 max(|g_ref|, 1e-3 max|g_ref|)
against the oracle; against nam_loss_backward the same element-wise bound, and a norm-relative
difference <= 1e-5 for the parameter gradients (fixed-order sums, grouped differently) and
<= 1e-4 for the texel gradients (float atomics, whose order differs between any two calls;
6.6e-6 measured at 200,000 samples on a 128 x 128 pyramid).
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


def _say(*a):
    print(*a, flush=True)


def problem(seed, n, tex=128, C=16, hidden=(64, 64, 64)):
    r = wl.rngs(seed)
    M = wl.full_chain(tex, tex)
    mat = wl.make_material(r[0], r[1], tex, tex, C, M, list(hidden))
    mat.params = (mat.params + 0.05 * r[1].standard_normal(mat.params.size)).astype(np.float32)
    q = wl.uniform_queries(r[2], n, 0.0, M - 1.0)
    q.uv[: n // 8] += r[2].integers(-2, 3, (n // 8, 2)).astype(np.float32)
    tgt = wl.make_analytic_material(r[3]).brdf(q.uv, q.wi, q.wo).astype(np.float32)
    return mat, q, tgt


def close(g, ref, name, norm_bound=1e-3):
    g, ref = np.asarray(g, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    norm_rel = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    bound = 1e-3 * np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    bad = np.abs(g - ref) > bound
    _say(f"{name}: norm-relative {norm_rel:.2e}, element-wise violations {bad.sum()} of {g.size}")
    assert norm_rel <= norm_bound, name
    assert not bad.any(), (name, np.flatnonzero(bad)[:5])


def run_both(nam, torch, ctx, mat, q, tgt):
    model = nam.Model.from_workload(ctx, mat)
    tex = torch.from_numpy(np.ascontiguousarray(nam.concat_levels(mat.levels), np.float32)).cuda()
    par = torch.from_numpy(np.ascontiguousarray(mat.params, np.float32)).cuda()
    tg = torch.from_numpy(np.ascontiguousarray(tgt, np.float32)).cuda()
    dq = nam.to_device(q)
    # outputs allocated ahead, so the no-allocation call itself allocates nothing
    d_tex_f = torch.zeros_like(tex)
    d_par_f = torch.empty_like(par)
    loss_f = torch.empty(1, dtype=torch.float32, device=tex.device)
    torch.cuda.synchronize()
    _say(f"noalloc call: n={len(q)}, {mat.width}x{mat.height}x{mat.channels}, dims {mat.dims}")
    model.loss_backward(tex, par, *dq, tg, d_texels=d_tex_f, d_params=d_par_f, loss=loss_f, noalloc=True)
    torch.cuda.synchronize()
    loss, d_tex, d_par = model.loss_backward(tex, par, *dq, tg)
    torch.cuda.synchronize()
    return (loss_f.item(), d_tex_f.cpu().numpy(), d_par_f.cpu().numpy()), (loss.item(), d_tex.cpu().numpy(),
                                                                         d_par.cpu().numpy())


def test_noalloc_matches_loss_backward_twice(nam, torch):
    ctx = nam.Context(0)
    for call, (seed, n) in enumerate(((71, 200_000), (72, 3_000))):
        mat, q, tgt = problem(seed, n)
        (lf, tf, pf), (l0, t0, p0) = run_both(nam, torch, ctx, mat, q, tgt)
        _say(f"call {call}: loss {lf:.8g} (noalloc) vs {l0:.8g}")
        assert abs(lf - l0) <= 1e-5 * abs(l0)
        close(pf, p0, f"call {call} params vs nam_loss_backward", 1e-5)
        close(tf, t0, f"call {call} texels vs nam_loss_backward", 1e-4)
        if n <= 10_000:
            L, dP, dL = oracle.loss_grad(mat.levels, mat.dims, mat.params, q.uv, q.lod, q.wi, q.wo, tgt)
            assert abs(lf - L) <= 1e-5 * L
            close(pf, dP, f"call {call} params vs oracle")
            close(tf, nam.concat_levels(dL), f"call {call} texels vs oracle")


def test_noalloc_vector_kernel_and_edges(nam, torch):
    """A decoder shape outside the matrix-core kernel (one hidden layer of 16) runs the vector
    kernel from the same region; n = 0 gives zero gradients and loss; deterministic mode is
    refused with NAM_E_UNSUPPORTED."""
    ctx = nam.Context(0)
    mat, q, tgt = problem(73, 5_000, tex=32, C=8, hidden=(16,))
    (lf, tf, pf), (l0, t0, p0) = run_both(nam, torch, ctx, mat, q, tgt)
    assert abs(lf - l0) <= 1e-5 * abs(l0)
    close(pf, p0, "vector kernel params vs nam_loss_backward", 1e-5)
    close(tf, t0, "vector kernel texels vs nam_loss_backward", 1e-4)
    L, dP, dL = oracle.loss_grad(mat.levels, mat.dims, mat.params, q.uv, q.lod, q.wi, q.wo, tgt)
    close(pf, dP, "vector kernel params vs oracle")

    model = nam.Model.from_workload(ctx, mat)
    tex = torch.from_numpy(np.ascontiguousarray(nam.concat_levels(mat.levels), np.float32)).cuda()
    par = torch.from_numpy(np.ascontiguousarray(mat.params, np.float32)).cuda()
    e = [torch.zeros((0, k), dtype=torch.float32, device="cuda") for k in (2, 3, 3, 3)]
    lod0 = torch.zeros(0, dtype=torch.float32, device="cuda")
    d_par = torch.full_like(par, 7.0)
    loss = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    model.loss_backward(tex, par, e[0], lod0, e[1], e[2], e[3], d_params=d_par, loss=loss, noalloc=True)
    torch.cuda.synchronize()
    assert float(d_par.abs().max()) == 0.0 and loss.item() == 0.0

    nam.check(nam.lib().nam_set_deterministic(ctx.handle, 1))
    dq = nam.to_device(q)
    tg = torch.from_numpy(np.ascontiguousarray(tgt, np.float32)).cuda()
    with pytest.raises(nam.NamError) as ei:
        model.loss_backward(tex, par, *dq, tg, noalloc=True)
    assert ei.value.status == nam.NAM_E_UNSUPPORTED
    nam.check(nam.lib().nam_set_deterministic(ctx.handle, 0))
