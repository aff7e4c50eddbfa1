"""The importance-sampling decoder and its analytic proxy (Sec. 4.3; App. A) through the C ABI,
against the FP64 oracle (orc_sampler_params, orc_proxy_pdf, orc_proxy_sample) on the same
inputs.

Tolerances (FP32 kernels against FP64): the proxy parameters within 1e-5 relative (a few FP32
roundings through at most five layers and smooth activations).  PDFs are compared where they
exceed 1e-3 within 1e-4 + 16 u kappa relative (u = 2^-24; 1e-7 absolute below), with kappa the
PDF's first-order condition at that query: the sum over its 15 inputs of |d log pdf / d x|
times the size of an FP32 rounding of x in units of u (1 for a component of a unit direction,
|x| for a proxy parameter), from central differences of the FP64 oracle.  The PDF's
sensitivity has several sources: the 1 / |wo . h| of the reflection Jacobian, the
normalisation of wi + wo near wo = -wi, the inverse of App. A's M (whose norm is
1 / sigma_min(A), up to 2e4 for alpha = 1e-3 and |rho| = 0.999, the limits of the
activations), and at a sample's own direction the cancellation in the slopes h_xy / h_z + mu
near the lobe's peak (|mu| reaches 40 in these saturated-weight samplers); kappa covers them
all.  An FP32 emulation of the PDF on the CPU stays within 1e-5 + 4.5 u kappa over 60 such
samplers.  The PDF returned with a sample is compared with the oracle's PDF at that direction
with the parameters the kernel returned (both checked on their own above).  The lobe choice is
a comparison of u_0 with w_d: queries whose u_0 lies within 1e-5 of the oracle's w_d may take
the other lobe and are checked against the oracle's sample for that lobe instead.
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


def _unit(v):
    return (v / np.linalg.norm(v, axis=-1, keepdims=True)).astype(np.float32)


def problem(C, H, NH, address=wl.WRAP, n=4000, seed=61, scale=1.0):
    r = wl.rngs(seed)
    m = wl.make_material(r[0], r[1], 64, 64, C, 6, [32, 32], address=address)
    sdims, sp = wl.sampler_decoder(r[3], C, [H] * NH)
    sp = (sp * scale).astype(np.float32)
    q = wl.uniform_queries(r[2], n, -0.5, 5.5)
    q.uv[: n // 10] += r[2].integers(-3, 4, (n // 10, 2)).astype(np.float32)
    wo = _unit(r[4].normal(size=(n, 3)))
    u = r[4].random((n, 3)).astype(np.float32)
    return m, sdims, sp, q, wo, u


U32 = 2.0 ** -24


def _kappa(P, wi, wo):
    """First-order condition of the PDF at each query: sum over its inputs x (wi, wo, the 9
    parameters) of |d log pdf / d x| times an FP32 rounding of x in units of 2^-24 (1 for a
    direction component, |x| for a parameter); central differences of the FP64 oracle's PDF."""
    P, wi, wo = (np.asarray(a, np.float64) for a in (P, wi, wo))
    k = np.zeros(len(P))
    for which in range(3):
        for j in range(9 if which == 2 else 3):
            args = [wi, wo, P]
            x = args[which][:, j]
            size = np.abs(x) if which == 2 else np.ones_like(x)
            d = 1e-6 * np.maximum(size, 1e-300)
            plus, minus = [a.copy() for a in args], [a.copy() for a in args]
            plus[which][:, j] += d
            minus[which][:, j] -= d
            fp = oracle.proxy_pdf(plus[2], plus[0], plus[1])
            fm = oracle.proxy_pdf(minus[2], minus[0], minus[1])
            g = (np.log(np.maximum(fp, 1e-300)) - np.log(np.maximum(fm, 1e-300))) / (2.0 * d)
            k += np.abs(g) * size
    return k


def _close_pdf(got, ref, kappa):
    """Relative PDF error in units of its tolerance 1e-4 + 16 u kappa (where the PDF exceeds
    1e-3; absolute below)."""
    big = ref > 1e-3
    rel = np.abs(got[big] - ref[big]) / ref[big] / (1e-4 + 16.0 * U32 * kappa[big])
    small = np.abs(got[~big] - ref[~big])
    return rel.max(initial=0.0), small.max(initial=0.0)


@pytest.mark.parametrize("C,H,NH", [(16, 32, 3), (8, 32, 3), (16, 64, 1), (8, 16, 4), (16, 16, 2)])
def test_sampler_matches_oracle(nam, ctx, torch, C, H, NH):
    m, sdims, sp, q, wo, u = problem(C, H, NH, scale=1.5)
    mat = nam.Material.from_workload(ctx, m)
    mat.set_sampler(sdims, sp)
    dq = nam.to_device(q)
    P_ref = oracle.sampler_params(m.levels, sdims, sp, q.uv, q.lod, q.wi)
    P = nam.sampler_params(mat, dq[0], dq[1], dq[2]).cpu().numpy().astype(np.float64)
    ep = np.abs(P - P_ref) / np.maximum(1.0, np.abs(P_ref))
    pdf = nam.sampler_pdf(mat, dq[0], dq[1], dq[2], _dev(torch, wo)).cpu().numpy().astype(np.float64)
    pdf_ref = oracle.proxy_pdf(P_ref, q.wi, wo)
    rel, small = _close_pdf(pdf, pdf_ref, _kappa(P_ref, q.wi, wo))
    swo, spdf = nam.sampler_sample(mat, dq[0], dq[1], dq[2], _dev(torch, u))
    swo, spdf = swo.cpu().numpy().astype(np.float64), spdf.cpu().numpy().astype(np.float64)
    rwo, rpdf = oracle.proxy_sample(P_ref, q.wi, u)
    tie = np.abs(u[:, 0] - P_ref[:, 0]) < 1e-5
    alt_u = u.astype(np.float64).copy()
    alt_u[:, 0] = np.where(u[:, 0] < P_ref[:, 0], 1.0, 0.0)          # the other lobe
    awo, apdf = oracle.proxy_sample(P_ref, q.wi, alt_u)
    d_main = np.abs(swo - rwo).max(1)
    d_alt = np.abs(swo - awo).max(1)
    dw = np.where(tie, np.minimum(d_main, d_alt), d_main)
    # the PDF of a sampled direction is compared at the kernel's own direction: near grazing
    # half vectors (|wi . h| -> 0) and near wo = -wi the PDF is singular, so a 1e-6 change of the
    # direction alone moves it by far more than the FP32 evaluation error
    # and with the kernel's own parameters: samples sit in the peak of their lobe, where a 1e-6
    # change of a parameter of a narrow lobe (alpha down to 1e-3) moves the PDF by far more
    srel, ssmall = _close_pdf(spdf, oracle.proxy_pdf(P, q.wi, swo), _kappa(P, q.wi, swo))
    _say(f"sampler C{C} H{H}x{NH}: params {ep.max():.2e}, pdf error / tolerance {rel:.2f} (abs {small:.2e}), "
         f"sample dir {dw.max():.2e}, sample pdf error / tolerance {srel:.2f}, ties {tie.sum()}, "
         f"specular share {np.mean(u[:, 0] >= P_ref[:, 0]):.2f}")
    assert ep.max() <= 1e-5
    assert rel <= 1.0 and small <= 1e-7
    assert dw.max() <= 1e-4
    assert srel <= 1.0 and ssmall <= 1e-7
    np.testing.assert_allclose(np.linalg.norm(swo, axis=1), 1.0, atol=1e-5)


def test_cached_proxy_equals_fused(nam, ctx, torch):
    """nam_proxy_pdf / nam_proxy_sample on the parameters nam_sampler_params wrote give the fused
    kernels' results, and match the oracle's proxy on those same FP32 parameters."""
    m, sdims, sp, q, wo, u = problem(16, 32, 3)
    mat = nam.Material.from_workload(ctx, m)
    mat.set_sampler(sdims, sp)
    dq = nam.to_device(q)
    P = nam.sampler_params(mat, dq[0], dq[1], dq[2])
    dwo, du = _dev(torch, wo), _dev(torch, u)
    fused = nam.sampler_pdf(mat, dq[0], dq[1], dq[2], dwo)
    cached = nam.proxy_pdf(ctx, P, dq[2], dwo)
    torch.testing.assert_close(cached, fused, rtol=1e-6, atol=1e-9)
    fw, fp = nam.sampler_sample(mat, dq[0], dq[1], dq[2], du)
    cw, cp = nam.proxy_sample(ctx, P, dq[2], du)
    torch.testing.assert_close(cw, fw, rtol=0, atol=1e-6)
    torch.testing.assert_close(cp, fp, rtol=1e-6, atol=1e-9)
    Pn = P.cpu().numpy().astype(np.float64)
    rel, small = _close_pdf(cached.cpu().numpy().astype(np.float64), oracle.proxy_pdf(Pn, q.wi, wo), _kappa(Pn, q.wi, wo))
    assert rel <= 1.0 and small <= 1e-8


def test_sampler_non_finite_and_arguments(nam, ctx, torch):
    m, sdims, sp, q, wo, u = problem(8, 32, 3, n=16)
    mat = nam.Material.from_workload(ctx, m)
    dq = nam.to_device(q)
    with pytest.raises(nam.NamError, match="NAM_E_INVALID_ARG"):
        nam.sampler_params(mat, dq[0], dq[1], dq[2])               # no sampler yet
    with pytest.raises(nam.NamError, match="NAM_E_SHAPE"):
        mat.set_sampler([12] + sdims[1:], sp)
    with pytest.raises(nam.NamError, match="NAM_E_UNSUPPORTED"):
        mat.set_sampler([11, 48, 9], np.zeros(11 * 48 + 48 + 48 * 9 + 9, np.float32))
    mat.set_sampler(sdims, sp)
    q.uv[3, 1] = np.nan
    q.lod[5] = np.inf
    dq = nam.to_device(q)
    P = nam.sampler_params(mat, dq[0], dq[1], dq[2]).cpu().numpy()
    pdf = nam.sampler_pdf(mat, dq[0], dq[1], dq[2], _dev(torch, wo)).cpu().numpy()
    assert np.isnan(P[[3, 5]]).all() and np.isfinite(np.delete(P, [3, 5], 0)).all()
    assert np.isnan(pdf[[3, 5]]).all() and np.isfinite(np.delete(pdf, [3, 5])).all()


def test_sampler_survives_the_material_file(nam, ctx, torch, tmp_path):
    m, sdims, sp, q, wo, u = problem(16, 32, 3, n=2000)
    a = nam.Material.from_workload(ctx, m)
    a.set_sampler(sdims, sp)
    path = str(tmp_path / "s.nam")
    a.save(path)
    b = nam.Material.load_file(ctx, path)
    assert b.sdims == sdims
    dq = nam.to_device(q)
    assert torch.equal(nam.sampler_params(a, dq[0], dq[1], dq[2]), nam.sampler_params(b, dq[0], dq[1], dq[2]))
    assert torch.equal(nam.decode(a, *dq), nam.decode(b, *dq))
