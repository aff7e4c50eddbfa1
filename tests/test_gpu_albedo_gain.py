"""What the albedo head learns (Sec. 6.4 "Albedo inference").

The decoder 22-64-64-64-6 and a 128^2 x 16 latent pyramid are trained on the GPU by the
library's own kernels (6000 Adam steps of 262,144 samples drawn from a pool of 2^20, learning
rate 3e-3 with cosine decay).  Each sample's target is the analytic Lambert + GGX material's
f(x, wi, wo) for the RGB outputs and a one-sample estimate of its directional albedo at
(x, wo) for the albedo outputs, drawn independently of wi (Sec. 5.2: L2 against one-sample
estimates converges to the mean): one sample per lobe from the lobe's own density, which weighs
rho for the Lambertian lobe and F G1 for a visible-normal sample of the GGX lobe.  On 512
held-out (x, wo) the predicted albedo is compared with Eq. albedo computed by quadrature
(192 x 192 cells of the cosine-hemisphere map), against
  (ii)  the untrained initialisation and
  (iii) a per-texel albedo texture at the level-0 resolution, fitted by least squares to the
        same one-sample estimates (the mean estimate in each texel): the classical texture
        method, which cannot follow the dependence on wo.
Margins: from the first measurement with the earlier cosine-sampled estimates (trained 0.088,
untrained 0.565), trained < 0.2 x untrained; from the first measurement with the per-lobe
estimates (trained 0.0252, per-texel fit 0.0395), trained < 0.9 x the per-texel fit.  The
training runs in the library's deterministic mode, so the result is one reproducible number.
"""
import numpy as np
import pytest

from paper_2305_02678_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_albedo_head_learns_the_directional_albedo():
    import torch
    from paper_2305_02678_amd import nam
    ctx = nam.Context(0)
    ctx.set_deterministic(True)
    tex, C, hidden = 128, 16, (64, 64, 64)
    w = wl.training(seed=1004, tex=tex, channels=C, n=1 << 20, hidden=hidden, albedo=True)
    m = w.material
    assert m.dims[-1] == 6 and w.targets.shape[1] == 6
    rh = wl.rngs(4243)[wl.CHILD_TARGETS]
    n_h = 512
    huv = rh.random((n_h, 2)).astype(np.float32)
    hwo = wl.cosine_hemisphere(rh, n_h)
    hwi = wl.cosine_hemisphere(rh, n_h)
    hlod = np.zeros(n_h, np.float32)
    truth = w.analytic.directional_albedo(huv.astype(np.float64), hwo, grid=192)

    model = nam.Model.from_workload(ctx, m)
    texels = torch.from_numpy(nam.concat_levels(m.levels)).cuda()
    params = torch.from_numpy(m.params.copy()).cuda()
    pool = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
            for a in (w.queries.uv, w.queries.lod, w.queries.wi, w.queries.wo, w.targets)]
    held = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in (huv, hlod, hwi, hwo)]

    def albedo_error():
        pred = model.forward(texels, params, *held).cpu().numpy()[:, 3:].astype(np.float64)
        return float(np.mean(np.abs(pred - truth) / truth))

    untrained = albedo_error()

    def texel_index(uv):
        x = np.floor((uv[:, 0] - np.floor(uv[:, 0])) * tex).astype(np.int64) % tex
        y = np.floor((uv[:, 1] - np.floor(uv[:, 1])) * tex).astype(np.int64) % tex
        return y * tex + x

    ti = texel_index(w.queries.uv)
    sums = np.zeros((tex * tex, 3))
    cnt = np.zeros(tex * tex)
    np.add.at(sums, ti, w.targets[:, 3:].astype(np.float64))
    np.add.at(cnt, ti, 1)
    fit = np.where(cnt[:, None] > 0, sums / np.maximum(cnt, 1)[:, None], w.targets[:, 3:].mean(0))
    per_texel = float(np.mean(np.abs(fit[texel_index(huv)] - truth) / truth))

    steps, batch, lr = 6000, 262144, 3e-3
    tr = nam.Trainer(model, texels, params, lr=lr)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    for s in range(steps):
        tr.cfg[0] = lr * 0.5 * (1.0 + np.cos(np.pi * s / steps))
        idx = torch.randint(0, 1 << 20, (batch,), device="cuda", generator=g)
        tr.step(*[p[idx].contiguous() for p in pool])
    trained = albedo_error()
    print(f"held-out directional albedo, mean relative error: trained {trained:.4f}, per-texel fit of the "
          f"estimates {per_texel:.4f}, untrained {untrained:.4f}; albedo range {truth.min():.3f}..{truth.max():.3f}",
          flush=True)
    assert np.isfinite(trained)
    assert trained < 0.2 * untrained
    assert trained < 0.9 * per_texel
