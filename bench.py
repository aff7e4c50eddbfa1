"""Decode-throughput benchmark of the neural appearance hot path on one MI355X.

One step = one fused decode (latent fetch + concatenation + decoder + softplus) of a full
1920x1080 frame of shading queries against a 2048^2 x 16-channel latent pyramid (full mip
chain) with a 22-64-64-64-3 decoder, inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Each path is timed over K launches after W untimed ones (defaults 100 and 300): under a
sustained load the GPU's clocks ramp up over the first few hundred decodes (a frame decodes in
about 70 us at launch 50 and about 57 us by launch 400), so the timed launches see the
steady state.

The headline is the FP16 matrix-core decode; the FP32 (vector ALU) and E4M3 decodes of the
same frame are timed beside it, each with its error against the FP64 oracle, and so are the
decode with the level chosen by Russian roulette, the decode through two learned shading
frames and the decode with the albedo head (keys "stochastic", "frames" and "albedo").
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shading queries/sec (fetch+decode) FP16-MFMA vs FP32 at stated err; p99 latency"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f32_valu": 157.3, "f32_mfma": 157.3, "f16_mfma": 2500.0, "fp8_mfma": 5000.0}


KERNEL_SOURCES = ["paper_2305_02678_amd/csrc/decode_mfma.h", "paper_2305_02678_amd/csrc/decode_mfma.hip",
                  "paper_2305_02678_amd/csrc/latent_fetch.h", "paper_2305_02678_amd/csrc/mfma_pack.h",
                  "paper_2305_02678_amd/csrc/decode_f32.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "decode_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def counted_traffic(precision):
    """HBM bytes per launch from the committed rocprofv3 counters (FETCH_SIZE and WRITE_SIZE,
    each scaled by a copy of known size), or None if the kernel sources changed since."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash() or precision not in d.get("kernels", {}):
        return None
    k = d["kernels"][precision]
    return k["fetch_kib"] * 1024 * d["fetch_scale"] + k["write_kib"] * 1024 * d["write_scale"]


def algorithmic_flops_per_query(dims):
    return sum(2 * dims[k] * dims[k + 1] for k in range(len(dims) - 1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_cpu_oracle(w, min_s=10.0, max_passes=20):
    """The FP64 oracle on the full frame (all host threads), repeated until at least
    min_s seconds of CPU work; returns its output and the median pass throughput."""
    import oracle
    m, q = w.material, w.queries
    lv64 = [l.astype(np.float64) for l in m.levels]          # conversion kept out of the timing
    times, ref = [], None
    t_all = time.perf_counter()
    while len(times) < max_passes and (time.perf_counter() - t_all < min_s or len(times) < 3):
        t0 = time.perf_counter()
        ref = oracle.decode(lv64, m.dims, m.params, q.uv, q.lod, q.wi, q.wo)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    cores = oracle.threads()
    # the same oracle on one thread, on the first 200,000 queries of the frame (median of 3)
    sub = q.subset(np.arange(min(len(q), 200000)))
    oracle.set_threads(1)
    t1 = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.decode(lv64, m.dims, m.params, sub.uv, sub.lod, sub.wi, sub.wo)
        t1.append(time.perf_counter() - t0)
    oracle.set_threads(cores)
    med1 = float(np.median(t1))
    return ref, {"value": len(q) / med, "unit": "queries/s", "cores": cores, "kind": "oracle",
                 "sample": f"the full frame ({len(q)} queries), {len(times)} passes of the FP64 C oracle "
                           f"(median {med:.2f} s per pass, {sum(times):.1f} s in total)",
                 "single_thread": {"value": len(sub) / med1, "unit": "queries/s", "cores": 1,
                                   "sample": f"the first {len(sub)} queries of the frame, median of 3 passes"}}


def run_precision(nam, torch, mat, dq, N, prec, steps, warmup, am=None, first16=False, xi=None):
    if prec == nam.F32:
        mat.set_precision(nam.F32)
    elif prec == nam.F16:
        mat.set_precision(nam.F16)
    else:
        mat.set_precision(nam.FP8_E4M3, act_absmax=am, first_layer_f16=first16)
    uv, lod, wi, wo = dq
    rgb = torch.empty((N, mat.dims[-1]), device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        nam.decode(mat, uv, lod, wi, wo, out=rgb, xi=xi)
    # throughput: the host clock around the K launches with a synchronisation on both sides
    # (value), and the kernel time as the span of launches 2..K between a pair of events on the
    # launch stream (kernel_ms = span / (K - 1)): the first event fires when launch 1 ends, so the
    # host's latency to its first launch after the synchronisation (a few hundred microseconds)
    # stays out of the kernel time while the launches run back to back
    first, last = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nam.decode(mat, uv, lod, wi, wo, out=rgb, xi=xi)
    first.record(stream)
    for k in range(steps - 1):
        nam.decode(mat, uv, lod, wi, wo, out=rgb, xi=xi)
    last.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    batch_ms = first.elapsed_time(last) / max(steps - 1, 1)
    prime = torch.empty(1 << 24, dtype=torch.float32, device="cuda")
    # latency: the same launches each between its own pair of events
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    prime.fill_(0.0)
    for k in range(steps):
        starts[k].record(stream)
        nam.decode(mat, uv, lod, wi, wo, out=rgb, xi=xi)
        ends[k].record(stream)
    torch.cuda.synchronize()
    per = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])   # ms per launch
    # cold-cache latency: a 1 GiB write between launches evicts the 256 MB Infinity Cache
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    cold = []
    for k in range(min(steps, 20)):
        flush.fill_(float(k))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        nam.decode(mat, uv, lod, wi, wo, out=rgb, xi=xi)
        b.record(stream)
        torch.cuda.synchronize()
        cold.append(a.elapsed_time(b))
    del flush
    return {"qps": N / (wall / steps), "ms_per_step": wall * 1e3 / steps, "kernel_ms": batch_ms,
            "p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99)),
            "cold_p50_ms": float(np.percentile(cold, 50)), "cold_p99_ms": float(np.percentile(cold, 99)),
            "rgb": rgb}


def roofline(prec_name, N, U, C, n_params, dims, kernel_ms, query_bytes=36, with_traffic=True, taps=8,
             traffic_key=None, out_bytes=None, fp32_mfma=False):
    """Algorithmic bytes: query_bytes in and out_bytes (by default 4 per decoder output,
    dims[-1]: 12 for RGB, 24 with the albedo head) out per query, the distinct texels U once, the
    decoder weights once; the no-reuse bound reads every tap of every query.  FP32 paths are
    priced against the vector ALU's FP32 peak, or the FP32 matrix cores' (the same 157.3 TFLOP/s)
    where the decode runs there (fp32_mfma: plain trilinear decodes, no frames)."""
    out_bytes = 4 * dims[-1] if out_bytes is None else out_bytes
    tex_bytes = 4 if prec_name == "fp32" else 2
    wbytes = {"fp32": 4, "fp16": 2, "fp8": 1}[prec_name] * n_params
    B = N * (query_bytes + out_bytes) + U * C * tex_bytes + wbytes
    F = N * algorithmic_flops_per_query(dims)
    t = kernel_ms * 1e-3
    peak_f = PEAK_TFLOPS[{"fp32": "f32_mfma" if fp32_mfma else "f32_valu", "fp16": "f16_mfma", "fp8": "fp8_mfma"}[prec_name]]
    t_hbm, t_flop = B / (PEAK_HBM_GBS * 1e9), F / (peak_f * 1e12)
    if prec_name == "fp32":
        r = {"bound": "mfma" if fp32_mfma else "alu", "achieved": F / t / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    elif t_hbm >= t_flop:
        r = {"bound": "hbm", "achieved": B / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        r = {"bound": "mfma", "achieved": F / t / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = counted_traffic(traffic_key or prec_name) if with_traffic else None
    r.update({"algorithmic_bytes": B, "algorithmic_flops": F, "distinct_texels": U, "kernel_ms": kernel_ms,
              "t_hbm_floor_us": t_hbm * 1e6, "t_compute_floor_us": t_flop * 1e6,
              "no_reuse_bytes": N * (query_bytes + out_bytes + taps * C * tex_bytes) + wbytes})
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-stochastic", action="store_true", help="skip the Russian-roulette level-choice decode")
    ap.add_argument("--no-frames", action="store_true", help="skip the decode with learned shading frames")
    ap.add_argument("--no-sampler", action="store_true", help="skip the importance-sampling decoder")
    ap.add_argument("--no-albedo", action="store_true", help="skip the decode with the albedo head")
    ap.add_argument("--no-encoder", action="store_true", help="skip the encoder's training phase and bake")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--counters-pass", choices=["fp16", "fp32", "fp8", "fp16-albedo", "train"], default=None,
                    help="short run for hardware-counter collection: 3 decodes of the frame in one precision "
                         "(or 3 training steps of 1,048,576 samples), then a 256 MiB device-to-device copy whose "
                         "byte count calibrates the counters")
    args = ap.parse_args()
    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the decode path is measured on a single MI355X "
              "(queries are independent; a multi-GPU split would give each GPU its own share of the frame).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_02678_amd import nam
    from paper_2305_02678_amd import workloads as wl

    if args.counters_pass == "train":
        w = wl.training()
        ctx = nam.Context(0)
        model = nam.Model.from_workload(ctx, w.material)
        tr = nam.Trainer(model, torch.from_numpy(nam.concat_levels(w.material.levels)).cuda(),
                         torch.from_numpy(w.material.params.copy()).cuda(), lr=1e-3)
        dq = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
              for a in (w.queries.uv, w.queries.lod, w.queries.wi, w.queries.wo, w.targets)]
        for _ in range(3):
            tr.step(*dq)
        torch.cuda.synchronize()
        log(f"counters pass train: 3 steps of {len(w.queries)} samples, loss {tr.loss.item():.5f}")
        return

    t0 = time.time()
    w = wl.frame()
    m, q = w.material, w.queries
    N = len(q)
    log(f"workload generated in {time.time() - t0:.1f} s: {w.name}, {N} queries")

    ctx = nam.Context(0)
    mat = nam.Material.from_workload(ctx, m)
    dq = nam.to_device(q)
    U = nam.texel_footprint(mat, dq[0], dq[1])
    calib = wl.frame(seed=99, n=65536)
    am = mat.calibrate(*nam.to_device(calib.queries))

    if args.counters_pass:
        if args.counters_pass == "fp16-albedo":            # the frame's decoder with the albedo head
            dims, params, _ = wl.decoder_for(wl.rngs(1002)[wl.CHILD_WEIGHTS], m.channels, m.dims[1:-1], albedo=True)
            mat = nam.Material.from_workload(ctx, wl.Material(m.width, m.height, m.channels, m.levels, dims, params,
                                                                 m.address))
        prec = {"fp16": nam.F16, "fp32": nam.F32, "fp8": nam.FP8_E4M3, "fp16-albedo": nam.F16}[args.counters_pass]
        r = run_precision(nam, torch, mat, dq, N, prec, 3, 0, am)
        src = torch.empty(1 << 26, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"counters pass {args.counters_pass}: kernel {r['kernel_ms'] * 1e3:.1f} us; copy of {src.numel() * 4} bytes")
        return

    res = {}
    for name, prec, f16first in (("fp16", nam.F16, False), ("fp32", nam.F32, False), ("fp8", nam.FP8_E4M3, False)):
        r = run_precision(nam, torch, mat, dq, N, prec, args.steps, args.warmup, am, f16first)
        r["rgb"] = r["rgb"].cpu().numpy().astype(np.float64)
        res[name] = r
        log(f"{name}: {r['qps'] / 1e9:.3f} G queries/s, kernel {r['kernel_ms'] * 1e3:.1f} us")

    head = res["fp16"]
    out = {
        "metric": METRIC, "value": head["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": w.name + ", decoder FP16 on MFMA (FP32 accumulate), texels FP16",
                   "queries": N, "precision": "fp16"},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"], "cold_p50": head["cold_p50_ms"],
                       "cold_p99": head["cold_p99_ms"]},
        "roofline": roofline("fp16", N, U, m.channels, m.params.size, m.dims, head["kernel_ms"]),
        "speedup_vs_fp32": head["qps"] / res["fp32"]["qps"],
        "compare": {},
    }
    ref = None
    if not args.no_cpu_baseline:
        ref, cpu = time_cpu_oracle(w, args.cpu_seconds)
        out["cpu_baseline"] = cpu
    for name, r in res.items():
        entry = {k: v for k, v in r.items() if k != "rgb"}
        entry["roofline"] = roofline(name, N, U, m.channels, m.params.size, m.dims, r["kernel_ms"], fp32_mfma=True)
        if ref is not None:
            e = np.abs(r["rgb"] - ref) / np.abs(ref)
            entry["error_vs_oracle"] = {"max_rel": float(e.max()), "mean_rel": float(e.mean()), "samples": int(e.size)}
        out["compare"][name] = entry
    if ref is not None:
        out["error_vs_oracle"] = out["compare"]["fp16"]["error_vs_oracle"]
    # achievable HBM bandwidth: a plain device copy of 1 GiB (reads and writes counted)
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = 2 * src.numel() * 4 * 10 / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    log(f"device copy: {out['copy_gbs']:.0f} GB/s")
    if not args.no_stochastic:
        out["stochastic"] = bench_stochastic(nam, torch, w, mat, dq, N, m, args, with_oracle=not args.no_cpu_baseline)
    if not args.no_sampler:
        out["sampler"] = bench_sampler(nam, torch, wl, ctx, w, mat, dq, U, args, with_oracle=not args.no_cpu_baseline)
    if not args.no_frames:
        out["frames"] = bench_frames(nam, torch, wl, ctx, w, U, args, with_oracle=not args.no_cpu_baseline)
    if not args.no_albedo:
        out["albedo"] = bench_albedo(nam, torch, wl, ctx, w, U, args, with_oracle=not args.no_cpu_baseline)
    del mat, dq, res
    if not args.no_train:
        out["train"] = bench_train(nam, torch, wl, ctx, with_oracle=not args.no_cpu_baseline)
    if not args.no_encoder:
        out["encoder"] = bench_encoder(nam, torch, wl, ctx, with_oracle=not args.no_cpu_baseline)
    if not args.no_serve:
        out["serving"] = bench_serving(nam, torch, wl, ctx)
    print(json.dumps(out), flush=True)


def bench_stochastic(nam, torch, w, mat, dq, N, m, args, with_oracle):
    """The same frame with the level chosen by Russian roulette (4 taps per query), seeded
    uniform draws; FP16 and FP32."""
    xi = np.random.default_rng(20240605).random(N).astype(np.float32)
    dxi = torch.from_numpy(xi).cuda()
    U = nam.texel_footprint(mat, dq[0], dq[1], xi=dxi)
    out = {"workload": w.name + ", level by Russian roulette (Sec. 4.1), seeded uniform draws",
           "distinct_texels": U}
    if with_oracle:
        import oracle                                  # the oracle side of the check, as for the baseline
        idx = np.random.default_rng(4).choice(N, 100000, replace=False)
        s = w.queries.subset(idx)
        ref = oracle.decode_rr(m.levels, m.dims, m.params, s.uv, s.lod, xi[idx], s.wi, s.wo)
    for name, prec in (("fp16", nam.F16), ("fp32", nam.F32)):
        r = run_precision(nam, torch, mat, dq, N, prec, args.steps, args.warmup, xi=dxi)
        entry = {k: v for k, v in r.items() if k != "rgb"}
        entry["roofline"] = roofline(name, N, U, m.channels, m.params.size, m.dims, r["kernel_ms"], query_bytes=40,
                                     with_traffic=False, taps=4)
        if with_oracle:
            e = np.abs(r["rgb"].cpu().numpy()[idx] - ref) / np.abs(ref)
            entry["error_vs_oracle"] = {"max_rel": float(e.max()), "mean_rel": float(e.mean()), "samples": int(e.size)}
        out[name] = entry
        log(f"stochastic {name}: {r['qps'] / 1e9:.3f} G queries/s, kernel {r['kernel_ms'] * 1e3:.1f} us")
    return out


def bench_frames(nam, torch, wl, ctx, w, U, args, with_oracle):
    """The same frame decoded by a material with two learned shading frames (Sec. 4.2): the
    16 -> 12 frame layer, normalised frames and T wi, T wo in FP32 in the fetch, then the decoder
    28-64-64-64-3; same latent pyramid and queries (so the same distinct texels U), decoder
    weights drawn for the wider input.  FP16 and FP32, trilinear filtering."""
    m = w.material
    N = len(w.queries)
    nf = 2
    dims, params, F = wl.decoder_for(wl.rngs(1002)[wl.CHILD_WEIGHTS], m.channels, m.dims[1:-1], nf)
    fm = wl.Material(m.width, m.height, m.channels, m.levels, dims, params, m.address, nf, F)
    mat = nam.Material.from_workload(ctx, fm)
    dq = nam.to_device(w.queries)
    out = {"workload": w.name.replace(f"MLP {'-'.join(str(d) for d in m.dims)}",
                                      f"MLP {'-'.join(str(d) for d in dims)}") + f", {nf} learned shading frames",
           "distinct_texels": U}
    if with_oracle:
        import oracle                                  # the oracle side of the check, as for the baseline
        idx = np.random.default_rng(6).choice(N, 100000, replace=False)
        s = w.queries.subset(idx)
        ref = oracle.decode_frames(fm.levels, dims, params, nf, F, s.uv, s.lod, s.wi, s.wo)
    # frame layer (2 C 6N) and the transform dot products (2 x 3N rows x 2 directions x 3) on top
    # of the decoder's matrix products
    extra_flops = 2 * m.channels * 6 * nf + 2 * 3 * (3 * nf) * 2
    for name, prec in (("fp16", nam.F16), ("fp32", nam.F32)):
        r = run_precision(nam, torch, mat, dq, N, prec, args.steps, args.warmup)
        entry = {k: v for k, v in r.items() if k != "rgb"}
        rf = roofline(name, N, U, m.channels, params.size + F.size, dims, r["kernel_ms"], with_traffic=False)
        rf["algorithmic_flops"] += N * extra_flops
        entry["roofline"] = rf
        if with_oracle:
            e = np.abs(r["rgb"].cpu().numpy()[idx] - ref) / np.abs(ref)
            entry["error_vs_oracle"] = {"max_rel": float(e.max()), "mean_rel": float(e.mean()), "samples": int(e.size)}
        out[name] = entry
        log(f"frames {name}: {r['qps'] / 1e9:.3f} G queries/s, kernel {r['kernel_ms'] * 1e3:.1f} us")
    mat.free()
    return out


def bench_albedo(nam, torch, wl, ctx, w, U, args, with_oracle):
    """The same frame decoded by a decoder with the albedo head (Sec. 6.4): 22-64-64-64-6, RGB
    then the directional albedo, 24 bytes out per query; same latent pyramid and queries (so
    the same distinct texels U), decoder weights drawn for the wider output.  FP16 and FP32,
    trilinear filtering."""
    m = w.material
    N = len(w.queries)
    dims, params, _ = wl.decoder_for(wl.rngs(1002)[wl.CHILD_WEIGHTS], m.channels, m.dims[1:-1], albedo=True)
    am = wl.Material(m.width, m.height, m.channels, m.levels, dims, params, m.address)
    mat = nam.Material.from_workload(ctx, am)
    dq = nam.to_device(w.queries)
    out = {"workload": w.name.replace(f"MLP {'-'.join(str(d) for d in m.dims)}",
                                      f"MLP {'-'.join(str(d) for d in dims)}") + ", albedo head",
           "distinct_texels": U}
    if with_oracle:
        import oracle                                  # the oracle side of the check, as for the baseline
        idx = np.random.default_rng(8).choice(N, 100000, replace=False)
        s = w.queries.subset(idx)
        ref = oracle.decode(am.levels, dims, params, s.uv, s.lod, s.wi, s.wo)
    for name, prec in (("fp16", nam.F16), ("fp32", nam.F32)):
        r = run_precision(nam, torch, mat, dq, N, prec, args.steps, args.warmup)
        entry = {k: v for k, v in r.items() if k != "rgb"}
        entry["roofline"] = roofline(name, N, U, m.channels, params.size, dims, r["kernel_ms"],
                                     with_traffic=name == "fp16", traffic_key="fp16-albedo", fp32_mfma=True)
        if with_oracle:
            e = np.abs(r["rgb"].cpu().numpy()[idx] - ref) / np.abs(ref)
            entry["error_vs_oracle"] = {"max_rel": float(e.max()), "mean_rel": float(e.mean()), "samples": int(e.size),
                                        "albedo_max_rel": float(e[:, 3:].max())}
        out[name] = entry
        log(f"albedo {name}: {r['qps'] / 1e9:.3f} G queries/s, kernel {r['kernel_ms'] * 1e3:.1f} us")
    mat.free()
    return out


def bench_sampler(nam, torch, wl, ctx, w, mat, dq, U, args, with_oracle):
    """Importance sampling on the same frame (Sec. 4.3, App. A): the paper's 3 x 32 sampling
    decoder on [z, wi] (19-32-32-32-9), in FP16 on the matrix cores (the precision Sec. 5.2
    converts the sampler to at load) and in FP32.  Timed per precision: the fused sample (fetch,
    decoder, activations, proxy sample and its PDF), the fused PDF of given directions and the
    fused proxy parameters; and sampling from cached proxy parameters (no fetch, no network).
    Roofline of the fused sample: 36 bytes in (uv, lod, wi, u) and 16 out (wo, pdf) per query,
    the distinct texels once."""
    m = w.material
    N = len(w.queries)
    sdims, sp = wl.sampler_decoder(wl.rngs(1002)[wl.CHILD_TARGETS], m.channels, (32, 32, 32))
    mat.set_sampler(sdims, sp)
    rng = np.random.default_rng(77)
    u = rng.random((N, 3), dtype=np.float32)
    wo = rng.normal(size=(N, 3))
    wo = (wo / np.linalg.norm(wo, axis=1, keepdims=True)).astype(np.float32)
    du, dwo = torch.from_numpy(u).cuda(), torch.from_numpy(wo).cuda()
    uv, lod, wi, _ = dq

    def timed(fn, reps):
        """Kernel time per launch after args.warmup launches (the clocks ramp up over the first
        few hundred): launches 2..reps back to back between a pair of events (the first event
        fires when launch 1 ends, after the host's latency to its first launch)."""
        for _ in range(args.warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        fn()
        a.record()
        for _ in range(reps - 1):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / max(reps - 1, 1)

    idx = np.random.default_rng(8).choice(N, 100000, replace=False) if with_oracle else None
    Pr = None
    if with_oracle:
        import oracle                                  # the oracle side of the check, as for the baseline
        s = w.queries.subset(idx)
        Pr = oracle.sampler_params(m.levels, sdims, sp, s.uv, s.lod, s.wi)
    out = {"workload": w.name.split(", MLP")[0] + f", sampling decoder {'-'.join(map(str, sdims))}"}
    P = None
    for name, prec in (("fp16", nam.F16), ("fp32", nam.F32)):
        mat.set_precision(prec)
        P = nam.sampler_params(mat, uv, lod, wi)
        t_sample = timed(lambda: nam.sampler_sample(mat, uv, lod, wi, du), args.steps)
        t_pdf = timed(lambda: nam.sampler_pdf(mat, uv, lod, wi, dwo), args.steps)
        t_params = timed(lambda: nam.sampler_params(mat, uv, lod, wi, out=P), args.steps)
        rf = roofline(name, N, U, m.channels, sp.size, sdims, t_sample, query_bytes=36, out_bytes=16,
                      with_traffic=False)
        e = {"sample": {"ms": t_sample, "queries_per_s": N / (t_sample * 1e-3), "roofline": rf},
             "pdf": {"ms": t_pdf, "queries_per_s": N / (t_pdf * 1e-3)},
             "params": {"ms": t_params, "queries_per_s": N / (t_params * 1e-3)}}
        if with_oracle:
            Pg = P.cpu().numpy()[idx].astype(np.float64)
            pdf_g = nam.sampler_pdf(mat, uv, lod, wi, dwo).cpu().numpy()[idx]
            pdf_r = oracle.proxy_pdf(Pr, s.wi, wo[idx])
            big = pdf_r > 1e-3
            e["error_vs_oracle"] = {
                "params_max_rel": float((np.abs(Pg - Pr) / np.maximum(1.0, np.abs(Pr))).max()),
                "params_mean_rel": float((np.abs(Pg - Pr) / np.maximum(1.0, np.abs(Pr))).mean()),
                "pdf_max_rel": float((np.abs(pdf_g[big] - pdf_r[big]) / pdf_r[big]).max()),
                "pdf_median_rel": float(np.median(np.abs(pdf_g[big] - pdf_r[big]) / pdf_r[big])),
                "samples": int(len(idx))}
            if name == "fp16":                         # against the oracle's FP16 sampler arithmetic
                qp = np.concatenate([np.concatenate([W.astype(np.float16).astype(np.float64).ravel(), b])
                                     for W, b in wl.unpack_params(sp.astype(np.float64), sdims)])
                Pq = oracle.sampler_params_quant([l.astype(np.float16).astype(np.float64) for l in m.levels], sdims,
                                                 qp, s.uv, s.lod, s.wi, address=m.address)
                ea = np.abs(Pg - Pq) / np.maximum(1.0, np.abs(Pq))
                e["error_vs_oracle"].update({"params_arith_max_rel": float(ea.max()),
                                             "params_arith_mean_rel": float(ea.mean()),
                                             "fp16_format_max_rel": float((np.abs(Pq - Pr) / np.maximum(1.0, np.abs(Pr))).max())})
        out[name] = e
        log(f"sampler {name}: sample {t_sample * 1e3:.1f} us ({N / t_sample / 1e6:.2f} G/s, {rf['bound']} "
            f"{rf['frac']:.2f}), pdf {t_pdf * 1e3:.1f} us, params {t_params * 1e3:.1f} us")
    t_cached = timed(lambda: nam.proxy_sample(ctx, P, wi, du), args.steps)
    out["cached_sample"] = {"ms": t_cached, "queries_per_s": N / (t_cached * 1e-3), "bytes": N * (36 + 12 + 12 + 12 + 4)}
    out["cached_sample"]["gbs"] = out["cached_sample"]["bytes"] / (t_cached * 1e-3) / 1e9
    log(f"sampler: cached sample {t_cached * 1e3:.1f} us")
    return out


def bench_encoder(nam, torch, wl, ctx, steps=20, warmup=10, with_oracle=False):
    """The encoder's first training phase (Sec. 5.1) on the training workload: 1,048,576 samples
    of the analytic material, its parameters (albedo, roughness) as a 1024^2 x 4 pyramid with 11
    levels, encoder 4-32-32-16, decoder 22-64-64-64-3.  One step = the codes of the samples
    (nam_encode_queries), the decoder's loss and gradients on them (nam_loss_backward_codes), the
    encoder's gradient (nam_encoder_backward) and Adam on both; FP32.  Then the bake of the
    latent pyramid (nam_encode_texels over its 1,398,101 texels).  Roofline of the encoder
    kernels: FP32 vector ALU, 2 (4 x 32 + 32 x 32 + 32 x 16) = 3,328 FLOP per code."""
    t0 = time.time()
    w = wl.training()
    m, q, am = w.material, w.queries, w.analytic
    attr = wl.material_parameters(am, m.width, m.n_levels)
    log(f"encoder workload generated in {time.time() - t0:.1f} s")
    dims_e, ep = wl.encoder_params(wl.rngs(5)[0], 4, m.channels, (32, 32))
    enc = nam.Encoder(ctx, dims_e, m.width, m.height, m.n_levels)
    model = nam.Model.from_workload(ctx, m)
    flat = torch.from_numpy(np.concatenate([l.reshape(-1, 4) for l in attr])).cuda()
    eparams = torch.from_numpy(ep.astype(np.float32)).cuda()
    params = torch.from_numpy(m.params.copy()).cuda()
    uv, lod, wi, wo, tgt = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
                            for a in (q.uv, q.lod, q.wi, q.wo, w.targets)]
    st = [torch.zeros_like(t) for t in (eparams, eparams, params, params)]
    n = len(q)
    counter = [0]

    def step():
        counter[0] += 1
        z = enc.encode_queries(eparams, flat, uv, lod)
        _, dz, dp = model.loss_backward_codes(params, z, wi, wo, tgt)
        de = enc.backward(eparams, flat, uv, lod, dz)
        nam.adam_update(ctx, eparams, st[0], st[1], de, counter[0], lr=1e-3)
        nam.adam_update(ctx, params, st[2], st[3], dp, counter[0], lr=1e-3)

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        fn()
        a.record()
        for _ in range(reps - 1):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / max(reps - 1, 1)

    t_step = timed(step, steps)
    z = enc.encode_queries(eparams, flat, uv, lod)
    _, dz, _ = model.loss_backward_codes(params, z, wi, wo, tgt)
    t_enc = timed(lambda: enc.encode_queries(eparams, flat, uv, lod), steps)
    t_codes = timed(lambda: model.loss_backward_codes(params, z, wi, wo, tgt), steps)
    t_bwd = timed(lambda: enc.backward(eparams, flat, uv, lod, dz), steps)
    t_bake = timed(lambda: enc.encode_texels(eparams, flat), steps)
    fl = 2 * sum(dims_e[k] * dims_e[k + 1] for k in range(len(dims_e) - 1))
    texels = flat.shape[0]

    def alu(flops, ms):
        a = flops / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": a, "peak": PEAK_TFLOPS["f32_valu"], "unit": "TFLOP/s",
                "frac": a / PEAK_TFLOPS["f32_valu"], "algorithmic_flops": flops}

    out = {"workload": f"encoder {'-'.join(map(str, dims_e))} on the {m.width}^2 x 4 parameter pyramid "
                       f"({m.n_levels} levels), decoder {'-'.join(map(str, m.dims))}, {n} samples, FP32",
           "step_ms": t_step, "samples_per_s": n / (t_step * 1e-3),
           "split": {"encode_queries_ms": t_enc, "codes_loss_backward_ms": t_codes, "encoder_backward_ms": t_bwd},
           "encode_queries_roofline": alu(n * fl, t_enc),
           "encoder_backward_roofline": alu(3 * n * fl, t_bwd),
           "bake": {"texels": texels, "ms": t_bake, "texels_per_s": texels / (t_bake * 1e-3),
                    "roofline": alu(texels * fl, t_bake)}}
    if with_oracle:
        import oracle                                  # the oracle side, as for the baseline
        k = 65536
        a = time.time()
        zr = oracle.encode_queries(attr, dims_e, ep, q.uv[:k], q.lod[:k])
        _, _, dzr = oracle.loss_grad_codes(m.dims, m.params, zr, q.wi[:k], q.wo[:k], w.targets[:k])
        oracle.encoder_backward(attr, dims_e, ep, q.uv[:k], q.lod[:k], dzr)
        out["cpu_baseline"] = {"value": k / (time.time() - a), "unit": "samples/s", "cores": oracle.threads(),
                               "kind": "oracle", "sample": f"one end-to-end gradient of the first {k} samples"}
    log(f"encoder: step {t_step:.2f} ms ({n / t_step / 1e3:.0f} M samples/s; codes {t_enc * 1e3:.0f} us, "
        f"codes loss {t_codes * 1e3:.0f} us, encoder backward {t_bwd * 1e3:.0f} us), bake of {texels} texels "
        f"{t_bake * 1e3:.0f} us")
    return out


def bench_train(nam, torch, wl, ctx, steps=20, warmup=3, with_oracle=False):
    """One training step = MSE loss and gradients of 1,048,576 samples into a 1024^2 x 16
    pyramid (11 levels) and a 22-64-64-64-3 decoder, then Adam (lr 1e-3) on every parameter and
    texel, all FP32."""
    t0 = time.time()
    w = wl.training()
    m, q = w.material, w.queries
    log(f"training workload generated in {time.time() - t0:.1f} s: {w.name}")
    model = nam.Model.from_workload(ctx, m)
    texels = torch.from_numpy(nam.concat_levels(m.levels)).cuda()
    params = torch.from_numpy(m.params.copy()).cuda()
    dq = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
          for a in (q.uv, q.lod, q.wi, q.wo, w.targets)]
    tr = nam.Trainer(model, texels, params, lr=1e-3)
    for _ in range(warmup):
        tr.step(*dq)
    first = tr.loss.item()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(steps):
        tr.step(*dq)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / steps
    n = len(q)
    flops = 3 * n * algorithmic_flops_per_query(m.dims)

    # split of the step: forward alone, loss with forward + backward + latent scatter (one fused
    # kernel plus the parameter-gradient reduction), Adam over every parameter and texel
    def timed(fn, reps=10):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    d_tex = torch.zeros_like(texels)
    grads = {}

    def lossgrad():
        grads["r"] = model.loss_backward(texels, params, *dq, d_texels=d_tex)

    t_fwd = timed(lambda: model.forward(texels, params, *dq[:4]))
    t_lb = timed(lossgrad)
    g_par = grads["r"][2]
    mt, vt, mp, vp = (torch.zeros_like(texels), torch.zeros_like(texels), torch.zeros_like(params),
                      torch.zeros_like(params))

    def adam():
        nam.adam_update(ctx, texels, mt, vt, d_tex, 1, lr=0.0)
        nam.adam_update(ctx, params, mp, vp, g_par, 1, lr=0.0)

    t_adam = timed(adam)
    # the same loss and gradients in the deterministic mode (fixed-point latent scatter)
    ctx.set_deterministic(True)
    t_det = timed(lossgrad, reps=5)
    ctx.set_deterministic(False)
    split = {"forward_ms": t_fwd, "loss_forward_backward_scatter_ms": t_lb,
             "backward_and_scatter_ms": t_lb - t_fwd, "adam_ms": t_adam, "step_ms": ms,
             "deterministic_loss_backward_ms": t_det}
    # a decoder with two learned shading frames (28-64-64-64-3, Sec. 4.2) on the same batch: loss
    # and gradients of the frame layer, decoder and texels (vector training kernel)
    rf = wl.rngs(77)
    fdims = [m.channels + 12] + list(m.dims[1:])
    fdec = wl.xavier_mlp(rf[1], fdims).astype(np.float32)
    fF = wl.frame_layer(rf[1], 2, m.channels)
    fmodel = nam.Model(ctx, m.width, m.height, m.channels, m.n_levels, fdims, m.address, n_frames=2)
    fpar = torch.from_numpy(np.concatenate([fF, fdec])).cuda()
    split["frames_loss_backward_ms"] = timed(lambda: fmodel.loss_backward(texels, fpar, *dq, d_texels=d_tex), reps=5)
    del d_tex, mt, vt, mp, vp, grads, fpar
    oracle_rate = None
    if with_oracle:
        import oracle                                  # the CPU-baseline leg: the oracle's gradient step
        k = 65536
        sub = q.subset(np.arange(k))
        lv64 = [l.astype(np.float64) for l in m.levels]
        t0 = time.perf_counter()
        oracle.loss_grad(lv64, m.dims, m.params, sub.uv, sub.lod, sub.wi, sub.wo, w.targets[:k])
        oracle_rate = {"value": k / (time.perf_counter() - t0), "unit": "samples/s", "cores": oracle.threads(),
                       "kind": "oracle", "sample": f"loss and exact gradients of the first {k} samples of the batch"}
    r = {"workload": w.name + ", MSE, Adam lr 1e-3, FP32", "ms_per_step": ms, "samples_per_s": n / (ms * 1e-3),
         "tflops_fwd_bwd_equiv": flops / (ms * 1e-3) / 1e12, "loss_first": first, "loss_last": tr.loss.item(),
         "steps": steps, "split": split}
    if oracle_rate is not None:
        r["cpu_baseline"] = oracle_rate
    log(f"train: {ms:.2f} ms/step, {r['samples_per_s'] / 1e6:.1f} M samples/s; loss and gradients: "
        f"deterministic {split['deterministic_loss_backward_ms']:.2f} ms, two learned frames "
        f"{split['frames_loss_backward_ms']:.2f} ms")
    del texels, params, dq, tr
    r["albedo"] = bench_train_albedo(nam, torch, wl, ctx, steps, warmup)
    return r


def bench_train_albedo(nam, torch, wl, ctx, steps, warmup):
    """The same training step with the albedo head (Sec. 6.4): decoder 22-64-64-64-6, each
    target row RGB plus a one-sample estimate of the directional albedo, the loss summing both
    L2 terms."""
    w = wl.training(albedo=True)
    m, q = w.material, w.queries
    model = nam.Model.from_workload(ctx, m)
    texels = torch.from_numpy(nam.concat_levels(m.levels)).cuda()
    params = torch.from_numpy(m.params.copy()).cuda()
    dq = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
          for a in (q.uv, q.lod, q.wi, q.wo, w.targets)]
    tr = nam.Trainer(model, texels, params, lr=1e-3)
    for _ in range(warmup):
        tr.step(*dq)
    first = tr.loss.item()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(steps):
        tr.step(*dq)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / steps
    r = {"workload": w.name + ", albedo head, MSE over RGB and albedo, Adam lr 1e-3, FP32", "ms_per_step": ms,
         "samples_per_s": len(q) / (ms * 1e-3), "loss_first": first, "loss_last": tr.loss.item(), "steps": steps}
    log(f"train with the albedo head: {ms:.2f} ms/step, {r['samples_per_s'] / 1e6:.1f} M samples/s")
    del texels, params, dq, tr
    return r


def bench_serving(nam, torch, wl, ctx, n_requests=2000, budget=2 << 30):
    """8 resident materials (side 512..4096, 8 or 16 channels, full chains), Poisson requests of
    log-uniform size in [4096, 8294400] queries, device-resident inputs, HBM budget 2 GiB for
    in-flight request buffers.  Saturated throughput first (all requests at once), then offered
    loads of 0.5, 0.8 and 1.1 times it; FP16 matrix-core decoders, then FP32 at 0.8."""
    t0 = time.time()
    mats = wl.serving_materials()
    log(f"serving materials generated in {time.time() - t0:.1f} s: sides {[m.width for m in mats]}, "
        f"channels {[m.channels for m in mats]}")
    handles = [nam.Material.from_workload(ctx, m) for m in mats]
    del mats
    # one 3840x2160 pool of queries per material (uv and directions shared, lod per texture size)
    smap_rng = wl.rngs(1005)[wl.CHILD_REQUESTS]
    smap = wl.random_screen_map(smap_rng, 2048, 2048, 3840, 2160)
    pool_q = wl.screen_queries(smap_rng, smap)
    P = len(pool_q)
    uv, lod2048, wi, wo = nam.to_device(pool_q)
    lods = {}
    outs = []
    for h in handles:
        side = h.desc.width
        if side not in lods:
            lods[side] = (lod2048 + float(np.log2(side / 2048.0))).contiguous()
        outs.append(torch.empty((P, 3), device="cuda"))
    rng = np.random.default_rng(1005)
    sizes = wl.request_sizes(rng, n_requests, 4096, 8294400)
    mids = rng.integers(0, len(handles), n_requests)
    offs = np.array([rng.integers(0, P - s + 1) for s in sizes])
    mean_q = float(sizes.mean())

    lead = 0.5      # every request is queued before the first arrival (submission costs ~20 us each)

    def run(server, ids, arrivals):
        server.reset_stats()                        # epoch for the replayed arrival times
        for k in range(n_requests):
            o, n_, mid = int(offs[k]), int(sizes[k]), int(mids[k])
            side = handles[mid].desc.width
            server.submit(ids[mid], uv[o:o + n_], lods[side][o:o + n_], wi[o:o + n_], wo[o:o + n_],
                          outs[mid][o:o + n_], arrival_s=lead + float(arrivals[k]))
        server.wait_all()
        st = server.stats()
        server.reset_stats()
        return st

    result = {"workload": "8 resident materials, Poisson requests of 4096..8294400 queries (log-uniform), "
                          "device-resident inputs, 2 GiB in-flight budget, 4 streams, tiles of 1M queries",
              "requests": n_requests, "mean_queries": mean_q, "loads": {}}
    for prec_name, prec in (("fp16", nam.F16), ("fp32", nam.F32)):
        for h in handles:
            h.set_precision(prec)
        server = nam.Server(ctx, budget_bytes=budget, n_streams=4, max_tile=1 << 20)
        ids = [server.add_material(h) for h in handles]
        sat = run(server, ids, np.zeros(n_requests))
        rate_sat = sat["queries_per_s"] / mean_q
        entry = {"saturated_queries_per_s": sat["queries_per_s"], "saturated_launches": sat["launches"],
                 "saturated_tiles": sat["tiles"]}
        if prec_name == "fp16":
            # the same saturated run with one launch per tile (grouped launches off)
            server.set_group(1)
            one = run(server, ids, np.zeros(n_requests))
            server.set_group(8)
            entry["saturated_queries_per_s_one_launch_per_tile"] = one["queries_per_s"]
            log(f"serving fp16 saturated: {sat['queries_per_s'] / 1e9:.2f} G q/s grouped ({sat['tiles']} tiles in "
                f"{sat['launches']} launches), {one['queries_per_s'] / 1e9:.2f} G q/s one launch per tile")
        for load in ((0.5, 0.8, 1.1) if prec_name == "fp16" else (0.8,)):
            gaps = rng.exponential(1.0 / (load * rate_sat), n_requests)
            st = run(server, ids, np.cumsum(gaps) - gaps[0])
            entry[f"load_{load}"] = {"queries_per_s": st["queries_per_s"], "p50_ms": st["p50_s"] * 1e3,
                                     "p99_ms": st["p99_s"] * 1e3, "mean_ms": st["mean_s"] * 1e3,
                                     "peak_budget_bytes": st["peak_reserved_bytes"], "launches": st["launches"],
                                     "tiles": st["tiles"],
                                     "peak_requests_on_device": st["peak_requests_on_device"],
                                     "peak_launches_on_device": st["peak_launches_on_device"]}
            log(f"serving {prec_name} load {load}: {st['queries_per_s'] / 1e9:.2f} G q/s, "
                f"p50 {st['p50_s'] * 1e3:.2f} ms, p99 {st['p99_s'] * 1e3:.2f} ms, up to "
                f"{st['peak_requests_on_device']} requests in {st['peak_launches_on_device']} launches on the device")
        result["loads"][prec_name] = entry
        server.close()

    # mode (ii): the FP16 decoders fed from pinned host memory, the H2D and D2H copies inside
    # each request's latency (one shared pinned output buffer per material)
    for h in handles:
        h.set_precision(nam.F16)
    h_uv, h_wi, h_wo = (t.cpu().pin_memory() for t in (uv, wi, wo))
    h_lods = {side: t.cpu().pin_memory() for side, t in lods.items()}
    h_out = torch.empty((P, 3), dtype=torch.float32).pin_memory()
    server = nam.Server(ctx, budget_bytes=budget, n_streams=4, max_tile=1 << 20)
    ids = [server.add_material(h) for h in handles]

    def run_host(arrivals):
        server.reset_stats()
        for k in range(n_requests):
            o, n_, mid = int(offs[k]), int(sizes[k]), int(mids[k])
            side = handles[mid].desc.width
            server.submit(ids[mid], h_uv[o:o + n_], h_lods[side][o:o + n_], h_wi[o:o + n_], h_wo[o:o + n_],
                          h_out[o:o + n_], arrival_s=lead + float(arrivals[k]))
        server.wait_all()
        st = server.stats()
        server.reset_stats()
        return st

    sat = run_host(np.zeros(n_requests))
    rate_sat = sat["queries_per_s"] / mean_q
    entry = {"saturated_queries_per_s": sat["queries_per_s"]}
    gaps = rng.exponential(1.0 / (0.8 * rate_sat), n_requests)
    st = run_host(np.cumsum(gaps) - gaps[0])
    entry["load_0.8"] = {"queries_per_s": st["queries_per_s"], "p50_ms": st["p50_s"] * 1e3,
                         "p99_ms": st["p99_s"] * 1e3, "mean_ms": st["mean_s"] * 1e3,
                         "peak_budget_bytes": st["peak_reserved_bytes"]}
    log(f"serving fp16 host inputs: saturated {sat['queries_per_s'] / 1e9:.2f} G q/s; load 0.8: "
        f"p50 {st['p50_s'] * 1e3:.2f} ms, p99 {st['p99_s'] * 1e3:.2f} ms")
    result["loads"]["fp16_host_inputs"] = entry
    server.close()
    return result


if __name__ == "__main__":
    main()
