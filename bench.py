"""Decode-throughput benchmark of the neural appearance hot path on one MI355X.

One step = one fused decode (latent fetch + concatenation + decoder + softplus) of a full
1920x1080 frame of shading queries against a 2048^2 x 16-channel latent pyramid (full mip
chain) with a 22-64-64-64-3 decoder, inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp16|fp32|fp8]
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
PEAK_TFLOPS = {"f32_valu": 157.3, "f16_mfma": 2500.0, "fp8_mfma": 5000.0}


def algorithmic_flops_per_query(dims):
    return sum(2 * dims[k] * dims[k + 1] for k in range(len(dims) - 1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_cpu_oracle(w, target_s=15.0, max_n=None):
    """The FP64 oracle on a bounded sample of the same frame, all host threads."""
    import oracle
    m, q = w.material, w.queries
    lv64 = [l.astype(np.float64) for l in m.levels]          # conversion kept out of the timing
    probe = q.subset(slice(0, 8192))
    t0 = time.perf_counter()
    oracle.decode(lv64, m.dims, m.params, probe.uv, probe.lod, probe.wi, probe.wo)
    rate = 8192 / (time.perf_counter() - t0)
    n = int(min(len(q), max(8192, rate * target_s)))
    if max_n:
        n = min(n, max_n)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(len(q), n, replace=False))
    s = q.subset(idx)
    t0 = time.perf_counter()
    ref = oracle.decode(lv64, m.dims, m.params, s.uv, s.lod, s.wi, s.wo)
    dt = time.perf_counter() - t0
    return idx, ref, {"value": n / dt, "unit": "queries/s", "cores": oracle.threads(), "kind": "oracle",
                      "sample": f"{n} of {len(q)} frame queries (random, seed 7), FP64 C oracle, "
                                f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "fp8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the decode path is measured on a single MI355X "
              "(queries are independent; a multi-GPU split would give each GPU its own share of the frame).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_02678_amd import nam
    from paper_2305_02678_amd import workloads as wl

    t0 = time.time()
    w = wl.frame()
    m, q = w.material, w.queries
    N = len(q)
    log(f"workload generated in {time.time() - t0:.1f} s: {w.name}, {N} queries")

    ctx = nam.Context(0)
    mat = nam.Material.from_workload(ctx, m)
    uv, lod, wi, wo = nam.to_device(q)
    prec = {"fp32": nam.F32, "fp16": nam.F16, "fp8": nam.FP8_E4M3}[args.precision]
    if prec == nam.FP8_E4M3:
        calib = wl.frame(seed=99, n=65536)
        am = mat.calibrate(*nam.to_device(calib.queries))
        mat.set_precision(prec, act_absmax=am)
    elif prec != nam.F32:
        mat.set_precision(prec)
    rgb = torch.empty((N, 3), device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        nam.decode(mat, uv, lod, wi, wo, out=rgb)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        nam.decode(mat, uv, lod, wi, wo, out=rgb)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    per = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])  # ms, per launch
    ms_step = wall * 1e3 / args.steps
    value = N / (wall / args.steps)

    # cold-cache latency: a 1 GiB write between launches evicts the 256 MB Infinity Cache
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    cold = []
    for k in range(min(args.steps, 20)):
        flush.fill_(float(k))
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        nam.decode(mat, uv, lod, wi, wo, out=rgb)
        e.record(stream)
        torch.cuda.synchronize()
        cold.append(s.elapsed_time(e))
    del flush

    # algorithmic traffic and work of one launch
    U = nam.texel_footprint(mat, uv, lod)
    tex_bytes = {nam.F32: 4, nam.F16: 2, nam.FP8_E4M3: 2}[prec]
    wbytes = {nam.F32: 4, nam.F16: 2, nam.FP8_E4M3: 1}[prec] * m.params.size
    B = N * (36 + 12) + U * m.channels * tex_bytes + wbytes
    F = N * algorithmic_flops_per_query(m.dims)
    t_launch = per.mean() * 1e-3
    peak_f = PEAK_TFLOPS[{nam.F32: "f32_valu", nam.F16: "f16_mfma", nam.FP8_E4M3: "fp8_mfma"}[prec]]
    t_hbm = B / (PEAK_HBM_GBS * 1e9)
    t_flop = F / (peak_f * 1e12)
    if prec == nam.F32:
        roof = {"bound": "alu", "achieved": F / t_launch / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    elif t_hbm >= t_flop:
        roof = {"bound": "hbm", "achieved": B / t_launch / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": F / t_launch / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["algorithmic_bytes"] = B
    roof["algorithmic_flops"] = F
    roof["distinct_texels"] = U
    roof["kernel_ms"] = per.mean()

    out = {
        "metric": METRIC, "value": value, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "fp16": "f16", "fp8": "fp8_e4m3"}[args.precision],
        "data": "synthetic",
        "config": {"workload": w.name + f", decoder {args.precision}" +
                   (", texels fp16" if prec != nam.F32 else ", texels fp32"),
                   "queries": N, "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99)),
                       "cold_p50": float(np.percentile(cold, 50)), "cold_p99": float(np.percentile(cold, 99))},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        idx, ref, cpu = time_cpu_oracle(w, args.cpu_seconds)
        got = rgb.cpu().numpy()[idx].astype(np.float64)
        e = np.abs(got - ref) / np.abs(ref)
        out["cpu_baseline"] = cpu
        out["error_vs_oracle"] = {"max_rel": float(e.max()), "mean_rel": float(e.mean()), "samples": int(len(idx))}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
