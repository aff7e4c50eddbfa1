"""Decode-throughput benchmark of the neural appearance hot path on one MI355X.

One step = one fused decode (latent fetch + concatenation + decoder + softplus) of a full
1920x1080 frame of shading queries against a 2048^2 x 16-channel latent pyramid (full mip
chain) with a 22-64-64-64-3 decoder, inputs resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

The headline is the FP16 matrix-core decode; the FP32 (vector ALU) and E4M3 decodes of the
same frame are timed beside it, each with its error against the FP64 oracle.
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
    return ref, {"value": len(q) / med, "unit": "queries/s", "cores": oracle.threads(), "kind": "oracle",
                 "sample": f"the full frame ({len(q)} queries), {len(times)} passes of the FP64 C oracle "
                           f"(median {med:.2f} s per pass, {sum(times):.1f} s in total)"}


def run_precision(nam, torch, mat, dq, N, prec, steps, warmup, am=None, first16=False):
    if prec == nam.F32:
        mat.set_precision(nam.F32)
    elif prec == nam.F16:
        mat.set_precision(nam.F16)
    else:
        mat.set_precision(nam.FP8_E4M3, act_absmax=am, first_layer_f16=first16)
    uv, lod, wi, wo = dq
    rgb = torch.empty((N, 3), device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        nam.decode(mat, uv, lod, wi, wo, out=rgb)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        nam.decode(mat, uv, lod, wi, wo, out=rgb)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])   # ms per launch
    # cold-cache latency: a 1 GiB write between launches evicts the 256 MB Infinity Cache
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    cold = []
    for k in range(min(steps, 20)):
        flush.fill_(float(k))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        nam.decode(mat, uv, lod, wi, wo, out=rgb)
        b.record(stream)
        torch.cuda.synchronize()
        cold.append(a.elapsed_time(b))
    del flush
    return {"qps": N / (wall / steps), "ms_per_step": wall * 1e3 / steps, "kernel_ms": float(per.mean()),
            "p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99)),
            "cold_p50_ms": float(np.percentile(cold, 50)), "cold_p99_ms": float(np.percentile(cold, 99)),
            "rgb": rgb}


def roofline(prec_name, N, U, C, n_params, dims, kernel_ms):
    tex_bytes = 4 if prec_name == "fp32" else 2
    wbytes = {"fp32": 4, "fp16": 2, "fp8": 1}[prec_name] * n_params
    B = N * (36 + 12) + U * C * tex_bytes + wbytes
    F = N * algorithmic_flops_per_query(dims)
    t = kernel_ms * 1e-3
    peak_f = PEAK_TFLOPS[{"fp32": "f32_valu", "fp16": "f16_mfma", "fp8": "fp8_mfma"}[prec_name]]
    t_hbm, t_flop = B / (PEAK_HBM_GBS * 1e9), F / (peak_f * 1e12)
    if prec_name == "fp32":
        r = {"bound": "alu", "achieved": F / t / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    elif t_hbm >= t_flop:
        r = {"bound": "hbm", "achieved": B / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        r = {"bound": "mfma", "achieved": F / t / 1e12, "peak": peak_f, "unit": "TFLOP/s"}
    r["frac"] = r["achieved"] / r["peak"]
    r["traffic"] = None
    r.update({"algorithmic_bytes": B, "algorithmic_flops": F, "distinct_texels": U, "kernel_ms": kernel_ms,
              "t_hbm_floor_us": t_hbm * 1e6, "t_compute_floor_us": t_flop * 1e6})
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--counters-pass", choices=["fp16", "fp32", "fp8"], default=None,
                    help="short run for hardware-counter collection: 3 decodes of the frame in one precision, "
                         "then a 256 MiB device-to-device copy whose byte count calibrates the counters")
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
    dq = nam.to_device(q)
    U = nam.texel_footprint(mat, dq[0], dq[1])
    calib = wl.frame(seed=99, n=65536)
    am = mat.calibrate(*nam.to_device(calib.queries))

    if args.counters_pass:
        prec = {"fp16": nam.F16, "fp32": nam.F32, "fp8": nam.FP8_E4M3}[args.counters_pass]
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
        entry["roofline"] = roofline(name, N, U, m.channels, m.params.size, m.dims, r["kernel_ms"])
        if ref is not None:
            e = np.abs(r["rgb"] - ref) / np.abs(ref)
            entry["error_vs_oracle"] = {"max_rel": float(e.max()), "mean_rel": float(e.mean()), "samples": int(e.size)}
        out["compare"][name] = entry
    if ref is not None:
        out["error_vs_oracle"] = out["compare"]["fp16"]["error_vs_oracle"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
