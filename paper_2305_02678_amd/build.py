"""Build libnam.so for gfx950 with hipcc (one object per source, compiled in parallel)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libnam.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# the matrix-core kernel families take longest and start first
SOURCES = ["train_mfma.hip", "decode_mfma.hip", "decode_mfma_frames.hip", "decode_mfma_albedo.hip", "decode_mfma_frames_albedo.hip",
           "sampler_mfma.hip", "encoder.hip", "train.hip", "train_frames.hip", "decode_f32.hip", "sampler.hip", "fetch.hip", "api.cpp", "material_file.cpp", "precision.cpp",
           "train_api.cpp", "server.cpp"]

# stand-alone measurement programs (probes/), built into _build/ beside the objects
PROBES = ["issue_cost.hip"]

# gfx950 only; packed-FP32 instructions are disabled (the compiler still uses scalar FP32).
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _compile_probe(src: str) -> str:
    exe = os.path.join(BUILD, os.path.splitext(src)[0])
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", os.path.join(HERE, "probes", src), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for probes/{src}:\n{r.stderr}")
    return exe


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        probes = [ex.submit(_compile_probe, p) for p in PROBES]
        objs = list(ex.map(_compile, SOURCES))
        for f in probes:
            f.result()
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
