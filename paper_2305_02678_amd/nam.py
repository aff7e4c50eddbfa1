"""Python binding of libnam (ctypes).  Argument marshalling only: every step of the decode
runs in the library's HIP kernels.  PyTorch supplies device memory and streams.

The library must be built (``python -m paper_2305_02678_amd.build`` or
``__graft_entry__.build()``); loading fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnam.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "nam.h")

NAM_OK, NAM_E_INVALID_ARG, NAM_E_SHAPE, NAM_E_UNSUPPORTED, NAM_E_OOM, NAM_E_BUDGET, NAM_E_HIP, NAM_E_BUSY, NAM_E_IO = range(9)
STATUS_NAMES = ["NAM_OK", "NAM_E_INVALID_ARG", "NAM_E_SHAPE", "NAM_E_UNSUPPORTED", "NAM_E_OOM", "NAM_E_BUDGET",
                "NAM_E_HIP", "NAM_E_BUSY", "NAM_E_IO"]
WRAP, CLAMP = 0, 1
F32, F16, FP8_E4M3 = 0, 1, 2


class NamError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {message}")


class PyramidDesc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("height", ctypes.c_int), ("channels", ctypes.c_int),
                ("levels", ctypes.c_int), ("address", ctypes.c_int)]


class MlpDesc(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int), ("dims", ctypes.POINTER(ctypes.c_int))]


_lib = None


def header_functions() -> List[str]:
    """Names of the functions declared in include/nam.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:nam_status|const char\*|int)\s+(nam_\w+)\s*\(", text, re.M)))


def lib(build_if_missing: bool = False):
    """Load libnam.so once.  torch is imported first so that the library binds to the HIP
    runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime first)
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"libnam is not built ({LIB_PATH} missing); run python -m paper_2305_02678_amd.build")
        from . import build as _b
        _b.build()
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, f32p = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
    L.nam_last_error.restype = ctypes.c_char_p
    L.nam_version.restype = ctypes.c_int
    for name in header_functions():
        fn = getattr(L, name)
        if name not in ("nam_last_error", "nam_version"):
            fn.restype = ctypes.c_int
    L.nam_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
    L.nam_destroy.argtypes = [vp]
    L.nam_pyramid_bytes.argtypes = [ctypes.POINTER(PyramidDesc), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.nam_material_load.argtypes = [vp, ctypes.POINTER(PyramidDesc), ctypes.POINTER(vp), ctypes.POINTER(MlpDesc),
                                    vp, ctypes.POINTER(vp)]
    L.nam_material_set_precision.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]
    L.nam_calibrate.argtypes = [vp, vp, i64, f32p, f32p, f32p, f32p, vp, vp]
    L.nam_material_footprint.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.nam_material_free.argtypes = [vp]
    L.nam_decode.argtypes = [vp, vp, i64, f32p, f32p, f32p, f32p, f32p, vp]
    L.nam_fetch.argtypes = [vp, vp, i64, f32p, f32p, f32p, vp]
    L.nam_texel_footprint.argtypes = [vp, vp, i64, f32p, f32p, ctypes.POINTER(ctypes.c_uint64), vp]
    _lib = L
    return L


def check(status: int):
    if status != NAM_OK:
        raise NamError(status, lib().nam_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, shape_tail, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n, {', '.join(map(str, shape_tail))}]")
    return ctypes.c_void_p(t.data_ptr())


def pyramid_bytes(width, height, channels, levels, texel_type=F16, address=WRAP) -> int:
    d = PyramidDesc(width, height, channels, levels, address)
    out = ctypes.c_size_t(0)
    check(lib().nam_pyramid_bytes(ctypes.byref(d), texel_type, ctypes.byref(out)))
    return out.value


class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        check(lib().nam_create(device, ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            check(lib().nam_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Material:
    """A latent pyramid plus decoder resident on the device."""

    def __init__(self, ctx: Context, levels: Sequence[np.ndarray], dims: Sequence[int], params: np.ndarray,
                 address: int = WRAP):
        levels = [np.ascontiguousarray(l, dtype=np.float32) for l in levels]
        H, W, C = levels[0].shape
        self.ctx = ctx
        self.desc = PyramidDesc(W, H, C, len(levels), address)
        self.dims = list(dims)
        self.channels = C
        self._dims_c = (ctypes.c_int * len(dims))(*dims)
        mlp = MlpDesc(len(dims) - 1, self._dims_c)
        ptrs = (ctypes.c_void_p * len(levels))(*[l.ctypes.data for l in levels])
        params = np.ascontiguousarray(params, dtype=np.float32)
        h = ctypes.c_void_p()
        check(lib().nam_material_load(ctx.handle, ctypes.byref(self.desc), ptrs, ctypes.byref(mlp),
                                      params.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.handle = h

    @classmethod
    def from_workload(cls, ctx: Context, mat) -> "Material":
        return cls(ctx, mat.levels, mat.dims, mat.params, mat.address)

    def set_precision(self, weights: int, texels: Optional[int] = None, act_absmax=None, first_layer_f16=False):
        if texels is None:
            texels = F32 if weights == F32 else F16
        am = None
        if act_absmax is not None:
            am = np.ascontiguousarray(act_absmax, dtype=np.float32)
        check(lib().nam_material_set_precision(self.ctx.handle, self.handle, weights, texels,
                                               am.ctypes.data_as(ctypes.c_void_p) if am is not None else None,
                                               int(bool(first_layer_f16))))

    def calibrate(self, uv, lod, wi, wo, stream=None) -> np.ndarray:
        n = lod.shape[0]
        out = np.zeros(len(self.dims) - 1, np.float32)
        check(lib().nam_calibrate(self.ctx.handle, self.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                  _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"),
                                  out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return out

    def footprint(self) -> int:
        out = ctypes.c_size_t(0)
        check(lib().nam_material_footprint(self.handle, ctypes.byref(out)))
        return out.value

    def free(self):
        if self.handle:
            check(lib().nam_material_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def decode(mat: Material, uv, lod, wi, wo, out=None, stream=None):
    import torch
    n = lod.shape[0]
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device=lod.device)
    check(lib().nam_decode(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                           _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"), _dev(out, (3,), "rgb"), _stream(stream)))
    return out


def fetch(mat: Material, uv, lod, out=None, stream=None):
    import torch
    n = lod.shape[0]
    if out is None:
        out = torch.empty((n, mat.channels), dtype=torch.float32, device=lod.device)
    check(lib().nam_fetch(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                          _dev(out, (mat.channels,), "z"), _stream(stream)))
    return out


def texel_footprint(mat: Material, uv, lod, stream=None) -> int:
    out = ctypes.c_uint64(0)
    check(lib().nam_texel_footprint(mat.ctx.handle, mat.handle, lod.shape[0], _dev(uv, (2,), "uv"),
                                    _dev(lod, (), "lod"), ctypes.byref(out), _stream(stream)))
    return out.value


def to_device(q, device="cuda"):
    """Queries (numpy) -> contiguous float32 CUDA tensors (uv, lod, wi, wo)."""
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
                 for a in (q.uv, q.lod, q.wi, q.wo))
