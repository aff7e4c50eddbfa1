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


class ModelDesc(ctypes.Structure):
    _fields_ = [("pyramid", PyramidDesc), ("mlp", MlpDesc), ("n_frames", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("queries", ctypes.c_int64), ("p50_s", ctypes.c_double),
                ("p99_s", ctypes.c_double), ("mean_s", ctypes.c_double), ("max_s", ctypes.c_double),
                ("span_s", ctypes.c_double), ("queries_per_s", ctypes.c_double),
                ("peak_reserved_bytes", ctypes.c_size_t), ("launches", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("peak_requests_on_device", ctypes.c_int64), ("peak_launches_on_device", ctypes.c_int64)]


class AdamCfg(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int64)]


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
    L.nam_material_set_sampler.argtypes = [vp, vp, ctypes.POINTER(MlpDesc), vp]
    L.nam_sampler_params.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    L.nam_sampler_pdf.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
    L.nam_sampler_sample.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp]
    L.nam_proxy_pdf.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    L.nam_proxy_sample.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.nam_server_set_group.argtypes = [vp, ctypes.c_int]
    L.nam_material_save.argtypes = [vp, ctypes.c_char_p]
    L.nam_material_load_file.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
    L.nam_material_load_framed.argtypes = [vp, ctypes.POINTER(PyramidDesc), ctypes.POINTER(vp),
                                           ctypes.POINTER(MlpDesc), vp, ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.nam_material_set_precision.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]
    L.nam_calibrate.argtypes = [vp, vp, i64, f32p, f32p, f32p, f32p, vp, vp]
    L.nam_material_footprint.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.nam_material_free.argtypes = [vp]
    L.nam_decode.argtypes = [vp, vp, i64, f32p, f32p, f32p, f32p, f32p, vp]
    L.nam_decode_stochastic.argtypes = [vp, vp, i64, f32p, f32p, f32p, f32p, f32p, f32p, vp]
    L.nam_fetch.argtypes = [vp, vp, i64, f32p, f32p, f32p, vp]
    L.nam_texel_footprint.argtypes = [vp, vp, i64, f32p, f32p, ctypes.POINTER(ctypes.c_uint64), vp]
    L.nam_texel_footprint_stochastic.argtypes = [vp, vp, i64, f32p, f32p, f32p, ctypes.POINTER(ctypes.c_uint64), vp]
    md = ctypes.POINTER(ModelDesc)
    L.nam_forward.argtypes = [vp, md, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    L.nam_backward.argtypes = [vp, md, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.nam_loss_backward.argtypes = [vp, md, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.nam_loss_backward_noalloc.argtypes = [vp, md, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.nam_loss_backward_codes.argtypes = [vp, md, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    mlp = ctypes.POINTER(MlpDesc)
    pd = ctypes.POINTER(PyramidDesc)
    L.nam_encode_texels.argtypes = [vp, mlp, vp, i64, vp, vp, vp]
    L.nam_encode_queries.argtypes = [vp, mlp, vp, pd, vp, i64, vp, vp, vp, vp]
    L.nam_encoder_backward.argtypes = [vp, mlp, vp, pd, vp, i64, vp, vp, vp, vp, vp]
    L.nam_adam_update.argtypes = [vp, i64, vp, vp, vp, vp, ctypes.POINTER(AdamCfg), vp]
    L.nam_set_deterministic.argtypes = [vp, ctypes.c_int]
    L.nam_train_step.argtypes = [vp, md, vp, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, ctypes.POINTER(AdamCfg),
                                 vp, vp]
    L.nam_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_int, i64, ctypes.POINTER(vp)]
    L.nam_server_add_material.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int)]
    L.nam_server_submit.argtypes = [vp, ctypes.c_int, i64, vp, vp, vp, vp, vp, ctypes.c_int, ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.nam_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    L.nam_server_cancel.argtypes = [vp, ctypes.c_uint64]
    L.nam_server_wait_all.argtypes = [vp]
    L.nam_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.nam_server_reset_stats.argtypes = [vp]
    L.nam_server_destroy.argtypes = [vp]
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

    def set_deterministic(self, on: bool = True) -> None:
        """Bitwise reproducible latent gradients in the training calls (nam_set_deterministic)."""
        check(lib().nam_set_deterministic(self.handle, 1 if on else 0))

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
                 address: int = WRAP, n_frames: int = 0, frame_params=None):
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
        self.n_frames = int(n_frames)
        if self.n_frames:
            fp = np.ascontiguousarray(frame_params, dtype=np.float32)
            check(lib().nam_material_load_framed(ctx.handle, ctypes.byref(self.desc), ptrs, ctypes.byref(mlp),
                                                 params.ctypes.data_as(ctypes.c_void_p), self.n_frames,
                                                 fp.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        else:
            check(lib().nam_material_load(ctx.handle, ctypes.byref(self.desc), ptrs, ctypes.byref(mlp),
                                          params.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self.handle = h

    def set_sampler(self, sdims, sparams):
        """nam_material_set_sampler: the importance-sampling decoder on [z, wi] (9 outputs)."""
        self.sdims = list(sdims)
        self._sdims_c = (ctypes.c_int * len(sdims))(*sdims)
        sp = np.ascontiguousarray(sparams, dtype=np.float32)
        check(lib().nam_material_set_sampler(self.ctx.handle, self.handle,
                                             ctypes.byref(MlpDesc(len(sdims) - 1, self._sdims_c)),
                                             sp.ctypes.data_as(ctypes.c_void_p)))

    def save(self, path: str):
        """nam_material_save: the FP32 master copy (pyramid, decoder, frames) to a file."""
        check(lib().nam_material_save(self.handle, os.fsencode(path)))

    @classmethod
    def load_file(cls, ctx: Context, path: str) -> "Material":
        """nam_material_load_file; the descriptors kept on the Python side are read back from the
        file's header."""
        h = ctypes.c_void_p()
        check(lib().nam_material_load_file(ctx.handle, os.fsencode(path), ctypes.byref(h)))
        with open(path, "rb") as f:
            head = np.frombuffer(f.read(8 + 4 * 6), dtype="<i4", offset=8)
            n_layers = int(head[5])
            dims = [int(v) for v in np.frombuffer(f.read(4 * (n_layers + 1)), dtype="<i4")]
            nf, s_layers = (int(v) for v in np.frombuffer(f.read(8), dtype="<i4"))
            sdims = [int(v) for v in np.frombuffer(f.read(4 * (s_layers + 1)), dtype="<i4")] if s_layers else None
        self = cls.__new__(cls)
        self.ctx = ctx
        self.desc = PyramidDesc(int(head[0]), int(head[1]), int(head[2]), int(head[3]), int(head[4]))
        self.dims = dims
        self.channels = int(head[2])
        self._dims_c = (ctypes.c_int * len(dims))(*dims)
        self.n_frames = nf
        if sdims:
            self.sdims = sdims
        self.handle = h
        return self

    @classmethod
    def from_workload(cls, ctx: Context, mat) -> "Material":
        return cls(ctx, mat.levels, mat.dims, mat.params, mat.address, getattr(mat, "n_frames", 0),
                   getattr(mat, "frame_params", None))

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


def sampler_params(mat: Material, uv, lod, wi, out=None, stream=None):
    """nam_sampler_params -> params [n, 9]."""
    import torch
    n = lod.shape[0]
    out = torch.empty((n, 9), dtype=torch.float32, device=lod.device) if out is None else out
    check(lib().nam_sampler_params(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                   _dev(wi, (3,), "wi"), _dev(out, (9,), "params"), _stream(stream)))
    return out


def sampler_pdf(mat: Material, uv, lod, wi, wo, out=None, stream=None):
    """nam_sampler_pdf -> pdf [n]."""
    import torch
    n = lod.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=lod.device) if out is None else out
    check(lib().nam_sampler_pdf(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"), _dev(out, (), "pdf"), _stream(stream)))
    return out


def sampler_sample(mat: Material, uv, lod, wi, u, stream=None):
    """nam_sampler_sample -> (wo [n, 3], pdf [n])."""
    import torch
    n = lod.shape[0]
    wo = torch.empty((n, 3), dtype=torch.float32, device=lod.device)
    pdf = torch.empty(n, dtype=torch.float32, device=lod.device)
    check(lib().nam_sampler_sample(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                   _dev(wi, (3,), "wi"), _dev(u, (3,), "u"), _dev(wo, (3,), "wo"),
                                   _dev(pdf, (), "pdf"), _stream(stream)))
    return wo, pdf


def proxy_pdf(ctx: Context, params, wi, wo, stream=None):
    """nam_proxy_pdf from cached proxy parameters -> pdf [n]."""
    import torch
    n = params.shape[0]
    pdf = torch.empty(n, dtype=torch.float32, device=params.device)
    check(lib().nam_proxy_pdf(ctx.handle, n, _dev(params, (9,), "params"), _dev(wi, (3,), "wi"),
                              _dev(wo, (3,), "wo"), _dev(pdf, (), "pdf"), _stream(stream)))
    return pdf


def proxy_sample(ctx: Context, params, wi, u, stream=None):
    """nam_proxy_sample from cached proxy parameters -> (wo [n, 3], pdf [n])."""
    import torch
    n = params.shape[0]
    wo = torch.empty((n, 3), dtype=torch.float32, device=params.device)
    pdf = torch.empty(n, dtype=torch.float32, device=params.device)
    check(lib().nam_proxy_sample(ctx.handle, n, _dev(params, (9,), "params"), _dev(wi, (3,), "wi"),
                                 _dev(u, (3,), "u"), _dev(wo, (3,), "wo"), _dev(pdf, (), "pdf"), _stream(stream)))
    return wo, pdf


def decode(mat: Material, uv, lod, wi, wo, out=None, stream=None, xi=None):
    """nam_decode; with `xi` (one draw per query) nam_decode_stochastic, the level chosen by
    Russian roulette.  out [n][3], or [n][6] (RGB, then albedo) for a decoder with the albedo
    head."""
    import torch
    n = lod.shape[0]
    ko = mat.dims[-1]
    if out is None:
        out = torch.empty((n, ko), dtype=torch.float32, device=lod.device)
    if xi is None:
        check(lib().nam_decode(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                               _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"), _dev(out, (ko,), "rgb"), _stream(stream)))
    else:
        check(lib().nam_decode_stochastic(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                          _dev(xi, (), "xi"), _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"),
                                          _dev(out, (ko,), "rgb"), _stream(stream)))
    return out


def fetch(mat: Material, uv, lod, out=None, stream=None):
    import torch
    n = lod.shape[0]
    if out is None:
        out = torch.empty((n, mat.channels), dtype=torch.float32, device=lod.device)
    check(lib().nam_fetch(mat.ctx.handle, mat.handle, n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                          _dev(out, (mat.channels,), "z"), _stream(stream)))
    return out


def texel_footprint(mat: Material, uv, lod, stream=None, xi=None) -> int:
    """Distinct texels the decode's taps address (with `xi`: the Russian-roulette taps)."""
    out = ctypes.c_uint64(0)
    if xi is None:
        check(lib().nam_texel_footprint(mat.ctx.handle, mat.handle, lod.shape[0], _dev(uv, (2,), "uv"),
                                        _dev(lod, (), "lod"), ctypes.byref(out), _stream(stream)))
    else:
        check(lib().nam_texel_footprint_stochastic(mat.ctx.handle, mat.handle, lod.shape[0], _dev(uv, (2,), "uv"),
                                                   _dev(lod, (), "lod"), _dev(xi, (), "xi"), ctypes.byref(out),
                                                   _stream(stream)))
    return out.value


def to_device(q, device="cuda"):
    """Queries (numpy) -> contiguous float32 CUDA tensors (uv, lod, wi, wo)."""
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
                 for a in (q.uv, q.lod, q.wi, q.wo))


# ------------------------------------------------------------------------------------------
# differentiation


def concat_levels(levels) -> np.ndarray:
    """Pyramid levels [H_l][W_l][C] -> one [texels][C] float32 array, level 0 first."""
    return np.ascontiguousarray(np.concatenate([l.reshape(-1, l.shape[-1]) for l in levels]), dtype=np.float32)


def split_levels(flat, width, height, n_levels):
    """Inverse of concat_levels (views into `flat`)."""
    out, o = [], 0
    for l in range(n_levels):
        w, h = max(1, width >> l), max(1, height >> l)
        out.append(flat[o:o + w * h].reshape(h, w, -1))
        o += w * h
    return out


class Model:
    """Shape of a trainable neural material (pyramid + decoder); tensors are the caller's."""

    def __init__(self, ctx: Context, width, height, channels, n_levels, dims, address=WRAP, n_frames=0):
        """n_frames > 0: learned shading frames, trained with the decoder; the parameter tensor
        then holds the frame layer (W_F[6N][C], b_F[6N]) ahead of the packed decoder."""
        self.ctx = ctx
        self.width, self.height, self.channels, self.n_levels = width, height, channels, n_levels
        self.dims = list(dims)
        self.n_frames = n_frames
        self._dims_c = (ctypes.c_int * len(dims))(*dims)
        self.desc = ModelDesc(PyramidDesc(width, height, channels, n_levels, address),
                              MlpDesc(len(dims) - 1, self._dims_c), n_frames)
        self.texel_count = sum(max(1, width >> l) * max(1, height >> l) for l in range(n_levels))
        self.frame_param_count = 6 * n_frames * channels + 6 * n_frames
        self.param_count = self.frame_param_count + sum(dims[k] * dims[k + 1] + dims[k + 1]
                                                        for k in range(len(dims) - 1))

    @classmethod
    def from_workload(cls, ctx, mat):
        return cls(ctx, mat.width, mat.height, mat.channels, mat.n_levels, mat.dims, mat.address,
                   getattr(mat, "n_frames", 0))

    def _check(self, texels, params):
        _dev(texels, (self.channels,), "texels")
        _dev(params, (), "params")
        if texels.shape[0] != self.texel_count or params.shape[0] != self.param_count:
            raise ValueError("texels / params do not match the model shape")

    def forward(self, texels, params, uv, lod, wi, wo, stream=None):
        import torch
        self._check(texels, params)
        n = lod.shape[0]
        ko = self.dims[-1]
        rgb = torch.empty((n, ko), dtype=torch.float32, device=lod.device)
        check(lib().nam_forward(self.ctx.handle, ctypes.byref(self.desc), _dev(texels, (self.channels,), "texels"),
                                _dev(params, (), "params"), n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"), _dev(rgb, (ko,), "rgb"), _stream(stream)))
        return rgb

    def backward(self, texels, params, uv, lod, wi, wo, d_rgb, d_texels=None, stream=None):
        """(d_texels += dL/dtexels, d_params = dL/dparams) for d_rgb = dL/drgb."""
        import torch
        self._check(texels, params)
        n = lod.shape[0]
        if d_texels is None:
            d_texels = torch.zeros_like(texels)
        d_params = torch.empty_like(params)
        check(lib().nam_backward(self.ctx.handle, ctypes.byref(self.desc), _dev(texels, (self.channels,), "texels"),
                                 _dev(params, (), "params"), n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"),
                                 _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"), _dev(d_rgb, (self.dims[-1],), "d_rgb"),
                                 _dev(d_texels, (self.channels,), "d_texels"), _dev(d_params, (), "d_params"),
                                 _stream(stream)))
        return d_texels, d_params

    def loss_backward(self, texels, params, uv, lod, wi, wo, target, d_texels=None, stream=None,
                      d_params=None, loss=None, noalloc=False):
        """Mean squared error against target: (loss tensor [1], d_texels (+=), d_params).
        noalloc=True calls nam_loss_backward_noalloc (the library allocates nothing; pass the
        output tensors to keep this call free of allocations too)."""
        import torch
        self._check(texels, params)
        n = lod.shape[0]
        if d_texels is None:
            d_texels = torch.zeros_like(texels)
        if d_params is None:
            d_params = torch.empty_like(params)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=lod.device)
        fn = lib().nam_loss_backward_noalloc if noalloc else lib().nam_loss_backward
        check(fn(self.ctx.handle, ctypes.byref(self.desc), _dev(texels, (self.channels,), "texels"),
                 _dev(params, (), "params"), n, _dev(uv, (2,), "uv"), _dev(lod, (), "lod"), _dev(wi, (3,), "wi"),
                 _dev(wo, (3,), "wo"), _dev(target, (self.dims[-1],), "target"),
                 _dev(d_texels, (self.channels,), "d_texels"), _dev(d_params, (), "d_params"),
                 ctypes.c_void_p(loss.data_ptr()), _stream(stream)))
        return loss, d_texels, d_params


    def loss_backward_codes(self, params, z, wi, wo, target, stream=None):
        """The decoder's mean squared error on given latent codes z [n, C] (the encoder's first
        training phase): (loss tensor [1], dz [n, C], d_params)."""
        import torch
        _dev(params, (), "params")
        n = z.shape[0]
        dz = torch.empty_like(z)
        d_params = torch.empty_like(params)
        loss = torch.empty(1, dtype=torch.float32, device=z.device)
        check(lib().nam_loss_backward_codes(self.ctx.handle, ctypes.byref(self.desc), _dev(params, (), "params"), n,
                                            _dev(z, (self.channels,), "z"), _dev(wi, (3,), "wi"), _dev(wo, (3,), "wo"),
                                            _dev(target, (self.dims[-1],), "target"), _dev(dz, (self.channels,), "dz"),
                                            _dev(d_params, (), "d_params"), ctypes.c_void_p(loss.data_ptr()),
                                            _stream(stream)))
        return loss, dz, d_params


class Encoder:
    """The encoder of Sec. 5.1 (dims [A, H, (H,) C]) over a pyramid of the material's
    parameters (A channels, levels concatenated); its parameters are the caller's tensor."""

    def __init__(self, ctx: Context, dims, width, height, n_levels, address=WRAP):
        self.ctx = ctx
        self.dims = list(dims)
        self.A, self.C = dims[0], dims[-1]
        self._dims_c = (ctypes.c_int * len(dims))(*dims)
        self.mlp = MlpDesc(len(dims) - 1, self._dims_c)
        self.pyramid = PyramidDesc(width, height, self.A, n_levels, address)
        self.param_count = sum(dims[k] * dims[k + 1] + dims[k + 1] for k in range(len(dims) - 1))

    def encode_texels(self, eparams, attrs, stream=None):
        """z [n, C] = E(attrs [n, A]): the bake of the latent texture."""
        import torch
        z = torch.empty((attrs.shape[0], self.C), dtype=torch.float32, device=attrs.device)
        check(lib().nam_encode_texels(self.ctx.handle, ctypes.byref(self.mlp), _dev(eparams, (), "eparams"),
                                      attrs.shape[0], _dev(attrs, (self.A,), "attrs"), _dev(z, (self.C,), "z"),
                                      _stream(stream)))
        return z

    def encode_queries(self, eparams, attrs, uv, lod, stream=None):
        """z [n, C] = E(parameters filtered at (uv, lod))."""
        import torch
        n = lod.shape[0]
        z = torch.empty((n, self.C), dtype=torch.float32, device=lod.device)
        check(lib().nam_encode_queries(self.ctx.handle, ctypes.byref(self.mlp), _dev(eparams, (), "eparams"),
                                       ctypes.byref(self.pyramid), _dev(attrs, (self.A,), "attrs"), n,
                                       _dev(uv, (2,), "uv"), _dev(lod, (), "lod"), _dev(z, (self.C,), "z"),
                                       _stream(stream)))
        return z

    def backward(self, eparams, attrs, uv, lod, dz, stream=None):
        """The gradient of sum_i dz_i . E(parameters filtered at query i) for the encoder's
        parameters."""
        import torch
        d = torch.empty_like(eparams)
        check(lib().nam_encoder_backward(self.ctx.handle, ctypes.byref(self.mlp), _dev(eparams, (), "eparams"),
                                         ctypes.byref(self.pyramid), _dev(attrs, (self.A,), "attrs"), lod.shape[0],
                                         _dev(uv, (2,), "uv"), _dev(lod, (), "lod"), _dev(dz, (self.C,), "dz"),
                                         _dev(d, (), "d_eparams"), _stream(stream)))
        return d


def adam_update(ctx: Context, p, m, v, g, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    cfg = AdamCfg(lr, beta1, beta2, eps, step)
    for t, name in ((p, "p"), (m, "m"), (v, "v"), (g, "g")):
        if not t.is_cuda or t.dtype.itemsize != 4 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    check(lib().nam_adam_update(ctx.handle, p.numel(), ctypes.c_void_p(p.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(g.data_ptr()), ctypes.byref(cfg),
                                _stream(stream)))


class Trainer:
    """Trainable texels and decoder with Adam state on the device; one nam_train_step per
    batch (loss and gradients of the mean squared error, then Adam on everything)."""

    def __init__(self, model: Model, texels, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        self.model = model
        self.texels = texels
        self.params = params
        self.m_tex = torch.zeros_like(texels)
        self.v_tex = torch.zeros_like(texels)
        self.m_par = torch.zeros_like(params)
        self.v_par = torch.zeros_like(params)
        self.cfg = [lr, beta1, beta2, eps]
        self.step_count = 0
        self.loss = torch.zeros(1, dtype=torch.float32, device=texels.device)

    def step(self, uv, lod, wi, wo, target, stream=None):
        self.step_count += 1
        cfg = AdamCfg(*self.cfg, self.step_count)
        md = self.model
        check(lib().nam_train_step(md.ctx.handle, ctypes.byref(md.desc),
                                   _dev(self.texels, (md.channels,), "texels"), _dev(self.params, (), "params"),
                                   _dev(self.m_tex, (md.channels,), "m_texels"),
                                   _dev(self.v_tex, (md.channels,), "v_texels"),
                                   _dev(self.m_par, (), "m_params"), _dev(self.v_par, (), "v_params"),
                                   lod.shape[0], _dev(uv, (2,), "uv"), _dev(lod, (), "lod"), _dev(wi, (3,), "wi"),
                                   _dev(wo, (3,), "wo"), _dev(target, (md.dims[-1],), "target"), ctypes.byref(cfg),
                                   ctypes.c_void_p(self.loss.data_ptr()), _stream(stream)))
        return self.loss


def _make_autograd():
    import torch

    class NeuralMaterialFn(torch.autograd.Function):
        """rgb = decode(texels, params; uv, lod, wi, wo) with the hand-written backward:
        gradients flow to the concatenated texels and the packed parameters only."""

        @staticmethod
        def forward(ctx, texels, params, uv, lod, wi, wo, model):
            ctx.save_for_backward(texels, params, uv, lod, wi, wo)
            ctx.model = model
            return model.forward(texels, params, uv, lod, wi, wo)

        @staticmethod
        def backward(ctx, d_rgb):
            texels, params, uv, lod, wi, wo = ctx.saved_tensors
            d_tex, d_par = ctx.model.backward(texels, params, uv, lod, wi, wo, d_rgb.contiguous())
            return d_tex, d_par, None, None, None, None, None

    return NeuralMaterialFn


_autograd_fn = None


def neural_material(texels, params, uv, lod, wi, wo, model: Model):
    """Differentiable decode (torch.autograd) through the library's forward and backward."""
    global _autograd_fn
    if _autograd_fn is None:
        _autograd_fn = _make_autograd()
    return _autograd_fn.apply(texels, params, uv, lod, wi, wo, model)


# ------------------------------------------------------------------------------------------
# serving


class Server:
    """Continuous-batching request loop over resident materials (see nam_server_* in nam.h)."""

    def __init__(self, ctx: Context, budget_bytes=2 << 30, n_streams=4, max_tile=1 << 20):
        h = ctypes.c_void_p()
        check(lib().nam_server_create(ctx.handle, budget_bytes, n_streams, max_tile, ctypes.byref(h)))
        self.handle = h
        self.ctx = ctx
        self._materials = []
        self._keep = {}

    def add_material(self, mat: Material) -> int:
        mid = ctypes.c_int(0)
        check(lib().nam_server_add_material(self.handle, mat.handle, ctypes.byref(mid)))
        self._materials.append(mat)
        return mid.value

    def submit(self, material_id, uv, lod, wi, wo, rgb, arrival_s=None) -> int:
        """Device tensors (host_io = 0) or pinned host tensors (host_io = 1, detected).
        arrival_s: None = now, else seconds after the server epoch (creation / reset_stats)."""
        host = not rgb.is_cuda
        n = lod.shape[0]
        ko = self._materials[material_id].dims[-1] if 0 <= material_id < len(self._materials) else 3
        for t, tail, name in ((uv, (2,), "uv"), (lod, (), "lod"), (wi, (3,), "wi"), (wo, (3,), "wo"),
                              (rgb, (ko,), "rgb")):
            if t.is_cuda == host or not t.is_contiguous() or tuple(t.shape[1:]) != tail:
                raise ValueError(f"{name}: all buffers on one side (host or device), contiguous, [n{', ' if tail else ''}"
                                 f"{', '.join(map(str, tail))}]")
        tk = ctypes.c_uint64(0)
        check(lib().nam_server_submit(self.handle, material_id, n, ctypes.c_void_p(uv.data_ptr()),
                                      ctypes.c_void_p(lod.data_ptr()), ctypes.c_void_p(wi.data_ptr()),
                                      ctypes.c_void_p(wo.data_ptr()), ctypes.c_void_p(rgb.data_ptr()), int(host),
                                      -1.0 if arrival_s is None else float(arrival_s), ctypes.byref(tk)))
        self._keep[tk.value] = (uv, lod, wi, wo, rgb)
        return tk.value

    def poll(self, ticket):
        done, lat = ctypes.c_int(0), ctypes.c_double(0.0)
        check(lib().nam_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(lat)))
        return bool(done.value), lat.value

    def cancel(self, ticket):
        check(lib().nam_server_cancel(self.handle, ticket))

    def wait_all(self):
        check(lib().nam_server_wait_all(self.handle))

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().nam_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def set_group(self, max_tiles: int):
        """nam_server_set_group: tiles per grouped launch (1 = one launch per tile)."""
        check(lib().nam_server_set_group(self.handle, int(max_tiles)))

    def reset_stats(self):
        check(lib().nam_server_reset_stats(self.handle))
        self._keep.clear()

    def close(self):
        if self.handle:
            check(lib().nam_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
