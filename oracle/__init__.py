"""FP64 CPU oracle of the neural appearance decode path (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import
this package; the HIP library never does, and this package imports nothing from it.

The arithmetic lives in ``nam_oracle.c`` (plain C, double precision, OpenMP over
queries).  This module only marshals numpy arrays: every floating input is converted to
float64 (exactly, from its stored float32/float16 value) before the call.  ``twin.py`` is
an independent brute-force numpy formulation of the fetch used to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nam_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

WRAP, CLAMP = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Pyr(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("height", ctypes.c_int), ("channels", ctypes.c_int),
                ("n_levels", ctypes.c_int), ("address", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        _lib.orc_proxy_pdf.restype = ctypes.c_double
        _lib.orc_proxy_sample.restype = ctypes.c_double
        _lib.orc_round_fp16.restype = ctypes.c_double
        _lib.orc_round_fp16.argtypes = [ctypes.c_double]
        _lib.orc_round_e4m3.restype = ctypes.c_double
        _lib.orc_round_e4m3.argtypes = [ctypes.c_double]
        _lib.orc_adam.argtypes = [ctypes.c_long, d, d, d, d, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_long]
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's parallel loops from now on (OpenMP)."""
    lib().orc_set_threads(ctypes.c_int(int(n)))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _Levels:
    """Keeps float64 copies of the levels alive and exposes a double** to them."""

    def __init__(self, levels: Sequence[np.ndarray]):
        self.arrs = [_f64(l) for l in levels]
        self.ptrs = (ctypes.c_void_p * len(self.arrs))(*[a.ctypes.data for a in self.arrs])


def _pyr(levels, address) -> _Pyr:
    h, w, c = levels[0].shape
    return _Pyr(w, h, c, len(levels), address)


def fetch(levels, uv, lod, address=WRAP) -> np.ndarray:
    L = _Levels(levels)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    n = lod.shape[0]
    z = np.empty((n, L.arrs[0].shape[2]), np.float64)
    lib().orc_fetch(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_long(n), _ptr(uv), _ptr(lod), _ptr(z))
    return z


def fetch_fp16(levels, uv, lod, address=WRAP) -> np.ndarray:
    """Latent codes filtered with the FP16 decoders' arithmetic (orc_fetch_fp16): FP16 weights,
    the taps summed in FP16 in stencil order.  Pass FP16-valued texels."""
    L = _Levels(levels)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    n = lod.shape[0]
    z = np.empty((n, L.arrs[0].shape[2]), np.float64)
    lib().orc_fetch_fp16(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_long(n), _ptr(uv), _ptr(lod),
                         _ptr(z))
    return z


def taps(levels, uv, lod, address=WRAP) -> np.ndarray:
    """Flat texel indices (level-concatenated pyramid) of the 8 taps of every query."""
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    n = lod.shape[0]
    out = np.empty((n, 8), np.int64)
    rc = lib().orc_taps(ctypes.byref(_pyr(levels, address)), ctypes.c_long(n), _ptr(uv), _ptr(lod), _ptr(out))
    assert rc == 0
    return out


def decode(levels, dims, params, uv, lod, wi, wo, address=WRAP, return_q=False):
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P = _f64(params)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    n = lod.shape[0]
    rgb = np.empty((n, dims[-1]), np.float64)
    q = np.empty((n, dims[-1]), np.float64) if return_q else None
    rc = lib().orc_decode(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(dims) - 1), dims_c,
                          _ptr(P), ctypes.c_long(n), _ptr(uv), _ptr(lod), _ptr(wi), _ptr(wo), _ptr(rgb),
                          _ptr(q) if q is not None else None)
    if rc != 0:
        raise ValueError("oracle decode: dims must be [C + 6, ..., 3 or 6]")
    return (rgb, q) if return_q else rgb


def decode_rr(levels, dims, params, uv, lod, xi, wi, wo, address=WRAP):
    """Decode with the level chosen by Russian roulette (orc_decode_rr): query i takes the
    coarser level when xi[i] < t (t the fractional part of its clamped level), the finer one
    otherwise, then filters bilinearly inside it."""
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P = _f64(params)
    uv, lod, xi = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1), _f64(xi).reshape(-1)
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    n = lod.shape[0]
    if xi.shape[0] != n:
        raise ValueError("oracle decode_rr: one draw per query")
    rgb = np.empty((n, dims[-1]), np.float64)
    rc = lib().orc_decode_rr(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(dims) - 1), dims_c,
                             _ptr(P), ctypes.c_long(n), _ptr(uv), _ptr(lod), _ptr(xi), _ptr(wi), _ptr(wo),
                             _ptr(rgb))
    if rc != 0:
        raise ValueError("oracle decode_rr: dims must be [C + 6, ..., 3 or 6]")
    return rgb


def frames(nf, fparams, z, wi, wo):
    """[T wi, T wo] (n x 6 nf) of latent codes z[n][C] under the learned-shading-frame layer
    fparams = W_F[6 nf][C] then b_F[6 nf] (orc_frames)."""
    z = _f64(z)
    n, C = z.shape
    F = _f64(fparams)
    if F.size != 6 * nf * C + 6 * nf:
        raise ValueError("oracle frames: fparams must hold W_F[6N][C] and b_F[6N]")
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    out = np.empty((n, 6 * nf), np.float64)
    rc = lib().orc_frames(ctypes.c_int(nf), ctypes.c_int(C), _ptr(F), ctypes.c_long(n), _ptr(z), _ptr(wi),
                          _ptr(wo), _ptr(out))
    assert rc == 0
    return out


def decode_frames(levels, dims, params, nf, fparams, uv, lod, wi, wo, xi=None, address=WRAP):
    """Decode with nf learned shading frames (orc_decode_frames): the decoder input is
    [z, T wi, T wo], dims[0] = C + 6 nf; xi selects the Russian-roulette fetch."""
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P, F = _f64(params), _f64(fparams)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    n = lod.shape[0]
    if xi is not None:
        xi = _f64(xi).reshape(-1)
        if xi.shape[0] != n:
            raise ValueError("oracle decode_frames: one draw per query")
    rgb = np.empty((n, dims[-1]), np.float64)
    rc = lib().orc_decode_frames(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(dims) - 1), dims_c,
                                 _ptr(P), ctypes.c_int(nf), _ptr(F), ctypes.c_long(n), _ptr(uv), _ptr(lod),
                                 _ptr(xi) if xi is not None else None, _ptr(wi), _ptr(wo), _ptr(rgb))
    if rc != 0:
        raise ValueError("oracle decode_frames: dims must be [C + 6 nf, ..., 3 or 6]")
    return rgb



def proxy_activate(raw):
    """The 9 proxy parameters {w_d, mu_dx, mu_dy, w_s, alpha_x, alpha_y, rho, mu_sx, mu_sy} from
    raw sampling-decoder outputs (orc_proxy_activate), row by row."""
    raw = _f64(raw).reshape(-1, 9)
    out = np.empty_like(raw)
    for i in range(raw.shape[0]):
        lib().orc_proxy_activate(_ptr(raw[i]), _ptr(out[i]))
    return out


def proxy_pdf(params, wi, wo):
    """PDF of wo under the analytic proxy (orc_proxy_pdf), params [n][9]."""
    P = _f64(params).reshape(-1, 9)
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    n = P.shape[0]
    pdf = np.empty(n)
    rc = lib().orc_proxy_batch(ctypes.c_long(n), _ptr(P), _ptr(wi), _ptr(wo), None, None, _ptr(pdf))
    assert rc == 0
    return pdf


def proxy_sample(params, wi, u):
    """(wo [n][3], pdf [n]) sampled with u [n][3] under the analytic proxy (orc_proxy_sample)."""
    P = _f64(params).reshape(-1, 9)
    wi, u = _f64(wi).reshape(-1, 3), _f64(u).reshape(-1, 3)
    n = P.shape[0]
    wo, pdf = np.empty((n, 3)), np.empty(n)
    rc = lib().orc_proxy_batch(ctypes.c_long(n), _ptr(P), _ptr(wi), None, _ptr(u), _ptr(wo), _ptr(pdf))
    assert rc == 0
    return wo, pdf


def sampler_params(levels, sdims, sparams, uv, lod, wi, address=WRAP):
    """Proxy parameters [n][9] of the sampling decoder on [z, wi] (orc_sampler_params)."""
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(sdims))(*sdims)
    P = _f64(sparams)
    uv, lod, wi = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1), _f64(wi).reshape(-1, 3)
    n = lod.shape[0]
    out = np.empty((n, 9))
    rc = lib().orc_sampler_params(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(sdims) - 1), dims_c,
                                  _ptr(P), ctypes.c_long(n), _ptr(uv), _ptr(lod), _ptr(wi), _ptr(out))
    if rc != 0:
        raise ValueError("oracle sampler_params: sdims must be [C + 3, ..., 9]")
    return out

def loss_grad(levels, dims, params, uv, lod, wi, wo, target, address=WRAP):
    """(loss, dparams, [dlevel_l]) of the mean squared error of the decoded outputs against
    target [n][dims[-1]] (RGB, or RGB then albedo; see orc_loss_grad)."""
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P = _f64(params)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    wi, wo, tg = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3), _f64(target).reshape(-1, dims[-1])
    n = lod.shape[0]
    dP = np.empty_like(P)
    dL = [np.empty_like(a) for a in L.arrs]
    dptrs = (ctypes.c_void_p * len(dL))(*[a.ctypes.data for a in dL])
    loss = ctypes.c_double(0.0)
    rc = lib().orc_loss_grad(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(dims) - 1), dims_c,
                             _ptr(P), ctypes.c_long(n), _ptr(uv), _ptr(lod), _ptr(wi), _ptr(wo), _ptr(tg),
                             ctypes.byref(loss), _ptr(dP), dptrs)
    if rc != 0:
        raise ValueError("oracle loss_grad: dims must be [C + 6, ..., 3 or 6]")
    return loss.value, dP, dL


def loss_grad_frames(levels, dims, params, fparams, n_frames, uv, lod, wi, wo, target, address=WRAP):
    """(loss, dparams, dfparams, [dlevel_l]) of the mean squared error of the decode with learned
    shading frames (see orc_loss_grad_frames); fparams = W_F[6N][C] then b_F[6N]."""
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P, F = _f64(params), _f64(fparams)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    wi, wo, tg = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3), _f64(target).reshape(-1, dims[-1])
    n = lod.shape[0]
    dP, dF = np.empty_like(P), np.empty_like(F)
    dL = [np.empty_like(a) for a in L.arrs]
    dptrs = (ctypes.c_void_p * len(dL))(*[a.ctypes.data for a in dL])
    loss = ctypes.c_double(0.0)
    rc = lib().orc_loss_grad_frames(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(dims) - 1),
                                    dims_c, _ptr(P), ctypes.c_int(n_frames), _ptr(F), ctypes.c_long(n), _ptr(uv),
                                    _ptr(lod), _ptr(wi), _ptr(wo), _ptr(tg), ctypes.byref(loss), _ptr(dP), _ptr(dF),
                                    dptrs)
    if rc != 0:
        raise ValueError("oracle loss_grad_frames: dims must be [C + 6 n_frames, ..., 3 or 6]")
    return loss.value, dP, dF, dL


def adam(p, m, v, g, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, step=1):
    """In-place Adam update of float64 arrays p, m, v with gradient g."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    dp = ctypes.POINTER(ctypes.c_double)
    lib().orc_adam(ctypes.c_long(p.size), p.ctypes.data_as(dp), m.ctypes.data_as(dp), v.ctypes.data_as(dp),
                   g.ctypes.data_as(dp), lr, b1, b2, eps, ctypes.c_long(step))


def round_fp16(x) -> np.ndarray:
    x = _f64(x)
    y = np.empty_like(x)
    lib().orc_round_array(ctypes.c_long(x.size), _ptr(x), _ptr(y), ctypes.c_int(0))
    return y


def round_e4m3(x) -> np.ndarray:
    x = _f64(x)
    y = np.empty_like(x)
    lib().orc_round_array(ctypes.c_long(x.size), _ptr(x), _ptr(y), ctypes.c_int(1))
    return y


FMT_FP16, FMT_E4M3, FMT_NONE = 0, 1, 2


def decode_quant(levels, dims, qparams, w_scales, a_scales, a_formats, uv, lod, wi, wo, address=WRAP,
                 blend_fp16=False):
    """Decode with reduced-precision decoder arithmetic (see orc_decode_quant); blend_fp16 filters
    the latent code in FP16 as the FP16 decoders do (orc_decode_quant_blend)."""
    L = _Levels(levels)
    K = len(dims) - 1
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P = _f64(qparams)
    sw, sa = _f64(w_scales), _f64(a_scales)
    af = (ctypes.c_int * K)(*a_formats)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    n = lod.shape[0]
    rgb = np.empty((n, dims[-1]), np.float64)
    rc = lib().orc_decode_quant_blend(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(K), dims_c,
                                      _ptr(P), _ptr(sw), _ptr(sa), af, ctypes.c_long(n), _ptr(uv), _ptr(lod),
                                      _ptr(wi), _ptr(wo), _ptr(rgb), ctypes.c_int(1 if blend_fp16 else 0))
    if rc != 0:
        raise ValueError("oracle decode_quant: bad dims")
    return rgb


def sampler_params_quant(levels, sdims, qparams, uv, lod, wi, address=WRAP, fmt=FMT_FP16, blend_fp16=True):
    """Proxy parameters [n][9] with the matrix-core sampling decoder's arithmetic
    (orc_sampler_params_quant): FP16-filtered code (blend_fp16), layer inputs rounded to FP16
    (fmt FMT_FP16) or kept (FMT_NONE), weights given already rounded, exact sums."""
    L = _Levels(levels)
    dims_c = (ctypes.c_int * len(sdims))(*sdims)
    P = _f64(qparams)
    uv, lod, wi = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1), _f64(wi).reshape(-1, 3)
    n = lod.shape[0]
    out = np.empty((n, 9))
    rc = lib().orc_sampler_params_quant(ctypes.byref(_pyr(levels, address)), L.ptrs, ctypes.c_int(len(sdims) - 1),
                                        dims_c, _ptr(P), ctypes.c_int(fmt), ctypes.c_long(n), _ptr(uv), _ptr(lod),
                                        _ptr(wi), _ptr(out), ctypes.c_int(1 if blend_fp16 else 0))
    if rc != 0:
        raise ValueError("oracle sampler_params_quant: sdims must be [C + 3, ..., 9], fmt FP16 or none")
    return out


def encode(edims, eparams, attrs):
    """The encoder on parameter rows (orc_encode): attrs [n][A] -> z [n][C]."""
    K = len(edims) - 1
    dims_c = (ctypes.c_int * len(edims))(*edims)
    P = _f64(eparams)
    A = _f64(attrs).reshape(-1, edims[0])
    z = np.empty((A.shape[0], edims[-1]))
    rc = lib().orc_encode(ctypes.c_int(K), dims_c, _ptr(P), ctypes.c_long(A.shape[0]), _ptr(A), _ptr(z))
    if rc != 0:
        raise ValueError("oracle encode: bad dims")
    return z


def encode_queries(attr_levels, edims, eparams, uv, lod, address=WRAP):
    """The encoder on the parameters filtered at each query (orc_encode_queries): z [n][C]."""
    L = _Levels(attr_levels)
    K = len(edims) - 1
    dims_c = (ctypes.c_int * len(edims))(*edims)
    P = _f64(eparams)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    z = np.empty((lod.shape[0], edims[-1]))
    rc = lib().orc_encode_queries(ctypes.byref(_pyr(attr_levels, address)), L.ptrs, ctypes.c_int(K), dims_c,
                                  _ptr(P), ctypes.c_long(lod.shape[0]), _ptr(uv), _ptr(lod), _ptr(z))
    if rc != 0:
        raise ValueError("oracle encode_queries: edims[0] must equal the parameter channels")
    return z


def loss_grad_codes(dims, params, z, wi, wo, target):
    """(loss, dparams, dz [n][C]) of the decoder's mean squared error on given latent codes
    (orc_loss_grad_codes)."""
    K = len(dims) - 1
    dims_c = (ctypes.c_int * len(dims))(*dims)
    P = _f64(params)
    z = _f64(z).reshape(-1, dims[0] - 6)
    n = z.shape[0]
    wi, wo = _f64(wi).reshape(-1, 3), _f64(wo).reshape(-1, 3)
    T = _f64(target).reshape(-1, dims[-1])
    dparams, dz, loss = np.empty(P.size), np.empty(z.shape), ctypes.c_double(0.0)
    rc = lib().orc_loss_grad_codes(ctypes.c_int(K), dims_c, _ptr(P), ctypes.c_long(n), _ptr(z), _ptr(wi), _ptr(wo),
                                   _ptr(T), ctypes.byref(loss), _ptr(dparams), _ptr(dz))
    if rc != 0:
        raise ValueError("oracle loss_grad_codes: bad dims")
    return loss.value, dparams, dz


def encoder_backward(attr_levels, edims, eparams, uv, lod, dz, address=WRAP):
    """Gradient of sum_i dz[i] . E(filtered parameters at query i) with respect to the
    encoder's parameters (orc_encoder_backward)."""
    L = _Levels(attr_levels)
    K = len(edims) - 1
    dims_c = (ctypes.c_int * len(edims))(*edims)
    P = _f64(eparams)
    uv, lod = _f64(uv).reshape(-1, 2), _f64(lod).reshape(-1)
    dz = _f64(dz).reshape(-1, edims[-1])
    out = np.empty(P.size)
    rc = lib().orc_encoder_backward(ctypes.byref(_pyr(attr_levels, address)), L.ptrs, ctypes.c_int(K), dims_c,
                                    _ptr(P), ctypes.c_long(lod.shape[0]), _ptr(uv), _ptr(lod), _ptr(dz), _ptr(out))
    if rc != 0:
        raise ValueError("oracle encoder_backward: edims[0] must equal the parameter channels")
    return out
