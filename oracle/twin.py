"""Brute-force numpy formulation of the latent fetch (test infrastructure).

An independent restatement of the filtered latent lookup of Sec. 4.1 ("Latent texture"):
inside one level, bilinear interpolation equals a sum of every texel weighted by the
separable tent kernel Lambda(d) = max(0, 1 - |d|) of its distance (in texels) to the
sample position, with texel x centred at (x + 1/2) / W.  Wrap addressing sums the tent
over the periodic images of the texture; clamp addressing extends the texture by edge
replication.  Across levels the two nearest levels are blended linearly.

No floor/fract/modulus logic is shared with the C oracle: this version never locates the
four neighbours, it weighs every texel.  Meant for textures of at most a few hundred
texels.
"""
from __future__ import annotations

import numpy as np

WRAP, CLAMP = 0, 1


def _tent(d):
    return np.maximum(0.0, 1.0 - np.abs(d))


def _axis_weights(coord: float, size: int, address: int) -> np.ndarray:
    """Weight of each texel index 0..size-1 along one axis for a sample at `coord` (uv units)."""
    s = coord * size - 0.5
    w = np.zeros(size)
    if address == WRAP:
        # periodic images: texel x also sits at x + k*size; coord may be any real number
        kmin = int(np.floor((s - size) / size)) - 1
        kmax = int(np.ceil((s + size) / size)) + 1
        for k in range(kmin, kmax + 1):
            w += _tent(s - (np.arange(size) + k * size))
    else:
        # edge replication: positions -2..size+1 beyond the edge carry the edge texel;
        # positions further out only matter for samples further out, handled by clipping s
        lo, hi = -1.0, size  # a sample beyond the last centre sees only the edge texel
        s_c = min(max(s, lo), hi)
        for x in range(-2, size + 2):
            xi = min(max(x, 0), size - 1)
            w[xi] += _tent(s_c - x)
    return w


def bilinear_level(level: np.ndarray, u: float, v: float, address: int = WRAP) -> np.ndarray:
    H, W, C = level.shape
    wx = _axis_weights(u, W, address)
    wy = _axis_weights(v, H, address)
    return np.einsum("y,x,yxc->c", wy, wx, level.astype(np.float64))


def fetch(levels, uv, lod, address: int = WRAP) -> np.ndarray:
    uv = np.asarray(uv, dtype=np.float64).reshape(-1, 2)
    lod = np.asarray(lod, dtype=np.float64).reshape(-1)
    M = len(levels)
    out = np.zeros((lod.shape[0], levels[0].shape[2]))
    for i in range(lod.shape[0]):
        lam = min(max(lod[i], 0.0), M - 1.0)
        # blend weight of every level: tent in the level index, so only the two neighbours of
        # lam (or lam itself when it is an integer) get a nonzero weight
        for l in range(M):
            wl = _tent(lam - l)
            if wl > 0.0:
                out[i] += wl * bilinear_level(levels[l], uv[i, 0], uv[i, 1], address)
    return out
