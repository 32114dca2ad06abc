"""FP64 CPU oracle for the camera's input conditioning and output encoding.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  Plain
numpy in double precision; it imports nothing from the GPU package.

Eq. (1) (Sec. III-A.1) attenuates with the distance d from the camera, which
the paper calls depth or range.  A renderer's depth buffer holds z-depth, the
distance along the optical axis; the line-of-sight range of pixel (u, v) under
a pinhole camera follows from back-projecting its centre (u + 1/2, v + 1/2).
Colour crosses the boundary as 8-bit sRGB, whose transfer function is the one
of IEC 61966-2-1; Eq. (1) acts on linear intensities.

Parity status: every function is pinned by tests (published sRGB values, the
inverse pair, geometric back-projection, the adjoint identity).
"""
from __future__ import annotations

import numpy as np


def srgb_to_linear(y):
    """IEC 61966-2-1 decoding: linear segment below 0.04045, power 2.4 above."""
    y = np.asarray(y, dtype=np.float64)
    return np.where(y <= 0.04045, y / 12.92, ((y + 0.055) / 1.055) ** 2.4)


def linear_to_srgb(x):
    """IEC 61966-2-1 encoding: linear segment up to 0.0031308, power 1/2.4 above."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= 0.0031308, 12.92 * x, 1.055 * np.abs(x) ** (1.0 / 2.4) - 0.055)


def decode_codes(codes):
    """8-bit codes -> linear intensities (fp64)."""
    return srgb_to_linear(np.asarray(codes, dtype=np.float64) / 255.0)


def encode_codes(x):
    """Linear intensities -> 8-bit codes: clamp to [0, 1] (NaN -> 0), then round
    255 * linear_to_srgb half up."""
    x = np.asarray(x, dtype=np.float64)
    x = np.where(np.isnan(x), 0.0, np.clip(x, 0.0, 1.0))
    return np.floor(255.0 * linear_to_srgb(x) + 0.5).astype(np.uint8)


def range_scale(H, W, fx, fy, cx, cy):
    """r / z for every pixel of an H x W pinhole image: the length of the
    back-projected ray ((u + 1/2 - cx) / fx, (v + 1/2 - cy) / fy, 1)."""
    a = (np.arange(W, dtype=np.float64) + 0.5 - cx) / fx
    b = (np.arange(H, dtype=np.float64) + 0.5 - cy) / fy
    return np.sqrt(1.0 + a[None, :] ** 2 + b[:, None] ** 2)


def condition(srgb=None, zdepth=None, fx=1.0, fy=1.0, cx=0.0, cy=0.0):
    """Forward conditioning of one frame.

    srgb: [H][W][3 or 4] uint8 (alpha ignored) or None; zdepth: [H][W] or None.
    Returns (J planar [3][H][W] fp64 or None, range [H][W] fp64 or None)."""
    J = rng = None
    if srgb is not None:
        J = np.ascontiguousarray(np.moveaxis(decode_codes(np.asarray(srgb)[..., :3]), -1, 0))
    if zdepth is not None:
        z = np.asarray(zdepth, dtype=np.float64)
        rng = z * range_scale(z.shape[0], z.shape[1], fx, fy, cx, cy)
    return J, rng


def condition_backward(grad_range, fx, fy, cx, cy):
    """Adjoint of the range conversion: dL/dz = dL/dr * r / z."""
    g = np.asarray(grad_range, dtype=np.float64)
    return g * range_scale(g.shape[0], g.shape[1], fx, fy, cx, cy)


def encode(I, channels_out=3):
    """Planar [3][H][W] linear image -> interleaved [H][W][channels_out] uint8
    (alpha 255)."""
    codes = np.moveaxis(encode_codes(I), 0, -1)
    if channels_out == 4:
        alpha = np.full(codes.shape[:2] + (1,), 255, dtype=np.uint8)
        codes = np.concatenate([codes, alpha], axis=-1)
    return np.ascontiguousarray(codes)
