"""Conversion between the oracle's projected quantities and the 12-float
splat record the C ABI exchanges between stages (test glue, not the method).

The record holds the conic as a scaled Cholesky factor M with
M M^T = C0 * conic, C0 = 1 / (2 ln 2), so that the rasteriser evaluates
alpha = sigma 2^-|M^T d|^2, plus log2 sigma, the colour, sigma and the packed
pixel box of the alpha >= 1/255 region.  The parity tests use these helpers
to feed oracle-made records to a single GPU stage and to read GPU records
back as FP64 (u, v, conic, sigma, rgb); nothing here feeds a GPU output to
the oracle's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

# scale between the conic and the splat record's factor: M M^T = C0 * conic
C0 = 0.5 / math.log(2.0)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def factor(conic):
    """Lower-triangular M with M M^T = C0 * conic (Cholesky factor, by definition)."""
    A, B, C = _d(conic)
    with np.errstate(invalid="ignore", divide="ignore"):
        m00 = np.sqrt(C0 * A)
        m10 = C0 * B / m00
        m11 = np.sqrt(C0 * C - m10 * m10)
    return np.stack([m00, m10, m11])


def to_record(pr):
    """The 12-float splat record of the C ABI for one view, from the oracle's
    projection (FP64 values rounded once to FP32).  Culled rows are zero."""
    N = pr["u"].shape[0]
    rec = np.zeros((N, 12), np.float64)
    vis = pr["visible"].astype(bool)
    m = factor(pr["conic"])
    rec[:, 0], rec[:, 1] = pr["u"], pr["v"]
    rec[:, 2], rec[:, 3], rec[:, 4] = m[0], m[1], m[2]
    with np.errstate(divide="ignore"):
        rec[:, 5] = np.log2(pr["sigma"])
    rec[:, 6:9] = pr["rgb"].T
    rec[:, 9] = pr["sigma"]
    rec[~vis] = 0.0
    out = rec.astype(np.float32)
    bx, by = alpha_box(pr)
    out[:, 10] = np.where(vis, bx, 0).astype(np.int32).view(np.float32)
    out[:, 11] = np.where(vis, by, 0).astype(np.int32).view(np.float32)
    return out


def alpha_extent(pr):
    """Half-widths (x, y) of the region where alpha >= 1/255, i.e. of the
    ellipse d^T conic d <= 2 ln(255 sigma): sqrt(tau Sigma2_xx), sqrt(tau Sigma2_yy)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.maximum(2.0 * np.log(255.0 * pr["sigma"]), 0.0)
        return np.sqrt(tau * pr["cov"][0]), np.sqrt(tau * pr["cov"][2])


def alpha_box(pr):
    """The record's packed pixel ranges (lo | hi << 16, int16 each) of the
    alpha >= 1/255 region, widened by 1e-3 relative + one pixel: every pixel
    outside has alpha < 1/255."""
    ex, ey = alpha_extent(pr)

    def pack(c, e):
        with np.errstate(invalid="ignore"):
            lo = np.clip(np.floor(c - e * 1.001 - 0.5) - 1, -32768, 32767)
            hi = np.clip(np.ceil(c + e * 1.001 - 0.5) + 1, -32768, 32767)
        lo = np.nan_to_num(lo).astype(np.int64)
        hi = np.nan_to_num(hi).astype(np.int64)
        return ((lo & 0xFFFF) | (hi << 16)).astype(np.int64).astype(np.uint32).view(np.int32)

    return pack(pr["u"], ex), pack(pr["v"], ey)


def unpack_box(words):
    w = np.asarray(words).view(np.int32).astype(np.int64)
    lo = ((w & 0xFFFF) ^ 0x8000) - 0x8000
    return lo, w >> 16


def from_record(rec):
    """FP64 (u, v, conic A, B, C, sigma, rgb) read exactly from a float32 splat
    record: conic = M M^T / C0."""
    r = np.asarray(rec, np.float32).astype(np.float64)
    m00, m10, m11 = r[:, 2], r[:, 3], r[:, 4]
    A = m00 * m00 / C0
    B = m00 * m10 / C0
    C = (m10 * m10 + m11 * m11) / C0
    return dict(u=r[:, 0].copy(), v=r[:, 1].copy(), conic=np.stack([A, B, C]),
                sigma=r[:, 9].copy(), rgb=np.ascontiguousarray(r[:, 6:9].T))
