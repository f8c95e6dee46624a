"""fp64 numpy oracle of the quality measures of §IV.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For one frame pair and one motion field (a vector per block, pointing from
the block's position in the current frame to its match in the reference
frame):
  compensated frame  every block copied from the reference at its vector
  SAD, SSE per block sum of |cur - comp| and of (cur - comp)^2 over its pixels
  MAD, MSE           those sums over the frame divided by its pixel count
  PSNR               10 log10(255^2 / MSE) dB (+inf when MSE = 0)
  distance           Euclidean distance between the vector and the true
                     (full-search) vector, summed over blocks
  equal              number of blocks whose vector equals the true vector
The paper averages distance and probability over blocks and every measure
over frames; the per-pair sums here are what those averages are made of.
"""
from __future__ import annotations

import math

import numpy as np


def compensate(ref, mv, B):
    """The motion-compensated frame: block (by, bx) = ref at its position + mv."""
    H, W = ref.shape
    out = np.empty_like(ref)
    for by in range(H // B):
        for bx in range(W // B):
            dx, dy = int(mv[by, bx, 0]), int(mv[by, bx, 1])
            y0, x0 = by * B + dy, bx * B + dx
            if not (0 <= y0 <= H - B and 0 <= x0 <= W - B):
                raise ValueError("vector %r of block %r leaves the frame" % ((dx, dy), (bx, by)))
            out[by * B:(by + 1) * B, bx * B:(bx + 1) * B] = ref[y0:y0 + B, x0:x0 + B]
    return out


def block_errors(cur, comp, B):
    """Per-block SAD and SSE (int64 [H/B, W/B])."""
    H, W = cur.shape
    d = cur.astype(np.int64) - comp.astype(np.int64)
    a = np.abs(d).reshape(H // B, B, W // B, B).sum(axis=(1, 3))
    e = (d * d).reshape(H // B, B, W // B, B).sum(axis=(1, 3))
    return a, e


def pair_quality(cur, ref, mv, B, mv_true=None):
    """The measures of one pair; mv, mv_true: int [H/B, W/B, 2] as (x, y)."""
    comp = compensate(ref, mv, B)
    a, e = block_errors(cur, comp, B)
    n = cur.size
    sad, sse = int(a.sum()), int(e.sum())
    equal, dist = 0, 0.0
    if mv_true is not None:
        for by in range(mv.shape[0]):
            for bx in range(mv.shape[1]):
                dx = int(mv[by, bx, 0]) - int(mv_true[by, bx, 0])
                dy = int(mv[by, bx, 1]) - int(mv_true[by, bx, 1])
                equal += dx == 0 and dy == 0
                dist += math.sqrt(dx * dx + dy * dy)
    mse = sse / n
    return {
        "sad": sad, "sse": sse, "blocks": mv.shape[0] * mv.shape[1], "equal": equal, "dist": dist,
        "mad": sad / n, "mse": mse, "psnr": math.inf if sse == 0 else 10.0 * math.log10(255.0 ** 2 / mse),
        "block_sad": a, "block_sse": e,
    }
