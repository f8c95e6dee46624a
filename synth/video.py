"""Seeded synthetic luma sequences standing in for the paper's test sequences.

The paper measures on 8-bit luminance of standard sequences (§II-C, §IV) that
are not available here.  These generators imitate the statistics that matter
to the search: most motion vectors are zero or small, horizontal motion is
wider spread than vertical (Tables II-III), and some objects move far.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` only, so a
seed fixes the output bit for bit.  Pixels are rounded with ``np.rint`` and
clipped to 0..255.

Recipes (sizes W x H):
  1  QCIF 176x144, 2 frames.  f0 = blurred noise (sigma 1.5).  Per 16x16 block a
     motion vector: zero with probability 0.6, else (rint(Laplace(0, 2)),
     rint(Laplace(0, 1))) clipped to +-7 and to the frame; f1's block copies f0
     at block + mv; f1 += N(0, 2^2).  cur = f1, ref = f0.
  2  CIF 352x288, 300 frames, +-7: a blurred-noise background panning 1 px per
     frame to the left (motion vector (+1, 0)), 8 textured rectangles of side
     U{24..96} with constant integer velocity U{-6..6}^2, wrapping with a
     margin, N(0, 2^2) per frame.
  3  1920x1088, 60 frames, +-15: as 2 with object sizes scaled by 1920/352,
     32 objects, velocity (rint(Laplace(0, 4)), rint(Laplace(0, 2))) clipped.
  4  64 streams (16 each of QCIF, CIF, 1280x720, 1920x1088), 30 frames each,
     objects 2/8/20/32, the velocity law of 3, seeds 1000 + s.
  5  3840x2160, 60 frames, +-31, 64 objects, velocity Laplace(0, 8) /
     Laplace(0, 4) clipped to +-31; training sequences (1920x1088, 50 frames,
     the same law) use seeds 10000 + q, held-out ones 20000 + q.
  6  CIF 352x288, 60 frames, +-7, near the paper's operating point (most
     vectors zero, small motion, smooth texture): a static background of
     blurred noise (sigma 3) stretched to standard deviation 30 around 128;
     12 rectangles of side U{32..111} with texture of sigma 2 (the same
     stretch, plus a uniform offset in -40..40), at uniform positions inside
     the frame, velocity (rint Laplace(0, 2), rint Laplace(0, 1)) clipped to
     +-7, moving off the frame rather than wrapping; N(0, 1) per frame.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CIF_W = 352


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _gauss_kernel(sigma: float) -> np.ndarray:
    r = int(math.ceil(3.0 * sigma))
    k = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def _blur_axis(x: np.ndarray, g: np.ndarray, axis: int) -> np.ndarray:
    r = (len(g) - 1) // 2
    pad = [(0, 0)] * x.ndim
    pad[axis] = (r, r)
    xp = np.pad(x, pad, mode="reflect")
    out = np.zeros_like(x)
    n = x.shape[axis]
    for i, w in enumerate(g):
        sl = [slice(None)] * x.ndim
        sl[axis] = slice(i, i + n)
        out += w * xp[tuple(sl)]
    return out


def blurred_noise(rng: np.random.Generator, h: int, w: int, sigma: float) -> np.ndarray:
    """Uniform integers 0..255 smoothed by a separable Gaussian (radius ceil(3 sigma),
    reflect borders), rounded; returned as float32 (std is about 14 at sigma 1.5)."""
    x = rng.integers(0, 256, size=(h, w)).astype(np.float64)
    g = _gauss_kernel(sigma)
    x = _blur_axis(_blur_axis(x, g, 0), g, 1)
    return np.rint(x).astype(np.float32)


def _to_u8(x: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def qcif_pair(seed: int = 1, W: int = 176, H: int = 144, block: int = 16, R: int = 7):
    """Config 1: returns (cur, ref, truth_mv int16[Hb, Wb, 2])."""
    rng = _rng(seed)
    f0 = blurred_noise(rng, H, W, 1.5)
    hb, wb = H // block, W // block
    truth = np.zeros((hb, wb, 2), np.int16)
    f1 = f0.copy()
    for j in range(hb):
        for i in range(wb):
            x0, y0 = i * block, j * block
            if rng.random() < 0.6:
                dx = dy = 0
            else:
                dx = int(np.clip(np.rint(rng.laplace(0.0, 2.0)), -R, R))
                dy = int(np.clip(np.rint(rng.laplace(0.0, 1.0)), -R, R))
                dx = int(np.clip(dx, -x0, W - block - x0))
                dy = int(np.clip(dy, -y0, H - block - y0))
            truth[j, i] = (dx, dy)
            f1[y0:y0 + block, x0:x0 + block] = f0[y0 + dy:y0 + dy + block, x0 + dx:x0 + dx + block]
    f1 = f1 + rng.normal(0.0, 2.0, size=f1.shape).astype(np.float32)
    return _to_u8(f1), _to_u8(f0), truth


@dataclass
class _Obj:
    w: int
    h: int
    tex: np.ndarray
    x: int
    y: int
    vx: int
    vy: int


@dataclass
class SequenceSpec:
    W: int
    H: int
    frames: int
    n_objects: int
    vel_law: str = "uniform6"  # "uniform6" | "laplace4x2" | "laplace8x4"
    vel_clip: int = 15
    seed: int = 0
    margin: int = field(default=0)


def _velocity(rng: np.random.Generator, law: str, clip: int):
    if law == "uniform6":
        return int(rng.integers(-6, 7)), int(rng.integers(-6, 7))
    if law == "laplace4x2":
        sx, sy = 4.0, 2.0
    elif law == "laplace8x4":
        sx, sy = 8.0, 4.0
    else:
        raise ValueError(law)
    vx = int(np.clip(np.rint(rng.laplace(0.0, sx)), -clip, clip))
    vy = int(np.clip(np.rint(rng.laplace(0.0, sy)), -clip, clip))
    return vx, vy


def moving_sequence(spec: SequenceSpec) -> np.ndarray:
    """Panning blurred-noise background plus textured moving rectangles.

    Returns uint8 frames [T, H, W].  The background of frame t is the canvas
    cropped at x = M + t, so cur = frame t matches ref = frame t-1 one pixel to
    the right: motion vector (+1, 0).  Object k is at p_k + v_k t (wrapping
    toroidally over the frame plus a margin), so its vector is -v_k.
    """
    rng = _rng(spec.seed)
    W, H, T = spec.W, spec.H, spec.frames
    scale = W / CIF_W
    M = 8
    canvas = blurred_noise(rng, H + 2 * M, W + T + 2 * M, 1.5)
    objs = []
    lo, hi = int(round(24 * scale)), int(round(96 * scale))
    margin = spec.margin or hi
    for _ in range(spec.n_objects):
        w = int(rng.integers(lo, hi + 1))
        h = int(rng.integers(lo, hi + 1))
        tex = blurred_noise(rng, h, w, 1.0) + float(rng.uniform(-40.0, 40.0))
        x = int(rng.integers(-margin, W + margin))
        y = int(rng.integers(-margin, H + margin))
        vx, vy = _velocity(rng, spec.vel_law, spec.vel_clip)
        objs.append(_Obj(w, h, tex, x, y, vx, vy))
    out = np.empty((T, H, W), np.uint8)
    span_x, span_y = W + 2 * margin, H + 2 * margin
    for t in range(T):
        f = canvas[M:M + H, M + t:M + t + W].copy()
        for o in objs:
            px = (o.x + o.vx * t + margin) % span_x - margin
            py = (o.y + o.vy * t + margin) % span_y - margin
            x0, y0 = max(px, 0), max(py, 0)
            x1, y1 = min(px + o.w, W), min(py + o.h, H)
            if x1 <= x0 or y1 <= y0:
                continue
            f[y0:y1, x0:x1] = o.tex[y0 - py:y1 - py, x0 - px:x1 - px]
        f += rng.normal(0.0, 2.0, size=f.shape).astype(np.float32)
        out[t] = _to_u8(f)
    return out


def _stretched(rng: np.random.Generator, h: int, w: int, sigma: float) -> np.ndarray:
    """Blurred noise rescaled to mean 128 and standard deviation 30."""
    x = blurred_noise(rng, h, w, sigma)
    c = x - x.mean()
    return 128.0 + c * (30.0 / c.std())


def paperlike_sequence(seed: int = 6, W: int = 352, H: int = 288, frames: int = 60, n_objects: int = 12,
                       R: int = 7) -> np.ndarray:
    """Config 6: a static smooth background and slowly moving smooth objects.

    Object k is at p_k + v_k t (clipped by the frame, not wrapped), so inside
    it the true vector is -v_k; the background's is (0, 0).
    """
    rng = _rng(seed)
    bg = _stretched(rng, H, W, 3.0)
    objs = []
    for _ in range(n_objects):
        w = int(rng.integers(32, 112))
        h = int(rng.integers(32, 112))
        tex = _stretched(rng, h, w, 2.0) + float(rng.uniform(-40.0, 40.0))
        x = int(rng.integers(0, W - w))
        y = int(rng.integers(0, H - h))
        vx = int(np.clip(np.rint(rng.laplace(0.0, 2.0)), -R, R))
        vy = int(np.clip(np.rint(rng.laplace(0.0, 1.0)), -R, R))
        objs.append(_Obj(w, h, tex, x, y, vx, vy))
    out = np.empty((frames, H, W), np.uint8)
    for t in range(frames):
        f = bg.astype(np.float32).copy()
        for o in objs:
            px, py = o.x + o.vx * t, o.y + o.vy * t
            x0, y0 = max(px, 0), max(py, 0)
            x1, y1 = min(px + o.w, W), min(py + o.h, H)
            if x1 <= x0 or y1 <= y0:
                continue
            f[y0:y1, x0:x1] = o.tex[y0 - py:y1 - py, x0 - px:x1 - px]
        f += rng.normal(0.0, 1.0, size=f.shape).astype(np.float32)
        out[t] = _to_u8(f)
    return out


# Stream kinds of the batched configuration: (W, H, objects).
BATCH_KINDS = [(176, 144, 2), (352, 288, 8), (1280, 720, 20), (1920, 1088, 32)]


def batch_streams(n_streams: int = 64, frames: int = 30, base_seed: int = 1000):
    """Config 4: list of uint8 [T, H, W] sequences, 16 of each kind for 64 streams."""
    seqs = []
    for s in range(n_streams):
        W, H, nobj = BATCH_KINDS[s % len(BATCH_KINDS)]
        seqs.append(moving_sequence(SequenceSpec(W, H, frames, nobj, "laplace4x2", 15, base_seed + s)))
    return seqs


def training_sequence(q: int, frames: int = 50, held_out: bool = False, W: int = 1920, H: int = 1088):
    """Learned-start training (seed 10000 + q) or held-out (20000 + q) sequence."""
    seed = (20000 if held_out else 10000) + q
    return moving_sequence(SequenceSpec(W, H, frames, 32 if W <= 1920 else 64, "laplace8x4", 31, seed))


@dataclass
class ConfigInfo:
    name: str
    W: int
    H: int
    frames: int
    blocks: tuple
    R: int


CONFIGS = {
    1: ConfigInfo("qcif_176x144_2f_r7", 176, 144, 2, (16,), 7),
    2: ConfigInfo("cif_352x288_300f_r7", 352, 288, 300, (16,), 7),
    3: ConfigInfo("1080p_1920x1088_60f_r15", 1920, 1088, 60, (16, 8), 15),
    4: ConfigInfo("batch_64streams_30f_r15", 0, 0, 30, (16,), 15),
    5: ConfigInfo("4k_3840x2160_60f_r31", 3840, 2160, 60, (16,), 31),
    6: ConfigInfo("paperlike_cif_352x288_60f_r7", 352, 288, 60, (16,), 7),
}


def make_config(k: int, seed: int | None = None, frames: int | None = None):
    """Frames [T, H, W] uint8 of config k (1, 2, 3, 5 or 6); seed defaults to k."""
    seed = k if seed is None else seed
    if k == 1:
        cur, ref, _ = qcif_pair(seed)
        return np.stack([ref, cur])
    if k == 2:
        spec = SequenceSpec(352, 288, frames or 300, 8, "uniform6", 6, seed)
    elif k == 3:
        spec = SequenceSpec(1920, 1088, frames or 60, 32, "laplace4x2", 15, seed)
    elif k == 5:
        spec = SequenceSpec(3840, 2160, frames or 60, 64, "laplace8x4", 31, seed)
    elif k == 6:
        return paperlike_sequence(seed, frames=frames or 60)
    else:
        raise ValueError("config %r has no single sequence; use batch_streams" % k)
    return moving_sequence(spec)
