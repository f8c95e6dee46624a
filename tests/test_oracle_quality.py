"""Pins of the quality oracle (oracle/quality.py): the compensated frame
against the C oracle's own SAD, closed forms for a constant brightness
offset, the Cauchy-Schwarz bounds between SAD and SSE, per-pixel brute force,
and the distance/probability definitions on hand-made fields."""
import math

import numpy as np
import pytest

import oracle
from oracle import quality as q
from synth import make_config, qcif_pair


def random_field(rng, H, W, B, R):
    """Valid vectors (the reference block stays inside the frame, |v| <= R)."""
    hb, wb = H // B, W // B
    mv = np.zeros((hb, wb, 2), np.int16)
    for by in range(hb):
        for bx in range(wb):
            lox, hix = max(-R, -bx * B), min(R, W - B - bx * B)
            loy, hiy = max(-R, -by * B), min(R, H - B - by * B)
            mv[by, bx] = (rng.integers(lox, hix + 1), rng.integers(loy, hiy + 1))
    return mv


@pytest.mark.parametrize("search", ["fs", "dcds"])
def test_compensated_sad_equals_the_search_sad(search):
    """SAD of the compensated blocks (numpy) = SAD the C oracle reported at
    its vectors: two independent codings of the same displacement."""
    cur, ref, _ = qcif_pair(5)
    fn = oracle.fullsearch if search == "fs" else oracle.dcds
    mv, sad, _ = fn(cur, ref, 16, 7)
    r = q.pair_quality(cur, ref, mv, 16)
    np.testing.assert_array_equal(r["block_sad"], sad.astype(np.int64))
    assert r["sad"] == int(sad.astype(np.int64).sum())


def test_constant_offset_closed_form():
    rng = np.random.default_rng(3)
    ref = rng.integers(20, 200, (48, 64)).astype(np.uint8)
    cur = (ref.astype(np.int64) + 7).astype(np.uint8)
    mv = np.zeros((3, 4, 2), np.int16)
    r = q.pair_quality(cur, ref, mv, 16)
    assert r["mad"] == 7.0 and r["mse"] == 49.0
    assert np.all(r["block_sse"] == 49 * 256)
    assert r["psnr"] == pytest.approx(10 * math.log10(65025 / 49), rel=1e-15)


def test_cauchy_schwarz_bounds():
    """Per block of N pixels: SAD^2 / N <= SSE <= 255 SAD."""
    seq = make_config(2, seed=4, frames=3)
    rng = np.random.default_rng(0)
    for B in (8, 16):
        mv = random_field(rng, 288, 352, B, 7)
        r = q.pair_quality(seq[1], seq[0], mv, B)
        a, e = r["block_sad"], r["block_sse"]
        assert np.all(a * a <= e * B * B)
        assert np.all(e <= 255 * a)


def test_brute_force_per_pixel():
    rng = np.random.default_rng(11)
    H, W, B = 24, 32, 8
    cur = rng.integers(0, 256, (H, W)).astype(np.uint8)
    ref = rng.integers(0, 256, (H, W)).astype(np.uint8)
    mv = random_field(rng, H, W, B, 5)
    r = q.pair_quality(cur, ref, mv, B)
    for by in range(H // B):
        for bx in range(W // B):
            s = e = 0
            for v in range(B):
                for u in range(B):
                    c = int(cur[by * B + v, bx * B + u])
                    p = int(ref[by * B + v + mv[by, bx, 1], bx * B + u + mv[by, bx, 0]])
                    s += abs(c - p)
                    e += (c - p) ** 2
            assert r["block_sad"][by, bx] == s and r["block_sse"][by, bx] == e


def test_identical_frames():
    ref = np.random.default_rng(1).integers(0, 256, (32, 32)).astype(np.uint8)
    mv = np.zeros((2, 2, 2), np.int16)
    r = q.pair_quality(ref, ref, mv, 16, mv_true=mv)
    assert r["sse"] == 0 and r["psnr"] == math.inf
    assert r["equal"] == 4 and r["dist"] == 0.0


def test_distance_and_probability():
    ref = np.zeros((32, 64), np.uint8)
    mv = np.zeros((2, 4, 2), np.int16)
    tv = np.zeros((2, 4, 2), np.int16)
    tv[0, 1] = (3, 4)     # distance 5
    tv[1, 2] = (-1, 0)    # distance 1
    mv[1, 3] = (0, -2)    # distance 2 (truth 0)
    mv[0, 0] = tv[0, 0] = (1, 1)  # equal, non-zero
    mv = np.clip(mv, -16, 16)
    r = q.pair_quality(ref, ref, mv, 16, mv_true=tv)
    assert r["equal"] == 5
    assert r["dist"] == pytest.approx(8.0, abs=1e-15)


def test_transposed_vector_is_caught():
    """A field read as (y, x) instead of (x, y) changes the SSE (asymmetric fields)."""
    cur, ref, _ = qcif_pair(2)
    mv, _, _ = oracle.fullsearch(cur, ref, 16, 7)
    asym = (mv[..., 0] != mv[..., 1]).any()
    assert asym
    good = q.pair_quality(cur, ref, mv, 16)["sse"]
    swapped = np.ascontiguousarray(mv[..., ::-1])
    try:
        bad = q.pair_quality(cur, ref, swapped, 16)["sse"]
    except ValueError:
        return  # a swapped vector left the frame
    assert bad != good
