"""FS oracle against an independent numpy brute force (the definition of §I:
minimise the block distortion over every candidate of the window), and the
SAD the DCDS oracle reports against the same brute force."""
import numpy as np
import pytest

import oracle


def brute_fs(cur, ref, B, R):
    """Numpy statement of FS with the tie order (SAD, |dx|+|dy|, dy, dx)."""
    H, W = cur.shape
    hb, wb = H // B, W // B
    mv = np.zeros((hb, wb, 2), np.int64)
    sad = np.zeros((hb, wb), np.int64)
    nsp = np.zeros((hb, wb), np.int64)
    c32, r32 = cur.astype(np.int32), ref.astype(np.int32)
    for j in range(hb):
        for i in range(wb):
            x0, y0 = i * B, j * B
            blk = c32[y0:y0 + B, x0:x0 + B]
            keys = []
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    x, y = x0 + dx, y0 + dy
                    if x < 0 or y < 0 or x + B > W or y + B > H:
                        continue
                    s = int(np.abs(blk - r32[y:y + B, x:x + B]).sum())
                    keys.append((s, abs(dx) + abs(dy), dy, dx))
            best = min(keys)
            mv[j, i] = (best[3], best[2])
            sad[j, i] = best[0]
            nsp[j, i] = len(keys)
    return mv, sad, nsp


def _frames(kind, H, W, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        cur = rng.integers(0, 256, (H, W), dtype=np.uint8)
        ref = rng.integers(0, 256, (H, W), dtype=np.uint8)
    elif kind == "lowentropy":  # two grey levels: many exact ties
        cur = (rng.integers(0, 2, (H, W)) * 3).astype(np.uint8)
        ref = (rng.integers(0, 2, (H, W)) * 3).astype(np.uint8)
    elif kind == "checker":  # zero SAD exactly where dx + dy is odd: ties at equal |dx|+|dy|
        yy, xx = np.mgrid[0:H, 0:W]
        ref = (((xx + yy) % 2) * 9).astype(np.uint8)
        cur = (9 - ref).astype(np.uint8)
    elif kind == "flat":  # every candidate ties
        cur = np.full((H, W), 7, np.uint8)
        ref = np.full((H, W), 9, np.uint8)
    else:  # extremes: SAD reaches its maximum
        cur = np.zeros((H, W), np.uint8)
        ref = np.full((H, W), 255, np.uint8)
    return cur, ref


CASES = [
    (32, 32, 8, 1), (32, 32, 8, 2), (32, 32, 8, 3),
    (32, 48, 16, 7), (24, 40, 8, 5), (16, 16, 16, 3), (16, 32, 8, 15),
]


@pytest.mark.parametrize("H,W,B,R", CASES)
@pytest.mark.parametrize("kind", ["uniform", "lowentropy", "checker", "flat", "extreme"])
def test_fs_oracle_equals_brute_force(H, W, B, R, kind):
    cur, ref = _frames(kind, H, W, seed=H * 1000 + W * 10 + R)
    mv, sad, nsp = oracle.fullsearch(cur, ref, B, R)
    bmv, bsad, bnsp = brute_fs(cur, ref, B, R)
    np.testing.assert_array_equal(sad, bsad)
    np.testing.assert_array_equal(nsp, bnsp)
    np.testing.assert_array_equal(mv, bmv)


@pytest.mark.parametrize("H,W,B,R", CASES)
def test_dcds_sad_is_the_block_sad_at_its_vector(H, W, B, R):
    cur, ref = _frames("uniform", H, W, seed=7 + R)
    mv, sad, nsp = oracle.dcds(cur, ref, B, R)
    c32, r32 = cur.astype(np.int32), ref.astype(np.int32)
    for j in range(H // B):
        for i in range(W // B):
            dx, dy = int(mv[j, i, 0]), int(mv[j, i, 1])
            x, y = i * B + dx, j * B + dy
            assert 0 <= x <= W - B and 0 <= y <= H - B and abs(dx) <= R and abs(dy) <= R
            s = np.abs(c32[j * B:j * B + B, i * B:i * B + B] - r32[y:y + B, x:x + B]).sum()
            assert sad[j, i] == s
            assert oracle.block_sad(cur, ref, B, i * B, j * B, dx, dy) == s


def test_fs_translation_recovered_exactly():
    """A pure global translation (no noise): FS finds the shift on every block
    whose displaced block stays in the frame (the texture makes it unique)."""
    from synth import blurred_noise
    rng = np.random.Generator(np.random.PCG64(5))
    big = blurred_noise(rng, 96 + 32, 128 + 32, 1.5).astype(np.uint8)
    for sx, sy in [(0, 0), (1, 0), (-3, 2), (6, -5), (7, 7)]:
        ref = big[16:16 + 96, 16:16 + 128]
        cur = big[16 + sy:16 + sy + 96, 16 + sx:16 + sx + 128]
        # cur(x) = ref(x + s): the motion vector is s.
        mv, sad, _ = oracle.fullsearch(cur, ref, 16, 7)
        for j in range(6):
            for i in range(8):
                x, y = i * 16 + sx, j * 16 + sy
                if 0 <= x <= 128 - 16 and 0 <= y <= 96 - 16:
                    assert tuple(mv[j, i]) == (sx, sy) and sad[j, i] == 0


@pytest.mark.parametrize("B,R", [(16, 31), (8, 7), (16, 5)])
def test_crop_fs_equals_whole_frame(B, R):
    """The crop rule the 3840x2160 GPU test samples FS with: on every block
    of a small frame (most of them edge blocks), FS on the crop equals FS on
    the whole frame."""
    from conftest import crop_fs
    from synth import make_config
    seq = make_config(5, seed=17, frames=2)[:, :160, :256]
    cur, ref = seq[1], seq[0]
    mv, sad, nsp = oracle.fullsearch(cur, ref, B, R)
    for by in range(160 // B):
        for bx in range(256 // B):
            emv, esad, ensp = crop_fs(cur, ref, B, R, bx, by)
            assert (mv[by, bx] == emv).all() and sad[by, bx] == esad and nsp[by, bx] == ensp, (bx, by)
