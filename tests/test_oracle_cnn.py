"""Pins of the proposer oracle (oracle/cnn.py): the convolution against an
explicit index loop, the backward pass against finite differences, the loss
against closed forms, and bf16 rounding against known values."""
import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, w, b, s):
    H, W, Ci = x.shape
    Co = w.shape[3]
    Ho, Wo = (H - 1) // s + 1, (W - 1) // s + 1
    out = np.zeros((Ho, Wo, Co))
    for oy in range(Ho):
        for ox in range(Wo):
            for co in range(Co):
                acc = b[co]
                for ky in range(3):
                    for kx in range(3):
                        iy, ix = oy * s + ky - 1, ox * s + kx - 1
                        if 0 <= iy < H and 0 <= ix < W:
                            for ci in range(Ci):
                                acc += x[iy, ix, ci] * w[ky, kx, ci, co]
                out[oy, ox, co] = acc
    return out


@pytest.mark.parametrize("H,W,s", [(5, 7, 1), (6, 9, 2), (8, 8, 2), (1, 3, 1)])
def test_conv_matches_index_loop(H, W, s):
    rng = np.random.default_rng(H * 10 + W)
    x = rng.normal(size=(H, W, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    b = rng.normal(size=4)
    np.testing.assert_allclose(cnn.conv(x, w, b, s), brute_conv(x, w, b, s), rtol=1e-12, atol=1e-12)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3, 65504.0])
    got = cnn.bf16(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: ties go to the even significand (1.0);
    # 1 + 3*2^-8 is a tie between 1 + 2^-7 and 1 + 2^-6: even is 1 + 2^-6.
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -7 and got[3] == 1.0 + 2 ** -6
    assert got[4] == -2.5
    assert abs(got[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    assert got[6] == 65536.0  # 65504 rounds up with 8 significant bits


def test_loss_closed_forms():
    head = np.zeros((1, 3, 3))
    # Block 0: u - tx = 0.5 (quadratic branch), v - ty = 0, o = 0 with label 0.
    # Block 1: u - tx = -3 (linear branch), ty = 0, o = 0.
    # Block 2: tx = 0, ty = 16 (label vertical), o = 0.
    head[0, 0] = [0.5, 0.0, 0.0]
    head[0, 1] = [-3.0, 0.0, 0.0]
    tgt = np.array([[[0, 0], [0, 0], [0, 16]]])
    loss, dh = cnn.loss_and_dhead(head, tgt)
    hub = 0.125 + 2.5 + (2.0 - 0.5)
    bce = 3 * np.log(2.0)
    assert loss == pytest.approx((hub + 0.25 * bce) / 3, rel=1e-12)
    assert dh[0, 0, 0] == pytest.approx(0.5 / 3)
    assert dh[0, 1, 0] == pytest.approx(-1.0 / 3)
    assert dh[0, 2, 1] == pytest.approx(-1.0 / 3)
    assert dh[0, 2, 2] == pytest.approx(0.25 * (0.5 - 1.0) / 3)


def test_loss_is_a_mean_over_every_block():
    rng = np.random.default_rng(3)
    heads = rng.normal(size=(2, 3, 4, 3))
    tg = rng.integers(-9, 10, (2, 3, 4, 2))
    l_all, d_all = cnn.loss_and_dhead(heads, tg)
    parts = [cnn.loss_and_dhead(heads[k], tg[k]) for k in range(2)]
    assert l_all == pytest.approx(0.5 * (parts[0][0] + parts[1][0]), rel=1e-12)
    np.testing.assert_allclose(d_all[0], 0.5 * parts[0][1], rtol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    cur = rng.integers(0, 256, (32, 64)).astype(np.uint8)
    ref = rng.integers(0, 256, (32, 64)).astype(np.uint8)
    x0 = cnn.downdiff(cur, ref, round_=False)
    ps = cnn.init_params(1)
    ps = [(w, rng.normal(0, 0.1, b.shape)) for w, b in ps]
    tgt = rng.integers(-20, 21, (2, 4, 2))

    def L(flat):
        head, _ = cnn.forward(x0, cnn.unflatten(flat), round_=False)
        return cnn.loss_and_dhead(head, tgt)[0]

    flat = cnn.flatten(ps)
    head, acts = cnn.forward(x0, ps, round_=False)
    assert head.shape == (2, 4, 3)
    _, dh = cnn.loss_and_dhead(head, tgt)
    g = cnn.flatten(cnn.backward(acts, ps, dh, round_=False))
    idx = rng.choice(len(flat), 60, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = eps
        num = (L(flat + e) - L(flat - e)) / (2 * eps)
        assert num == pytest.approx(g[i], rel=1e-4, abs=1e-8), i


def test_shapes_and_counts():
    assert cnn.num_params() == 2 * 16 * 9 + 16 + 16 * 32 * 9 + 32 + 32 * 32 * 9 + 32 + 32 * 3 * 9 + 3
    x0 = cnn.downdiff(np.zeros((1088, 1920), np.uint8), np.zeros((1088, 1920), np.uint8))
    assert x0.shape == (272, 480, 2)
    head, acts = cnn.forward(x0, cnn.init_params(0))
    assert head.shape == (68, 120, 3) and [a.shape[2] for a in acts] == [2, 16, 32, 32]


def test_downdiff_on_known_box_means():
    """x0 from frames whose 4x4 box means are known by construction: each 4x4
    box of cur holds four copies of a, b, c, d (mean (a+b+c+d)/4), ref a
    constant; channel 0 is (mean - ref) / 32, channel 1 (mean - 128) / 64."""
    rng = np.random.default_rng(5)
    hb, wb = 3, 5
    vals = rng.integers(0, 256, (hb, wb, 4))
    cur = np.zeros((4 * hb, 4 * wb), np.uint8)
    for j in range(hb):
        for i in range(wb):
            box = np.repeat(vals[j, i], 4).reshape(4, 4)  # rows a a a a / b b b b / ...
            cur[4 * j:4 * j + 4, 4 * i:4 * i + 4] = box
    ref = np.full_like(cur, 100)
    x = cnn.downdiff(cur, ref, round_=False)
    mean = vals.sum(axis=-1) / 4.0
    assert x.shape == (hb, wb, 2)
    np.testing.assert_array_equal(x[..., 0], (mean - 100.0) / 32.0)
    np.testing.assert_array_equal(x[..., 1], (mean - 128.0) / 64.0)
    # A box is never mixed with its neighbours: one changed pixel moves one cell.
    cur2 = cur.copy()
    cur2[5, 9] = cur2[5, 9] ^ 4
    d = cnn.downdiff(cur2, ref, round_=False) - x
    assert np.count_nonzero(d[..., 0]) == 1 and d[1, 2, 0] != 0
    # Rounded input: the bf16 value nearest the exact one (8 significant bits).
    xr = cnn.downdiff(cur, ref)
    assert np.all(np.abs(xr - x) <= np.abs(x) * 2.0 ** -8)


def test_decode_rounding_and_clamp():
    """Start = 8 (u, v) rounded half to even (rint), clamped to +-R; vertical
    when o > 0 (o = 0 is horizontal)."""
    u = np.array([0.0625, 0.1875, 0.3125, -0.0625, -0.1875, 0.06, 0.07, 10.0, -10.0, 1.9375])
    # 8u = 0.5, 1.5, 2.5, -0.5, -1.5, 0.48, 0.56, 80, -80, 15.5
    want = np.array([0, 2, 2, 0, -2, 0, 1, 15, -15, 15])
    head = np.zeros((1, len(u), 3))
    head[0, :, 0] = u
    head[0, :, 1] = -u
    head[0, :, 2] = np.array([1e-9, 0.0, -1e-9, 5, -5, 0, 0, 0, 0, 0])
    s, o = cnn.decode(head, 15)
    np.testing.assert_array_equal(s[0, :, 0], want)
    np.testing.assert_array_equal(s[0, :, 1], -want)
    np.testing.assert_array_equal(o[0], [1, 0, 0, 1, 0, 0, 0, 0, 0, 0])
    s7, _ = cnn.decode(head, 7)
    np.testing.assert_array_equal(s7[0, :, 0], np.clip(want, -7, 7))
    assert s.dtype == np.int16 and o.dtype == np.uint8
