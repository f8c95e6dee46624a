"""The proposer's GPU kernels against the fp64 oracle (oracle/cnn.py), which
mirrors the GPU's bf16 storage points.  What remains between the two is fp32
accumulation order and the rare bf16 rounding decision it flips; the bounds
below follow from that (one flip moves a value by at most 2^-8 of itself)."""
import numpy as np
import pytest

from oracle import cnn
from synth import make_config

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.fixture(scope="module")
def frames():
    seq = make_config(3, seed=77, frames=3)[:, :256, :384]
    return seq


def close(got, ref, what, rel, cos_min):
    """Elementwise |got - ref| <= rel * (|ref| + rms(ref)), and cosine >= cos_min."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    rms = np.sqrt(np.mean(ref * ref)) + 1e-30
    err = np.abs(got - ref)
    worst = float(np.max(err / (np.abs(ref) + rms)))
    cos = float(got @ ref / (np.linalg.norm(got) * np.linalg.norm(ref) + 1e-30))
    say("%s: worst scaled error %.3e, cosine %.9f" % (what, worst, cos))
    assert worst <= rel, (what, worst)
    assert cos >= cos_min, (what, cos)


# bf16 keeps 8 significant bits: one rounding flip moves a stored value by
# <= 2^-8 of itself, while fp32 summation-order effects are ~1e-6 relative.
# The head (fp32, read from bf16 layer-3 activations) is bounded by one flip
# at its own scale.  Gradients sum products over many pixels, which dilutes
# a flip far below that: they are bounded tighter.
REL = 2.0 ** -8        # head and loss: elementwise, scaled
COS = 1.0 - 2.0 ** -16  # head: cosine
REL_G = 2.0 ** -12     # gradients: elementwise, scaled
COS_G = 1.0 - 2.0 ** -20


def test_forward_matches_oracle(frames):
    p = me.Proposer(seed=3)
    w = p.get_weights()
    cur, ref = frames[1:], frames[:-1]
    head = p.forward(dev(cur), dev(ref)).cpu().numpy()
    ps = cnn.unflatten(w)
    for k in range(2):
        x0 = cnn.downdiff(cur[k], ref[k])
        h, _ = cnn.forward(x0, ps)
        close(head[k], h, "head pair %d" % k, REL, COS)


def test_backward_matches_oracle(frames):
    p = me.Proposer(seed=4)
    w = p.get_weights()
    cur, ref = frames[1:2], frames[0:1]
    head = p.forward(dev(cur), dev(ref))
    rng = np.random.default_rng(0)
    dh = rng.normal(0, 1e-3, head.shape).astype(np.float32)
    p.backward(dev(dh))
    g = p.get_grads()
    ps = cnn.unflatten(w)
    x0 = cnn.downdiff(cur[0], ref[0])
    _, acts = cnn.forward(x0, ps)
    gref = cnn.flatten(cnn.backward(acts, ps, dh[0].astype(np.float64)))
    shapes = cnn.param_shapes()
    at = 0
    for li, (ws, bs) in enumerate(shapes):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        close(g[at:at + nw], gref[at:at + nw], "dW layer %d" % (li + 1), REL_G, COS_G)
        close(g[at + nw:at + nw + nb], gref[at + nw:at + nw + nb], "db layer %d" % (li + 1), REL_G, COS_G)
        at += nw + nb


def test_train_step_loss_and_adam(frames):
    p = me.Proposer(seed=5)
    w0 = p.get_weights().astype(np.float64)
    cur, ref = frames[1:], frames[:-1]
    rng = np.random.default_rng(1)
    tgt = rng.integers(-31, 32, (2, 16, 24, 2)).astype(np.int16)
    lr = 1e-3
    loss = float(p.train_step(dev(cur), dev(ref), dev(tgt), lr).cpu()[0])
    ps = cnn.unflatten(w0)
    heads = [cnn.forward(cnn.downdiff(cur[k], ref[k]), ps)[0] for k in range(2)]
    lref, dhead = cnn.loss_and_dhead(np.stack(heads), tgt)
    say("loss gpu %.7f oracle %.7f" % (loss, lref))
    assert abs(loss - lref) <= REL * abs(lref)
    # The gradient train_step built (loss gradient through both pairs)
    # against the oracle's backward of the oracle's loss gradient.
    g = p.get_grads().astype(np.float64)
    gref = sum(cnn.flatten(cnn.backward(cnn.forward(cnn.downdiff(cur[k], ref[k]), ps)[1], ps, dhead[k]))
               for k in range(2))
    at = 0
    for li, (ws, bs) in enumerate(cnn.param_shapes()):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        close(g[at:at + nw], gref[at:at + nw], "train dW layer %d" % (li + 1), REL_G, COS_G)
        close(g[at + nw:at + nw + nb], gref[at + nw:at + nw + nb], "train db layer %d" % (li + 1), REL_G, COS_G)
        at += nw + nb
    # Adam's first step from zero moments on the GPU's own gradient.
    m = 0.1 * g
    v = 0.001 * g * g
    step = lr * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    w1 = p.get_weights().astype(np.float64)
    np.testing.assert_allclose(w1, w0 - step, rtol=0, atol=1e-6 * lr + 1e-7)
    mm, vv, st = p.get_state()
    assert st == 1
    np.testing.assert_allclose(mm, m, rtol=1e-6, atol=1e-12)


def test_training_is_deterministic_and_resumable(frames):
    cur, ref = dev(frames[1:]), dev(frames[:-1])
    tgt = dev(np.random.default_rng(2).integers(-31, 32, (2, 16, 24, 2)).astype(np.int16))
    a = me.Proposer(seed=6)
    b = me.Proposer(seed=6)
    for _ in range(3):
        a.train_step(cur, ref, tgt, 2e-3)
    for _ in range(2):
        b.train_step(cur, ref, tgt, 2e-3)
    w, (m, v, st) = b.get_weights(), b.get_state()
    c = me.Proposer()
    c.set_weights(w)
    c.set_state(m, v, st)
    c.train_step(cur, ref, tgt, 2e-3)
    b.train_step(cur, ref, tgt, 2e-3)
    wa, wb, wc = a.get_weights(), b.get_weights(), c.get_weights()
    assert np.array_equal(wa, wb), "two identical runs differ"
    assert np.array_equal(wa, wc), "a resumed run differs"
    assert c.get_state()[2] == 3


def test_infer_decodes_the_head(frames):
    p = me.Proposer(seed=7)
    cur, ref = dev(frames[1:]), dev(frames[:-1])
    head = p.forward(cur, ref).cpu().numpy()
    s, o = p.infer(cur, ref, 31)
    es, eo = cnn.decode(head.astype(np.float32), 31)
    # The same fp32 values decide on both sides.
    es = np.clip(np.rint(head[..., :2].astype(np.float32) * np.float32(8)), -31, 31).astype(np.int16)
    assert np.array_equal(s.cpu().numpy(), es)
    assert np.array_equal(o.cpu().numpy(), eo)


@pytest.mark.parametrize("crop", [(8, 216, 4, 340), (0, 144, 0, 384), (16, 48, 32, 64)])
def test_infer_ragged_views(frames, crop):
    """The fused inference kernel on frames whose block grid leaves partial
    tiles (13x21, 9x24, 2x2 blocks), read through views whose rows start
    4-byte (not 16-byte) aligned, equals forward() + decode on a copy."""
    y0, y1, x0, x1 = crop
    p = me.Proposer(seed=9)
    full = dev(frames)
    cur, ref = full[1:, y0:y1, x0:x1], full[:-1, y0:y1, x0:x1]
    say("crop", crop, "pitch", cur.stride(-2), "pointer mod 16", cur.data_ptr() % 16)
    head = p.forward(cur.contiguous(), ref.contiguous()).cpu().numpy()
    s, o = p.infer(cur, ref, 15)
    es = np.clip(np.rint(head[..., :2].astype(np.float32) * np.float32(8)), -15, 15).astype(np.int16)
    eo = (head[..., 2] > 0).astype(np.uint8)
    assert s.shape == (2, (y1 - y0) // 16, (x1 - x0) // 16, 2)
    assert np.array_equal(s.cpu().numpy(), es)
    assert np.array_equal(o.cpu().numpy(), eo)


@pytest.mark.parametrize("shape", [(5, 256, 512), (4, 1088, 1920), (3, 2160, 3840)])
def test_infer_tile_order(shape):
    """Grids that are multiples of 8 workgroups take the XCD-local tile
    order (32 tiles on 32 workgroups; 405 tiles, and at 4K 1020 tiles with a
    partial last tile row, on at most 256): every block still gets exactly
    forward() + decode."""
    P, H, W = shape
    seq = (make_config(5, seed=21, frames=P) if H > 1088 else make_config(3, seed=21, frames=P))[:, :H, :W]
    p = me.Proposer(seed=11)
    cur, ref = dev(seq[1:]), dev(seq[:-1])
    head = p.forward(cur, ref).cpu().numpy()
    s, o = p.infer(cur, ref, 31)
    es = np.clip(np.rint(head[..., :2].astype(np.float32) * np.float32(8)), -31, 31).astype(np.int16)
    eo = (head[..., 2] > 0).astype(np.uint8)
    say("shape", shape, "tiles", (P - 1) * ((H // 16 + 7) // 8) * ((W // 16 + 7) // 8))
    assert np.array_equal(s.cpu().numpy(), es)
    assert np.array_equal(o.cpu().numpy(), eo)


def test_dcds_learned_equals_seeded_dcds(frames):
    p = me.Proposer(seed=8)
    cur, ref = dev(frames[1:]), dev(frames[:-1])
    got = me.dcds_learned(p, cur, ref, 31)
    s, o = p.infer(cur, ref, 31)
    exp = me.dcds(cur, ref, 16, 31, start=s, orient=o)
    for x, y in zip(got, exp):
        assert torch.equal(x, y)
    plain = me.dcds_learned(None, cur, ref, 31)
    for x, y in zip(plain, me.dcds(cur, ref, 16, 31)):
        assert torch.equal(x, y)


def test_set_weights_rejects_non_finite():
    p = me.Proposer()
    w = np.zeros(p.n, np.float32)
    w[5] = np.nan
    with pytest.raises(me.MEError):
        p.set_weights(w)


def test_forward_grid_limits():
    """forward and train_step put rows and pairs on grid dimensions y and z:
    more than 65535 pairs, or height/4 above 65535, is refused before any
    device work (the frame pointers here are never read)."""
    p = me.Proposer()
    fake = 0x1000
    L = me.lib()
    # 65536 pairs of 16x16 frames.
    assert L.me_proposer_forward(p.h, fake, fake, 16, 16, 16, 256, 65536, fake, None) == me.ME_EUNSUPPORTED
    # One 16x262160 frame: height/4 = 65540.
    assert L.me_proposer_forward(p.h, fake, fake, 16, 262160, 16, 16 * 262160, 1, fake, None) == me.ME_EUNSUPPORTED
    assert L.me_proposer_train_step(p.h, fake, fake, 16, 16, 16, 256, 65536, fake, 0.001, fake,
                                    None) == me.ME_EUNSUPPORTED
    # 16449 pairs of 1920x1088: 2^31 layer-1 pixels or more.
    W, H = 1920, 1088
    assert L.me_proposer_train_step(p.h, fake, fake, W, H, W, W * H, 16449, fake, 0.001, fake,
                                    None) == me.ME_EUNSUPPORTED
