"""Calls over more pairs than one launch holds.  A dispatch counts its
work-items in 32 bits, so the library splits a call into launches of at most
2^31 - 1 work-items over consecutive pair ranges.  The pairs on both sides of
a split must equal a call over them alone, and the oracle."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ITEMS = 2**31 - 1  # work-items per launch at most


def say(*a):
    print(*a, flush=True)


def same(a, b, what):
    for x, y, name in zip(a, b, ("mv", "sad", "nsp")):
        assert torch.equal(x, y), "%s: %s differs" % (what, name)


def check_oracle(got, seq, pairs, fn, B, R):
    mv, sad, nsp = [t.cpu().numpy() for t in got]
    for p in pairs:
        cur, ref = seq[p + 1].cpu().numpy(), seq[p].cpu().numpy()
        emv, esad, ensp = fn(cur, ref, B, R)
        assert np.array_equal(mv[p].reshape(emv.shape), emv), p
        assert np.array_equal(sad[p].reshape(esad.shape).astype(np.int64), esad.astype(np.int64)), p
        assert np.array_equal(nsp[p].reshape(ensp.shape).astype(np.int64), ensp.astype(np.int64)), p


def noise_sequence(frames, H, W, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return torch.randint(0, 256, (frames, H, W), dtype=torch.uint8, device=DEV, generator=g)


def test_dcds_split_over_launches():
    """16x16 frames, 8x8 blocks, one 8x8-block tile of 512 lanes per pair
    (rows per lane 1, 8 waves): 2^31 - 1 work-items hold 4 194 303 pairs, so
    4 194 306 pairs take two launches."""
    B, R, cfg = 8, 7, (1, 8)
    per = ITEMS // 512
    P = per + 3
    assert me.me_set_config(B, R, cfg) == me.ME_OK
    try:
        seq = noise_sequence(P + 1, 16, 16, seed=41)
        say("case dcds split: %d pairs, %d per launch" % (P, per))
        full = me.dcds(seq[1:], seq[:-1], B, R)
        lo = per - 2
        part = me.dcds(seq[lo + 1:], seq[lo:-1], B, R)
        same([t[lo:] for t in full], part, "dcds across the split")
        check_oracle(full, seq, (per - 1, per, P - 1), oracle.dcds, B, R)
        del seq, full, part
    finally:
        me.me_set_config(B, R, None)
        torch.cuda.empty_cache()


def test_fullsearch_split_over_launches():
    """1920x1088 at +-15: 8160 blocks of 256 lanes per pair, so one launch
    holds 1028 pairs and 1030 pairs take two."""
    B, R = 16, 15
    per = ITEMS // (8160 * 256)
    assert per == 1028
    P = per + 2
    seq = noise_sequence(P + 1, 1088, 1920, seed=42)
    say("case fs split: %d pairs, %d per launch" % (P, per))
    full = me.fullsearch(seq[1:], seq[:-1], B, R)
    lo = per - 2
    part = me.fullsearch(seq[lo + 1:], seq[lo:-1], B, R)
    same([t[lo:] for t in full], part, "fs across the split")
    check_oracle(full, seq, (per,), oracle.fullsearch, B, R)
    del seq, full, part
    torch.cuda.empty_cache()
