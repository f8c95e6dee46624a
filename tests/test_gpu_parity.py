"""GPU parity: the HIP kernels (through the C ABI) against the CPU oracle,
bit-exact in motion vector, SAD and NSP for FS, DCDS, simplified DCDS and
seeded DCDS, on the seeded synthetic configurations, ragged tilings, every
supported range, both block sizes, and the cost-surface path (Table VII)."""
import numpy as np
import pytest

import oracle
from conftest import crop_fs, load_golden
from synth import blurred_noise, make_config, qcif_pair

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def assert_same(got, exp, what):
    gmv, gsad, gnsp = [t.cpu().numpy() for t in got]
    emv, esad, ensp = exp
    gmv = gmv.reshape(emv.shape)
    gsad = gsad.reshape(esad.shape)
    gnsp = gnsp.reshape(ensp.shape)
    bad = np.nonzero((gmv != emv).any(-1) | (gsad != esad.astype(np.int64)) | (gnsp != ensp.astype(np.int64)))
    if len(bad[0]):
        k = tuple(b[0] for b in bad)
        raise AssertionError("%s: %d blocks differ; first %s gpu mv=%s sad=%s nsp=%s oracle mv=%s sad=%s nsp=%s" % (
            what, len(bad[0]), k, gmv[k], gsad[k], gnsp[k], emv[k], esad[k], ensp[k]))


def oracle_pairs(fn, cur, ref, B, R, **kw):
    outs = [fn(cur[p], ref[p], B, R, **kw) for p in range(cur.shape[0])]
    return tuple(np.stack([o[i] for o in outs]) for i in range(3))


def random_pair(H, W, B, R, seed, kind="shifted"):
    if kind == "shifted":
        cur, ref, _ = qcif_pair(seed, W=W, H=H, block=B, R=R)
        return cur, ref
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(0, 256, (H, W), dtype=np.uint8), rng.integers(0, 256, (H, W), dtype=np.uint8)
    if kind == "flat":
        return np.full((H, W), 5, np.uint8), np.full((H, W), 5, np.uint8)
    if kind == "extreme":
        return np.zeros((H, W), np.uint8), np.full((H, W), 255, np.uint8)
    if kind == "checker":
        yy, xx = np.mgrid[0:H, 0:W]
        ref = (((xx + yy) % 2) * 9).astype(np.uint8)
        return (9 - ref).astype(np.uint8), ref
    raise ValueError(kind)


def run_all(cur, ref, B, R, label, seeded=True):
    """FS, DCDS, DCDS^S and seeded DCDS on [P, H, W] frames vs the oracle."""
    tc, tr = to_dev(cur), to_dev(ref)
    say("case", label, "B=%d R=%d shape=%s" % (B, R, cur.shape))
    assert_same(me.fullsearch(tc, tr, B, R), oracle_pairs(oracle.fullsearch, cur, ref, B, R), label + " fs")
    assert_same(me.dcds(tc, tr, B, R), oracle_pairs(oracle.dcds, cur, ref, B, R), label + " dcds")
    assert_same(me.dcds(tc, tr, B, R, algo=me.ME_ALGO_DCDS_S),
                oracle_pairs(oracle.dcds, cur, ref, B, R, variant=oracle.VARIANT_DCDS_S), label + " dcds_s")
    if seeded:
        P, H, W = cur.shape
        rng = np.random.default_rng(B * 100 + R)
        start = rng.integers(-R - 2, R + 3, (P, H // B, W // B, 2)).astype(np.int16)
        orient = rng.integers(0, 2, (P, H // B, W // B)).astype(np.uint8)
        got = me.dcds(tc, tr, B, R, start=to_dev(start), orient=to_dev(orient))
        exp = tuple(np.stack(x) for x in zip(*[oracle.dcds(cur[p], ref[p], B, R, start=start[p], orient=orient[p])
                                                for p in range(P)]))
        assert_same(got, exp, label + " seeded")


def test_qcif_config1():
    cur, ref, _ = qcif_pair(1)
    run_all(cur[None], ref[None], 16, 7, "qcif")


@pytest.mark.parametrize("B", [16, 8])
@pytest.mark.parametrize("R", [1, 2, 3, 4, 7, 8, 15, 31])
def test_ranges_and_ragged_tiles(B, R):
    # 80 x 48 is 5 x 3 blocks at B = 16 (ragged in both tile directions).
    cur, ref = random_pair(48, 80, B, min(R, 7), seed=R * 7 + B)
    run_all(cur[None], ref[None], B, R, "ragged")


@pytest.mark.parametrize("H,W,B", [(16, 16, 16), (8, 8, 8), (16, 64, 16), (64, 16, 16), (24, 8, 8), (8, 136, 8)])
def test_degenerate_frames(H, W, B):
    for kind in ["uniform", "shifted"]:
        cur, ref = random_pair(H, W, B, 3, seed=H + W, kind=kind)
        for R in (1, 7, 31):
            run_all(cur[None], ref[None], B, R, "degenerate-" + kind)


@pytest.mark.parametrize("kind", ["flat", "extreme", "checker", "uniform"])
def test_ties_and_extremes(kind):
    for B in (16, 8):
        cur, ref = random_pair(64, 96, B, 7, seed=3, kind=kind)
        run_all(cur[None], ref[None], B, 7, kind)


def test_cif_multi_pair_call():
    seq = make_config(2, frames=7)
    cur, ref = seq[1:], seq[:-1]
    for B in (16, 8):
        tseq = to_dev(seq)
        tc, tr = tseq[1:], tseq[:-1]
        say("case cif 6 pairs B=%d" % B)
        assert_same(me.dcds(tc, tr, B, 7), oracle_pairs(oracle.dcds, cur, ref, B, 7), "cif dcds")
        assert_same(me.fullsearch(tc, tr, B, 7), oracle_pairs(oracle.fullsearch, cur, ref, B, 7), "cif fs")


def test_paperlike_all_pairs():
    """Config 6 (the paper's operating point), all 59 pairs in one call:
    DCDS, DCDS^S and FS against the oracle."""
    seq = make_config(6)
    cur, ref = seq[1:], seq[:-1]
    tseq = to_dev(seq)
    tc, tr = tseq[1:], tseq[:-1]
    say("case config 6, 59 pairs, B=16, R=7")
    assert_same(me.dcds(tc, tr, 16, 7), oracle_pairs(oracle.dcds, cur, ref, 16, 7), "config 6 dcds")
    assert_same(me.dcds(tc, tr, 16, 7, algo=me.ME_ALGO_DCDS_S),
                oracle_pairs(oracle.dcds, cur, ref, 16, 7, variant=oracle.VARIANT_DCDS_S), "config 6 dcds_s")
    assert_same(me.fullsearch(tc, tr, 16, 7), oracle_pairs(oracle.fullsearch, cur, ref, 16, 7), "config 6 fs")


@pytest.mark.parametrize("case", range(24))
def test_random_configurations(case):
    """Seeded random shapes, ranges, block sizes, pair counts, row pitches and
    4-byte frame offsets: every search against the oracle."""
    rng = np.random.default_rng(1000 + case)
    B = int(rng.choice([8, 16]))
    R = int(rng.integers(1, 32))
    bh, bw, P = int(rng.integers(1, 9)), int(rng.integers(1, 13)), int(rng.integers(1, 4))
    H, W = bh * B, bw * B
    pad = 4 * int(rng.integers(0, 5))      # extra row bytes
    off = 4 * int(rng.integers(0, 4))      # frame start offset inside its row
    kind = str(rng.choice(["shifted", "uniform", "checker"]))
    frames = [random_pair(H, W, B, min(R, 7), seed=2000 + case * 10 + p, kind=kind) for p in range(P)]
    cur = np.stack([f[0] for f in frames])
    ref = np.stack([f[1] for f in frames])
    big = np.zeros((2, P, H, off + W + pad), np.uint8)
    big[0, :, :, off:off + W], big[1, :, :, off:off + W] = cur, ref
    tb = to_dev(big)
    tc, tr = tb[0, :, :, off:off + W], tb[1, :, :, off:off + W]
    label = "random case %d B=%d R=%d %dx%d P=%d pad=%d off=%d %s" % (case, B, R, H, W, P, pad, off, kind)
    say(label)
    assert_same(me.fullsearch(tc, tr, B, R), oracle_pairs(oracle.fullsearch, cur, ref, B, R), label + " fs")
    assert_same(me.dcds(tc, tr, B, R), oracle_pairs(oracle.dcds, cur, ref, B, R), label + " dcds")
    assert_same(me.dcds(tc, tr, B, R, algo=me.ME_ALGO_DCDS_S),
                oracle_pairs(oracle.dcds, cur, ref, B, R, variant=oracle.VARIANT_DCDS_S), label + " dcds_s")
    start = rng.integers(-R - 2, R + 3, (P, bh, bw, 2)).astype(np.int16)
    orient = rng.integers(0, 2, (P, bh, bw)).astype(np.uint8)
    got = me.dcds(tc, tr, B, R, start=to_dev(start), orient=to_dev(orient))
    exp = tuple(np.stack(x) for x in zip(*[oracle.dcds(cur[p], ref[p], B, R, start=start[p], orient=orient[p])
                                            for p in range(P)]))
    assert_same(got, exp, label + " seeded")


def test_pitch_wider_than_frame():
    cur, ref = random_pair(64, 96, 16, 7, seed=9)
    big_c = np.zeros((64, 128), np.uint8)
    big_r = np.zeros((64, 128), np.uint8)
    big_c[:, :96], big_r[:, :96] = cur, ref
    tc, tr = to_dev(big_c)[:, :96], to_dev(big_r)[:, :96]
    assert tc.stride(0) == 128
    say("case pitch 128 width 96")
    assert_same(me.dcds(tc, tr, 16, 7), oracle_pairs(oracle.dcds, cur[None], ref[None], 16, 7), "pitch dcds")
    assert_same(me.fullsearch(tc, tr, 16, 7), oracle_pairs(oracle.fullsearch, cur[None], ref[None], 16, 7), "pitch fs")


def test_pitch_of_2_23_bytes_and_more():
    """Frames of few rows may have row pitches beyond 24-bit products (height *
    pitch < 2^31 is the only limit): 16 rows at a pitch of 2^23 + 16 bytes."""
    cur, ref = random_pair(16, 32, 16, 7, seed=12)
    pitch = (1 << 23) + 16
    big = torch.zeros((2, 16, pitch), dtype=torch.uint8, device=DEV)
    big[0, :, :32], big[1, :, :32] = to_dev(cur), to_dev(ref)
    tc, tr = big[0:1, :, :32], big[1:2, :, :32]
    assert tc.stride(1) == pitch
    for R in (7, 15):
        say("case pitch 2^23 + 16, R=%d" % R)
        assert_same(me.fullsearch(tc, tr, 16, R), oracle_pairs(oracle.fullsearch, cur[None], ref[None], 16, R),
                    "wide pitch fs")
        assert_same(me.dcds(tc, tr, 16, R), oracle_pairs(oracle.dcds, cur[None], ref[None], 16, R),
                    "wide pitch dcds")
    del big
    torch.cuda.empty_cache()


def test_caller_tensors_are_checked_before_any_launch():
    """Outputs, start vectors and orientations that do not match the block
    grid raise in the binding; nothing is launched."""
    cur, ref = random_pair(32, 64, 16, 7, seed=5)
    tc, tr = to_dev(cur), to_dev(ref)
    mv = torch.zeros((1, 2, 4, 2), dtype=torch.int16, device=DEV)
    small = torch.zeros((1, 2, 3), dtype=torch.int32, device=DEV)
    ok = torch.zeros((1, 2, 4), dtype=torch.int32, device=DEV)
    with pytest.raises(ValueError):
        me.dcds(tc, tr, 16, 7, out=(mv, small, ok))
    with pytest.raises(ValueError):
        me.fullsearch(tc, tr, 16, 7, out=(mv, ok, ok.to(torch.int16)))
    with pytest.raises(ValueError):
        me.dcds(tc, tr, 16, 7, start=torch.zeros((1, 2, 3, 2), dtype=torch.int16, device=DEV))
    with pytest.raises(ValueError):
        me.search(tc, tr, 16, 7, sse=True, out=(mv, ok, ok.clone(), small))
    got = me.dcds(tc, tr, 16, 7, out=(mv, ok, ok.clone()))
    assert_same(got, oracle_pairs(oracle.dcds, cur[None], ref[None], 16, 7), "checked outputs")


def test_zero_pairs_is_a_no_op():
    t = torch.zeros((0, 32, 32), dtype=torch.uint8, device=DEV)
    mv, sad, nsp = me.dcds(t, t, 16, 7)
    assert mv.shape == (0, 2, 2, 2)
    me.fullsearch(t, t, 16, 7)
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def seq1080():
    say("generating the 1920x1088 sequence")
    return make_config(3)


@pytest.mark.parametrize("B", [16, 8])
def test_1080p_all_pairs_dcds_in_one_call(seq1080, B):
    """The benchmark's launch: all 59 pairs of the 1920x1088 sequence in one call."""
    tseq = to_dev(seq1080)
    say("case 1080p 59 pairs DCDS B=%d" % B)
    got = me.dcds(tseq[1:], tseq[:-1], B, 15)
    exp = oracle_pairs(oracle.dcds, seq1080[1:], seq1080[:-1], B, 15)
    assert_same(got, exp, "1080p dcds")
    got2 = me.dcds(tseq[1:], tseq[:-1], B, 15)
    for a, b in zip(got, got2):
        assert torch.equal(a, b), "DCDS is not deterministic"


@pytest.mark.parametrize("B", [16, 8])
def test_1080p_dcds_with_4_byte_loads(seq1080, B):
    """Three 1920x1088 pairs read through views 4 bytes off a 16-byte
    boundary (4-byte loads), so that interior tiles (whose window rows all
    lie in the frame) and border tiles both take the 4-byte staging."""
    P = 3
    big = np.zeros((P + 1, 1088, 1920 + 16), np.uint8)
    big[:, :, 4:1924] = seq1080[:P + 1]
    tb = to_dev(big)
    view = tb[:, :, 4:1924]
    assert view.data_ptr() % 16 == 4 and view.stride(1) % 16 == 0
    say("case 1080p 4-byte loads B=%d" % B)
    got = me.dcds(view[1:], view[:-1], B, 15)
    assert_same(got, oracle_pairs(oracle.dcds, seq1080[1:P + 1], seq1080[:P], B, 15), "1080p dcds 4-byte loads")


@pytest.mark.parametrize("B", [16, 8])
def test_1080p_fs_sampled_pairs(seq1080, B):
    """FS over all 59 pairs in one call; the oracle checks three sampled pairs."""
    tseq = to_dev(seq1080)
    say("case 1080p 59 pairs FS B=%d" % B)
    mv, sad, nsp = me.fullsearch(tseq[1:], tseq[:-1], B, 15)
    for p in (0, 29, 58):
        exp = oracle.fullsearch(seq1080[p + 1], seq1080[p], B, 15)
        assert_same((mv[p], sad[p], nsp[p]), exp, "1080p fs pair %d" % p)


@pytest.fixture(scope="module")
def seq4k():
    say("generating 3 frames of the 3840x2160 sequence")
    return make_config(5, frames=3)


def test_4k_r31_dcds_all_blocks(seq4k):
    """The 3840x2160, +-31 configuration: DCDS, DCDS^S and seeded DCDS over
    two whole pairs (64 800 blocks) against the oracle."""
    run = seq4k
    cur, ref = run[1:], run[:-1]
    tc, tr = to_dev(cur), to_dev(ref)
    say("case 4k R=31 dcds")
    assert_same(me.dcds(tc, tr, 16, 31), oracle_pairs(oracle.dcds, cur, ref, 16, 31), "4k dcds")
    assert_same(me.dcds(tc, tr, 16, 31, algo=me.ME_ALGO_DCDS_S),
                oracle_pairs(oracle.dcds, cur, ref, 16, 31, variant=oracle.VARIANT_DCDS_S), "4k dcds_s")
    P, H, W = cur.shape
    rng = np.random.default_rng(31)
    start = rng.integers(-33, 34, (P, H // 16, W // 16, 2)).astype(np.int16)
    orient = rng.integers(0, 2, (P, H // 16, W // 16)).astype(np.uint8)
    got = me.dcds(tc, tr, 16, 31, start=to_dev(start), orient=to_dev(orient))
    exp = tuple(np.stack(x) for x in zip(*[oracle.dcds(cur[p], ref[p], 16, 31, start=start[p], orient=orient[p])
                                            for p in range(P)]))
    assert_same(got, exp, "4k seeded")


def test_4k_r31_fs_sampled_blocks(seq4k):
    """FS at 3840x2160, +-31 (3969 candidates per block): the whole frame on
    the GPU, the oracle on the four corners, edge blocks and random interior
    blocks, each from a crop that holds its search window."""
    cur, ref = seq4k[2], seq4k[1]
    bh, bw = cur.shape[0] // 16, cur.shape[1] // 16
    mv, sad, nsp = [t.cpu().numpy() for t in me.fullsearch(to_dev(cur), to_dev(ref), 16, 31)]
    mv, sad, nsp = mv.reshape(bh, bw, 2), sad.reshape(bh, bw), nsp.reshape(bh, bw)
    rng = np.random.default_rng(5)
    picks = [(0, 0), (bw - 1, 0), (0, bh - 1), (bw - 1, bh - 1), (1, 1), (bw // 2, 0), (0, bh // 2), (bw - 2, bh - 2)]
    picks += [(int(rng.integers(0, bw)), int(rng.integers(0, bh))) for _ in range(40)]
    say("case 4k R=31 fs, %d sampled blocks" % len(picks))
    for bx, by in picks:
        emv, esad, ensp = crop_fs(cur, ref, 16, 31, bx, by)
        assert (mv[by, bx] == emv).all() and sad[by, bx] == esad and nsp[by, bx] == ensp, (
            "block", bx, by, mv[by, bx], sad[by, bx], nsp[by, bx], emv, esad, ensp)


def ideal_cost(t, R):
    ys, xs = np.mgrid[-R:R + 1, -R:R + 1]
    return ((xs - t[0]) ** 2 + (ys - t[1]) ** 2).astype(np.int32)


def test_table7_on_device():
    """The ideal condition of §III-C run by the GPU control flow: Table VII."""
    R = 7
    table = load_golden("table7_dcds_nsp.txt", int)
    ts = [(x, y) for y in range(-R, R + 1) for x in range(-R, R + 1)]
    cost = np.stack([ideal_cost(t, R) for t in ts])
    mv, c, nsp = me.dcds_surface(to_dev(cost))
    mv, c, nsp = mv.cpu().numpy(), c.cpu().numpy(), nsp.cpu().numpy()
    for i, t in enumerate(ts):
        assert tuple(mv[i]) == t and c[i] == 0
        assert nsp[i] == table[abs(t[1]), abs(t[0])], t


@pytest.mark.parametrize("R", [2, 3, 7, 15, 31])
def test_random_surfaces_vs_oracle(R):
    rng = np.random.default_rng(R)
    n, side = 400, 2 * R + 1
    cost = rng.integers(0, 40, (n, side, side)).astype(np.int32)
    valid = np.zeros((n, side, side), np.uint8)
    start = rng.integers(-R, R + 1, (n, 2)).astype(np.int16)
    orient = rng.integers(0, 2, n).astype(np.uint8)
    for i in range(n):
        lx, hx = sorted(rng.integers(-R, R + 1, 2))
        ly, hy = sorted(rng.integers(-R, R + 1, 2))
        lx, hx, ly, hy = min(lx, 0), max(hx, 0), min(ly, 0), max(hy, 0)
        valid[i, ly + R:hy + R + 1, lx + R:hx + R + 1] = 1
        start[i, 0] = np.clip(start[i, 0], lx, hx)
        start[i, 1] = np.clip(start[i, 1], ly, hy)
    for algo, variant in [(me.ME_ALGO_DCDS, oracle.VARIANT_DCDS), (me.ME_ALGO_DCDS_S, oracle.VARIANT_DCDS_S)]:
        for seeded in (False, True):
            got = me.dcds_surface(to_dev(cost), to_dev(valid), algo=algo,
                                  start=to_dev(start) if seeded else None, orient=to_dev(orient) if seeded else None)
            gmv, gc, gn = [x.cpu().numpy() for x in got]
            for i in range(n):
                kw = dict(start=start[i], orient_v=bool(orient[i])) if seeded else {}
                emv, ec, en = oracle.dcds_surface(cost[i], valid[i], variant=variant, **kw)
                assert (tuple(gmv[i]), gc[i], gn[i]) == (emv, ec, en), (R, algo, seeded, i)


CONFIGS16 = [(r, w) for r in (1, 2, 4) for w in (1, 2, 4, 8)]
CONFIGS8 = [(r, w) for r in (1, 2) for w in (1, 2, 4, 8)]


@pytest.mark.parametrize("B,cfg", [(16, c) for c in CONFIGS16] + [(8, c) for c in CONFIGS8])
def test_every_kernel_configuration(B, cfg, seq1080):
    """Each rows-per-lane x waves-per-group layout gives the oracle's results:
    ragged small frames at every range class, with 16-byte and with 4-byte
    loads (frames 4 bytes off a 16-byte boundary), and two 1920x1088 pairs."""
    try:
        for R in (3, 7, 8, 15, 16, 31):
            assert me.me_set_config(B, R, cfg) == me.ME_OK
            cur, ref = random_pair(48, 80, B, min(R, 7), seed=R * 11 + B)
            say("case config", cfg, "B=%d R=%d ragged" % (B, R))
            tc, tr = to_dev(cur[None]), to_dev(ref[None])
            assert_same(me.dcds(tc, tr, B, R), oracle_pairs(oracle.dcds, cur[None], ref[None], B, R), "cfg dcds")
            assert_same(me.dcds(tc, tr, B, R, algo=me.ME_ALGO_DCDS_S),
                        oracle_pairs(oracle.dcds, cur[None], ref[None], B, R, variant=oracle.VARIANT_DCDS_S),
                        "cfg dcds_s")
            say("case config", cfg, "B=%d R=%d ragged, 4-byte loads" % (B, R))
            big = np.zeros((2, 1, 48, 96), np.uint8)
            big[0, 0, :, 4:84], big[1, 0, :, 4:84] = cur, ref
            tb = to_dev(big)
            assert_same(me.dcds(tb[0, :, :, 4:84], tb[1, :, :, 4:84], B, R),
                        oracle_pairs(oracle.dcds, cur[None], ref[None], B, R), "cfg dcds 4-byte loads")
        tseq = to_dev(seq1080[:3])
        say("case config", cfg, "B=%d 1080p" % B)
        assert_same(me.dcds(tseq[1:], tseq[:-1], B, 15),
                    oracle_pairs(oracle.dcds, seq1080[1:3], seq1080[:2], B, 15), "cfg 1080p")
    finally:
        for R in (7, 15, 31):
            me.me_set_config(B, R, None)
