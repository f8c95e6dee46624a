"""The quality epilogue on the GPU against the oracle: the per-block squared
error of the motion-compensated block (fused into FS, DCDS, DCDS^S, seeded
DCDS and the batched launch) bit-exact, and the per-pair records of
me_frame_quality (integer sums exact, floating measures to 1e-12)."""
import math

import numpy as np
import pytest

import oracle
from oracle import quality as q
from synth import make_config, qcif_pair
from test_oracle_quality import random_field

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ALGOS = {"fs": me.ME_ALGO_FS, "dcds": me.ME_ALGO_DCDS, "dcds_s": me.ME_ALGO_DCDS_S}


def say(*a):
    print(*a, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def oracle_search(algo, cur, ref, B, R, start=None):
    if algo == "fs":
        return oracle.fullsearch(cur, ref, B, R)
    v = oracle.VARIANT_DCDS_S if algo == "dcds_s" else oracle.VARIANT_DCDS
    return oracle.dcds(cur, ref, B, R, start=start, variant=v)


def check_pairs(cur, ref, B, R, algo, label, starts=None, pairs=None):
    """cur, ref: [P, H, W] numpy; compares every pair in `pairs` (default all)."""
    say("case %s %s B=%d R=%d" % (label, algo, B, R))
    st = to_dev(starts) if starts is not None else None
    mv, sad, nsp, sse = me.search(to_dev(cur), to_dev(ref), B, R, ALGOS[algo], start=st, sse=True)
    mv, sad, nsp, sse = [t.cpu().numpy() for t in (mv, sad, nsp, sse)]
    for p in (range(cur.shape[0]) if pairs is None else pairs):
        emv, esad, ensp = oracle_search(algo, cur[p], ref[p], B, R, None if starts is None else starts[p])
        assert np.array_equal(mv[p], emv) and np.array_equal(sad[p], esad.astype(np.int64)), (label, p)
        assert np.array_equal(nsp[p], ensp.astype(np.int64)), (label, p)
        r = q.pair_quality(cur[p], ref[p], emv, B)
        np.testing.assert_array_equal(sse[p], r["block_sse"], err_msg="%s pair %d" % (label, p))


@pytest.mark.parametrize("algo", ["fs", "dcds", "dcds_s"])
@pytest.mark.parametrize("B", [16, 8])
def test_sse_qcif(algo, B):
    cur, ref, _ = qcif_pair(9)
    check_pairs(cur[None], ref[None], B, 7, algo, "qcif")


@pytest.mark.parametrize("algo", ["fs", "dcds"])
def test_sse_extreme_values(algo):
    """0 against 255 everywhere: 255^2 * 256 = 16 646 400 per 16x16 block, near the 2^24 bound."""
    cur = np.zeros((1, 64, 96), np.uint8)
    ref = np.full((1, 64, 96), 255, np.uint8)
    check_pairs(cur, ref, 16, 7, algo, "extreme")
    got = me.search(to_dev(cur), to_dev(ref), 16, 7, ALGOS[algo], sse=True)[3]
    assert int(got.max()) == 255 * 255 * 256


@pytest.mark.parametrize("algo", ["fs", "dcds", "dcds_s"])
def test_sse_cif_multi_pair(algo):
    seq = make_config(2, seed=21, frames=4)
    check_pairs(seq[1:], seq[:-1], 16, 15, algo, "cif")


def test_sse_seeded():
    seq = make_config(2, seed=22, frames=3)
    cur, ref = seq[1:], seq[:-1]
    rng = np.random.default_rng(5)
    starts = rng.integers(-15, 16, (2, 18, 22, 2)).astype(np.int16)
    check_pairs(cur, ref, 16, 15, "dcds", "cif seeded", starts=starts)


def test_sse_1088p_sampled():
    seq = make_config(3, frames=6)
    check_pairs(seq[1:], seq[:-1], 16, 15, "dcds", "1088p", pairs=[0, 4])


def test_batch_sse_equals_search():
    seqs = [make_config(1, seed=s) for s in (30, 31)] + [make_config(2, seed=32, frames=3)]
    pairs = [(to_dev(s[1:]), to_dev(s[:-1])) for s in seqs]
    for algo in ("fs", "dcds"):
        sses = [torch.empty((c.shape[0], c.shape[1] // 16, c.shape[2] // 16), dtype=torch.int32, device=DEV)
                for c, _ in pairs]
        outs = me.batch(pairs, 16, 15, ALGOS[algo], sses=sses)
        for (c, r), o, e in zip(pairs, outs, sses):
            ref_out = me.search(c, r, 16, 15, ALGOS[algo], sse=True)
            for x, y in zip(tuple(o) + (e,), ref_out):
                assert torch.equal(x, y), algo


@pytest.mark.parametrize("B", [16, 8])
def test_frame_quality_matches_oracle(B):
    seq = make_config(2, seed=40, frames=4)
    cur, ref = seq[1:], seq[:-1]
    rng = np.random.default_rng(B)
    P, H, W = cur.shape
    mv = np.stack([random_field(rng, H, W, B, 7) for _ in range(P)])
    tv = np.stack([random_field(rng, H, W, B, 7) for _ in range(P)])
    tv[:, ::3] = mv[:, ::3]  # some blocks agree
    exp = [q.pair_quality(cur[p], ref[p], mv[p], B, mv_true=tv[p]) for p in range(P)]
    sad = np.stack([e["block_sad"] for e in exp]).astype(np.int32)
    sse = np.stack([e["block_sse"] for e in exp]).astype(np.int32)
    got = me.frame_quality(to_dev(mv), to_dev(sad), to_dev(sse), to_dev(tv), block=B)
    for p in range(P):
        g, e = got[p], exp[p]
        say("pair %d: psnr %.6f mad %.4f dist %.4f equal %d" % (p, g["psnr"], g["mad"], g["dist"], g["equal"]))
        assert int(g["sad"]) == e["sad"] and int(g["sse"]) == e["sse"]
        assert int(g["blocks"]) == e["blocks"] and int(g["equal"]) == e["equal"]
        assert g["mad"] == pytest.approx(e["mad"], rel=1e-15) and g["mse"] == pytest.approx(e["mse"], rel=1e-15)
        assert g["psnr"] == pytest.approx(e["psnr"], rel=1e-12)
        assert g["dist"] == pytest.approx(e["dist"], rel=1e-12)
    none = me.frame_quality(to_dev(mv), to_dev(sad), to_dev(sse), None, block=B)
    assert np.all(none["equal"] == 0) and np.all(none["dist"] == 0.0)
    assert np.array_equal(none["sse"], got["sse"])


def test_frame_quality_perfect_match():
    ref = np.random.default_rng(2).integers(0, 256, (1, 32, 48)).astype(np.uint8)
    mv, sad, nsp, sse = me.search(to_dev(ref), to_dev(ref), 16, 7, me.ME_ALGO_DCDS, sse=True)
    rec = me.frame_quality(mv, sad, sse, mv, block=16)[0]
    assert rec["sse"] == 0 and math.isinf(rec["psnr"]) and rec["equal"] == 6 and rec["dist"] == 0.0


def test_table9_columns_on_qcif():
    """FS and DCDS on config 1 with FS as the truth: the GPU's records equal
    the oracle's, and FS has the smaller MAD and probability 1."""
    cur, ref, _ = qcif_pair(1)
    c, r = to_dev(cur[None]), to_dev(ref[None])
    fmv, fsad, _, fsse = me.search(c, r, 16, 7, me.ME_ALGO_FS, sse=True)
    dmv, dsad, _, dsse = me.search(c, r, 16, 7, me.ME_ALGO_DCDS, sse=True)
    fq = me.frame_quality(fmv, fsad, fsse, fmv)[0]
    dq = me.frame_quality(dmv, dsad, dsse, fmv)[0]
    emv_fs = oracle.fullsearch(cur, ref, 16, 7)[0]
    emv_d = oracle.dcds(cur, ref, 16, 7)[0]
    e = q.pair_quality(cur, ref, emv_d, 16, mv_true=emv_fs)
    say("FS mad %.4f psnr %.3f | DCDS mad %.4f psnr %.3f dist %.4f p %.4f" % (
        fq["mad"], fq["psnr"], dq["mad"], dq["psnr"], dq["dist"] / dq["blocks"], dq["equal"] / dq["blocks"]))
    assert fq["equal"] == fq["blocks"] and fq["mad"] <= dq["mad"]
    assert int(dq["sse"]) == e["sse"] and int(dq["equal"]) == e["equal"]
    assert dq["dist"] == pytest.approx(e["dist"], rel=1e-12)
