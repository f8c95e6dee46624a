"""Batched persistent launches (me_batch) and the autotuner on the GPU: every
job of a mixed-size batch equals the single-call result and the oracle, over
several replays of the captured graph with different job mixes."""
import numpy as np
import pytest

import oracle
from synth import SequenceSpec, moving_sequence, qcif_pair

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


KINDS = [(176, 144, 2), (352, 288, 8), (1280, 720, 20), (1920, 1088, 32)]


@pytest.fixture(scope="module")
def streams():
    out = []
    for s in range(8):
        W, H, nobj = KINDS[s % 4]
        frames = 3 if W >= 1280 else 4
        seq = moving_sequence(SequenceSpec(W, H, frames, nobj, "laplace4x2", 15, 1000 + s))
        out.append((seq, dev(seq)))
    return out


def pairs_of(streams, idx):
    return [(t[1:], t[:-1]) for (_, t) in (streams[i] for i in idx)]


def equal(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("algo", ["dcds", "dcds_s", "fs"])
@pytest.mark.parametrize("B,R", [(16, 15), (8, 7), (16, 31)])
def test_batch_equals_single_calls_over_replays(streams, algo, B, R):
    code = {"dcds": me.ME_ALGO_DCDS, "dcds_s": me.ME_ALGO_DCDS_S, "fs": me.ME_ALGO_FS}[algo]
    mixes = [[0, 1, 2, 3], [3, 2, 1, 0, 4, 5], [1, 5], [0, 1, 2, 3, 4, 5, 6, 7]]
    for rep, mix in enumerate(mixes):
        say("case batch", algo, "B=%d R=%d replay %d jobs %s" % (B, R, rep, mix))
        pairs = pairs_of(streams, mix)
        got = me.batch(pairs, B, R, algo=code)
        # Eager work between replays (the graph must not depend on it).
        junk = torch.arange(1 << 20, device=DEV).sum()
        for (cur, ref), g in zip(pairs, got):
            if code == me.ME_ALGO_FS:
                exp = me.fullsearch(cur, ref, B, R)
            else:
                exp = me.dcds(cur, ref, B, R, algo=code)
            assert equal(g, exp), (algo, B, R, rep)
        torch.cuda.synchronize()
        del junk
    # Oracle on the QCIF and CIF jobs of the last mix.
    for i in (0, 1):
        seq = streams[i][0]
        g = got[i]
        for p in range(seq.shape[0] - 1):
            fn = oracle.fullsearch if code == me.ME_ALGO_FS else oracle.dcds
            kw = {} if code != me.ME_ALGO_DCDS_S else {"variant": oracle.VARIANT_DCDS_S}
            emv, esad, ensp = fn(seq[p + 1], seq[p], B, R, **kw)
            assert np.array_equal(g[0][p].cpu().numpy(), emv)
            assert np.array_equal(g[1][p].cpu().numpy(), esad.astype(np.int32))
            assert np.array_equal(g[2][p].cpu().numpy(), ensp.astype(np.int32))


def test_batch_seeded_jobs(streams):
    pairs = pairs_of(streams, [0, 1, 3])
    rng = np.random.default_rng(5)
    starts, orients = [], []
    for cur, _ in pairs:
        P, H, W = cur.shape
        starts.append(dev(rng.integers(-17, 18, (P, H // 16, W // 16, 2)).astype(np.int16)))
        orients.append(dev(rng.integers(0, 2, (P, H // 16, W // 16)).astype(np.uint8)))
    got = me.batch(pairs, 16, 15, starts=starts, orients=orients)
    for (cur, ref), s, o, g in zip(pairs, starts, orients, got):
        assert equal(g, me.dcds(cur, ref, 16, 15, start=s, orient=o))


def test_autotune_and_cache_roundtrip(streams, tmp_path):
    pairs = pairs_of(streams, [0, 1, 2])
    try:
        cfg, ms = me.autotune(pairs, 16, 15, reps=2)
        say("autotune best", cfg, ms)
        assert cfg[0] in (1, 2, 4) and cfg[1] in (1, 2, 4, 8) and cfg[2] in (1, 2, 4, 8, 16) and ms > 0
        assert me.me_get_config(16, 15) == cfg
        got = me.batch(pairs, 16, 15)
        for (cur, ref), g in zip(pairs, got):
            exp = oracle.dcds(cur[0].cpu().numpy(), ref[0].cpu().numpy(), 16, 15)
            assert np.array_equal(g[0][0].cpu().numpy(), exp[0])
        path = tmp_path / "tune.txt"
        assert me.me_autotune_save(str(path)) == me.ME_OK
        me.set_config(16, 15, None)
        rc, applied, rejected = me.me_autotune_load(str(path))
        assert rc == me.ME_OK and applied >= 1 and rejected == 0
        assert me.me_get_config(16, 15) == cfg
        # A reloaded result replaces the one recorded for the same key.
        path2 = tmp_path / "tune2.txt"
        assert me.me_autotune_save(str(path2)) == me.ME_OK
        rows = [ln.split() for ln in path2.read_text().splitlines() if ln and not ln.startswith("#")]
        keys = [tuple(r[:4]) for r in rows]
        assert len(keys) == len(set(keys)), "a reloaded result is recorded twice"
    finally:
        me.set_config(16, 15, None)


@pytest.mark.parametrize("grab", [1, 2, 8, 16])
def test_tiles_per_grab(streams, grab):
    """Every tiles-per-grab setting gives the single calls' results, in me_batch
    and in me_batch_noalloc."""
    pairs = pairs_of(streams, [3, 0, 2, 1, 5])
    try:
        rpl, wpg, _ = me.me_get_config(16, 15)
        me.set_config(16, 15, (rpl, wpg, grab))
        assert me.me_get_config(16, 15)[2] == grab
        got = me.batch(pairs, 16, 15)
        got2 = me.batch_noalloc(pairs, 16, 15)
        for (cur, ref), g, g2 in zip(pairs, got, got2):
            exp = me.dcds(cur, ref, 16, 15)
            assert equal(g, exp) and equal(g2, exp), grab
    finally:
        me.set_config(16, 15, None)


def test_shutdown_then_reuse(streams):
    pairs = pairs_of(streams, [0, 1])
    a = me.batch(pairs, 16, 15)
    torch.cuda.synchronize()
    assert me.me_shutdown() == me.ME_OK
    b = me.batch(pairs, 16, 15)
    for x, y in zip(a, b):
        assert equal(x, y)


def test_config4_scale_rotated_tables():
    """The benchmarked batch at full size: 64 streams (16 each of 176x144,
    352x288, 1280x720, 1920x1088), 30 frames, 16x16, +-15, 5.69 M blocks per
    launch.  Four job tables (the stream list rotated by 16) replay one
    captured graph; every job equals its single call element by element, and
    one sampled pair per size class equals the oracle."""
    from synth import batch_streams
    seqs_np = batch_streams(64, 30)
    seqs = [dev(s) for s in seqs_np]
    pairs = [(s[1:], s[:-1]) for s in seqs]
    single = [me.dcds(c, r, 16, 15) for c, r in pairs]
    stream = torch.cuda.current_stream().cuda_stream
    tables = []
    for k in range(4):
        order = [(i + 16 * k) % 64 for i in range(64)]
        tables.append((order, me.make_jobs([pairs[i] for i in order], 16)))
    for rep in range(2):  # two passes over the four tables
        for k, (order, (jobs, outs)) in enumerate(tables):
            say("case config4 pass %d table %d" % (rep, k))
            for o in outs:
                for x in o:
                    x.fill_(-1)
            assert me.me_batch(jobs, 64, me.ME_ALGO_DCDS, 16, 15, stream) == me.ME_OK
            for i, o in zip(order, outs):
                assert equal(o, single[i]), (rep, k, i)
    rng = np.random.default_rng(44)
    for kind in range(4):
        s = kind + 4 * int(rng.integers(0, 16))
        p = int(rng.integers(0, 29))
        emv, esad, ensp = oracle.dcds(seqs_np[s][p + 1], seqs_np[s][p], 16, 15)
        order, (jobs, outs) = tables[1]
        g = outs[order.index(s)]
        assert np.array_equal(g[0][p].cpu().numpy(), emv), (s, p)
        assert np.array_equal(g[1][p].cpu().numpy(), esad.astype(np.int32)), (s, p)
        assert np.array_equal(g[2][p].cpu().numpy(), ensp.astype(np.int32)), (s, p)
