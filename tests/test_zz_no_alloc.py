"""me_batch_noalloc (the batch for callers that cannot allocate) against
me_batch, through the C ABI: two calls in a row on one stream, the second
with a smaller input, each job's outputs equal to me_batch's element by
element.  The first call spans more than one table-copy kernel (16 jobs
each); the second leaves most of the first call's table behind in the shared
array, which must not leak into its results."""
import ctypes
import functools

import numpy as np
import pytest

from synth import SequenceSpec, moving_sequence

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


KINDS = [(176, 144, 2), (352, 288, 8), (1280, 720, 20), (1920, 1088, 32)]


@functools.lru_cache(maxsize=None)
def sequences(n, frames, base_seed):
    out = []
    for s in range(n):
        W, H, nobj = KINDS[s % 4] if s % 5 else KINDS[0]
        out.append(dev(moving_sequence(SequenceSpec(W, H, frames, nobj, "laplace4x2", 15, base_seed + s))))
    return out


def poisoned(pairs, B):
    """Outputs pre-filled with a value no search writes."""
    outs = []
    for cur, _ in pairs:
        P, H, W = cur.shape
        outs.append((torch.full((P, H // B, W // B, 2), -32768, dtype=torch.int16, device=DEV),
                     torch.full((P, H // B, W // B), -1, dtype=torch.int32, device=DEV),
                     torch.full((P, H // B, W // B), -1, dtype=torch.int32, device=DEV)))
    return outs


@pytest.mark.parametrize("algo,B,R,seeded", [("dcds", 16, 15, False), ("dcds_s", 8, 7, False),
                                             ("fs", 16, 7, False), ("dcds", 16, 31, True)])
def test_noalloc_equals_batch_on_two_calls(algo, B, R, seeded):
    code = {"dcds": me.ME_ALGO_DCDS, "dcds_s": me.ME_ALGO_DCDS_S, "fs": me.ME_ALGO_FS}[algo]
    big = sequences(20, 3, 3000)
    small = sequences(3, 2, 4000)[:3]
    small = [s[:, :144, :176].contiguous() for s in small]   # a smaller input: QCIF crops
    rng = np.random.default_rng(7)
    for call, seqs in enumerate((big, small)):
        pairs = [(t[1:], t[:-1]) for t in seqs]
        starts = orients = None
        if seeded:
            starts = [dev(rng.integers(-R - 2, R + 3, (c.shape[0], c.shape[1] // B, c.shape[2] // B, 2))
                          .astype(np.int16)) for c, _ in pairs]
            orients = [dev(rng.integers(0, 2, (c.shape[0], c.shape[1] // B, c.shape[2] // B)).astype(np.uint8))
                       for c, _ in pairs]
        say("case noalloc %s B=%d R=%d seeded=%s call %d: %d jobs, %d blocks" %
            (algo, B, R, seeded, call, len(pairs), sum(c.shape[0] * (c.shape[1] // B) * (c.shape[2] // B)
                                                        for c, _ in pairs)))
        exp = me.batch(pairs, B, R, algo=code, starts=starts, orients=orients)
        got = me.batch_noalloc(pairs, B, R, algo=code, starts=starts, orients=orients, outs=poisoned(pairs, B))
        torch.cuda.synchronize()
        for j, (g, e) in enumerate(zip(got, exp)):
            for name, x, y in zip(("mv", "sad", "nsp"), g, e):
                assert torch.equal(x, y), "call %d job %d %s differs" % (call, j, name)


def test_noalloc_sse_and_limits():
    B, R = 16, 15
    seqs = sequences(5, 3, 5000)
    pairs = [(t[1:], t[:-1]) for t in seqs]
    sse_a = [torch.zeros((c.shape[0], c.shape[1] // B, c.shape[2] // B), dtype=torch.int32, device=DEV)
             for c, _ in pairs]
    sse_b = [torch.full_like(x, -1) for x in sse_a]
    exp = me.batch(pairs, B, R, sses=sse_a)
    got = me.batch_noalloc(pairs, B, R, sses=sse_b, outs=poisoned(pairs, B))
    torch.cuda.synchronize()
    for g, e, sa, sb in zip(got, exp, sse_a, sse_b):
        assert all(torch.equal(x, y) for x, y in zip(g, e)) and torch.equal(sa, sb)
    # Sizes beyond the array are refused before anything runs; none is a no-op.
    cur, ref = pairs[0]
    jobs, _ = me.make_jobs([(cur, ref)] * 513, B)
    assert me.me_batch_noalloc(jobs, 513, me.ME_ALGO_DCDS, B, R, 0) == me.ME_EUNSUPPORTED
    assert me.me_batch_noalloc(None, 0, me.ME_ALGO_DCDS, B, R, 0) == me.ME_OK
    jobs, _ = me.make_jobs([(cur, ref)], B)
    assert me.me_batch_noalloc(jobs, 1, me.ME_ALGO_DCDS, 12, R, 0) == me.ME_EUNSUPPORTED
    assert me.me_batch_noalloc(ctypes.cast(None, ctypes.POINTER(me.MeJob)), 1, me.ME_ALGO_DCDS, B, R, 0) \
        == me.ME_EINVAL
