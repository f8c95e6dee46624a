"""MVP statistics (§II-C) on the GPU against the oracle: the counters of
me_mvp_stats bit-exact (full-search vector, best point of the CDS cross and
of the 5x5 square per block), accumulation across calls, and the tables of
me_mvp_tables equal to the oracle's to the last bit of fp64."""
import numpy as np
import pytest

from oracle import mvp
from synth import make_config, qcif_pair

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(counts):
    return tuple(c.cpu().numpy().astype(np.int64).reshape(-1) for c in counts)


def check_counts(cur, ref, B, R, label):
    """cur, ref: [P, H, W] numpy."""
    say("case %s B=%d R=%d pairs=%d" % (label, B, R, cur.shape[0]))
    got = host(me.mvp_stats(to_dev(cur), to_dev(ref), B, R))
    acc = None
    for p in range(cur.shape[0]):
        acc = mvp.counts(cur[p], ref[p], B, R, acc)
    for g, e, name in zip(got, acc, ("hist", "d1", "d2")):
        np.testing.assert_array_equal(g, e.reshape(-1), err_msg="%s %s" % (label, name))
    return got


@pytest.mark.parametrize("B", [16, 8])
def test_counts_qcif(B):
    cur, ref, _ = qcif_pair(3)
    check_counts(cur[None], ref[None], B, 7, "qcif")


@pytest.mark.parametrize("R", [7, 15, 2])
def test_counts_cif(R):
    seq = make_config(2, seed=50, frames=3)
    check_counts(seq[1:], seq[:-1], 16, R, "cif")


def test_accumulation_across_calls():
    seq = make_config(2, seed=51, frames=4)
    cur, ref = to_dev(seq[1:]), to_dev(seq[:-1])
    once = host(me.mvp_stats(cur, ref, 16, 7))
    c = me.mvp_stats(cur[:1], ref[:1], 16, 7)
    c = me.mvp_stats(cur[1:], ref[1:], 16, 7, counts=c)
    for a, b in zip(once, host(c)):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("R", [7, 1, 31])
def test_tables_match_oracle(R):
    seq = make_config(2, seed=52, frames=3)
    counts = me.mvp_stats(to_dev(seq[1:]), to_dev(seq[:-1]), 16, R)
    got = me.mvp_tables(counts, R)
    exp = mvp.tables(*host(counts), R)
    for k, e in exp.items():
        np.testing.assert_allclose(got[k], e, rtol=1e-15, atol=0, err_msg=k)
    say("R=%d: P(0,0) %.4f Bx(+-1) %.4f %.4f By(+-1) %.4f %.4f eta %s" % (
        R, got["quarter"][0, 0], got["bx"][R - 1] if R else 0, got["bx"][R + 1], got["by"][R - 1], got["by"][R + 1],
        np.round(got["eta"], 4)))


def test_empty_counters_give_zero_tables():
    n = 15
    counts = (torch.zeros(n * n, dtype=torch.int32, device=DEV), torch.zeros((9, n * n), dtype=torch.int32, device=DEV),
              torch.zeros((n * n, 25), dtype=torch.int32, device=DEV))
    t = me.mvp_tables(counts, 7)
    assert all(np.all(v == 0) for v in t.values())
