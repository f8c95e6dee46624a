"""What the trained proposer gains over DCDS without it, on held-out seeds
(never seen in training): the learned start must keep mean SAD within 1% of
plain DCDS and is expected to save search points; every block stays no better
than FS (the exhaustive reference).  Uses the committed checkpoint written by
paper_0806_0689_amd/train.py."""
import os

import numpy as np
import pytest

from synth import make_config, training_sequence

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")
from paper_0806_0689_amd import train  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def proposer():
    assert os.path.exists(train.DEFAULT_WEIGHTS), "trained checkpoint missing"
    return train.load_proposer()


def stats(seq, p, R):
    t = torch.from_numpy(seq).to(DEV)
    cur, ref = t[1:], t[:-1]
    _, fs, _ = me.fullsearch(cur, ref, 16, R)
    _, ps, pn = me.dcds(cur, ref, 16, R)
    _, ls, ln = me.dcds_learned(p, cur, ref, R)
    assert bool((ls >= fs).all()) and bool((ps >= fs).all())
    return {k: float(v.double().mean()) for k, v in
            (("fs", fs), ("plain", ps), ("learned", ls), ("plain_nsp", pn), ("learned_nsp", ln))}


@pytest.mark.parametrize("q", [0, 1])
def test_gain_on_held_out_1080p(proposer, q):
    s = stats(training_sequence(q, frames=12, held_out=True), proposer, 31)
    say("held-out 1080p seq %d:" % q, s)
    assert s["learned"] <= 1.01 * s["plain"]
    assert s["learned_nsp"] < s["plain_nsp"]


def test_gain_on_4k_sample(proposer):
    seq = make_config(5, seed=20005, frames=4)
    s = stats(seq, proposer, 31)
    say("held-out 4K sample:", s)
    assert s["learned"] <= 1.01 * s["plain"]
    assert s["learned_nsp"] < s["plain_nsp"]


def test_checkpoint_loads_without_pickle():
    with np.load(train.DEFAULT_WEIGHTS, allow_pickle=False) as z:
        assert z["weights"].dtype == np.float32 and len(z["weights"]) == me.lib().me_proposer_num_params()
        assert np.isfinite(z["weights"]).all()
