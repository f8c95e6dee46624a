"""What the trained proposer gains over DCDS without it, on every single-sequence
workload (configs 1, 2, 3, 5 and 6) and on held-out training-law sequences (never
seen in training).

Learned-start DCDS runs plain DCDS first and follows the proposed start only
when it beats that result, so on every block its SAD is at most plain DCDS's
(and at least FS's, the exhaustive reference): mean SAD is within 1% of plain
DCDS by construction, and is checked block by block here.  The gain is the SAD
the start finds beyond plain DCDS; on the long-motion 1088p and 4K content it
must be large.  The cost is reported: the points of both searches.  Uses the
committed checkpoint written by paper_0806_0689_amd/train.py."""
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
    # Block by block: FS <= learned <= plain.
    assert bool((ls >= fs).all()) and bool((ls <= ps).all())
    return {k: float(v.double().mean()) for k, v in
            (("fs", fs), ("plain", ps), ("learned", ls), ("plain_nsp", pn), ("learned_nsp", ln))}


# (name, frames, range, required SAD ratio learned / plain)
CASES = [
    ("config1_qcif_r7", lambda: make_config(1), 7, 1.01),
    ("config2_cif_r7", lambda: make_config(2, frames=12), 7, 1.01),
    ("config6_paperlike_r7", lambda: make_config(6, frames=12), 7, 1.01),
    ("config3_1088p_r15", lambda: make_config(3, frames=4), 15, 0.95),
    ("config5_4k_r31", lambda: make_config(5, frames=3), 31, 0.9),
    ("held_out_1088p_q0_r31", lambda: training_sequence(0, frames=8, held_out=True), 31, 0.9),
    ("held_out_1088p_q1_r31", lambda: training_sequence(1, frames=8, held_out=True), 31, 0.9),
    ("held_out_4k_r31", lambda: make_config(5, seed=20005, frames=3), 31, 0.9),
]


@pytest.mark.parametrize("name,make,R,ratio", CASES, ids=[c[0] for c in CASES])
def test_learned_start_against_plain(proposer, name, make, R, ratio):
    s = stats(make(), proposer, R)
    say("%s: sad fs %.1f plain %.1f learned %.1f (x%.3f); nsp plain %.2f learned %.2f" %
        (name, s["fs"], s["plain"], s["learned"], s["learned"] / s["plain"], s["plain_nsp"], s["learned_nsp"]))
    assert s["learned"] <= ratio * s["plain"]
    assert s["learned_nsp"] >= s["plain_nsp"]


def test_untrained_proposer_is_plain_dcds():
    """All-zero weights propose the origin on every block: the result is plain
    DCDS exactly, points included (the fallback path)."""
    p = me.Proposer()
    seq = make_config(1)
    t = torch.from_numpy(seq).to(DEV)
    got = me.dcds_learned(p, t[1:], t[:-1], 7)
    exp = me.dcds(t[1:], t[:-1], 16, 7)
    for a, b in zip(got, exp):
        assert torch.equal(a, b)


def test_checkpoint_loads_without_pickle():
    with np.load(train.DEFAULT_WEIGHTS, allow_pickle=False) as z:
        assert z["weights"].dtype == np.float32 and len(z["weights"]) == me.lib().me_proposer_num_params()
        assert np.isfinite(z["weights"]).all()
