"""The Python binding checks every caller tensor that a kernel indexes by
block (outputs, start vectors, orientations, counters) before any call:
device, dtype, contiguity and element count."""
import pytest

torch = pytest.importorskip("torch")
me = pytest.importorskip("paper_0806_0689_amd")


def test_accepts_a_matching_tensor():
    t = torch.zeros((2, 3, 4, 2), dtype=torch.int16)
    assert me._arg(t, 48, torch.int16, t.device, "mv") is t
    assert me._arg(None, 48, torch.int16, t.device, "start") is None


@pytest.mark.parametrize("make, why", [
    (lambda: torch.zeros(47, dtype=torch.int16), "too few elements"),
    (lambda: torch.zeros(49, dtype=torch.int16), "too many elements"),
    (lambda: torch.zeros(48, dtype=torch.int32), "wrong dtype"),
    (lambda: torch.zeros((2, 48), dtype=torch.int16)[:, ::2].T, "not contiguous"),
    (lambda: torch.zeros(48, dtype=torch.int16, device="meta"), "another device"),
])
def test_rejects(make, why):
    with pytest.raises(ValueError):
        me._arg(make(), 48, torch.int16, torch.device("cpu"), why)


def test_block_arguments_and_outputs():
    cpu = torch.device("cpu")
    P, hb, wb = 2, 3, 4
    start = torch.zeros((P, hb, wb, 2), dtype=torch.int16)
    orient = torch.zeros((P, hb, wb), dtype=torch.uint8)
    assert me._block_args(P, hb, wb, cpu, start, orient) == (start, orient)
    with pytest.raises(ValueError):
        me._block_args(P, hb, wb, cpu, start[:1], orient)
    with pytest.raises(ValueError):
        me._block_args(P, hb, wb, cpu, start, orient.to(torch.int16))
    mv = torch.zeros((P, hb, wb, 2), dtype=torch.int16)
    sad = torch.zeros((P, hb, wb), dtype=torch.int32)
    assert me._outputs(P, hb, wb, cpu, (mv, sad, sad.clone()))[0] is mv
    with pytest.raises(ValueError):
        me._outputs(P, hb, wb, cpu, (mv, sad[:1], sad))


def test_mvp_counters():
    cpu = torch.device("cpu")
    n = 2 * 7 + 1
    ok = (torch.zeros(n * n, dtype=torch.int32), torch.zeros((9, n * n), dtype=torch.int32),
          torch.zeros((n * n, 25), dtype=torch.int32))
    assert me._mvp_counts(ok, 7, cpu)[2] is ok[2]
    with pytest.raises(ValueError):
        me._mvp_counts(ok, 8, cpu)  # counters of another range
