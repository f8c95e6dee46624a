"""The C ABI (include/me.h): the library loads without a GPU, exports every
declared symbol, and rejects bad arguments on the host before any launch
(these calls return before touching the device, so they run on the CPU)."""
import os
import re

import pytest

import paper_0806_0689_amd as me
from conftest import ROOT


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(me_[a-z_0-9]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported():
    L = me.lib()
    declared = _declared()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(me.EXPORTS)


def test_status_strings():
    for s in (me.ME_OK, me.ME_EINVAL, me.ME_EUNSUPPORTED, me.ME_ENOMEM, me.ME_EDEVICE):
        assert me.status_string(s)
    assert me.status_string(12345) == "unknown status"


# A fake but 4-aligned "device" address: only reached by calls that must fail
# their host-side checks (or do nothing), never dereferenced.
P = 0x1000


def _frame_call(fn, **kw):
    a = dict(cur=P, ref=P, width=64, height=32, pitch=64, pair_stride=64 * 32, n_pairs=1, block=16, range_=7,
             mv=P, sad=P, nsp=P)
    a.update(kw)
    return fn(a["cur"], a["ref"], a["width"], a["height"], a["pitch"], a["pair_stride"], a["n_pairs"], a["block"],
              a["range_"], a["mv"], a["sad"], a["nsp"], 0)


def _search_fs(*a):
    return me.me_search(*a[:9], me.ME_ALGO_FS, None, None, *a[9:12], None, a[12])


def _search_dcds_sse(*a):
    return me.me_search(*a[:9], me.ME_ALGO_DCDS_S, None, None, *a[9:12], P, a[12])


@pytest.mark.parametrize("fn", [me.me_fullsearch, me.me_dcds, _search_fs, _search_dcds_sse])
@pytest.mark.parametrize("kw,status", [
    (dict(cur=None), me.ME_EINVAL),
    (dict(ref=None), me.ME_EINVAL),
    (dict(mv=None), me.ME_EINVAL),
    (dict(sad=None), me.ME_EINVAL),
    (dict(nsp=None), me.ME_EINVAL),
    (dict(width=0), me.ME_EINVAL),
    (dict(height=-16), me.ME_EINVAL),
    (dict(n_pairs=-1), me.ME_EINVAL),
    (dict(width=72), me.ME_EINVAL),           # not a multiple of the block
    (dict(height=40), me.ME_EINVAL),
    (dict(pitch=60), me.ME_EINVAL),           # pitch < width
    (dict(pitch=66), me.ME_EINVAL),           # pitch not a multiple of 4
    (dict(cur=P + 2), me.ME_EINVAL),          # misaligned frame
    (dict(ref=P + 1), me.ME_EINVAL),
    (dict(pair_stride=6), me.ME_EINVAL),
    (dict(block=12), me.ME_EUNSUPPORTED),
    (dict(block=32), me.ME_EUNSUPPORTED),
    (dict(range_=0), me.ME_EUNSUPPORTED),
    (dict(range_=32), me.ME_EUNSUPPORTED),
    (dict(n_pairs=0), me.ME_OK),              # empty input: nothing to do
    (dict(n_pairs=0, cur=None, mv=None), me.ME_OK),
    (dict(n_pairs=0, block=12), me.ME_EUNSUPPORTED),
    (dict(height=65536, pitch=32768, n_pairs=0), me.ME_EUNSUPPORTED),  # one frame of 2 GiB
    (dict(height=32768, pitch=65532, n_pairs=0), me.ME_OK),             # just below 2^31 bytes
])
def test_frame_argument_checks(fn, kw, status):
    assert _frame_call(fn, **kw) == status


def test_dcds_ex_checks():
    base = (P, P, 64, 32, 64, 2048, 1, 16, 7)
    assert me.me_dcds_ex(*base, 7, None, None, P, P, P, 0) == me.ME_EUNSUPPORTED  # unknown algo
    assert me.me_dcds_ex(*base, me.ME_ALGO_FS, None, None, P, P, P, 0) == me.ME_EUNSUPPORTED
    assert me.me_dcds_ex(*base, me.ME_ALGO_DCDS, None, P, P, P, P, 0) == me.ME_EINVAL  # orient without start
    assert me.me_dcds_ex(P, P, 64, 32, 64, 2048, 0, 16, 7, me.ME_ALGO_DCDS_S, P, P, P, P, P, 0) == me.ME_OK


def test_search_checks():
    base = (P, P, 64, 32, 64, 2048, 1, 16, 7)
    assert me.me_search(*base, 7, None, None, P, P, P, None, 0) == me.ME_EUNSUPPORTED  # unknown algo
    assert me.me_search(*base, me.ME_ALGO_FS, P, None, P, P, P, None, 0) == me.ME_EINVAL  # FS has no start
    assert me.me_search(*base, me.ME_ALGO_DCDS, None, P, P, P, P, P, 0) == me.ME_EINVAL  # orient without start
    assert me.me_search(P, P, 64, 32, 64, 2048, 0, 16, 7, me.ME_ALGO_FS, None, None, P, P, P, P, 0) == me.ME_OK


def test_frame_quality_checks():
    q = me.me_frame_quality
    assert q(P, P, P, None, 64, 32, 1, 16, P + 4, 0) == me.ME_EINVAL      # misaligned record array
    assert q(None, P, P, None, 64, 32, 1, 16, P, 0) == me.ME_EINVAL
    assert q(P, P, None, None, 64, 32, 1, 16, P, 0) == me.ME_EINVAL
    assert q(P, P, P, None, 64, 32, 1, 16, None, 0) == me.ME_EINVAL
    assert q(P, P, P, None, 0, 32, 1, 16, P, 0) == me.ME_EINVAL
    assert q(P, P, P, None, 72, 32, 1, 16, P, 0) == me.ME_EINVAL          # not a multiple of the block
    assert q(P, P, P, None, 64, 32, -1, 16, P, 0) == me.ME_EINVAL
    assert q(P, P, P, None, 64, 32, 1, 12, P, 0) == me.ME_EUNSUPPORTED
    assert q(None, None, None, None, 64, 32, 0, 16, None, 0) == me.ME_OK  # nothing to do


def test_mvp_checks():
    base = (P, P, 64, 32, 64, 2048, 1, 16, 7)
    assert me.me_mvp_stats(*base, None, P, P, 0) == me.ME_EINVAL
    assert me.me_mvp_stats(*base, P, P, P + 2, 0) == me.ME_EINVAL          # misaligned counter
    assert me.me_mvp_stats(P, P, 64, 32, 64, 2048, 1, 16, 32, P, P, P, 0) == me.ME_EUNSUPPORTED
    assert me.me_mvp_stats(P, P, 64, 32, 64, 2048, 0, 16, 7, None, None, None, 0) == me.ME_OK
    assert me.me_mvp_tables_size(0) == me.ME_EUNSUPPORTED and me.me_mvp_tables_size(32) == me.ME_EUNSUPPORTED
    n = 15
    assert me.me_mvp_tables_size(7) == 8 * 8 + 4 * n + 10 + 9 * n * n + 25 * n * n + 50
    assert me.me_mvp_tables(P, P, P, 7, P + 4, 0) == me.ME_EINVAL          # misaligned output
    assert me.me_mvp_tables(None, P, P, 7, P, 0) == me.ME_EINVAL
    assert me.me_mvp_tables(P, P, P, 0, P, 0) == me.ME_EUNSUPPORTED


def test_surface_checks():
    assert me.me_dcds_surface(None, None, 1, 7, 1, None, None, P, P, P, 0) == me.ME_EINVAL
    assert me.me_dcds_surface(P, None, -1, 7, 1, None, None, P, P, P, 0) == me.ME_EINVAL
    assert me.me_dcds_surface(P, None, 1, 0, 1, None, None, P, P, P, 0) == me.ME_EUNSUPPORTED
    assert me.me_dcds_surface(P, None, 1, 7, 0, None, None, P, P, P, 0) == me.ME_EUNSUPPORTED
    assert me.me_dcds_surface(P, None, 1, 7, 1, None, P, P, P, P, 0) == me.ME_EINVAL
    assert me.me_dcds_surface(P, None, 0, 7, 1, None, None, P, P, P, 0) == me.ME_OK


def test_product_path_does_not_import_the_oracle():
    """The HIP package and the oracle share no code and neither imports the other."""
    pkg = os.path.join(ROOT, "paper_0806_0689_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), fn
                assert "me_oracle" not in text, fn
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".py", ".c", ".h")):
            text = open(os.path.join(ROOT, "oracle", fn)).read()
            assert not re.search(r"^\s*(import|from)\s+paper_0806_0689_amd\b", text, re.M), fn
            assert '#include "me' not in text and "csrc" not in text, fn


def test_config_set_get_and_checks():
    d16 = me.me_get_config(16, 15)
    assert d16[2] == 4                              # default tiles per grab
    assert me.me_set_config(16, 15, (4, 2)) == me.ME_OK
    assert me.me_get_config(16, 15) == (4, 2, 4)
    assert me.me_get_config(16, 9) == (4, 2, 4)    # same range class 8..15
    assert me.me_set_config(16, 15, (4, 2, 16)) == me.ME_OK
    assert me.me_get_config(16, 15) == (4, 2, 16)
    assert me.me_set_config(16, 15, (4, 2, 3)) == me.ME_EUNSUPPORTED  # grabs: 1, 2, 4, 8, 16
    assert me.me_set_config(16, 15, (4, 2, 32)) == me.ME_EUNSUPPORTED
    assert me.me_get_config(16, 15) == (4, 2, 16)
    assert me.me_get_config(16, 7) == me.me_get_config(16, 1)
    assert me.me_set_config(16, 15, None) == me.ME_OK
    assert me.me_get_config(16, 15) == d16
    assert me.me_set_config(8, 15, (4, 2)) == me.ME_EUNSUPPORTED   # 8x8 blocks: 1 or 2 rows per lane
    assert me.me_set_config(16, 15, (3, 2)) == me.ME_EUNSUPPORTED
    assert me.me_set_config(16, 15, (2, 16)) == me.ME_EUNSUPPORTED
    assert me.me_set_config(16, 15, (2, 8)) == me.ME_OK
    assert me.me_set_config(12, 15, (2, 2)) == me.ME_EUNSUPPORTED
    assert me.me_set_config(16, 0, (2, 2)) == me.ME_EUNSUPPORTED
    assert me.lib().me_get_config(16, 15, None) == me.ME_EINVAL


def test_batch_argument_checks():
    J = me.MeJob
    good = J(P, P, 64, 32, 64, 1, 64 * 32, P, P, P, None, None)
    arr = (J * 2)(good, good)
    assert me.me_batch(None, -1, me.ME_ALGO_DCDS, 16, 7) == me.ME_EINVAL
    assert me.me_batch(None, me.MAX_JOBS + 1, me.ME_ALGO_DCDS, 16, 7) == me.ME_EINVAL
    assert me.me_batch(None, 1, me.ME_ALGO_DCDS, 16, 7) == me.ME_EINVAL
    assert me.me_batch(None, 0, me.ME_ALGO_DCDS, 16, 7) == me.ME_OK     # empty batch
    assert me.me_batch(arr, 2, 9, 16, 7) == me.ME_EUNSUPPORTED
    assert me.me_batch(arr, 2, me.ME_ALGO_DCDS, 12, 7) == me.ME_EUNSUPPORTED
    assert me.me_batch(arr, 2, me.ME_ALGO_DCDS, 16, 40) == me.ME_EUNSUPPORTED
    bad = (J * 2)(good, J(P, P, 60, 32, 64, 1, 64 * 32, P, P, P, None, None))   # width not a multiple of 16
    assert me.me_batch(bad, 2, me.ME_ALGO_DCDS, 16, 7) == me.ME_EINVAL
    bad = (J * 1)(J(P, P, 64, 32, 64, 1, 64 * 32, P, P, P, None, P))           # orient without start
    assert me.me_batch(bad, 1, me.ME_ALGO_DCDS, 16, 7) == me.ME_EINVAL
    bad = (J * 1)(J(P, P, 64, 32, 64, 1, 64 * 32, P, P, P, P, None))           # start with FS
    assert me.me_batch(bad, 1, me.ME_ALGO_FS, 16, 7) == me.ME_EINVAL
    empty = (J * 1)(J(None, None, 64, 32, 64, 0, 0, None, None, None, None, None))  # zero pairs
    assert me.me_batch(empty, 1, me.ME_ALGO_DCDS, 16, 7) == me.ME_OK
    # More than 2^30 work tiles in one call (FS: one tile per block), rejected
    # before any device work: 1024 blocks per pair, 2^20 + 1 pairs.
    huge = (J * 1)(J(P, P, 16384, 16, 16384, (1 << 20) + 1, 16 * 16384, P, P, P, None, None))
    assert me.me_batch(huge, 1, me.ME_ALGO_FS, 16, 7) == me.ME_EUNSUPPORTED


def test_autotune_argument_checks(tmp_path):
    J = me.MeJob
    arr = (J * 1)(J(P, P, 64, 32, 64, 1, 64 * 32, P, P, P, None, None))
    assert me.me_autotune(arr, 1, me.ME_ALGO_FS, 16, 7, 3)[0] == me.ME_EUNSUPPORTED
    assert me.me_autotune(arr, 1, me.ME_ALGO_DCDS, 12, 7, 3)[0] == me.ME_EUNSUPPORTED
    assert me.me_autotune(arr, 1, me.ME_ALGO_DCDS, 16, 0, 3)[0] == me.ME_EUNSUPPORTED
    assert me.me_autotune(arr, 1, me.ME_ALGO_DCDS, 16, 7, 0)[0] == me.ME_EINVAL
    assert me.me_autotune(None, 0, me.ME_ALGO_DCDS, 16, 7, 3)[0] == me.ME_EINVAL
    # Cache file: missing -> EINVAL (defaults stay); malformed lines are counted and skipped.
    assert me.me_autotune_load(str(tmp_path / "missing.txt"))[0] == me.ME_EINVAL
    f = tmp_path / "cache.txt"
    # Lines of 7 fields (without tiles_per_grab) and of 8 fields are read.
    f.write_text("# header\nnot a line\ngfx950 70000000 16 1 3 4 0.1\ngfx950 70000000 16 9 2 4 0.1\n"
                 "otherarch 1 16 1 2 4 0.5\n"
                 "gfx950 70000000 16 1 2 4 3 0.1\ngfx950 70000000 16 1 2 4 8 0.1 extra\n"
                 "otherarch 1 16 1 2 4 8 0.5\n")
    rc, applied, rejected = me.me_autotune_load(str(f))
    assert rc == me.ME_OK and rejected == 5 and applied == 0
    assert me.me_autotune_save(str(tmp_path / "out.txt")) == me.ME_OK
    assert (tmp_path / "out.txt").read_text().startswith("# me autotune cache v2")


def test_proposer_host_checks():
    from oracle import cnn
    assert me.lib().me_proposer_num_params() == cnn.num_params()
    assert me.lib().me_proposer_create(None) == me.ME_EINVAL
    assert me.lib().me_proposer_destroy(None) == me.ME_OK
    assert me.lib().me_proposer_init(None, 1) == me.ME_EINVAL
    assert me.lib().me_proposer_forward(None, P, P, 64, 32, 64, 2048, 1, P, None) == me.ME_EINVAL
    assert me.lib().me_proposer_backward(None, P, None) == me.ME_EINVAL
