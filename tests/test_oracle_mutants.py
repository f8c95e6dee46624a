"""The pins must catch plausible mistakes.  Each case plants one mistake in a
copy of the oracle's C source (on the CPU, in a temporary directory), builds
it, and checks that at least one pin fails for it while the real oracle passes
the same pin."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from conftest import load_golden
from test_oracle_bruteforce import _frames, brute_fs
from test_oracle_rules import PINS as RULE_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "me_oracle.c")

MUTANTS = {
    # Pattern geometry: the cross's vertical arms at distance 2 instead of 1.
    "hcsp_shape": ("{0, -1}, {0, 1}};\n/* The transposed", "{0, -2}, {0, 2}};\n/* The transposed"),
    # Switching strategy one inverted.
    "strategy_one": ("(b.dy == c.dy) ? PAT_H : PAT_V", "(b.dy == c.dy) ? PAT_V : PAT_H"),
    # Switching strategy two inverted (switch on distant points).
    "strategy_two": ("abs(b.dy - c.dy) == 1)", "abs(b.dy - c.dy) == 2)"),
    # Step 4 skipped.
    "no_step4": ("b = pattern_bmp(st, c, list, 3, &d);", "b = pattern_bmp(st, c, list, 1, &d);"),
    # Ties leave the centre.
    "ties_leave_centre": ("if (!have || d < best_d) {", "if (!have || d <= best_d) {"),
    # Revisited points counted again.
    "count_revisits": ("        st->nsp += 1;\n    }", "    }\n    st->nsp += 1;"),
    # HDSP distant points at distance 3.
    "hdsp_shape": ("HDSP[5] = {{0, 0}, {-2, 0}, {2, 0}", "HDSP[5] = {{0, 0}, {-3, 0}, {3, 0}"),
    # FS tie order: left-most before top-most.
    "fs_tie_order": ("(dy < by || (dy == by && dx < bx))", "(dx < bx || (dx == bx && dy < by))"),
    # SAD without the absolute value.
    "sad_no_abs": ("s += abs((int)c[u] - (int)r[u]);", "s += ((int)c[u] - (int)r[u]) & 0xff;"),
    # Frame edge: the last valid column dropped.
    "frame_edge": ("x <= f->W - f->B", "x < f->W - f->B"),
    # Reference rows taken from the current frame's row (dy ignored in SAD).
    "sad_row": ("(size_t)(f->y0 + dy + v) * f->pitch", "(size_t)(f->y0 + v) * f->pitch"),
    # DCDS^S: the middle point on the side of the larger distant point.
    "dcds_s_side_flip": ("list[1] = (sp < sn) ? mid[1] : mid[0];", "list[1] = (sp < sn) ? mid[0] : mid[1];"),
    # DCDS^S: with one distant point outside V, only the valid partner's side.
    "dcds_s_edge_one_side": ("        if (vn && vp) {\n            list[1] = (sp < sn) ? mid[1] : mid[0];",
                             "        if (vn || vp) {\n            list[1] = (vn && vp ? sp < sn : vp) ? mid[1] : mid[0];"),
    # Learned start: the proposer's orientation ignored (always HCSP).
    "seeded_vcsp_ignored": ("first_vertical ? VCSP : HCSP", "HCSP"),
    # Learned start: the second search only when the start beats plain DCDS's result.
    "seeded_gate_plain": ("|| ds >= st->bdm[widx(st, 0, 0)])", "|| ds >= dp)"),
    # Learned start: the second search's result always kept (no fallback to plain DCDS).
    "seeded_no_fallback": ("if (dq < dp) {", "if (1) {"),
    # Learned start: a tie between the two searches goes to the seeded one.
    "seeded_tie_to_start": ("if (dq < dp) {", "if (dq <= dp) {"),
}


def _table7_ok():
    table = load_golden("table7_dcds_nsp.txt", int)
    R = 7
    ys, xs = np.mgrid[-R:R + 1, -R:R + 1]
    for sy in (1, -1):
        for sx in (1, -1):
            for y in range(8):
                for x in range(8):
                    t = (sx * x, sy * y)
                    mv, d, nsp = oracle.dcds_surface((xs - t[0]) ** 2 + (ys - t[1]) ** 2)
                    if mv != t or nsp != table[y, x]:
                        return False
    return True


def _brute_ok():
    for kind in ("uniform", "lowentropy", "checker"):
        for (H, W, B, R) in [(32, 32, 8, 3), (32, 48, 16, 7)]:
            cur, ref = _frames(kind, H, W, seed=H + W + R)
            got = oracle.fullsearch(cur, ref, B, R)
            exp = brute_fs(cur, ref, B, R)
            if not all(np.array_equal(a, b) for a, b in zip(got, exp)):
                return False
            # DCDS's reported SAD must be the true SAD at its vector.
            mv, sad, _ = oracle.dcds(cur, ref, B, R)
            c32, r32 = cur.astype(np.int32), ref.astype(np.int32)
            for j in range(H // B):
                for i in range(W // B):
                    dx, dy = int(mv[j, i, 0]), int(mv[j, i, 1])
                    y, x = j * B + dy, i * B + dx
                    if not (0 <= x <= W - B and 0 <= y <= H - B):
                        return False
                    s = np.abs(c32[j * B:j * B + B, i * B:i * B + B] - r32[y:y + B, x:x + B]).sum()
                    if s != sad[j, i]:
                        return False
    return True


def _rules_ok():
    for pin in RULE_PINS:
        try:
            pin()
        except AssertionError:
            return False
    return True


def _all_pins_ok():
    return _table7_ok() and _brute_ok() and _rules_ok()


def test_real_oracle_passes_pins():
    assert _all_pins_ok()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not unique: %s" % name
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", *oracle.CC_FLAGS, "-o", str(so), str(path)])
    saved = oracle._lib
    try:
        oracle._lib = oracle.load_library(str(so))
        assert not _all_pins_ok(), "mutant %s passed every pin" % name
    finally:
        oracle._lib = saved
