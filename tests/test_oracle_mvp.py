"""Pins of the MVP-statistics oracle (oracle/mvp.py): its tables rebuilt from
the paper's own Tables II and III and Fig. 3 (Table VI's efficiencies
included), the structural zeros of the conditional distributions, and a
brute-force window search on tiny frames."""
import numpy as np
import pytest

from conftest import load_golden
from oracle import mvp
from synth import make_config

R = 7
N_ = 2 * R + 1


def paper_histogram():
    """Counts (per 10^4 blocks) with the paper's axis distributions Bx, By
    (Table III) on the axes and Table II's off-axis quarter in one quadrant."""
    t2 = load_golden("table2_mvp_quarter.txt")
    t3 = load_golden("table3_mvp_1d.txt")
    h = np.zeros((N_, N_), np.int64)  # [y + R, x + R]
    for d in range(-R, R + 1):
        h[R, d + R] = round(t3[2, d + R] * 1e4)
        if d:
            h[d + R, R] = round(t3[3, d + R] * 1e4)
    for qy in range(1, R + 1):
        for qx in range(1, R + 1):
            h[qy + R, qx + R] = round(t2[qy, qx] * 1e4)
    return h


def empty_conditionals():
    return np.zeros((9, N_ * N_), np.int64), np.zeros((N_ * N_, 25), np.int64)


def test_tables_reproduce_tables_ii_and_iii():
    h = paper_histogram()
    t = mvp.tables(h.ravel(), *empty_conditionals(), R)
    t2 = load_golden("table2_mvp_quarter.txt")
    t3 = load_golden("table3_mvp_1d.txt")
    scale = h.sum() / 1e4  # the printed fractions sum to 1 only up to rounding
    np.testing.assert_allclose(t["quarter"] * scale, t2, atol=1.5e-4)
    np.testing.assert_allclose(t["bx"] * scale, t3[2], atol=1e-9)
    np.testing.assert_allclose(t["by"] * scale, t3[3], atol=1e-9)
    # Folded marginals: A(d) + A(-d) equals the column (row) sums of Table II.
    for d in range(1, R + 1):
        assert (t["ax"][R + d] + t["ax"][R - d]) * scale == pytest.approx(t3[0, R + d] + t3[0, R - d], abs=1.2e-3)
        assert (t["ay"][R + d] + t["ay"][R - d]) * scale == pytest.approx(t3[1, R + d] + t3[1, R - d], abs=1.2e-3)
    assert t["ax"].sum() == pytest.approx(1.0) and t["ay"].sum() == pytest.approx(1.0)


def test_regions_and_first_step_efficiency_from_fig3():
    """Fig. 3's cells (the 5x5 centre, fractions of 10^4 blocks; the rest of
    the mass elsewhere) give the printed P values and Table VI's eta_1."""
    fig3 = load_golden("fig3_regional.txt")
    h = np.zeros((N_, N_), np.int64)
    h[R - 2:R + 3, R - 2:R + 3] = np.rint(fig3 * 1e4).astype(np.int64)
    h[R + 7, R + 7] = 10000 - h.sum()
    t = mvp.tables(h.ravel(), *empty_conditionals(), R)
    printed = [0.8745, 0.8557, 0.8315, 0.7899, 0.8248]
    np.testing.assert_allclose(t["regions"], printed, atol=13 * 5e-5)
    # Table VI: P_1 / n_1 for BBGDS, DS, CDS, HEXBS, HCSP.
    np.testing.assert_allclose(t["eta"], [0.0878, 0.6705 / 9, 0.0924, 0.0922, 0.1178], atol=6e-5)
    assert t["eta"][4] == max(t["eta"])  # HCSP has the highest efficiency


@pytest.fixture(scope="module")
def cif_counts():
    seq = make_config(2, seed=8, frames=3)
    acc = None
    for p in range(2):
        acc = mvp.counts(seq[p + 1], seq[p], 16, R, acc)
    return acc


def test_counter_totals(cif_counts):
    hist, d1, d2 = cif_counts
    blocks = 2 * 18 * 22
    assert hist.sum() == d1.sum() == d2.sum() == blocks
    np.testing.assert_array_equal(d1.sum(axis=0), hist)
    np.testing.assert_array_equal(d2.sum(axis=1), hist)


def test_structural_zeros(cif_counts):
    """A full-search vector on the cross (in the square) is itself the best
    point there: D1 vanishes at the other cross points, D2 is a unit row."""
    hist, d1, d2 = cif_counts
    for p, s in enumerate(mvp.CROSS):
        v = (s[1] + R) * N_ + (s[0] + R)
        for q in range(9):
            if q != p:
                assert d1[q, v] == 0
    for qi, (x, y) in enumerate(mvp.SQUARE):
        v = (y + R) * N_ + (x + R)
        assert d2[v].sum() == d2[v, qi]
    t = mvp.tables(hist, d1, d2, R)
    rows = t["d1"].reshape(9, -1).sum(axis=1)
    assert np.all((np.abs(rows - 1) < 1e-12) | (rows == 0))


def test_brute_force_tiny():
    rng = np.random.default_rng(4)
    H, W, B, r = 32, 40, 8, 3
    base = rng.integers(0, 256, (H + 8, W + 8)).astype(np.uint8)
    ref = base[4:4 + H, 4:4 + W].copy()
    cur = base[3:3 + H, 5:5 + W].copy()  # global motion (+1, -1) inside the window
    hist, d1, d2 = mvp.counts(cur, ref, B, r)
    n = 2 * r + 1
    exp_h = np.zeros(n * n, np.int64)
    exp_1 = np.zeros((9, n * n), np.int64)
    exp_2 = np.zeros((n * n, 25), np.int64)
    for by in range(H // B):
        for bx in range(W // B):
            keys = {}
            for y in range(-r, r + 1):
                for x in range(-r, r + 1):
                    if 0 <= bx * B + x <= W - B and 0 <= by * B + y <= H - B:
                        s = 0
                        for v in range(B):
                            for u in range(B):
                                s += abs(int(cur[by * B + v, bx * B + u]) - int(ref[by * B + v + y, bx * B + u + x]))
                        keys[(x, y)] = (s, abs(x) + abs(y), y, x)
            best = min(keys, key=keys.get)
            vi = (best[1] + r) * n + best[0] + r
            exp_h[vi] += 1
            p = min((keys[c], i) for i, c in enumerate(mvp.CROSS) if c in keys)[1]
            q = min((keys[c], i) for i, c in enumerate(mvp.SQUARE) if c in keys)[1]
            exp_1[p, vi] += 1
            exp_2[vi, q] += 1
    np.testing.assert_array_equal(hist, exp_h)
    np.testing.assert_array_equal(d1, exp_1)
    np.testing.assert_array_equal(d2, exp_2)
    assert hist[(-1 + r) * n + (1 + r)] > 0  # the planted motion is found
