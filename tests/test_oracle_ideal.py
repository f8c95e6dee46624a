"""Pins of the DCDS oracle against what the paper prints (§II-C, §III).

The ideal condition of §III-C: the true motion vector t has zero distortion and
every other point's distortion is its Euclidean distance to t.  Squared
distance has the same order and the same ties, and stays integer.
"""
import os

import numpy as np
import pytest

import oracle
from conftest import GOLDEN, load_golden

R = 7


def ideal_cost(tx, ty, r=R):
    ys, xs = np.mgrid[-r:r + 1, -r:r + 1]
    return (xs - tx) ** 2 + (ys - ty) ** 2


@pytest.mark.parametrize("sx,sy", [(1, 1), (-1, 1), (1, -1), (-1, -1)])
def test_table7_exact_all_quadrants(sx, sy):
    """Table VII (DCDS block): NSP at every true-MV position, and the MV found."""
    table = load_golden("table7_dcds_nsp.txt", int)
    for y in range(8):
        for x in range(8):
            t = (sx * x, sy * y)
            mv, d, nsp = oracle.dcds_surface(ideal_cost(*t))
            assert mv == t and d == 0, (t, mv)
            assert nsp == table[y, x], (t, nsp, table[y, x])


def test_half_way_stop_and_small_vectors():
    """§III-C 1): 7 points for a zero MV; 10 for (+-1, 0); 11 for (0, +-1)."""
    assert oracle.dcds_surface(ideal_cost(0, 0))[2] == 7
    for t in [(1, 0), (-1, 0)]:
        assert oracle.dcds_surface(ideal_cost(*t))[2] == 10
    for t in [(0, 1), (0, -1)]:
        assert oracle.dcds_surface(ideal_cost(*t))[2] == 11


def test_fig6_example_path():
    """Fig. 6 works an example with the MV at (1, 3); Table VII gives 17 points.

    The walk: HCSP (7) -> VDSP at (0,1) (+3) -> VDSP at (0,3) (+3, near point
    wins, switch) -> HDSP at (1,3) centre wins (+3) -> one new middle point.
    """
    mv, d, nsp, trace = oracle.dcds_surface(ideal_cost(1, 3), want_trace=True)
    assert mv == (1, 3) and nsp == 17
    assert trace == [7, 10, 13, 16, 17]


def _s_after_halt():
    # A surface whose minimum is the origin: DCDS stops after Step 1, so S is
    # exactly the first pattern.
    _, _, nsp, S = oracle.dcds_surface(ideal_cost(0, 0), want_set=True)
    pts = [(x - R, y - R) for y, x in zip(*np.nonzero(S))]
    return nsp, pts


def test_hcsp_shape_from_fig3_and_table6():
    """The first pattern, read back from the oracle, covers exactly P = 0.8248 of Fig. 3
    and so has eta_1 = 0.8248 / 7 = 0.1178 (Eq. 7, Table VI)."""
    fig3 = load_golden("fig3_regional.txt")
    nsp, pts = _s_after_halt()
    assert nsp == 7 and len(pts) == 7
    assert all(abs(x) <= 2 and abs(y) <= 2 for x, y in pts)
    p1 = sum(fig3[y + 2, x + 2] for x, y in pts)
    assert p1 == pytest.approx(0.8248, abs=5e-5)
    assert round(p1 / 7, 4) == 0.1178


def test_fig3_fixture_against_printed_regional_sums():
    """Regional sums printed beside Fig. 3 and in Table VI, recomputed from its cells
    (pins the transcription of the fixture; each cell is rounded to 1e-4)."""
    fig3 = load_golden("fig3_regional.txt")
    ys, xs = np.mgrid[-2:3, -2:3]
    regions = {
        "P_square5": np.ones_like(xs, bool),
        "P_diamond5": (abs(xs) + abs(ys)) <= 2,
        "P_cross5": (xs == 0) | (ys == 0),
        "P_square3": (abs(xs) <= 1) & (abs(ys) <= 1),
        "P_flatdiamond": (ys == 0) | ((xs == 0) & (abs(ys) <= 1)),
        "eta_DS": ((abs(xs) + abs(ys)) == 2) & ((xs == 0) | (ys == 0) | (abs(xs) == 1)) | ((xs == 0) & (ys == 0)),
        "eta_HEXBS": ((xs == 0) & (ys == 0)) | ((abs(xs) == 2) & (ys == 0)) | ((abs(xs) == 1) & (abs(ys) == 2)),
    }
    printed = {}
    with open(os.path.join(GOLDEN, "regional_sums.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, val, n = line.split()
            printed[name] = (float(val), int(n))
    for name, mask in regions.items():
        val, n = printed[name]
        assert int(mask.sum()) == n, name
        assert fig3[mask].sum() == pytest.approx(val, abs=n * 5e-5 + 1e-9), name
    # Table VI's remaining ratios.
    for name in ["eta_BBGDS", "eta_CDS", "eta_HCSP"]:
        val, n = printed[name]
        assert round(val / n, 4) == {"eta_BBGDS": 0.0878, "eta_CDS": 0.0924, "eta_HCSP": 0.1178}[name]


def test_ansp_distribution2():
    """Table VIII: DCDS ANSP on distribution 2 (Table II) is printed as 9.7."""
    t2 = load_golden("table2_mvp_quarter.txt")
    nsp = np.zeros((8, 8))
    for y in range(8):
        for x in range(8):
            nsp[y, x] = oracle.dcds_surface(ideal_cost(x, y))[2]
    ansp = float((t2 * nsp).sum() / t2.sum())
    assert ansp == pytest.approx(9.7, abs=0.05)


def _all_t():
    for ty in range(-R, R + 1):
        for tx in range(-R, R + 1):
            yield tx, ty


def test_eq8_upper_bound_and_three_new_points_per_step():
    """Eq. (8) counts 7 + 3n + {1, 2}; with distinct points it is an upper bound.
    §III-C 1): each intermediate step checks at most three new points."""
    for t in _all_t():
        mv, d, nsp, trace = oracle.dcds_surface(ideal_cost(*t), want_trace=True)
        assert trace[0] <= 7
        if mv == (0, 0):
            assert trace == [7] and nsp == 7
            continue
        n = len(trace) - 2  # diamonds evaluated (Step 2 + repeats of Step 3)
        assert n >= 1
        assert nsp <= 7 + 3 * n + 2
        assert -3 <= nsp - (7 + 3 * n) <= 2
        steps = np.diff(trace)
        assert all(0 <= s <= 3 for s in steps[:-1]), (t, trace)
        assert 0 <= steps[-1] <= 2
        assert trace[-1] == nsp


def test_ideal_finds_true_vector_everywhere():
    """The ideal surface is unimodal, so DCDS always reaches t (§III-C 2))."""
    for t in _all_t():
        mv, d, _ = oracle.dcds_surface(ideal_cost(*t))
        assert mv == t and d == 0
