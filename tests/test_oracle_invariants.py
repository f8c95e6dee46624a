"""Properties the DCDS oracle must have on real SAD (§III-B), independent of
the printed tables: it never beats FS, it returns the best point it evaluated,
the half-way stop is exactly the zero vector, its frame path agrees with its
cost-surface path (pinned by Table VII), mirror symmetry on tie-free costs, and
the relations of the simplified and seeded variants to plain DCDS."""
import numpy as np
import pytest

import oracle
from synth import blurred_noise, make_config, qcif_pair

HCSP_PTS = [(0, 0), (-1, 0), (1, 0), (-2, 0), (2, 0), (0, -1), (0, 1)]


def _surface(cur, ref, B, R, i, j):
    """Brute-force cost surface of one block and its validity mask."""
    H, W = cur.shape
    n = 2 * R + 1
    cost = np.zeros((n, n), np.int64)
    valid = np.zeros((n, n), np.uint8)
    c32, r32 = cur.astype(np.int32), ref.astype(np.int32)
    blk = c32[j * B:j * B + B, i * B:i * B + B]
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            x, y = i * B + dx, j * B + dy
            if 0 <= x <= W - B and 0 <= y <= H - B:
                valid[dy + R, dx + R] = 1
                cost[dy + R, dx + R] = np.abs(blk - r32[y:y + B, x:x + B]).sum()
    return cost, valid


def _pairs():
    cur, ref, _ = qcif_pair(1)
    yield "qcif", cur, ref, 16, 7
    seq = make_config(2, frames=3)
    yield "cif", seq[1], seq[0], 16, 7
    rng = np.random.default_rng(3)
    a = blurred_noise(rng, 64, 96, 1.5).astype(np.uint8)
    b = np.roll(a, (2, -3), axis=(0, 1))
    yield "rolled8", a, b, 8, 5


@pytest.mark.parametrize("name,cur,ref,B,R", list(_pairs()), ids=lambda v: v if isinstance(v, str) else "")
def test_dcds_invariants_on_frames(name, cur, ref, B, R):
    fmv, fsad, fnsp = oracle.fullsearch(cur, ref, B, R)
    mv, sad, nsp = oracle.dcds(cur, ref, B, R)
    H, W = cur.shape
    assert (sad >= fsad).all()
    assert (nsp <= fnsp).all()
    for j in range(H // B):
        for i in range(W // B):
            cost, valid = _surface(cur, ref, B, R, i, j)
            # FS visits every valid point.
            assert fnsp[j, i] == valid.sum()
            # The frame path equals the surface path on the block's own surface.
            smv, sd, sn, S = oracle.dcds_surface(cost, valid, want_set=True)
            assert smv == tuple(mv[j, i]) and sd == sad[j, i] and sn == nsp[j, i]
            # S only holds valid points; the result is the minimum over S.
            assert not (S & (valid == 0)).any()
            assert S.sum() == nsp[j, i]
            assert sad[j, i] == cost[S].min()
            # Half-way stop <=> zero vector <=> NSP equals the valid cross points.
            n_cross = sum(valid[dy + R, dx + R] for dx, dy in HCSP_PTS)
            zero = tuple(mv[j, i]) == (0, 0)
            assert zero == (nsp[j, i] == n_cross and S.sum() == n_cross)


def test_mirror_symmetry_on_tie_free_costs():
    """With all-distinct costs the scan order never matters, and the patterns are
    symmetric under x- and y-mirroring, so DCDS commutes with both mirrors."""
    rng = np.random.default_rng(11)
    for R in (3, 7, 15):
        n = 2 * R + 1
        for _ in range(200):
            cost = rng.permutation(n * n).reshape(n, n).astype(np.int64)
            mv, d, nsp = oracle.dcds_surface(cost)
            mx = oracle.dcds_surface(cost[:, ::-1])
            my = oracle.dcds_surface(cost[::-1, :])
            assert mx[0] == (-mv[0], mv[1]) and mx[1:] == (d, nsp)
            assert my[0] == (mv[0], -mv[1]) and my[1:] == (d, nsp)


def test_simplified_dcds_relations():
    """DCDS^S (§IV-C) follows DCDS up to Step 4 and checks a subset of its final
    candidates: never more points, never a smaller SAD."""
    rng = np.random.default_rng(12)
    for R in (2, 7, 15):
        n = 2 * R + 1
        for _ in range(300):
            cost = rng.integers(0, 50, (n, n)).astype(np.int64)
            a = oracle.dcds_surface(cost, want_trace=True)
            b = oracle.dcds_surface(cost, variant=oracle.VARIANT_DCDS_S, want_trace=True)
            assert a[3][:-1] == b[3][:-1]
            assert b[2] <= a[2] and b[1] >= a[1]
    cur, ref, _ = qcif_pair(2)
    mv, sad, nsp = oracle.dcds(cur, ref, 16, 7)
    ms, ss, ns = oracle.dcds(cur, ref, 16, 7, variant=oracle.VARIANT_DCDS_S)
    assert (ns <= nsp).all() and (ss >= sad).all()


def test_seeded_start_relations():
    """Learned start (not in the paper): a zero start is plain DCDS; a start that
    does not beat the origin leaves plain DCDS's result (plus its probe point);
    otherwise the result is never worse than plain DCDS's."""
    seq = make_config(2, frames=2)
    cur, ref = seq[1], seq[0]
    B, R = 16, 7
    mv, sad, nsp = oracle.dcds(cur, ref, B, R)
    hb, wb = cur.shape[0] // B, cur.shape[1] // B
    zero = np.zeros((hb, wb, 2), np.int16)
    m0, s0, n0 = oracle.dcds(cur, ref, B, R, start=zero)
    np.testing.assert_array_equal(m0, mv)
    np.testing.assert_array_equal(s0, sad)
    np.testing.assert_array_equal(n0, nsp)
    rng = np.random.default_rng(4)
    start = rng.integers(-R, R + 1, (hb, wb, 2)).astype(np.int16)
    orient = rng.integers(0, 2, (hb, wb)).astype(np.uint8)
    m1, s1, n1 = oracle.dcds(cur, ref, B, R, start=start, orient=orient)
    fmv, fsad, _ = oracle.fullsearch(cur, ref, B, R)
    assert (s1 >= fsad).all()
    for j in range(hb):
        for i in range(wb):
            cost, valid = _surface(cur, ref, B, R, i, j)
            # Clamp the start into V as the oracle does.
            xs = np.nonzero(valid.any(axis=0))[0] - R
            ys = np.nonzero(valid.any(axis=1))[0] - R
            s = (int(np.clip(start[j, i, 0], xs.min(), xs.max())), int(np.clip(start[j, i, 1], ys.min(), ys.max())))
            ds = cost[s[1] + R, s[0] + R]
            if s == (0, 0) or ds >= cost[R, R]:
                _, _, _, S = oracle.dcds_surface(cost, valid, want_set=True)
                assert tuple(m1[j, i]) == tuple(mv[j, i]) and s1[j, i] == sad[j, i]
                assert n1[j, i] == nsp[j, i] + (0 if S[s[1] + R, s[0] + R] else 1)
            else:
                assert s1[j, i] <= min(ds, sad[j, i]) and n1[j, i] >= nsp[j, i]
            # The surface entry clamps nothing: give it the clamped start.
            r = oracle.dcds_surface(cost, valid, start=s, orient_v=bool(orient[j, i]))
            assert r[0] == tuple(m1[j, i]) and r[1] == s1[j, i] and r[2] == n1[j, i]


def test_dcds_translation_inside_cross_recovered_exactly():
    """A pure global translation by a point of the first cross: DCDS stops on it
    (Step 1 then the diamonds see zero SAD there) on every interior block."""
    rng = np.random.Generator(np.random.PCG64(6))
    big = blurred_noise(rng, 96 + 32, 128 + 32, 1.5).astype(np.uint8)
    for sx, sy in HCSP_PTS:
        ref = big[16:16 + 96, 16:16 + 128]
        cur = big[16 + sy:16 + sy + 96, 16 + sx:16 + sx + 128]
        mv, sad, nsp = oracle.dcds(cur, ref, 16, 7)
        for j in range(6):
            for i in range(8):
                x, y = i * 16 + sx, j * 16 + sy
                if 0 <= x <= 128 - 16 and 0 <= y <= 96 - 16:
                    assert tuple(mv[j, i]) == (sx, sy) and sad[j, i] == 0
