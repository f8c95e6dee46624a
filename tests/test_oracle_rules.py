"""Pins for oracle rules that Table VII does not reach.

* DCDS^S (§IV-C): Step 4 checks only the middle point on the side of the
  smaller distant point.  Hand-built cost surfaces fix which middle point is
  evaluated, and the ideal condition of §III-C (the distortion grows with the
  distance to the true vector) fixes that DCDS^S must still end on the true
  vector at every position of the window, edges included.
* Learned start (this library's addition, not the paper's): the seeded first
  cross is HCSP or its transpose around the start; the search from the start
  runs when the start beats the origin, and the better of the two searches'
  results is kept, so the result is never worse than plain DCDS.

Each pin is a function that raises AssertionError; the mutant tests run them
against oracles with one planted mistake.
"""
import numpy as np

import oracle
from synth import make_config, qcif_pair

FILL = 1000  # filler distortion: every unnamed point is worse than any named one


def surface(R, pts, transpose=False):
    """Cost surface of side 2R+1: the named points {(dx, dy): cost}, every other
    point a distinct filler above FILL (no ties among fillers)."""
    n = 2 * R + 1
    cost = FILL + np.arange(n * n, dtype=np.int64).reshape(n, n)
    for (dx, dy), c in pts.items():
        if transpose:
            dx, dy = dy, dx
        cost[dy + R, dx + R] = c
    return cost


def in_set(S, R, p, transpose=False):
    dx, dy = p
    if transpose:
        dx, dy = dy, dx
    return bool(S[dy + R, dx + R])


def walk(side, mids, R=7, vertical=False):
    """A surface on which DCDS walks (0,0) -> (2,0) -> (4,0) and keeps (4,0):
    Step 1's cross picks (2,0) (horizontal, so the horizontal diamond follows),
    the diamond at (2,0) picks its distant point (4,0), and the diamond at
    (4,0) keeps its centre (cost 10).  Step 4 then faces the middle points
    (3,0) and (5,0), neither evaluated before, with distortions `mids`, and the
    distant points (2,0) (cost 60) and (6,0) (cost `side`).

    vertical=True: the same walk along y, which starts with the cross's
    vertical near point (0,1) (cost 60): the vertical diamond moves to (0,3),
    keeps it, and Step 4 faces (0,2), (0,4) with distant points (0,1), (0,5)."""
    if not vertical:
        return surface(R, {(0, 0): 100, (2, 0): 60, (4, 0): 10, (6, 0): side, (3, 0): mids[0], (5, 0): mids[1]})
    return surface(R, {(0, 0): 100, (0, 1): 60, (0, 3): 10, (0, 5): side, (0, 2): mids[0], (0, 4): mids[1]})


def pin_simplified_side_rule():
    """The middle point on the side of the smaller distant point, and only it,
    is checked; ties go to the negative side.  The middle distortions are set
    against the chosen side, so a rule that looked at them would differ."""
    for vertical in (False, True):
        lo, hi = ((0, 2), (0, 4)) if vertical else ((3, 0), (5, 0))
        base = 15  # plain DCDS's NSP on this walk: 7 (cross) + 3 + 3 (diamonds) + 2 (middles)
        # Plain DCDS checks both middles and takes the better (lo, cost 3).
        mv, d, nsp, S = oracle.dcds_surface(walk(50, (3, 7), vertical=vertical), want_set=True)
        assert (mv, d, nsp) == (lo, 3, base), (vertical, mv, d, nsp)
        for side, mids, pick, cost in ((50, (3, 7), hi, 7),    # (6,0) beats (2,0): positive side only
                                       (70, (7, 3), lo, 7),    # (2,0) beats (6,0): negative side only
                                       (60, (7, 3), lo, 7)):   # a tie: the negative side
            c = walk(side, mids, vertical=vertical)
            mv, d, nsp, S = oracle.dcds_surface(c, variant=oracle.VARIANT_DCDS_S, want_set=True)
            other = hi if pick == lo else lo
            assert (mv, d, nsp) == (pick, cost, base - 1), (vertical, side, mv, d, nsp)
            assert in_set(S, 7, pick) and not in_set(S, 7, other), (vertical, side)


def pin_simplified_edge_reading():
    """When a distant point of the final diamond lies outside the candidate
    set there is no comparison to make: both middle points are checked.  Here
    the window is +-5, so the distant point (6,0) of the diamond at (4,0) is
    outside it; the better middle point (5,0) must be found."""
    c = surface(5, {(0, 0): 100, (2, 0): 60, (4, 0): 10, (3, 0): 7, (5, 0): 3})
    mv, d, nsp, S = oracle.dcds_surface(c, variant=oracle.VARIANT_DCDS_S, want_set=True)
    assert (mv, d, nsp) == ((5, 0), 3, 14), (mv, d, nsp)
    assert in_set(S, 5, (3, 0)) and in_set(S, 5, (5, 0))


def pin_simplified_ideal_condition():
    """Under §III-C's ideal condition the distortion grows with the distance to
    the true vector t, so the distant point nearer t is the smaller one and its
    side's middle point is the one nearer t: DCDS^S must end on t wherever
    DCDS does (every t of the window, edges included), with no more points."""
    for R in (3, 7, 10):
        ys, xs = np.mgrid[-R:R + 1, -R:R + 1]
        for ty in range(-R, R + 1):
            for tx in range(-R, R + 1):
                c = (xs - tx) ** 2 + (ys - ty) ** 2
                a = oracle.dcds_surface(c)
                b = oracle.dcds_surface(c, variant=oracle.VARIANT_DCDS_S)
                assert a[0] == (tx, ty), (R, tx, ty, a)
                assert b[0] == (tx, ty) and b[2] <= a[2], (R, tx, ty, b, a)


def cross_points(c, vertical):
    along = [(-1, 0), (1, 0), (-2, 0), (2, 0)]
    across = [(0, -1), (0, 1)]
    pts = [(0, 0)] + (along + across if not vertical else [(y, x) for x, y in along + across])
    return {(c[0] + dx, c[1] + dy) for dx, dy in pts}


def pin_seeded_first_cross():
    """Plain DCDS stops at the origin (distortion 50); the start s = (4, 3)
    (distortion 5) beats that, so DCDS runs again from s, whose cross keeps s.
    S must be exactly the origin's cross plus s's cross: the transposed cross
    when the proposer says vertical, HCSP otherwise."""
    R, s = 7, (4, 3)
    pts = {p: 80 + k for k, p in enumerate(sorted(cross_points((0, 0), False)))}
    pts[(0, 0)] = 50
    for k, p in enumerate(sorted(cross_points(s, False) | cross_points(s, True))):
        pts[p] = 30 + k
    pts[s] = 5
    c = surface(R, pts)
    for vertical in (False, True):
        mv, d, nsp, S = oracle.dcds_surface(c, start=s, orient_v=vertical, want_set=True)
        want = cross_points((0, 0), False) | cross_points(s, vertical)
        got = {(x - R, y - R) for y, x in zip(*np.nonzero(S))}
        assert got == want, (vertical, sorted(got ^ want))
        assert (mv, d, nsp) == (s, 5, 14)


def pin_seeded_switching():
    """After a vertical first cross, switching strategy one still follows the
    direction of the move: the cross's vertical distant point s + (0, 2) wins,
    so the vertical diamond follows and evaluates s + (0, 4) and s + (+-1, 2);
    a win on the cross's horizontal arm s + (1, 0) gives the horizontal diamond
    (s + (3, 0), s + (1, +-1))."""
    R, s = 7, (3, -4)
    for arm, ahead, sides in (((0, 2), (0, 4), ((-1, 2), (1, 2))), ((1, 0), (3, 0), ((1, -1), (1, 1)))):
        pts = {(0, 0): 50, s: 20, (s[0] + arm[0], s[1] + arm[1]): 10}
        c = surface(R, pts)
        mv, d, nsp, S = oracle.dcds_surface(c, start=s, orient_v=True, want_set=True)
        assert (mv, d) == ((s[0] + arm[0], s[1] + arm[1]), 10), (arm, mv, d)
        for p in (ahead,) + sides:
            assert in_set(S, R, (s[0] + p[0], s[1] + p[1])), (arm, p)


def pin_seeded_gate():
    """The second search runs when the start beats the origin, and the result
    is the better of the two searches (a tie keeps plain DCDS's).  Plain DCDS
    walks from the origin (100) to (2, 0) (10) with 11 points: the cross, the
    diamond's (4, 0), (2, +-1) and the middle point (3, 0).  The start
    s = (-5, 5) costs 20: better than the origin, not than 10.  From s the
    second search moves to (-4, 5) and stops there (6 new cross points, 3 new
    diamond points, both middle points already in S), so both searches and the
    probe make 21 points.  With (-4, 5) at 3 the second search wins (a rule
    that only follows starts better than plain DCDS's result would miss it);
    at 15, and at 10 (a tie), plain DCDS's result stays.  A start worse than
    the origin (120) runs no second search: 11 points plus the probe."""
    R, s = 7, (-5, 5)
    for v, want in ((3, ((-4, 5), 3, 21)), (15, ((2, 0), 10, 21)), (10, ((2, 0), 10, 21))):
        c = surface(R, {(0, 0): 100, (2, 0): 10, s: 20, (-4, 5): v})
        plain = oracle.dcds_surface(c)
        assert plain == ((2, 0), 10, 11), plain
        got = oracle.dcds_surface(c, start=s, orient_v=False)
        assert got == want, (v, got)
    c = surface(R, {(0, 0): 100, (2, 0): 10, s: 120, (-4, 5): 3})
    assert oracle.dcds_surface(c, start=s, orient_v=False) == ((2, 0), 10, 12)


def pin_seeded_never_worse():
    """On random surfaces and starts the learned-start result is never worse
    than plain DCDS, and equals it (plus the probe) whenever the start does not
    beat the origin."""
    rng = np.random.default_rng(31)
    for R in (3, 7):
        n = 2 * R + 1
        for _ in range(400):
            c = rng.integers(0, 60, (n, n)).astype(np.int64)
            s = tuple(int(v) for v in rng.integers(-R, R + 1, 2))
            v = bool(rng.integers(0, 2))
            p = oracle.dcds_surface(c, want_set=True)
            r = oracle.dcds_surface(c, start=s, orient_v=v)
            assert r[1] <= p[1] and r[2] >= p[2]
            if s == (0, 0) or c[s[1] + R, s[0] + R] >= c[R, R]:
                assert r[:2] == p[:2] and r[2] == p[2] + (0 if p[3][s[1] + R, s[0] + R] else 1)


PINS = [pin_simplified_side_rule, pin_simplified_edge_reading, pin_simplified_ideal_condition,
        pin_seeded_first_cross, pin_seeded_switching, pin_seeded_gate, pin_seeded_never_worse]


def test_simplified_side_rule():
    pin_simplified_side_rule()


def test_simplified_edge_reading():
    pin_simplified_edge_reading()


def test_simplified_ideal_condition():
    pin_simplified_ideal_condition()


def test_seeded_first_cross():
    pin_seeded_first_cross()


def test_seeded_switching():
    pin_seeded_switching()


def test_seeded_gate():
    pin_seeded_gate()


def test_seeded_never_worse():
    pin_seeded_never_worse()


def test_seeded_never_worse_on_frames():
    """Per block of real frames: learned-start DCDS from random starts and
    orientations never ends worse than plain DCDS."""
    for cur, ref, R in ((*qcif_pair(3)[:2], 7), (*make_config(2, frames=2)[::-1], 7)):
        hb, wb = cur.shape[0] // 16, cur.shape[1] // 16
        rng = np.random.default_rng(R + hb)
        start = rng.integers(-R, R + 1, (hb, wb, 2)).astype(np.int16)
        orient = rng.integers(0, 2, (hb, wb)).astype(np.uint8)
        _, sad, nsp = oracle.dcds(cur, ref, 16, R)
        _, ls, ln = oracle.dcds(cur, ref, 16, R, start=start, orient=orient)
        assert (ls <= sad).all()
        assert (ln >= nsp).all()
