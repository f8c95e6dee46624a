"""Oracle of the MVP statistics of §II-C (plain numpy and Python loops).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Counters over blocks, n = 2R + 1, vector index (y + R) n + (x + R):
  hist[v]        the full-search vector of the block (the "true" MV);
  d1[p][v]       the vector, given p = the best point of the CDS first-step
                 cross S (Eq. (3): the point of minimum distortion in S) --
                 the prior distribution D1 of Eq. (4);
  d2[v][q]       q = the best point of the central 5x5 square, given the
                 vector -- the posterior distribution D2 of Eq. (6).
"Best" follows full search's order (SAD, |x| + |y|, y, x) over the points of
the block's candidate set.  The tables (Tables II, III, VI, Fig. 3, Eqs. (4),
(6), (7)) are fractions of these counts.
"""
from __future__ import annotations

import numpy as np

import oracle

# The CDS first-step cross, in the index order of the d1 counter.
CROSS = [(-2, 0), (-1, 0), (0, 0), (1, 0), (2, 0), (0, -2), (0, -1), (0, 1), (0, 2)]
# The central 5x5 square, index (y + 2) 5 + (x + 2).
SQUARE = [(x, y) for y in range(-2, 3) for x in range(-2, 3)]


def _sad(cur, ref, B, bx, by, x, y):
    c = cur[by * B:(by + 1) * B, bx * B:(bx + 1) * B].astype(np.int64)
    r = ref[by * B + y:(by + 1) * B + y, bx * B + x:(bx + 1) * B + x].astype(np.int64)
    return int(np.abs(c - r).sum())


def _best(cur, ref, B, R, bx, by, points):
    H, W = cur.shape
    cand = []
    for i, (x, y) in enumerate(points):
        if abs(x) <= R and abs(y) <= R and 0 <= bx * B + x <= W - B and 0 <= by * B + y <= H - B:
            cand.append(((_sad(cur, ref, B, bx, by, x, y), abs(x) + abs(y), y, x), i))
    return min(cand)[1]


def counts(cur, ref, B, R, acc=None):
    """Adds one frame pair's blocks to (hist, d1, d2) (int64 arrays)."""
    n = 2 * R + 1
    if acc is None:
        acc = (np.zeros(n * n, np.int64), np.zeros((9, n * n), np.int64), np.zeros((n * n, 25), np.int64))
    hist, d1, d2 = acc
    mv, _, _ = oracle.fullsearch(cur, ref, B, R)
    for by in range(mv.shape[0]):
        for bx in range(mv.shape[1]):
            x, y = int(mv[by, bx, 0]), int(mv[by, bx, 1])
            v = (y + R) * n + (x + R)
            hist[v] += 1
            d1[_best(cur, ref, B, R, bx, by, CROSS), v] += 1
            d2[v, _best(cur, ref, B, R, bx, by, SQUARE)] += 1
    return acc


def _region_masks():
    ys, xs = np.mgrid[-2:3, -2:3]
    ax, ay = abs(xs), abs(ys)
    regions = [np.ones_like(xs, bool), ax + ay <= 2, (xs == 0) | (ys == 0), (ax <= 1) & (ay <= 1),
               (ys == 0) | ((xs == 0) & (ay <= 1))]
    patterns = [(ax <= 1) & (ay <= 1), ((xs == 0) & (ys == 0)) | (ax + ay == 2), (xs == 0) | (ys == 0),
                ((xs == 0) & (ys == 0)) | ((ax == 2) & (ys == 0)) | ((ax == 1) & (ay == 2)),
                (ys == 0) | ((xs == 0) & (ay <= 1))]
    return regions, patterns


def tables(hist, d1, d2, R):
    """The derived tables from the counters (same names and shapes as the
    library's mvp_tables)."""
    n = 2 * R + 1
    h = np.asarray(hist, np.int64).reshape(n, n)  # [y + R, x + R]
    N = int(h.sum())
    fr = (lambda c: c / N) if N else (lambda c: 0.0)
    quarter = np.zeros((R + 1, R + 1))
    for qy in range(R + 1):
        for qx in range(R + 1):
            c = 0
            for sy in ({qy, -qy}):
                for sx in ({qx, -qx}):
                    c += int(h[sy + R, sx + R])
            quarter[qy, qx] = fr(c)
    ax = np.array([fr(int(h[:, d + R].sum())) for d in range(-R, R + 1)])
    ay = np.array([fr(int(h[d + R, :].sum())) for d in range(-R, R + 1)])
    bx = np.array([fr(int(h[R, d + R])) for d in range(-R, R + 1)])
    by = np.array([fr(int(h[d + R, R])) for d in range(-R, R + 1)])
    c5 = np.zeros((5, 5), np.int64)
    for y in range(-2, 3):
        for x in range(-2, 3):
            if abs(x) <= R and abs(y) <= R:
                c5[y + 2, x + 2] = h[y + R, x + R]
    rmasks, pmasks = _region_masks()
    regions = np.array([fr(int(c5[m].sum())) for m in rmasks])
    eta = np.array([fr(int(c5[m].sum())) / int(m.sum()) for m in pmasks])
    d1 = np.asarray(d1, np.int64).reshape(9, n * n)
    rows = d1.sum(axis=1)
    d1n = np.array([d1[p] / rows[p] if rows[p] else np.zeros(n * n) for p in range(9)]).reshape(9, n, n)
    d2 = np.asarray(d2, np.int64).reshape(n * n, 25)
    rs = d2.sum(axis=1)
    d2n = np.array([d2[v] / rs[v] if rs[v] else np.zeros(25) for v in range(n * n)]).reshape(n, n, 5, 5)
    t = []
    for x0 in (4, -7):
        c = np.zeros(25, np.int64)
        for y in range(4, 8):
            for x in range(x0, x0 + 4):
                if abs(x) <= R and abs(y) <= R:
                    c += d2[(y + R) * n + (x + R)]
        t.append((c / c.sum() if c.sum() else np.zeros(25)).reshape(5, 5))
    return {"quarter": quarter, "ax": ax, "ay": ay, "bx": bx, "by": by, "regions": regions, "eta": eta,
            "d1": d1n, "d2": d2n, "t1": t[0], "t2": t[1]}
