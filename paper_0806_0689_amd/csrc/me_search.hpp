// DCDS control flow (§III-B), shared by the frame kernels and the cost-surface
// kernel.  One group of L lanes runs one search; every value below is uniform
// across the group, and different groups of a wave diverge freely (EXEC masks).
//
// Visited points never win.  Within one search, the centre is the minimum of
// every point that search has met (it only moves to a point of strictly
// smaller distortion, and ties keep the centre), so a point it evaluated
// before cannot beat it.  Consequences used below:
//  - each small-diamond step evaluates only its three new points: the distant
//    point behind the centre (on the side it came from) is always a point of
//    the previous pattern;
//  - the set S of visited points serves to count distinct points (NSP): it
//    is a bitmap in LDS, one bit per window point, set for every valid point
//    evaluated, and NSP is its popcount; Step 4 of a search that has it to
//    itself also skips the middle points already in it.
// The DCDS^S rule of Step 4 compares the two distant points of the final
// diamond, so the cost of the one behind the centre is carried along.
//
// Points are (x, y) with the pattern's long arm along x for the horizontal
// patterns (HCSP, HDSP) and along y for the vertical ones.
#pragma once

#include "me_device.hpp"

namespace me {

enum { ALGO_FS = 0, ALGO_DCDS = 1, ALGO_DCDS_S = 2 };

struct Bounds {
    int lox, hix, loy, hiy;  // candidate set: lox <= x <= hix, loy <= y <= hiy
};

struct SearchOut {
    int x, y;
    uint32_t cost, nsp;
};

// Room of a centre inside the candidate set: how far it may move towards
// -x, +x, -y, +y.  A point at distance d along one axis is valid iff the room
// on that side is at least d.
struct Room {
    int xl, xh, yl, yh;
    __device__ __forceinline__ void at(const Bounds& bd, int cx, int cy) {
        xl = cx - bd.lox;
        xh = bd.hix - cx;
        yl = cy - bd.loy;
        yh = bd.hiy - cy;
    }
    // Along the arm (x unless t) and across it.
    __device__ __forceinline__ int am(bool t) const { return t ? yl : xl; }
    __device__ __forceinline__ int ap(bool t) const { return t ? yh : xh; }
    __device__ __forceinline__ int pm(bool t) const { return t ? xl : yl; }
    __device__ __forceinline__ int pp(bool t) const { return t ? xh : yh; }
};

// The visited-point bitmap of one search: one bit per window point,
// (2R + 1)^2 bits, in bitmap_words(RMAX) words.  To count, each of the L
// lanes reads the same number of words; the last read of some lanes lies
// past the bitmap (and is ignored), so an array of bitmaps is followed by
// bitmap_slack(L, RMAX) more words.
__host__ __device__ constexpr int bitmap_words(int R) { return ((2 * R + 1) * (2 * R + 1) + 31) / 32; }
__host__ __device__ constexpr int bitmap_slack(int L, int RMAX) {
    return (bitmap_words(RMAX) + L - 1) / L * L - bitmap_words(RMAX);
}

__device__ __forceinline__ uint32_t key(bool valid, uint32_t cost, uint32_t idx) {
    return valid ? ((cost << 3) | idx) : 0xFFFFFFFFu;
}

// Ev (all costs uniform over the group, each < 2^28).  A point is named by an
// address that is affine in (x, y): a(x, y) = a00 + y * row() + x.
//   cross0(c[7])              HCSP at the origin (Step 1)
//   cross(a, t, c[7])         the cross centred at address a; t = vertical
//   pair(a0, a1, c0, c1)      two points
//   one(a0)                   one point
// HCSP order: centre, -1, +1, -2, +2 along the arm, -1, +1 across it.
// Points outside the candidate set may be evaluated on any finite data; their
// results are masked here.

struct WalkOut {
    int x, y;
    uint32_t cost;
    uint32_t c0;  // cost of the first cross's centre
};

// Sets bit k of the group's bitmap when act (fire and forget).
__device__ __forceinline__ void mark_point(uint32_t* bm, bool act, int k) {
    if (act) (void)atomicOr(&bm[k >> 5], 1u << (k & 31));
}

// NSP: the number of bits set in the group's bitmap (the group's own LDS
// operations complete in order, so every mark is visible here).  Words past
// the window's bits are zero; every lane reads NW words, and a last word
// beyond the bitmap is dropped.
template <int L, int RMAX>
__device__ __forceinline__ uint32_t count_points(const uint32_t* bm, int g) {
    constexpr int WMAX = bitmap_words(RMAX), NW = (WMAX + L - 1) / L;
    uint32_t n = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        const uint32_t w = bm[g + j * L];
        n += __popc(j < NW - 1 || g + j * L < WMAX ? w : 0u);
    }
    return group_sum<L>(n);
}

// Steps 1-4 of DCDS with the first cross centred at (cx, cy): HCSP, or its
// transpose when t.  AT_ORIGIN: the paper's start, (0, 0) with HCSP (its
// cross reads the centre row once).  Every point evaluated is marked in bm.
// Returns the final vector and its cost; the caller counts the points.
// SKIP_VISITED: bm holds only this search's points, so Step 4 may skip a
// middle point already in it (a point met before never beats the centre).
template <int L, bool SIMPLIFIED, bool AT_ORIGIN, bool SKIP_VISITED, class Ev>
__device__ __forceinline__ WalkOut dcds_walk(const Ev& ev, int R, const Bounds& bd, uint32_t* bm, int g, int cx,
                                             int cy, bool t) {
    const int S = 2 * R + 1;      // bitmap row length
    const int k00 = R * S + R;    // bitmap index of the origin
    const int rs = ev.row();

    uint32_t c7[7];
    if constexpr (AT_ORIGIN) {
        cx = 0;
        cy = 0;
        t = false;
        ev.cross0(c7);
    } else {
        ev.cross(ev.a00 + __mul24(cy, rs) + cx, t, c7);
    }

    // Step 1: the cross centred at (cx, cy).
    Room rc;
    rc.at(bd, cx, cy);
    const bool am1 = rc.am(t) >= 1, ap1 = rc.ap(t) >= 1, am2 = rc.am(t) >= 2, ap2 = rc.ap(t) >= 2;
    const bool pm1 = rc.pm(t) >= 1, pp1 = rc.pp(t) >= 1;
    {
        // Lane g marks cross point g (and g + L when L = 4).
#pragma unroll
        for (int r = 0; r < (7 + L - 1) / L; ++r) {
            const int i = g + r * L;
            const int oa = i == 1 ? -1 : i == 2 ? 1 : i == 3 ? -2 : i == 4 ? 2 : 0;  // along the arm
            const int op = i == 5 ? -1 : i == 6 ? 1 : 0;                             // across it
            const bool v = i == 0 || (i == 1 && am1) || (i == 2 && ap1) || (i == 3 && am2) || (i == 4 && ap2) ||
                           (i == 5 && pm1) || (i == 6 && pp1);
            const int dx = t ? op : oa, dy = t ? oa : op;
            mark_point(bm, v, k00 + __mul24(cy + dy, S) + (cx + dx));
        }
    }
    uint32_t m = c7[0] << 3;
    m = min(m, key(am1, c7[1], 1u));
    m = min(m, key(ap1, c7[2], 2u));
    m = min(m, key(am2, c7[3], 3u));
    m = min(m, key(ap2, c7[4], 4u));
    m = min(m, key(pm1, c7[5], 5u));
    m = min(m, key(pp1, c7[6], 6u));
    const uint32_t w = m & 7u;
    if (w == 0) return WalkOut{cx, cy, m >> 3, c7[0]};  // half-way stop

    // Move to the BMP.  Switching strategy one: a BMP along x selects the
    // horizontal diamond, otherwise the vertical one.  dir: the last move
    // (its sign says which way is ahead); the point behind the new centre is
    // the opposite cross point (or the cross's centre after a step of 2).
    int dir;
    uint32_t kcost = 0;  // cost of the distant point behind the centre
    {
        // Offset of cross point w (1..6) along its axis, from a table of
        // 4-bit fields holding o + 2: -1, +1, -2, +2, -1, +1.
        const int o = (int)((0x3140310u >> (w << 2)) & 15u) - 2;
        const bool along_x = (w <= 4) != t;
        if (along_x) cx += o; else cy += o;
        t = !along_x;
        dir = o;
        if (SIMPLIFIED) kcost = w == 1 ? c7[2] : w == 2 ? c7[1] : w <= 4 ? c7[0] : w == 5 ? c7[6] : c7[5];
    }
    uint32_t cc8 = m & ~7u;  // centre cost << 3

    // Steps 2 and 3: the current diamond around the BMP until the centre
    // wins.  New points: F (distant, ahead), N- and N+ (near).
    uint32_t cF = 0;
    rc.at(bd, cx, cy);
    int ca = ev.a00 + __mul24(cy, rs) + cx;  // address of the centre
    int kc = k00 + __mul24(cy, S) + cx;      // its bitmap index
    // Bitmap offsets of this lane's point (F for lane 0, N- for lane 1, N+
    // for lane 2) in the horizontal and vertical diamonds, F ahead on +.
    const int kh = g == 0 ? 2 : g == 1 ? -S : S;
    const int kv = g == 0 ? 2 * S : g == 1 ? -1 : 1;
    const int kmax = S * S;
    for (int it = 0; it < kmax; ++it) {
        const bool s = dir > 0;
        const int ram = rc.am(t), rap = rc.ap(t);
        const bool vF = (s ? rap : ram) >= 2;
        const bool vNm = rc.pm(t) != 0, vNp = rc.pp(t) != 0;
        const int arm2 = t ? 2 * rs : 2, perp = t ? 1 : rs;
        {
            // Marked before the evaluation, so that no masked store splits
            // the sums' DPP steps (which then fold into their adds).
            const int ko = t ? kv : kh;
            mark_point(bm, (g == 0 && vF) || (g == 1 && vNm) || (g == 2 && vNp), kc + ((g == 0 && !s) ? -ko : ko));
        }
        uint32_t cNm, cNp;
        ev.pair(ca + (s ? arm2 : -arm2), ca - perp, cF, cNm);
        cNp = ev.one(ca + perp);
        uint32_t mm = cc8;
        mm = min(mm, key(vF, cF, 1u));
        mm = min(mm, key(vNm, cNm, 3u));
        mm = min(mm, key(vNp, cNp, 4u));
        const uint32_t ww = mm & 7u;
        if (ww == 0) break;
        if (SIMPLIFIED) kcost = ww == 1 ? (cc8 >> 3) : ww == 3 ? cNp : cNm;
        cc8 = mm & ~7u;
        // Distant point: keep the pattern.  Near point: switching strategy
        // two, to the other diamond, moving across the old arm.
        const bool isF = ww == 1;
        const int a = isF ? (s ? 2 : -2) : (ww == 4 ? 1 : -1);
        const bool along_x = isF != t;
        const int ax = along_x ? a : 0, ay = along_x ? 0 : a;
        rc.xl += ax;
        rc.xh -= ax;
        rc.yl += ay;
        rc.yh -= ay;
        ca += __mul24(ay, rs) + ax;
        kc += __mul24(ay, S) + ax;
        t = isF ? t : !t;
        dir = a;
    }
    cx = rc.xl + bd.lox;
    cy = rc.yl + bd.loy;

    // Step 4: the centre and the two middle points of the current diamond.
    bool r0 = rc.am(t) >= 1, r1 = rc.ap(t) >= 1;
    if (SIMPLIFIED) {
        // Simplified DCDS (§IV-C): with both distant points in the set, only
        // the middle point on the side of the smaller one (ties -> negative
        // side).  With a distant point outside the set there is nothing to
        // compare, and both middle points are checked.
        if (rc.am(t) >= 2 && rc.ap(t) >= 2) {
            const uint32_t d0 = dir > 0 ? kcost : cF, d1 = dir > 0 ? cF : kcost;
            r0 = !(d1 < d0);
            r1 = d1 < d0;
        }
    }
    // A middle point this search visited before cannot beat the centre (nor
    // tie it: ties keep the centre), so with SKIP_VISITED only unvisited ones
    // are evaluated, and the wave skips the evaluation when none of its
    // searches has one.  Reading the bitmap after this group's marks is
    // ordered (LDS operations of a wave complete in order).
    const int arm = t ? rs : 1;
    const int ka = t ? S : 1;
    bool n0 = r0, n1 = r1;
    if constexpr (SKIP_VISITED) {
        const int k0 = max(kc - ka, 0), k1 = min(kc + ka, S * S - 1);  // in the bitmap even when not used
        n0 = n0 && !((bm[k0 >> 5] >> (k0 & 31)) & 1u);
        n1 = n1 && !((bm[k1 >> 5] >> (k1 & 31)) & 1u);
    }
    mark_point(bm, (g == 0 && n0) || (g == 1 && n1), g == 0 ? kc - ka : kc + ka);
    uint32_t mf = cc8;
    if (__ballot(n0 && n1)) {
        uint32_t mc0, mc1;
        ev.pair(ca - arm, ca + arm, mc0, mc1);
        mf = min(mf, key(n0, mc0, 1u));
        mf = min(mf, key(n1, mc1, 2u));
    } else if (__ballot(n0 || n1)) {
        const uint32_t mc = ev.one(n0 ? ca - arm : ca + arm);
        mf = min(mf, key(n0 || n1, mc, n0 ? 1u : 2u));
    }
    const uint32_t wf = mf & 7u;
    if (wf != 0) {
        const int o = wf == 1 ? -1 : 1;
        if (t) cy += o; else cx += o;
    }
    return WalkOut{cx, cy, mf >> 3, c7[0]};
}

// The search of one block.  SIMPLIFIED: Step 4 of DCDS^S.  SEEDED: learned
// start (sx, sy, orient_v; this library's addition): plain DCDS runs first;
// the start, clamped into the candidate set, is then probed, and if it beats
// the origin DCDS runs again with its first cross centred there (HCSP, or
// its transpose when orient_v).  The better of the two results is kept (a
// tie keeps plain DCDS's), so it is never worse than plain DCDS's.  Points
// shared by both searches are counted once (the bitmap is common); the second
// search may meet points of the first that beat its centre, so it evaluates
// every point of its patterns but the one it came from, as plain DCDS does,
// and its Step 4 skips nothing.
// bm: the group's bitmap, bitmap_words(RMAX) words, all zero on entry.
template <int L, int RMAX, bool SIMPLIFIED, bool SEEDED, class Ev>
__device__ SearchOut dcds_search(const Ev& ev, int R, const Bounds& bd, uint32_t* bm, int g, int sx, int sy,
                                 bool orient_v) {
    static_assert(L == 4 || L == 8 || L == 16, "group of 4, 8 or 16 lanes");
    WalkOut r = dcds_walk<L, SIMPLIFIED, true, true>(ev, R, bd, bm, g, 0, 0, false);
    if constexpr (SEEDED) {
        sx = clampi(sx, bd.lox, bd.hix);
        sy = clampi(sy, bd.loy, bd.hiy);
        if (sx != 0 || sy != 0) {
            const int S = 2 * R + 1;
            mark_point(bm, g == 0, R * S + R + __mul24(sy, S) + sx);
            const uint32_t ps = ev.one(ev.a00 + __mul24(sy, ev.row()) + sx);
            if (ps < r.c0) {
                const WalkOut q = dcds_walk<L, SIMPLIFIED, false, false>(ev, R, bd, bm, g, sx, sy, orient_v);
                if (q.cost < r.cost) r = q;
            }
        }
    }
    return SearchOut{r.x, r.y, r.cost, count_points<L, RMAX>(bm, g)};
}

}  // namespace me
