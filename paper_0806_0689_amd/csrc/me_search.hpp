// DCDS control flow (§III-B), shared by the frame kernels and the cost-surface
// kernel.  One group of L lanes runs one search; every value below is uniform
// across the group, and different groups of a wave diverge freely (EXEC masks).
//
// Each step evaluates the whole pattern, including points met before: a point
// already in S has a distortion no smaller than the current centre (the
// centre is the minimum of S by induction, since it only moves to a strictly
// smaller value), and ties keep the centre, so recomputing such a point never
// changes a decision.  The set S itself is kept as a bitmap in LDS, one bit
// per window point, and only serves to count distinct points (NSP).
//
// All pattern points lie on the two axes through the pattern centre.  The
// horizontal patterns of §III-A are listed below as (offset along the arm, arm
// index) pairs; the vertical ones are their transposes.
#pragma once

#include "me_device.hpp"

namespace me {

enum { ALGO_FS = 0, ALGO_DCDS = 1, ALGO_DCDS_S = 2 };

// Horizontal cross (HCSP), centre first: (0,0) (-1,0) (+1,0) (-2,0) (+2,0) (0,-1) (0,+1).
__host__ __device__ constexpr int cross_x(int i) { return i == 1 ? -1 : i == 2 ? 1 : i == 3 ? -2 : i == 4 ? 2 : 0; }
__host__ __device__ constexpr int cross_y(int i) { return i == 5 ? -1 : i == 6 ? 1 : 0; }
// Horizontal diamond (HDSP) without its centre: distant (-2,0) (+2,0), near (0,-1) (0,+1).
__host__ __device__ constexpr int diam_x(int i) { return i == 0 ? -2 : i == 1 ? 2 : 0; }
__host__ __device__ constexpr int diam_y(int i) { return i == 2 ? -1 : i == 3 ? 1 : 0; }
// Middle points of the horizontal diamond: (-1,0) (+1,0).
__host__ __device__ constexpr int mid_x(int i) { return i == 0 ? -1 : 1; }

struct Bounds {
    int lox, hix, loy, hiy;  // candidate set: lox <= x <= hix, loy <= y <= hiy
    __device__ __forceinline__ bool inx(int x) const { return (unsigned)(x - lox) <= (unsigned)(hix - lox); }
    __device__ __forceinline__ bool iny(int y) const { return (unsigned)(y - loy) <= (unsigned)(hiy - loy); }
    __device__ __forceinline__ bool in(int x, int y) const { return inx(x) && iny(y); }
};

// Lane roles for NSP counting: lane g of a group marks point g (and g + L, ...)
// of the pattern being evaluated.  Offsets are stored for the horizontal
// orientation and transposed on use.
template <int L>
struct Roles {
    static constexpr int NR = (7 + L - 1) / L;  // rounds needed for 7 points
    int8_t cx[NR], cy[NR], dx[NR], dy[NR], mx[NR];
    bool cv[NR], dv[NR], mv[NR];
    __device__ __forceinline__ void init(int g) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = g + r * L;
            cx[r] = (int8_t)(i == 1 ? -1 : i == 2 ? 1 : i == 3 ? -2 : i == 4 ? 2 : 0);
            cy[r] = (int8_t)(i == 5 ? -1 : i == 6 ? 1 : 0);
            cv[r] = i < 7;
            dx[r] = (int8_t)(i == 0 ? -2 : i == 1 ? 2 : 0);
            dy[r] = (int8_t)(i == 2 ? -1 : i == 3 ? 1 : 0);
            dv[r] = i < 4;
            mx[r] = (int8_t)(i == 0 ? -1 : 1);
            mv[r] = i < 2;
        }
    }
};

// Marks one point per lane (when `act`) in the group's bitmap; returns the
// number of points of the group that were not marked before.
template <int L>
__device__ __forceinline__ int mark(uint32_t* bm, int R, int gbase, bool act, int x, int y) {
    bool fresh = false;
    if (act) {
        const int k = __mul24(y + R, 2 * R + 1) + (x + R);
        const uint32_t bit = 1u << (k & 31);
        const uint32_t old = atomicOr(&bm[k >> 5], bit);
        fresh = (old & bit) == 0;
    }
    const uint64_t b = __builtin_amdgcn_ballot_w64(fresh);
    const uint64_t m = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
    return __popcll((b >> gbase) & m);
}

struct SearchOut {
    int x, y;
    uint32_t cost, nsp;
};

__device__ __forceinline__ uint32_t key(bool valid, uint32_t cost, uint32_t idx) {
    return valid ? ((cost << 3) | idx) : 0xFFFFFFFFu;
}

// Ev provides, for the group (all costs uniform over the group, each < 2^28):
//   cross0(c[7])               HCSP at the origin (the paper's Step 1)
//   cross(cx, cy, vert, c[7])  the cross at any centre (learned start)
//   diamond(cx, cy, vert, c[4])
//   mids(cx, cy, vert, c[2])
//   probe(sx, sy, c[2])        origin and one start point
// Points outside the candidate set may be evaluated on any finite data; their
// results are masked here.
// simplified: DCDS^S Step 4; seeded: learned start (sx, sy, orient_v).
template <int L, class Ev>
__device__ SearchOut dcds_search(const Ev& ev, int R, const Bounds& bd, uint32_t* bm, const Roles<L>& ro, int gbase,
                                 bool simplified, bool seeded, int sx, int sy, bool orient_v) {
    constexpr int NR = Roles<L>::NR;
    int nsp = 0;
    int cx = 0, cy = 0;
    bool t = false;  // current pattern is vertical

    uint32_t c7[7];
    if (seeded) {
        // Learned start: probe the origin and the (clamped) start.
        sx = clampi(sx, bd.lox, bd.hix);
        sy = clampi(sy, bd.loy, bd.hiy);
        const bool moved = (sx != 0) || (sy != 0);
        uint32_t pc[2];
        ev.probe(sx, sy, pc);
        // Lane 0 of the group marks the origin, lane 1 the start.
        const bool is_start = ro.mx[0] > 0;
        nsp += mark<L>(bm, R, gbase, ro.mv[0] && (!is_start || moved), is_start ? sx : 0, is_start ? sy : 0);
        if (moved && pc[1] < pc[0]) {
            cx = sx;
            cy = sy;
            t = orient_v;
        }
        ev.cross(cx, cy, t, c7);
    } else {
        ev.cross0(c7);
    }

    // Step 1: the cross centred at (cx, cy).
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int ox = t ? ro.cy[r] : ro.cx[r], oy = t ? ro.cx[r] : ro.cy[r];
        const int x = cx + ox, y = cy + oy;
        nsp += mark<L>(bm, R, gbase, ro.cv[r] && bd.in(x, y), x, y);
    }
    uint32_t km;
    {
        uint32_t m = key(true, c7[0], 0);
#pragma unroll
        for (int i = 1; i < 7; ++i) {
            // Points 1-4 lie on the cross's long arm, 5-6 on the short one.
            const int o = i <= 4 ? cross_x(i) : cross_y(i);
            const bool along_x = (i <= 4) != t;
            const bool v = along_x ? bd.inx(cx + o) : bd.iny(cy + o);
            m = min(m, key(v, c7[i], (uint32_t)i));
        }
        km = m;
    }
    const int w = (int)(km & 7u);
    if (w == 0) return SearchOut{cx, cy, km >> 3, (uint32_t)nsp};  // half-way stop
    {
        const int o = w <= 4 ? cross_x(w) : cross_y(w);
        const bool along_x = (w <= 4) != t;
        // Switching strategy one: a BMP in the horizontal direction selects
        // the horizontal diamond, otherwise the vertical one.
        if (along_x) cx += o; else cy += o;
        t = !along_x;
    }
    uint32_t ccost = km >> 3;

    // Steps 2 and 3: the current diamond around the BMP until the centre wins.
    uint32_t d0 = 0, d1 = 0;
    bool v0 = false, v1 = false;
    int guard = (2 * R + 1) * (2 * R + 1);
    for (;;) {
        uint32_t q[4];
        ev.diamond(cx, cy, t, q);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int ox = t ? ro.dy[r] : ro.dx[r], oy = t ? ro.dx[r] : ro.dy[r];
            const int x = cx + ox, y = cy + oy;
            nsp += mark<L>(bm, R, gbase, ro.dv[r] && bd.in(x, y), x, y);
        }
        // Distant points lie on the long arm (x for HDSP), near points on the other.
        v0 = t ? bd.iny(cy - 2) : bd.inx(cx - 2);
        v1 = t ? bd.iny(cy + 2) : bd.inx(cx + 2);
        const bool v2 = t ? bd.inx(cx - 1) : bd.iny(cy - 1);
        const bool v3 = t ? bd.inx(cx + 1) : bd.iny(cy + 1);
        d0 = q[0];
        d1 = q[1];
        uint32_t m = ccost << 3;
        m = min(m, key(v0, q[0], 1u));
        m = min(m, key(v1, q[1], 2u));
        m = min(m, key(v2, q[2], 3u));
        m = min(m, key(v3, q[3], 4u));
        const int ww = (int)(m & 7u);
        if (ww == 0 || --guard <= 0) break;
        ccost = m >> 3;
        if (ww <= 2) {
            // Distant point: keep the pattern.
            const int o = ww == 1 ? -2 : 2;
            if (t) cy += o; else cx += o;
        } else {
            // Near point: switching strategy two, to the other diamond.
            const int o = ww == 3 ? -1 : 1;
            if (t) cx += o; else cy += o;
            t = !t;
        }
    }

    // Step 4: the centre and the two middle points of the current diamond.
    bool r0 = t ? bd.iny(cy - 1) : bd.inx(cx - 1);
    bool r1 = t ? bd.iny(cy + 1) : bd.inx(cx + 1);
    if (simplified) {
        // Simplified DCDS (§IV-C): only the middle point on the side of the
        // smaller distant point; ties -> negative side; with one distant
        // point outside the set, its valid partner's side; with none, both.
        bool use0 = true, use1 = true;
        if (v0 && v1) {
            use1 = d1 < d0;
            use0 = !use1;
        } else if (v0) {
            use1 = false;
        } else if (v1) {
            use0 = false;
        }
        r0 = r0 && use0;
        r1 = r1 && use1;
    }
    uint32_t mc[2];
    ev.mids(cx, cy, t, mc);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int ox = t ? 0 : ro.mx[r], oy = t ? ro.mx[r] : 0;
        const bool act = ro.mv[r] && (ro.mx[r] < 0 ? r0 : r1);
        nsp += mark<L>(bm, R, gbase, act, cx + ox, cy + oy);
    }
    uint32_t m = ccost << 3;
    m = min(m, key(r0, mc[0], 1u));
    m = min(m, key(r1, mc[1], 2u));
    const int wf = (int)(m & 7u);
    if (wf != 0) {
        const int o = wf == 1 ? -1 : 1;
        if (t) cy += o; else cx += o;
    }
    return SearchOut{cx, cy, m >> 3, (uint32_t)nsp};
}

}  // namespace me
