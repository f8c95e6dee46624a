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
#pragma once

#include "me_device.hpp"

namespace me {

enum { ALGO_FS = 0, ALGO_DCDS = 1, ALGO_DCDS_S = 2 };

// Offsets of the horizontal patterns of §III-A; the vertical ones are their
// transposes.  Index 0 of the cross is its centre.
__device__ constexpr int kCrossX[7] = {0, -1, 1, -2, 2, 0, 0};
__device__ constexpr int kCrossY[7] = {0, 0, 0, 0, 0, -1, 1};
// Horizontal diamond without its centre: two distant points, two near points.
__device__ constexpr int kDiamX[4] = {-2, 2, 0, 0};
__device__ constexpr int kDiamY[4] = {0, 0, -1, 1};

struct Bounds {
    int lox, hix, loy, hiy;  // candidate set: lox <= x <= hix, loy <= y <= hiy
    __device__ bool in(int x, int y) const { return x >= lox && x <= hix && y >= loy && y <= hiy; }
};

// Marks the n points in the group's bitmap (lane i of the group handles point
// i) and returns how many of the valid ones were not there before.
template <int L, int N>
__device__ __forceinline__ int visit(uint32_t* bm, int R, int lane_g, int gbase, const int (&px)[N],
                                     const int (&py)[N], const bool (&pv)[N]) {
    bool fresh = false;
    int x = 0, y = 0;
    bool v = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (lane_g == i) {
            x = px[i];
            y = py[i];
            v = pv[i];
        }
    }
    if (v) {
        const int k = (y + R) * (2 * R + 1) + (x + R);
        const uint32_t bit = 1u << (k & 31);
        const uint32_t old = atomicOr(&bm[k >> 5], bit);
        fresh = (old & bit) == 0;
    }
    const uint64_t b = __builtin_amdgcn_ballot_w64(fresh);
    const uint64_t m = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
    return __popcll((b >> gbase) & m);
}

template <int N>
__device__ __forceinline__ uint32_t min_key(const uint32_t (&k)[N]) {
    uint32_t m = k[0];
#pragma unroll
    for (int i = 1; i < N; ++i) m = min(m, k[i]);
    return m;
}

struct SearchOut {
    int x, y;
    uint32_t cost, nsp;
};

// Ev: functor with  template <int N> void operator()(const int (&x)[N], const int (&y)[N], uint32_t (&c)[N])
// returning the full distortion of N in-window points (uniform over the group).
// Costs must stay below 2^28 so that (cost << 3 | index) fits a 32-bit key.
template <int L, int ALGO, class Ev>
__device__ SearchOut dcds_search(Ev& ev, int R, const Bounds& bd, uint32_t* bm, int lane_g, int gbase,
                                 bool has_start, int sx, int sy, bool orient_v) {
    int nsp = 0;
    int cx = 0, cy = 0;
    bool vcross = false;

    if (has_start) {
        // Learned start: probe the origin and the (clamped) start.
        sx = clampi(sx, bd.lox, bd.hix);
        sy = clampi(sy, bd.loy, bd.hiy);
        const bool moved = (sx != 0) || (sy != 0);
        int px[2] = {0, sx}, py[2] = {0, sy};
        bool pv[2] = {true, moved};
        uint32_t pc[2];
        ev(px, py, pc);
        nsp += visit<L, 2>(bm, R, lane_g, gbase, px, py, pv);
        if (moved && pc[1] < pc[0]) {
            cx = sx;
            cy = sy;
            vcross = orient_v;
        }
    }

    // Step 1: the cross centred at (cx, cy).
    {
        int px[7], py[7], ex[7], ey[7];
        bool pv[7];
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const int ox = vcross ? kCrossY[i] : kCrossX[i];
            const int oy = vcross ? kCrossX[i] : kCrossY[i];
            px[i] = cx + ox;
            py[i] = cy + oy;
            pv[i] = bd.in(px[i], py[i]);
            ex[i] = pv[i] ? px[i] : cx;
            ey[i] = pv[i] ? py[i] : cy;
        }
        uint32_t c[7], k[7];
        ev(ex, ey, c);
        nsp += visit<L, 7>(bm, R, lane_g, gbase, px, py, pv);
#pragma unroll
        for (int i = 0; i < 7; ++i) k[i] = pv[i] ? ((c[i] << 3) | (uint32_t)i) : 0xFFFFFFFFu;
        const uint32_t km = min_key(k);
        const int w = (int)(km & 7u);
        if (w == 0) return SearchOut{cx, cy, km >> 3, (uint32_t)nsp};  // half-way stop
        const int ox = vcross ? kCrossY[w] : kCrossX[w];
        const int oy = vcross ? kCrossX[w] : kCrossY[w];
        // Switching strategy one: horizontal BMP -> horizontal diamond.
        vcross = (oy != 0);
        cx += ox;
        cy += oy;
        uint32_t ccost = km >> 3;

        // Steps 2/3: diamonds until the centre wins.
        bool patv = vcross;
        uint32_t dist_c0 = 0, dist_c1 = 0;
        bool dist_v0 = false, dist_v1 = false;
        int guard = (2 * R + 1) * (2 * R + 1);
        for (;;) {
            int qx[4], qy[4], fx[4], fy[4];
            bool qv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int dx = patv ? kDiamY[i] : kDiamX[i];
                const int dy = patv ? kDiamX[i] : kDiamY[i];
                qx[i] = cx + dx;
                qy[i] = cy + dy;
                qv[i] = bd.in(qx[i], qy[i]);
                fx[i] = qv[i] ? qx[i] : cx;
                fy[i] = qv[i] ? qy[i] : cy;
            }
            uint32_t q[4], kk[5];
            ev(fx, fy, q);
            nsp += visit<L, 4>(bm, R, lane_g, gbase, qx, qy, qv);
            kk[0] = ccost << 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) kk[i + 1] = qv[i] ? ((q[i] << 3) | (uint32_t)(i + 1)) : 0xFFFFFFFFu;
            const uint32_t m = min_key(kk);
            const int ww = (int)(m & 7u);
            dist_c0 = q[0];
            dist_c1 = q[1];
            dist_v0 = qv[0];
            dist_v1 = qv[1];
            if (ww == 0 || --guard <= 0) break;
            const int dx = patv ? kDiamY[ww - 1] : kDiamX[ww - 1];
            const int dy = patv ? kDiamX[ww - 1] : kDiamY[ww - 1];
            // Switching strategy two: a near point switches to the other diamond.
            if (abs(dx) + abs(dy) == 1) patv = !patv;
            cx += dx;
            cy += dy;
            ccost = m >> 3;
        }

        // Step 4: the centre and the two middle points of the current diamond.
        const int mx = patv ? 0 : 1, my = patv ? 1 : 0;
        int rx[2] = {cx - mx, cx + mx}, ry[2] = {cy - my, cy + my};
        bool rv[2] = {bd.in(rx[0], ry[0]), bd.in(rx[1], ry[1])};
        if (ALGO == ALGO_DCDS_S) {
            // Simplified DCDS (§IV-C): only the middle point on the side of the
            // smaller distant point; ties -> negative side; with one distant
            // point outside the set, its valid partner's side; with none, both.
            bool use0 = true, use1 = true;
            if (dist_v0 && dist_v1) {
                use1 = dist_c1 < dist_c0;
                use0 = !use1;
            } else if (dist_v0) {
                use1 = false;
            } else if (dist_v1) {
                use0 = false;
            }
            rv[0] = rv[0] && use0;
            rv[1] = rv[1] && use1;
        }
        int gx[2] = {rv[0] ? rx[0] : cx, rv[1] ? rx[1] : cx};
        int gy[2] = {rv[0] ? ry[0] : cy, rv[1] ? ry[1] : cy};
        uint32_t r[2], kr[3];
        ev(gx, gy, r);
        nsp += visit<L, 2>(bm, R, lane_g, gbase, rx, ry, rv);
        kr[0] = ccost << 3;
        kr[1] = rv[0] ? ((r[0] << 3) | 1u) : 0xFFFFFFFFu;
        kr[2] = rv[1] ? ((r[1] << 3) | 2u) : 0xFFFFFFFFu;
        const uint32_t m = min_key(kr);
        const int wf = (int)(m & 7u);
        const int fxo = wf == 0 ? cx : rx[wf - 1];
        const int fyo = wf == 0 ? cy : ry[wf - 1];
        return SearchOut{fxo, fyo, m >> 3, (uint32_t)nsp};
    }
}

}  // namespace me
