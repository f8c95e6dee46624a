// DCDS over caller cost surfaces (the ideal-condition analysis of §III-C on
// the device).
#pragma once

#include "me_dcds.hpp"

namespace me {

// ---------------------------------------------------------------------------
// DCDS over cost surfaces (ideal-condition analysis of §III-C).  16 lanes per
// surface; the "distortion" of a point is read from the caller's table.
// Points outside the window read a clamped table entry (their results are masked).
// ---------------------------------------------------------------------------
struct SurfaceEval {
    const int32_t* cost;
    int S;    // 2R + 1
    int a00;  // address of (0, 0): R * S + R
    __device__ __forceinline__ int row() const { return S; }
    __device__ __forceinline__ uint32_t at(int a) const { return (uint32_t)cost[clampi(a, 0, S * S - 1)]; }
    __device__ __forceinline__ void pair(int a0, int a1, uint32_t& c0, uint32_t& c1) const {
        c0 = at(a0);
        c1 = at(a1);
    }
    __device__ __forceinline__ uint32_t one(int a0) const { return at(a0); }
    __device__ __forceinline__ void cross(int a, bool t, uint32_t (&c)[7]) const {
        const int arm = t ? S : 1, perp = t ? 1 : S;
        c[0] = at(a);
        c[1] = at(a - arm);
        c[2] = at(a + arm);
        c[3] = at(a - 2 * arm);
        c[4] = at(a + 2 * arm);
        c[5] = at(a - perp);
        c[6] = at(a + perp);
    }
    __device__ __forceinline__ void cross0(uint32_t (&c)[7]) const { cross(a00, false, c); }
};

__global__ __launch_bounds__(256) void k_dcds_surface(const int32_t* __restrict__ cost, const uint8_t* __restrict__ valid,
                                                      int n, int R, bool simplified, const int16_t* __restrict__ start,
                                                      const uint8_t* __restrict__ orient, int16_t* __restrict__ mv,
                                                      uint32_t* __restrict__ out_cost, uint32_t* __restrict__ nsp) {
    constexpr int L = 16;
    constexpr int BMW = bitmap_words(31);
    extern __shared__ uint32_t smem[];
    const int gi = threadIdx.x / L, g = threadIdx.x % L;
    const long long s = (long long)blockIdx.x * (256 / L) + gi;
    uint32_t* bm = smem + gi * BMW;
    for (int i = g; i < BMW; i += L) bm[i] = 0u;
    __syncthreads();
    if (s >= n) return;
    const int side = 2 * R + 1;
    SurfaceEval ev{cost + s * side * side, side, R * side + R};
    // The candidate set is the bounding box of the valid mask, plus the origin.
    Bounds bd{-R, R, -R, R};
    if (valid) {
        const uint8_t* vm = valid + s * side * side;
        int lox = R + 1, hix = -R - 1, loy = R + 1, hiy = -R - 1;
        for (int i = g; i < side * side; i += L) {
            if (vm[i]) {
                const int yy = i / side - R, xx = i % side - R;
                lox = min(lox, xx);
                hix = max(hix, xx);
                loy = min(loy, yy);
                hiy = max(hiy, yy);
            }
        }
        // The origin always belongs to the set (keeps every read in the table).
        bd.lox = min(0, (int)group_min<16>((uint32_t)(lox + 64)) - 64);
        bd.hix = max(0, 64 - (int)group_min<16>((uint32_t)(64 - hix)));
        bd.loy = min(0, (int)group_min<16>((uint32_t)(loy + 64)) - 64);
        bd.hiy = max(0, 64 - (int)group_min<16>((uint32_t)(64 - hiy)));
    }
    const bool seeded = start != nullptr;
    int sx = 0, sy = 0;
    bool ov = false;
    if (seeded) {
        sx = start[2 * s];
        sy = start[2 * s + 1];
        ov = orient != nullptr && orient[s] != 0;
    }
    const SearchOut r =
        seeded ? (simplified ? dcds_search<L, 31, true, true>(ev, R, bd, bm, g, sx, sy, ov)
                             : dcds_search<L, 31, false, true>(ev, R, bd, bm, g, sx, sy, ov))
               : (simplified ? dcds_search<L, 31, true, false>(ev, R, bd, bm, g, sx, sy, ov)
                             : dcds_search<L, 31, false, false>(ev, R, bd, bm, g, sx, sy, ov));
    if (g == 0) {
        mv[2 * s] = (int16_t)r.x;
        mv[2 * s + 1] = (int16_t)r.y;
        out_cost[s] = r.cost;
        nsp[s] = r.nsp;
    }
}

}  // namespace me
