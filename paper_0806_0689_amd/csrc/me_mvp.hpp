// Tables of the MVP statistics (§II-C) from the counters of k_fs_stats.
// One workgroup; every output is a sum over counters by one thread in a
// fixed order, divided once, so repeated runs are identical.
#pragma once

#include "me_device.hpp"

namespace me {

// Offsets (in doubles) of the output, n = 2R + 1, m = n^2.
struct MvpLayout {
    int quarter, ax, ay, bx, by, regions, eta, d1, d2, t1, t2, total;
    __host__ __device__ explicit MvpLayout(int R) {
        const int n = 2 * R + 1, m = n * n;
        quarter = 0;
        ax = (R + 1) * (R + 1);
        ay = ax + n;
        bx = ay + n;
        by = bx + n;
        regions = by + n;
        eta = regions + 5;
        d1 = eta + 5;
        d2 = d1 + 9 * m;
        t1 = d2 + 25 * m;
        t2 = t1 + 25;
        total = t2 + 25;
    }
};

// Membership of (x, y), |x|, |y| <= 2, in the five regions of Fig. 3 and the
// five first-step patterns of Table VI (bit i = region or pattern i).
__device__ __forceinline__ int mvp_regions(int x, int y) {
    const int ax = abs(x), ay = abs(y);
    int r = 1;                                          // 5x5 square
    r |= (ax + ay <= 2) << 1;                           // 5x5 diamond
    r |= (x == 0 || y == 0) << 2;                       // 5x5 cross
    r |= (ax <= 1 && ay <= 1) << 3;                     // 3x3 square
    r |= (y == 0 || (x == 0 && ay <= 1)) << 4;          // flat 5x3 diamond (HCSP)
    return r;
}
__device__ __forceinline__ int mvp_patterns(int x, int y) {
    const int ax = abs(x), ay = abs(y);
    int r = (ax <= 1 && ay <= 1);                                            // BBGDS 3x3 square
    r |= ((x == 0 && y == 0) || ax + ay == 2) << 1;                          // DS large diamond
    r |= (x == 0 || y == 0) << 2;                                            // CDS 5x5 cross
    r |= ((x == 0 && y == 0) || (ax == 2 && y == 0) || (ax == 1 && ay == 2)) << 3;  // HEXBS hexagon
    r |= (y == 0 || (x == 0 && ay <= 1)) << 4;                               // DCDS HCSP
    return r;
}

__global__ __launch_bounds__(256) void k_mvp_tables(const uint32_t* __restrict__ hist, const uint32_t* __restrict__ d1,
                                                    const uint32_t* __restrict__ d2, int R, double* __restrict__ out) {
    __shared__ unsigned long long s_total;
    __shared__ double s_rows1[9];
    const MvpLayout L(R);
    const int n = 2 * R + 1, m = n * n, t = threadIdx.x;
    if (t == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < m; ++i) s += hist[i];
        s_total = s;
    }
    if (t < 9) {
        unsigned long long s = 0;
        for (int i = 0; i < m; ++i) s += d1[t * m + i];
        s_rows1[t] = (double)s;
    }
    __syncthreads();
    const double N = (double)s_total;
    auto frac = [&](unsigned long long c) { return N > 0 ? (double)c / N : 0.0; };
    auto h = [&](int x, int y) -> unsigned long long {
        return (abs(x) <= R && abs(y) <= R) ? hist[(y + R) * n + (x + R)] : 0ull;
    };
    // Table II: the distribution folded into one quarter (|x|, |y|).
    for (int i = t; i < (R + 1) * (R + 1); i += 256) {
        const int qy = i / (R + 1), qx = i % (R + 1);
        unsigned long long c = 0;
        for (int sy = 0; sy < (qy ? 2 : 1); ++sy)
            for (int sx = 0; sx < (qx ? 2 : 1); ++sx) c += h(sx ? -qx : qx, sy ? -qy : qy);
        out[L.quarter + i] = frac(c);
    }
    // Table III: marginals A and axis distributions B.
    for (int d = t - R; d <= R; d += 256) {
        unsigned long long cx = 0, cy = 0;
        for (int o = -R; o <= R; ++o) {
            cx += h(d, o);
            cy += h(o, d);
        }
        out[L.ax + d + R] = frac(cx);
        out[L.ay + d + R] = frac(cy);
        out[L.bx + d + R] = frac(h(d, 0));
        out[L.by + d + R] = frac(h(0, d));
    }
    // Fig. 3 regions and Table VI first-step efficiencies (eq. (7)).
    if (t < 10) {
        const int i = t % 5;
        unsigned long long c = 0;
        int pts = 0;
        for (int y = -2; y <= 2; ++y)
            for (int x = -2; x <= 2; ++x) {
                const int in = (t < 5 ? mvp_regions(x, y) : mvp_patterns(x, y)) >> i & 1;
                c += in ? h(x, y) : 0ull;
                pts += in;
            }
        if (t < 5) out[L.regions + i] = frac(c);
        else out[L.eta + i] = frac(c) / pts;
    }
    // Eq. (4): D1 normalised per conditioning point.
    for (int i = t; i < 9 * m; i += 256) {
        const double r = s_rows1[i / m];
        out[L.d1 + i] = r > 0 ? (double)d1[i] / r : 0.0;
    }
    // Eq. (6): D2 normalised per vector.
    for (int v = t; v < m; v += 256) {
        unsigned long long s = 0;
        for (int j = 0; j < 25; ++j) s += d2[v * 25 + j];
        for (int j = 0; j < 25; ++j) out[L.d2 + v * 25 + j] = s ? (double)d2[v * 25 + j] / (double)s : 0.0;
    }
    // D2 given a vector in T1 = [4, 7] x [4, 7] or T2 = [-7, -4] x [4, 7].
    if (t < 50) {
        const int j = t % 25, x0 = t < 25 ? 4 : -7;
        unsigned long long c = 0, s = 0;
        for (int y = 4; y <= 7 && y <= R; ++y)
            for (int x = x0; x <= x0 + 3; ++x) {
                if (abs(x) > R) continue;
                const int v = (y + R) * n + (x + R);
                c += d2[v * 25 + j];
                for (int k = 0; k < 25; ++k) s += d2[v * 25 + k];
            }
        out[(t < 25 ? L.t1 : L.t2) + j] = s ? (double)c / (double)s : 0.0;
    }
}

}  // namespace me
