// Per-pair quality of a motion field (§IV): the sums behind MAD, MSE and the
// PSNR of the motion-compensated frame, and the distance from and agreement
// with reference (full-search) vectors.  One workgroup per frame pair; every
// thread sums a fixed stride of blocks and a fixed tree combines them, so
// the floating-point distance sum is reproducible run to run.
#pragma once

#include "me_device.hpp"

namespace me {

struct QualityOut {  // the layout of me_quality
    unsigned long long sad, sse;
    uint32_t blocks, equal;
    double dist, mad, mse, psnr;
};

__global__ __launch_bounds__(256) void k_frame_quality(const int16_t* __restrict__ mv, const uint32_t* __restrict__ sad,
                                                       const uint32_t* __restrict__ sse,
                                                       const int16_t* __restrict__ mv_true, int nb, int B,
                                                       QualityOut* __restrict__ out) {
    __shared__ unsigned long long s_sad[256], s_sse[256];
    __shared__ uint32_t s_eq[256];
    __shared__ double s_dist[256];
    const int t = threadIdx.x;
    const long long base = (long long)blockIdx.x * nb;
    unsigned long long a = 0, e = 0;
    uint32_t q = 0;
    double d = 0.0;
    for (int i = t; i < nb; i += 256) {
        const long long j = base + i;
        a += sad[j];
        e += sse[j];
        if (mv_true) {
            const int dx = (int)mv[2 * j] - (int)mv_true[2 * j];
            const int dy = (int)mv[2 * j + 1] - (int)mv_true[2 * j + 1];
            q += (dx == 0 && dy == 0) ? 1u : 0u;
            d += sqrt((double)(dx * dx + dy * dy));
        }
    }
    s_sad[t] = a;
    s_sse[t] = e;
    s_eq[t] = q;
    s_dist[t] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            s_sad[t] += s_sad[t + s];
            s_sse[t] += s_sse[t + s];
            s_eq[t] += s_eq[t + s];
            s_dist[t] += s_dist[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        QualityOut r;
        r.sad = s_sad[0];
        r.sse = s_sse[0];
        r.blocks = (uint32_t)nb;
        r.equal = s_eq[0];
        r.dist = s_dist[0];
        const double px = (double)nb * B * B;
        r.mad = (double)r.sad / px;
        r.mse = (double)r.sse / px;
        r.psnr = r.sse == 0 ? __builtin_huge_val() : 10.0 * log10(65025.0 * px / (double)r.sse);
        out[blockIdx.x] = r;
    }
}

}  // namespace me
