// Full search over frame pairs, and DCDS over cost surfaces.
#pragma once

#include "me_dcds.hpp"

namespace me {

// Copies rows [ys, ys + rows) x words [xs/4, xs/4 + words) of a frame into
// LDS; words outside the frame read as 0 (no valid candidate ever uses them).
__device__ __forceinline__ void stage_window(uint32_t* dst, const uint8_t* frame, int W, int H, int pitch, int xs,
                                             int ys, int rows, int words, int tid, int nthreads) {
    const int n = rows * words;
    for (int i = tid; i < n; i += nthreads) {
        const int r = i / words;
        const int w = i - r * words;
        const int gx = xs + 4 * w, gy = ys + r;
        uint32_t v = 0;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H)
            v = *reinterpret_cast<const uint32_t*>(frame + (size_t)gy * pitch + gx);
        dst[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Full search.  One workgroup per block.  Work item (y, g): candidate row y
// and four horizontally adjacent candidates x = x_g .. x_g + 3, all four
// evaluated at once by v_qsad_pk_u16_u8 on an 8-byte reference window
// against each 4-byte current word.
// Key of a candidate: SAD << 13 | (|x|+|y|) << 7 | (y + 31) << 1 | (x > 0),
// whose minimum is the tie order (SAD, |x|+|y|, y, x).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int fs_groups(int R) { return margin_words(R) + (R + 1 + 3) / 4; }
__host__ __device__ constexpr int fs_window_words(int B, int R) { return fs_groups(R) + B / 4; }
template <int B>
__host__ __device__ constexpr size_t fs_lds_bytes(int R) {
    return (size_t)4 * ((B + 2 * R) * fs_window_words(B, R)) + (size_t)B * B + 4 * 4;
}

__device__ __forceinline__ uint32_t fs_key(uint32_t s, int x, int y) {
    return (s << 13) | ((uint32_t)(abs(x) + abs(y)) << 7) | ((uint32_t)(y + 31) << 1) | (x > 0 ? 1u : 0u);
}

// One block of one frame pair; all 256 threads of the workgroup call it.
template <int B>
__device__ __forceinline__ void fs_block(uint32_t* smem, const FrameArgs& a, int pair, int bx, int by,
                                         int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                         uint32_t* __restrict__ nsp) {
    const int R = a.R;
    const int MW = margin_words(R);
    const int G = fs_groups(R);
    const int WD = fs_window_words(B, R);
    const int WR = B + 2 * R;
    uint32_t* win = smem;
    uint32_t* curs = smem + WR * WD;
    uint32_t* part = curs + B * B / 4;

    const uint8_t* curf = a.cur + (long long)pair * a.pair_stride;
    const uint8_t* reff = a.ref + (long long)pair * a.pair_stride;
    const int x0 = bx * B, y0 = by * B;
    stage_window(win, reff, a.W, a.H, a.pitch, x0 - 4 * MW, y0 - R, WR, WD, threadIdx.x, 256);
    stage_window(curs, curf, a.W, a.H, a.pitch, x0, y0, B, B / 4, threadIdx.x, 256);
    __syncthreads();

    const int lox = max(-R, -x0), hix = min(R, a.W - B - x0);
    const int loy = max(-R, -y0), hiy = min(R, a.H - B - y0);
    uint32_t best = 0xFFFFFFFFu;
    const int items = (2 * R + 1) * G;
    for (int it = threadIdx.x; it < items; it += 256) {
        const int yi = it / G, g = it - yi * G;
        const int y = yi - R;
        uint64_t acc = 0;
        for (int v = 0; v < B; ++v) {
            const uint32_t* row = win + (yi + v) * WD + g;
            uint32_t d[B / 4 + 1];
#pragma unroll
            for (int k = 0; k <= B / 4; ++k) d[k] = row[k];
#pragma unroll
            for (int k = 0; k < B / 4; ++k)
                acc = __builtin_amdgcn_qsad_pk_u16_u8(((uint64_t)d[k + 1] << 32) | d[k], curs[v * (B / 4) + k], acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = -4 * MW + 4 * g + i;
            const uint32_t s = (uint32_t)(acc >> (16 * i)) & 0xFFFFu;
            const bool ok = x >= lox && x <= hix && y >= loy && y <= hiy;
            best = min(best, ok ? fs_key(s, x, y) : 0xFFFFFFFFu);
        }
    }
    // Workgroup minimum.
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t k = min(min(part[0], part[1]), min(part[2], part[3]));
        const int sgn = (int)(k & 1u);
        const int y = (int)((k >> 1) & 63u) - 31;
        const int l1 = (int)((k >> 7) & 63u);
        const int ax = l1 - abs(y);
        const long long idx = ((long long)pair * a.bh + by) * a.bw + bx;
        mv[2 * idx] = (int16_t)(sgn ? ax : -ax);
        mv[2 * idx + 1] = (int16_t)y;
        sad[idx] = k >> 13;
        nsp[idx] = (uint32_t)((hix - lox + 1) * (hiy - loy + 1));
    }
}

template <int B>
__global__ __launch_bounds__(256) void k_fs(FrameArgs a, int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                            uint32_t* __restrict__ nsp) {
    extern __shared__ uint32_t smem[];
    int t = blockIdx.x;
    const int bx = t % a.bw;
    t /= a.bw;
    const int by = t % a.bh;
    const int pair = t / a.bh;
    fs_block<B>(smem, a, pair, bx, by, mv, sad, nsp);
}

}  // namespace me
