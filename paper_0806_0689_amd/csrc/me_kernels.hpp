// FS and DCDS kernels over frame pairs, and DCDS over cost surfaces.
#pragma once

#include "me_search.hpp"

namespace me {

struct FrameArgs {
    const uint8_t* cur;
    const uint8_t* ref;
    long long pair_stride;  // bytes between consecutive pairs
    int W, H, pitch;
    int R;
    int bw, bh;             // blocks per row / column
    int tiles_x, tiles_y;   // DCDS tiles per row / column
};

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
// DCDS over frames.  A workgroup of WPG waves owns a tile of BPW x WPG blocks
// (BPW = 64 / B blocks side by side per wave, B lanes per block, one row per
// lane).  The tile's window, widened by the range on every side, is staged in
// LDS once; each block keeps its visited-point bitmap in LDS too.
// ---------------------------------------------------------------------------
template <int B>
struct FrameEval {
    const uint32_t* win;
    int WD;       // words per LDS row
    int rowbase;  // LDS row of this lane's current-block row at y offset 0
    int colbase;  // LDS byte column of the block's left edge at x offset 0
    uint32_t cur[B / 4];

    template <int N>
    __device__ __forceinline__ void operator()(const int (&x)[N], const int (&y)[N], uint32_t (&c)[N]) const {
#pragma unroll
        for (int i = 0; i < N; i += 2) {
            uint32_t acc = row_sad_lo<B>(win + (rowbase + y[i]) * WD, colbase + x[i], cur, 0u);
            if (i + 1 < N) acc = row_sad_hi<B>(win + (rowbase + y[i + 1]) * WD, colbase + x[i + 1], cur, acc);
            acc = group_sum<B>(acc);
            c[i] = acc & 0xFFFFu;
            if (i + 1 < N) c[i + 1] = acc >> 16;
        }
    }
};

__host__ __device__ constexpr int dcds_window_words(int tile_w, int R) { return tile_w / 4 + 2 * margin_words(R) + 1; }
__host__ __device__ constexpr int bitmap_words(int R) { return ((2 * R + 1) * (2 * R + 1) + 31) / 32; }

template <int B, int WPG>
__host__ __device__ constexpr size_t dcds_lds_bytes(int R) {
    return (size_t)4 * ((WPG * B + 2 * R) * dcds_window_words((64 / B) * B, R) + (64 / B) * WPG * bitmap_words(R));
}

template <int B, int WPG, int ALGO>
__global__ __launch_bounds__(64 * WPG) void k_dcds(FrameArgs a, const int16_t* __restrict__ start,
                                                    const uint8_t* __restrict__ orient, int16_t* __restrict__ mv,
                                                    uint32_t* __restrict__ sad, uint32_t* __restrict__ nsp) {
    constexpr int L = B, BPW = 64 / B, TW = BPW * B, TH = WPG * B;
    extern __shared__ uint32_t smem[];
    const int R = a.R;
    const int MW = margin_words(R);
    const int WD = dcds_window_words(TW, R);
    const int WR = TH + 2 * R;
    const int BMW = bitmap_words(R);
    uint32_t* win = smem;
    uint32_t* bms = smem + WR * WD;

    int t = blockIdx.x;
    const int tx = t % a.tiles_x;
    t /= a.tiles_x;
    const int ty = t % a.tiles_y;
    const int pair = t / a.tiles_y;
    const uint8_t* curf = a.cur + (long long)pair * a.pair_stride;
    const uint8_t* reff = a.ref + (long long)pair * a.pair_stride;
    const int X0 = tx * TW, Y0 = ty * TH;

    stage_window(win, reff, a.W, a.H, a.pitch, X0 - 4 * MW, Y0 - R, WR, WD, threadIdx.x, 64 * WPG);

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = lane / L, v = lane % L;
    const int bx = tx * BPW + b, by = ty * WPG + wave;
    const bool exists = bx < a.bw && by < a.bh;
    uint32_t* bm = bms + (wave * BPW + b) * BMW;
    for (int i = v; i < BMW; i += L) bm[i] = 0u;

    FrameEval<B> ev;
    ev.win = win;
    ev.WD = WD;
    ev.rowbase = wave * B + v + R;
    ev.colbase = b * B + 4 * MW;
    const int x0 = bx * B, y0 = by * B;
    if (exists) {
        const uint32_t* crow = reinterpret_cast<const uint32_t*>(curf + (size_t)(y0 + v) * a.pitch + x0);
#pragma unroll
        for (int k = 0; k < B / 4; ++k) ev.cur[k] = crow[k];
    }
    __syncthreads();
    if (!exists) return;

    Bounds bd;
    bd.lox = max(-R, -x0);
    bd.hix = min(R, a.W - B - x0);
    bd.loy = max(-R, -y0);
    bd.hiy = min(R, a.H - B - y0);
    const long long idx = ((long long)pair * a.bh + by) * a.bw + bx;
    const bool has_start = start != nullptr;
    int sx = 0, sy = 0;
    bool ov = false;
    if (has_start) {
        sx = start[2 * idx];
        sy = start[2 * idx + 1];
        ov = orient != nullptr && orient[idx] != 0;
    }
    const SearchOut r = dcds_search<L, ALGO>(ev, R, bd, bm, v, b * L, has_start, sx, sy, ov);
    if (v == 0) {
        mv[2 * idx] = (int16_t)r.x;
        mv[2 * idx + 1] = (int16_t)r.y;
        sad[idx] = r.cost;
        nsp[idx] = r.nsp;
    }
}

// ---------------------------------------------------------------------------
// DCDS over cost surfaces (ideal-condition analysis).  16 lanes per surface;
// the "distortion" of a point is read from the caller's table.
// ---------------------------------------------------------------------------
struct SurfaceEval {
    const int32_t* cost;
    int R;
    template <int N>
    __device__ __forceinline__ void operator()(const int (&x)[N], const int (&y)[N], uint32_t (&c)[N]) const {
#pragma unroll
        for (int i = 0; i < N; ++i) c[i] = (uint32_t)cost[(y[i] + R) * (2 * R + 1) + (x[i] + R)];
    }
};

template <int ALGO>
__global__ __launch_bounds__(256) void k_dcds_surface(const int32_t* __restrict__ cost, const uint8_t* __restrict__ valid,
                                                      int n, int R, const int16_t* __restrict__ start,
                                                      const uint8_t* __restrict__ orient, int16_t* __restrict__ mv,
                                                      uint32_t* __restrict__ out_cost, uint32_t* __restrict__ nsp) {
    constexpr int L = 16;
    extern __shared__ uint32_t smem[];
    const int BMW = bitmap_words(R);
    const int g = threadIdx.x / L, v = threadIdx.x % L;
    const long long s = (long long)blockIdx.x * (256 / L) + g;
    uint32_t* bm = smem + g * BMW;
    for (int i = v; i < BMW; i += L) bm[i] = 0u;
    __syncthreads();
    if (s >= n) return;
    const int side = 2 * R + 1;
    SurfaceEval ev{cost + s * side * side, R};
    // The candidate set is the bounding box of the valid mask (the frame case
    // always yields a rectangle).
    Bounds bd{-R, R, -R, R};
    if (valid) {
        const uint8_t* vm = valid + s * side * side;
        int lox = R + 1, hix = -R - 1, loy = R + 1, hiy = -R - 1;
        for (int i = v; i < side * side; i += L) {
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
    const bool has_start = start != nullptr;
    int sx = 0, sy = 0;
    bool ov = false;
    if (has_start) {
        sx = start[2 * s];
        sy = start[2 * s + 1];
        ov = orient != nullptr && orient[s] != 0;
    }
    const int lane = threadIdx.x & 63;
    const SearchOut r = dcds_search<L, ALGO>(ev, R, bd, bm, v, (lane / L) * L, has_start, sx, sy, ov);
    if (v == 0) {
        mv[2 * s] = (int16_t)r.x;
        mv[2 * s + 1] = (int16_t)r.y;
        out_cost[s] = r.cost;
        nsp[s] = r.nsp;
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

template <int B>
__global__ __launch_bounds__(256) void k_fs(FrameArgs a, int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                            uint32_t* __restrict__ nsp) {
    extern __shared__ uint32_t smem[];
    const int R = a.R;
    const int MW = margin_words(R);
    const int G = fs_groups(R);
    const int WD = fs_window_words(B, R);
    const int WR = B + 2 * R;
    uint32_t* win = smem;
    uint32_t* curs = smem + WR * WD;
    uint32_t* part = curs + B * B / 4;

    int t = blockIdx.x;
    const int bx = t % a.bw;
    t /= a.bw;
    const int by = t % a.bh;
    const int pair = t / a.bh;
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

}  // namespace me
