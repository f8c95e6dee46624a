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
// Full search.  One workgroup per block.  Work item (y-group, g): J
// consecutive candidate rows y and four horizontally adjacent candidates
// x = x_g .. x_g + 3; v_qsad_pk_u16_u8 evaluates the four x at once on an
// 8-byte reference window against each 4-byte current word, and each
// reference row read from LDS serves the J rows it belongs to.  The current
// block is wave-uniform (scalar loads).
// Key of a candidate: SAD << 13 | (|x|+|y|) << 7 | (y + 31) << 1 | (x > 0),
// whose minimum is the tie order (SAD, |x|+|y|, y, x).
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int fs_groups(int R) { return margin_words(R) + (R + 1 + 3) / 4; }
__host__ __device__ constexpr int fs_window_words(int B, int R) { return fs_groups(R) + B / 4; }
__host__ __device__ constexpr int fs_rows_per_item(int R) { return R <= 7 ? 1 : 4; }
__host__ __device__ constexpr int fs_items(int R) {
    return fs_groups(R) * ((2 * R + 1 + fs_rows_per_item(R) - 1) / fs_rows_per_item(R));
}
__host__ __device__ constexpr int fs_threads(int R) {
    return fs_items(R) <= 64 ? 64 : (fs_items(R) <= 128 ? 128 : 256);
}
template <int B>
__host__ __device__ constexpr size_t fs_lds_bytes(int R) {
    const int J = fs_rows_per_item(R);
    const int rows = ((2 * R + 1 + J - 1) / J) * J + B - 1;
    return (size_t)4 * rows * fs_window_words(B, R) + 4 * 12;
}

__device__ __forceinline__ uint32_t fs_key(uint32_t s, int x, int y) {
    return (s << 13) | ((uint32_t)(abs(x) + abs(y)) << 7) | ((uint32_t)(y + 31) << 1) | (x > 0 ? 1u : 0u);
}

__device__ __forceinline__ void fs_decode(uint32_t k, int& x, int& y) {
    y = (int)((k >> 1) & 63u) - 31;
    const int ax = (int)((k >> 7) & 63u) - abs(y);
    x = (k & 1u) ? ax : -ax;
}

// Counters of the MVP statistics (§II-C), n = 2R + 1, vector index
// (y + R) n + (x + R):
//   hist[n^2]       full-search vectors (Tables II-III, Fig. 3)
//   d1[9][n^2]      vector given the best point P of the CDS first-step cross
//                   (Eq. (4)); P index: (x + 2) for (x, 0), x = -2..2, then
//                   5..8 for (0, -2), (0, -1), (0, 1), (0, 2)
//   d2[n^2][25]     best point of the central 5x5 square given the vector
//                   (Eq. (6)); point index (y + 2) 5 + (x + 2)
struct MvpCounts {
    uint32_t* hist;
    uint32_t* d1;
    uint32_t* d2;
    uint32_t* lds;  // the workgroup's hash tables (mvp_hash_words words)
};

// Per-workgroup aggregation of the counters: one open-addressing table of
// (key, count) per counter array in LDS, filled by thread 0 only, flushed
// with one global atomic per distinct key.  A key that finds no slot within
// kMvpProbe probes is counted in global memory directly.
constexpr int kMvpSlots = 256;
constexpr int kMvpProbe = 16;
constexpr uint32_t kMvpEmpty = 0xFFFFFFFFu;
__host__ __device__ constexpr int mvp_hash_words() { return 3 * 2 * kMvpSlots; }

__device__ __forceinline__ void mvp_add(uint32_t* tab, uint32_t key, uint32_t* global) {
    uint32_t* keys = tab;
    uint32_t* cnt = tab + kMvpSlots;
    const uint32_t h = (key * 2654435761u) >> 24;
    for (int i = 0; i < kMvpProbe; ++i) {
        const uint32_t s = (h + i) & (kMvpSlots - 1);
        if (keys[s] == key) {
            cnt[s] += 1u;
            return;
        }
        if (keys[s] == kMvpEmpty) {
            keys[s] = key;
            cnt[s] = 1u;
            return;
        }
    }
    atomicAdd(&global[key], 1u);
}

// J candidate rows per item; nt threads per workgroup.  The block rows are
// taken V at a time (a runtime loop, so that only V rows of the current block
// are live in scalar registers); each step reads the V + J - 1 reference rows
// it needs from LDS.
// ST: also the minima over the CDS first-step cross (c1) and over the
// central 5x5 square (c2), with the same keys.
template <int B, int J, bool ST>
__device__ __forceinline__ uint32_t fs_items_min(const uint32_t* win, int WD, int G, int items, int R, int MW,
                                                 const uint32_t* cur, int cpw, int lox, int hix, int loy, int hiy,
                                                 int nt, uint32_t& c1, uint32_t& c2) {
    constexpr int K = B / 4;
    constexpr int V = 4;
    constexpr int Q = V + J - 1;
    uint32_t best = 0xFFFFFFFFu;
    for (int it = threadIdx.x; it < items; it += nt) {
        const int yg = it / G, g = it - yg * G;
        const int y0 = yg * J;  // first candidate row index (y = y0 - R)
        uint64_t acc[J];
#pragma unroll
        for (int j = 0; j < J; ++j) acc[j] = 0;
#pragma unroll 1
        for (int vb = 0; vb < B; vb += V) {
            uint32_t c[V][K];
#pragma unroll
            for (int u = 0; u < V; ++u)
#pragma unroll
                for (int k = 0; k < K; ++k) c[u][k] = cur[(vb + u) * cpw + k];
            uint32_t d[Q][K + 1];
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int k = 0; k <= K; ++k) d[q][k] = win[(y0 + vb + q) * WD + g + k];
#pragma unroll
            for (int u = 0; u < V; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j)
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        acc[j] = __builtin_amdgcn_qsad_pk_u16_u8(((uint64_t)d[u + j][k + 1] << 32) | d[u + j][k],
                                                                 c[u][k], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int y = y0 + j - R;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int x = -4 * MW + 4 * g + i;
                const uint32_t s = (uint32_t)(acc[j] >> (16 * i)) & 0xFFFFu;
                const bool ok = x >= lox && x <= hix && y >= loy && y <= hiy;
                const uint32_t kk = ok ? fs_key(s, x, y) : 0xFFFFFFFFu;
                best = min(best, kk);
                if (ST) {
                    const bool sq = abs(x) <= 2 && abs(y) <= 2;
                    c2 = min(c2, sq ? kk : 0xFFFFFFFFu);
                    c1 = min(c1, sq && (x == 0 || y == 0) ? kk : 0xFFFFFFFFu);
                }
            }
        }
    }
    return best;
}

// One block of one frame pair; all nt threads of the workgroup call it.
// J = fs_rows_per_item(R) (checked by the caller).
// ST: instead of the per-block outputs (mv, sad, nsp may be NULL), count
// the block in the MVP statistics.
template <int B, int J, bool ST = false>
__device__ __forceinline__ void fs_block(uint32_t* smem, const FrameArgs& a, int pair, int bx, int by,
                                         int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                         uint32_t* __restrict__ nsp, uint32_t* __restrict__ sse, int nt,
                                         MvpCounts mc = MvpCounts{nullptr, nullptr, nullptr}) {
    const int R = a.R;
    const int MW = margin_words(R);
    const int G = fs_groups(R);
    const int WD = fs_window_words(B, R);
    const int DG = (2 * R + 1 + J - 1) / J;
    const int WR = DG * J + B - 1;
    uint32_t* win = smem;
    uint32_t* part = smem + WR * WD;

    const uint8_t* curf = a.cur + (long long)pair * a.pair_stride;
    const uint8_t* reff = a.ref + (long long)pair * a.pair_stride;
    const int x0 = bx * B, y0 = by * B;
    stage_window(win, reff, a.W, a.H, a.pitch, x0 - 4 * MW, y0 - R, WR, WD, threadIdx.x, nt);
    // The current block is read straight from global memory: the same words
    // for every lane (scalar loads).
    const uint32_t* cur = reinterpret_cast<const uint32_t*>(curf + (size_t)y0 * a.pitch + x0);
    __syncthreads();

    const int lox = max(-R, -x0), hix = min(R, a.W - B - x0);
    const int loy = max(-R, -y0), hiy = min(R, a.H - B - y0);
    const int items = G * DG;
    uint32_t c1 = 0xFFFFFFFFu, c2 = 0xFFFFFFFFu;
    uint32_t best =
        fs_items_min<B, J, ST>(win, WD, G, items, R, MW, cur, a.pitch / 4, lox, hix, loy, hiy, nt, c1, c2);
    // Workgroup minimum: every thread reads the per-wave minima.
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        best = min(best, (uint32_t)__shfl_xor((int)best, o, 64));
        if (ST) {
            c1 = min(c1, (uint32_t)__shfl_xor((int)c1, o, 64));
            c2 = min(c2, (uint32_t)__shfl_xor((int)c2, o, 64));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        part[threadIdx.x >> 6] = best;
        part[4 + (threadIdx.x >> 6)] = c1;
        part[8 + (threadIdx.x >> 6)] = c2;
    }
    __syncthreads();
    uint32_t k = part[0];
    for (int w = 1; w < nt / 64; ++w) k = min(k, part[w]);
    int x, y;
    fs_decode(k, x, y);
    const long long idx = ((long long)pair * a.bh + by) * a.bw + bx;
    if (ST && threadIdx.x == 0) {
        uint32_t k1 = part[4], k2 = part[8];
        for (int w = 1; w < nt / 64; ++w) {
            k1 = min(k1, part[4 + w]);
            k2 = min(k2, part[8 + w]);
        }
        int x1, y1, x2, y2;
        fs_decode(k1, x1, y1);
        fs_decode(k2, x2, y2);
        const int n = 2 * R + 1;
        const int v = (y + R) * n + (x + R);
        const int p1 = y1 == 0 ? x1 + 2 : (y1 < 0 ? 7 + y1 : 6 + y1);
        const int p2 = (y2 + 2) * 5 + (x2 + 2);
        mvp_add(mc.lds, (uint32_t)v, mc.hist);
        mvp_add(mc.lds + 2 * kMvpSlots, (uint32_t)(p1 * n * n + v), mc.d1);
        mvp_add(mc.lds + 4 * kMvpSlots, (uint32_t)(v * 25 + p2), mc.d2);
    }
    if (!ST && threadIdx.x == 0) {
        mv[2 * idx] = (int16_t)x;
        mv[2 * idx + 1] = (int16_t)y;
        sad[idx] = k >> 13;
        nsp[idx] = (uint32_t)((hix - lox + 1) * (hiy - loy + 1));
    }
    // Optional epilogue: squared error of the compensated block, one word of
    // the block per lane of the first wave (sum (f - c)^2 = f.f + c.c - 2 f.c
    // with v_dot4_u32_u8, exact modulo 2^32).
    if (sse && threadIdx.x < 64) {
        constexpr int K = B / 4;
        uint32_t e = 0;
        if (threadIdx.x < B * K) {
            const int v = threadIdx.x / K, kw = threadIdx.x % K;
            const int b = x + 4 * MW + 4 * kw;  // byte column in the window row
            const uint32_t* row = win + (y + R + v) * WD + (b >> 2);
            const uint32_t f = __builtin_amdgcn_alignbyte(row[1], row[0], (uint32_t)b);
            const uint32_t c = cur[v * (a.pitch / 4) + kw];
            e = __builtin_amdgcn_udot4(f, f, 0u, false) + __builtin_amdgcn_udot4(c, c, 0u, false) -
                2u * __builtin_amdgcn_udot4(f, c, 0u, false);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) e += (uint32_t)__shfl_xor((int)e, o, 64);
        if (threadIdx.x == 0) sse[idx] = e;
    }
}

template <int B, int J>
__global__ __launch_bounds__(256) void k_fs(FrameArgs a, int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                            uint32_t* __restrict__ nsp, uint32_t* __restrict__ sse) {
    extern __shared__ uint32_t smem[];
    int t = blockIdx.x;
    const int bx = t % a.bw;
    t /= a.bw;
    const int by = t % a.bh;
    const int pair = t / a.bh;
    fs_block<B, J>(smem, a, pair, bx, by, mv, sad, nsp, sse, blockDim.x);
}

// Persistent: workgroup w takes blocks [w chunk, (w + 1) chunk) of the
// flattened (pair, by, bx) space.  LDS: window, reduction scratch, then the
// hash tables.
template <int B, int J>
__global__ __launch_bounds__(256) void k_fs_stats(FrameArgs a, MvpCounts mc, int total, int chunk) {
    extern __shared__ uint32_t smem[];
    const int R = a.R;
    const int DG = (2 * R + 1 + J - 1) / J;
    mc.lds = smem + (DG * J + B - 1) * fs_window_words(B, R) + 12;
    for (int i = threadIdx.x; i < mvp_hash_words(); i += blockDim.x)
        mc.lds[i] = (i / kMvpSlots) % 2 == 0 ? kMvpEmpty : 0u;
    const int lo = blockIdx.x * chunk, hi = min(total, lo + chunk);
    for (int b = lo; b < hi; ++b) {
        __syncthreads();
        int t = b;
        const int bx = t % a.bw;
        t /= a.bw;
        const int by = t % a.bh;
        const int pair = t / a.bh;
        fs_block<B, J, true>(smem, a, pair, bx, by, nullptr, nullptr, nullptr, nullptr, blockDim.x, mc);
    }
    __syncthreads();
    uint32_t* const dst[3] = {mc.hist, mc.d1, mc.d2};
    for (int i = threadIdx.x; i < 3 * kMvpSlots; i += blockDim.x) {
        const uint32_t* tab = mc.lds + 2 * kMvpSlots * (i / kMvpSlots);
        const int s = i % kMvpSlots;
        if (tab[s] != kMvpEmpty) atomicAdd(&dst[i / kMvpSlots][tab[s]], tab[kMvpSlots + s]);
    }
}

}  // namespace me
