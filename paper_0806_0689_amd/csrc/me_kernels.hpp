// Full search over frame pairs, and DCDS over cost surfaces.
#pragma once

#include "me_dcds.hpp"

namespace me {

// Copies rows [ys, ys + rows) x words [xs/4, xs/4 + words) of a frame into
// LDS; words outside the frame read as 0 (no valid candidate ever uses them).
// xs and W are multiples of 4, so a word is wholly inside or outside.  A
// thread steps its (row, word) position without dividing; every load reads a
// clamped in-frame address (positions past the window too, whose values are
// dropped), and four loads are issued before any is stored.
__device__ __forceinline__ void stage_window(uint32_t* dst, const uint8_t* frame, int W, int H, int pitch, int xs,
                                             int ys, int rows, int words, int tid, int nthreads) {
    constexpr int U = 4;
    const int n = rows * words;
    int r = tid / words, w = tid - r * words;
    const int dr = nthreads / words, dw = nthreads - dr * words;
    for (int i0 = tid; i0 < n; i0 += U * nthreads) {
        uint32_t v[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int gx = xs + 4 * w, gy = ys + r;
            in[u] = gx >= 0 && gx < W && gy >= 0 && gy < H;
            const int cx = min(max(gx, 0), W - 4), cy = min(max(gy, 0), H - 1);
            // In-frame offset: below 2^31, as height * pitch is.  (A 24-bit
            // product would not do: a frame of few rows may have a pitch of
            // 2^23 bytes or more.)
            v[u] = *reinterpret_cast<const uint32_t*>(frame + (uint32_t)(cy * pitch + cx));
            w += dw;
            r += dr;
            if (w >= words) {
                w -= words;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * nthreads < n) dst[i0 + u * nthreads] = in[u] ? v[u] : 0u;
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
// Candidate rows are taken 4 at a time.
__host__ __device__ constexpr int fs_row_groups(int R) { return (2 * R + 1 + 3) / 4; }
__host__ __device__ constexpr int fs_window_rows(int B, int R) { return 4 * fs_row_groups(R) + B - 1; }
// Up to +-7 a block has too few candidates to give 64 lanes 4 whole
// candidate rows each: the block rows are split over a lane quad instead.
__host__ __device__ constexpr bool fs_split(int R) { return R <= 7; }
__host__ __device__ constexpr int fs_items(int R) {
    return fs_groups(R) * fs_row_groups(R) * (fs_split(R) ? 4 : 1);
}
__host__ __device__ constexpr int fs_threads(int R) {
    return fs_items(R) <= 64 ? 64 : (fs_items(R) <= 128 ? 128 : 256);
}
template <int B>
__host__ __device__ constexpr size_t fs_lds_bytes(int R) {
    return (size_t)4 * fs_window_rows(B, R) * fs_window_words(B, R) + 4 * 12;
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

// The position part of a key splits into a column part and a row part:
// (|x| + |y|) << 7 | (y + 31) << 1 | (x > 0) = X(x) + Y(y) with
// X = |x| << 7 | (x > 0) and Y = |y| << 7 + (y + 31) << 1 (the fields never
// carry into each other), so a lane builds the parts of its 4 columns and
// 4 rows once and keys each candidate with an add.
struct FsAxis {
    uint32_t part;
    bool ok, sq, zero;  // inside the candidate set; within +-2; zero
};
__device__ __forceinline__ FsAxis fs_axis_x(int x, int lo, int hi) {
    return FsAxis{((uint32_t)abs(x) << 7) | (x > 0 ? 1u : 0u), x >= lo && x <= hi, abs(x) <= 2, x == 0};
}
__device__ __forceinline__ FsAxis fs_axis_y(int y, int lo, int hi) {
    return FsAxis{((uint32_t)abs(y) << 7) + ((uint32_t)(y + 31) << 1), y >= lo && y <= hi, abs(y) <= 2, y == 0};
}

// Keys one candidate into the running minima.
// ST: also the minima over the CDS first-step cross (c1) and over the
// central 5x5 square (c2), with the same keys.
template <bool ST>
__device__ __forceinline__ void fs_take(uint32_t s, const FsAxis& ax, const FsAxis& ay, uint32_t& best, uint32_t& c1,
                                        uint32_t& c2) {
    const uint32_t kk = ax.ok && ay.ok ? (s << 13) + ax.part + ay.part : 0xFFFFFFFFu;
    best = min(best, kk);
    if (ST) {
        const bool sq = ax.sq && ay.sq;
        c2 = min(c2, sq ? kk : 0xFFFFFFFFu);
        c1 = min(c1, sq && (ax.zero || ay.zero) ? kk : 0xFFFFFFFFu);
    }
}

// 4 candidate rows per item; nt threads per workgroup.  The block rows are
// taken V at a time (a runtime loop, so that only V rows of the current block
// are live in scalar registers); each step reads the V + J - 1 reference rows
// it needs from LDS.
template <int B, bool ST>
__device__ __forceinline__ uint32_t fs_items_min(const uint32_t* win, int WD, int G, int items, int R, int MW,
                                                 const uint32_t* cur, int cpw, int lox, int hix, int loy, int hiy,
                                                 int nt, uint32_t& c1, uint32_t& c2) {
    constexpr int K = B / 4;
    constexpr int J = 4;
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
        FsAxis ax[4], ay[J];
#pragma unroll
        for (int i = 0; i < 4; ++i) ax[i] = fs_axis_x(-4 * MW + 4 * g + i, lox, hix);
#pragma unroll
        for (int j = 0; j < J; ++j) ay[j] = fs_axis_y(y0 + j - R, loy, hiy);
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                fs_take<ST>((uint32_t)(acc[j] >> (16 * i)) & 0xFFFFu, ax[i], ay[j], best, c1, c2);
    }
    return best;
}

// Small ranges (fs_split): an item is (group of 4 candidate rows, x group g,
// quarter q of the block rows), q fastest, so the four quarters of one
// (row group, g) are one lane quad.  A lane sums its B/4 block rows for the
// 4 candidate rows x 4 shifts; two DPP steps add the quad's partial sums
// (each 16-bit field holds a block SAD, at most 255 B^2 < 2^16), after which
// lane q keys candidate row q.  The block rows differ within a quad, so
// they are vector loads here.  items is a multiple of 4 and at most nt.
template <int B, bool ST>
__device__ __forceinline__ uint32_t fs_items_min_split(const uint32_t* win, int WD, int G, int items, int R, int MW,
                                                       const uint32_t* cur, int cpw, int lox, int hix, int loy,
                                                       int hiy, uint32_t& c1, uint32_t& c2) {
    constexpr int K = B / 4;
    constexpr int J = 4;
    constexpr int V = B / 4;  // block rows per quarter
    constexpr int Q = V + J - 1;
    uint32_t best = 0xFFFFFFFFu;
    const int it = threadIdx.x;
    if (it < items) {  // whole quads only
        const int q = it & 3, item = it >> 2;
        const int yg = item / G, g = item - yg * G;
        const int y0 = yg * J;
        const int vb = q * V;
        uint32_t c[V][K];
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) c[u][k] = cur[(vb + u) * cpw + k];
        uint32_t d[Q][K + 1];
#pragma unroll
        for (int r = 0; r < Q; ++r)
#pragma unroll
            for (int k = 0; k <= K; ++k) d[r][k] = win[(y0 + vb + r) * WD + g + k];
        uint64_t acc[J];
#pragma unroll
        for (int j = 0; j < J; ++j) acc[j] = 0;
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
            for (int j = 0; j < J; ++j)
#pragma unroll
                for (int k = 0; k < K; ++k)
                    acc[j] = __builtin_amdgcn_qsad_pk_u16_u8(((uint64_t)d[u + j][k + 1] << 32) | d[u + j][k], c[u][k],
                                                             acc[j]);
        uint32_t lo = 0, hi = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t l = group_sum<4>((uint32_t)acc[j]), h = group_sum<4>((uint32_t)(acc[j] >> 32));
            lo = q == j ? l : lo;
            hi = q == j ? h : hi;
        }
        const FsAxis ay = fs_axis_y(y0 + q - R, loy, hiy);
        fs_take<ST>(lo & 0xFFFFu, fs_axis_x(-4 * MW + 4 * g, lox, hix), ay, best, c1, c2);
        fs_take<ST>(lo >> 16, fs_axis_x(-4 * MW + 4 * g + 1, lox, hix), ay, best, c1, c2);
        fs_take<ST>(hi & 0xFFFFu, fs_axis_x(-4 * MW + 4 * g + 2, lox, hix), ay, best, c1, c2);
        fs_take<ST>(hi >> 16, fs_axis_x(-4 * MW + 4 * g + 3, lox, hix), ay, best, c1, c2);
    }
    return best;
}

// One block of one frame pair; all nt threads of the workgroup call it.
// SPLIT = fs_split(R) (checked by the caller).
// ST: instead of the per-block outputs (mv, sad, nsp may be NULL), count
// the block in the MVP statistics.
template <int B, bool SPLIT, bool ST = false>
__device__ __forceinline__ void fs_block(uint32_t* smem, const FrameArgs& a, int pair, int bx, int by,
                                         int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                         uint32_t* __restrict__ nsp, uint32_t* __restrict__ sse, int nt,
                                         MvpCounts mc = MvpCounts{nullptr, nullptr, nullptr}) {
    const int R = a.R;
    const int MW = margin_words(R);
    const int G = fs_groups(R);
    const int WD = fs_window_words(B, R);
    const int WR = fs_window_rows(B, R);
    uint32_t* win = smem;
    uint32_t* part = smem + WR * WD;

    const uint8_t* curf = a.cur + (long long)pair * a.pair_stride;
    const uint8_t* reff = a.ref + (long long)pair * a.pair_stride;
    const int x0 = bx * B, y0 = by * B;
    // The current block is read straight from global memory (with whole
    // candidate rows per lane, the same words for every lane: scalar loads).
    const uint32_t* cur = reinterpret_cast<const uint32_t*>(curf + (size_t)y0 * a.pitch + x0);
    stage_window(win, reff, a.W, a.H, a.pitch, x0 - 4 * MW, y0 - R, WR, WD, threadIdx.x, nt);
    __syncthreads();

    const int lox = max(-R, -x0), hix = min(R, a.W - B - x0);
    const int loy = max(-R, -y0), hiy = min(R, a.H - B - y0);
    const int items = fs_items(R);
    uint32_t c1 = 0xFFFFFFFFu, c2 = 0xFFFFFFFFu;
    uint32_t best;
    if constexpr (SPLIT)
        best = fs_items_min_split<B, ST>(win, WD, G, items, R, MW, cur, a.pitch / 4, lox, hix, loy, hiy, c1, c2);
    else
        best = fs_items_min<B, ST>(win, WD, G, items, R, MW, cur, a.pitch / 4, lox, hix, loy, hiy, nt, c1, c2);
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

template <int B, bool SPLIT>
__global__ __launch_bounds__(256) void k_fs(FrameArgs a, int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                            uint32_t* __restrict__ nsp, uint32_t* __restrict__ sse) {
    extern __shared__ uint32_t smem[];
    int t = blockIdx.x;
    const int bx = t % a.bw;
    t /= a.bw;
    const int by = t % a.bh;
    const int pair = t / a.bh;
    fs_block<B, SPLIT>(smem, a, pair, bx, by, mv, sad, nsp, sse, blockDim.x);
}

// Persistent: workgroup w takes blocks [w chunk, (w + 1) chunk) of the
// flattened (pair, by, bx) space.  LDS: window, reduction scratch, then the
// hash tables.
template <int B, bool SPLIT>
__global__ __launch_bounds__(256) void k_fs_stats(FrameArgs a, MvpCounts mc, int total, int chunk) {
    extern __shared__ uint32_t smem[];
    const int R = a.R;
    mc.lds = smem + fs_window_rows(B, R) * fs_window_words(B, R) + 12;
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
        fs_block<B, SPLIT, true>(smem, a, pair, bx, by, nullptr, nullptr, nullptr, nullptr, blockDim.x, mc);
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
