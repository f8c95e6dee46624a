// DCDS over frame pairs.
//
// Layout.  A workgroup of WPG waves owns a tile of BPW x WPG blocks: each wave
// takes BPW = 64 / L blocks side by side, each block L = B / RPL lanes, each
// lane RPL rows of its block, at most 4 apart (each row's B/4 words in
// VGPRs; FrameEval gives the mapping).  The
// tile's reference window, widened by RMAX + 2 rows and at least as many
// columns on every side (so every point a pattern can reach from a valid
// centre is in LDS), is staged once; each block keeps its visited-point bitmap
// in LDS.  RMAX is the range class (7, 15 or 31): it fixes the window geometry
// at compile time, the actual range R <= RMAX only bounds the candidate set.
//
// SAD of a point: per lane, two aligned LDS words per 4 pixels, one
// v_alignbyte_b32 and one v_sad_u8 (or v_sad_hi_u8, which accumulates into the
// high half so that two points share one register), then a DPP sum over the
// block's L lanes.  The paper's first step at the origin reads its centre row
// once: v_qsad_pk_u16_u8 gives four horizontal shifts per instruction.
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
    int tiles_x, tiles_y;   // tiles per row / column
    DivU div_tx, div_ty;    // division by tiles_x, tiles_y
};

__host__ __device__ constexpr int round_up(int v, int m) { return (v + m - 1) / m * m; }

template <int B, int RPL, int WPG, int RMAX>
struct DcdsGeo {
    static constexpr int K = B / 4;          // words per block row
    static constexpr int L = B / RPL;        // lanes per block
    static constexpr int D = L < 4 ? L : 4;  // rows between a lane's rows
    static constexpr int BPW = 64 / L;       // blocks per wave
    static constexpr int TW = BPW * B;       // tile width (pixels)
    static constexpr int TH = WPG * B;       // tile height
    static constexpr int MR = RMAX + 2;      // rows above and below the tile
    static constexpr int ML = round_up(MR, 16);              // bytes left of the tile
    static constexpr int NEED = round_up(ML + TW + RMAX + 6, 16) / 4;  // words a row must hold
    // Odd row pitch: the lanes of a block read consecutive rows at one
    // column, and an odd pitch puts those 8 or 16 reads in distinct banks.
    // No wider than needed, so that six tiles fit a CU's LDS at +-15.
    // (Giving each lane adjacent rows would let one ds_read2 fetch both, but
    // spreads a block over every other bank and nearly doubles the bank
    // conflicts between the blocks of a wave.)
    static constexpr int WDW = NEED | 1;
    static constexpr int WR = TH + 2 * MR;   // LDS rows
    static constexpr int WIN_WORDS = WR * WDW;
    static_assert(L >= 2 && BPW * L == 64, "lanes per block must divide the wave");
};

// LDS of one workgroup: the window, then one bitmap per block, each sized
// for the range class, and the bitmaps' slack.
template <int B, int RPL, int WPG, int RMAX>
__host__ __device__ constexpr size_t dcds_lds_bytes() {
    using G = DcdsGeo<B, RPL, WPG, RMAX>;
    return (size_t)4 * (G::WIN_WORDS + G::BPW * WPG * bitmap_words(RMAX) + bitmap_slack(G::L, RMAX));
}

// Stages column c (CH bytes at window x offset c * CH) of the window rows
// r0, r0 + RS, ... (NP of them) into LDS.  Only the last of them can reach
// past the window; it is replaced by row WR - 1, which then gets the same
// chunk from two threads (so no store is conditional).  The window's x
// origin xs and W are multiples of CH, so a chunk lies wholly inside or
// outside the frame.  Every load reads a clamped in-frame address, at a
// 32-bit offset (a frame spans less than 2^31 bytes), so a chunk outside the
// frame holds a copy of frame pixels: no valid candidate reads it, and the
// searches mask every point they evaluate outside the candidate set, which
// only needs finite data there.  Up to four loads are in flight before the
// first store.
template <int CH, int WDW, int WR, int RS, int NP>
__device__ __forceinline__ void stage_column(uint32_t* win, const uint8_t* frame, int W, int H, int pitch, int xs,
                                             int ys, int c, int r0) {
    constexpr int CW = CH / 4;  // words per chunk
    constexpr int U = 4;        // loads per batch
    const int cx = min(max(xs + c * CH, 0), W - CH);
    for (int p0 = 0; p0 < NP; p0 += U) {
        uint32_t v[U][CW];
        int r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            r[u] = r0 + (p0 + u) * RS;
            if (p0 + u == NP - 1) r[u] = min(r[u], WR - 1);
            const int cy = min(max(ys + r[u], 0), H - 1);
            const uint8_t* src = frame + (uint32_t)(cy * pitch + cx);
            if (p0 + u < NP) {
                if constexpr (CW == 4) {
                    const uint4 q = *reinterpret_cast<const uint4*>(src);
                    v[u][0] = q.x;
                    v[u][1] = q.y;
                    v[u][2] = q.z;
                    v[u][3] = q.w;
                } else {
                    v[u][0] = *reinterpret_cast<const uint32_t*>(src);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p0 + u < NP) {
                uint32_t* dst = win + r[u] * WDW + c * CW;
#pragma unroll
                for (int k = 0; k < CW; ++k) dst[k] = v[u][k];
            }
        }
    }
}

// Copies the tile window (WR rows of WB bytes, LDS pitch WDW words) of the
// reference frame into LDS with NT threads.  VEC: 16-byte chunks (frame base,
// pitch and width multiples of 16); otherwise 4-byte chunks.  A thread keeps
// one column over every RS-th row while a row has at most NT chunks, else it
// takes whole columns.
template <int WB, int WDW, int WR, int NT, bool VEC>
__device__ __forceinline__ void stage(uint32_t* win, const uint8_t* frame, int W, int H, int pitch, int xs, int ys) {
    constexpr int CH = VEC ? 16 : 4;  // bytes per chunk
    constexpr int CPR = WB / CH;      // chunks per row
    const int t = threadIdx.x;
    if constexpr (CPR <= NT) {
        constexpr int RS = NT / CPR;  // rows per pass
        const int c = t % CPR, r0 = t / CPR;
        if (r0 < RS) stage_column<CH, WDW, WR, RS, (WR + RS - 1) / RS>(win, frame, W, H, pitch, xs, ys, c, r0);
    } else {
        for (int c = t; c < CPR; c += NT) stage_column<CH, WDW, WR, 1, WR>(win, frame, W, H, pitch, xs, ys, c, 0);
    }
}

// Lane g of a block holds rows row0(g) + j D, j < RPL, D = min(L, 4):
// rows at most 4 apart, so one ds_read2 fetches a word of two of them, and
// the first rows of a block's lanes, (g mod D) + RPL D (g / D), are distinct
// mod 32 for an odd pitch.  A point's address is the LDS byte offset of its
// reference pixel for this lane's first row: a00 + y * ROWB + x.
template <int RPL, int L>
__host__ __device__ constexpr int row0(int g) {
    constexpr int D = L < 4 ? L : 4;
    return g % D + RPL * D * (g / D);
}

template <int B, int RPL, int WDW>
struct FrameEval {
    static constexpr int K = B / 4;
    static constexpr int L = B / RPL;
    static constexpr int D = L < 4 ? L : 4;
    static constexpr int ROWB = WDW * 4;
    static constexpr int JW = D * WDW;  // words between a lane's rows
    int a00;             // address of point (0, 0): an LDS byte address
    uint32_t cur[RPL][K];

    __device__ __forceinline__ int row() const { return ROWB; }

    // Partial SAD of the point at address a over this lane's rows, added into
    // the low (HI = false) or high (HI = true) half of acc.
    template <bool HI>
    __device__ __forceinline__ uint32_t pt(int a, uint32_t acc) const {
        const lds_words w = lds_at((uint32_t)a & ~3u);
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            uint32_t d[K + 1];
#pragma unroll
            for (int k = 0; k <= K; ++k) d[k] = w[j * JW + k];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = __builtin_amdgcn_alignbyte(d[k + 1], d[k], (uint32_t)a);
                acc = HI ? __builtin_amdgcn_sad_hi_u8(f, cur[j][k], acc) : __builtin_amdgcn_sad_u8(f, cur[j][k], acc);
            }
        }
        return acc;
    }

    __device__ __forceinline__ void pair(int a0, int a1, uint32_t& c0, uint32_t& c1) const {
        uint32_t acc = pt<false>(a0, 0u);
        acc = pt<true>(a1, acc);
        acc = group_sum<L>(acc);
        c0 = acc & 0xFFFFu;
        c1 = acc >> 16;
    }

    __device__ __forceinline__ uint32_t one(int a0) const { return group_sum<L>(pt<false>(a0, 0u)); }

    // Sum of squared differences between the block and the reference block at
    // address a (the motion-compensated block), over the whole group:
    // sum (f - c)^2 = sum f^2 + sum c^2 - 2 sum f c, each term one
    // v_dot4_u32_u8 per word; the u32 arithmetic is exact modulo 2^32 and the
    // result is below 2^24.
    __device__ __forceinline__ uint32_t sse(int a) const {
        const lds_words w = lds_at((uint32_t)a & ~3u);
        uint32_t ff = 0, fc = 0, cc = 0;
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            uint32_t d[K + 1];
#pragma unroll
            for (int k = 0; k <= K; ++k) d[k] = w[j * JW + k];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const uint32_t f = __builtin_amdgcn_alignbyte(d[k + 1], d[k], (uint32_t)a);
                ff = __builtin_amdgcn_udot4(f, f, ff, false);
                fc = __builtin_amdgcn_udot4(f, cur[j][k], fc, false);
                cc = __builtin_amdgcn_udot4(cur[j][k], cur[j][k], cc, false);
            }
        }
        return group_sum<L>(ff + cc - 2u * fc);
    }

    // HCSP at the origin: the centre row is read once (K + 2 words from 4
    // bytes left of the block), shifted by 2 bytes, and v_qsad_pk_u16_u8
    // yields the offsets -2, -1, 0, +1 together; the rows above and below are
    // word aligned.
    __device__ __forceinline__ void cross0(uint32_t (&c)[7]) const {
        uint64_t q = 0;
        uint32_t s2 = 0, s3 = 0;
        const lds_words w = lds_at((uint32_t)(a00 - 4));
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            uint32_t d[K + 2], up[K], dn[K];
#pragma unroll
            for (int k = 0; k < K + 2; ++k) d[k] = w[j * JW + k];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                up[k] = w[j * JW - WDW + 1 + k];
                dn[k] = w[j * JW + WDW + 1 + k];
            }
            uint32_t f[K + 1];
#pragma unroll
            for (int k = 0; k <= K; ++k) f[k] = __builtin_amdgcn_alignbyte(d[k + 1], d[k], 2u);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                q = __builtin_amdgcn_qsad_pk_u16_u8(((uint64_t)f[k + 1] << 32) | f[k], cur[j][k], q);
                s2 = __builtin_amdgcn_sad_u8(f[k + 1], cur[j][k], s2);    // (+2, 0)
                s2 = __builtin_amdgcn_sad_hi_u8(up[k], cur[j][k], s2);    // (0, -1)
                s3 = __builtin_amdgcn_sad_u8(dn[k], cur[j][k], s3);       // (0, +1)
            }
        }
        const uint32_t lo = group_sum<L>((uint32_t)q);          // (-2) | (-1) << 16
        const uint32_t hi = group_sum<L>((uint32_t)(q >> 32));  // (0) | (+1) << 16
        s2 = group_sum<L>(s2);
        s3 = group_sum<L>(s3);
        c[0] = hi & 0xFFFFu;
        c[1] = lo >> 16;
        c[2] = hi >> 16;
        c[3] = lo & 0xFFFFu;
        c[4] = s2 & 0xFFFFu;
        c[5] = s2 >> 16;
        c[6] = s3;
    }

    // The cross centred at address a, t = vertical orientation.
    __device__ __forceinline__ void cross(int a, bool t, uint32_t (&c)[7]) const {
        const int arm = t ? ROWB : 1, perp = t ? 1 : ROWB;
        pair(a, a - arm, c[0], c[1]);
        pair(a + arm, a - 2 * arm, c[2], c[3]);
        pair(a + 2 * arm, a - perp, c[4], c[5]);
        c[6] = one(a + perp);
    }
};

// XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
// give each XCD a contiguous run of tiles (neighbouring tiles share window
// rows through that XCD's L2).
__device__ __forceinline__ int xcd_remap(int i, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = i & 7, k = i >> 3;
    return x * q + min(x, r) + k;
}

// flags: DCDS_SIMPLIFIED (Step 4 of DCDS^S), DCDS_VEC16 (16-byte loads allowed).
enum { DCDS_SIMPLIFIED = 1, DCDS_VEC16 = 2 };

// One tile (BPW x WPG blocks) of one frame pair.  All threads of the
// workgroup call it; it ends with every wave done with the LDS window except
// for the final search, so callers that loop must barrier before restaging.
template <int B, int RPL, int WPG, int RMAX>
__device__ __forceinline__ void dcds_tile(uint32_t* smem, const FrameArgs& a, int flags, int pair, int tx, int ty,
                                          const int16_t* __restrict__ start, const uint8_t* __restrict__ orient,
                                          int16_t* __restrict__ mv, uint32_t* __restrict__ sad,
                                          uint32_t* __restrict__ nsp, uint32_t* __restrict__ sse) {
    using G = DcdsGeo<B, RPL, WPG, RMAX>;
    constexpr int L = G::L, K = G::K;
    constexpr int BMW = bitmap_words(RMAX);
    const int R = a.R;
    uint32_t* win = smem;
    uint32_t* bms = smem + G::WIN_WORDS;
    const uint8_t* curf = a.cur + (long long)pair * a.pair_stride;
    const uint8_t* reff = a.ref + (long long)pair * a.pair_stride;
    const int X0 = tx * G::TW, Y0 = ty * G::TH;

    const bool vec = (flags & DCDS_VEC16) != 0;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b = lane / L, g = lane % L;
    // The block of this lane within the tile.  LDS serves a wave in quarters
    // of 16 lanes.  With 8 lanes per block a quarter holds two blocks; one
    // above the other they are B * WDW words apart, which for the odd pitch
    // puts their lanes' words in disjoint banks when both blocks sit at the
    // same displacement (a shared pan, the common case), while side by side,
    // B / 4 words apart, they collide.  So a wave covers 4 columns x 2 rows
    // of blocks, and two waves one band of two tile rows (measured: half the
    // bank conflicts, 0.085 -> 0.081 ms at 1088p +-15).  With 4 lanes per
    // block, four stacked blocks measured slower, so that layout stays a row.
    int bxl = b, byl = wave;
    if constexpr (L == 8 && WPG % 2 == 0) {
        bxl = 4 * (wave & 1) + (lane >> 4);
        byl = 2 * (wave >> 1) + ((lane >> 3) & 1);
    }
    const int bx = tx * G::BPW + bxl, by = ty * WPG + byl;
    const bool exists = bx < a.bw && by < a.bh;
    FrameEval<B, RPL, G::WDW> ev;
    ev.a00 = (int)lds_offset(win) + (G::MR + byl * B + row0<RPL, L>(g)) * (G::WDW * 4) + G::ML + bxl * B;
    const int x0 = bx * B, y0 = by * B;
    // The block's rows are loaded first, so that they are in flight while
    // the window is staged.
    if (exists) {
#pragma unroll
        for (int j = 0; j < RPL; ++j) {
            const uint8_t* row = curf + (size_t)(y0 + row0<RPL, L>(g) + j * G::D) * a.pitch + x0;
            if (K == 4 && vec) {
                const uint4 v = *reinterpret_cast<const uint4*>(row);
                ev.cur[j][0] = v.x;
                ev.cur[j][1] = v.y;
                ev.cur[j][2] = v.z;
                ev.cur[j][3] = v.w;
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) ev.cur[j][k] = reinterpret_cast<const uint32_t*>(row)[k];
            }
        }
    }
    if (vec)
        stage<G::NEED * 4, G::WDW, G::WR, 64 * WPG, true>(win, reff, a.W, a.H, a.pitch, X0 - G::ML, Y0 - G::MR);
    else
        stage<G::NEED * 4, G::WDW, G::WR, 64 * WPG, false>(win, reff, a.W, a.H, a.pitch, X0 - G::ML, Y0 - G::MR);
    // Every bitmap of the tile starts empty: the workgroup clears them
    // together.
    {
        constexpr int NT = 64 * WPG, N = G::BPW * WPG * BMW;
#pragma unroll
        for (int j = 0; j < (N + NT - 1) / NT; ++j)
            if ((j + 1) * NT <= N || (int)threadIdx.x + j * NT < N) bms[threadIdx.x + j * NT] = 0u;
    }
    uint32_t* bm = bms + (wave * G::BPW + b) * BMW;
    __syncthreads();
    if (exists) {
        Bounds bd;
        bd.lox = max(-R, -x0);
        bd.hix = min(R, a.W - B - x0);
        bd.loy = max(-R, -y0);
        bd.hiy = min(R, a.H - B - y0);
        // Below 2^31 (a call covers at most 2^31 - 1 blocks), so 2 idx + 1
        // fits in 32 unsigned bits.
        const uint32_t idx = (uint32_t)((pair * a.bh + by) * a.bw + bx);
        const bool seeded = start != nullptr;
        int sx = 0, sy = 0;
        bool ov = false;
        if (seeded) {
            sx = start[2u * idx];
            sy = start[2u * idx + 1u];
            ov = orient != nullptr && orient[idx] != 0;
        }
        const bool simp = (flags & DCDS_SIMPLIFIED) != 0;
        const SearchOut r =
            seeded ? (simp ? dcds_search<L, RMAX, true, true>(ev, R, bd, bm, g, sx, sy, ov)
                           : dcds_search<L, RMAX, false, true>(ev, R, bd, bm, g, sx, sy, ov))
                   : (simp ? dcds_search<L, RMAX, true, false>(ev, R, bd, bm, g, sx, sy, ov)
                           : dcds_search<L, RMAX, false, false>(ev, R, bd, bm, g, sx, sy, ov));
        // Optional epilogue: the squared error of the compensated block.
        const uint32_t e = sse ? ev.sse(ev.a00 + __mul24(r.y, G::WDW * 4) + r.x) : 0u;
        if (g == 0) {
            mv[2u * idx] = (int16_t)r.x;
            mv[2u * idx + 1u] = (int16_t)r.y;
            sad[idx] = r.cost;
            nsp[idx] = r.nsp;
            if (sse) sse[idx] = e;
        }
    }
}

template <int B, int RPL, int WPG, int RMAX>
__global__ __launch_bounds__(64 * WPG) void k_dcds(FrameArgs a, int flags, const int16_t* __restrict__ start,
                                                    const uint8_t* __restrict__ orient, int16_t* __restrict__ mv,
                                                    uint32_t* __restrict__ sad, uint32_t* __restrict__ nsp,
                                                    uint32_t* __restrict__ sse) {
    extern __shared__ uint32_t smem[];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int r = a.div_tx.div(t), tx = t - r * a.tiles_x;
    const int pair = a.div_ty.div(r), ty = r - pair * a.tiles_y;
    dcds_tile<B, RPL, WPG, RMAX>(smem, a, flags, pair, tx, ty, start, orient, mv, sad, nsp, sse);
}

}  // namespace me
