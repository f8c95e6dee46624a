// C ABI of the motion-estimation library (declared in include/me.h): argument
// checks on the host, then stream-ordered kernel launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "me.h"
#include "me_host.hpp"
#include "me_kernels.hpp"
#include "me_mvp.hpp"
#include "me_quality.hpp"
#include "me_surface.hpp"

using namespace me;
using namespace me::host;

namespace me {
namespace host {

bool aligned(const void* p, uintptr_t m) { return ((uintptr_t)p & (m - 1)) == 0; }

int check_frames(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                 int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, const void* mv,
                 const void* sad, const void* nsp) {
    if (width <= 0 || height <= 0 || n_pairs < 0) return ME_EINVAL;
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (width % block || height % block) return ME_EINVAL;
    if (pitch < width || (pitch & 3)) return ME_EINVAL;
    // Offsets within one frame are 32-bit (and rows 24-bit products) in the kernels.
    if ((int64_t)height * pitch > (int64_t)INT32_MAX) return ME_EUNSUPPORTED;
    if (n_pairs == 0) return ME_OK;  // nothing to read or write; pointers may be NULL
    if (!cur || !ref || !mv || !sad || !nsp) return ME_EINVAL;
    if (!aligned(cur, 4) || !aligned(ref, 4) || (pair_stride & 3)) return ME_EINVAL;
    if ((int64_t)(width / block) * (height / block) * n_pairs > (int64_t)INT32_MAX) return ME_EUNSUPPORTED;
    return ME_OK;
}

FrameArgs frame_args(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                     int64_t pair_stride, int32_t block, int32_t range, int tile_w, int tile_h) {
    FrameArgs a;
    a.cur = cur;
    a.ref = ref;
    a.pair_stride = pair_stride;
    a.W = width;
    a.H = height;
    a.pitch = pitch;
    a.R = range;
    a.bw = width / block;
    a.bh = height / block;
    a.tiles_x = (a.bw + tile_w - 1) / tile_w;
    a.tiles_y = (a.bh + tile_h - 1) / tile_h;
    a.div_tx = make_divu(a.tiles_x);
    a.div_ty = make_divu(a.tiles_y);
    return a;
}

int launched() { return hipGetLastError() == hipSuccess ? ME_OK : ME_EDEVICE; }

// A dispatch counts its work-items in 32 bits, so one launch stays below 2^31
// of them: a call over more pairs is split into launches over consecutive
// pair ranges, each with its pointers offset to its first pair.
int pairs_per_launch(long long items_per_pair) {
    return (int)std::max<long long>(1, std::min<long long>(INT32_MAX, (long long)INT32_MAX / items_per_pair));
}

// ---------------------------------------------------------------------------
// DCDS kernel configurations: rows per lane x waves per workgroup, per block
// size and range class.  Defaults come from measurements on MI355X; the
// autotuner may replace them.
// ---------------------------------------------------------------------------
int range_class(int R) { return R <= 7 ? 0 : (R <= 15 ? 1 : 2); }

// [block 8/16][range class] = grab << 8 | rpl << 4 | wpg; a zero layout
// (low byte) means the built-in layout, a zero grab the default grab.
std::atomic<int> g_cfg[2][3];
// Built-in defaults (rows per lane * 16 + waves per group) per block size and
// range class (1-7, 8-15, 16-31): the fastest measured on MI355X over a
// 1920x1088 sequence (59 pairs) at ranges 7, 15 and 31.
int default_cfg(int block, int rc) {
    static const int kDefault[2][3] = {
        {2 * 16 + 4, 2 * 16 + 8, 1 * 16 + 8},   // 8x8 blocks
        {2 * 16 + 4, 2 * 16 + 8, 2 * 16 + 8},   // 16x16 blocks
    };
    return kDefault[block == 16][rc];
}
void current_cfg(int block, int rc, int* rpl, int* wpg) {
    int v = g_cfg[block == 16][rc].load(std::memory_order_relaxed) & 255;
    if (!v) v = default_cfg(block, rc);
    *rpl = v / 16;
    *wpg = v % 16;
}
int current_grab(int block, int rc) {
    const int g = g_cfg[block == 16][rc].load(std::memory_order_relaxed) >> 8;
    return g ? g : kDefaultGrab;
}
bool valid_grab(int grab) { return grab == 0 || grab == 1 || grab == 2 || grab == 4 || grab == 8 || grab == 16; }
bool valid_cfg(int block, int rpl, int wpg) {
    const bool r_ok = block == 16 ? (rpl == 1 || rpl == 2 || rpl == 4) : (rpl == 1 || rpl == 2);
    return r_ok && (wpg == 1 || wpg == 2 || wpg == 4 || wpg == 8);
}
int dcds_flags(int32_t algo, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t pitch,
               int64_t pair_stride) {
    int flags = algo == ME_ALGO_DCDS_S ? DCDS_SIMPLIFIED : 0;
    if (aligned(cur, 16) && aligned(ref, 16) && (pitch % 16) == 0 && (width % 16) == 0 && (pair_stride % 16) == 0)
        flags |= DCDS_VEC16;
    return flags;
}

}  // namespace host
}  // namespace me

namespace {

template <int B, int RPL, int WPG, int RMAX>
int launch_dcds_cfg(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                    int64_t pair_stride, int32_t n_pairs, int32_t range, int flags, const me_mv* start,
                    const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp, uint32_t* sse,
                    hipStream_t st) {
    using G = DcdsGeo<B, RPL, WPG, RMAX>;
    const size_t lds = dcds_lds_bytes<B, RPL, WPG, RMAX>();
    if (lds > kMaxLds) return ME_EUNSUPPORTED;
    if (lds > 65536) {
        // Windows above 64 KiB need the kernel's dynamic-LDS limit raised once.
        static std::atomic<int> raised{0};
        if (!raised.load()) {
            if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dcds<B, RPL, WPG, RMAX>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds) != hipSuccess)
                return ME_EUNSUPPORTED;
            raised.store(1);
        }
    }
    const FrameArgs a0 = frame_args(cur, ref, width, height, pitch, pair_stride, B, range, G::BPW, WPG);
    const long long tiles = (long long)a0.tiles_x * a0.tiles_y, blocks = (long long)a0.bw * a0.bh;
    const int ppl = pairs_per_launch(tiles * 64 * WPG);
    for (int p0 = 0; p0 < n_pairs; p0 += ppl) {
        const int np = std::min(ppl, n_pairs - p0);
        const long long o = p0 * blocks;
        FrameArgs a = a0;
        a.cur = cur + p0 * pair_stride;
        a.ref = ref + p0 * pair_stride;
        hipLaunchKernelGGL((k_dcds<B, RPL, WPG, RMAX>), dim3((unsigned)(tiles * np)), dim3(64 * WPG), lds, st, a,
                           flags, start ? reinterpret_cast<const int16_t*>(start + o) : nullptr,
                           orient ? orient + o : nullptr, reinterpret_cast<int16_t*>(mv + o), sad + o, nsp + o,
                           sse ? sse + o : nullptr);
        const int rc = launched();
        if (rc != ME_OK) return rc;
    }
    return ME_OK;
}

template <int B, int RPL, int RMAX>
int launch_dcds_wpg(int wpg, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                    int64_t pair_stride, int32_t n_pairs, int32_t range, int flags, const me_mv* start,
                    const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp, uint32_t* sse, hipStream_t st) {
#define ME_ARGS cur, ref, width, height, pitch, pair_stride, n_pairs, range, flags, start, orient, mv, sad, nsp, sse, st
    if (wpg == 1) return launch_dcds_cfg<B, RPL, 1, RMAX>(ME_ARGS);
    if (wpg == 2) return launch_dcds_cfg<B, RPL, 2, RMAX>(ME_ARGS);
    if (wpg == 4) return launch_dcds_cfg<B, RPL, 4, RMAX>(ME_ARGS);
    return launch_dcds_cfg<B, RPL, 8, RMAX>(ME_ARGS);
}

template <int B, int RMAX>
int launch_dcds_rpl(int rpl, int wpg, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height,
                    int32_t pitch, int64_t pair_stride, int32_t n_pairs, int32_t range, int flags,
                    const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp,
                    uint32_t* sse, hipStream_t st) {
    if (rpl == 1) return launch_dcds_wpg<B, 1, RMAX>(wpg, ME_ARGS);
    if constexpr (B == 16) {
        if (rpl == 4) return launch_dcds_wpg<B, 4, RMAX>(wpg, ME_ARGS);
    }
    return launch_dcds_wpg<B, 2, RMAX>(wpg, ME_ARGS);
}

int launch_dcds(int32_t block, int rpl, int wpg, const uint8_t* cur, const uint8_t* ref, int32_t width,
                int32_t height, int32_t pitch, int64_t pair_stride, int32_t n_pairs, int32_t range, int flags,
                const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp, uint32_t* sse,
                hipStream_t st) {
    const int rc = range_class(range);
    if (block == 16) {
        if (rc == 0) return launch_dcds_rpl<16, 7>(rpl, wpg, ME_ARGS);
        if (rc == 1) return launch_dcds_rpl<16, 15>(rpl, wpg, ME_ARGS);
        return launch_dcds_rpl<16, 31>(rpl, wpg, ME_ARGS);
    }
    if (rc == 0) return launch_dcds_rpl<8, 7>(rpl, wpg, ME_ARGS);
    if (rc == 1) return launch_dcds_rpl<8, 15>(rpl, wpg, ME_ARGS);
    return launch_dcds_rpl<8, 31>(rpl, wpg, ME_ARGS);
#undef ME_ARGS
}

}  // namespace

ME_EXPORT const char* me_status_string(int status) {
    switch (status) {
        case ME_OK: return "ok";
        case ME_EINVAL: return "invalid argument (NULL pointer, size, alignment or pitch)";
        case ME_EUNSUPPORTED: return "unsupported block size, search range or configuration";
        case ME_ENOMEM: return "out of memory";
        case ME_EDEVICE: return "HIP launch or runtime error";
        default: return "unknown status";
    }
}

ME_EXPORT int me_set_config(int32_t block, int32_t range, const me_config* cfg) {
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    const int rc = range_class(range);
    if (!cfg) {
        g_cfg[block == 16][rc].store(0);
        return ME_OK;
    }
    if (!valid_cfg(block, cfg->rows_per_lane, cfg->waves_per_group) || !valid_grab(cfg->tiles_per_grab))
        return ME_EUNSUPPORTED;
    g_cfg[block == 16][rc].store(cfg->tiles_per_grab << 8 | cfg->rows_per_lane << 4 | cfg->waves_per_group);
    return ME_OK;
}

ME_EXPORT int me_get_config(int32_t block, int32_t range, me_config* cfg) {
    if (!cfg) return ME_EINVAL;
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    int rpl, wpg;
    current_cfg(block, range_class(range), &rpl, &wpg);
    cfg->rows_per_lane = rpl;
    cfg->waves_per_group = wpg;
    cfg->tiles_per_grab = current_grab(block, range_class(range));
    return ME_OK;
}

ME_EXPORT int me_search(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                        int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, int32_t algo,
                        const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp,
                        uint32_t* sse, void* stream) {
    int rc = check_frames(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, mv, sad, nsp);
    if (rc != ME_OK) return rc;
    if (algo != ME_ALGO_FS && algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    if (orient && !start) return ME_EINVAL;
    if (algo == ME_ALGO_FS && start) return ME_EINVAL;
    if (n_pairs == 0) return ME_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (algo == ME_ALGO_FS) {
        const FrameArgs a0 = frame_args(cur, ref, width, height, pitch, pair_stride, block, range, 1, 1);
        const long long blocks = (long long)a0.bw * a0.bh;
        const int nt = fs_threads(range);
        const bool split = fs_split(range);
        const size_t lds = block == 16 ? fs_lds_bytes<16>(range) : fs_lds_bytes<8>(range);
        const void* fn = block == 16 ? (split ? reinterpret_cast<const void*>(&k_fs<16, true>)
                                              : reinterpret_cast<const void*>(&k_fs<16, false>))
                                     : (split ? reinterpret_cast<const void*>(&k_fs<8, true>)
                                              : reinterpret_cast<const void*>(&k_fs<8, false>));
        const int ppl = pairs_per_launch(blocks * nt);
        for (int p0 = 0; p0 < n_pairs; p0 += ppl) {
            const int np = std::min(ppl, n_pairs - p0);
            const long long o = p0 * blocks;
            FrameArgs a = a0;
            a.cur = cur + p0 * pair_stride;
            a.ref = ref + p0 * pair_stride;
            int16_t* mvp = reinterpret_cast<int16_t*>(mv + o);
            uint32_t *sadp = sad + o, *nspp = nsp + o, *ssep = sse ? sse + o : nullptr;
            void* args[] = {&a, &mvp, &sadp, &nspp, &ssep};
            if (hipLaunchKernel(fn, dim3((unsigned)(blocks * np)), dim3(nt), args, lds, st) != hipSuccess)
                return ME_EDEVICE;
        }
        return ME_OK;
    }
    const int flags = dcds_flags(algo, cur, ref, width, pitch, pair_stride);
    int rpl, wpg;
    current_cfg(block, range_class(range), &rpl, &wpg);
    return launch_dcds(block, rpl, wpg, cur, ref, width, height, pitch, pair_stride, n_pairs, range, flags, start,
                       orient, mv, sad, nsp, sse, st);
}

ME_EXPORT int me_fullsearch(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                            int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, me_mv* mv,
                            uint32_t* sad, uint32_t* nsp, void* stream) {
    return me_search(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, ME_ALGO_FS, nullptr,
                     nullptr, mv, sad, nsp, nullptr, stream);
}

ME_EXPORT int me_dcds_ex(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                         int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, int32_t algo,
                         const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp,
                         void* stream) {
    if (algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    return me_search(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, algo, start, orient, mv,
                     sad, nsp, nullptr, stream);
}

ME_EXPORT int me_dcds(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                      int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, me_mv* mv, uint32_t* sad,
                      uint32_t* nsp, void* stream) {
    return me_search(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, ME_ALGO_DCDS, nullptr,
                     nullptr, mv, sad, nsp, nullptr, stream);
}

ME_EXPORT int me_frame_quality(const me_mv* mv, const uint32_t* sad, const uint32_t* sse, const me_mv* mv_true,
                               int32_t width, int32_t height, int32_t n_pairs, int32_t block, me_quality* out,
                               void* stream) {
    if (width <= 0 || height <= 0 || n_pairs < 0) return ME_EINVAL;
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (width % block || height % block) return ME_EINVAL;
    if (n_pairs == 0) return ME_OK;
    if (!mv || !sad || !sse || !out) return ME_EINVAL;
    if (!aligned(out, 8)) return ME_EINVAL;
    const long long nb = (long long)(width / block) * (height / block);
    if (nb * n_pairs > (long long)INT32_MAX) return ME_EUNSUPPORTED;
    const int ppl = pairs_per_launch(256);
    for (int p0 = 0; p0 < n_pairs; p0 += ppl) {
        const int np = std::min(ppl, n_pairs - p0);
        const long long o = p0 * nb;
        hipLaunchKernelGGL(k_frame_quality, dim3((unsigned)np), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                           reinterpret_cast<const int16_t*>(mv + o), sad + o, sse + o,
                           mv_true ? reinterpret_cast<const int16_t*>(mv_true + o) : nullptr, (int)nb, block,
                           reinterpret_cast<QualityOut*>(out) + p0);
        const int rc = launched();
        if (rc != ME_OK) return rc;
    }
    return ME_OK;
}

ME_EXPORT int me_mvp_stats(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                           int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, uint32_t* hist,
                           uint32_t* d1, uint32_t* d2, void* stream) {
    int rc = check_frames(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, hist, d1, d2);
    if (rc != ME_OK || n_pairs == 0) return rc;
    if (!aligned(hist, 4) || !aligned(d1, 4) || !aligned(d2, 4)) return ME_EINVAL;
    const FrameArgs a = frame_args(cur, ref, width, height, pitch, pair_stride, block, range, 1, 1);
    const long long total = (long long)a.bw * a.bh * n_pairs;
    if (total > INT32_MAX) return ME_EUNSUPPORTED;
    // Chunks of consecutive blocks per workgroup, at most 4096 workgroups.
    const int chunk = (int)((total + 4095) / 4096);
    const unsigned grid = (unsigned)((total + chunk - 1) / chunk);
    const int nt = fs_threads(range);
    const bool split = fs_split(range);
    const MvpCounts mc{hist, d1, d2, nullptr};
    const size_t hash = 4 * (size_t)mvp_hash_words();
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int tb = (int)total;
    if (block == 16) {
        const size_t lds = fs_lds_bytes<16>(range) + hash;
        if (split) hipLaunchKernelGGL((k_fs_stats<16, true>), dim3(grid), dim3(nt), lds, st, a, mc, tb, chunk);
        else hipLaunchKernelGGL((k_fs_stats<16, false>), dim3(grid), dim3(nt), lds, st, a, mc, tb, chunk);
    } else {
        const size_t lds = fs_lds_bytes<8>(range) + hash;
        if (split) hipLaunchKernelGGL((k_fs_stats<8, true>), dim3(grid), dim3(nt), lds, st, a, mc, tb, chunk);
        else hipLaunchKernelGGL((k_fs_stats<8, false>), dim3(grid), dim3(nt), lds, st, a, mc, tb, chunk);
    }
    return launched();
}

ME_EXPORT int32_t me_mvp_tables_size(int32_t range) {
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    return MvpLayout(range).total;
}

ME_EXPORT int me_mvp_tables(const uint32_t* hist, const uint32_t* d1, const uint32_t* d2, int32_t range, double* out,
                            void* stream) {
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (!hist || !d1 || !d2 || !out) return ME_EINVAL;
    if (!aligned(hist, 4) || !aligned(d1, 4) || !aligned(d2, 4) || !aligned(out, 8)) return ME_EINVAL;
    hipLaunchKernelGGL(k_mvp_tables, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), hist, d1, d2,
                       range, out);
    return launched();
}

ME_EXPORT int me_dcds_surface(const int32_t* cost, const uint8_t* valid, int32_t n, int32_t range, int32_t algo,
                              const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* cost_out,
                              uint32_t* nsp, void* stream) {
    if (n < 0) return ME_EINVAL;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    if (orient && !start) return ME_EINVAL;
    if (n == 0) return ME_OK;
    if (!cost || !mv || !cost_out || !nsp) return ME_EINVAL;
    const size_t lds = (size_t)4 * (16 * bitmap_words(31) + bitmap_slack(16, 31));
    const long long side2 = (long long)(2 * range + 1) * (2 * range + 1);
    const int per = pairs_per_launch(16) / 16 * 16;  // surfaces per launch, whole workgroups
    for (int s0 = 0; s0 < n; s0 += per) {
        const int ns = std::min(per, n - s0);
        hipLaunchKernelGGL(k_dcds_surface, dim3((unsigned)((ns + 15) / 16)), dim3(256), lds,
                           reinterpret_cast<hipStream_t>(stream), cost + s0 * side2, valid ? valid + s0 * side2 : nullptr,
                           ns, range, algo == ME_ALGO_DCDS_S,
                           start ? reinterpret_cast<const int16_t*>(start + s0) : nullptr, orient ? orient + s0 : nullptr,
                           reinterpret_cast<int16_t*>(mv + s0), cost_out + s0, nsp + s0);
        const int rc = launched();
        if (rc != ME_OK) return rc;
    }
    return ME_OK;
}
