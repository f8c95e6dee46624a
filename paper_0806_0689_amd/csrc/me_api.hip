// C ABI of the motion-estimation library (declared in include/me.h): argument
// checks on the host, then stream-ordered kernel launches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me.h"
#include "me_kernels.hpp"

using namespace me;

namespace {

constexpr int kDcdsWavesPerGroup = 4;

bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

int check_frames(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                 int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, const void* mv,
                 const void* sad, const void* nsp) {
    if (width <= 0 || height <= 0 || n_pairs < 0) return ME_EINVAL;
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (width % block || height % block) return ME_EINVAL;
    if (pitch < width || (pitch & 3)) return ME_EINVAL;
    if (n_pairs == 0) return ME_OK;  // nothing to read or write; pointers may be NULL
    if (!cur || !ref || !mv || !sad || !nsp) return ME_EINVAL;
    if (!aligned4(cur) || !aligned4(ref) || (pair_stride & 3)) return ME_EINVAL;
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
    return a;
}

int launched() { return hipGetLastError() == hipSuccess ? ME_OK : ME_EDEVICE; }

template <int B, int ALGO>
int launch_dcds(const FrameArgs& a, int32_t n_pairs, const me_mv* start, const uint8_t* orient, me_mv* mv,
                uint32_t* sad, uint32_t* nsp, hipStream_t st) {
    constexpr int WPG = kDcdsWavesPerGroup;
    const size_t lds = dcds_lds_bytes<B, WPG>(a.R);
    const long long grid = (long long)a.tiles_x * a.tiles_y * n_pairs;
    hipLaunchKernelGGL((k_dcds<B, WPG, ALGO>), dim3((unsigned)grid), dim3(64 * WPG), lds, st, a,
                       reinterpret_cast<const int16_t*>(start), orient, reinterpret_cast<int16_t*>(mv), sad, nsp);
    return launched();
}

}  // namespace

extern "C" {

const char* me_status_string(int status) {
    switch (status) {
        case ME_OK: return "ok";
        case ME_EINVAL: return "invalid argument (NULL pointer, size, alignment or pitch)";
        case ME_EUNSUPPORTED: return "unsupported block size or search range";
        case ME_ENOMEM: return "out of memory";
        case ME_EDEVICE: return "HIP launch or runtime error";
        default: return "unknown status";
    }
}

int me_fullsearch(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                  int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, me_mv* mv, uint32_t* sad,
                  uint32_t* nsp, void* stream) {
    int rc = check_frames(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, mv, sad, nsp);
    if (rc != ME_OK || n_pairs == 0) return rc;
    const FrameArgs a = frame_args(cur, ref, width, height, pitch, pair_stride, block, range, 1, 1);
    const long long grid = (long long)a.bw * a.bh * n_pairs;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (block == 16)
        hipLaunchKernelGGL(k_fs<16>, dim3((unsigned)grid), dim3(256), fs_lds_bytes<16>(range), st, a,
                           reinterpret_cast<int16_t*>(mv), sad, nsp);
    else
        hipLaunchKernelGGL(k_fs<8>, dim3((unsigned)grid), dim3(256), fs_lds_bytes<8>(range), st, a,
                           reinterpret_cast<int16_t*>(mv), sad, nsp);
    return launched();
}

int me_dcds_ex(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
               int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, int32_t algo,
               const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* sad, uint32_t* nsp, void* stream) {
    int rc = check_frames(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, mv, sad, nsp);
    if (rc != ME_OK) return rc;
    if (algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    if (orient && !start) return ME_EINVAL;
    if (n_pairs == 0) return ME_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int tw = 64 / block;
    const FrameArgs a =
        frame_args(cur, ref, width, height, pitch, pair_stride, block, range, tw, kDcdsWavesPerGroup);
    if (block == 16)
        return algo == ME_ALGO_DCDS ? launch_dcds<16, ALGO_DCDS>(a, n_pairs, start, orient, mv, sad, nsp, st)
                                    : launch_dcds<16, ALGO_DCDS_S>(a, n_pairs, start, orient, mv, sad, nsp, st);
    return algo == ME_ALGO_DCDS ? launch_dcds<8, ALGO_DCDS>(a, n_pairs, start, orient, mv, sad, nsp, st)
                                : launch_dcds<8, ALGO_DCDS_S>(a, n_pairs, start, orient, mv, sad, nsp, st);
}

int me_dcds(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
            int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, me_mv* mv, uint32_t* sad,
            uint32_t* nsp, void* stream) {
    return me_dcds_ex(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range, ME_ALGO_DCDS, nullptr,
                      nullptr, mv, sad, nsp, stream);
}

int me_dcds_surface(const int32_t* cost, const uint8_t* valid, int32_t n, int32_t range, int32_t algo,
                    const me_mv* start, const uint8_t* orient, me_mv* mv, uint32_t* cost_out, uint32_t* nsp,
                    void* stream) {
    if (n < 0) return ME_EINVAL;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    if (orient && !start) return ME_EINVAL;
    if (n == 0) return ME_OK;
    if (!cost || !mv || !cost_out || !nsp) return ME_EINVAL;
    const size_t lds = (size_t)4 * 16 * bitmap_words(range);
    const unsigned grid = (unsigned)((n + 15) / 16);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (algo == ME_ALGO_DCDS)
        hipLaunchKernelGGL(k_dcds_surface<ALGO_DCDS>, dim3(grid), dim3(256), lds, st, cost, valid, n, range,
                           reinterpret_cast<const int16_t*>(start), orient, reinterpret_cast<int16_t*>(mv), cost_out,
                           nsp);
    else
        hipLaunchKernelGGL(k_dcds_surface<ALGO_DCDS_S>, dim3(grid), dim3(256), lds, st, cost, valid, n, range,
                           reinterpret_cast<const int16_t*>(start), orient, reinterpret_cast<int16_t*>(mv), cost_out,
                           nsp);
    return launched();
}

}  // extern "C"
