// Host-side helpers shared by the entry points (argument checks, geometry,
// kernel configuration table).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "me.h"
#include "me_dcds.hpp"

#define ME_EXPORT extern "C" __attribute__((visibility("default")))

namespace me {
namespace host {

constexpr size_t kMaxLds = 160 * 1024;  // LDS per compute unit on gfx950

bool aligned(const void* p, uintptr_t m);
int check_frames(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                 int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, const void* mv,
                 const void* sad, const void* nsp);
FrameArgs frame_args(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                     int64_t pair_stride, int32_t block, int32_t range, int tile_w, int tile_h);
int range_class(int R);
// rows per lane and waves per group of DCDS for (block, range class)
void current_cfg(int block, int rc, int* rpl, int* wpg);
// tiles per grab of the batched DCDS launches for (block, range class)
int current_grab(int block, int rc);
bool valid_cfg(int block, int rpl, int wpg);
bool valid_grab(int grab);  // 0 (default), 1, 2, 4, 8 or 16
constexpr int kDefaultGrab = 4;
// DCDS flags for one job: simplified Step 4, 16-byte loads when aligned.
int dcds_flags(int32_t algo, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t pitch,
               int64_t pair_stride);
int launched();

}  // namespace host
}  // namespace me
