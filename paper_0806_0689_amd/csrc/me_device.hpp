// Device helpers for block matching on gfx950 (CDNA4, wave64).
//
// Data layout used by every kernel: a search window is staged in LDS as rows
// of 32-bit words; word w of a row holds frame bytes xs + 4w .. xs + 4w + 3
// (little endian), with xs a multiple of 4, so any byte column is reached
// with two aligned LDS words and one v_alignbyte_b32.  Sums over the lanes of
// one block use DPP (the lanes of a block never straddle a 16-lane DPP row).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

// DPP controls (GCN/CDNA encoding).
constexpr int DPP_QUAD_XOR1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141; // row_half_mirror: lane i <-> 7-i in each 8-lane half
constexpr int DPP_ROR8 = 0x128;       // row_ror:8
constexpr int DPP_ROR4 = 0x124;
constexpr int DPP_ROR2 = 0x122;
constexpr int DPP_ROR1 = 0x121;

// Every control used here reads a lane of the same row, so bound_ctrl never
// applies; setting it lets the move fold into the consuming add or min.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, true);
}

// Sum over aligned groups of L lanes (L = 4, 8 or 16); every lane of the group
// receives the total.  Packed 2 x u16 sums add without carries as long as each
// half's total stays below 2^16.
template <int L>
__device__ __forceinline__ uint32_t group_sum(uint32_t x);

template <>
__device__ __forceinline__ uint32_t group_sum<16>(uint32_t x) {
    x += dpp<DPP_ROR8>(x);
    x += dpp<DPP_ROR4>(x);
    x += dpp<DPP_ROR2>(x);
    x += dpp<DPP_ROR1>(x);
    return x;
}

template <>
__device__ __forceinline__ uint32_t group_sum<4>(uint32_t x) {
    x += dpp<DPP_QUAD_XOR1>(x);
    x += dpp<DPP_QUAD_XOR2>(x);
    return x;
}

template <>
__device__ __forceinline__ uint32_t group_sum<8>(uint32_t x) {
    x += dpp<DPP_QUAD_XOR1>(x);
    x += dpp<DPP_QUAD_XOR2>(x);
    x += dpp<DPP_HALF_MIRROR>(x);
    return x;
}

template <int L>
__device__ __forceinline__ uint32_t group_min(uint32_t x);

template <>
__device__ __forceinline__ uint32_t group_min<16>(uint32_t x) {
    x = min(x, dpp<DPP_ROR8>(x));
    x = min(x, dpp<DPP_ROR4>(x));
    x = min(x, dpp<DPP_ROR2>(x));
    x = min(x, dpp<DPP_ROR1>(x));
    return x;
}

// LDS addressing by byte offset (a 32-bit LDS address, not a generic pointer).
typedef const __attribute__((address_space(3))) uint32_t* lds_words;
__device__ __forceinline__ lds_words lds_at(uint32_t byte) { return (lds_words)(uintptr_t)byte; }
__device__ __forceinline__ uint32_t lds_offset(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Number of 4-byte words of window margin left of a tile for range R.
__host__ __device__ constexpr int margin_words(int R) { return (R + 3) / 4; }

// Division of 0 <= n < 2^31 by a divisor d >= 1 fixed at launch, as one
// 32 x 32 -> 64-bit multiply and a shift (scalar instructions when n is
// uniform; the compiler's division by a run-time value goes through the
// vector float reciprocal).  With 2^l >= d and m = ceil(2^(31+l) / d),
// floor(n m / 2^(31+l)) = floor(n / d): m d - 2^(31+l) = e is in [0, d), so
// the error n e / (d 2^(31+l)) is below 2^-l <= 1/d.  m < 2^32.
struct DivU {
    uint32_t m;
    int s;
    __host__ __device__ constexpr int div(int n) const { return (int)(((uint64_t)(uint32_t)n * m) >> s); }
};
__host__ __device__ constexpr DivU make_divu(int d) {
    int l = 0;
    while ((1LL << l) < d) ++l;
    return DivU{(uint32_t)(((1ULL << (31 + l)) + (uint64_t)d - 1) / (uint64_t)d), 31 + l};
}
static_assert(make_divu(1).div(2147483647) == 2147483647, "divide by 1");
static_assert(make_divu(15).div(2147483647) == 2147483647 / 15, "divide by 15");
static_assert(make_divu(15).div(14) == 0 && make_divu(15).div(15) == 1, "divide by 15 at the step");
static_assert(make_divu(9).div(8) == 0 && make_divu(9).div(9) == 1 && make_divu(9).div(2147483646) == 2147483646 / 9,
              "divide by 9");
static_assert(make_divu(1 << 20).div(2147483647) == 2047, "divide by a power of two");
static_assert(make_divu(2147483647).div(2147483646) == 0 && make_divu(2147483647).div(2147483647) == 1,
              "divide by the largest divisor");
static_assert(make_divu(1000003).div(1000003 * 2147 - 1) == 2146, "divide by a large prime");

}  // namespace me
