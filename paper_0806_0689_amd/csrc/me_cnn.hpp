// Kernels of the learned start proposer: a 4-layer convolutional network on a
// 4x-downsampled current/reference pair, bf16 storage, fp32 accumulation.
// This network is not part of the paper's method; its output only chooses
// where DCDS starts.
//
// Tensors are NHWC bf16 (raw uint16).  The head writes 4 channels internally
// (the last is zero).
//
// Forward convolutions (training and the fused inference kernel alike) are
// implicit GEMMs on v_mfma_f32_16x16x32_bf16, one wave per 16x16 output tile:
// lane l holds A[l%16][8(l/16)+i] and B[8(l/16)+i][l%16], i = 0..7, and
// receives D[4(l/16)+i][l%16], i = 0..3.  A lane's 8 reduction indices are
// one 16-byte operand: 8 channels of one tap for layers of 16 or more input
// channels; for the 2-channel input of the first layer the taps of a kernel
// row are paired by column (index (ky 4 + kx) 2 + ci, with a zero column
// kx = 3 and a zero row ky = 3), so that the 8 indices are 4 adjacent pixels
// of one row and the whole reduction is one k-step.  The reduction is padded
// to a multiple of 32 with zero weights.
//
// The backward kernels use v_mfma_f32_16x16x16_bf16 (lane l holds
// A[l%16][4(l/16)+i] and B[4(l/16)+i][l%16], i = 0..3), with reductions
// padded to a multiple of 16.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace me {
namespace cnn {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct LayerDim {
    int cin, cout, stride;
    bool relu;
};
// Internal layer shapes (last output padded to 4 channels).
constexpr LayerDim kLayers[4] = {{2, 16, 1, true}, {16, 32, 2, true}, {32, 32, 2, true}, {32, 4, 1, false}};
// Exposed (trained) shapes: 2 input channels, 3 head channels.
constexpr int kExposedCin[4] = {2, 16, 32, 32};
constexpr int kExposedCout[4] = {16, 32, 32, 3};

__host__ __device__ constexpr int pad16(int v) { return (v + 15) / 16 * 16; }
__host__ __device__ constexpr int pad32(int v) { return (v + 31) / 32 * 32; }
// Reduction length of the forward weights Wf[co][k] of a layer.
__host__ __device__ constexpr int fwd_kp(int cin) { return pad32(9 * cin); }

// Reduction index k of a layer with cin input channels: its tap and channel,
// or tap = -1 for a padding index (zero weight).  cin = 2: the taps of a
// kernel row paired by column, k = (ky 4 + kx) 2 + ci (32 indices, 18 used);
// otherwise k = tap cin + ci.
__host__ __device__ constexpr int ktap(int cin, int k) {
    if (cin == 2) {
        const int ky = k >> 3, kx = (k >> 1) & 3;
        return ky < 3 && kx < 3 ? 3 * ky + kx : -1;
    }
    return k < 9 * cin ? k / cin : -1;
}
__host__ __device__ constexpr int kchan(int cin, int k) { return cin == 2 ? (k & 1) : k % cin; }

// Round to bfloat16, nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ v4s as_v4s(uint2 v) { return __builtin_bit_cast(v4s, v); }
__device__ __forceinline__ v8bf as_v8bf(uint4 v) { return __builtin_bit_cast(v8bf, v); }

// n / D for 0 <= n < N by one 24-bit multiply and a shift, where the
// compiler's division by a constant takes a 32-bit high multiply: the
// multiplier is ceil(2^K / D) for the smallest K exact on every n < N
// (checked here, at compile time, for each n).
template <int D, int N>
struct SmallDiv {
    static constexpr int pick() {
        for (int k = 0; k < 24; ++k) {
            const long long m = ((1LL << k) + D - 1) / D;
            bool ok = (N - 1) * m < (1LL << 24);
            for (int n = 0; ok && n < N; ++n) ok = ((n * m) >> k) == n / D;
            if (ok) return k;
        }
        return -1;
    }
    static constexpr int K = pick();
    static_assert(K >= 0, "no exact 24-bit multiplier");
    static constexpr unsigned MUL = (unsigned)(((1LL << K) + D - 1) / D);
    __device__ static __forceinline__ int div(int n) { return (int)(__umul24((unsigned)n, MUL) >> K); }
};

// max(x, 0) for finite x as one integer max on the bit pattern (negative
// floats, -0 included, are negative integers); fmaxf would first quiet x.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// max(x, 0) of both bfloat16 halves of a packed pair, as signed 16-bit
// integers (negative values, -0 included, have the sign bit set).
typedef short v2s __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf2(uint32_t x) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(v2s, x), (v2s){0, 0}));
}

// Two floats to a packed pair of bfloat16 (low = a), each rounded as f2bf.
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){a, b}, v2bf));
}

// LDS addressing by 32-bit byte address.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(3))) T* lds_ptr(uint32_t a) {
    return (__attribute__((address_space(3))) T*)(uintptr_t)a;
}

// ---------------------------------------------------------------------------
// Input: 4x4 box means of cur and ref -> [(c - r) / 32, (c - 128) / 64].
// One thread per output pixel; rows of 4 pixels are one aligned word.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_downdiff(const uint8_t* __restrict__ cur, const uint8_t* __restrict__ ref,
                                                  int pitch, long long pair_stride, int H4, int W4,
                                                  uint16_t* __restrict__ x0) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y, p = blockIdx.z;
    if (x >= W4) return;
    const uint8_t* c = cur + (long long)p * pair_stride + (size_t)(4 * y) * pitch + 4 * x;
    const uint8_t* r = ref + (long long)p * pair_stride + (size_t)(4 * y) * pitch + 4 * x;
    uint32_t sc = 0, sr = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        sc = __builtin_amdgcn_sad_u8(*reinterpret_cast<const uint32_t*>(c + (size_t)i * pitch), 0u, sc);
        sr = __builtin_amdgcn_sad_u8(*reinterpret_cast<const uint32_t*>(r + (size_t)i * pitch), 0u, sr);
    }
    const float mc = (float)sc * (1.0f / 16.0f), mr = (float)sr * (1.0f / 16.0f);
    const uint16_t a = f2bf((mc - mr) * (1.0f / 32.0f));
    const uint16_t b = f2bf((mc - 128.0f) * (1.0f / 64.0f));
    *reinterpret_cast<uint32_t*>(x0 + (((long long)p * H4 + y) * W4 + x) * 2) = (uint32_t)a | ((uint32_t)b << 16);
}

// ---------------------------------------------------------------------------
// Forward convolution: out[p][oy][ox][co] = bias[co] + sum_{tap, ci}
//   in[p][oy*S + ky - 1][ox*S + kx - 1][ci] * W[tap][ci][co]    (tap = 3 ky + kx),
// accumulated from the bias.
// GEMM M = 16 output pixels of one row, N = COUT, K = 9 CIN in the order of
// ktap/kchan.  Wf: [COUT][KP] bf16, KP = fwd_kp(CIN), zero at padding indices.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int S, bool RELU, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ in, const uint16_t* __restrict__ Wf,
                                                  const float* __restrict__ bias, void* __restrict__ out, int Hi,
                                                  int Wi, int Ho, int Wo) {
    constexpr int KP = fwd_kp(CIN);
    constexpr int NT = (COUT + 15) / 16;
    static_assert(CIN == 2 || CIN % 8 == 0, "8 reduction indices of a lane share one tap");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int seg = blockIdx.x * 4 + wave;
    const int oy = blockIdx.y, p = blockIdx.z;
    if (seg * 16 >= Wo) return;
    const int m = lane & 15, kq = lane >> 4;
    const int ox = seg * 16 + m;
    // The bias is the accumulator's initial value (the fused inference
    // kernel starts from it too, so both round alike).
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][r] = t * 16 + 4 * kq + r < COUT ? bias[t * 16 + 4 * kq + r] : 0.f;
    const uint16_t* inp = in + (long long)p * Hi * Wi * CIN;
#pragma unroll 3
    for (int ks = 0; ks < KP / 32; ++ks) {
        const int k = ks * 32 + 8 * kq;
        uint4 av = make_uint4(0u, 0u, 0u, 0u);
        if constexpr (CIN == 2) {
            // Kernel row ky = kq: the taps kx = 0..2, both channels each (kx = 3
            // and ky = 3 are zero padding).
            const int ky = k >> 3;
            const int iy = oy * S + ky - 1, ix = ox * S - 1;
            if (ky < 3 && ox < Wo && iy >= 0 && iy < Hi) {
                const uint32_t* row = reinterpret_cast<const uint32_t*>(inp + (long long)iy * Wi * 2);
                if (ix >= 0) av.x = row[ix];
                if (ix + 1 < Wi) av.y = row[ix + 1];
                if (ix + 2 < Wi) av.z = row[ix + 2];
            }
        } else {
            const int tap = k / CIN, ci = k % CIN;
            if (tap < 9 && ox < Wo) {
                const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
                if (iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
                    av = *reinterpret_cast<const uint4*>(inp + ((long long)iy * Wi + ix) * CIN + ci);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = t * 16 + m;
            uint4 bv = make_uint4(0u, 0u, 0u, 0u);
            if (n < COUT) bv = *reinterpret_cast<const uint4*>(Wf + (long long)n * KP + k);
            // Weights as the row operand: lane (m, kq) receives channels
            // 16 t + 4 kq .. + 3 of pixel ox.
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_v8bf(bv), as_v8bf(av), acc[t], 0, 0, 0);
        }
    }
    if (ox >= Wo) return;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n0 = t * 16 + 4 * kq;
        if (n0 >= COUT) continue;
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = RELU ? relu(acc[t][r]) : acc[t][r];
        const long long o = (((long long)p * Ho + oy) * Wo + ox) * COUT + n0;
        if (F32OUT) *reinterpret_cast<float4*>(reinterpret_cast<float*>(out) + o) = make_float4(v[0], v[1], v[2], v[3]);
        else *reinterpret_cast<uint2*>(reinterpret_cast<uint16_t*>(out) + o) = make_uint2(pack_bf2(v[0], v[1]), pack_bf2(v[2], v[3]));
    }
}

// ---------------------------------------------------------------------------
// Backward with respect to the input: gin[p][iy][ix][ci] = mask * sum_{tap, co}
//   gout[p][(iy + 1 - ky)/S][(ix + 1 - kx)/S][co] * W[tap][ci][co]
// (terms whose division is not exact or out of range vanish), mask = the
// layer input's ReLU (in > 0).  GEMM M = 16 input pixels of one row, N = CIN,
// K = 9 COUT (k = tap*COUT + co).  Wb: [CIN][KB] bf16, KB = pad16(9 COUT).
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int S>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const uint16_t* __restrict__ gout,
                                                       const uint16_t* __restrict__ Wb,
                                                       const uint16_t* __restrict__ in, uint16_t* __restrict__ gin,
                                                       int Hi, int Wi, int Ho, int Wo) {
    constexpr int KB = pad16(9 * COUT);
    constexpr int NT = (CIN + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int seg = blockIdx.x * 4 + wave;
    const int iy = blockIdx.y, p = blockIdx.z;
    if (seg * 16 >= Wi) return;
    const int m = lane & 15, kq = lane >> 4;
    const int ix = seg * 16 + m;
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const uint16_t* gp = gout + (long long)p * Ho * Wo * COUT;
#pragma unroll 2
    for (int ks = 0; ks < KB / 16; ++ks) {
        const int k = ks * 16 + 4 * kq;
        const int tap = k / COUT, co = k % COUT;
        uint2 av = make_uint2(0u, 0u);
        if (tap < 9 && ix < Wi) {
            const int ty = iy + 1 - tap / 3, tx = ix + 1 - tap % 3;
            if (ty >= 0 && tx >= 0 && ty % S == 0 && tx % S == 0 && ty / S < Ho && tx / S < Wo)
                av = *reinterpret_cast<const uint2*>(gp + ((long long)(ty / S) * Wo + tx / S) * COUT + co);
        }
        const v4s a = as_v4s(av);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = t * 16 + m;
            uint2 bv = make_uint2(0u, 0u);
            if (n < CIN) bv = *reinterpret_cast<const uint2*>(Wb + (long long)n * KB + k);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, as_v4s(bv), acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = t * 16 + m;
        if (n >= CIN) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = seg * 16 + 4 * kq + i;
            if (x >= Wi) continue;
            const long long o = (((long long)p * Hi + iy) * Wi + x) * CIN + n;
            const bool on = (int16_t)in[o] > 0;  // bf16 > +0 (negative zero and negatives excluded)
            gin[o] = on ? f2bf(acc[t][i]) : (uint16_t)0;
        }
    }
}

// ---------------------------------------------------------------------------
// Backward with respect to the weights, over one chunk of CH output pixels
// (flattened over pairs, rows and columns):
//   part[c][(tap*CIN + ci)*COUT + co] = sum_{q in chunk} in[pos(q, tap)][ci] * gout[q][co]
//   part[c][9 CIN COUT + co]          = sum_{q in chunk} gout[q][co]
// GEMM M = 9 CIN, N = COUT, K = pixels.  Chunks are summed afterwards in a
// fixed order (k_sum_chunks), so results do not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int kChunk = 256;

template <int CIN, int COUT, int S>
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const uint16_t* __restrict__ in,
                                                         const uint16_t* __restrict__ gout, float* __restrict__ part,
                                                         int Hi, int Wi, int Ho, int Wo, long long total) {
    constexpr int M = 9 * CIN, MT = (M + 15) / 16, NT = (COUT + 15) / 16, LEN = M * COUT + COUT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const long long q0 = (long long)blockIdx.x * kChunk;
    float* dst = part + (long long)blockIdx.x * LEN;
    const long long hw = (long long)Ho * Wo;
    for (int tile = wave; tile < MT * NT; tile += 4) {
        const int mt = tile / NT, nt = tile % NT;
        const int row = mt * 16 + m;  // (tap, ci) of this lane's A row
        const int tap = row / CIN, ci = row % CIN;
        const int n = nt * 16 + m;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        for (int ks = 0; ks < kChunk / 16; ++ks) {
            v4s a, b;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long q = q0 + ks * 16 + 4 * kq + i;
                uint16_t av = 0, bv = 0;
                if (q < total) {
                    const int p = (int)(q / hw);
                    const int r = (int)(q - (long long)p * hw);
                    const int oy = r / Wo, ox = r - oy * Wo;
                    if (row < M) {
                        const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
                        if (iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
                            av = in[(((long long)p * Hi + iy) * Wi + ix) * CIN + ci];
                    }
                    if (n < COUT) bv = gout[q * COUT + n];
                }
                a[i] = (short)av;
                b[i] = (short)bv;
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int mr = mt * 16 + 4 * kq + i;
            if (mr < M && n < COUT) dst[mr * COUT + n] = acc[i];
        }
    }
    if (threadIdx.x < COUT) {
        float s = 0.f;
        for (int i = 0; i < kChunk; ++i) {
            const long long q = q0 + i;
            if (q < total) s += bf2f(gout[q * COUT + threadIdx.x]);
        }
        dst[M * COUT + threadIdx.x] = s;
    }
}

// out[i] = sum_c part[c][i], in chunk order.
__global__ __launch_bounds__(256) void k_sum_chunks(const float* __restrict__ part, int nchunk, int len,
                                                    float* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
    for (int c = 0; c < nchunk; ++c) s += part[(long long)c * len + i];
    out[i] = s;
}

// ---------------------------------------------------------------------------
// Loss over n blocks: huber(u - tx) + huber(v - ty) + 0.25 bce(o, |ty| > |tx|),
// t = target / 8, mean over blocks.  Writes the head gradient (bf16, 4
// channels, the last zero) and one partial loss sum per workgroup.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_head_loss(const float* __restrict__ head, const int16_t* __restrict__ target,
                                                   int n, uint16_t* __restrict__ ghead, float* __restrict__ loss_part) {
    __shared__ float red[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const float inv = 1.0f / (float)n;
        const float tx = (float)target[2 * i] * 0.125f, ty = (float)target[2 * i + 1] * 0.125f;
        const float du = head[4 * i] - tx, dv = head[4 * i + 1] - ty, o = head[4 * i + 2];
        const float au = fabsf(du), av = fabsf(dv);
        l = (au <= 1.f ? 0.5f * du * du : au - 0.5f) + (av <= 1.f ? 0.5f * dv * dv : av - 0.5f);
        const float lab = fabsf(ty) > fabsf(tx) ? 1.f : 0.f;
        const float sp = fmaxf(o, 0.f) + log1pf(expf(-fabsf(o)));
        l += 0.25f * (sp - lab * o);
        const float sig = 1.f / (1.f + expf(-o));
        uint2 g;
        g.x = (uint32_t)f2bf(fminf(fmaxf(du, -1.f), 1.f) * inv) |
              ((uint32_t)f2bf(fminf(fmaxf(dv, -1.f), 1.f) * inv) << 16);
        g.y = (uint32_t)f2bf(0.25f * (sig - lab) * inv);
        *reinterpret_cast<uint2*>(ghead + 4 * i) = g;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Head gradient given by the caller (fp32, 3 channels) -> bf16, 4 channels.
__global__ __launch_bounds__(256) void k_pack_ghead(const float* __restrict__ dhead, int n, uint16_t* __restrict__ g) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint2 v;
    v.x = (uint32_t)f2bf(dhead[3 * i]) | ((uint32_t)f2bf(dhead[3 * i + 1]) << 16);
    v.y = (uint32_t)f2bf(dhead[3 * i + 2]);
    *reinterpret_cast<uint2*>(g + 4 * i) = v;
}

// Deterministic total of the loss partials, divided by the block count.
__global__ void k_loss_total(const float* __restrict__ part, int nparts, int n, float* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    float s = 0.f;
    for (int i = 0; i < nparts; ++i) s += part[i];
    loss[0] = s / (float)n;
}

// Adam on fp32 master parameters (bias-corrected).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 operand layouts of one layer from its fp32 master W[tap][ci][co]:
// forward Wf[co][k] (k in the order of ktap/kchan) and input-gradient
// Wb[ci][tap*COUT + co].
__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ W, int cin, int cout,
                                                      uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
    const int kp = fwd_kp(cin), kb = pad16(9 * cout);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < cout * kp) {
        const int co = i / kp, k = i % kp;
        const int tap = ktap(cin, k);
        wf[i] = tap >= 0 ? f2bf(W[(tap * cin + kchan(cin, k)) * cout + co]) : (uint16_t)0;
    }
    if (wb && i < cin * kb) {
        const int ci = i / kb, k = i % kb;
        wb[i] = k < 9 * cout ? f2bf(W[((k / cout) * cin + ci) * cout + k % cout]) : (uint16_t)0;
    }
}

// Start vectors and orientations from the head: s = clamp(rint(8 (u, v)), -R, R),
// vertical when o > 0.
__global__ __launch_bounds__(256) void k_head_decode(const float* __restrict__ head, int n, int R,
                                                     int16_t* __restrict__ start, uint8_t* __restrict__ orient) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float u = rintf(head[4 * i] * 8.f), v = rintf(head[4 * i + 1] * 8.f);
    start[2 * i] = (int16_t)fminf(fmaxf(u, (float)-R), (float)R);
    start[2 * i + 1] = (int16_t)fminf(fmaxf(v, (float)-R), (float)R);
    orient[i] = head[4 * i + 2] > 0.f ? 1 : 0;
}

// Head [n][4] (internal) -> [n][3] for callers.
__global__ __launch_bounds__(256) void k_head_export(const float* __restrict__ head, int n, float* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    out[3 * i] = head[4 * i];
    out[3 * i + 1] = head[4 * i + 1];
    out[3 * i + 2] = head[4 * i + 2];
}


// ---------------------------------------------------------------------------
// Fused inference: all four layers for a tile of kTB x kTB blocks, with every
// activation in LDS, then the start-vector decode.  Each output takes exactly
// the operands and the k-step order of k_downdiff + k_conv_fwd + k_head_decode
// (same bf16 values, same 32-wide MFMA k-steps in the same order, zero padding
// outside each layer's image), so the two paths give identical results.
//
// Tile sides (with the halo each 3x3 layer needs): L3 kN3 = kTB + 2, L2
// kN2 = 2 kN3 + 1, L1 kN1 = 2 kN2 + 1, input kN0 = kN1 + 2.  Persistent: one
// workgroup per CU stages the weights once and walks the tiles.
//
// LDS layouts are chosen so that the 16 lanes reading one operand row read
// 16 consecutive 16-byte words (one ds_read_b128 each, free of bank
// conflicts):
// - activations (Planar): 8 channels of a pixel are one 16-byte slot; the
//   channel groups are separate planes; and where the next layer reads with
//   stride 2 each row keeps its even columns first, so that one tap of 16
//   consecutive stride-2 outputs is 16 consecutive slots;
// - weights: the 16-byte chunk (k-step, lane group, output channel), output
//   channel fastest.
// The 2-channel input tile is one dword per pixel.
// ---------------------------------------------------------------------------
constexpr int kTB = 8;
constexpr int kN3 = kTB + 2, kN2 = 2 * kN3 + 1, kN1 = 2 * kN2 + 1, kN0 = kN1 + 2;

template <int N, int C, bool SPLIT>
struct Planar {
    static_assert(C % 8 == 0, "whole 16-byte slots");
    static constexpr int kEven = (N + 1) / 2;                // even columns per row
    static constexpr int kPlane = (N * N + 15) / 16 * 16;    // plane stride in slots (a 256-byte multiple)
    static constexpr int kBytes = 16 * (C / 8) * kPlane;
    __host__ __device__ static constexpr int col(int x) { return SPLIT ? ((x & 1) ? kEven + (x >> 1) : (x >> 1)) : x; }
    // The column stored at position c of a row (the inverse of col).
    __host__ __device__ static constexpr int xof(int c) { return SPLIT ? 2 * c - (c < kEven ? 0 : 2 * kEven - 1) : c; }
};
typedef Planar<kN1, 16, true> L1Tile;   // L1 output, read by L2 (stride 2)
typedef Planar<kN2, 32, true> L2Tile;   // L2 output, read by L3 (stride 2)
typedef Planar<kN3, 32, false> L3Tile;  // L3 output, read by the head (stride 1)
typedef Planar<kTB, 8, false> HeadTile;  // head output: 4 fp32 channels per pixel
constexpr int kIn0Bytes = 4 * (kN0 * kN0 + 1);  // input tile and the pixel after it
static_assert(kIn0Bytes <= L2Tile::kBytes, "the input tile lives in layer 2's buffer");

// Weights in LDS: layer l as 16-byte chunks [KS][4][COUT].
__host__ __device__ constexpr int wbytes(int l) { return fwd_kp(kLayers[l].cin) / 8 * 16 * kLayers[l].cout; }
constexpr int kWOff1 = wbytes(0), kWOff2 = kWOff1 + wbytes(1), kWOff3 = kWOff2 + wbytes(2), kWAll = kWOff3 + wbytes(3);
constexpr int kBias = 16 + 32 + 32 + 4;
// LDS (bytes): l1, l2 (also the input tile), l3, the weights, the fp32 head
// and the biases.
constexpr int kOffL2 = L1Tile::kBytes, kOffL3 = kOffL2 + L2Tile::kBytes, kOffW = kOffL3 + L3Tile::kBytes;
constexpr int kOffHead = kOffW + kWAll, kOffBias = kOffHead + 4 * 4 * kTB * kTB;
// A 16-byte slot per lane that stores with nothing to store go to (instead of
// branching around them).
constexpr int kOffDummy = (kOffBias + 4 * kBias + 15) / 16 * 16;
constexpr size_t kFusedLds = (size_t)kOffDummy + 16 * 64;
constexpr int kFusedThreads = 1024;
static_assert(kOffL2 % 16 == 0 && kOffL3 % 16 == 0 && kOffW % 16 == 0 && kOffHead % 16 == 0,
              "16-byte aligned buffers");
static_assert(kFusedLds <= 160 * 1024, "one workgroup's LDS");

// One 3x3 layer from an LDS tile to an LDS tile (or, for the head, to the
// head buffer: fp32, 4 channels, 16 bytes per pixel).  LI/LO: input/output
// layouts (LI unused for the 2-channel input: one dword per pixel, side NI);
// NO: output tile side; wb: this layer's weight chunks; dummy: 16 bytes per lane
// for stores with nothing to store; (oy0, ox0): output
// tile origin in its layer's grid of Ho x Wo (outputs outside are written as
// 0, the next layer's padding).  The weights are the MFMA row operand and 16
// output pixels the column operand, so lane (m, kq) receives channels
// 16 t + 4 kq .. + 3 of pixel m and stores them as one 8-byte word.
//
// Output pixels are numbered in the output layout's stored order (so a
// lane's store address is its index times 16 plus a lane constant) and cut
// into PARTS bands of HR rows: an M-tile of the first band and the M-tiles
// HR rows below it in the other bands are computed together, at constant
// offsets from the first one's addresses.  Rows past the layer (in the last
// band) read inside LDS and are not stored.
template <int CIN, int COUT, int S, int NI, class LI, int NO, class LO, int PARTS, bool RELU, bool HEAD>
__device__ __forceinline__ void conv_tile(uint32_t ib, uint32_t ob, uint32_t wb, const float* bias, int oy0, int ox0,
                                          int Ho, int Wo, uint32_t dummy) {
    constexpr int KP = fwd_kp(CIN);
    constexpr int KS = KP / 32;
    constexpr int NT = (COUT + 15) / 16;
    constexpr int M = NO * NO;
    constexpr int HR = (NO + PARTS - 1) / PARTS, MB = HR * NO;
    // Weights stay in registers across a wave's M-tiles when it has more
    // than one; otherwise each k-step reads its own.
    constexpr bool kCache = MB > 16 * (kFusedThreads / 64);
    // k-steps whose operand reads are issued together (register budget:
    // 4 VGPRs per B operand and band, 4 NT more per k-step without cached
    // weights).
    constexpr int CMAX = kCache ? (PARTS == 1 ? 9 : 4) : (PARTS == 1 ? 5 : 3);
    constexpr int CH = KS < CMAX ? KS : CMAX;
    constexpr uint32_t kPix = CIN == 2 ? 4u : 16u;  // input bytes per pixel (per plane)
    constexpr uint32_t kInBand = kPix * (uint32_t)(S * HR * NI), kOutBand = 16u * (uint32_t)MB;
    static_assert(CIN == 2 || CIN % 8 == 0, "8 reduction indices of a lane share one tap");
    static_assert(CIN == 2 || S == 1 || (S == 2 && LI::col(2) == 1), "stride-2 inputs split even and odd columns");
    static_assert(!HEAD || (COUT == 4 && LO::kPlane >= M), "head: one 16-byte fp32 word per pixel");
    const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave * 16 >= MB) return;  // no output tile for this wave: skip the weight reads
    const int m = lane & 15, kq = lane >> 4;
    auto weights = [&](int ks, int t) {
        const int n = t * 16 + m;
        v4u bv = v4u{0u, 0u, 0u, 0u};
        if (n < COUT) bv = *lds_ptr<const v4u>(wb + 16u * (uint32_t)((ks * 4 + kq) * COUT + n));
        return __builtin_bit_cast(v8bf, bv);
    };
    v8bf w[kCache ? KS : 1][NT];
    // Operand byte offset of k-step ks: the tap and channel group of the
    // lane's 8 indices; with CIN = 2 the pixels (ky, 0..3) of kernel row
    // ky = kq.  A padding index reads the pixel itself (ky = 3, or a padding
    // tap), or the pixel right of the window (kx = 3: one pixel past a tile
    // row or, at the last one, past the tile, which is kept finite): finite
    // data against zero weights adds exact zeros.
    uint32_t aoff[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        if constexpr (CIN == 2) {
            aoff[ks] = 4u * (uint32_t)(kq < 3 ? kq * NI : 0);
        } else {
            const int k = 32 * ks + 8 * kq, tap = k / CIN < 9 ? k / CIN : 0, plane = k % CIN / 8;
            const int kx = tap % 3;
            // Column of tap kx relative to the output's first one.
            const int cx = S == 2 ? (kx == 0 ? 0 : kx == 1 ? LI::kEven : 1) : kx;
            aoff[ks] = 16u * (uint32_t)(plane * LI::kPlane + (tap / 3) * NI + cx);
        }
        if constexpr (kCache)
#pragma unroll
            for (int t = 0; t < NT; ++t) w[ks][t] = weights(ks, t);
    }
    // The bias is each accumulator's initial value.
    v4f bn[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) bn[t][r] = t * 16 + 4 * kq + r < COUT ? bias[t * 16 + 4 * kq + r] : 0.f;
    // Store address of the lane's channels 4 kq .. + 3 (t = 0) for stored
    // index 0: plane kq / 2, half kq & 1 of the slot.
    const uint32_t obl = HEAD ? ob : ob + 16u * (uint32_t)((kq >> 1) * LO::kPlane) + 8u * (uint32_t)(kq & 1);
    const bool interior = oy0 >= 0 && ox0 >= 0 && oy0 + NO <= Ho && ox0 + NO <= Wo;
    // The M-tile loop, with the test for outputs outside the layer's grid only
    // where a tile reaches past it (BORDER; uniform per tile).
    auto run = [&](auto border) {
        constexpr bool BORDER = decltype(border)::value;
        for (int tile = wave; tile * 16 < MB; tile += nw) {
            // This lane's output pixel in band 0 (stored index po: row ay,
            // stored column sc, column ax); past the band it takes the last
            // pixel and stores nothing.
            const int po = tile * 16 + m;
            const int pa = min(po, MB - 1);
            const int ay = SmallDiv<NO, MB>::div(pa), sc = pa - __mul24(ay, NO);
            const int ax = LO::xof(sc);
            // The output's first input pixel: (S ay, S ax), at column ax of a
            // split row (even columns first) when S = 2.
            const uint32_t ab = ib + kPix * (uint32_t)(S * ay * NI + ax);
            v4f acc[PARTS][NT];
#pragma unroll
            for (int r = 0; r < PARTS; ++r)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[r][t] = bn[t];
            // The k-steps in chunks of CH: every operand read of a chunk is
            // issued before its MFMA chain starts (a scheduling barrier keeps
            // the reads from sinking to their uses), so the reads' latencies
            // overlap instead of adding up.
#pragma unroll
            for (int k0 = 0; k0 < KS; k0 += CH) {
                v8bf a[PARTS][CH];
                v8bf wk[kCache ? 1 : CH][NT];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int ks = k0 + c;
                    if (ks >= KS) break;
#pragma unroll
                    for (int r = 0; r < PARTS; ++r) {
                        const uint32_t ad = ab + aoff[ks] + (uint32_t)r * kInBand;
                        if constexpr (CIN == 2) {
                            // 4 pixels at a 4-byte boundary: dword reads (two
                            // ds_read2_b32); wider reads off their alignment
                            // are much slower.
                            const __attribute__((address_space(3))) uint32_t* q = lds_ptr<const uint32_t>(ad);
                            a[r][c] = __builtin_bit_cast(v8bf, v4u{q[0], q[1], q[2], q[3]});
                        } else {
                            a[r][c] = __builtin_bit_cast(v8bf, *lds_ptr<const v4u>(ad));
                        }
                    }
                    if constexpr (!kCache)
#pragma unroll
                        for (int t = 0; t < NT; ++t) wk[c][t] = weights(ks, t);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int ks = k0 + c;
                    if (ks >= KS) break;
#pragma unroll
                    for (int r = 0; r < PARTS; ++r)
#pragma unroll
                        for (int t = 0; t < NT; ++t)
                            acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                kCache ? w[kCache ? ks : 0][t] : wk[kCache ? 0 : c][t], a[r][c], acc[r][t], 0, 0, 0);
                }
            }
            // A lane past its band, past the layer or without channels stores
            // into its dummy slot instead of branching around the store.
            const uint32_t dl = dummy + 16u * (uint32_t)lane;
#pragma unroll
            for (int r = 0; r < PARTS; ++r) {
                const bool vr = po < MB && (r == 0 || po + r * MB < M);
                // Outputs outside the layer's grid are the next layer's zero padding.
                bool inside = true;
                if constexpr (BORDER)
                    inside = oy0 + ay + r * HR >= 0 && oy0 + ay + r * HR < Ho && ox0 + ax >= 0 && ox0 + ax < Wo;
                const uint32_t od = obl + 16u * (uint32_t)po + (uint32_t)r * kOutBand;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const bool vt = vr && 16 * t + 4 * kq < COUT;
                    if constexpr (HEAD) {
                        *lds_ptr<v4f>(vt ? od : dl) = acc[r][t];
                    } else {
                        // ReLU on the packed bf16 pair: one signed 16-bit max
                        // each (a negative value, -0 included, has its sign bit
                        // set), the same values as ReLU before the rounding.
                        v2u o = v2u{pack_bf2(acc[r][t][0], acc[r][t][1]), pack_bf2(acc[r][t][2], acc[r][t][3])};
                        if (RELU) {
                            o.x = relu_bf2(o.x);
                            o.y = relu_bf2(o.y);
                        }
                        if (BORDER && !inside) o = v2u{0u, 0u};
                        // Channels 16 t + 4 kq .. + 3: plane 2 t + kq / 2.
                        *lds_ptr<v2u>(vt ? od + 32u * (uint32_t)(t * LO::kPlane) : dl) = o;
                    }
                }
            }
        }
    };
    if (HEAD || interior) run(std::false_type{});
    else run(std::true_type{});
}

// The input tile (4x4 box means of cur and ref, as k_downdiff; 0 outside).
// A work item is 4 adjacent input pixels of one row: 16 bytes of each of 4
// source rows in each frame.  The tile origin and the input grid's width are
// multiples of 4 pixels, so the 4 pixels are all inside the frame or all
// outside; outside items read a clamped in-frame address and use zeros, so
// every load of an item is issued before any is used.  Rows are 4-byte
// aligned, which is all a 16-byte global load (u32x4a4: one dwordx4) needs.
typedef uint32_t u32x4a4 __attribute__((ext_vector_type(4), aligned(4)));
constexpr int kInG = (kN0 + 3) / 4;  // items per row; the last holds kN0 - 4 (kInG - 1) tile pixels
constexpr int kInItems = kN0 * kInG;

__device__ __forceinline__ void input_item(int it, const uint8_t* cp, const uint8_t* rp, int pitch, int y0, int x0,
                                           int H4, int W4, uint32_t (&o)[4]) {
    const int i = it / kInG, q = it - (it / kInG) * kInG;
    const int gy = y0 + i, gx = x0 + 4 * q;
    const bool in = gy >= 0 && gy < H4 && gx >= 0 && gx < W4;
    const int cy = min(max(gy, 0), H4 - 1), cx = min(max(gx, 0), W4 - 4);
    const size_t off = (size_t)(4 * cy) * pitch + 4 * cx;
    u32x4a4 c[4], r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const size_t a = off + (size_t)j * pitch;
        c[j] = *reinterpret_cast<const u32x4a4*>(cp + a);
        r[j] = *reinterpret_cast<const u32x4a4*>(rp + a);
    }
    uint32_t sc[4] = {0u, 0u, 0u, 0u}, sr[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        sc[0] = __builtin_amdgcn_sad_u8(c[j].x, 0u, sc[0]);
        sc[1] = __builtin_amdgcn_sad_u8(c[j].y, 0u, sc[1]);
        sc[2] = __builtin_amdgcn_sad_u8(c[j].z, 0u, sc[2]);
        sc[3] = __builtin_amdgcn_sad_u8(c[j].w, 0u, sc[3]);
        sr[0] = __builtin_amdgcn_sad_u8(r[j].x, 0u, sr[0]);
        sr[1] = __builtin_amdgcn_sad_u8(r[j].y, 0u, sr[1]);
        sr[2] = __builtin_amdgcn_sad_u8(r[j].z, 0u, sr[2]);
        sr[3] = __builtin_amdgcn_sad_u8(r[j].w, 0u, sr[3]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const float mc = (float)sc[u] * (1.0f / 16.0f), mr = (float)sr[u] * (1.0f / 16.0f);
        o[u] = in ? (uint32_t)f2bf((mc - mr) * (1.0f / 32.0f)) | ((uint32_t)f2bf((mc - 128.0f) * (1.0f / 64.0f)) << 16)
                  : 0u;
    }
}

__device__ __forceinline__ void input_store(uint32_t* x, int it, const uint32_t (&o)[4]) {
    const int i = it / kInG, q = it - (it / kInG) * kInG;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (4 * q + u < kN0) x[i * kN0 + 4 * q + u] = o[u];
}

// Layer 3's M-tiles take waves [0, kW3); the rest load the next tile's input
// meanwhile.
constexpr int kW3 = (kN3 * kN3 + 15) / 16;
static_assert((kFusedThreads / 64 - kW3) * 64 >= kInItems, "input prefetch needs one item per idle lane");
// L2 warming of the next tile's source rows: 3 dwords per raw row of each
// frame (4 kN0 raw rows of 4 kN0 bytes; 128-byte lines).
// One per thread (register budget): the touches past the thread count, the
// last rows of the reference frame, are left out.
constexpr int kWarm = 2 * 4 * kN0 * 3;
constexpr int kWarmPer = 1;
static_assert(4 * kN0 <= 176 + 4 && 4 * kN0 > 128, "bytes 0, 128 and 176 reach every line of a raw row");

// grid: min(tiles, CUs) workgroups of kFusedThreads threads, kFusedLds bytes.
// wf/bias: the packed layer weights ([COUT][KP], KP = fwd_kp(CIN)) and biases.
//
// Per tile: L1 (input -> l1), L2 (l1 -> l2), then L3 (l2 -> l3) while the
// idle waves fetch and reduce the next tile's input, then the head (l3 ->
// head) while they store it into l2's buffer, whose last reader was L3.
__global__ __launch_bounds__(kFusedThreads) void k_proposer_infer(
    const uint8_t* __restrict__ cur, const uint8_t* __restrict__ ref, int pitch, long long pair_stride, int Hb, int Wb,
    int n_pairs, const uint16_t* __restrict__ wf0, const uint16_t* __restrict__ wf1,
    const uint16_t* __restrict__ wf2, const uint16_t* __restrict__ wf3, const float* __restrict__ b0,
    const float* __restrict__ b1, const float* __restrict__ b2, const float* __restrict__ b3, int R,
    int16_t* __restrict__ start, uint8_t* __restrict__ orient) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    uint32_t* x0 = reinterpret_cast<uint32_t*>(lds + kOffL2);  // the input tile, in layer 2's buffer
    float* head = reinterpret_cast<float*>(lds + kOffHead);
    float* bl = reinterpret_cast<float*>(lds + kOffBias);
    const uint32_t a1 = lds_addr(lds), a2 = a1 + kOffL2, a3 = a1 + kOffL3, aw = a1 + kOffW, ah = a1 + kOffHead,
                   ad = a1 + kOffDummy;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Weights and biases, once.  Chunk c of row n of layer l (indices
    // 8c .. 8c + 7 of W[n][.], 16 bytes) goes to the layer's LDS chunk
    // c COUT + n.  The loads are issued here, the stores after the first
    // input tile's loads (below), so that all of them are in flight together.
    constexpr int kC0 = fwd_kp(kLayers[0].cin) / 8, kC1 = fwd_kp(kLayers[1].cin) / 8,
                  kC2 = fwd_kp(kLayers[2].cin) / 8, kC3 = fwd_kp(kLayers[3].cin) / 8;
    constexpr int kE0 = kLayers[0].cout * kC0, kE1 = kE0 + kLayers[1].cout * kC1, kE2 = kE1 + kLayers[2].cout * kC2,
                  kE3 = kE2 + kLayers[3].cout * kC3;
    constexpr int kPer = (kE3 + kFusedThreads - 1) / kFusedThreads;
    v4u wq[kPer];
    uint32_t wdst[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int i = (int)threadIdx.x + j * kFusedThreads;
        wdst[j] = 0xFFFFFFFFu;
        if (i >= kE3) continue;
        const int l = i < kE0 ? 0 : i < kE1 ? 1 : i < kE2 ? 2 : 3;
        const int r = i - (l == 0 ? 0 : l == 1 ? kE0 : l == 2 ? kE1 : kE2);
        const int cpr = l == 0 ? kC0 : l == 1 ? kC1 : l == 2 ? kC2 : kC3;
        const int rows = l == 0 ? kLayers[0].cout : l == 1 ? kLayers[1].cout : l == 2 ? kLayers[2].cout
                                                                                      : kLayers[3].cout;
        const int n = r / cpr, c = r - n * cpr;
        const uint16_t* src = l == 0 ? wf0 : l == 1 ? wf1 : l == 2 ? wf2 : wf3;
        wq[j] = *reinterpret_cast<const v4u*>(src + (size_t)(n * cpr + c) * 8);
        const int woff = l == 0 ? 0 : l == 1 ? kWOff1 : l == 2 ? kWOff2 : kWOff3;
        wdst[j] = aw + (uint32_t)woff + 16u * (uint32_t)(c * rows + n);
    }
    const int H4 = 4 * Hb, W4 = 4 * Wb, H8 = 2 * Hb, W8 = 2 * Wb;
    const int tx = (Wb + kTB - 1) / kTB, ty = (Hb + kTB - 1) / kTB;
    const int total = tx * ty * n_pairs;
    // Tile order: blocks are dealt to the 8 XCDs round-robin, so when the
    // grid is a multiple of 8 the workgroups of one XCD take one contiguous
    // eighth of the tiles, side by side, and a tile's halo has mostly been
    // read through the same L2 by its neighbour.
    int first = blockIdx.x, step = gridDim.x, end = total;
    if (gridDim.x % 8 == 0) {
        const int x = blockIdx.x % 8;
        first = (int)((long long)total * x / 8) + blockIdx.x / 8;
        end = (int)((long long)total * (x + 1) / 8);
        step = gridDim.x / 8;
    }
    // Tile t: its pair and first block.  Its input tile starts 8 input
    // pixels (the halo of three 3x3 layers, two of stride 2) before the
    // first block's 4 input pixels per block, at (4 by0 - 8, 4 bx0 - 8).
    auto place = [&](int t, int& p, int& by0, int& bx0) {
        p = t / (tx * ty);
        const int r = t - p * (tx * ty);
        bx0 = (r % tx) * kTB;
        by0 = (r / tx) * kTB;
    };
    // The pixel after the input tile (read against zero weights) starts
    // finite; later it holds layer-2 values, finite too.
    if (threadIdx.x == 0) x0[kN0 * kN0] = 0;
    if (first < end) {
        int p, by0, bx0;
        place(first, p, by0, bx0);
        for (int it = threadIdx.x; it < kInItems; it += blockDim.x) {
            uint32_t o[4];
            input_item(it, cur + (long long)p * pair_stride, ref + (long long)p * pair_stride, pitch, 4 * by0 - 8,
                       4 * bx0 - 8, H4, W4, o);
            input_store(x0, it, o);
        }
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j)
        if (wdst[j] != 0xFFFFFFFFu) *lds_ptr<v4u>(wdst[j]) = wq[j];
    for (int i = threadIdx.x; i < kBias; i += blockDim.x)
        bl[i] = i < 16 ? b0[i] : i < 48 ? b1[i - 16] : i < 80 ? b2[i - 48] : b3[i - 80];
    __syncthreads();
    for (int t = first; t < end; t += step) {
        int p, by0, bx0;
        place(t, p, by0, bx0);
        // Tile origins per layer (grid coordinates of local (0, 0)).
        const int y3 = by0 - 1, x3 = bx0 - 1;
        const int y2 = 2 * y3 - 1, x2 = 2 * x3 - 1;
        const int y1 = 2 * y2 - 1, x1 = 2 * x2 - 1;
        // Every earlier global access is complete here (the previous tile's
        // fetch was consumed, its decode stores are the only ones left), so
        // after this wait nothing but the warming loads below is pending, and
        // layer 1 has no reason to wait for them (s_waitcnt vmcnt(0)).
        __builtin_amdgcn_s_waitcnt(0x0F70);
        // Warm the L2 with the next tile's source rows while layers 1 and 2
        // run: one dword at bytes 0, 128 and 176 of each raw row's 180-byte
        // stretch (so every 128-byte line of it), both frames, as far as one
        // per thread goes; the fetch under layer 3 then reads from the L2.
        // The dwords are only held, to keep the loads.
        uint32_t warm[kWarmPer];
        {
            int pn, byn, bxn;
            place(min(t + step, end - 1), pn, byn, bxn);
            const bool next = t + step < end;
#pragma unroll
            for (int k = 0; k < kWarmPer; ++k) {
                const int u = (int)threadIdx.x + k * kFusedThreads;
                warm[k] = 0u;
                if (!next || u >= kWarm) continue;
                const int f = u / (kWarm / 2), rem = u - f * (kWarm / 2);
                const int r = rem / 3, sgm = rem - 3 * r;
                const int cy = min(max(4 * byn - 8 + (r >> 2), 0), H4 - 1);
                const int rx = min(max(16 * bxn - 32 + (sgm == 0 ? 0 : sgm == 1 ? 128 : 176), 0), 4 * W4 - 4);
                const uint8_t* frame = (f ? ref : cur) + (long long)pn * pair_stride;
                warm[k] = *reinterpret_cast<const uint32_t*>(frame + (size_t)(4 * cy + (r & 3)) * pitch + rx);
            }
        }
        conv_tile<2, 16, 1, kN0, L1Tile, kN1, L1Tile, 2, true, false>(a2, a1, aw, bl, y1, x1, H4, W4, ad);
        __syncthreads();
        conv_tile<16, 32, 2, kN1, L1Tile, kN2, L2Tile, 1, true, false>(a1, a2, aw + kWOff1, bl + 16, y2, x2, H8, W8, ad);
        __syncthreads();
        conv_tile<32, 32, 2, kN2, L2Tile, kN3, L3Tile, 1, true, false>(a2, a3, aw + kWOff2, bl + 48, y3, x3, Hb, Wb, ad);
#pragma unroll
        for (int k = 0; k < kWarmPer; ++k) asm volatile("" ::"v"(warm[k]));
        const int it = (int)threadIdx.x - 64 * kW3;
        const bool fetch = wave >= kW3 && t + step < end && it < kInItems;
        uint32_t o[4];
        if (fetch) {
            int pn, byn, bxn;
            place(t + step, pn, byn, bxn);
            input_item(it, cur + (long long)pn * pair_stride, ref + (long long)pn * pair_stride, pitch, 4 * byn - 8,
                       4 * bxn - 8, H4, W4, o);
        }
        __syncthreads();
        // Head over the kTB x kTB blocks: local L3 (1 + i, 1 + j) is block (by0 + i, bx0 + j).
        conv_tile<32, 4, 1, kN3, L3Tile, kTB, HeadTile, 1, false, true>(a3, ah, aw + kWOff3, bl + 80, by0, bx0, Hb, Wb, ad);
        if (fetch) input_store(x0, it, o);
        __syncthreads();
        if (threadIdx.x < kTB * kTB) {
            const int i = threadIdx.x / kTB, j = threadIdx.x % kTB;
            const int by = by0 + i, bx = bx0 + j;
            if (by < Hb && bx < Wb) {
                const float* h = head + threadIdx.x * 4;
                const long long o = ((long long)p * Hb + by) * Wb + bx;
                const float u = rintf(h[0] * 8.f), v = rintf(h[1] * 8.f);
                start[2 * o] = (int16_t)fminf(fmaxf(u, (float)-R), (float)R);
                start[2 * o + 1] = (int16_t)fminf(fmaxf(v, (float)-R), (float)R);
                orient[o] = h[2] > 0.f ? 1 : 0;
            }
        }
    }
}

}  // namespace cnn
}  // namespace me
