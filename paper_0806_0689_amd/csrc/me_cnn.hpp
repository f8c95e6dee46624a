// Kernels of the learned start proposer: a 4-layer convolutional network on a
// 4x-downsampled current/reference pair, bf16 storage, fp32 accumulation.
// This network is not part of the paper's method; its output only chooses
// where DCDS starts.
//
// Tensors are NHWC bf16 (raw uint16).  Internally the first layer reads 4
// input channels (the last two are zero) and the head writes 4 channels (the
// last is zero), so that every 4 consecutive reduction indices (tap, channel)
// of a convolution are one 8-byte load.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16 (one wave per
// 16x16 output tile).  Lane l holds A[l%16][4(l/16)+i] and B[4(l/16)+i][l%16],
// and receives D[4(l/16)+i][l%16], i = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {
namespace cnn {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct LayerDim {
    int cin, cout, stride;
    bool relu;
};
// Internal layer shapes (first input and last output padded to 4 channels).
constexpr LayerDim kLayers[4] = {{4, 16, 1, true}, {16, 32, 2, true}, {32, 32, 2, true}, {32, 4, 1, false}};
// Exposed (trained) shapes: 2 input channels, 3 head channels.
constexpr int kExposedCin[4] = {2, 16, 32, 32};
constexpr int kExposedCout[4] = {16, 32, 32, 3};

__host__ __device__ constexpr int pad16(int v) { return (v + 15) / 16 * 16; }

__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ v4s as_v4s(uint2 v) {
    v4s r;
    r[0] = (short)(v.x & 0xFFFFu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFFu);
    r[3] = (short)(v.y >> 16);
    return r;
}

// ---------------------------------------------------------------------------
// Input: 4x4 box means of cur and ref -> [(c - r) / 32, (c - 128) / 64, 0, 0].
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
    uint2 out;
    out.x = (uint32_t)a | ((uint32_t)b << 16);
    out.y = 0u;
    *reinterpret_cast<uint2*>(x0 + (((long long)p * H4 + y) * W4 + x) * 4) = out;
}

// ---------------------------------------------------------------------------
// Forward convolution: out[p][oy][ox][co] = bias[co] + sum_{tap, ci}
//   in[p][oy*S + ky - 1][ox*S + kx - 1][ci] * W[tap][ci][co]    (tap = 3 ky + kx)
// GEMM M = 16 output pixels of one row, N = COUT, K = 9 CIN (k = tap*CIN + ci).
// Wf: [COUT][KP] bf16, KP = pad16(9 CIN), zero beyond 9 CIN.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, int S, bool RELU, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t* __restrict__ in, const uint16_t* __restrict__ Wf,
                                                  const float* __restrict__ bias, void* __restrict__ out, int Hi,
                                                  int Wi, int Ho, int Wo) {
    constexpr int KP = pad16(9 * CIN);
    constexpr int NT = (COUT + 15) / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int seg = blockIdx.x * 4 + wave;
    const int oy = blockIdx.y, p = blockIdx.z;
    if (seg * 16 >= Wo) return;
    const int m = lane & 15, kq = lane >> 4;
    const int ox = seg * 16 + m;
    v4f acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const uint16_t* inp = in + (long long)p * Hi * Wi * CIN;
#pragma unroll 2
    for (int ks = 0; ks < KP / 16; ++ks) {
        const int k = ks * 16 + 4 * kq;
        const int tap = k / CIN, ci = k % CIN;
        uint2 av = make_uint2(0u, 0u);
        if (tap < 9 && ox < Wo) {
            const int iy = oy * S + tap / 3 - 1, ix = ox * S + tap % 3 - 1;
            if (iy >= 0 && iy < Hi && ix >= 0 && ix < Wi)
                av = *reinterpret_cast<const uint2*>(inp + ((long long)iy * Wi + ix) * CIN + ci);
        }
        const v4s a = as_v4s(av);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = t * 16 + m;
            uint2 bv = make_uint2(0u, 0u);
            if (n < COUT) bv = *reinterpret_cast<const uint2*>(Wf + (long long)n * KP + k);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, as_v4s(bv), acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = t * 16 + m;
        if (n >= COUT) continue;
        const float bn = bias[n];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int x = seg * 16 + 4 * kq + i;
            if (x >= Wo) continue;
            float v = acc[t][i] + bn;
            if (RELU) v = fmaxf(v, 0.f);
            const long long o = (((long long)p * Ho + oy) * Wo + x) * COUT + n;
            if (F32OUT) reinterpret_cast<float*>(out)[o] = v;
            else reinterpret_cast<uint16_t*>(out)[o] = f2bf(v);
        }
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
// forward Wf[co][tap*CIN + ci] and input-gradient Wb[ci][tap*COUT + co].
__global__ __launch_bounds__(256) void k_pack_weights(const float* __restrict__ W, int cin, int cout,
                                                      uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
    const int kp = pad16(9 * cin), kb = pad16(9 * cout);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < cout * kp) {
        const int co = i / kp, k = i % kp;
        wf[i] = k < 9 * cin ? f2bf(W[(k / cin * cin + k % cin) * cout + co]) : (uint16_t)0;
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

}  // namespace cnn
}  // namespace me
