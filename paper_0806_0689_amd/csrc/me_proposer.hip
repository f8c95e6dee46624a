// Learned start proposer (me_proposer_*) and DCDS from its proposals
// (me_dcds_learned).  The network and its training are this library's
// addition; the search it seeds is DCDS (§III-B) with the start rule of
// me_dcds_ex.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <random>
#include <vector>

#include "me.h"
#include "me_cnn.hpp"
#include "me_host.hpp"

using namespace me;
using namespace me::host;
using namespace me::cnn;

namespace {

// Parameter offsets in the internal (padded) and exposed flat layouts:
// per layer W[tap][ci][co] then bias[co].
struct Offsets {
    int w[4], b[4], total;
};
Offsets internal_offsets() {
    Offsets o;
    int at = 0;
    for (int l = 0; l < 4; ++l) {
        o.w[l] = at;
        at += 9 * kLayers[l].cin * kLayers[l].cout;
        o.b[l] = at;
        at += kLayers[l].cout;
    }
    o.total = at;
    return o;
}
Offsets exposed_offsets() {
    Offsets o;
    int at = 0;
    for (int l = 0; l < 4; ++l) {
        o.w[l] = at;
        at += 9 * kExposedCin[l] * kExposedCout[l];
        o.b[l] = at;
        at += kExposedCout[l];
    }
    o.total = at;
    return o;
}

// Copies between the exposed and internal layouts (padding entries are 0).
void exposed_to_internal(const float* e, float* in) {
    const Offsets oi = internal_offsets(), oe = exposed_offsets();
    memset(in, 0, sizeof(float) * oi.total);
    for (int l = 0; l < 4; ++l) {
        const int ci_i = kLayers[l].cin, co_i = kLayers[l].cout, ci_e = kExposedCin[l], co_e = kExposedCout[l];
        for (int t = 0; t < 9; ++t)
            for (int ci = 0; ci < ci_e; ++ci)
                for (int co = 0; co < co_e; ++co)
                    in[oi.w[l] + (t * ci_i + ci) * co_i + co] = e[oe.w[l] + (t * ci_e + ci) * co_e + co];
        for (int co = 0; co < co_e; ++co) in[oi.b[l] + co] = e[oe.b[l] + co];
    }
}
void internal_to_exposed(const float* in, float* e) {
    const Offsets oi = internal_offsets(), oe = exposed_offsets();
    for (int l = 0; l < 4; ++l) {
        const int ci_i = kLayers[l].cin, co_i = kLayers[l].cout, ci_e = kExposedCin[l], co_e = kExposedCout[l];
        for (int t = 0; t < 9; ++t)
            for (int ci = 0; ci < ci_e; ++ci)
                for (int co = 0; co < co_e; ++co)
                    e[oe.w[l] + (t * ci_e + ci) * co_e + co] = in[oi.w[l] + (t * ci_i + ci) * co_i + co];
        for (int co = 0; co < co_e; ++co) e[oe.b[l] + co] = in[oi.b[l] + co];
    }
}

template <class T>
int grow(T** p, size_t* cap, size_t n) {
    if (*cap >= n) return ME_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return ME_ENOMEM;
    }
    *cap = n;
    return ME_OK;
}

unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

struct me_proposer {
    int device = -1;
    int n_int = 0;  // internal parameter count
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    long long step = 0;
    uint16_t* wf[4] = {nullptr, nullptr, nullptr, nullptr};
    uint16_t* wb[4] = {nullptr, nullptr, nullptr, nullptr};
    // Activations and gradients of the last forward (capacity in elements).
    uint16_t *x0 = nullptr, *x1 = nullptr, *x2 = nullptr, *x3 = nullptr;
    uint16_t *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *g4 = nullptr;
    size_t cx0 = 0, cx1 = 0, cx2 = 0, cx3 = 0, cg1 = 0, cg2 = 0, cg3 = 0, cg4 = 0;
    float* head = nullptr;
    size_t chead = 0;
    float* part = nullptr;
    size_t cpart = 0;
    float* lpart = nullptr;
    size_t clpart = 0;
    int16_t* start = nullptr;
    size_t cstart = 0;
    uint8_t* orient = nullptr;
    size_t corient = 0;
    int P = 0, H4 = 0, W4 = 0;  // geometry of the last forward
};

namespace {

int pack_all(me_proposer* p, hipStream_t st) {
    const Offsets oi = internal_offsets();
    for (int l = 0; l < 4; ++l) {
        const int ci = kLayers[l].cin, co = kLayers[l].cout;
        const int n = std::max(co * fwd_kp(ci), ci * pad16(9 * co));
        hipLaunchKernelGGL(k_pack_weights, dim3(cdiv(n, 256)), dim3(256), 0, st, p->w + oi.w[l], ci, co, p->wf[l],
                           l > 0 ? p->wb[l] : nullptr);
    }
    return launched();
}

int check_pairs(const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
                int64_t pair_stride, int32_t n_pairs) {
    // The proposer works on 16x16 block grids; its reads are plain frame reads.
    int rc = check_frames(cur, ref, width, height, pitch, pair_stride, n_pairs, 16, 1, cur, cur, cur);
    if (rc != ME_OK) return rc;
    return ME_OK;
}

// Forward pass over n_pairs frame pairs; keeps activations for backward.
int forward(me_proposer* p, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height, int32_t pitch,
            int64_t pair_stride, int32_t n_pairs, hipStream_t st) {
    const int H4 = height / 4, W4 = width / 4, H8 = H4 / 2, W8 = W4 / 2, H16 = H8 / 2, W16 = W8 / 2;
    // The per-layer kernels put rows and pairs on grid dimensions y and z;
    // the weight gradients take one work-item per layer-1 pixel in one
    // dimension (a dispatch counts work-items in 32 bits).
    if (H4 > 65535 || n_pairs > 65535) return ME_EUNSUPPORTED;
    if ((long long)n_pairs * H4 * W4 > (long long)INT32_MAX) return ME_EUNSUPPORTED;
    const long long P = n_pairs;
    int rc = ME_OK;
    if ((rc = grow(&p->x0, &p->cx0, (size_t)(P * H4 * W4 * 2))) ||
        (rc = grow(&p->x1, &p->cx1, (size_t)(P * H4 * W4 * 16))) ||
        (rc = grow(&p->x2, &p->cx2, (size_t)(P * H8 * W8 * 32))) ||
        (rc = grow(&p->x3, &p->cx3, (size_t)(P * H16 * W16 * 32))) ||
        (rc = grow(&p->head, &p->chead, (size_t)(P * H16 * W16 * 4))))
        return rc;
    p->P = n_pairs;
    p->H4 = H4;
    p->W4 = W4;
    const Offsets oi = internal_offsets();
    hipLaunchKernelGGL(k_downdiff, dim3(cdiv(W4, 256), H4, n_pairs), dim3(256), 0, st, cur, ref, pitch, pair_stride,
                       H4, W4, p->x0);
    hipLaunchKernelGGL((k_conv_fwd<2, 16, 1, true, false>), dim3(cdiv(W4, 64), H4, n_pairs), dim3(256), 0, st, p->x0,
                       p->wf[0], p->w + oi.b[0], (void*)p->x1, H4, W4, H4, W4);
    hipLaunchKernelGGL((k_conv_fwd<16, 32, 2, true, false>), dim3(cdiv(W8, 64), H8, n_pairs), dim3(256), 0, st, p->x1,
                       p->wf[1], p->w + oi.b[1], (void*)p->x2, H4, W4, H8, W8);
    hipLaunchKernelGGL((k_conv_fwd<32, 32, 2, true, false>), dim3(cdiv(W16, 64), H16, n_pairs), dim3(256), 0, st,
                       p->x2, p->wf[2], p->w + oi.b[2], (void*)p->x3, H8, W8, H16, W16);
    hipLaunchKernelGGL((k_conv_fwd<32, 4, 1, false, true>), dim3(cdiv(W16, 64), H16, n_pairs), dim3(256), 0, st,
                       p->x3, p->wf[3], p->w + oi.b[3], (void*)p->head, H16, W16, H16, W16);
    return launched();
}

// One layer's weight gradient: chunks, then a fixed-order sum into p->g.
template <int CIN, int COUT, int S>
int weight_grad(me_proposer* p, int layer, const uint16_t* in, const uint16_t* gout, int Hi, int Wi, int Ho, int Wo,
                hipStream_t st) {
    constexpr int LEN = 9 * CIN * COUT + COUT;
    const long long total = (long long)p->P * Ho * Wo;
    const int nchunk = (int)((total + kChunk - 1) / kChunk);
    int rc = grow(&p->part, &p->cpart, (size_t)nchunk * LEN);
    if (rc) return rc;
    hipLaunchKernelGGL((k_conv_bwd_weight<CIN, COUT, S>), dim3(nchunk), dim3(256), 0, st, in, gout, p->part, Hi, Wi, Ho,
                       Wo, total);
    const Offsets oi = internal_offsets();
    // W and bias are adjacent in the internal layout, as in the chunk rows.
    hipLaunchKernelGGL(k_sum_chunks, dim3(cdiv(LEN, 256)), dim3(256), 0, st, p->part, nchunk, LEN, p->g + oi.w[layer]);
    return launched();
}

// Backward from the head gradient in p->g4 to every parameter gradient.
int backward(me_proposer* p, hipStream_t st) {
    const int H4 = p->H4, W4 = p->W4, H8 = H4 / 2, W8 = W4 / 2, H16 = H8 / 2, W16 = W8 / 2;
    const long long P = p->P;
    int rc = ME_OK;
    if ((rc = grow(&p->g1, &p->cg1, (size_t)(P * H4 * W4 * 16))) ||
        (rc = grow(&p->g2, &p->cg2, (size_t)(P * H8 * W8 * 32))) ||
        (rc = grow(&p->g3, &p->cg3, (size_t)(P * H16 * W16 * 32))))
        return rc;
    if ((rc = weight_grad<32, 4, 1>(p, 3, p->x3, p->g4, H16, W16, H16, W16, st))) return rc;
    hipLaunchKernelGGL((k_conv_bwd_data<32, 4, 1>), dim3(cdiv(W16, 64), H16, p->P), dim3(256), 0, st, p->g4, p->wb[3],
                       p->x3, p->g3, H16, W16, H16, W16);
    if ((rc = weight_grad<32, 32, 2>(p, 2, p->x2, p->g3, H8, W8, H16, W16, st))) return rc;
    hipLaunchKernelGGL((k_conv_bwd_data<32, 32, 2>), dim3(cdiv(W8, 64), H8, p->P), dim3(256), 0, st, p->g3, p->wb[2],
                       p->x2, p->g2, H8, W8, H16, W16);
    if ((rc = weight_grad<16, 32, 2>(p, 1, p->x1, p->g2, H4, W4, H8, W8, st))) return rc;
    hipLaunchKernelGGL((k_conv_bwd_data<16, 32, 2>), dim3(cdiv(W4, 64), H4, p->P), dim3(256), 0, st, p->g2, p->wb[1],
                       p->x1, p->g1, H4, W4, H8, W8);
    if ((rc = weight_grad<2, 16, 1>(p, 0, p->x0, p->g1, H4, W4, H4, W4, st))) return rc;
    return launched();
}

int set_device_params(me_proposer* p, const std::vector<float>& internal) {
    if (hipMemcpy(p->w, internal.data(), sizeof(float) * p->n_int, hipMemcpyHostToDevice) != hipSuccess)
        return ME_EDEVICE;
    int rc = pack_all(p, nullptr);
    if (rc) return rc;
    return hipDeviceSynchronize() == hipSuccess ? ME_OK : ME_EDEVICE;
}

}  // namespace

ME_EXPORT int32_t me_proposer_num_params(void) { return exposed_offsets().total; }

ME_EXPORT int me_proposer_create(me_proposer** out) {
    if (!out) return ME_EINVAL;
    *out = nullptr;
    me_proposer* p = new (std::nothrow) me_proposer();
    if (!p) return ME_ENOMEM;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return ME_EDEVICE;
    }
    p->n_int = internal_offsets().total;
    bool ok = hipMalloc(&p->w, sizeof(float) * p->n_int) == hipSuccess &&
              hipMalloc(&p->g, sizeof(float) * p->n_int) == hipSuccess &&
              hipMalloc(&p->m, sizeof(float) * p->n_int) == hipSuccess &&
              hipMalloc(&p->v, sizeof(float) * p->n_int) == hipSuccess;
    for (int l = 0; l < 4 && ok; ++l) {
        const int ci = kLayers[l].cin, co = kLayers[l].cout;
        ok = hipMalloc(&p->wf[l], sizeof(uint16_t) * co * fwd_kp(ci)) == hipSuccess;
        if (ok && l > 0) ok = hipMalloc(&p->wb[l], sizeof(uint16_t) * ci * pad16(9 * co)) == hipSuccess;
    }
    if (ok) ok = hipMemset(p->w, 0, sizeof(float) * p->n_int) == hipSuccess &&
                 hipMemset(p->g, 0, sizeof(float) * p->n_int) == hipSuccess &&
                 hipMemset(p->m, 0, sizeof(float) * p->n_int) == hipSuccess &&
                 hipMemset(p->v, 0, sizeof(float) * p->n_int) == hipSuccess;
    if (ok) ok = pack_all(p, nullptr) == ME_OK && hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        me_proposer_destroy(p);
        return ME_ENOMEM;
    }
    *out = p;
    return ME_OK;
}

ME_EXPORT int me_proposer_destroy(me_proposer* p) {
    if (!p) return ME_OK;
    void* bufs[] = {p->w, p->g, p->m, p->v, p->x0, p->x1, p->x2, p->x3, p->g1, p->g2, p->g3, p->g4,
                    p->head, p->part, p->lpart, p->start, p->orient};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int l = 0; l < 4; ++l) {
        if (p->wf[l]) (void)hipFree(p->wf[l]);
        if (p->wb[l]) (void)hipFree(p->wb[l]);
    }
    delete p;
    return ME_OK;
}

ME_EXPORT int me_proposer_init(me_proposer* p, uint64_t seed) {
    if (!p) return ME_EINVAL;
    // He-normal weights (std sqrt(2 / (9 cin)) over the exposed fan-in), zero biases.
    std::mt19937_64 rng(seed);
    std::vector<float> e(exposed_offsets().total, 0.f);
    const Offsets oe = exposed_offsets();
    for (int l = 0; l < 4; ++l) {
        std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (9.0 * kExposedCin[l])));
        for (int i = oe.w[l]; i < oe.b[l]; ++i) e[i] = (float)nd(rng);
    }
    return me_proposer_set_weights(p, e.data(), (int32_t)e.size());
}

ME_EXPORT int me_proposer_set_weights(me_proposer* p, const float* host, int32_t n) {
    if (!p || !host) return ME_EINVAL;
    if (n != exposed_offsets().total) return ME_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return ME_EINVAL;
    std::vector<float> in(p->n_int);
    exposed_to_internal(host, in.data());
    return set_device_params(p, in);
}

static int get_internal(const float* dev, int n_int, float* host, int32_t n) {
    if (!host || n != exposed_offsets().total) return ME_EINVAL;
    std::vector<float> in(n_int);
    if (hipDeviceSynchronize() != hipSuccess) return ME_EDEVICE;
    if (hipMemcpy(in.data(), dev, sizeof(float) * n_int, hipMemcpyDeviceToHost) != hipSuccess) return ME_EDEVICE;
    internal_to_exposed(in.data(), host);
    return ME_OK;
}

ME_EXPORT int me_proposer_get_weights(me_proposer* p, float* host, int32_t n) {
    if (!p) return ME_EINVAL;
    return get_internal(p->w, p->n_int, host, n);
}

ME_EXPORT int me_proposer_get_grads(me_proposer* p, float* host, int32_t n) {
    if (!p) return ME_EINVAL;
    return get_internal(p->g, p->n_int, host, n);
}

ME_EXPORT int me_proposer_get_state(me_proposer* p, float* m, float* v, int64_t* step, int32_t n) {
    if (!p || !step) return ME_EINVAL;
    int rc = get_internal(p->m, p->n_int, m, n);
    if (rc == ME_OK) rc = get_internal(p->v, p->n_int, v, n);
    *step = p->step;
    return rc;
}

ME_EXPORT int me_proposer_set_state(me_proposer* p, const float* m, const float* v, int64_t step, int32_t n) {
    if (!p || !m || !v || step < 0 || n != exposed_offsets().total) return ME_EINVAL;
    std::vector<float> im(p->n_int), iv(p->n_int);
    exposed_to_internal(m, im.data());
    exposed_to_internal(v, iv.data());
    if (hipMemcpy(p->m, im.data(), sizeof(float) * p->n_int, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->v, iv.data(), sizeof(float) * p->n_int, hipMemcpyHostToDevice) != hipSuccess)
        return ME_EDEVICE;
    p->step = step;
    return ME_OK;
}

ME_EXPORT int me_proposer_forward(me_proposer* p, const uint8_t* cur, const uint8_t* ref, int32_t width,
                                  int32_t height, int32_t pitch, int64_t pair_stride, int32_t n_pairs, float* head,
                                  void* stream) {
    if (!p) return ME_EINVAL;
    int rc = check_pairs(cur, ref, width, height, pitch, pair_stride, n_pairs);
    if (rc != ME_OK || n_pairs == 0) return rc;
    if (!head) return ME_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = forward(p, cur, ref, width, height, pitch, pair_stride, n_pairs, st);
    if (rc) return rc;
    const int n = n_pairs * (height / 16) * (width / 16);
    hipLaunchKernelGGL(k_head_export, dim3(cdiv(n, 256)), dim3(256), 0, st, p->head, n, head);
    return launched();
}

ME_EXPORT int me_proposer_backward(me_proposer* p, const float* dhead, void* stream) {
    if (!p || !dhead) return ME_EINVAL;
    if (p->P == 0) return ME_EINVAL;  // no forward yet
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n = p->P * (p->H4 / 4) * (p->W4 / 4);
    int rc = grow(&p->g4, &p->cg4, (size_t)n * 4);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pack_ghead, dim3(cdiv(n, 256)), dim3(256), 0, st, dhead, n, p->g4);
    return backward(p, st);
}

ME_EXPORT int me_proposer_train_step(me_proposer* p, const uint8_t* cur, const uint8_t* ref, int32_t width,
                                     int32_t height, int32_t pitch, int64_t pair_stride, int32_t n_pairs,
                                     const me_mv* target, float lr, float* loss, void* stream) {
    if (!p) return ME_EINVAL;
    int rc = check_pairs(cur, ref, width, height, pitch, pair_stride, n_pairs);
    if (rc != ME_OK) return rc;
    if (n_pairs == 0 || !target || !loss || !(lr >= 0.f) || !std::isfinite(lr)) return ME_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    rc = forward(p, cur, ref, width, height, pitch, pair_stride, n_pairs, st);
    if (rc) return rc;
    const int n = n_pairs * (height / 16) * (width / 16);
    const int nb = (int)cdiv(n, 256);
    if ((rc = grow(&p->g4, &p->cg4, (size_t)n * 4)) || (rc = grow(&p->lpart, &p->clpart, (size_t)nb))) return rc;
    hipLaunchKernelGGL(k_head_loss, dim3(nb), dim3(256), 0, st, p->head, reinterpret_cast<const int16_t*>(target), n,
                       p->g4, p->lpart);
    hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(64), 0, st, p->lpart, nb, n, loss);
    if ((rc = backward(p, st))) return rc;
    p->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)p->step), c2 = 1.f - std::pow(b2, (float)p->step);
    hipLaunchKernelGGL(k_adam, dim3(cdiv(p->n_int, 256)), dim3(256), 0, st, p->w, p->g, p->m, p->v, p->n_int, lr, b1,
                       b2, 1e-8f, c1, c2);
    if ((rc = launched())) return rc;
    return pack_all(p, st);
}

ME_EXPORT int me_proposer_infer(me_proposer* p, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height,
                                int32_t pitch, int64_t pair_stride, int32_t n_pairs, int32_t range, me_mv* start,
                                uint8_t* orient, void* stream) {
    if (!p) return ME_EINVAL;
    int rc = check_pairs(cur, ref, width, height, pitch, pair_stride, n_pairs);
    if (rc != ME_OK) return rc;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (n_pairs == 0) return ME_OK;
    if (!start || !orient) return ME_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // One fused launch: every layer of a tile of blocks stays in LDS (the
    // results equal forward() followed by the head decode).
    static std::atomic<int> raised{0};
    if (!raised.load()) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_proposer_infer),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLds) != hipSuccess)
            return ME_EDEVICE;
        raised.store(1);
    }
    const Offsets oi = internal_offsets();
    const int Hb = height / 16, Wb = width / 16;
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return ME_EDEVICE;
        cus = prop.multiProcessorCount;
    }
    const long long tiles = (long long)cdiv(Wb, kTB) * cdiv(Hb, kTB) * n_pairs;
    if (tiles > INT32_MAX) return ME_EUNSUPPORTED;
    const unsigned grid = (unsigned)std::min<long long>(tiles, cus);
    hipLaunchKernelGGL(k_proposer_infer, dim3(grid), dim3(kFusedThreads), kFusedLds, st, cur, ref, pitch,
                       (long long)pair_stride, Hb, Wb, n_pairs, p->wf[0], p->wf[1], p->wf[2], p->wf[3],
                       p->w + oi.b[0], p->w + oi.b[1], p->w + oi.b[2], p->w + oi.b[3], range,
                       reinterpret_cast<int16_t*>(start), orient);
    return launched();
}

ME_EXPORT int me_dcds_learned(me_proposer* p, const uint8_t* cur, const uint8_t* ref, int32_t width, int32_t height,
                              int32_t pitch, int64_t pair_stride, int32_t n_pairs, int32_t range, int32_t algo,
                              me_mv* mv, uint32_t* sad, uint32_t* nsp, void* stream) {
    if (!p)  // no proposer: plain DCDS (the fallback)
        return me_dcds_ex(cur, ref, width, height, pitch, pair_stride, n_pairs, 16, range, algo, nullptr, nullptr, mv,
                          sad, nsp, stream);
    int rc = check_frames(cur, ref, width, height, pitch, pair_stride, n_pairs, 16, range, mv, sad, nsp);
    if (rc != ME_OK || n_pairs == 0) return rc;
    if (algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    const size_t n = (size_t)n_pairs * (height / 16) * (width / 16);
    if ((rc = grow(&p->start, &p->cstart, n * 2)) || (rc = grow(&p->orient, &p->corient, n))) return rc;
    rc = me_proposer_infer(p, cur, ref, width, height, pitch, pair_stride, n_pairs, range,
                           reinterpret_cast<me_mv*>(p->start), p->orient, stream);
    if (rc) return rc;
    return me_dcds_ex(cur, ref, width, height, pitch, pair_stride, n_pairs, 16, range, algo,
                      reinterpret_cast<const me_mv*>(p->start), p->orient, mv, sad, nsp, stream);
}
