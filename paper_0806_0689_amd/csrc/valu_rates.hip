// Issue rates of the VALU instructions the searches are built on, measured
// on the current device: each thread runs 16 independent chains of one
// instruction, 8 waves per SIMD.  Prints one JSON object: cycles per wave64
// instruction per SIMD, and the absolute differences per second that the
// byte-SAD instructions reach at that rate (v_sad_u8: 4 per lane,
// v_qsad_pk_u16_u8: 16 per lane).  The full search's VALU roofline is the
// v_qsad_pk_u16_u8 figure.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHECK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

constexpr int kChains = 16;

template <int OP>
__global__ __launch_bounds__(256) void k_rate(uint64_t* out, int iters) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    const uint32_t b = t * 2654435761u;
    uint64_t q[kChains];
    uint32_t a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        q[j] = (uint64_t)(t + j) * 0x9E3779B97F4A7C15ull;
        a[j] = t + 77u * j;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            if constexpr (OP == 0) q[j] = __builtin_amdgcn_qsad_pk_u16_u8(q[(j + 1) % kChains], b, q[j]);
            if constexpr (OP == 1) a[j] = __builtin_amdgcn_sad_u8(a[(j + 1) % kChains], b, a[j]);
            if constexpr (OP == 2) a[j] = __builtin_amdgcn_alignbyte(a[j], a[(j + 1) % kChains], b);
            if constexpr (OP == 3) a[j] = __builtin_amdgcn_udot4(a[(j + 1) % kChains], b, a[j], false);
            if constexpr (OP == 4) a[j] = a[j] + (a[(j + 1) % kChains] ^ b);
        }
    }
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += q[j] + a[j];
    out[t] = s;
}

int main() {
    int dev = 0;
    hipDeviceProp_t prop;
    CHECK(hipGetDevice(&dev));
    CHECK(hipGetDeviceProperties(&prop, dev));
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    const int iters = 2048;
    const double clock_hz = 2.4e9;  // the MI355X peak engine clock
    uint64_t* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(uint64_t) * (size_t)blocks * 256));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const char* names[5] = {"v_qsad_pk_u16_u8", "v_sad_u8", "v_alignbyte_b32", "v_dot4_u32_u8", "v_xad_u32"};
    void (*fns[5])(uint64_t*, int) = {k_rate<0>, k_rate<1>, k_rate<2>, k_rate<3>, k_rate<4>};
    double cyc[5];
    for (int f = 0; f < 5; ++f) {
        hipLaunchKernelGGL(fns[f], dim3(blocks), dim3(256), 0, 0, out, 8);
        CHECK(hipGetLastError());
        CHECK(hipDeviceSynchronize());
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            CHECK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(fns[f], dim3(blocks), dim3(256), 0, 0, out, iters);
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            best = ms < best ? ms : best;
        }
        const double winst = (double)blocks * 4 * iters * kChains;  // wave instructions
        cyc[f] = (best * 1e-3) * (double)cus * 4 * clock_hz / winst;
    }
    CHECK(hipFree(out));
    const double simd_cycles_per_s = (double)cus * 4 * clock_hz;
    printf("{\"device\": \"%s\", \"cus\": %d, \"clock_ghz\": 2.4, \"cycles_per_wave_instruction\": {", prop.gcnArchName,
           cus);
    for (int f = 0; f < 5; ++f) printf("%s\"%s\": %.3f", f ? ", " : "", names[f], cyc[f]);
    printf("}, \"absdiff_per_s\": {\"v_qsad_pk_u16_u8\": %.4g, \"v_sad_u8\": %.4g}}\n",
           simd_cycles_per_s / cyc[0] * 64 * 16, simd_cycles_per_s / cyc[1] * 64 * 4);
    return 0;
}
