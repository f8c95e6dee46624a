// Batched persistent launches (me_batch), the configuration autotuner
// (me_autotune, me_autotune_save, me_autotune_load) and me_shutdown.
//
// A batch is a table of jobs (one frame sequence each, any size).  The table
// travels through a pinned host buffer into device memory, a tiny kernel
// resets the tile counter, and one persistent kernel drains all tiles.  The
// three steps are captured once per kernel variant into a hipGraph and
// replayed; sizes change through the table, not the graph.  Two slots (pinned
// buffer, device table, counter, graphs) alternate, so the host can fill one
// while the other is in flight.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "me.h"
#include "me_batch.hpp"
#include "me_host.hpp"

using namespace me;
using namespace me::host;

namespace {

constexpr int kMaxJobs = 4096;
constexpr int kSlots = 2;

enum { KIND_DCDS = 1, KIND_FS = 2 };
constexpr size_t kStaticLdsReserve = 1024;  // static LDS of the persistent kernels (bytes, upper bound)

// kind, B, rpl, wpg, range class, kernel, threads, lds, cap: everything a captured graph bakes in.
using GraphKey = std::tuple<int, int, int, int, int, const void*, int, size_t, int>;

struct Slot {
    BatchTable* host = nullptr;  // pinned
    BatchTable* dev = nullptr;
    int* counter = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

struct BatchState {
    std::mutex mu;
    Slot slots[kSlots];
    int next = 0;
    int device = -1;
    hipStream_t cap = nullptr;
    int cus = 0;
};
BatchState g_batch;

struct TuneEntry {
    std::string arch;
    int runtime;
    int block, rclass, rpl, wpg, grab;
    float ms;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int ensure_slot(Slot& s) {
    if (s.host) return ME_OK;
    const size_t bytes = batch_table_bytes(kMaxJobs);
    if (hipHostMalloc(reinterpret_cast<void**>(&s.host), bytes, hipHostMallocDefault) != hipSuccess) {
        s.host = nullptr;
        return ME_ENOMEM;
    }
    if (hipMalloc(reinterpret_cast<void**>(&s.dev), bytes) != hipSuccess) {
        s.dev = nullptr;
        return ME_ENOMEM;
    }
    if (hipMalloc(reinterpret_cast<void**>(&s.counter), 64) != hipSuccess) {
        s.counter = nullptr;
        return ME_ENOMEM;
    }
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return ME_EDEVICE;
    return ME_OK;
}

int ensure_state() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ME_EDEVICE;
    if (g_batch.device >= 0 && g_batch.device != dev) return ME_EUNSUPPORTED;  // one device per process
    if (g_batch.device < 0) {
        if (hipStreamCreateWithFlags(&g_batch.cap, hipStreamNonBlocking) != hipSuccess) return ME_EDEVICE;
        if (hipDeviceGetAttribute(&g_batch.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return ME_EDEVICE;
        g_batch.device = dev;
    }
    return ME_OK;
}

// The persistent kernel of one variant, its block size, LDS bytes and grid.
struct Variant {
    const void* fn;
    int threads;
    size_t lds;
};

template <int B, int RPL, int WPG, int RMAX>
Variant dcds_variant() {
    return Variant{reinterpret_cast<const void*>(&k_dcds_batch<B, RPL, WPG, RMAX>), 64 * WPG,
                   dcds_lds_bytes<B, RPL, WPG, RMAX>() + 16};
}

template <int B, int RPL, int RMAX>
Variant dcds_variant_w(int wpg) {
    if (wpg == 1) return dcds_variant<B, RPL, 1, RMAX>();
    if (wpg == 2) return dcds_variant<B, RPL, 2, RMAX>();
    if (wpg == 4) return dcds_variant<B, RPL, 4, RMAX>();
    return dcds_variant<B, RPL, 8, RMAX>();
}

template <int B, int RMAX>
Variant dcds_variant_r(int rpl, int wpg) {
    if (rpl == 1) return dcds_variant_w<B, 1, RMAX>(wpg);
    if constexpr (B == 16) {
        if (rpl == 4) return dcds_variant_w<B, 4, RMAX>(wpg);
    }
    return dcds_variant_w<B, 2, RMAX>(wpg);
}

Variant pick_variant(int kind, int B, int rpl, int wpg, int R) {
    if (kind == KIND_FS) {
        const size_t lds = (B == 16 ? fs_lds_bytes<16>(R) : fs_lds_bytes<8>(R)) + 16;
        const bool split = fs_split(R);
        const void* fn = B == 16 ? (split ? reinterpret_cast<const void*>(&k_fs_batch<16, true>)
                                          : reinterpret_cast<const void*>(&k_fs_batch<16, false>))
                                 : (split ? reinterpret_cast<const void*>(&k_fs_batch<8, true>)
                                          : reinterpret_cast<const void*>(&k_fs_batch<8, false>));
        return Variant{fn, fs_threads(R), lds};
    }
    const int rc = range_class(R);
    if (B == 16) {
        if (rc == 0) return dcds_variant_r<16, 7>(rpl, wpg);
        if (rc == 1) return dcds_variant_r<16, 15>(rpl, wpg);
        return dcds_variant_r<16, 31>(rpl, wpg);
    }
    if (rc == 0) return dcds_variant_r<8, 7>(rpl, wpg);
    if (rc == 1) return dcds_variant_r<8, 15>(rpl, wpg);
    return dcds_variant_r<8, 31>(rpl, wpg);
}

// Enqueues copy + reset + persistent kernel on `st` (capturing or not).
int enqueue(Slot& s, const Variant& v, unsigned grid, size_t table_bytes, hipStream_t st) {
    if (hipMemcpyAsync(s.dev, s.host, table_bytes, hipMemcpyHostToDevice, st) != hipSuccess) return ME_EDEVICE;
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, st, s.counter);
    void* args[] = {&s.dev, &s.counter};
    if (hipLaunchKernel(v.fn, dim3(grid), dim3(v.threads), args, v.lds, st) != hipSuccess) return ME_EDEVICE;
    return ME_OK;
}

// Argument checks shared by me_batch and me_batch_noalloc (nothing is
// launched on an error).  Returns the kernel kind, its configuration (rows
// per lane, waves per group, tiles per grab) and the tile shape in blocks.
int check_batch(const me_job* jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range, int* kind,
                int* rpl, int* wpg, int* grab, int* tile_w, int* tile_h) {
    if (n_jobs < 0 || n_jobs > kMaxJobs) return ME_EINVAL;
    if (algo != ME_ALGO_FS && algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (n_jobs > 0 && !jobs) return ME_EINVAL;
    for (int i = 0; i < n_jobs; ++i) {
        const me_job& j = jobs[i];
        const int rc = check_frames(j.cur, j.ref, j.width, j.height, j.pitch, j.pair_stride, j.n_pairs, block, range,
                                    j.mv, j.sad, j.nsp);
        if (rc != ME_OK) return rc;
        if (j.orient && !j.start) return ME_EINVAL;
        if (algo == ME_ALGO_FS && (j.start || j.orient)) return ME_EINVAL;
    }
    *kind = algo == ME_ALGO_FS ? KIND_FS : KIND_DCDS;
    *rpl = 1;
    *wpg = 1;
    *grab = kDefaultGrab;
    if (*kind == KIND_DCDS) {
        current_cfg(block, range_class(range), rpl, wpg);
        *grab = current_grab(block, range_class(range));
    }
    *tile_w = *kind == KIND_FS ? 1 : 64 * *rpl / block;
    *tile_h = *kind == KIND_FS ? 1 : *wpg;
    return ME_OK;
}

// The device record of one job whose tiles start at tile_begin.
BatchJob make_job(const me_job& j, int32_t algo, int32_t block, int32_t range, int tile_w, int tile_h,
                  long long tile_begin) {
    BatchJob b;
    b.a = frame_args(j.cur, j.ref, j.width, j.height, j.pitch, j.pair_stride, block, range, tile_w, tile_h);
    b.flags = dcds_flags(algo, j.cur, j.ref, j.width, j.pitch, j.pair_stride);
    b.tile_begin = (int)tile_begin;
    b.start = reinterpret_cast<const int16_t*>(j.start);
    b.orient = j.orient;
    b.mv = reinterpret_cast<int16_t*>(j.mv);
    b.sad = j.sad;
    b.nsp = j.nsp;
    b.sse = j.sse;
    return b;
}

long long job_tiles(const BatchJob& b, int n_pairs) { return (long long)b.a.tiles_x * b.a.tiles_y * n_pairs; }

// The shared tile counter runs past the total by one grab (at most
// kMaxGrab tiles) for every workgroup before each has seen the end: 2^30
// keeps it far from int overflow.
constexpr long long kMaxTiles = 1LL << 30;

// Grid of a persistent kernel: resident workgroups per CU x CUs.  The
// persistent kernels also hold a little static LDS (the grabbed tile index):
// their dynamic limit leaves room for it.
int persistent_grid(const Variant& v, int cus, unsigned* grid) {
    if (v.lds > 65536 && hipFuncSetAttribute(v.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(kMaxLds - kStaticLdsReserve)) != hipSuccess)
        return ME_EUNSUPPORTED;
    // The runtime's occupancy answer, bounded by the LDS each workgroup takes
    // (the query can report 0 for windows above 64 KiB even after the limit
    // was raised; the LDS bound is then what applies).
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.fn, v.threads, v.lds) != hipSuccess) per_cu = 0;
    const int by_lds = (int)(kMaxLds / std::max<size_t>(v.lds, 1));
    if (per_cu < 1) per_cu = std::min(by_lds, 2048 / v.threads);
    if (per_cu < 1) return ME_EUNSUPPORTED;
    *grid = (unsigned)(per_cu * cus);
    return ME_OK;
}

int batch_launch(const me_job* jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range, hipStream_t st) {
    int kind = 0, rpl = 1, wpg = 1, grab = kDefaultGrab, tile_w = 1, tile_h = 1;
    int rc = check_batch(jobs, n_jobs, algo, block, range, &kind, &rpl, &wpg, &grab, &tile_w, &tile_h);
    if (rc != ME_OK) return rc;

    // Table contents (host side, before touching shared state).
    std::vector<BatchJob> tab;
    tab.reserve(n_jobs);
    long long total = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const me_job& j = jobs[i];
        if (j.n_pairs == 0) continue;
        const BatchJob b = make_job(j, algo, block, range, tile_w, tile_h, total);
        total += job_tiles(b, j.n_pairs);
        if (total > kMaxTiles) return ME_EUNSUPPORTED;
        tab.push_back(b);
    }
    if (tab.empty()) return ME_OK;

    const Variant v = pick_variant(kind, block, rpl, wpg, range);
    if (v.lds > kMaxLds - kStaticLdsReserve) return ME_EUNSUPPORTED;

    std::lock_guard<std::mutex> lock(g_batch.mu);
    rc = ensure_state();
    if (rc != ME_OK) return rc;
    Slot& s = g_batch.slots[g_batch.next];
    g_batch.next = (g_batch.next + 1) % kSlots;
    rc = ensure_slot(s);
    if (rc != ME_OK) return rc;
    if (s.pending && hipEventSynchronize(s.done) != hipSuccess) return ME_EDEVICE;
    s.pending = false;

    s.host->n_jobs = (int)tab.size();
    s.host->total_tiles = (int)total;
    s.host->grab = grab;
    memcpy(s.host->jobs, tab.data(), tab.size() * sizeof(BatchJob));
    int cap = 64;
    while (cap < (int)tab.size()) cap *= 2;
    const size_t table_bytes = batch_table_bytes(cap);

    unsigned grid = 0;
    rc = persistent_grid(v, g_batch.cus, &grid);
    if (rc != ME_OK) return rc;

    const GraphKey key{kind, block, rpl, wpg, range_class(range), v.fn, v.threads, v.lds, cap};
    auto it = s.graphs.find(key);
    if (it == s.graphs.end()) {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = hipStreamBeginCapture(g_batch.cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const int erc = enqueue(s, v, grid, table_bytes, g_batch.cap);
            ok = hipStreamEndCapture(g_batch.cap, &graph) == hipSuccess && erc == ME_OK && graph;
        }
        if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        it = s.graphs.emplace(key, ok ? exec : nullptr).first;
    }
    if (it->second) {
        if (hipGraphLaunch(it->second, st) != hipSuccess) return ME_EDEVICE;
    } else {
        // Capture unavailable: the same three steps as direct launches.
        rc = enqueue(s, v, grid, table_bytes, st);
        if (rc != ME_OK) return rc;
    }
    if (hipEventRecord(s.done, st) != hipSuccess) return ME_EDEVICE;
    s.pending = true;
    return ME_OK;
}

int device_identity(std::string* arch, int* runtime) {
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return ME_EDEVICE;
    if (hipRuntimeGetVersion(runtime) != hipSuccess) return ME_EDEVICE;
    *arch = p.gcnArchName;
    const size_t colon = arch->find(':');
    if (colon != std::string::npos) arch->resize(colon);
    return ME_OK;
}

}  // namespace

ME_EXPORT int me_batch(const me_job* jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range, void* stream) {
    return batch_launch(jobs, n_jobs, algo, block, range, reinterpret_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// me_batch_noalloc: the same persistent launch with its job table and tile
// counter in a file-scope device array instead of library allocations.  The
// table reaches the array through the arguments of small copy kernels (16
// jobs each), so the call needs no pinned buffer, no device allocation and no
// host-to-device copy of pageable memory; a header kernel then writes the job
// count and total and resets the counter (a kernel, not a memset), and the
// persistent kernel reads them in stream order.  Each device holds its own
// copy of the array; its address comes from hipGetSymbolAddress on the first
// call on that device.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoAllocJobs = 512;
constexpr size_t kScratchHead = 256;  // the tile counter, alone in its cache line
constexpr size_t kScratchBytes = kScratchHead + batch_table_bytes(kNoAllocJobs);

}  // namespace

// Job table and tile counter of me_batch_noalloc (one copy per device).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kChunkJobs = 16;
struct JobChunk {
    BatchJob jobs[kChunkJobs];  // 2 KiB of kernel arguments
};
static_assert(sizeof(BatchJob) % 4 == 0, "jobs are copied as 32-bit words");

__global__ __launch_bounds__(256) void k_table_write(JobChunk c, BatchTable* __restrict__ tab, int first, int n) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(c.jobs);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&tab->jobs[first]);
    const int words = n * (int)(sizeof(BatchJob) / 4);
    for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

__global__ void k_table_head(BatchTable* __restrict__ tab, int* __restrict__ counter, int n_jobs, int total,
                             int grab) {
    if (threadIdx.x == 0) {
        tab->n_jobs = n_jobs;
        tab->total_tiles = total;
        tab->grab = grab;
        counter[0] = 0;
    }
}

constexpr int kMaxDevices = 64;
struct ScratchOfDevice {
    std::atomic<bool> ready{false};
    unsigned char* ptr = nullptr;  // device address of this device's copy of `scratch`
    int cus = 0;
};
ScratchOfDevice g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// This device's copy of the array and its CU count (set up once per device,
// with that device current).
int scratch_of_device(unsigned char** ptr, int* cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return ME_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return ME_EUNSUPPORTED;
    ScratchOfDevice& d = g_scratch[dev];
    if (!d.ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!d.ready.load(std::memory_order_relaxed)) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ME_EDEVICE;
            int n = 0;
            if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
                return ME_EDEVICE;
            d.ptr = static_cast<unsigned char*>(p);
            d.cus = n;
            d.ready.store(true, std::memory_order_release);
        }
    }
    *ptr = d.ptr;
    *cus = d.cus;
    return ME_OK;
}

}  // namespace

ME_EXPORT int me_batch_noalloc(const me_job* jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range,
                               void* stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int kind = 0, rpl = 1, wpg = 1, grab = kDefaultGrab, tile_w = 1, tile_h = 1;
    int rc = check_batch(jobs, n_jobs, algo, block, range, &kind, &rpl, &wpg, &grab, &tile_w, &tile_h);
    if (rc != ME_OK) return rc;
    if (n_jobs > kNoAllocJobs) return ME_EUNSUPPORTED;
    long long total = 0;
    int n = 0;
    for (int i = 0; i < n_jobs; ++i) {
        if (jobs[i].n_pairs == 0) continue;
        total += job_tiles(make_job(jobs[i], algo, block, range, tile_w, tile_h, 0), jobs[i].n_pairs);
        if (total > kMaxTiles) return ME_EUNSUPPORTED;
        ++n;
    }
    if (n == 0) return ME_OK;
    const Variant v = pick_variant(kind, block, rpl, wpg, range);
    if (v.lds > kMaxLds - kStaticLdsReserve) return ME_EUNSUPPORTED;
    unsigned char* base = nullptr;
    int cus = 0;
    rc = scratch_of_device(&base, &cus);
    if (rc != ME_OK) return rc;
    unsigned grid = 0;
    rc = persistent_grid(v, cus, &grid);
    if (rc != ME_OK) return rc;

    int* counter = reinterpret_cast<int*>(base);
    BatchTable* tab = reinterpret_cast<BatchTable*>(base + kScratchHead);
    JobChunk chunk;
    int in_chunk = 0, first = 0;
    long long begin = 0;
    for (int i = 0; i < n_jobs; ++i) {
        if (jobs[i].n_pairs == 0) continue;
        chunk.jobs[in_chunk] = make_job(jobs[i], algo, block, range, tile_w, tile_h, begin);
        begin += job_tiles(chunk.jobs[in_chunk], jobs[i].n_pairs);
        if (++in_chunk == kChunkJobs || first + in_chunk == n) {
            hipLaunchKernelGGL(k_table_write, dim3(1), dim3(256), 0, st, chunk, tab, first, in_chunk);
            if (launched() != ME_OK) return ME_EDEVICE;  // no search over a partial table
            first += in_chunk;
            in_chunk = 0;
        }
    }
    hipLaunchKernelGGL(k_table_head, dim3(1), dim3(64), 0, st, tab, counter, n, (int)total, grab);
    if (launched() != ME_OK) return ME_EDEVICE;
    void* args[] = {&tab, &counter};
    if (hipLaunchKernel(v.fn, dim3(grid), dim3(v.threads), args, v.lds, st) != hipSuccess) return ME_EDEVICE;
    return launched();
}

// Records a tuning result, replacing an earlier one for the same device,
// runtime, block size and range class.
static void remember(const TuneEntry& e) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (auto& t : g_tune) {
        if (t.arch == e.arch && t.runtime == e.runtime && t.block == e.block && t.rclass == e.rclass) {
            t = e;
            return;
        }
    }
    g_tune.push_back(e);
}

ME_EXPORT int me_autotune(const me_job* jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range,
                          int32_t reps, me_config* best, float* best_ms, void* stream) {
    if (algo != ME_ALGO_DCDS && algo != ME_ALGO_DCDS_S) return ME_EUNSUPPORTED;
    if (block != 8 && block != 16) return ME_EUNSUPPORTED;
    if (range < 1 || range > 31) return ME_EUNSUPPORTED;
    if (reps < 1 || n_jobs < 1 || !jobs) return ME_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return ME_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return ME_EDEVICE;
    }
    me_config saved;
    me_get_config(block, range, &saved);
    me_config top{0, 0, 0};
    float top_ms = 0.f;
    int rc = ME_OK;
    // Mean time per launch of configuration c over `reps` launches (after a
    // warm-up that also builds the graph); ME_EUNSUPPORTED if c does not fit.
    auto time_cfg = [&](const me_config& c, float* ms) -> int {
        if (me_set_config(block, range, &c) != ME_OK) return ME_EUNSUPPORTED;
        int r = batch_launch(jobs, n_jobs, algo, block, range, st);
        if (r != ME_OK) return r;
        if (hipEventRecord(e0, st) != hipSuccess) return ME_EDEVICE;
        for (int i = 0; i < reps && r == ME_OK; ++i) r = batch_launch(jobs, n_jobs, algo, block, range, st);
        if (r != ME_OK) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ME_EDEVICE;
        if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return ME_EDEVICE;
        *ms /= (float)reps;
        return ME_OK;
    };
    // Every layout at the default grab, then every grab with the best layout.
    const int rpls[3] = {1, 2, 4};
    const int wpgs[4] = {1, 2, 4, 8};
    for (int ri = 0; ri < 3 && rc == ME_OK; ++ri) {
        for (int wi = 0; wi < 4 && rc == ME_OK; ++wi) {
            const me_config c{rpls[ri], wpgs[wi], kDefaultGrab};
            float ms = 0.f;
            const int r = time_cfg(c, &ms);
            if (r == ME_EUNSUPPORTED) continue;
            if (r != ME_OK) {
                rc = r;
                break;
            }
            if (top.rows_per_lane == 0 || ms < top_ms) {
                top = c;
                top_ms = ms;
            }
        }
    }
    const int grabs[4] = {1, 2, 8, 16};
    for (int gi = 0; gi < 4 && rc == ME_OK && top.rows_per_lane != 0; ++gi) {
        const me_config c{top.rows_per_lane, top.waves_per_group, grabs[gi]};
        float ms = 0.f;
        const int r = time_cfg(c, &ms);
        if (r != ME_OK) {
            rc = r;
            break;
        }
        if (ms < top_ms) {
            top = c;
            top_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != ME_OK || top.rows_per_lane == 0) {
        me_set_config(block, range, &saved);
        return rc != ME_OK ? rc : ME_EUNSUPPORTED;
    }
    me_set_config(block, range, &top);
    if (best) *best = top;
    if (best_ms) *best_ms = top_ms;
    TuneEntry e;
    if (device_identity(&e.arch, &e.runtime) == ME_OK) {
        e.block = block;
        e.rclass = range_class(range);
        e.rpl = top.rows_per_lane;
        e.wpg = top.waves_per_group;
        e.grab = top.tiles_per_grab;
        e.ms = top_ms;
        remember(e);
    }
    return ME_OK;
}

ME_EXPORT int me_autotune_save(const char* path) {
    if (!path) return ME_EINVAL;
    FILE* f = fopen(path, "w");
    if (!f) return ME_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    fprintf(f, "# me autotune cache v2: arch runtime block range_class rows_per_lane waves_per_group tiles_per_grab "
               "ms\n");
    for (const auto& t : g_tune)
        fprintf(f, "%s %d %d %d %d %d %d %.6f\n", t.arch.c_str(), t.runtime, t.block, t.rclass, t.rpl, t.wpg, t.grab,
                t.ms);
    const int bad = ferror(f);
    fclose(f);
    return bad ? ME_EINVAL : ME_OK;
}

ME_EXPORT int me_autotune_load(const char* path, int32_t* applied, int32_t* rejected) {
    if (!path) return ME_EINVAL;
    if (applied) *applied = 0;
    if (rejected) *rejected = 0;
    FILE* f = fopen(path, "r");
    if (!f) return ME_EINVAL;
    std::string arch;
    int runtime = 0;
    const bool have_id = device_identity(&arch, &runtime) == ME_OK;
    char line[512];
    int n_ok = 0, n_bad = 0;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        // v2 lines carry tiles_per_grab before the time; v1 lines (without
        // it) keep the default grab.
        char a[128];
        int rt, blk, rcl, rpl, wpg, grab = kDefaultGrab;
        float ms;
        char extra[2];
        int tokens = 0;
        for (const char* q = line; *q;) {
            while (*q == ' ' || *q == '\t' || *q == '\n' || *q == '\r') ++q;
            if (!*q) break;
            ++tokens;
            while (*q && *q != ' ' && *q != '\t' && *q != '\n' && *q != '\r') ++q;
        }
        bool ok = false;
        if (tokens == 8)
            ok = sscanf(line, "%127s %d %d %d %d %d %d %f %1s", a, &rt, &blk, &rcl, &rpl, &wpg, &grab, &ms, extra) == 8;
        else if (tokens == 7)
            ok = sscanf(line, "%127s %d %d %d %d %d %f %1s", a, &rt, &blk, &rcl, &rpl, &wpg, &ms, extra) == 7;
        if (!ok || rcl < 0 || rcl > 2 || (blk != 8 && blk != 16) || !valid_cfg(blk, rpl, wpg) || grab == 0 ||
            !valid_grab(grab)) {
            ++n_bad;
            continue;
        }
        if (!have_id || arch != a || rt != runtime) continue;  // tuned on other hardware or runtime
        const int rep_range = rcl == 0 ? 7 : (rcl == 1 ? 15 : 31);
        me_config c{rpl, wpg, grab};
        if (me_set_config(blk, rep_range, &c) == ME_OK) {
            ++n_ok;
            remember(TuneEntry{a, rt, blk, rcl, rpl, wpg, grab, ms});
        }
    }
    fclose(f);
    if (applied) *applied = n_ok;
    if (rejected) *rejected = n_bad;
    return ME_OK;
}

ME_EXPORT int me_shutdown(void) {
    std::lock_guard<std::mutex> lock(g_batch.mu);
    int rc = ME_OK;
    for (auto& s : g_batch.slots) {
        if (s.pending && hipEventSynchronize(s.done) != hipSuccess) rc = ME_EDEVICE;
        s.pending = false;
        for (auto& kv : s.graphs)
            if (kv.second) (void)hipGraphExecDestroy(kv.second);
        s.graphs.clear();
        if (s.host) (void)hipHostFree(s.host);
        if (s.dev) (void)hipFree(s.dev);
        if (s.counter) (void)hipFree(s.counter);
        if (s.done) (void)hipEventDestroy(s.done);
        s.host = nullptr;
        s.dev = nullptr;
        s.counter = nullptr;
        s.done = nullptr;
    }
    if (g_batch.cap) (void)hipStreamDestroy(g_batch.cap);
    g_batch.cap = nullptr;
    g_batch.device = -1;
    return rc;
}
