// Persistent kernels over a device job table: many frame sequences of any
// size in one launch.  Each workgroup takes the next tile from an atomic
// counter until the table is exhausted, so streams of uneven resolution share
// the GPU without per-stream launches.
#pragma once

#include "me_kernels.hpp"

namespace me {

struct BatchJob {
    FrameArgs a;             // geometry of this job (tiles per the current configuration)
    int flags;               // DCDS flags (simplified, 16-byte loads)
    int tile_begin;          // first tile of this job in the flattened index space
    const int16_t* start;    // optional learned start vectors
    const uint8_t* orient;   // optional first-cross orientations
    int16_t* mv;
    uint32_t* sad;
    uint32_t* nsp;
    uint32_t* sse;           // optional compensated-block squared error
};

struct BatchTable {
    int n_jobs;
    int total_tiles;
    int grab;  // tiles a workgroup takes per grab from the counter
    int pad0;
    BatchJob jobs[1];  // n_jobs entries (the allocation holds the capacity)
};

__host__ __device__ constexpr size_t batch_table_bytes(int cap) {
    return sizeof(BatchTable) + (size_t)(cap - 1) * sizeof(BatchJob);
}

static __global__ void k_batch_reset(int* counter) {
    if (threadIdx.x == 0) counter[0] = 0;
}

// Index of the job holding tile t: the last job whose tile_begin <= t.
__device__ __forceinline__ int batch_job_of(const BatchTable* tab, int t) {
    int lo = 0, hi = tab->n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab->jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Tiles are taken `grab` at a time (the table's, 1 to 16): one atomic and
// one job lookup serve several tiles, which are then walked in order
// (crossing job boundaries with one comparison each).
constexpr int kMaxGrab = 16;

// Takes the next chunk for the whole workgroup; every wave leaves the previous
// tile (and its LDS) before the new index is published.
__device__ __forceinline__ int batch_next(int* counter, int grab, int* s_tile) {
    __syncthreads();
    if (threadIdx.x == 0) *s_tile = atomicAdd(counter, grab);
    __syncthreads();
    return *s_tile;
}

template <int B, int RPL, int WPG, int RMAX>
__global__ __launch_bounds__(64 * WPG) void k_dcds_batch(const BatchTable* __restrict__ tab, int* __restrict__ counter) {
    extern __shared__ uint32_t smem[];
    __shared__ int s_tile;
    const int total = tab->total_tiles;
    const int n = tab->n_jobs;
    const int grab = tab->grab;
    for (;;) {
        const int t0 = batch_next(counter, grab, &s_tile);
        if (t0 >= total) break;
        int j = batch_job_of(tab, t0);
        const int t1 = min(t0 + grab, total);
        for (int t = t0; t < t1; ++t) {
            while (j + 1 < n && tab->jobs[j + 1].tile_begin <= t) ++j;
            const BatchJob& jb = tab->jobs[j];
            const int i = t - jb.tile_begin;
            const int r = jb.a.div_tx.div(i), tx = i - r * jb.a.tiles_x;
            const int pair = jb.a.div_ty.div(r), ty = r - pair * jb.a.tiles_y;
            if (t != t0) __syncthreads();  // the previous tile's waves are done with LDS
            dcds_tile<B, RPL, WPG, RMAX>(smem, jb.a, jb.flags, pair, tx, ty, jb.start, jb.orient, jb.mv, jb.sad,
                                         jb.nsp, jb.sse);
        }
    }
}

template <int B, bool SPLIT>
__global__ __launch_bounds__(256) void k_fs_batch(const BatchTable* __restrict__ tab, int* __restrict__ counter) {
    extern __shared__ uint32_t smem[];
    __shared__ int s_tile;
    const int total = tab->total_tiles;
    const int n = tab->n_jobs;
    const int grab = tab->grab;
    for (;;) {
        const int t0 = batch_next(counter, grab, &s_tile);
        if (t0 >= total) break;
        int j = batch_job_of(tab, t0);
        const int t1 = min(t0 + grab, total);
        for (int t = t0; t < t1; ++t) {
            while (j + 1 < n && tab->jobs[j + 1].tile_begin <= t) ++j;
            const BatchJob& jb = tab->jobs[j];
            int r = t - jb.tile_begin;
            const int bx = r % jb.a.bw;
            r /= jb.a.bw;
            const int by = r % jb.a.bh;
            const int pair = r / jb.a.bh;
            if (t != t0) __syncthreads();
            fs_block<B, SPLIT>(smem, jb.a, pair, bx, by, jb.mv, jb.sad, jb.nsp, jb.sse, blockDim.x);
        }
    }
}

}  // namespace me
