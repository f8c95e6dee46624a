/*
 * me.h -- block-matching motion estimation on AMD Instinct MI355X (gfx950).
 *
 * The problem (Jia & Zhang, §I): a frame is cut into non-overlapping,
 * equal-sized B x B blocks; for each block of the current frame, find the
 * displacement of the best-matching block of the reference (previous) frame
 * inside a window centred on the block's own position, by minimising a block
 * distortion measure.  This library uses SAD (the paper's MAD times B^2: the
 * same argmin and the same ties).
 *
 * Two searches:
 *   full search (FS): every candidate of the window (§I);
 *   directional cross diamond search (DCDS, §III-B): a horizontal cross
 *   pattern first, then horizontal/vertical diamonds until the centre wins,
 *   then the two middle points.
 *
 * Conventions shared by every entry point
 *   - Frames are 8-bit luma, row-major, `pitch` bytes between rows, in device
 *     memory owned by the caller.  width and height must be multiples of
 *     `block`; pitch must be >= width and a multiple of 4; frame pointers must
 *     be 4-byte aligned.  One frame must span less than 2 GiB (height * pitch
 *     < 2^31; larger frames give ME_EUNSUPPORTED).
 *   - A motion vector (x, y) places the reference block at (x0 + x, y0 + y)
 *     for the current block at (x0, y0); +x right, +y down.
 *   - Candidate set of a block: |x|, |y| <= range and the displaced block wholly
 *     inside the frame (restricted vectors, no padding).  Points outside it are
 *     never evaluated and never counted.
 *   - nsp = number of distinct candidates whose SAD was evaluated (the paper's
 *     NSP, §III-B Eq. (8), §IV).
 *   - FS tie order: smallest (SAD, |x|+|y|, y, x).  DCDS ties keep the pattern
 *     centre; among other points the order is: cross (0,0), (-1,0), (+1,0),
 *     (-2,0), (+2,0), (0,-1), (0,+1); horizontal diamond (-2,0), (+2,0), (0,-1),
 *     (0,+1); vertical diamond (0,-2), (0,+2), (-1,0), (+1,0); middle points
 *     negative side first.
 *   - Sequences: a call covers `n_pairs` frame pairs; pair p reads
 *     cur + p * pair_stride and ref + p * pair_stride (bytes).  For a sequence
 *     stored as frames [T][height][pitch], pass cur = frame 1, ref = frame 0,
 *     pair_stride = height * pitch and n_pairs = T - 1.  A call over more
 *     pairs than one kernel launch holds (2^31 - 1 work-items) is issued as
 *     several launches over consecutive pair ranges, in order on `stream`.
 *   - Outputs are device arrays of n_pairs * (height/block) * (width/block)
 *     entries in pair-major, then raster block order, owned by the caller.
 *   - Calls are asynchronous and ordered on `stream` (a hipStream_t; NULL is
 *     the default stream).  Outputs are valid once the stream has reached the
 *     call.
 *   - Argument errors are detected on the host before anything is launched;
 *     no exception crosses this interface.  A call with n_pairs == 0 (or
 *     n == 0) does nothing and returns ME_OK once the sizes are valid; its
 *     pointers may then be NULL.
 */
#ifndef ME_H
#define ME_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int16_t x, y;
} me_mv;

/* Status codes.  Every entry point returns one of these.                    */
enum {
    ME_OK = 0,
    ME_EINVAL = -1,       /* NULL pointer, bad size, misaligned pointer or pitch */
    ME_EUNSUPPORTED = -2, /* block not 8 or 16, range outside 1..31, ...        */
    ME_ENOMEM = -3,       /* the library could not allocate its workspace       */
    ME_EDEVICE = -4       /* a HIP launch or runtime call failed                */
};

/* Search algorithms.                                                        */
enum {
    ME_ALGO_FS = 0,     /* full search                                         */
    ME_ALGO_DCDS = 1,   /* DCDS, §III-B                                         */
    ME_ALGO_DCDS_S = 2  /* simplified DCDS, §IV-C: one middle point in Step 4   */
};

/* Human-readable text for a status code (static storage).                   */
const char *me_status_string(int status);

/*
 * Kernel configuration of the DCDS searches (me_dcds, me_dcds_ex, me_batch):
 * how many rows of a block one lane holds (1, 2 or 4 for 16x16 blocks; 1 or 2
 * for 8x8), how many waves share one staged reference window (1, 2, 4 or 8;
 * each wave takes 64 * rows_per_lane / block blocks side by side) and, for the
 * batched launches, how many work tiles a workgroup takes per grab from the
 * shared counter (1, 2, 4, 8 or 16; 0 = the default, 4).  Results do not
 * depend on it, only speed.  Kept per block size and range class (1-7, 8-15,
 * 16-31) for the process; me_set_config with cfg == NULL restores the
 * built-in default; ME_EUNSUPPORTED for values outside the lists (and, at call
 * time, for a configuration whose window exceeds the 160 KiB of LDS of a
 * compute unit).  me_get_config reports the values in force (tiles_per_grab
 * never 0).  Not meant to change while searches of that class are being
 * enqueued from another thread.
 */
typedef struct {
    int32_t rows_per_lane;
    int32_t waves_per_group;
    int32_t tiles_per_grab;
} me_config;

int me_set_config(int32_t block, int32_t range, const me_config *cfg);
int me_get_config(int32_t block, int32_t range, me_config *cfg);

/*
 * Full search (§I; Table IX row "FS").  Every candidate of the window is
 * evaluated; mv/sad hold the tie-ordered minimum, nsp the candidate count.
 */
int me_fullsearch(const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height, int32_t pitch,
                  int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range,
                  me_mv *mv, uint32_t *sad, uint32_t *nsp, void *stream);

/*
 * DCDS (§III-B, Steps 1-4 with switching strategies one and two), from the
 * window origin.
 */
int me_dcds(const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height, int32_t pitch,
            int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range,
            me_mv *mv, uint32_t *sad, uint32_t *nsp, void *stream);

/*
 * DCDS with options.  algo: ME_ALGO_DCDS or ME_ALGO_DCDS_S.
 * start (optional, device, one per block): a proposed start vector, clamped
 * into the block's candidate set.  Plain DCDS runs first, from the origin;
 * then the start is evaluated, and only if its SAD is below the origin's does
 * DCDS run again, with its first cross centred on the start, over the same
 * evaluated point set.  The better of the two results is returned (a tie
 * keeps the plain one), so the result is never worse than plain DCDS.
 * orient (optional, device, one byte per block): 0 = horizontal cross (the
 * paper's), 1 = vertical cross for that second search's first pattern.  nsp
 * counts every distinct point of both searches and the probe.  The learned
 * start is this library's addition, not part of the paper's method.
 */
int me_dcds_ex(const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height, int32_t pitch,
               int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, int32_t algo,
               const me_mv *start, const uint8_t *orient,
               me_mv *mv, uint32_t *sad, uint32_t *nsp, void *stream);

/*
 * Any search with every option: algo ME_ALGO_FS, ME_ALGO_DCDS or
 * ME_ALGO_DCDS_S; start/orient as me_dcds_ex (DCDS only, else ME_EINVAL).
 * sse (optional, device, one per block): the sum of squared differences
 * between the block and the reference block at its vector -- the
 * motion-compensated block behind the MSE and PSNR of §IV -- computed from
 * the data already staged for the search (no extra frame reads).
 * me_fullsearch, me_dcds and me_dcds_ex are this call without sse.
 */
int me_search(const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height, int32_t pitch,
              int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range, int32_t algo,
              const me_mv *start, const uint8_t *orient,
              me_mv *mv, uint32_t *sad, uint32_t *nsp, uint32_t *sse, void *stream);

/*
 * Quality of a motion field per frame pair, the measures of §IV (Tables I,
 * VIII-X): MAD and MSE per pixel and the PSNR of the motion-compensated
 * frame, and -- given the true vectors (those of full search) -- the mean
 * distance from them and the probability of finding them.
 * Inputs are the per-block outputs of one search over n_pairs pairs of
 * width x height frames (mv, sad, sse from me_search; device) and optional
 * true vectors mv_true (device, same layout).  out (device, 8-byte aligned)
 * receives one record per pair.  Distance is Euclidean; a block finds the
 * true vector when both components are equal.  The sums run in a fixed order.
 */
typedef struct {
    uint64_t sad;     /* sum of the blocks' SAD */
    uint64_t sse;     /* sum of the blocks' squared error */
    uint32_t blocks;  /* blocks per pair */
    uint32_t equal;   /* blocks whose vector equals the true one (0 without mv_true) */
    double dist;      /* sum of the Euclidean distances to the true vectors (0 without mv_true) */
    double mad;       /* sad / (blocks * block^2) */
    double mse;       /* sse / (blocks * block^2) */
    double psnr;      /* 10 log10(255^2 / mse) in dB; +inf when mse = 0 */
} me_quality;

int me_frame_quality(const me_mv *mv, const uint32_t *sad, const uint32_t *sse, const me_mv *mv_true,
                     int32_t width, int32_t height, int32_t n_pairs, int32_t block, me_quality *out,
                     void *stream);

/*
 * Statistics of the motion-vector probability (MVP) distribution of §II-C,
 * from full search over n_pairs frame pairs (frames as me_fullsearch).  With
 * n = 2 range + 1 and vector index (y + range) n + (x + range), the call adds
 * every block to three device counter arrays (uint32; the caller zeroes
 * them, so several sequences can be accumulated as the paper does):
 *   hist[n*n]      the full-search vector (Tables II and III, Fig. 3);
 *   d1[9][n*n]     the vector given P, the best point of the CDS first-step
 *                  cross {(x, 0): |x| <= 2} U {(0, y): |y| <= 2} -- the prior
 *                  distribution of Eq. (4); P index x + 2 for (x, 0), then
 *                  5, 6, 7, 8 for (0, -2), (0, -1), (0, 1), (0, 2);
 *   d2[n*n][25]    the best point of the central 5x5 square given the vector
 *                  -- the posterior distribution of Eq. (6); point index
 *                  (y + 2) 5 + (x + 2).
 * "Best" uses full search's order (SAD, then |x| + |y|, then y, then x) over
 * the points inside the block's candidate set.  +y points down the frame.
 */
int me_mvp_stats(const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height, int32_t pitch,
                 int64_t pair_stride, int32_t n_pairs, int32_t block, int32_t range,
                 uint32_t *hist, uint32_t *d1, uint32_t *d2, void *stream);

/*
 * The tables of §II-C from those counters, as me_mvp_tables_size(range)
 * doubles at out (device, 8-byte aligned), in this order (N = total count):
 *   quarter[(range+1)^2]  Table II: count at (+-x, +-y) / N, row |y|, column |x|
 *   Ax[n], Ay[n]          Table III: marginal of x (of y) / N, index d + range
 *   Bx[n], By[n]          Table III: vectors (d, 0) (and (0, d)) / N
 *   regions[5]            Fig. 3: 5x5 square, 5x5 diamond, 5x5 cross, 3x3
 *                         square, 5x3 flat diamond
 *   eta[5]                Table VI / Eq. (7): P_1 / n_1 of the 3x3 square
 *                         (BBGDS), large diamond (DS), 5x5 cross (CDS),
 *                         hexagon (HEXBS) and HCSP (DCDS)
 *   d1[9][n*n]            Eq. (4), each row normalised to 1 (0 if empty)
 *   d2[n*n][25]           Eq. (6), each row normalised to 1 (0 if empty)
 *   t1[25], t2[25]        d2 given a vector in T1 = [4,7] x [4,7] and
 *                         T2 = [-7,-4] x [4,7], normalised to 1
 * me_mvp_tables_size returns ME_EUNSUPPORTED for a range outside 1..31.
 */
int32_t me_mvp_tables_size(int32_t range);
int me_mvp_tables(const uint32_t *hist, const uint32_t *d1, const uint32_t *d2, int32_t range, double *out,
                  void *stream);

/*
 * DCDS over caller-given cost surfaces instead of frames: the ideal-condition
 * analysis of §III-C (Table VII) runs the search on a distortion defined for
 * every window point.  cost: device int32 [n][2*range+1][2*range+1] (row = y +
 * range, column = x + range); valid: optional device uint8 of the same shape
 * (0 = outside the candidate set; NULL = whole window).  The set is taken
 * as the bounding rectangle of the marked points plus the origin, which is
 * always a candidate (frame clipping always yields such a rectangle).  start/orient as in
 * me_dcds_ex (one per surface, optional).  Outputs per surface: mv, the
 * distortion at mv (cost_out) and nsp.  Costs must lie in 0 .. 2^28 - 1.
 */
int me_dcds_surface(const int32_t *cost, const uint8_t *valid, int32_t n, int32_t range, int32_t algo,
                    const me_mv *start, const uint8_t *orient,
                    me_mv *mv, uint32_t *cost_out, uint32_t *nsp, void *stream);

/*
 * Batched search over many sequences in one persistent launch (this
 * library's addition; the search itself is the one above).  A job is one
 * frame sequence (its own size, pitch and pair count; the block size and the
 * range are the batch's).  Each job's arguments follow me_search; start/orient
 * must be NULL for ME_ALGO_FS.  Up to 4096 jobs and 2^30 work tiles (a
 * tile is one block for FS and one workgroup's blocks, at most 128, for DCDS;
 * ME_EUNSUPPORTED beyond).
 *
 * The host copies the job table into a pinned buffer; the device work is
 * {table copy, counter reset, persistent kernel}, captured once per kernel
 * variant into a hipGraph and replayed on `stream`, so sizes may change from
 * call to call without re-capture.  Two internal slots alternate: a call waits
 * (on the host) for the call two before it to finish before reusing its slot.
 * Results equal me_fullsearch / me_dcds_ex on each job.  One device per
 * process (ME_EUNSUPPORTED if the current device changes).
 */
typedef struct {
    const uint8_t *cur, *ref;
    int32_t width, height, pitch, n_pairs;
    int64_t pair_stride;
    me_mv *mv;
    uint32_t *sad, *nsp;
    const me_mv *start;    /* optional (DCDS only) */
    const uint8_t *orient; /* optional (DCDS only; needs start) */
    uint32_t *sse;         /* optional: compensated-block squared error, as me_search */
} me_job;

int me_batch(const me_job *jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range, void *stream);

/*
 * me_batch for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * results as me_batch, but the library allocates nothing on any call: the job
 * table and the tile counter live in one fixed device array of this library
 * (about 64 KiB, held by every GPU the library runs on until the process
 * ends), filled by small kernels on `stream` whose arguments carry the table.
 * At most 512 jobs and 2^30 work tiles per call (ME_EUNSUPPORTED beyond).
 * Every call on one GPU shares that array: calls must not overlap on a GPU
 * (issue them on one stream, or order their streams); overlapping calls race
 * and give undefined results.  The first call on a device looks the array up
 * (hipGetSymbolAddress); later calls only launch.
 */
int me_batch_noalloc(const me_job *jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range, void *stream);

/*
 * Autotuner: times every DCDS kernel layout (rows_per_lane x waves_per_group)
 * on the given batch with `reps` launches each (me_batch on `stream`,
 * synchronising it), then every tiles_per_grab with the fastest layout,
 * keeps the fastest configuration for (block, range class) via me_set_config,
 * and returns it with its time per launch in milliseconds (best, best_ms may
 * be NULL).
 * algo: ME_ALGO_DCDS or ME_ALGO_DCDS_S.  Outputs of the jobs are overwritten.
 *
 * me_autotune_save writes every result of this process (and every entry
 * loaded) as a text file keyed by GPU architecture and HIP runtime version.
 * me_autotune_load applies the entries that match the current device and
 * runtime; malformed lines are skipped and counted in *rejected, entries for
 * other hardware are ignored.  ME_EINVAL if the file cannot be opened (the
 * built-in defaults then stay in force).
 */
int me_autotune(const me_job *jobs, int32_t n_jobs, int32_t algo, int32_t block, int32_t range, int32_t reps,
                me_config *best, float *best_ms, void *stream);
int me_autotune_save(const char *path);
int me_autotune_load(const char *path, int32_t *applied, int32_t *rejected);

/*
 * Learned start proposer (this library's addition, not the paper's method).
 * A 4-layer convolutional network with bf16 storage and fp32 accumulation
 * reads a 4x-downsampled pair: input channels (cur4 - ref4)/32 and
 * (cur4 - 128)/64, where cur4, ref4 are 4x4 box means.  Layers: 3x3 conv
 * 2->16 (ReLU), 3x3 stride 2 16->32 (ReLU), 3x3 stride 2 32->32 (ReLU), 3x3
 * 32->3 (head u, v, o), all padded by 1, one head per 16x16 block.  Start
 * vector = clamp(rint(8 u), rint(8 v)) to +-range; first cross vertical when
 * o > 0.  Frames follow me_dcds (16x16 blocks).
 *
 * Parameters travel as one flat fp32 host vector of me_proposer_num_params()
 * values: per layer W[ky][kx][ci][co] then bias[co].  Training minimises,
 * averaged over blocks, huber(u - tx) + huber(v - ty) + 0.25 bce(o, |ty| >
 * |tx|) with t = target vector / 8, by Adam (0.9, 0.999, 1e-8) on fp32 master
 * weights.  Every reduction runs in a fixed order: repeated runs and resumed
 * runs are bit-identical.
 *
 * A proposer belongs to the device current at creation.  Calls on one
 * proposer must not overlap (they share its activation buffers, grown on
 * demand with hipMalloc).  create/init/set/get synchronise the device; the
 * others are stream-ordered.
 */
typedef struct me_proposer me_proposer;

int32_t me_proposer_num_params(void);
int me_proposer_create(me_proposer **out);                 /* all parameters 0             */
int me_proposer_destroy(me_proposer *p);
int me_proposer_init(me_proposer *p, uint64_t seed);       /* He-normal weights, 0 biases   */
int me_proposer_set_weights(me_proposer *p, const float *host, int32_t n); /* EINVAL if not finite */
int me_proposer_get_weights(me_proposer *p, float *host, int32_t n);
int me_proposer_get_grads(me_proposer *p, float *host, int32_t n);          /* last backward */
/* Adam moments (host, flat layout) and step count, for checkpoints.        */
int me_proposer_get_state(me_proposer *p, float *m, float *v, int64_t *step, int32_t n);
int me_proposer_set_state(me_proposer *p, const float *m, const float *v, int64_t step, int32_t n);
/* head: device fp32 [n_pairs][height/16][width/16][3].  forward and
 * train_step take at most 65535 pairs, height/4 <= 65535, and
 * n_pairs * (height/4) * (width/4) < 2^31 per call (16448 pairs of
 * 1920x1088; ME_EUNSUPPORTED beyond).                                      */
int me_proposer_forward(me_proposer *p, const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height,
                        int32_t pitch, int64_t pair_stride, int32_t n_pairs, float *head, void *stream);
/* Parameter gradients (me_proposer_get_grads) for a head gradient of the
 * same shape (device fp32), through the activations of the last forward.  */
int me_proposer_backward(me_proposer *p, const float *dhead, void *stream);
/* One Adam step on the loss above; target: device FS vectors, one per block;
 * loss: device float receiving the mean loss before the step.             */
int me_proposer_train_step(me_proposer *p, const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height,
                           int32_t pitch, int64_t pair_stride, int32_t n_pairs, const me_mv *target, float lr,
                           float *loss, void *stream);
/* Proposals: start (device, one per block) and orient (device bytes).     */
int me_proposer_infer(me_proposer *p, const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height,
                      int32_t pitch, int64_t pair_stride, int32_t n_pairs, int32_t range, me_mv *start,
                      uint8_t *orient, void *stream);
/* DCDS (16x16 blocks) from the proposer's starts with me_dcds_ex's fallback
 * rule; p == NULL runs plain DCDS.                                          */
int me_dcds_learned(me_proposer *p, const uint8_t *cur, const uint8_t *ref, int32_t width, int32_t height,
                    int32_t pitch, int64_t pair_stride, int32_t n_pairs, int32_t range, int32_t algo, me_mv *mv,
                    uint32_t *sad, uint32_t *nsp, void *stream);

/* Releases the library's device and pinned buffers, graphs and streams (no
 * batch may be in flight).  Later calls allocate them again.               */
int me_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* ME_H */
