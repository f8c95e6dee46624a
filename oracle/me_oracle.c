/*
 * CPU oracle for block-matching motion estimation with full search (FS) and
 * the directional cross diamond search (DCDS) of Jia & Zhang.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * statement of what the GPU library computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library: the pattern
 * tables below are written out here a second time on purpose.
 *
 * Conventions (each one a reading of the paper, restated where it is used):
 *   - A motion vector (dx, dy) means: the reference block sits at
 *     (x0 + dx, y0 + dy) when the current block sits at (x0, y0);
 *     +x is to the right, +y is down (the paper gives no axis convention).
 *   - The block distortion measure is SAD.  The paper uses MAD = SAD / B^2
 *     (§II-C, §IV); the divisor is a constant, so the argmin and every tie
 *     are the same.
 *   - The candidate set V of a block is every (dx, dy) with |dx|, |dy| <= R
 *     whose displaced block lies wholly inside the reference frame
 *     (restricted motion vectors, no padding).  A point outside V is neither
 *     evaluated nor counted.
 *   - NSP counts distinct evaluated points.
 *
 * Build: gcc -O2 -std=c99 -shared -fPIC (scalar, no intrinsics, no OpenMP).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -3

/* Pattern variants the oracle knows.                                       */
#define OR_VARIANT_DCDS 0   /* plain DCDS, §III-B Steps 1-4                */
#define OR_VARIANT_DCDS_S 1 /* simplified DCDS, §IV-C                       */

/* ------------------------------------------------------------------------ */
/* The three directional patterns of §III-A (Fig. 4, reconstructed from the */
/* text: HCSP has seven points and spans 5x1 horizontally plus the two      */
/* vertical neighbours; HDSP/VDSP have five points: the centre, two distant */
/* points at distance 2 on the long wing and two near points at distance 1  */
/* on the short wing).  The centre comes first, so a tie with the centre    */
/* keeps the centre.  Among the other points the scan order is the listed   */
/* order; the paper does not fix it.                                         */
/* ------------------------------------------------------------------------ */
typedef struct { int dx, dy; } pt;

static const pt HCSP[7] = {{0, 0}, {-1, 0}, {1, 0}, {-2, 0}, {2, 0}, {0, -1}, {0, 1}};
/* The transposed cross, used only when a learned start asks for a vertical
 * first pattern (not part of the paper's method).                          */
static const pt VCSP[7] = {{0, 0}, {0, -1}, {0, 1}, {0, -2}, {0, 2}, {-1, 0}, {1, 0}};
static const pt HDSP[5] = {{0, 0}, {-2, 0}, {2, 0}, {0, -1}, {0, 1}};
static const pt VDSP[5] = {{0, 0}, {0, -2}, {0, 2}, {-1, 0}, {1, 0}};
/* Middle points: distance 1 on the long wing, outside the pattern itself.   */
static const pt MID_H[2] = {{-1, 0}, {1, 0}};
static const pt MID_V[2] = {{0, -1}, {0, 1}};

enum { PAT_H = 0, PAT_V = 1 };

/* ------------------------------------------------------------------------ */
/* Evaluation context: the set S of evaluated points (Eq. 3), with the      */
/* distortion of each, over the (2R+1)^2 window.                             */
/* ------------------------------------------------------------------------ */
typedef int64_t (*cost_fn)(void *user, int dx, int dy);
typedef int (*valid_fn)(void *user, int dx, int dy);

typedef struct {
    int R;
    cost_fn cost;
    valid_fn valid;
    void *user;
    uint8_t *in_s;  /* 1 if the point is in S                     */
    int64_t *bdm;   /* its distortion, meaningful where in_s == 1 */
    int nsp;        /* |S|                                        */
    uint32_t *trace; /* optional: |S| after each pattern evaluation */
    int trace_n, trace_cap;
} search_state;

/* Records |S| after one pattern (or Step-4 set) has been evaluated.        */
static void note_step(search_state *st)
{
    if (st->trace && st->trace_n < st->trace_cap)
        st->trace[st->trace_n] = (uint32_t)st->nsp;
    st->trace_n += 1;
}

static int widx(const search_state *st, int dx, int dy)
{
    return (dy + st->R) * (2 * st->R + 1) + (dx + st->R);
}

static int in_window(const search_state *st, int dx, int dy)
{
    return dx >= -st->R && dx <= st->R && dy >= -st->R && dy <= st->R;
}

/* Returns 0 when (dx, dy) is outside V, else 1 and the point's distortion.
 * A point met for the first time is added to S and counted.               */
static int eval_point(search_state *st, int dx, int dy, int64_t *out)
{
    if (!in_window(st, dx, dy) || !st->valid(st->user, dx, dy))
        return 0;
    int k = widx(st, dx, dy);
    if (!st->in_s[k]) {
        st->bdm[k] = st->cost(st->user, dx, dy);
        st->in_s[k] = 1;
        st->nsp += 1;
    }
    *out = st->bdm[k];
    return 1;
}

/* Current BMP of one pattern placed at c: scan the points in list order and
 * keep the first strictly smaller distortion.  The centre is always in V.   */
static pt pattern_bmp(search_state *st, pt c, const pt *pat, int n, int64_t *best_out)
{
    pt best = c;
    int64_t best_d = 0;
    int have = 0;
    for (int i = 0; i < n; i++) {
        int64_t d;
        pt q = {c.dx + pat[i].dx, c.dy + pat[i].dy};
        if (!eval_point(st, q.dx, q.dy, &d))
            continue;
        if (!have || d < best_d) {
            best = q;
            best_d = d;
            have = 1;
        }
    }
    *best_out = best_d;
    return best;
}

static int same_pt(pt a, pt b) { return a.dx == b.dx && a.dy == b.dy; }

/* ------------------------------------------------------------------------ */
/* DCDS, §III-B.  start: the centre of the first pattern (the origin in the  */
/* paper's method).  first_vertical selects the transposed cross (learned    */
/* start only).  Returns the final motion vector and its distortion.         */
/* ------------------------------------------------------------------------ */
static pt dcds_from(search_state *st, pt start, int first_vertical, int variant, int64_t *bdm_out)
{
    int64_t d;
    /* Step 1: the cross search pattern centred at the start.              */
    pt c = start;
    pt b = pattern_bmp(st, c, first_vertical ? VCSP : HCSP, 7, &d);
    note_step(st);
    if (same_pt(b, c)) {
        /* Half-way stop: the centre is the best-matched point.             */
        *bdm_out = d;
        return c;
    }
    /* Switching strategy one: a BMP in the horizontal direction selects the
     * horizontal diamond, anything else the vertical one.                  */
    int p = (b.dy == c.dy) ? PAT_H : PAT_V;
    c = b;

    /* Steps 2 and 3: re-centre the current pattern on the BMP until the
     * centre wins.  The distortion at the centre strictly decreases each
     * time, so the loop ends; the guard only bounds a broken cost.          */
    int guard = (2 * st->R + 1) * (2 * st->R + 1) + 1;
    for (;;) {
        b = pattern_bmp(st, c, p == PAT_H ? HDSP : VDSP, 5, &d);
        note_step(st);
        if (same_pt(b, c) || --guard <= 0)
            break;
        /* Switching strategy two: a near point (distance 1) switches to the
         * other directional diamond; a distant point keeps the pattern.    */
        if (abs(b.dx - c.dx) + abs(b.dy - c.dy) == 1)
            p = (p == PAT_H) ? PAT_V : PAT_H;
        c = b;
    }

    /* Step 4: the BMP among the centre and the two middle points of the
     * current pattern is the motion vector.                                 */
    const pt *mid = (p == PAT_H) ? MID_H : MID_V;
    if (variant == OR_VARIANT_DCDS_S) {
        /* Simplified DCDS (§IV-C): the distortions of the two distant points
         * are compared, and only the middle point on the side of the smaller
         * one is checked; a tie goes to the negative side.  Reading: when a
         * distant point lies outside V there is no comparison to use, so both
         * middle points are checked, as in plain DCDS.                      */
        pt dn = {c.dx + 2 * mid[0].dx, c.dy + 2 * mid[0].dy};
        pt dp = {c.dx + 2 * mid[1].dx, c.dy + 2 * mid[1].dy};
        int64_t sn = 0, sp = 0;
        int vn = eval_point(st, dn.dx, dn.dy, &sn);
        int vp = eval_point(st, dp.dx, dp.dy, &sp);
        pt list[3] = {{0, 0}, mid[0], mid[1]};
        int n = 3;
        if (vn && vp) {
            list[1] = (sp < sn) ? mid[1] : mid[0];
            n = 2;
        }
        b = pattern_bmp(st, c, list, n, &d);
    } else {
        pt list[3] = {{0, 0}, mid[0], mid[1]};
        b = pattern_bmp(st, c, list, 3, &d);
    }
    note_step(st);
    *bdm_out = d;
    return b;
}

/* Learned start (not part of the paper's method).  Plain DCDS runs first,
 * from the origin; call its result p.  Then the proposed start s is probed;
 * if it beats the origin, DCDS runs a second time, with its first cross
 * (HCSP, or its transpose when orient_v) centred at s, over the same set S:
 * a point already in S keeps its distortion and is not counted again.  The
 * result is the better of the two searches' results (a tie keeps p), so it
 * is never worse than plain DCDS's.                                          */
static pt dcds_seeded(search_state *st, pt s, int orient_v, int variant, int64_t *bdm_out)
{
    int64_t dp, ds, dq;
    pt origin = {0, 0};
    pt p = dcds_from(st, origin, 0, variant, &dp);
    *bdm_out = dp;
    if (same_pt(s, origin) || !eval_point(st, s.dx, s.dy, &ds) || ds >= st->bdm[widx(st, 0, 0)])
        return p;
    pt q = dcds_from(st, s, orient_v, variant, &dq);
    if (dq < dp) {
        *bdm_out = dq;
        return q;
    }
    return p;
}

/* ------------------------------------------------------------------------ */
/* Frame pair context: SAD of one candidate (§I problem statement, BDM).    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *cur, *ref;
    int W, H, pitch, B, x0, y0;
} frame_ctx;

static int64_t frame_sad(void *user, int dx, int dy)
{
    const frame_ctx *f = (const frame_ctx *)user;
    int64_t s = 0;
    for (int v = 0; v < f->B; v++) {
        const uint8_t *c = f->cur + (size_t)(f->y0 + v) * f->pitch + f->x0;
        const uint8_t *r = f->ref + (size_t)(f->y0 + dy + v) * f->pitch + f->x0 + dx;
        for (int u = 0; u < f->B; u++)
            s += abs((int)c[u] - (int)r[u]);
    }
    return s;
}

static int frame_valid(void *user, int dx, int dy)
{
    const frame_ctx *f = (const frame_ctx *)user;
    int x = f->x0 + dx, y = f->y0 + dy;
    return x >= 0 && y >= 0 && x <= f->W - f->B && y <= f->H - f->B;
}

static int check_frame_args(const uint8_t *cur, const uint8_t *ref, int W, int H, int pitch, int B, int R)
{
    if (!cur || !ref || W <= 0 || H <= 0 || B <= 0 || R < 0 || pitch < W)
        return OR_EINVAL;
    if (W % B || H % B)
        return OR_EINVAL;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Full search: every point of V; the motion vector is the lexicographic    */
/* minimum of (SAD, |dx|+|dy|, dy, dx).  The paper assumes a unique FS      */
/* optimum; this tie order (centre-biased, then top-most, then left-most)   */
/* is the reading taken here.                                                 */
/* mv: 2 int16 per block (dx, dy); sad, nsp: one uint32 per block; raster. */
/* ------------------------------------------------------------------------ */
int oracle_fs(const uint8_t *cur, const uint8_t *ref, int W, int H, int pitch, int B, int R,
              int16_t *mv, uint32_t *sad, uint32_t *nsp)
{
    int rc = check_frame_args(cur, ref, W, H, pitch, B, R);
    if (rc)
        return rc;
    int bw = W / B, bh = H / B;
    for (int j = 0; j < bh; j++) {
        for (int i = 0; i < bw; i++) {
            frame_ctx f = {cur, ref, W, H, pitch, B, i * B, j * B};
            int have = 0, n = 0;
            int64_t bs = 0;
            int bx = 0, by = 0;
            for (int dy = -R; dy <= R; dy++) {
                for (int dx = -R; dx <= R; dx++) {
                    if (!frame_valid(&f, dx, dy))
                        continue;
                    n++;
                    int64_t s = frame_sad(&f, dx, dy);
                    int l1 = abs(dx) + abs(dy), bl1 = abs(bx) + abs(by);
                    int better = !have || s < bs ||
                                 (s == bs && (l1 < bl1 || (l1 == bl1 && (dy < by || (dy == by && dx < bx)))));
                    if (better) {
                        have = 1;
                        bs = s;
                        bx = dx;
                        by = dy;
                    }
                }
            }
            int k = j * bw + i;
            mv[2 * k] = (int16_t)bx;
            mv[2 * k + 1] = (int16_t)by;
            sad[k] = (uint32_t)bs;
            nsp[k] = (uint32_t)n;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* DCDS over a frame pair.                                                    */
/*   start, orient: NULL for the paper's method (origin start).  Otherwise    */
/*   one start vector (2 int16) and one orientation byte (0 = horizontal     */
/*   cross, 1 = vertical cross) per block; each start is clamped into V.     */
/*   variant: OR_VARIANT_DCDS or OR_VARIANT_DCDS_S.                          */
/* ------------------------------------------------------------------------ */
int oracle_dcds(const uint8_t *cur, const uint8_t *ref, int W, int H, int pitch, int B, int R,
                const int16_t *start, const uint8_t *orient, int variant,
                int16_t *mv, uint32_t *sad, uint32_t *nsp)
{
    int rc = check_frame_args(cur, ref, W, H, pitch, B, R);
    if (rc)
        return rc;
    int n = (2 * R + 1) * (2 * R + 1);
    uint8_t *in_s = (uint8_t *)malloc((size_t)n);
    int64_t *bdm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!in_s || !bdm) {
        free(in_s);
        free(bdm);
        return OR_ENOMEM;
    }
    int bw = W / B, bh = H / B;
    for (int j = 0; j < bh; j++) {
        for (int i = 0; i < bw; i++) {
            int k = j * bw + i;
            frame_ctx f = {cur, ref, W, H, pitch, B, i * B, j * B};
            search_state st = {R, frame_sad, frame_valid, &f, in_s, bdm, 0, NULL, 0, 0};
            memset(in_s, 0, (size_t)n);
            int64_t d;
            pt r;
            if (start) {
                int lox = -R, hix = R, loy = -R, hiy = R;
                if (-f.x0 > lox) lox = -f.x0;
                if (W - B - f.x0 < hix) hix = W - B - f.x0;
                if (-f.y0 > loy) loy = -f.y0;
                if (H - B - f.y0 < hiy) hiy = H - B - f.y0;
                pt s = {start[2 * k], start[2 * k + 1]};
                s.dx = s.dx < lox ? lox : (s.dx > hix ? hix : s.dx);
                s.dy = s.dy < loy ? loy : (s.dy > hiy ? hiy : s.dy);
                r = dcds_seeded(&st, s, orient ? (orient[k] != 0) : 0, variant, &d);
            } else {
                pt o = {0, 0};
                r = dcds_from(&st, o, 0, variant, &d);
            }
            mv[2 * k] = (int16_t)r.dx;
            mv[2 * k + 1] = (int16_t)r.dy;
            sad[k] = (uint32_t)d;
            nsp[k] = (uint32_t)st.nsp;
        }
    }
    free(in_s);
    free(bdm);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* DCDS over a caller-given cost surface, as in the ideal-condition analysis */
/* of §III-C (Table VII): cost[(dy+R)*(2R+1) + (dx+R)] is the distortion of  */
/* (dx, dy); valid (optional, same layout) marks the points of V, otherwise  */
/* the whole window is V.  Optional outputs: the set S as 0/1 flags in the   */
/* same layout, and |S| after each evaluated pattern (Step 1, every Step-2/3 */
/* diamond, Step 4; the seeded probes are not a pattern).                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int R;
    const int64_t *cost;
    const uint8_t *valid;
} surface_ctx;

static int64_t surface_cost(void *user, int dx, int dy)
{
    const surface_ctx *s = (const surface_ctx *)user;
    return s->cost[(dy + s->R) * (2 * s->R + 1) + (dx + s->R)];
}

static int surface_valid(void *user, int dx, int dy)
{
    const surface_ctx *s = (const surface_ctx *)user;
    return s->valid ? s->valid[(dy + s->R) * (2 * s->R + 1) + (dx + s->R)] != 0 : 1;
}

int oracle_dcds_surface(int R, const int64_t *cost, const uint8_t *valid, int start_dx, int start_dy,
                        int use_start, int orient_v, int variant, int16_t *mv, int64_t *bdm_out,
                        uint32_t *nsp, uint8_t *s_out, uint32_t *trace, int trace_cap, int *trace_n)
{
    if (R < 1 || !cost || !mv || !bdm_out || !nsp)
        return OR_EINVAL;
    int n = (2 * R + 1) * (2 * R + 1);
    uint8_t *in_s = (uint8_t *)calloc((size_t)n, 1);
    int64_t *bdm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!in_s || !bdm) {
        free(in_s);
        free(bdm);
        return OR_ENOMEM;
    }
    surface_ctx sc = {R, cost, valid};
    search_state st = {R, surface_cost, surface_valid, &sc, in_s, bdm, 0, trace, 0, trace_cap};
    int64_t d;
    pt r;
    if (use_start) {
        pt s = {start_dx, start_dy};
        r = dcds_seeded(&st, s, orient_v, variant, &d);
    } else {
        pt o = {0, 0};
        r = dcds_from(&st, o, 0, variant, &d);
    }
    mv[0] = (int16_t)r.dx;
    mv[1] = (int16_t)r.dy;
    *bdm_out = d;
    *nsp = (uint32_t)st.nsp;
    if (s_out)
        memcpy(s_out, in_s, (size_t)n);
    if (trace_n)
        *trace_n = st.trace_n;
    free(in_s);
    free(bdm);
    return OR_OK;
}

/* SAD of one candidate, exposed so tests can pin the distortion itself.     */
int64_t oracle_block_sad(const uint8_t *cur, const uint8_t *ref, int W, int H, int pitch, int B,
                         int x0, int y0, int dx, int dy)
{
    frame_ctx f = {cur, ref, W, H, pitch, B, x0, y0};
    if (!frame_valid(&f, dx, dy))
        return -1;
    return frame_sad(&f, dx, dy);
}
