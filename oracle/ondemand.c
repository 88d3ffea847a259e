/*
 * CPU on-demand baseline -- TEST AND BENCHMARK INFRASTRUCTURE.
 *
 * The paper's per-frame method done on the host with the oracle's own
 * routines and no other optimisation: mark the blocks the frame reads
 * (Method: Mark, with the whole filter footprint), list them, decode only
 * those MCUs by random access into the original entropy-coded segment from
 * a per-MCU index of start bits and DC predictors (Implementation details:
 * Indexing Table; the index is the oracle's own, recorded by a sequential
 * pass before timing), turn them into texels (fp64 IDCT by definition,
 * single rounding) and resolve (Method: Resolve).  Work items and pixel
 * rows are split over n threads (pthreads).  Shares no code with the GPU
 * library.
 */
#define _POSIX_C_SOURCE 199309L
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include "oracle.h"

static double now_s(void) {
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

typedef struct {
    /* scene */
    int n_tex;
    const int32_t *tex_first, *tex_count, *lev_w, *lev_h;
    const uint32_t *blk_base;
    int n_levels;
    uint64_t n_blocks;
    const orc_jpeg *const *jpegs;
    const uint64_t *const *mcu_bit;
    const int32_t *const *pred;
    uint8_t *const *level_rgb;
    /* frame */
    const orc_gpixel *g;
    int64_t n_px;
    int filter;
    uint32_t *frame;
    uint8_t *vis;
    uint32_t *list;
    uint64_t n_list;
    int n_threads;
    int failed;
} od_job;

typedef struct {
    od_job *job;
    int t;
    int64_t bad;
} od_arg;

static void run_threads(od_job *job, void *(*fn)(void *), od_arg *args) {
    pthread_t th[256];
    int n = job->n_threads;
    for (int t = 0; t < n; t++) {
        args[t].job = job; args[t].t = t; args[t].bad = 0;
        if (t) pthread_create(&th[t], NULL, fn, &args[t]);
    }
    fn(&args[0]);
    for (int t = 1; t < n; t++) pthread_join(th[t], NULL);
}

static void *mark_part(void *p) {
    od_arg *a = (od_arg *)p;
    od_job *J = a->job;
    int64_t lo = J->n_px * a->t / J->n_threads, hi = J->n_px * (a->t + 1) / J->n_threads;
    /* each thread marks into the shared byte map; orc_mark only ever
     * stores 1, so the threads' stores do not conflict in value */
    a->bad = orc_mark(J->n_tex, J->tex_first, J->tex_count, J->lev_w, J->lev_h, J->blk_base, J->g + lo, hi - lo,
                      J->filter, J->vis);
    return NULL;
}

static int level_of_block(const od_job *J, uint64_t b) {
    int lo = 0, hi = J->n_levels - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if ((uint64_t)J->blk_base[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

/* Decode one MCU through the index and copy its texels into the level image. */
static int decode_mcu_into(const od_job *J, int L, int mx, int my) {
    const orc_jpeg *j = J->jpegs[L];
    int64_t info[10];
    orc_info(j, info);
    const int w = (int)info[0], h = (int)info[1], sampling = (int)info[2], mcu_cols = (int)info[3];
    const int n_du = (int)info[6];
    const int ms = sampling == 420 ? 16 : 8;
    const int m = my * mcu_cols + mx;
    int16_t coef[6 * 64];
    uint8_t tile[16 * 16 * 3];
    uint64_t end;
    if (orc_decode_mcu_at(j, J->mcu_bit[L][m], J->pred[L] + 3 * m, coef, &end) != ORC_OK) return -1;
    if (end != J->mcu_bit[L][m + 1]) return -1;
    (void)n_du;
    orc_mcu_pixels(j, coef, tile, NULL);
    uint8_t *img = J->level_rgb[L];
    for (int ty = 0; ty < ms; ty++)
        for (int tx = 0; tx < ms; tx++) {
            const int x = mx * ms + tx, y = my * ms + ty;
            if (x >= w || y >= h) continue;
            memcpy(img + ((size_t)y * w + x) * 3, tile + ((size_t)ty * ms + tx) * 3, 3);
        }
    return 0;
}

static void *decode_part(void *p) {
    od_arg *a = (od_arg *)p;
    od_job *J = a->job;
    /* blocks dealt round-robin, so that long and short regions spread */
    for (uint64_t i = (uint64_t)a->t; i < J->n_list; i += (uint64_t)J->n_threads) {
        const uint64_t b = J->list[i];
        const int L = level_of_block(J, b);
        const uint64_t r = b - J->blk_base[L];
        const int bc = (J->lev_w[L] + 15) / 16;
        const int bx = (int)(r % (uint64_t)bc), by = (int)(r / (uint64_t)bc);
        int64_t info[10];
        orc_info(J->jpegs[L], info);
        if (info[2] == 420) {
            if (decode_mcu_into(J, L, bx, by)) a->bad++;
        } else {
            for (int q = 0; q < 4; q++) {
                const int mx = 2 * bx + (q & 1), my = 2 * by + (q >> 1);
                if (mx >= info[3] || my >= info[4]) continue;
                if (decode_mcu_into(J, L, mx, my)) a->bad++;
            }
        }
    }
    return NULL;
}

static void *resolve_part(void *p) {
    od_arg *a = (od_arg *)p;
    od_job *J = a->job;
    int64_t lo = J->n_px * a->t / J->n_threads, hi = J->n_px * (a->t + 1) / J->n_threads;
    a->bad = orc_resolve(J->n_tex, J->tex_first, J->tex_count, J->lev_w, J->lev_h,
                         (const uint8_t *const *)J->level_rgb, NULL, J->g + lo, hi - lo, J->filter, J->frame + lo,
                         NULL);
    return NULL;
}

int64_t orc_ondemand_frame(int n_tex, const int32_t *tex_first, const int32_t *tex_count, int n_levels,
                           const int32_t *lev_w, const int32_t *lev_h, const uint32_t *blk_base, uint64_t n_blocks,
                           const orc_jpeg *const *jpegs, const uint64_t *const *mcu_bit, const int32_t *const *pred,
                           uint8_t *const *level_rgb, const orc_gpixel *g, int64_t n_px, int filter,
                           uint32_t *frame, uint8_t *vis, uint32_t *list, int n_threads, double times[4],
                           uint64_t *n_decoded) {
    if (n_threads < 1 || n_threads > 256 || !vis || !list || !frame) return -1;
    od_job J = {n_tex, tex_first, tex_count, lev_w, lev_h, blk_base, n_levels, n_blocks, jpegs, mcu_bit, pred,
                level_rgb, g, n_px, filter, frame, vis, list, 0, n_threads, 0};
    od_arg args[256];
    int64_t bad = 0;
    double t0 = now_s();
    memset(vis, 0, n_blocks);
    run_threads(&J, mark_part, args);
    for (int t = 0; t < n_threads; t++) bad += args[t].bad;
    double t1 = now_s();
    uint64_t n = 0;
    for (uint64_t b = 0; b < n_blocks; b++)
        if (vis[b]) list[n++] = (uint32_t)b;
    J.n_list = n;
    double t2 = now_s();
    run_threads(&J, decode_part, args);
    for (int t = 0; t < n_threads; t++) bad += args[t].bad;
    double t3 = now_s();
    run_threads(&J, resolve_part, args);
    double t4 = now_s();
    if (times) {
        times[0] = t1 - t0; times[1] = t2 - t1; times[2] = t3 - t2; times[3] = t4 - t3;
    }
    if (n_decoded) *n_decoded = n;
    return bad;
}
