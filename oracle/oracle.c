/*
 * Reference clusterer for Timepix pixel hits -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the parity oracle.  It is plain, sequential, single-threaded C
 * written straight from the paper's definition of a cluster, and it shares no
 * code, header, table or helper with the GPU library.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.
 *
 * What it computes (paper, Section 2, conditions (i), (ii) and (iii)(a)):
 *   Two hits a != b are adjacent when
 *     - their pixels are 8-neighbours or the same pixel
 *       (Chebyshev distance max(|dx|,|dy|) <= 1; Section 4.1 searches a
 *       hit's own pixel and its eight neighbours), and
 *     - |toa(a) - toa(b)| <= dt  (the dynamic local-time-neighbourhood
 *       variant, Section 2 (iii)(a), read as "there is a path whose every
 *       step is spatially adjacent and time-close").
 *   Clusters are the connected components of that adjacency graph (the
 *   maximality condition (i) plus the path conditions (ii)/(iii)(a)); the
 *   frame-based Section 2.1 states the same graph formulation.
 *   Each hit's label is the smallest input index in its cluster.
 *
 * Algorithm (deliberately the obvious one):
 *   1. reject any hit with x >= width or y >= height;
 *   2. order all hits by (toa, input index);
 *   3. bucket that order per pixel (counting pass), so each pixel's hits
 *      are listed in time order;
 *   4. for i = 0..n-1 in input order, if hit i is unlabelled, breadth-first
 *      search from it: for a popped hit h, for each in-sensor pixel q within
 *      Chebyshev distance 1 of h (h's own pixel included), binary-search q's
 *      list for the first hit with toa >= toa(h) - dt (saturating) and label
 *      every unlabelled hit up to toa(h) + dt (saturating).  Every index
 *      below i is already labelled, so i is the smallest index of its
 *      component;
 *   5. features per cluster (the paper motivates them in Sections 1 and 6;
 *      it fixes no formula): size, sum of ToT, min/max ToA, sum of x*ToT and
 *      y*ToT, all exact integers, then the ToT-weighted centroid
 *      cx = (double)sum(x*ToT) / (double)sum(ToT)  (and cy likewise), or the
 *      plain mean of x (y) when every ToT of the cluster is zero.  Clusters
 *      are listed in ascending label order.
 *
 * dt is in ToA ticks and inclusive; dt = UINT64_MAX means no time limit.
 * Parity: pinned by brute force, closed forms, a library reduction and
 * invariant checks in the CPU test suite (no worked example is printed in the
 * paper to pin against).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t toa;
    uint16_t x, y, tot, reserved;
} oc_hit;

typedef struct {
    int32_t label;
    uint32_t size;
    uint64_t sum_tot, toa_min, toa_max, sum_x_tot, sum_y_tot;
    double cx, cy;
} oc_features;

enum { OC_OK = 0, OC_ERR_ARG = -1, OC_ERR_RANGE = -2, OC_ERR_NOMEM = -9 };

/* sort key of step 2: (toa, input index); the pair carries its own ToA, so
 * the comparison needs no outside state and concurrent calls are safe */
typedef struct {
    uint64_t toa;
    int64_t idx;
} oc_key;

static int cmp_time_then_index(const void* pa, const void* pb)
{
    const oc_key* a = (const oc_key*)pa;
    const oc_key* b = (const oc_key*)pb;
    if (a->toa < b->toa) return -1;
    if (a->toa > b->toa) return 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx) ? 1 : 0;
}

static uint64_t sat_sub(uint64_t a, uint64_t b) { return a > b ? a - b : 0; }
static uint64_t sat_add(uint64_t a, uint64_t b) { return (UINT64_MAX - a < b) ? UINT64_MAX : a + b; }

/* Returns OC_OK and fills labels[n], feats[*n_clusters]; OC_ERR_RANGE if a hit
 * lies outside the width x height sensor (outputs then untouched). */
int oracle_cluster(const oc_hit* hits, int64_t n, uint32_t width, uint32_t height,
                   uint64_t dt, int32_t* labels, oc_features* feats, int64_t* n_clusters)
{
    if (n < 0 || n > INT32_MAX || width == 0 || height == 0 || !n_clusters) return OC_ERR_ARG;
    if (n > 0 && (!hits || !labels)) return OC_ERR_ARG;
    for (int64_t i = 0; i < n; i++)
        if (hits[i].x >= width || hits[i].y >= height) return OC_ERR_RANGE;
    *n_clusters = 0;
    if (n == 0) return OC_OK;

    int64_t npix = (int64_t)width * (int64_t)height;
    int64_t* order = malloc((size_t)n * sizeof(int64_t));
    int64_t* start = calloc((size_t)npix + 1, sizeof(int64_t));
    int64_t* fill = malloc((size_t)npix * sizeof(int64_t));
    int64_t* list = malloc((size_t)n * sizeof(int64_t));
    int64_t* queue = malloc((size_t)n * sizeof(int64_t));
    if (!order || !start || !fill || !list || !queue) {
        free(order); free(start); free(fill); free(list); free(queue);
        return OC_ERR_NOMEM;
    }

    /* step 2: time order, ties by input index */
    oc_key* keys = malloc((size_t)n * sizeof(oc_key));
    if (!keys) {
        free(order); free(start); free(fill); free(list); free(queue);
        return OC_ERR_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) {
        keys[i].toa = hits[i].toa;
        keys[i].idx = i;
    }
    qsort(keys, (size_t)n, sizeof(oc_key), cmp_time_then_index);
    for (int64_t k = 0; k < n; k++) order[k] = keys[k].idx;
    free(keys);

    /* step 3: per-pixel lists in time order */
    for (int64_t i = 0; i < n; i++)
        start[(int64_t)hits[i].y * width + hits[i].x + 1]++;
    for (int64_t p = 0; p < npix; p++) start[p + 1] += start[p];
    memcpy(fill, start, (size_t)npix * sizeof(int64_t));
    for (int64_t k = 0; k < n; k++) {
        int64_t i = order[k];
        int64_t p = (int64_t)hits[i].y * width + hits[i].x;
        list[fill[p]++] = i;
    }

    /* step 4: breadth-first search over the adjacency relation */
    for (int64_t i = 0; i < n; i++) labels[i] = -1;
    for (int64_t seed = 0; seed < n; seed++) {
        if (labels[seed] != -1) continue;
        int64_t head = 0, tail = 0;
        labels[seed] = (int32_t)seed;
        queue[tail++] = seed;
        while (head < tail) {
            int64_t h = queue[head++];
            int64_t hx = hits[h].x, hy = hits[h].y;
            uint64_t lo = sat_sub(hits[h].toa, dt), hi = sat_add(hits[h].toa, dt);
            for (int64_t qy = hy - 1; qy <= hy + 1; qy++) {
                if (qy < 0 || qy >= (int64_t)height) continue;
                for (int64_t qx = hx - 1; qx <= hx + 1; qx++) {
                    if (qx < 0 || qx >= (int64_t)width) continue;
                    int64_t q = qy * width + qx;
                    /* first entry of q's list with toa >= lo */
                    int64_t a = start[q], b = start[q + 1];
                    while (a < b) {
                        int64_t m = a + (b - a) / 2;
                        if (hits[list[m]].toa < lo) a = m + 1; else b = m;
                    }
                    for (int64_t k = a; k < start[q + 1] && hits[list[k]].toa <= hi; k++) {
                        int64_t j = list[k];
                        if (labels[j] == -1) {
                            labels[j] = (int32_t)seed;
                            queue[tail++] = j;
                        }
                    }
                }
            }
        }
    }

    /* step 5: features, accumulated per label in input order */
    if (feats) {
        uint32_t* size = calloc((size_t)n, sizeof(uint32_t));
        uint64_t* acc = malloc((size_t)n * 7 * sizeof(uint64_t));
        if (!size || !acc) {
            free(size); free(acc);
            free(order); free(start); free(fill); free(list); free(queue);
            return OC_ERR_NOMEM;
        }
        uint64_t *st = acc, *tmin = acc + n, *tmax = acc + 2 * n, *sxt = acc + 3 * n,
                 *syt = acc + 4 * n, *sx = acc + 5 * n, *sy = acc + 6 * n;
        for (int64_t i = 0; i < n; i++) {
            st[i] = sxt[i] = syt[i] = sx[i] = sy[i] = 0;
            tmin[i] = UINT64_MAX;
            tmax[i] = 0;
        }
        for (int64_t i = 0; i < n; i++) {
            int64_t c = labels[i];
            uint64_t x = hits[i].x, y = hits[i].y, t = hits[i].tot;
            size[c] += 1;
            st[c] += t;
            if (hits[i].toa < tmin[c]) tmin[c] = hits[i].toa;
            if (hits[i].toa > tmax[c]) tmax[c] = hits[i].toa;
            sxt[c] += x * t;
            syt[c] += y * t;
            sx[c] += x;
            sy[c] += y;
        }
        int64_t k = 0;
        for (int64_t c = 0; c < n; c++) {
            if (labels[c] != c) continue;
            oc_features* f = &feats[k++];
            f->label = (int32_t)c;
            f->size = size[c];
            f->sum_tot = st[c];
            f->toa_min = tmin[c];
            f->toa_max = tmax[c];
            f->sum_x_tot = sxt[c];
            f->sum_y_tot = syt[c];
            if (st[c] > 0) {
                f->cx = (double)sxt[c] / (double)st[c];
                f->cy = (double)syt[c] / (double)st[c];
            } else {
                f->cx = (double)sx[c] / (double)size[c];
                f->cy = (double)sy[c] / (double)size[c];
            }
        }
        *n_clusters = k;
        free(size);
        free(acc);
    } else {
        int64_t k = 0;
        for (int64_t c = 0; c < n; c++) k += (labels[c] == c);
        *n_clusters = k;
    }

    free(order); free(start); free(fill); free(list); free(queue);
    return OC_OK;
}
