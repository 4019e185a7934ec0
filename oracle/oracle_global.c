/*
 * Reference clusterer for the paper's second cluster definition -- TEST
 * INFRASTRUCTURE ONLY (loaded by the test suite; the product never does).
 *
 * Section 2, conditions (i), (ii) and (iii)(b), the dynamic global-time-
 * neighbourhood variant: a set C of hits is a cluster when
 *   (ii)  every two hits of C are joined by a path inside C whose steps are
 *         spatially 8-neighbouring (or identical) pixels -- no time limit on
 *         a step; and
 *   (iii)(b) every hit of C except the earliest has another hit of C whose
 *         ToA lies in [toa - dt, toa]: sorted by ToA, the hits of C leave no
 *         gap longer than dt; and
 *   (i)   C is maximal.
 * Read literally, maximality against single added hits does not partition
 * the hits (a hit s can be maximal alone while {s, x, y} is a cluster in
 * which y bridges the time gap between s and x); it is read as maximal under
 * inclusion.  Two clusters that share a hit have a union that is again
 * spatially connected and gap-free, so the maximal sets are disjoint and
 * cover every hit: a partition.
 *
 * Algorithm (deliberately plain): start with one part holding every hit and
 * refine until nothing changes:
 *   1. split every part where its ToAs, sorted, jump by more than dt;
 *   2. split every resulting segment into its spatial components
 *      (breadth-first search over hits of the segment at the 9 pixels around
 *      a hit, any ToA).
 * A set that is spatially connected and gap-free never straddles a split
 * (a gap of the part would be a gap of the set; a set of hits of one
 * segment that is connected lies in one component), so every cluster stays
 * inside one part, and the parts left when nothing splits any more are
 * themselves spatially connected and gap-free: they are the clusters.
 * Labels: the smallest input index of each cluster (the breadth-first
 * searches are seeded in input-index order).
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    uint64_t toa;
    uint16_t x, y, tot, reserved;
} og_hit;

typedef struct {  /* sort record: part, then ToA or pixel, then input index */
    int64_t part;
    uint64_t key;
    int64_t idx;
} og_rec;

static int cmp_rec(const void* pa, const void* pb)
{
    const og_rec* a = (const og_rec*)pa;
    const og_rec* b = (const og_rec*)pb;
    if (a->part != b->part) return a->part < b->part ? -1 : 1;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx < b->idx) ? -1 : (a->idx > b->idx) ? 1 : 0;
}

/* first record of recs[0..n) that is not below (part, key) */
static int64_t lower(const og_rec* recs, int64_t n, int64_t part, uint64_t key)
{
    int64_t a = 0, b = n;
    while (a < b) {
        int64_t m = a + (b - a) / 2;
        if (recs[m].part < part || (recs[m].part == part && recs[m].key < key)) a = m + 1; else b = m;
    }
    return a;
}

/* labels[n]: smallest input index of every hit's cluster; returns the number
 * of clusters, -2 when a hit lies off the sensor, -9 when out of memory. */
int64_t oracle_cluster_global(const og_hit* hits, int64_t n, uint32_t width, uint32_t height, uint64_t dt,
                              int32_t* labels)
{
    if (n < 0 || n > INT32_MAX || width == 0 || height == 0) return -1;
    for (int64_t i = 0; i < n; i++)
        if (hits[i].x >= width || hits[i].y >= height) return -2;
    if (n == 0) return 0;
    int64_t* part = malloc((size_t)n * sizeof(int64_t));
    int64_t* seg = malloc((size_t)n * sizeof(int64_t));
    og_rec* recs = malloc((size_t)n * sizeof(og_rec));
    int64_t* queue = malloc((size_t)n * sizeof(int64_t));
    if (!part || !seg || !recs || !queue) {
        free(part); free(seg); free(recs); free(queue);
        return -9;
    }
    for (int64_t i = 0; i < n; i++) part[i] = 0;
    int64_t n_parts = 1;
    for (;;) {
        /* 1. ToA gaps larger than dt split a part; a segment is named by the
         *    input index of its earliest hit */
        for (int64_t i = 0; i < n; i++) {
            recs[i].part = part[i];
            recs[i].key = hits[i].toa;
            recs[i].idx = i;
        }
        qsort(recs, (size_t)n, sizeof(og_rec), cmp_rec);
        int64_t name = recs[0].idx;
        for (int64_t k = 0; k < n; k++) {
            if (k > 0 && (recs[k].part != recs[k - 1].part || recs[k].key - recs[k - 1].key > dt))
                name = recs[k].idx;
            seg[recs[k].idx] = name;
        }
        /* 2. spatial components of every segment */
        for (int64_t i = 0; i < n; i++) {
            recs[i].part = seg[i];
            recs[i].key = (uint64_t)hits[i].y * width + hits[i].x;
            recs[i].idx = i;
        }
        qsort(recs, (size_t)n, sizeof(og_rec), cmp_rec);
        for (int64_t i = 0; i < n; i++) labels[i] = -1;
        int64_t count = 0;
        for (int64_t s0 = 0; s0 < n; s0++) {
            if (labels[s0] != -1) continue;
            count++;
            int64_t head = 0, tail = 0;
            labels[s0] = (int32_t)s0;
            queue[tail++] = s0;
            while (head < tail) {
                int64_t h = queue[head++];
                int64_t hx = hits[h].x, hy = hits[h].y;
                for (int64_t qy = hy - 1; qy <= hy + 1; qy++) {
                    if (qy < 0 || qy >= (int64_t)height) continue;
                    for (int64_t qx = hx - 1; qx <= hx + 1; qx++) {
                        if (qx < 0 || qx >= (int64_t)width) continue;
                        uint64_t q = (uint64_t)qy * width + (uint64_t)qx;
                        for (int64_t k = lower(recs, n, seg[h], q); k < n && recs[k].part == seg[h] && recs[k].key == q;
                             k++) {
                            int64_t j = recs[k].idx;
                            if (labels[j] == -1) {
                                labels[j] = (int32_t)s0;
                                queue[tail++] = j;
                            }
                        }
                    }
                }
            }
        }
        for (int64_t i = 0; i < n; i++) part[i] = labels[i];
        if (count == n_parts) break; /* parts only ever split: same count, same partition */
        n_parts = count;
    }
    free(part); free(seg); free(recs); free(queue);
    return n_parts;
}
