/*
 * oracle.c -- plain, slow CPU oracle for the buffer k-d tree exact kNN query.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It shares no code, header or table with the HIP path.
 *
 * Paper: Gieseke, Oancea, Mahabal, Igel, Heskes, "Bigger Buffer k-d Trees on
 * Multi-Many-Core Systems" (arXiv 1512.02831).
 *
 * Contents (each function names the passage it follows):
 *   orc_build          canonical median split tree      Section 2.3 (construction), Section 3.1
 *   orc_brute_f64      exhaustive kNN in float64        Section 2.2 (problem statement)
 *   orc_brute_f32c     exhaustive kNN, float32 keys     Section 2.2 + the float32 distance reading
 *   orc_kdtree_f64     classical k-d tree kNN search    Section 2.3 (search), timed CPU baseline
 *   orc_replay_*       LazySearch schedule replay       Algorithm 1 (Section 2.4), Section 3.2
 *   orc_traverse_f32   one query's leaf sequence        Section 2.3 search phases, stackless form
 *   orc_chunk_bounds   leaf-structure chunk bounds      Section 3.2 ("Processing the Leaf Structure")
 *   orc_leaf_chunks    leaf-aligned chunk plan          Section 3.2 (chunks of whole leaves)
 *   orc_build_rules    variant tree: longest-side split Section 2.3 (footnote on splitting rules)
 *   orc_node_boxes     node bounding boxes              Section 2.3 (search phase, pruning)
 *   orc_traverse_*_rules  walk with per-node dimensions and bounding-box pruning
 *
 * Readings of the paper used here (the paper is silent or loose on them):
 *   - "height h" = h internal levels, 2^h leaves; h = 0 is a single leaf.
 *   - a node holding c points orders them by (coordinate, original index);
 *     the left child takes the floor(c/2) smallest, split value = coordinate
 *     of the smallest point on the right; a query goes left iff q[dim] < split.
 *   - leaf points are stored in ascending original index.
 *   - distances: float32 inputs; float32 keys use t = q_j - x_j rounded to
 *     float32, acc = fmaf(t, t, acc) for j = 0..d-1 starting from +0.
 *   - hyperplane test: t = q[dim] - split (float32), h2 = t*t (float32);
 *     the far child is visited iff h2 <= current k-th best squared distance
 *     (+inf while fewer than k candidates are known).
 *   - key = (bits of float32 d2) << 32 | original index; the k smallest keys
 *     form a query's list, so ties are broken by smaller index.
 *   - queues are FIFO; a fetch takes reinsert first, then input; half-full
 *     means a buffer holds >= ceil(B/2) indices; processed indices are
 *     appended to reinsert leaf by leaf (ascending leaf), in buffer order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EMPTY_KEY 0x7F800000FFFFFFFFull
#define ORC_FRESH (-2)
#define ORC_DONE (-1)

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Canonical build (Section 2.3 construction rule; Section 3.1 host build).  */

typedef struct {
    float v;
    int32_t i;
} vi_t;

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int less_vi(const vi_t *x, const vi_t *y)
{
    return x->v < y->v || (x->v == y->v && x->i < y->i);
}

/*
 * Selection of rank r under the total order (value, index) (Hoare's FIND):
 * afterwards a[r] is the element of rank r, every element before it is
 * smaller and every element after it larger.  Only which elements land on
 * either side matters to the build, and that is fixed by the order alone, so
 * any exact selection gives the same tree (the paper's host build uses
 * linear-time median selection).  The pivot position is drawn from a
 * fixed-seed generator, so the expected cost is linear for every input.
 */
static void select_vi(vi_t *a, int64_t c, int64_t r)
{
    int64_t lo = 0, hi = c - 1;
    uint64_t state = 0x9E3779B97F4A7C15ull ^ (uint64_t)c;
    while (lo < hi) {
        state = state * 6364136223846793005ull + 1442695040888963407ull;
        const int64_t pi = lo + (int64_t)((state >> 33) % (uint64_t)(hi - lo + 1));
        const vi_t pv = a[pi];
        a[pi] = a[hi];
        a[hi] = pv;
        int64_t store = lo;
        for (int64_t i = lo; i < hi; i++) {
            if (less_vi(&a[i], &pv)) {
                const vi_t t = a[i];
                a[i] = a[store];
                a[store] = t;
                store++;
            }
        }
        a[hi] = a[store];
        a[store] = pv;
        if (store == r) return;
        if (store < r) lo = store + 1;
        else hi = store - 1;
    }
}

static int level_of(int64_t v)
{
    int l = 0;
    while (v + 1 >= (int64_t)2 << l) l++;
    return l;
}

/*
 * split[2^h - 1]   splitting values in heap order (children of v: 2v+1, 2v+2)
 * leaf_off[2^h+1]  leaf l holds leaf-structure positions [leaf_off[l], leaf_off[l+1])
 * perm[n]          original index of the point at each leaf-structure position
 * Returns 0, or -1 on invalid arguments / allocation failure.
 */
/*
 * Splitting dimension of a node (Section 2.3).  rule 0: level mod d (the
 * original k-d tree).  rule 1: the longest side of the bounding box of the
 * node's points (the footnote's alternative rule): the j with the largest
 * float32 side fl32(max_j - min_j), the smaller j on ties.
 */
static int split_dim(const float *P, int d, const int32_t *perm, int64_t a, int64_t c, int level, int rule)
{
    if (rule == 0) return level % d;
    int best = 0;
    float best_side = -1.0f;
    for (int j = 0; j < d; j++) {
        float mn = INFINITY, mx = -INFINITY;
        for (int64_t i = 0; i < c; i++) {
            float v = P[(int64_t)perm[a + i] * d + j];
            if (v < mn) mn = v;
            if (v > mx) mx = v;
        }
        float side = mx - mn;
        if (side > best_side) {
            best_side = side;
            best = j;
        }
    }
    return best;
}

int orc_build_rules(const float *P, int64_t n, int32_t d, int32_t h, int32_t rule, float *split, int32_t *dims,
                    int64_t *leaf_off, int32_t *perm);

int orc_build(const float *P, int64_t n, int32_t d, int32_t h, float *split, int64_t *leaf_off, int32_t *perm)
{
    return orc_build_rules(P, n, d, h, 0, split, NULL, leaf_off, perm);
}

/* The same construction with a choice of splitting rule; dims[v] (if not NULL) receives the
   splitting dimension of internal node v. */
int orc_build_rules(const float *P, int64_t n, int32_t d, int32_t h, int32_t rule, float *split, int32_t *dims,
                    int64_t *leaf_off, int32_t *perm)
{
    if (!P || n < 1 || d < 1 || h < 0 || h > 30 || ((int64_t)1 << h) > n || rule < 0 || rule > 1) return -1;
    int64_t nleaf = (int64_t)1 << h;
    int64_t nnodes = 2 * nleaf - 1;
    int64_t *lo = (int64_t *)malloc(sizeof(int64_t) * nnodes);
    int64_t *hi = (int64_t *)malloc(sizeof(int64_t) * nnodes);
    if (!lo || !hi) { free(lo); free(hi); return -1; }
    for (int64_t i = 0; i < n; i++) perm[i] = (int32_t)i;
    lo[0] = 0;
    hi[0] = n;
    for (int l = 0; l < h; l++) {
        int64_t first = ((int64_t)1 << l) - 1, count = (int64_t)1 << l;
        int failed = 0;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t t = 0; t < count; t++) {
            int64_t v = first + t;
            int64_t a = lo[v], c = hi[v] - lo[v];
            int dim = split_dim(P, d, perm, a, c, l, rule);
            if (dims) dims[v] = dim;
            vi_t *tmp = (vi_t *)malloc(sizeof(vi_t) * (size_t)c);
            if (!tmp) { failed = 1; continue; }
            for (int64_t i = 0; i < c; i++) {
                tmp[i].i = perm[a + i];
                tmp[i].v = P[(int64_t)tmp[i].i * d + dim];
            }
            /* the left child takes the floor(c/2) smallest; the split value is the
               smallest value on the right */
            int64_t nl = c / 2;
            select_vi(tmp, c, nl);
            for (int64_t i = 0; i < c; i++) perm[a + i] = tmp[i].i;
            split[v] = tmp[nl].v;
            lo[2 * v + 1] = a;
            hi[2 * v + 1] = a + nl;
            lo[2 * v + 2] = a + nl;
            hi[2 * v + 2] = a + c;
            free(tmp);
        }
        if (failed) { free(lo); free(hi); return -1; }
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t l = 0; l < nleaf; l++) {
        int64_t v = nleaf - 1 + l;
        qsort(perm + lo[v], (size_t)(hi[v] - lo[v]), sizeof(int32_t), cmp_i32);
    }
    for (int64_t l = 0; l < nleaf; l++) leaf_off[l] = lo[nleaf - 1 + l];
    leaf_off[nleaf] = n;
    free(lo);
    free(hi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Distances.                                                               */

/* float32 squared distance under the stated rounding reading. */
static float dist2_f32(const float *q, const float *x, int d)
{
    float acc = 0.0f;
    for (int j = 0; j < d; j++) {
        float t = q[j] - x[j];
        acc = fmaf(t, t, acc);
    }
    return acc;
}

static double dist2_f64(const float *q, const float *x, int d)
{
    double acc = 0.0;
    for (int j = 0; j < d; j++) {
        double t = (double)q[j] - (double)x[j];
        acc += t * t;
    }
    return acc;
}

static uint64_t make_key(float d2, int32_t idx)
{
    uint32_t b;
    memcpy(&b, &d2, 4);
    return ((uint64_t)b << 32) | (uint32_t)idx;
}

/* Keep the k smallest keys in ascending order (insertion into a sorted list). */
static void insert_key(uint64_t *list, int k, uint64_t key)
{
    if (key >= list[k - 1]) return;
    int i = k - 1;
    while (i > 0 && list[i - 1] > key) {
        list[i] = list[i - 1];
        i--;
    }
    list[i] = key;
}

/* Same for (d2, idx) pairs in float64, ordered by d2 then idx. */
static void insert_pair(double *dl, int64_t *il, int k, double d2, int64_t idx)
{
    double dk = dl[k - 1];
    if (d2 > dk || (d2 == dk && idx >= il[k - 1])) return;
    int i = k - 1;
    while (i > 0 && (dl[i - 1] > d2 || (dl[i - 1] == d2 && il[i - 1] > idx))) {
        dl[i] = dl[i - 1];
        il[i] = il[i - 1];
        i--;
    }
    dl[i] = d2;
    il[i] = idx;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive kNN (Section 2.2): every (query, reference) distance.          */

int orc_brute_f64(const float *P, int64_t n, const float *Q, int64_t m, int32_t d, int32_t k,
                  int64_t *out_idx, double *out_d2, int32_t nthreads)
{
    if (!P || !Q || n < 1 || m < 0 || d < 1 || k < 1 || k > n) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < m; qi++) {
        double *dl = out_d2 + qi * k;
        int64_t *il = out_idx + qi * k;
        for (int i = 0; i < k; i++) { dl[i] = INFINITY; il[i] = INT64_MAX; }
        const float *q = Q + qi * d;
        for (int64_t j = 0; j < n; j++) insert_pair(dl, il, k, dist2_f64(q, P + j * d, d), j);
    }
    return 0;
}

int orc_brute_f32c(const float *P, int64_t n, const float *Q, int64_t m, int32_t d, int32_t k,
                   uint64_t *out_keys, int32_t nthreads)
{
    if (!P || !Q || n < 1 || m < 0 || d < 1 || k < 1 || k > n) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < m; qi++) {
        uint64_t *kl = out_keys + qi * k;
        for (int i = 0; i < k; i++) kl[i] = ORC_EMPTY_KEY;
        const float *q = Q + qi * d;
        for (int64_t j = 0; j < n; j++) insert_key(kl, k, make_key(dist2_f32(q, P + j * d, d), (int32_t)j));
    }
    return 0;
}

/* float32 hyperplane term of node v for query q. */
static float plane2_f32(const float *q, const float *split, int64_t v, int d)
{
    float t = q[level_of(v) % d] - split[v];
    return t * t;
}

/* ------------------------------------------------------------------------ */
/* Classical k-d tree search in float64 (Section 2.3): descend to the cell,  */
/* then on the way back visit the far child when the hyperplane is no       */
/* farther than the current k-th candidate.  Used as the timed CPU baseline.*/

typedef struct {
    const float *P, *split;
    const int64_t *leaf_off;
    const int32_t *perm;
    int64_t first_leaf;
    int d, k;
} kd64_t;

static void kd64_search(const kd64_t *t, int64_t v, const float *q, double *dl, int64_t *il)
{
    if (v >= t->first_leaf) {
        int64_t l = v - t->first_leaf;
        for (int64_t p = t->leaf_off[l]; p < t->leaf_off[l + 1]; p++) {
            int64_t o = t->perm[p];
            insert_pair(dl, il, t->k, dist2_f64(q, t->P + o * t->d, t->d), o);
        }
        return;
    }
    int dim = level_of(v) % t->d;
    double s = t->split[v];
    int64_t nearc = ((double)q[dim] < s) ? 2 * v + 1 : 2 * v + 2;
    int64_t farc = (nearc == 2 * v + 1) ? 2 * v + 2 : 2 * v + 1;
    kd64_search(t, nearc, q, dl, il);
    double g = (double)q[dim] - s;
    if (g * g <= dl[t->k - 1]) kd64_search(t, farc, q, dl, il);
}

/*
 * Classical k-d tree with leaves of about `leaf_size` points (height
 * floor(log2(n / leaf_size))), built once, queried many times.
 */
typedef struct {
    kd64_t t;
    float *split;
    int64_t *leaf_off;
    int32_t *perm;
} kd64_tree_t;

void orc_kdtree_f64_free(kd64_tree_t *T)
{
    if (!T) return;
    free(T->split); free(T->leaf_off); free(T->perm); free(T);
}

kd64_tree_t *orc_kdtree_f64_build(const float *P, int64_t n, int32_t d, int32_t leaf_size, int32_t nthreads)
{
    if (!P || n < 1 || d < 1 || leaf_size < 1) return NULL;
    set_threads(nthreads);
    int h = 0;
    while (((int64_t)leaf_size << (h + 1)) <= n && h < 30) h++;
    int64_t nleaf = (int64_t)1 << h;
    kd64_tree_t *T = (kd64_tree_t *)calloc(1, sizeof(kd64_tree_t));
    if (!T) return NULL;
    T->split = (float *)malloc(sizeof(float) * (size_t)(nleaf > 1 ? nleaf - 1 : 1));
    T->leaf_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nleaf + 1));
    T->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!T->split || !T->leaf_off || !T->perm || orc_build(P, n, d, h, T->split, T->leaf_off, T->perm) != 0) {
        orc_kdtree_f64_free(T);
        return NULL;
    }
    kd64_t t = {P, T->split, T->leaf_off, T->perm, nleaf - 1, d, 0};
    T->t = t;
    return T;
}

/* P must stay alive while the tree is used (the tree refers to it). */
int orc_kdtree_f64_query(kd64_tree_t *T, const float *Q, int64_t m, int32_t k, int64_t *out_idx, double *out_d2,
                         int32_t nthreads)
{
    if (!T || !Q || m < 0 || k < 1) return -1;
    set_threads(nthreads);
    kd64_t t = T->t;
    t.k = k;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t qi = 0; qi < m; qi++) {
        double *dl = out_d2 + qi * k;
        int64_t *il = out_idx + qi * k;
        for (int i = 0; i < k; i++) { dl[i] = INFINITY; il[i] = INT64_MAX; }
        kd64_search(&t, 0, Q + qi * t.d, dl, il);
    }
    return 0;
}

int orc_kdtree_f64(const float *P, int64_t n, const float *Q, int64_t m, int32_t d, int32_t k, int32_t leaf_size,
                   int64_t *out_idx, double *out_d2, int32_t nthreads)
{
    if (!P || !Q || n < 1 || m < 0 || d < 1 || k < 1 || k > n || leaf_size < 1) return -1;
    kd64_tree_t *T = orc_kdtree_f64_build(P, n, d, leaf_size, nthreads);
    if (!T) return -1;
    int rc = orc_kdtree_f64_query(T, Q, m, k, out_idx, out_d2, nthreads);
    orc_kdtree_f64_free(T);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Stackless traversal (FindLeafBatch for one query; Sections 2.3, 2.4).    */

static int64_t descend(const float *q, const float *split, int64_t v, int64_t first_leaf, int d)
{
    while (v < first_leaf) v = (q[level_of(v) % d] < split[v]) ? 2 * v + 1 : 2 * v + 2;
    return v;
}

/*
 * state: ORC_FRESH, ORC_DONE or the heap index of the last visited leaf.
 * Returns the heap index of the next leaf, or ORC_DONE once the walk back
 * reaches the root a second time.  kth: current k-th best float32 d2.
 */
static int64_t next_leaf(int64_t state, const float *q, float kth, const float *split, int64_t first_leaf, int d)
{
    if (state == ORC_DONE) return ORC_DONE;
    if (state == ORC_FRESH) return descend(q, split, 0, first_leaf, d);
    int64_t u = state;
    while (u != 0) {
        int64_t p = (u - 1) / 2;
        int dim = level_of(p) % d;
        int64_t nearc = (q[dim] < split[p]) ? 2 * p + 1 : 2 * p + 2;
        if (u == nearc && plane2_f32(q, split, p, d) <= kth) {
            int64_t sib = (nearc == 2 * p + 1) ? 2 * p + 2 : 2 * p + 1;
            return descend(q, split, sib, first_leaf, d);
        }
        u = p;
    }
    return ORC_DONE;
}

static float kth_of(const uint64_t *list, int k)
{
    uint32_t b = (uint32_t)(list[k - 1] >> 32);
    float f;
    memcpy(&f, &b, 4);
    return f;
}

/* Scan every point of leaf l against query q (float32 keys). */
static void scan_leaf(const float *P, int d, const int64_t *leaf_off, const int32_t *perm, int64_t l, const float *q,
                      uint64_t *list, int k)
{
    for (int64_t p = leaf_off[l]; p < leaf_off[l + 1]; p++) {
        int32_t o = perm[p];
        insert_key(list, k, make_key(dist2_f32(q, P + (int64_t)o * d, d), o));
    }
}

/*
 * One query's complete traversal: the sequence of leaves it visits and its
 * final keys.  A query's sequence depends only on its own data, not on the
 * batching schedule, so this checks sampled queries of large runs.
 * Returns the number of leaves visited (may exceed max_leaves; only the
 * first max_leaves are stored).
 */
int64_t orc_traverse_f32(const float *P, int32_t d, int32_t h, const float *split, const int64_t *leaf_off,
                         const int32_t *perm, const float *q, int32_t k, int32_t *out_leaves, int64_t max_leaves,
                         uint64_t *out_keys)
{
    int64_t first_leaf = ((int64_t)1 << h) - 1;
    for (int i = 0; i < k; i++) out_keys[i] = ORC_EMPTY_KEY;
    int64_t state = ORC_FRESH, count = 0;
    for (;;) {
        state = next_leaf(state, q, kth_of(out_keys, k), split, first_leaf, d);
        if (state == ORC_DONE) break;
        if (count < max_leaves) out_leaves[count] = (int32_t)(state - first_leaf);
        count++;
        scan_leaf(P, d, leaf_off, perm, state - first_leaf, q, out_keys, k);
    }
    return count;
}

/* Same for many queries in parallel: keys and leaf-visit counts only. */
int orc_traverse_many_f32(const float *P, int32_t d, int32_t h, const float *split, const int64_t *leaf_off,
                          const int32_t *perm, const float *Q, int64_t m, int32_t k, uint64_t *out_keys,
                          int64_t *out_visits, int64_t *out_pairs, int32_t nthreads)
{
    set_threads(nthreads);
    int64_t first_leaf = ((int64_t)1 << h) - 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < m; qi++) {
        uint64_t *kl = out_keys + qi * k;
        const float *q = Q + qi * d;
        for (int i = 0; i < k; i++) kl[i] = ORC_EMPTY_KEY;
        int64_t state = ORC_FRESH, count = 0, pairs = 0;
        for (;;) {
            state = next_leaf(state, q, kth_of(kl, k), split, first_leaf, d);
            if (state == ORC_DONE) break;
            int64_t l = state - first_leaf;
            count++;
            pairs += leaf_off[l + 1] - leaf_off[l];
            scan_leaf(P, d, leaf_off, perm, l, q, kl, k);
        }
        if (out_visits) out_visits[qi] = count;
        if (out_pairs) out_pairs[qi] = pairs;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Variant tree: a splitting dimension per node and bounding-box pruning     */
/* (Section 2.3: the footnote's other splitting rules; the search phase     */
/* prunes a subtree whose points are all farther than the current k-th      */
/* candidate -- the box of its points gives a tighter such bound than the   */
/* splitting hyperplane).                                                   */

/*
 * Bounding box of every node's points, heap order over all 2^(h+1) - 1
 * nodes (internal nodes, then leaves): box[v * 2d + j] = min of coordinate j,
 * box[v * 2d + d + j] = max.  A node's points are the leaf-structure
 * positions of the leaves below it.
 */
int orc_node_boxes(const float *P, int32_t d, int32_t h, const int64_t *leaf_off, const int32_t *perm, float *box)
{
    if (!P || d < 1 || h < 0 || h > 30) return -1;
    int64_t nleaf = (int64_t)1 << h, first_leaf = nleaf - 1;
    for (int64_t l = 0; l < nleaf; l++) {
        float *b = box + (first_leaf + l) * 2 * d;
        for (int j = 0; j < d; j++) {
            b[j] = INFINITY;
            b[d + j] = -INFINITY;
        }
        for (int64_t p = leaf_off[l]; p < leaf_off[l + 1]; p++) {
            const float *x = P + (int64_t)perm[p] * d;
            for (int j = 0; j < d; j++) {
                if (x[j] < b[j]) b[j] = x[j];
                if (x[j] > b[d + j]) b[d + j] = x[j];
            }
        }
    }
    for (int64_t v = first_leaf - 1; v >= 0; v--) {
        float *b = box + v * 2 * d;
        const float *l = box + (2 * v + 1) * 2 * d, *r = box + (2 * v + 2) * 2 * d;
        for (int j = 0; j < d; j++) {
            b[j] = l[j] < r[j] ? l[j] : r[j];
            b[d + j] = l[d + j] > r[d + j] ? l[d + j] : r[d + j];
        }
    }
    return 0;
}

/*
 * float32 box term of query q and box b: g_j = the distance of q_j to
 * [min_j, max_j] (0 inside), rounded to float32, accumulated as the distance
 * is: acc = fmaf(g_j, g_j, acc) for j = 0..d-1 from +0.  For every point x in
 * the box, |fl32(q_j - x_j)| >= g_j and rounding is monotone, so the term
 * never exceeds the float32 squared distance of x.
 */
static float box2_f32(const float *q, const float *b, int d)
{
    float acc = 0.0f;
    for (int j = 0; j < d; j++) {
        float g = 0.0f;
        if (q[j] < b[j]) g = b[j] - q[j];
        else if (q[j] > b[d + j]) g = q[j] - b[d + j];
        acc = fmaf(g, g, acc);
    }
    return acc;
}

static int node_dim(const int32_t *dims, int64_t v, int d) { return dims ? dims[v] : level_of(v) % d; }

static int64_t descend_r(const float *q, const float *split, const int32_t *dims, int64_t v, int64_t first_leaf, int d)
{
    while (v < first_leaf) v = (q[node_dim(dims, v, d)] < split[v]) ? 2 * v + 1 : 2 * v + 2;
    return v;
}

/* The stackless walk of next_leaf with per-node dimensions (dims, NULL: level mod d) and the
   far child's box term in place of the plane term (box, NULL: the plane). */
static int64_t next_leaf_r(int64_t state, const float *q, float kth, const float *split, const int32_t *dims,
                           const float *box, int64_t first_leaf, int d)
{
    if (state == ORC_DONE) return ORC_DONE;
    if (state == ORC_FRESH) return descend_r(q, split, dims, 0, first_leaf, d);
    int64_t u = state;
    while (u != 0) {
        int64_t p = (u - 1) / 2;
        int dim = node_dim(dims, p, d);
        int64_t nearc = (q[dim] < split[p]) ? 2 * p + 1 : 2 * p + 2;
        int64_t sib = (nearc == 2 * p + 1) ? 2 * p + 2 : 2 * p + 1;
        if (u == nearc) {
            float t = q[dim] - split[p];
            float bound = box ? box2_f32(q, box + sib * 2 * d, d) : t * t;
            if (bound <= kth) return descend_r(q, split, dims, sib, first_leaf, d);
        }
        u = p;
    }
    return ORC_DONE;
}

int64_t orc_traverse_f32_rules(const float *P, int32_t d, int32_t h, const float *split, const int32_t *dims,
                               const float *box, const int64_t *leaf_off, const int32_t *perm, const float *q, int32_t k,
                               int32_t *out_leaves, int64_t max_leaves, uint64_t *out_keys)
{
    int64_t first_leaf = ((int64_t)1 << h) - 1;
    for (int i = 0; i < k; i++) out_keys[i] = ORC_EMPTY_KEY;
    int64_t state = ORC_FRESH, count = 0;
    for (;;) {
        state = next_leaf_r(state, q, kth_of(out_keys, k), split, dims, box, first_leaf, d);
        if (state == ORC_DONE) break;
        if (count < max_leaves) out_leaves[count] = (int32_t)(state - first_leaf);
        count++;
        scan_leaf(P, d, leaf_off, perm, state - first_leaf, q, out_keys, k);
    }
    return count;
}

int orc_traverse_many_f32_rules(const float *P, int32_t d, int32_t h, const float *split, const int32_t *dims,
                                const float *box, const int64_t *leaf_off, const int32_t *perm, const float *Q,
                                int64_t m, int32_t k, uint64_t *out_keys, int64_t *out_visits, int32_t nthreads)
{
    set_threads(nthreads);
    int64_t first_leaf = ((int64_t)1 << h) - 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t qi = 0; qi < m; qi++) {
        uint64_t *kl = out_keys + qi * k;
        const float *q = Q + qi * d;
        for (int i = 0; i < k; i++) kl[i] = ORC_EMPTY_KEY;
        int64_t state = ORC_FRESH, count = 0;
        for (;;) {
            state = next_leaf_r(state, q, kth_of(kl, k), split, dims, box, first_leaf, d);
            if (state == ORC_DONE) break;
            count++;
            scan_leaf(P, d, leaf_off, perm, state - first_leaf, q, kl, k);
        }
        if (out_visits) out_visits[qi] = count;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* LazySearch schedule replay (Algorithm 1).                                */

typedef struct {
    int64_t m;
    int32_t k;
    uint64_t *keys;       /* m x k final lists                            */
    int64_t ncalls;       /* ProcessAllBuffers calls                       */
    int64_t nfetch;       /* fetches (FindLeafBatch invocations)           */
    int64_t pairs;        /* (query, leaf point) pairs scanned             */
    /* trace: per call, the fetched (query, leaf) pairs in fetch order since */
    /* the previous call, leaf -1 = traversal finished                      */
    int64_t tlen, tcap, ccap;
    int64_t *call_off;
    int64_t *tq;
    int32_t *tr;
} orc_replay_t;

static int trace_push(orc_replay_t *r, int64_t q, int32_t leaf)
{
    if (r->tlen == r->tcap) {
        int64_t nc = r->tcap ? 2 * r->tcap : 1024;
        int64_t *a = (int64_t *)realloc(r->tq, sizeof(int64_t) * (size_t)nc);
        if (!a) return -1;
        r->tq = a;
        int32_t *b = (int32_t *)realloc(r->tr, sizeof(int32_t) * (size_t)nc);
        if (!b) return -1;
        r->tr = b;
        r->tcap = nc;
    }
    r->tq[r->tlen] = q;
    r->tr[r->tlen] = leaf;
    r->tlen++;
    return 0;
}

static int call_push(orc_replay_t *r)
{
    if (r->ncalls + 2 > r->ccap) {
        int64_t nc = r->ccap ? 2 * r->ccap : 64;
        int64_t *a = (int64_t *)realloc(r->call_off, sizeof(int64_t) * (size_t)nc);
        if (!a) return -1;
        r->call_off = a;
        r->ccap = nc;
    }
    r->ncalls++;
    r->call_off[r->ncalls] = r->tlen;
    return 0;
}

void orc_replay_free(orc_replay_t *r)
{
    if (!r) return;
    free(r->keys);
    free(r->call_off);
    free(r->tq);
    free(r->tr);
    free(r);
}

/*
 * B: buffer size (a buffer is half-full at >= ceil(B/2) indices); B <= 0
 *    means buffers never count as half-full (process only on empty queues).
 * M: indices fetched per iteration; M <= 0 means all available.
 * The tree arrays are the canonical ones from orc_build.
 */
orc_replay_t *orc_replay_run(const float *P, int64_t n, int32_t d, int32_t h, const float *split,
                             const int64_t *leaf_off, const int32_t *perm, const float *Q, int64_t m, int32_t k,
                             int64_t B, int64_t M, int32_t record_trace, int32_t nthreads)
{
    if (!P || !Q || n < 1 || d < 1 || k < 1 || k > n || m < 0) return NULL;
    set_threads(nthreads);
    int64_t nleaf = (int64_t)1 << h, first_leaf = nleaf - 1;
    int64_t half = B > 0 ? (B + 1) / 2 : INT64_MAX;
    int64_t fetch = M > 0 ? M : INT64_MAX;
    orc_replay_t *r = (orc_replay_t *)calloc(1, sizeof(orc_replay_t));
    int64_t *state = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int64_t *reinsert = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1)); /* ring */
    int64_t *fetched = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int64_t *leafof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
    int64_t *bcnt = (int64_t *)calloc((size_t)nleaf, sizeof(int64_t));
    int64_t *boff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nleaf + 1));
    int64_t *buf = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));   /* buffered, arrival order */
    int64_t *bl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));    /* leaf of buffered entry */
    int64_t *flat = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));  /* buffers, leaf order */
    if (!r || !state || !reinsert || !fetched || !leafof || !bcnt || !boff || !buf || !bl || !flat) goto fail;
    r->m = m;
    r->k = k;
    r->keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m ? m : 1) * (size_t)k);
    r->call_off = (int64_t *)malloc(sizeof(int64_t) * 64);
    r->ccap = 64;
    if (!r->keys || !r->call_off) goto fail;
    r->call_off[0] = 0;
    for (int64_t i = 0; i < m * k; i++) r->keys[i] = ORC_EMPTY_KEY;
    for (int64_t i = 0; i < m; i++) state[i] = ORC_FRESH;

    int64_t in_head = 0;            /* input holds queries in_head..m-1 */
    int64_t re_head = 0, re_len = 0; /* reinsert ring                     */
    int64_t nbuf = 0, maxcnt = 0;    /* buffered entries                  */
    while (in_head < m || re_len > 0) {
        /* Fetch up to M indices, reinsert first, then input. */
        int64_t nf = 0;
        while (nf < fetch && re_len > 0) {
            fetched[nf++] = reinsert[re_head];
            re_head = (re_head + 1) % m;
            re_len--;
        }
        while (nf < fetch && in_head < m) fetched[nf++] = in_head++;
        r->nfetch++;
        /* FindLeafBatch. */
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t j = 0; j < nf; j++) {
            int64_t qi = fetched[j];
            int64_t s = next_leaf(state[qi], Q + qi * d, kth_of(r->keys + qi * k, k), split, first_leaf, d);
            state[qi] = s;
            leafof[j] = (s == ORC_DONE) ? -1 : s - first_leaf;
        }
        /* Insert into the buffers in fetch order. */
        for (int64_t j = 0; j < nf; j++) {
            if (record_trace && trace_push(r, fetched[j], (int32_t)leafof[j])) goto fail;
            if (leafof[j] < 0) continue;
            buf[nbuf] = fetched[j];
            bl[nbuf] = leafof[j];
            nbuf++;
            if (++bcnt[leafof[j]] > maxcnt) maxcnt = bcnt[leafof[j]];
        }
        int queues_empty = (in_head == m && re_len == 0);
        if (maxcnt >= half || queues_empty) {
            /* ProcessAllBuffers: every buffered query against its leaf. */
            boff[0] = 0;
            for (int64_t l = 0; l < nleaf; l++) boff[l + 1] = boff[l] + bcnt[l];
            for (int64_t l = 0; l < nleaf; l++) bcnt[l] = 0;
            for (int64_t j = 0; j < nbuf; j++) flat[boff[bl[j]] + bcnt[bl[j]]++] = buf[j];
            int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pairs)
            for (int64_t j = 0; j < nbuf; j++) {
                int64_t qi = flat[j];
                int64_t l = state[qi] - first_leaf;
                scan_leaf(P, d, leaf_off, perm, l, Q + qi * d, r->keys + qi * k, k);
                pairs += leaf_off[l + 1] - leaf_off[l];
            }
            r->pairs += pairs;
            /* Reinsert every processed index, ascending leaf, buffer order. */
            for (int64_t j = 0; j < nbuf; j++) {
                reinsert[(re_head + re_len) % m] = flat[j];
                re_len++;
            }
            for (int64_t l = 0; l < nleaf; l++) bcnt[l] = 0;
            nbuf = 0;
            maxcnt = 0;
            if (call_push(r)) goto fail;
        }
    }
    free(state); free(reinsert); free(fetched); free(leafof); free(bcnt); free(boff); free(buf); free(bl); free(flat);
    return r;
fail:
    free(state); free(reinsert); free(fetched); free(leafof); free(bcnt); free(boff); free(buf); free(bl); free(flat);
    orc_replay_free(r);
    return NULL;
}

int64_t orc_replay_ncalls(const orc_replay_t *r) { return r->ncalls; }
int64_t orc_replay_nfetch(const orc_replay_t *r) { return r->nfetch; }
int64_t orc_replay_pairs(const orc_replay_t *r) { return r->pairs; }
int64_t orc_replay_trace_len(const orc_replay_t *r) { return r->tlen; }

void orc_replay_get(const orc_replay_t *r, uint64_t *keys, int64_t *call_off, int64_t *trace_q, int32_t *trace_r)
{
    if (keys) memcpy(keys, r->keys, sizeof(uint64_t) * (size_t)(r->m * r->k));
    if (call_off) memcpy(call_off, r->call_off, sizeof(int64_t) * (size_t)(r->ncalls + 1));
    if (trace_q && r->tlen) memcpy(trace_q, r->tq, sizeof(int64_t) * (size_t)r->tlen);
    if (trace_r && r->tlen) memcpy(trace_r, r->tr, sizeof(int32_t) * (size_t)r->tlen);
}

/* ------------------------------------------------------------------------ */
/* Chunk bounds of the leaf structure (Section 3.2): chunk j of N covers    */
/* positions [ceil((j-1) n / N), ceil(j n / N)), read half-open.            */

/*
 * Leaf-aligned chunks (the reading of Section 3.2 in which a chunk holds whole
 * leaves, so a leaf never straddles two chunks): chunk j holds leaves
 * [first[j], first[j+1]).  With N > 0 the leaf range is cut by the same
 * ceiling rule as positions: chunk j of N holds leaves [ceil((j-1) L / N),
 * ceil(j L / N)) of the L = 2^h leaves.  With N = 0 the leaves are packed in
 * order, as many whole leaves per chunk as fit cap_bytes at (4d + 4) bytes per
 * point (a leaf larger than the capacity is a chunk of its own).  first gets
 * up to L + 1 entries; returns the number of chunks, or -1.
 */
int64_t orc_leaf_chunks(const int64_t *leaf_off, int32_t h, int32_t d, int64_t N, int64_t cap_bytes, int64_t *first)
{
    int64_t L = (int64_t)1 << h;
    if (!leaf_off || d < 1 || N < 0 || (N == 0 && cap_bytes < 1)) return -1;
    if (N > 0) {
        if (N > L) N = L;
        for (int64_t j = 0; j <= N; j++) first[j] = (j * L + N - 1) / N;
        return N;
    }
    int64_t count = 0, l = 0, bpp = 4 * (int64_t)d + 4;
    while (l < L) {
        int64_t e = l + 1;
        while (e < L && (leaf_off[e + 1] - leaf_off[l]) * bpp <= cap_bytes) e++;
        first[count++] = l;
        l = e;
    }
    first[count] = L;
    return count;
}

int orc_chunk_bounds(int64_t n, int64_t N, int64_t *lo, int64_t *hi)
{
    if (n < 1 || N < 1) return -1;
    for (int64_t j = 1; j <= N; j++) {
        /* ceil(a / N) for a >= 0 in exact integer arithmetic */
        lo[j - 1] = ((j - 1) * n + N - 1) / N;
        hi[j - 1] = (j * n + N - 1) / N;
    }
    return 0;
}
