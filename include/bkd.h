/*
 * bkd.h -- C ABI of the MI355X buffer k-d tree exact kNN library.
 *
 * Method: Gieseke, Oancea, Mahabal, Igel, Heskes, "Bigger Buffer k-d Trees on
 * Multi-Many-Core Systems" (arXiv 1512.02831).  The problem solved is the one
 * of Section 2.2: for every query q in Q, the k >= 1 nearest points of the
 * reference set P under the Euclidean distance.  A query runs the buffered
 * loop of Algorithm 1 (Section 2.4) on one AMD Instinct MI355X (gfx950):
 * queries are routed through a top tree (FindLeafBatch), parked in per-leaf
 * buffers, and all buffers are then processed by a brute-force leaf scan with
 * a top-k merge (ProcessAllBuffers).  When the leaf structure exceeds the
 * device budget it is streamed in chunks with copy/compute overlap
 * (Section 3.2).
 *
 * Conventions shared by every entry point
 *   - Every function returns BKD_OK (0) or a negative BKD_E* code.  No C++
 *     exception, abort or exit crosses this boundary.  bkd_last_error()
 *     returns a thread-local message describing the last failure.
 *   - Points are float32, row-major [count][d].  Indices are 0-based rows of P.
 *   - Results are row-major [m][k]: the k nearest points of each query in
 *     ascending distance; exact distance ties are broken by smaller index.
 *     Distances are Euclidean (the square root of the float32 squared
 *     distance defined under bkd_query).
 *   - On error the outputs are unspecified, bkd_build creates nothing and an
 *     existing tree stays valid.
 *   - A tree may be used by one query at a time (the served API interleaves
 *     requests on shared trees itself).
 */
#ifndef BKD_H
#define BKD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define BKD_OK 0
#define BKD_EINVAL (-1)   /* invalid argument (NULL, range, non-finite value)          */
#define BKD_ENOMEM (-2)   /* host, pinned or device allocation failed                   */
#define BKD_EBUDGET (-3)  /* leaf budget smaller than two leaves of the leaf structure  */
#define BKD_EDEVICE (-4)  /* a HIP call failed; the message holds hipGetErrorString     */
#define BKD_EBUSY (-5)    /* served form: no capacity left and the call is non-blocking */
#define BKD_ETIMEOUT (-6) /* served form: bkd_wait timed out                            */
#define BKD_ENOTFOUND (-7)/* served form: unknown request or tree id                    */

#define BKD_MAX_DIM 32
#define BKD_MAX_K 64
#define BKD_MAX_HEIGHT 24

/* Chunk partition of the leaf structure (Section 3.2). */
#define BKD_CHUNK_LEAF 0     /* chunks hold whole leaves, packed up to the chunk capacity      */
#define BKD_CHUNK_POSITION 1 /* chunk j of N holds positions [ceil((j-1)n/N), ceil(jn/N))      */

/* Option flags. */
#define BKD_FLAG_TRACE 1  /* record every fetch's (query, leaf) pairs (for parity checks)     */
#define BKD_FLAG_TIMING 2 /* time every leaf-scan launch with HIP events                       */
#define BKD_FLAG_SQUARED 4 /* out_dist receives the float32 squared distance, not its root      */
#define BKD_FLAG_NO_TAIL 8 /* lock-step rounds to the end: no hand-over of the last few pending  */
                           /* queries to one-workgroup-per-query traversals (results identical)  */
#define BKD_FLAG_DEVICE_BUILD 16 /* build the top tree on the device: one stable radix sort per     */
                                 /* level (the same canonical tree as the host build, Section 2.3); */
                                 /* needs about 8d + 32 bytes of device memory per point meanwhile  */
#define BKD_FLAG_DEVICE_PTRS 32 /* batched form: every instance's P, Q, out_idx and out_dist are    */
                                /* device pointers on the batch's device (else host pointers)       */

/* Splitting rule and pruning bound of the tree (Section 2.3).  The original k-d tree splits
   dimension (level mod d) and prunes with the splitting hyperplane; the footnote on splitting
   rules names the longest side as an alternative, and the bounding box of a subtree's points
   bounds its distances more tightly than the hyperplane.  Results are the same for every rule
   and bound (exact kNN); the leaves a query visits differ. */
#define BKD_SPLIT_CYCLIC 0  /* dimension (level mod d)                                        */
#define BKD_SPLIT_LONGEST 1 /* the longest side of the bounding box of the node's points:      */
                            /* the j with the largest float32 fl32(max_j - min_j), smaller j    */
                            /* on ties; median split as in the original rule                    */
#define BKD_PRUNE_PLANE 0   /* enter the far child iff fl32(q[dim] - s)^2 <= current k-th d2     */
#define BKD_PRUNE_BOX 1     /* enter it iff its box term <= current k-th d2: g_j = fl32 distance */
                            /* of q_j to the far child's [min_j, max_j] (0 inside), accumulated */
                            /* acc = fma(g_j, g_j, acc) from +0 as the distance is; never above */
                            /* the float32 distance of a point in the box, never below the plane */

typedef struct bkd_tree bkd_tree;

/*
 * Schedule and memory options of a tree.  Zero-initialised fields take the
 * defaults of Section 4.1 (footnote on parameters): B = 2^(24-h), M = 10 B.
 *   buffer_size   B.  A ProcessAllBuffers call is triggered once a buffer holds
 *                 at least ceil(B/2) query indices (Algorithm 1).  < 0: never
 *                 half-full; buffers are processed only when both queues are
 *                 empty.  Buffers are pooled, so B only sets the trigger.
 *   fetch_size    M, indices fetched per iteration (reinsert first, then
 *                 input, both FIFO).  < 0: fetch everything available, which
 *                 makes every iteration one lock-step round over all active
 *                 queries.  Results do not depend on B or M.
 *   leaf_budget_bytes  device bytes reserved for the leaf structure.  0 (and
 *                 num_chunks 0): the whole structure is resident on the
 *                 device.  Otherwise, if the structure does not fit, it stays
 *                 in pinned host memory and is streamed through two device
 *                 chunk buffers of budget/2 bytes each (Section 3.1, 3.2).
 *   chunk_mode    BKD_CHUNK_LEAF or BKD_CHUNK_POSITION.
 *   num_chunks    > 0 forces streaming with exactly this many chunks (testing
 *                 and the chunked-versus-resident comparison).
 *   device        HIP device ordinal.
 *   flags         BKD_FLAG_* bits.
 *   tail_max      lock-step schedule: on a resident structure, once a round
 *                 starts with at most this many pending queries, the rounds
 *                 stop and each of them finishes its traversal alone (one
 *                 workgroup per query); on a structure streamed in N
 *                 leaf-aligned chunks, a resident chunk with at most
 *                 max(1, tail_max / N) pending queries is drained that way
 *                 (each query walks on while its next leaf is in the chunk).
 *                 0: the default (32768); < 0: rounds to the end (as
 *                 BKD_FLAG_NO_TAIL).
 *   split_rule    BKD_SPLIT_CYCLIC (0) or BKD_SPLIT_LONGEST (host build only:
 *                 BKD_FLAG_DEVICE_BUILD with BKD_SPLIT_LONGEST is BKD_EINVAL).
 *   prune         BKD_PRUNE_PLANE (0) or BKD_PRUNE_BOX; the boxes take
 *                 (2^(h+1) - 1) 8d bytes of device memory.
 *   leaf_path     NULL: a streamed leaf structure is kept in pinned host
 *                 memory.  Otherwise the path of a file the library creates
 *                 (truncating any file there), writes the streamed structure
 *                 to (leaf-block layout, (4d + 4) n bytes) and removes at
 *                 bkd_free, for a reference set whose structure does not fit
 *                 in host memory (Section 3.2, last paragraph of "Processing
 *                 the Leaf Structure").  Chunks then travel disk -> pinned
 *                 staging buffer -> device in three overlapped stages: a
 *                 reader thread fills one of two staging buffers (direct I/O
 *                 where the file system allows it) while the other's copy to
 *                 the device and the scans of the resident chunk run.  Host
 *                 memory: two staging buffers of the chunk capacity.  Only
 *                 used when the structure is streamed (leaf_budget_bytes or
 *                 num_chunks).  The path is copied.
 * Results are identical for every value of these options.
 */
typedef struct bkd_options {
    int64_t buffer_size;
    int64_t fetch_size;
    int64_t leaf_budget_bytes;
    int32_t chunk_mode;
    int32_t num_chunks;
    int32_t device;
    int32_t flags;
    int64_t tail_max;
    int32_t split_rule;
    int32_t prune;
    const char *leaf_path;
} bkd_options;

/* Static facts of a built tree. */
typedef struct bkd_tree_info {
    int64_t n;            /* reference points                                  */
    int32_t d;            /* dimension                                         */
    int32_t height;       /* h: 2^h leaves, 2^h - 1 splitting values           */
    int64_t buffer_size;  /* effective B (-1: never half-full)                 */
    int64_t fetch_size;   /* effective M (-1: everything available)            */
    int32_t num_chunks;   /* 1 when resident                                   */
    int32_t resident;     /* 1: leaf structure lives on the device             */
    int64_t leaf_bytes;   /* bytes of the leaf structure (points + indices)    */
    int64_t chunk_capacity_bytes; /* bytes of one device chunk buffer          */
    int32_t on_disk;      /* 1: the streamed structure is read from leaf_path      */
    int32_t direct_io;    /* 1: reads bypass the page cache (O_DIRECT)             */
} bkd_tree_info;

/* Counters of the last query on a tree. */
typedef struct bkd_stats {
    int64_t queries;        /* m                                                  */
    int64_t fetches;        /* FindLeafBatch invocations                          */
    int64_t calls;          /* ProcessAllBuffers invocations                      */
    int64_t pairs;          /* (query, leaf point) pairs scanned                  */
    int64_t visits;         /* (query, leaf) visits                               */
    int64_t dense_launches; /* launches of the dense leaf scan (lane per query)    */
    int64_t dense_pairs;    /* pairs scanned by it                                */
    int64_t sparse_launches;/* launches of the sparse leaf scan (wave per query)  */
    int64_t sparse_pairs;   /* pairs scanned by it                                */
    int64_t chunk_copies;   /* host-to-device chunk copies                        */
    int64_t bytes_h2d;      /* bytes of those copies                              */
    double dense_ms;        /* sum of dense-scan launch durations (BKD_FLAG_TIMING)  */
    double sparse_ms;       /* sum of sparse-scan and tail launch durations (BKD_FLAG_TIMING) */
    double total_ms;        /* wall time of the query call on the host            */
    /* Algorithmic work.  A ProcessAllBuffers call reads every buffered leaf once    */
    /* (4d + 4 bytes per point: coordinates and index) and, per buffered query, its  */
    /* coordinates, its key list (read and written, 8 bytes per key each way) and    */
    /* its buffer entry: 4d + 16k + 4 bytes per visit.  A tail visit reads its leaf  */
    /* for its one query.                                                            */
    int64_t dense_visits;       /* visits scanned by the dense leaf scan              */
    int64_t leaf_points_dense;  /* points of the leaves the dense scan read, per call */
    int64_t leaf_points_other;  /* the same for the sparse scan and the tail          */
    int64_t alg_bytes;          /* leaf points (4d + 4) + visits (4d + 16k + 4)       */
    int64_t alg_bytes_dense;    /* the dense scan's part of alg_bytes                 */
    /* Phases (device time from HIP events with BKD_FLAG_TIMING, else 0).           */
    double find_ms;         /* FindLeafBatch launches (first round; routing inside   */
                            /* the scans of later rounds is part of the scans' time) */
    double group_ms;        /* buffer insertion: grouping by leaf, offsets, chunk      */
                            /* sweep redistribution                                   */
    double copy_ms;         /* host-to-device chunk copies (streamed structures)     */
    double wait_ms;         /* host time spent waiting for the device (readbacks and */
                            /* synchronisations inside the call) or for chunk reads   */
                            /* from a leaf file, always measured                     */
    int64_t bytes_disk;     /* bytes read from the leaf file (leaf_path), aligned reads */
    double disk_ms;         /* time the reader thread spent in those reads            */
} bkd_stats;

/* Thread-local description of the last error on this thread ("" if none). */
const char *bkd_last_error(void);

/* Library version string. */
const char *bkd_version(void);

/* Fill *out with the defaults for a tree of the given height.  Host only. */
int bkd_default_options(int32_t height, bkd_options *out);

/*
 * Build a buffer k-d tree (Section 2.3 construction, Section 3.1 host build).
 *   P       host pointer, row-major [n][d] float32, caller-owned; the library
 *           copies what it needs and keeps no pointer to P.
 *   n       1 <= n <= 2^31 - 1.
 *   d       1 <= d <= BKD_MAX_DIM.
 *   height  0 <= h <= BKD_MAX_HEIGHT and 2^h <= n.  A node holding c points
 *           splits dimension (level mod d) at the point of rank floor(c/2)
 *           under the order (coordinate, index): the left child takes the
 *           floor(c/2) smallest, the split value is the coordinate of the
 *           smallest point on the right, and a query goes left iff its
 *           coordinate is below the split value.  Leaves keep ascending index.
 *   opt     NULL for defaults.
 *   out     receives the tree handle, owned by the library until bkd_free.
 * Errors: BKD_EINVAL (NULL, ranges, non-finite P), BKD_EBUDGET, BKD_ENOMEM,
 * BKD_EDEVICE.
 */
int bkd_build(const float *P, int64_t n, int32_t d, int32_t height, const bkd_options *opt, bkd_tree **out);

/* Release a tree and all of its host and device memory.  NULL is a no-op. */
int bkd_free(bkd_tree *tree);

/*
 * Exact kNN of m queries (Algorithm 1), host pointers, blocking.
 *   Q         host [m][d] float32 (finite), caller-owned.
 *   m         0 <= m <= 2^31 - 1.
 *   k         1 <= k <= min(n, BKD_MAX_K).
 *   out_idx   host [m][k] int64, caller-owned.
 *   out_dist  host [m][k] float32, caller-owned.
 * Squared distances are computed in float32 as t_j = q_j - x_j (rounded),
 * acc = fma(t_j, t_j, acc) for j = 0..d-1 from +0; out_dist = sqrt(acc).
 * Errors: BKD_EINVAL, BKD_ENOMEM, BKD_EDEVICE.
 */
int bkd_query(bkd_tree *tree, const float *Q, int64_t m, int32_t k, int64_t *out_idx, float *out_dist);

/*
 * Same with device pointers, ordered on `stream` (a hipStream_t; NULL = the
 * null stream).  dQ, d_idx and d_dist must stay valid until the work on the
 * stream has completed.  The host takes part in the loop's control flow
 * (reading a few counters per iteration), so the call returns once the last
 * kernel is enqueued; synchronise the stream before reading the outputs.
 */
int bkd_query_async(bkd_tree *tree, const float *dQ, int64_t m, int32_t k, int64_t *d_idx, float *d_dist,
                    void *stream);

/*
 * bkd_query_async with no allocation, for callers that cannot allocate device
 * memory during a call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and ordering as
 * bkd_query_async.  The call's workspace is a fixed 64 MiB device array of the
 * library (one per device, held until the process ends) instead of the tree's
 * own buffers, so the call makes no hipMalloc, hipFree or other allocating
 * call.  The workspace a call needs is about m (8K + 4d + 33) + 20 * 2^h +
 * 8 KiB bytes (fifteen arrays, each rounded up to 256 bytes), K = the key
 * capacity >= k from {1, 2, 4, 5, 8, 10, 16, 32, 64}: about 440,000 queries
 * at d = 10, k = 10, h = 10.  Calls on one device share
 * the array: calls that overlap on one device (on different streams or host
 * threads) race and must not be made.  The tree must be resident (no leaf
 * budget) and built without BKD_FLAG_TRACE; per-launch timing is not recorded.
 * Errors: BKD_EINVAL (as bkd_query_async; a streamed or traced tree; a query
 * whose workspace exceeds 64 MiB, with both sizes in the message), BKD_EDEVICE.
 */
int bkd_query_async_noalloc(bkd_tree *tree, const float *dQ, int64_t m, int32_t k, int64_t *d_idx, float *d_dist,
                            void *stream);

/*
 * Proximity-based outlier scores (Section 4, large-scale outlier detection):
 * the all-nearest-neighbours problem over the tree's own reference set.  The
 * score of reference point i is the mean of the float32 distances (as
 * bkd_query returns them) to its k nearest other reference points: the k + 1
 * nearest are searched with the tree's query path, i's own entry is dropped
 * (when more than k other points share i's coordinates with smaller indices
 * it is not among them, and the first k are kept), and the k distances are
 * summed in ascending order in float64 and divided by k.  The ranking lists
 * the points by score, largest first, equal scores by smaller index.
 *   tree       built from P.
 *   P          host [n][d] float32, row-major: the same array the tree was
 *              built from (rows are matched to tree points by index).
 *   n          must equal the tree's n.
 *   k          1 <= k <= min(n - 1, BKD_MAX_K - 1).
 *   out_score  host [n] float32, caller-owned: out_score[i] is point i's score.
 *   out_order  host [n] int64, caller-owned: point indices, highest score first.
 * Blocking.  Uses the tree's host-pointer stream, like bkd_query, and
 * allocates device memory for the sort during the call.
 * Errors: BKD_EINVAL (NULL pointers, n or k out of range, non-finite P),
 * BKD_ENOMEM, BKD_EDEVICE.
 */
int bkd_outlier_scores(bkd_tree *tree, const float *P, int64_t n, int32_t k, float *out_score, int64_t *out_order);

/* Static facts of the tree. */
int bkd_tree_info_get(const bkd_tree *tree, bkd_tree_info *out);

/*
 * Copy out the serialized tree: split [2^h - 1] (heap order), leaf_off
 * [2^h + 1] (leaf l holds leaf-structure positions [leaf_off[l],
 * leaf_off[l+1])) and perm [n] (index of the point at each position).
 * Any pointer may be NULL to skip that array.
 */
int bkd_tree_export(const bkd_tree *tree, float *split, int64_t *leaf_off, int32_t *perm);

/*
 * The tree's splitting dimensions and node boxes: dims [2^h - 1] receives the
 * dimension of every internal node (heap order; level mod d under
 * BKD_SPLIT_CYCLIC); box [(2^(h+1) - 1) * 2d], heap order over all nodes
 * (internal, then leaves), node v's minima at box[v*2d .. v*2d + d) and maxima
 * after them, is filled for a tree built with BKD_PRUNE_BOX (BKD_EINVAL
 * otherwise).  Either pointer may be NULL.
 */
int bkd_tree_rules_export(const bkd_tree *tree, int32_t *dims, float *box);

/* Chunk bounds (positions [lo[j], hi[j])) of the streaming plan; num_chunks entries. */
int bkd_chunk_plan(const bkd_tree *tree, int64_t *lo, int64_t *hi);

/* Counters of the last query. */
int bkd_last_stats(const bkd_tree *tree, bkd_stats *out);

/*
 * Trace of the last query when BKD_FLAG_TRACE is set: for every
 * ProcessAllBuffers call c, the (query, leaf) pairs fetched since the
 * previous call in fetch order, entries call_off[c] .. call_off[c+1]-1;
 * leaf -1 marks a query whose traversal finished.  bkd_trace_size gives the
 * sizes; bkd_trace_get fills caller arrays of those sizes.
 */
int bkd_trace_size(const bkd_tree *tree, int64_t *ncalls, int64_t *length);
int bkd_trace_get(const bkd_tree *tree, int64_t *call_off, int32_t *query, int32_t *leaf);

/* ------------------------------------------------------------------------ */
/* Batched form: many independent instances in one persistent launch.       */
/*                                                                          */
/* Every instance is a complete problem of Section 2.2 with its own P, Q, d, */
/* k and height, answered by the buffered search of Algorithm 1 in lock-step */
/* rounds.  All instances run inside one persistent kernel, captured in a    */
/* HIP graph: a device task queue hands out routing tasks (FindLeafBatch and */
/* buffer insertion of one instance, one workgroup) and scan tasks (the leaf */
/* scans of a group of that instance's buffered leaves), and each instance   */
/* advances to its next round as soon as its own scans are done, with no    */
/* barrier across instances.  Within a leaf the order of buffered queries is */
/* unspecified in this form; results are the same as bkd_query's.           */

typedef struct bkd_instance {
    const float *P;     /* [n][d] float32, finite; host (device: BKD_FLAG_DEVICE_PTRS) */
    int64_t n;          /* 1 <= n <= 2^31 - 1                                       */
    const float *Q;     /* [m][d] float32, finite; host (device: BKD_FLAG_DEVICE_PTRS) */
    int64_t m;          /* 0 <= m <= 2^31 - 1                                       */
    int32_t d;          /* 1 <= d <= BKD_MAX_DIM                                    */
    int32_t k;          /* 1 <= k <= min(n, BKD_MAX_K)                              */
    int32_t height;     /* 0 <= h <= 12 and 2^h <= n                                */
    int64_t *out_idx;   /* [m][k], filled by bkd_batch_results; host or device      */
    float *out_dist;    /* [m][k], filled by bkd_batch_results; host or device      */
} bkd_instance;

/* Schedule of the persistent launch (results do not depend on it). */
typedef struct bkd_tuning {
    int32_t leaves_per_task; /* pieces per scan task (1..256; a piece: up to 32 buffered      */
                             /* queries of one leaf); 0: default 8                           */
    int32_t groups_per_cu;   /* persistent workgroups per compute unit (1..16); 0: default 4  */
    int32_t solo_max;        /* once an instance has at most this many active queries, each  */
                             /* finishes its traversal alone (one wave per query); 0: 2048   */
} bkd_tuning;

typedef struct bkd_batch_stats {
    int64_t instances, queries;
    int64_t tasks;      /* tasks executed by the last run                          */
    int64_t rounds;     /* sum over instances of lock-step rounds                   */
    int64_t pairs;      /* (query, leaf point) pairs scanned                        */
    int64_t flops;      /* 3 d flops per pair, summed over instances                */
    double run_ms;      /* device time of the last run (graph launch)               */
    int32_t error;      /* nonzero: the last run stopped early (queue overflow or   */
                        /* stall guard); its results are not valid                  */
    int32_t workgroups; /* persistent workgroups of the last run                    */
    double claim_wait_ms; /* time workgroups spent waiting for a task, summed       */
} bkd_batch_stats;

typedef struct bkd_batch bkd_batch;

/*
 * Build every instance's tree on the host (Section 3.1) and upload trees and
 * queries to `device`.  The library copies P and Q; the out_* pointers are
 * kept and written by bkd_batch_results.  flags: BKD_FLAG_SQUARED and
 * BKD_FLAG_DEVICE_PTRS (P, Q and the outputs of every instance are device
 * memory on `device`: P and Q are read back for the host build, results are
 * copied device to device).  Errors: BKD_EINVAL (any instance's arguments,
 * with its index in the message, including a pointer that is not device
 * memory under BKD_FLAG_DEVICE_PTRS), BKD_ENOMEM, BKD_EDEVICE.
 */
int bkd_batch_create(const bkd_instance *inst, int32_t count, int32_t device, int32_t flags, bkd_batch **out);

/*
 * Answer every instance: one launch of the captured graph (state reset, then
 * the persistent kernel) on `stream` (a hipStream_t; NULL = null stream).
 * tune NULL: the tuning chosen by bkd_batch_autotune, else the defaults.
 * Results stay in device memory; the call returns once the graph is launched.
 */
int bkd_batch_run(bkd_batch *batch, const bkd_tuning *tune, void *stream);

/* Synchronise and copy every instance's results to its out_idx / out_dist. */
int bkd_batch_results(bkd_batch *batch);

/*
 * Time a set of candidate tunings on this batch (each run in full, after one
 * warm-up run) and keep the fastest for later bkd_batch_run(batch, NULL, ...).
 * *best and *best_ms (either may be NULL) receive the winner.
 */
int bkd_batch_autotune(bkd_batch *batch, bkd_tuning *best, double *best_ms);

/*
 * Persistent tuning cache (a text file, one line per batch signature: the device's architecture
 * name and compute-unit count and every instance's n, m, d, k and height).  _save writes the
 * batch's tuning (from bkd_batch_autotune or an earlier _load) in place of any line of the same
 * signature; BKD_EINVAL if the batch is untuned or the file cannot be written.  _load makes the
 * cached tuning the batch's own, as bkd_batch_autotune would, and copies it to *tuning (may be
 * NULL); BKD_ENOTFOUND if the file or its line is missing.  The caller owns the path string.
 */
int bkd_batch_tuning_save(const bkd_batch *batch, const char *path);
int bkd_batch_tuning_load(bkd_batch *batch, const char *path, bkd_tuning *tuning);

int bkd_batch_stats_get(const bkd_batch *batch, bkd_batch_stats *out);
int bkd_batch_free(bkd_batch *batch);

/* ------------------------------------------------------------------------ */
/* Served form: resident trees, continuous batching of query requests.      */
/*                                                                          */
/* A server answers requests (a batch of m queries, its own k, on one of its */
/* trees) as they arrive.  Each (tree, key capacity) pair is served by a    */
/* session that runs lock-step rounds of Algorithm 1 continuously on its own */
/* stream; between two rounds it admits waiting requests, in arrival order, */
/* whose queries fit into its free query slots (on-the-fly insertion of new */
/* indices, Section 3.2).  Admitted queries share the leaf buffers of every */
/* query already in flight on that tree.  A request completes when its last */
/* query finishes; its results are then copied to the caller's arrays.     */
/* Results are the same as bkd_query's, alone or in any mix of requests.    */

#define BKD_REQ_WAITING 0
#define BKD_REQ_RUNNING 1
#define BKD_REQ_DONE 2
#define BKD_REQ_CANCELLED 3

typedef struct bkd_server_opts {
    int64_t slots_per_session; /* query slots of one session (its memory: 4d + 8K + 36 bytes     */
                               /* per slot, K = key capacity >= k); 0: 2^20                       */
    int32_t max_requests;      /* requests in flight per session; 0: 4096                        */
    int32_t device;            /* HIP device of the server (trees must live there)               */
    int32_t flags;             /* BKD_FLAG_SQUARED or 0                                          */
    int32_t age_max;           /* > 0: a query still travelling after this many rounds leaves     */
                               /* the rounds and walks the rest of its traversal alone (one       */
                               /* workgroup), so long walks do not hold a request; 0: never       */
    int64_t tail_max;          /* a round with at most this many queries in flight hands them    */
                               /* all to single walks; 0: 16384; < 0: never                       */
    int32_t straggle_max;      /* > 0: once a request has at most this many queries travelling,   */
                               /* they leave the rounds for single walks (its slowest walks do    */
                               /* not hold it one round per leaf); 0: never                       */
} bkd_server_opts;

typedef struct bkd_server bkd_server;

int bkd_server_create(const bkd_server_opts *opts, bkd_server **out);

/* Serve a built, resident tree (leaf_budget_bytes 0); the tree must outlive the server. */
int bkd_server_add_tree(bkd_server *srv, bkd_tree *tree, int32_t *tree_id);

/*
 * Submit a request: Q host [m][d] (copied), 1 <= m <= slots_per_session,
 * 1 <= k <= min(n, 64); out_idx [m][k] and out_dist [m][k] are host arrays the
 * caller keeps valid until the request is done.  Returns at once with
 * *req_id.  Errors: BKD_EINVAL, BKD_ENOTFOUND (tree id), BKD_EBUSY (m larger
 * than a session's slots: it could never be admitted), BKD_EDEVICE.
 */
int bkd_submit(bkd_server *srv, int32_t tree_id, const float *Q, int64_t m, int32_t k, int64_t *out_idx,
               float *out_dist, int64_t *req_id);

/* Request state: BKD_REQ_*. */
int bkd_poll(bkd_server *srv, int64_t req_id, int32_t *state);

/* Block until the request is done or cancelled; timeout_us < 0 waits forever (else BKD_ETIMEOUT). */
int bkd_wait(bkd_server *srv, int64_t req_id, int64_t timeout_us);

/* Cancel a request: a waiting request is dropped; a running one completes with state CANCELLED. */
int bkd_cancel(bkd_server *srv, int64_t req_id);

/* Host steady-clock times (seconds) of submission, admission and completion. */
int bkd_request_times(bkd_server *srv, int64_t req_id, double *submit_s, double *admit_s, double *done_s);

/* Forget a finished request (its id becomes unknown). */
int bkd_release(bkd_server *srv, int64_t req_id);

/* Counters of a server since its creation, summed over its sessions. */
typedef struct bkd_server_stats {
    int32_t sessions;       /* (tree, key capacity) sessions created                         */
    int64_t rounds;         /* routing rounds                                                 */
    int64_t scan_rounds;    /* rounds that scanned buffers with the dense/sparse kernels      */
    int64_t tail_rounds;    /* rounds handed to the one-workgroup-per-query tail kernel       */
    int64_t queries;        /* queries admitted                                               */
    double busy_s;          /* host wall time inside rounds, summed over sessions             */
    double admit_s;         /* host wall time admitting requests (copies in), summed          */
    double complete_s;      /* host wall time delivering results (copies out), summed         */
    int64_t direct_launches;/* launches of the direct path: requests of at most 2048 queries  */
                            /* skip the rounds, each query walking its whole traversal in one */
                            /* workgroup right after admission                                 */
    int64_t aged_queries;   /* queries handed from the rounds to single walks (age_max,       */
                            /* straggle_max)                                                  */
} bkd_server_stats;

int bkd_server_stats_get(bkd_server *srv, bkd_server_stats *out);

/* Stop every session and free the server (trees are not freed). */
int bkd_server_destroy(bkd_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* BKD_H */
