// internal.h -- shared host-side declarations of the bkd library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/bkd.h"

namespace bkd {

// ---------------------------------------------------------------------------
// Errors: every failure becomes a BkdError caught at the ABI boundary.

struct BkdError {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void set_error(int code, const std::string &msg);
void clear_error();

#define BKD_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            ::bkd::fail(e_ == hipErrorOutOfMemory ? BKD_ENOMEM : BKD_EDEVICE,                      \
                        std::string(#call) + ": " + hipGetErrorString(e_));                        \
    } while (0)

// Parallel loop on host threads (no OpenMP runtime inside the library).
void parallel_for(int64_t count, const std::function<void(int64_t, int64_t)> &body, int64_t grain = 1);
int host_threads();

// ---------------------------------------------------------------------------
// Device buffers.

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need);  // grow (contents not preserved)
    void release();
    template <class T> T *as() const { return static_cast<T *>(p); }
    ~DevBuf() { release(); }
};

struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void ensure(size_t need);
    void release();
    template <class T> T *as() const { return static_cast<T *>(p); }
    ~PinnedBuf() { release(); }
};

// ---------------------------------------------------------------------------
// Canonical tree on the host.

struct HostTree {
    int64_t n = 0;
    int d = 0;
    int h = 0;
    std::vector<float> split;      // 2^h - 1
    std::vector<int64_t> leaf_off; // 2^h + 1
    std::vector<int32_t> perm;     // n
    std::vector<uint8_t> dims;     // 2^h - 1 splitting dimensions (BKD_SPLIT_LONGEST); empty: level mod d
    std::vector<float> box;        // (2^(h+1) - 1) x 2d node boxes (BKD_PRUNE_BOX); empty: plane pruning
};

// Build the canonical tree of P (row-major n x d) under a splitting rule (BKD_SPLIT_*);
// parallel = use the host thread pool.
void build_canonical(const float *P, int64_t n, int d, int h, HostTree &t, bool parallel = true,
                     int rule = BKD_SPLIT_CYCLIC);
// Bounding boxes of every node's points (HostTree::box) from the built tree.
void build_boxes(const float *P, HostTree &t);
// The same tree built on the current device (one segmented sort per level); blocking on s.
void build_canonical_device(const float *P, int64_t n, int d, int h, HostTree &t, hipStream_t s);

// Leaf-block layout of the leaf structure: leaf l occupies 4-byte words
// [blk[l], blk[l+1]): d rows of len_l float32 coordinates (row j holds
// coordinate j of the leaf's points in position order), then len_l int32
// original indices.  Any run of consecutive leaves is one contiguous range.
//
// One chunk of the streaming plan: it serves positions [lo, hi) and holds the
// whole blocks of leaves [leaf_first, leaf_last] (host words [word_lo, word_hi)).
struct Chunk {
    int64_t lo, hi;
    int32_t leaf_first, leaf_last;
    int64_t word_lo, word_hi;
};

// Device control words (one small array per tree, read back by the host).
enum Ctl : int {
    CTL_MAXCNT = 0,   // largest buffer fill since the last call
    CTL_WIDE = 1,     // a query coordinate beyond +-FILTER_RANGE seen (the dense scan then skips its filter)
    CTL_V = 2,        // buffered entries of the current call
    CTL_T = 3,        // work items of the current call
    CTL_BAD = 4,      // non-finite query coordinate seen
    CTL_S = 5,        // sparse (one wave per buffered query) items of the current call
    CTL_VISITS_LO = 6, // 64-bit counters (two words each)
    CTL_DPAIRS_LO = 8,
    CTL_SPAIRS_LO = 10,
    CTL_LPD_LO = 12,     // points of the leaves scanned densely, each leaf once per call
    CTL_LPS_LO = 14,     // points of the leaves scanned sparsely, and the tail's leaf reads
    CTL_DVISITS_LO = 16, // visits scanned densely
    CTL_AGED = 18,       // served form: routed queries handed to the tail for their age
    CTL_WORDS = 24
};

// Query-tile width of the dense leaf scan (queries per work item), and the
// buffer fill below which a leaf is scanned with one wave per buffered query.
// A single call scans every buffered leaf densely: one staged read of a leaf
// with the matrix-core filter costs about what one wave streaming the whole
// leaf for one query does, and less from two queries on.  1 against 4: 0.8%
// faster on the 2^22-point, 4096-point-leaf workload (55.2 -> 54.8 ms per
// call), 7.5% on the 2^28-point, 16384-point-leaf one streamed in 12 chunks
// (4.91 -> 4.54 s) and 1.7% resident; 2 within 0.4% of 4.  (4 against 32 had
// measured 1.3% and 19% faster.)
constexpr int SCAN_QT = 256;
constexpr int SCAN_DENSE_MIN = 1;

// Disk-backed leaf structure (bkd_options.leaf_path): chunks are read from the
// file into two pinned staging buffers by a reader thread, then copied to the
// device chunk buffers (leaffile.cpp).
struct LeafFile;
void leaffile_create(struct Tree &t, const float *P, const char *path);
void leaffile_destroy(struct Tree &t);
// Ask for chunk j to be read ahead (no-op if it is already read, being read, or no
// staging buffer is free).
void leaffile_prefetch(struct Tree &t, int j);
// Copy chunk j to device buffer dst on stream s (after the copy stream waits for
// `after`): waits until the chunk is in a staging buffer, queues the copy, and
// releases the staging buffer once the copy completes.  Returns the host wait in ms.
double leaffile_copy(struct Tree &t, int j, void *dst, hipStream_t s);
// Bytes read and milliseconds spent reading since the last call (per query statistics).
void leaffile_take_stats(struct Tree &t, int64_t *bytes, double *ms);
bool leaffile_direct(const struct Tree &t);
// Write the blocks of leaves [lf, ll] of P's leaf structure to dst (word 0 = first word of leaf lf).
void gather_leaves(const float *P, const struct Tree &t, int lf, int ll, void *dst);

struct Tree {
    HostTree host;
    bkd_options opt{};
    int64_t B = 0, M = 0;  // effective; -1 = unlimited
    int device = 0;
    int nleaf = 1;

    // device top tree and leaf bounds; per-node dimensions and boxes of a variant tree
    DevBuf d_split, d_leaf_off, d_dims, d_box;

    // leaf structure
    std::vector<int64_t> leaf_blk; // [nleaf+1] word offsets of the leaf blocks
    DevBuf d_leaf_blk;
    DevBuf d_centers;              // [nleaf][d] float32 bounding-box midpoints, then [nleaf] leaf scales
    bool resident = true;
    // buffers of at least this many queries go to the dense scan: SCAN_DENSE_MIN, or never
    // (INT32_MAX) when a leaf holds 2^30 points or more (the dense scan addresses a leaf's
    // rows with 32-bit byte offsets)
    int dense_min = SCAN_DENSE_MIN;
    bool wide = false;             // a reference coordinate beyond +-FILTER_RANGE
    bool sweep = false;            // streaming with the chunk-sweep schedule
    std::vector<Chunk> chunks;
    size_t chunk_cap_bytes = 0;
    DevBuf d_chunk[2];     // resident: d_chunk[0] holds everything
    int chunk_in[2] = {-1, -1};
    PinnedBuf h_leaf;      // streaming: pinned host copy of the leaf structure (no leaf file)
    LeafFile *leaf_file = nullptr;  // streaming from a file (leaf_path), else null
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_copied[2] = {nullptr, nullptr};
    hipEvent_t ev_used[2] = {nullptr, nullptr};
    hipEvent_t ev_rb = nullptr;  // readback of the control words

    // query workspace
    DevBuf d_Q, d_outi, d_outd;
    DevBuf d_Qp, d_perm;  // lock-step rounds: queries renumbered in first-leaf order
    DevBuf d_keys, d_kth, d_node, d_ring, d_pleaf, d_pq, d_tleaf, d_tq, d_hist;
    DevBuf d_cnt, d_cnt0, d_off, d_tiles, d_ctl;  // d_cnt0: run starts of the sorted pending list
    DevBuf d_chunk_of, d_rleaf, d_rq, d_rcnt;  // chunk sweep: leaf -> chunk, per-chunk pending regions
    PinnedBuf h_rcnt;
    PinnedBuf h_ctl, h_tiles;  // h_tiles: dense tiles, sparse items, buffer offsets (3 x (nleaf+1))

    // variant-tree arrays on the device, or null under the original rules
    const uint8_t *dims_dev() const { return host.dims.empty() ? nullptr : d_dims.as<uint8_t>(); }
    const float *boxes_dev() const { return host.box.empty() ? nullptr : d_box.as<float>(); }

    // results of the last query
    bkd_stats stats{};
    std::vector<int64_t> trace_off;
    std::vector<int32_t> trace_q, trace_leaf;
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels.hip, scan_*.hip).

struct FetchSpec {
    const int32_t *ring;  // reinsert ring
    int64_t ring_head, ring_count, ring_cap;
    int64_t in_start, in_count;  // input queue part: queries in_start .. in_start + in_count - 1
    const int32_t *in_list = nullptr;  // if set, the input part holds in_list[in_start ..] instead
    // served form: owning request, outstanding-query counters and the completion list
    const int32_t *req_of = nullptr;
    int32_t *req_left = nullptr;
    int32_t *done_list = nullptr;  // done_list[0] = count, then request table indices
    // Algorithm 1 schedule: record the largest buffer fill (the half-full trigger);
    // other schedules only need the per-leaf counts, and the lock-step rounds take
    // those from the sorted list instead (count_leaves false: no atomics).
    bool track_fill = false;
    bool count_leaves = true;
    // variant tree (Section 2.3): per-node splitting dimensions (null: level mod d) and node
    // boxes for the pruning test (null: the splitting hyperplane)
    const uint8_t *dims = nullptr;
    const float *boxes = nullptr;
    // served form: rounds each query has been routed (null: not tracked); a query routed more
    // than age_max times leaves the rounds: its entry gets the key 2^h + 1 (sorted after the
    // finished ones) and it is counted in ctl[CTL_AGED]
    int32_t *age = nullptr;
    int32_t age_max = 0;
    // served form: a query whose request has at most this many queries still travelling
    // leaves the rounds the same way (0: never; needs req_of and req_left)
    int32_t strag_max = 0;
};

void launch_init_state(int32_t *node, uint64_t *keys, uint32_t *kth, int64_t m, int K, hipStream_t s);
void launch_check_finite(const float *Q, int64_t count, int32_t *ctl, hipStream_t s);
void launch_find_leaf(const FetchSpec &f, const float *Q, int d, int32_t *node, const uint32_t *kth,
                      const float *split, int h, uint32_t *pend_leaf, int32_t *pend_q, int64_t pend_base,
                      int32_t *cnt, int32_t *ctl, hipStream_t s);
// Stable sort of (leaf, query) pairs by leaf; returns which buffer holds the result (0: a, 1: b).
// With dcount the pair count is read on the device (*dcount <= count; count sizes the grids).
int launch_sort_pairs(uint32_t *key_a, int32_t *val_a, uint32_t *key_b, int32_t *val_b, int64_t count, int key_bits,
                      uint32_t *hist, hipStream_t s, const int32_t *dcount = nullptr);
size_t sort_hist_words(int64_t count);
// Grouping of (leaf, query) pairs by leaf in one pass, order within a leaf unspecified, for
// at most bucket_max_keys() distinct keys: launch_bucket_count writes per-block key counts
// and their column prefixes into hist and returns the key totals (inside hist);
// launch_bucket_scatter then places the pairs, key k starting at off[k].  Keys are counted
// relative to key_base (key - key_base in [0, nb); others are skipped) and written as they
// are; with dcount the pair count is read on the device and count only bounds it.
int bucket_max_keys();
const int32_t *launch_bucket_count(const uint32_t *keys, int64_t count, int nb, uint32_t *hist,
                                   hipStream_t s, uint32_t key_base = 0, const int32_t *dcount = nullptr);
void launch_bucket_scatter(const uint32_t *kin, const int32_t *vin, uint32_t *kout, int32_t *vout, int64_t count,
                           int nb, const uint32_t *hist, const int32_t *off, hipStream_t s, uint32_t key_base = 0,
                           const int32_t *dcount = nullptr);
// tiles: [2][nleaf+1] -- dense work-item offsets, then sparse (per buffered query) offsets.
// count_work: also add the visits and pairs of scanning every buffer to the ctl counters.
void launch_leaf_offsets(const int32_t *cnt, const int32_t *start, const int32_t *leaf_off, int nleaf, int qt,
                         int dense_min, int32_t *off, int32_t *tiles, int32_t *sparse, int32_t *ctl, hipStream_t s,
                         bool count_work = false);
void launch_run_bounds(const uint32_t *leaf, int64_t count, int nleaf, int32_t *start, int32_t *end, hipStream_t s,
                       const int32_t *dcount = nullptr);
// The chunk sweep's distribution counts its targets (the chunks and a side buffer) in LDS.
constexpr int DISTRIBUTE_MAX_TARGETS = 1024;
void launch_distribute(const uint32_t *leaf, const int32_t *q, int64_t n, int nleaf, const int32_t *chunk_of, int c,
                       uint32_t *rleaf, int32_t *rq, int64_t rcap, int32_t *rcnt, uint32_t *sleaf, int32_t *sq,
                       int nchunks, hipStream_t s, const int32_t *dn = nullptr);
void launch_restore(const uint32_t *sleaf, const int32_t *sq, int64_t n, uint32_t *rleaf, int32_t *rq, int32_t *rcnt,
                    int c, int nchunks, hipStream_t s);
void launch_count_work(const int32_t *off, const int32_t *leaf_off, int lf, int ll, int dense_min, int32_t *ctl,
                       hipStream_t s);
void launch_ring_append(int32_t *ring, int64_t cap, int64_t tail, const int32_t *src, int64_t count, hipStream_t s);
void launch_finalize(const uint64_t *keys, int K, int k, int64_t m, const int32_t *perm, int64_t *idx, float *dist,
                     bool squared, hipStream_t s);
void launch_localize(int32_t *ids, const uint32_t *leaf, int64_t m, int d, const float *Q, float *Qp, int32_t *perm,
                     int32_t *node, int h, hipStream_t s);
void launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s);

// Leaves at least this large get the tail kernel's 512-lane workgroups.
constexpr int TAIL_WIDE_LEAF = 2048;

struct ScanArgs {
    const int32_t *tiles;     // [nleaf+1] dense work-item offsets
    const int32_t *sparse;    // [nleaf+1] sparse work-item offsets
    const int32_t *off;       // [nleaf+1] buffer offsets
    const int32_t *bufq;      // buffered query ids, leaf order
    const int32_t *leaf_off;  // [nleaf+1] leaf positions
    const float *base;        // device buffer holding the leaf blocks of this launch
    const int64_t *blk;       // [nleaf+1] word offsets of the leaf blocks in the whole structure
    int64_t blk_shift;        // added to blk[l] to address the buffer (minus the buffer's first word)
    int64_t chunk_lo, chunk_hi;  // positions served by this launch
    int32_t item_first, item_count;    // dense items of this launch
    int exact_only;                    // dense scan: exact distances for every pair, no filter
    const int32_t *wide_flag;          // dense scan: if set and nonzero on the device, likewise
    const int32_t *dev_counts;         // if set, the dense item count is dev_counts[CTL_T] and
                                       // item_count is only an upper bound that sizes the grid
    // lock-step rounds: if set, every scanned query also takes its next FindLeafBatch step
    // here (node[q] updated, its next leaf, or 2^h when done, stored at its list position)
    uint32_t *route_leaf;
    int32_t sitem_first, sitem_count;  // sparse items of this launch
    int32_t leaf_first, leaf_last;
    const float *Q;           // [m][d]
    int d;
    uint64_t *keys;           // [m][K]
    uint32_t *kth;            // [m] high word of each query's k-th key (its pruning distance)
    const float *centers;     // [nleaf][d] leaf centres of the inner-product filter
    const float *scales;      // [nleaf] power of two bringing a leaf's centred coordinates into [-1, 1]
    // tail of the lock-step schedule (resident structure): pending (leaf, query) entries
    // that each finish their whole traversal in one workgroup
    const uint32_t *tail_leaf;
    const int32_t *tail_q;
    int32_t tail_count;
    int tail_counted;         // the first visit of each tail entry is already in the work counters
    int tail_wide;            // tail workgroups of 512 lanes (leaves of TAIL_WIDE_LEAF points and more)
    int tail_from_node;       // each tail entry starts at the leaf in node[q] (tail_leaf unused)
    int32_t *node;            // [m] traversal state, set to DONE at the end
    const float *split;       // [2^h - 1]
    int h, k;                 // tree height; k of the query (pruning uses the k-th key)
    int32_t *ctl;             // visit and pair counters
    // served form: per-query k (else k), owning request, outstanding-query counters, completion list
    const int32_t *kq;
    const int32_t *req_of;
    int32_t *req_left;
    int32_t *done_list;
    // variant tree: per-node splitting dimensions and node boxes (null: the original rules)
    const uint8_t *dims;
    const float *boxes;
};

// Default number of pending queries at or below which the lock-step rounds hand over to
// the tail kernel (bkd_options.tail_max).
constexpr int64_t TAIL_MAX = 32768;

// Coordinates up to this magnitude keep every quantity of the dense scan's
// inner-product filter (centred coordinates, the leaf scales and the scaled
// query offsets) finite and normal-ranged at d <= 32; beyond it the scan takes
// its exact path for every point.
constexpr float FILTER_RANGE = 0x1p59f;

// Dispatch on padded dimension and key capacity; sparse = 0: dense items, 1: sparse items,
// 2: the tail (tail_count pending entries, one workgroup each).
void launch_leaf_scan(const ScanArgs &a, int K, int sparse, hipStream_t s);
int padded_dim(int d);
int key_capacity(int k);

// ---------------------------------------------------------------------------
// Host driver (query.cpp).

void tree_build(Tree &t, const float *P, int64_t n, int d, int h, const bkd_options &opt);
int guarded_call(const std::function<void()> &f);

// Device workspace of one query call on a resident structure: key lists,
// traversal state, the reinsert ring, the two pending-pair buffers, grouping
// scratch, per-leaf counts and offsets, and the renumbered query copy.
struct Workspace {
    uint64_t *keys;
    uint32_t *kth;
    int32_t *node, *ring;
    uint32_t *pleaf, *tleaf;
    int32_t *pq, *tq;
    uint32_t *hist;
    int32_t *cnt, *cnt0, *off, *tiles;
    float *Qp;
    int32_t *perm;
};

// Bytes of that workspace for m queries with k neighbours on tree t (each array
// 256-byte aligned), and its layout inside a caller-provided region.
size_t workspace_bytes(const Tree &t, int64_t m, int k);
Workspace workspace_in(const Tree &t, int64_t m, int k, void *region);

// One query call.  region == nullptr: the tree's own workspace, grown on demand.
// Otherwise the call uses `region` (workspace_bytes(t, m, k) bytes of device
// memory) and allocates nothing: the structure must be resident, and neither
// the trace nor per-launch timing is recorded.
void tree_query_device(Tree &t, const float *dQ, int64_t m, int k, int64_t *d_idx, float *d_dist, hipStream_t s,
                       void *region = nullptr);

}  // namespace bkd

// The ABI's tree handle.
struct bkd_tree {
    bkd::Tree t;
    hipStream_t stream = nullptr;  // stream of the host-pointer entry point
};
