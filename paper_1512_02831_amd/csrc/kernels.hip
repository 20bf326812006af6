// kernels.hip -- integer and traversal kernels of the query loop (gfx950, wave64).
//
//   k_find_leaf     FindLeafBatch (Algorithm 1; search phases of Section 2.3)
//   k_radix_*       stable buffer insertion: fetched (leaf, query) pairs are
//                   grouped by leaf in fetch order (Algorithm 1, buffer insert)
//   k_leaf_offsets  buffer offsets and work items of one ProcessAllBuffers call
//   k_ring_append   reinsert queue append (Algorithm 1)
//   k_finalize      keys -> (index, Euclidean distance)
#include <hip/hip_runtime.h>

#include <climits>

#include "internal.h"
#include "traverse.h"

namespace bkd {

namespace {


inline unsigned grid_for(int64_t count, int threads) { return (unsigned)((count + threads - 1) / threads); }

__device__ inline uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

constexpr int FIND_LDS_SPLITS = 2047;  // heap nodes of the top 11 levels
constexpr int FIND_LDS_DIMS = 16;      // queries of up to this dimension walk from LDS

// ---------------------------------------------------------------------------

__global__ void k_init_state(int32_t *node, uint64_t *keys, uint32_t *kth, int64_t m, int K)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        node[i] = NODE_FRESH;
        kth[i] = (uint32_t)(EMPTY_KEY >> 32);
    }
    int64_t total = m * K;
    for (int64_t j = i; j < total; j += (int64_t)gridDim.x * blockDim.x) keys[j] = EMPTY_KEY;
}

__global__ void k_check_finite(const float *Q, int64_t count, int32_t *ctl)
{
    bool bad = false, wide = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = Q[i];
        bad |= !isfinite(v);
        wide |= fabsf(v) > FILTER_RANGE;
    }
    if (__ballot(bad) != 0ull && __lane_id() == 0) atomicOr(&ctl[CTL_BAD], 1);
    if (__ballot(wide) != 0ull && __lane_id() == 0) atomicOr(&ctl[CTL_WIDE], 1);
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ __launch_bounds__(256) void k_find_leaf(FetchSpec f, const float *__restrict__ Q, int d,
                                                   int32_t *__restrict__ node, const uint32_t *__restrict__ kth,
                                                   const float *__restrict__ split, int h,
                                                   uint32_t *__restrict__ pend_leaf, int32_t *__restrict__ pend_q,
                                                   int64_t pend_base, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ ctl)
{
    // the upper levels of the split array, shared by every walk of the block, and each
    // lane's query (coordinate-major, so lanes at different levels hit distinct banks)
    __shared__ float split_lds[FIND_LDS_SPLITS];
    __shared__ float q_lds[FIND_LDS_DIMS * 256];
    const int lds_nodes = min((1 << h) - 1, FIND_LDS_SPLITS);
    for (int i = threadIdx.x; i < lds_nodes; i += blockDim.x) split_lds[i] = split[i];
    __syncthreads();
    const int64_t total = f.ring_count + f.in_count;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t first = (1 << h) - 1;
    const uint32_t nleaf = 1u << h;
    int32_t fill = 0;
    bool valid = false;
    uint32_t leaf = nleaf;
    if (j < total) {
        int32_t q;
        if (j < f.ring_count) {
            int64_t r = f.ring_head + j;  // ring_head < ring_cap and ring_count <= ring_cap
            if (r >= f.ring_cap) r -= f.ring_cap;
            q = f.ring[r];
        }
        else if (f.in_list) q = f.in_list[f.in_start + (j - f.ring_count)];
        else q = (int32_t)(f.in_start + (j - f.ring_count));
        const float *qp = Q + (int64_t)q * d;
        const int32_t st = node[q];
        int32_t v;
        if (f.dims || f.boxes) {
            v = next_leaf_rules(st, qp, kth + q, split, f.dims, f.boxes, h, d);
        } else if (d <= FIND_LDS_DIMS) {
            float *ql = q_lds + threadIdx.x;
            for (int c = 0; c < d; c++) ql[c * 256] = qp[c];
            v = next_leaf(st, ql, kth + q, split, split_lds, lds_nodes, h, d, 256);
        } else {
            v = next_leaf(st, qp, kth + q, split, split_lds, lds_nodes, h, d);
        }
        node[q] = v;
        if (f.req_left && v == NODE_DONE && st != NODE_DONE) {
            // last query of its request: record the request as complete
            const int32_t r = f.req_of[q];
            if (atomicSub(&f.req_left[r], 1) == 1) f.done_list[1 + atomicAdd(&f.done_list[0], 1)] = r;
        }
        leaf = (v >= 0) ? (uint32_t)(v - first) : nleaf;
        if (f.age && v >= 0 && ++f.age[q] > f.age_max) {
            // a long traversal leaves the rounds: the tail walks it to its end from node[q]
            leaf = nleaf + 1;
            atomicAdd(&ctl[CTL_AGED], 1);
        } else if (f.strag_max > 0 && v >= 0 && f.req_left[f.req_of[q]] <= f.strag_max) {
            // one of its request's last few travelling queries: leaves the rounds likewise, so
            // the request does not wait out its slowest walks one round at a time (the count
            // is read while other queries of the request may finish: at worst a query hands
            // over a round early or late)
            leaf = nleaf + 1;
            atomicAdd(&ctl[CTL_AGED], 1);
        }
        pend_leaf[pend_base + j] = leaf;
        pend_q[pend_base + j] = q;
        valid = leaf < nleaf;
    }
    // Buffer fills: lanes bound for the same leaf are counted with one atomic
    // (fetched queries arrive grouped by their previous leaf, so a wave holds
    // few distinct leaves).  Under the Algorithm 1 schedule each lane also
    // learns its fill for the half-full trigger, which needs the atomic's
    // return value; otherwise the atomics are fire-and-forget.
    uint64_t todo = __ballot(valid);
    if (!f.count_leaves) return;
    if (f.track_fill) {
        const uint64_t below = lanemask_lt();
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const uint32_t ll = (uint32_t)__builtin_amdgcn_readlane((int)leaf, leader);
            const uint64_t grp = __ballot(valid && leaf == ll);
            int32_t old = 0;
            if (__lane_id() == leader) old = atomicAdd(&cnt[ll], (int32_t)__popcll(grp));
            old = __builtin_amdgcn_readlane(old, leader);
            if ((grp >> __lane_id()) & 1ull) fill = old + (int32_t)__popcll(grp & below) + 1;
            todo &= ~grp;
        }
        int32_t mx = fill;
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
        if (__lane_id() == 0 && mx > 0) atomicMax(&ctl[CTL_MAXCNT], mx);
    } else {
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const uint32_t ll = (uint32_t)__builtin_amdgcn_readlane((int)leaf, leader);
            const uint64_t grp = __ballot(valid && leaf == ll);
            if (__lane_id() == leader) atomicAdd(&cnt[ll], (int32_t)__popcll(grp));
            todo &= ~grp;
        }
    }
}

// Per-leaf counts of a pending list sorted by leaf, without atomics: the run
// of leaf l occupies [start[l], end[l]); both arrays are zero for absent leaves.
// With dcount the element count is *dcount (count only bounds the grid).
__global__ void k_run_bounds(const uint32_t *__restrict__ leaf, int64_t count, const int32_t *__restrict__ dcount,
                             uint32_t nleaf, int32_t *__restrict__ start, int32_t *__restrict__ end)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (dcount) count = *dcount;
    if (i >= count) return;
    const uint32_t l = leaf[i];
    if (l >= nleaf) return;
    if (i == 0 || leaf[i - 1] != l) start[l] = (int32_t)i;
    if (i + 1 == count || leaf[i + 1] != l) end[l] = (int32_t)(i + 1);
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (leaf, query) pairs, 8-bit digits.

constexpr int SORT_THREADS = 256;
constexpr int SORT_ROUNDS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ROUNDS;

__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t count,
                                                             const int32_t *__restrict__ dcount, int shift,
                                                             uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t hcount[256];
    const int tid = threadIdx.x;
    if (dcount) count = *dcount;
    hcount[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ROUNDS; r++) {
        int64_t i = base + r * SORT_THREADS + tid;
        if (i < count) atomicAdd(&hcount[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nblocks + blockIdx.x] = hcount[tid];
}

// Exclusive scan of each digit's column of the histogram (hist is digit-major:
// hist[digit * nblocks + block]); totals[digit] receives the column sum.
__global__ __launch_bounds__(256) void k_scan_columns(uint32_t *__restrict__ hist, int nblocks,
                                                      uint32_t *__restrict__ totals)
{
    __shared__ uint32_t lds[256];
    uint32_t *col = hist + (int64_t)blockIdx.x * nblocks;
    const int tid = threadIdx.x;
    uint32_t carry = 0;
    for (int base = 0; base < nblocks; base += 256) {
        const int i = base + tid;
        const uint32_t v = i < nblocks ? col[i] : 0u;
        lds[tid] = v;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            uint32_t add = tid >= o ? lds[tid - o] : 0u;
            __syncthreads();
            lds[tid] += add;
            __syncthreads();
        }
        if (i < nblocks) col[i] = carry + lds[tid] - v;
        carry += lds[255];
        __syncthreads();
    }
    if (tid == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                                const int32_t *__restrict__ vin,
                                                                uint32_t *__restrict__ kout,
                                                                int32_t *__restrict__ vout, int64_t count,
                                                                const int32_t *__restrict__ dcount, int shift,
                                                                const uint32_t *__restrict__ hist, int nblocks,
                                                                const uint32_t *__restrict__ totals)
{
    if (dcount) count = *dcount;
    constexpr int W = SORT_THREADS / 64;
    __shared__ uint32_t run[256];      // next output position per digit for this block
    __shared__ uint32_t wcount[W][256];
    __shared__ uint32_t wstart[W][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    {
        // digit base = exclusive scan of the column totals
        const uint32_t tot = totals[tid];
        run[tid] = tot;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            uint32_t add = tid >= o ? run[tid - o] : 0u;
            __syncthreads();
            run[tid] += add;
            __syncthreads();
        }
        const uint32_t base = run[tid] - tot;
        __syncthreads();
        run[tid] = base + hist[(int64_t)tid * nblocks + blockIdx.x];
    }
    for (int w = 0; w < W; w++) wcount[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ROUNDS; r++) {
        const int64_t i = base + r * SORT_THREADS + tid;
        const bool valid = i < count;
        uint32_t key = valid ? kin[i] : 0u;
        int32_t val = valid ? vin[i] : 0;
        uint32_t digit = (key >> shift) & 255u;
        uint64_t mask = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            bool bit = (digit >> b) & 1u;
            uint64_t bal = __ballot(valid && bit);
            mask &= bit ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(mask & lanemask_lt());
        if (valid && rank == 0) wcount[wave][digit] = (uint32_t)__popcll(mask);
        __syncthreads();
        {
            uint32_t p = run[tid];
            for (int w = 0; w < W; w++) {
                uint32_t c = wcount[w][tid];
                wstart[w][tid] = p;
                wcount[w][tid] = 0;
                p += c;
            }
            run[tid] = p;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = wstart[wave][digit] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
    }
}

// ---------------------------------------------------------------------------
// Single-pass grouping by leaf for at most BK_MAX distinct keys.  The lock-step
// rounds need every buffer's queries together but not in any particular order,
// so each element claims its output position with an LDS atomic on its key's
// running counter.  Pass 1 writes each block's key counts (key-major), the
// column scan turns them into per-block prefixes and key totals (the per-leaf
// counts), the buffer offsets follow from the totals, and pass 2 scatters.

constexpr int BK_THREADS = 1024;
constexpr int BK_PER = 8;
constexpr int BK_TILE = BK_THREADS * BK_PER;
constexpr int BK_MAX = 2048;

__global__ __launch_bounds__(BK_THREADS) void k_bucket_hist(const uint32_t *__restrict__ keys, int64_t count, int nb,
                                                            uint32_t *__restrict__ hist, int nblocks,
                                                            uint32_t key_base, const int32_t *__restrict__ dcount)
{
    __shared__ uint32_t h[BK_MAX];
    if (dcount) count = *dcount;
    for (int i = threadIdx.x; i < nb; i += BK_THREADS) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BK_TILE + threadIdx.x;
    uint32_t kr[BK_PER];
#pragma unroll
    for (int r = 0; r < BK_PER; r++) {
        const int64_t i = base + (int64_t)r * BK_THREADS;
        kr[r] = i < count ? keys[i] - key_base : 0u;
    }
#pragma unroll
    for (int r = 0; r < BK_PER; r++)
        if (base + (int64_t)r * BK_THREADS < count && kr[r] < (uint32_t)nb) atomicAdd(&h[kr[r]], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += BK_THREADS) hist[(int64_t)i * nblocks + blockIdx.x] = h[i];
}

// hist: per-block exclusive prefixes within each key (after the column scan);
// off: start of each key's run in the output.
__global__ __launch_bounds__(BK_THREADS) void k_bucket_scatter(const uint32_t *__restrict__ kin,
                                                               const int32_t *__restrict__ vin,
                                                               uint32_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                               int64_t count, int nb,
                                                               const uint32_t *__restrict__ hist, int nblocks,
                                                               const int32_t *__restrict__ off, uint32_t key_base,
                                                               const int32_t *__restrict__ dcount)
{
    __shared__ uint32_t run[BK_MAX];
    if (dcount) count = *dcount;
    for (int i = threadIdx.x; i < nb; i += BK_THREADS)
        run[i] = (uint32_t)off[i] + hist[(int64_t)i * nblocks + blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * BK_TILE + threadIdx.x;
    uint32_t kr[BK_PER];
    int32_t vr[BK_PER];
#pragma unroll
    for (int r = 0; r < BK_PER; r++) {
        const int64_t i = base + (int64_t)r * BK_THREADS;
        kr[r] = i < count ? kin[i] : 0u;
        vr[r] = i < count ? vin[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < BK_PER; r++) {
        const uint32_t lk = kr[r] - key_base;
        if (base + (int64_t)r * BK_THREADS < count && lk < (uint32_t)nb) {
            const uint32_t pos = atomicAdd(&run[lk], 1u);
            kout[pos] = kr[r];
            vout[pos] = vr[r];
        }
    }
}

// ---------------------------------------------------------------------------

// Buffer offsets (exclusive scan of the fills), work items of one call and
// the pair / visit counters.  A leaf holding at least dense_min buffered
// queries is scanned in tiles of `qt` queries (one lane per query); a leaf
// holding fewer gets one wave per buffered query (lanes over points).
__global__ __launch_bounds__(1024) void k_leaf_offsets(const int32_t *__restrict__ cnt,
                                                       const int32_t *__restrict__ start,
                                                       const int32_t *__restrict__ leaf_off, int nleaf, int qt,
                                                       int dense_min, int32_t *__restrict__ off,
                                                       int32_t *__restrict__ tiles, int32_t *__restrict__ sparse,
                                                       int32_t *__restrict__ ctl, int count_work)
{
    // columns: buffered entries, dense items, sparse items (prefix sums); then the work of a
    // full scan: dense pairs, sparse pairs, points of the dense leaves, points of the sparse
    // leaves, dense visits (totals)
    constexpr int NC = 8;
    __shared__ long long wsum[16][NC], wpre[16][3], wtot[NC];
    const int tid = threadIdx.x;
    const int seg = (nleaf + 1023) / 1024;
    const int lo = min(nleaf, tid * seg), hi = min(nleaf, lo + seg);
    long long sc = 0, st = 0, ss = 0;
    long long red[5] = {0, 0, 0, 0, 0};
    // count of leaf l: cnt[l], or end - start of its run when start is given
    for (int l = lo; l < hi; l++) {
        int c = cnt[l] - (start ? start[l] : 0);
        const int len = leaf_off[l + 1] - leaf_off[l];
        const long long pr = (long long)c * len;
        sc += c;
        if (c >= dense_min) {
            st += (c + qt - 1) / qt;
            red[0] += pr;
            red[2] += len;
            red[4] += c;
        } else {
            ss += c;
            red[1] += pr;
            if (c > 0) red[3] += len;
        }
    }
    // one pass: inclusive sums of the three running counts within each wave
    // (shuffles), the wave totals through LDS, and sixteen threads turn those
    // into per-wave prefixes and the block totals
    const int lane = tid & 63, wave = tid >> 6;
    int32_t inc[3] = {(int32_t)sc, (int32_t)st, (int32_t)ss};
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const int32_t u = __shfl_up(inc[i], o);
            if (lane >= o) inc[i] += u;
        }
    }
    if (count_work) {
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int i = 0; i < 5; i++) red[i] += __shfl_xor(red[i], o);
        }
    }
    if (lane == 63) {
        wsum[wave][0] = inc[0];
        wsum[wave][1] = inc[1];
        wsum[wave][2] = inc[2];
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < 5; i++) wsum[wave][3 + i] = red[i];
    }
    __syncthreads();
    if (tid < NC) {
        // column tid: exclusive prefix over the waves (counts) or the total (work)
        long long run = 0;
        for (int w = 0; w < 16; w++) {
            const long long v = wsum[w][tid];
            if (tid < 3) wpre[w][tid] = run;
            run += v;
        }
        wtot[tid] = run;
    }
    __syncthreads();
    long long rc = wpre[wave][0] + inc[0] - sc, rt = wpre[wave][1] + inc[1] - st, rs = wpre[wave][2] + inc[2] - ss;
    const long long tc = wtot[0], tt = wtot[1], ts = wtot[2];
    if (count_work && tid == 0) {
        // visits, pairs and leaf points of a full scan of these buffers (as k_count_work does)
        auto add = [&](int w, long long v) {
            if (v) atomicAdd((unsigned long long *)(ctl + w), (unsigned long long)v);
        };
        add(CTL_VISITS_LO, tc);
        add(CTL_DPAIRS_LO, wtot[3]);
        add(CTL_SPAIRS_LO, wtot[4]);
        add(CTL_LPD_LO, wtot[5]);
        add(CTL_LPS_LO, wtot[6]);
        add(CTL_DVISITS_LO, wtot[7]);
    }
    for (int l = lo; l < hi; l++) {
        int c = cnt[l] - (start ? start[l] : 0);
        off[l] = (int32_t)rc;
        tiles[l] = (int32_t)rt;
        sparse[l] = (int32_t)rs;
        rc += c;
        if (c >= dense_min) rt += (c + qt - 1) / qt;
        else rs += c;
    }
    if (tid == 0) {
        off[nleaf] = (int32_t)tc;
        tiles[nleaf] = (int32_t)tt;
        sparse[nleaf] = (int32_t)ts;
        ctl[CTL_V] = (int32_t)tc;
        ctl[CTL_T] = (int32_t)tt;
        ctl[CTL_S] = (int32_t)ts;
    }
}

// Visits and (query, point) pairs of the leaves [lf, ll] about to be scanned, split by scan kernel.
__global__ __launch_bounds__(256) void k_count_work(const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ leaf_off, int lf, int ll,
                                                    int dense_min, int32_t *__restrict__ ctl)
{
    long long w[6] = {0, 0, 0, 0, 0, 0};  // visits, dense pairs, sparse pairs, dense / sparse leaf points, dense visits
    for (int l = lf + threadIdx.x; l <= ll; l += blockDim.x) {
        const int c = off[l + 1] - off[l];
        const int len = leaf_off[l + 1] - leaf_off[l];
        const long long pr = (long long)c * len;
        w[0] += c;
        if (c >= dense_min) {
            w[1] += pr;
            w[3] += len;
            w[5] += c;
        } else {
            w[2] += pr;
            if (c > 0) w[4] += len;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int i = 0; i < 6; i++) w[i] += __shfl_xor(w[i], o);
    }
    if (__lane_id() == 0) {
        const int word[6] = {CTL_VISITS_LO, CTL_DPAIRS_LO, CTL_SPAIRS_LO, CTL_LPD_LO, CTL_LPS_LO, CTL_DVISITS_LO};
#pragma unroll
        for (int i = 0; i < 6; i++)
            if (w[i]) atomicAdd((unsigned long long *)(ctl + word[i]), (unsigned long long)w[i]);
    }
}

// Chunk sweep: route entries of the drained chunk c to the pending regions of
// their next chunk; entries staying in c go to a side buffer, finished ones are dropped.
// The order inside a region is free (a region is grouped by leaf before its scan),
// so a block first counts its entries per target in LDS and then reserves each
// target's range with one device-scope atomic: a few atomics per 1024 entries
// instead of one per entry on a handful of words.
__global__ __launch_bounds__(1024) void k_distribute(const uint32_t *__restrict__ leaf, const int32_t *__restrict__ q,
                                                     int64_t n, const int32_t *__restrict__ dn, uint32_t nleaf,
                                                     const int32_t *__restrict__ chunk_of,
                                                     int c, uint32_t *__restrict__ rleaf, int32_t *__restrict__ rq,
                                                     int64_t rcap, int32_t *__restrict__ rcnt,
                                                     uint32_t *__restrict__ sleaf, int32_t *__restrict__ sq, int nchunks)
{
    __shared__ int32_t cnt[DISTRIBUTE_MAX_TARGETS], base[DISTRIBUTE_MAX_TARGETS];
    if (dn) n = *dn;
    for (int j = threadIdx.x; j <= nchunks; j += blockDim.x) cnt[j] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t l = i < n ? leaf[i] : nleaf;
    int t = -1, pos = 0;
    if (l < nleaf) {
        const int tc = chunk_of[l];
        t = tc == c ? nchunks : tc;
        pos = atomicAdd(&cnt[t], 1);
    }
    __syncthreads();
    for (int j = threadIdx.x; j <= nchunks; j += blockDim.x)
        if (cnt[j]) base[j] = atomicAdd(&rcnt[j], cnt[j]);
    __syncthreads();
    if (t < 0) return;
    pos += base[t];
    if (t == nchunks) {
        sleaf[pos] = l;
        sq[pos] = q[i];
    } else {
        rleaf[(int64_t)t * rcap + pos] = l;
        rq[(int64_t)t * rcap + pos] = q[i];
    }
}

__global__ void k_restore(const uint32_t *__restrict__ sleaf, const int32_t *__restrict__ sq, int64_t n,
                          uint32_t *__restrict__ rleaf, int32_t *__restrict__ rq, int32_t *__restrict__ rcnt, int c,
                          int nchunks)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t stay = rcnt[nchunks];
    if (i < stay) {
        rleaf[i] = sleaf[i];
        rq[i] = sq[i];
    }
    if (i == 0) rcnt[c] = stay;
}

__global__ void k_ring_append(int32_t *ring, int64_t cap, int64_t tail, const int32_t *src, int64_t count)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) ring[(tail + i) % cap] = src[i];
}

__global__ void k_finalize(const uint64_t *__restrict__ keys, int K, int k, int64_t m, const int32_t *__restrict__ perm,
                           int64_t *__restrict__ idx, float *__restrict__ dist, int squared)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * k) return;
    int64_t q = i / k;
    int s = (int)(i - q * k);
    uint64_t key = keys[q * K + s];
    const int64_t o = (perm ? (int64_t)perm[q] : q) * k + s;  // row of the caller's query
    idx[o] = (int64_t)(uint32_t)key;
    float d2 = __uint_as_float((uint32_t)(key >> 32));
    dist[o] = squared ? d2 : sqrtf(d2);
}

// Renumber the queries in the order of a pending list sorted by leaf: slot i
// takes query q = ids[i] (perm[i] = q, coordinates copied, node = its leaf) and
// ids[i] becomes i.  Queries sharing a buffer then have neighbouring numbers,
// so per-query state is read and written in contiguous runs.
__global__ void k_localize(int32_t *__restrict__ ids, const uint32_t *__restrict__ leaf, int64_t m,
                           int32_t *__restrict__ perm, int32_t *__restrict__ node, int32_t first, uint32_t nleaf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    perm[i] = ids[i];
    node[i] = leaf[i] < nleaf ? first + (int32_t)leaf[i] : NODE_DONE;
    ids[i] = (int32_t)i;
}

// Coordinates in the new numbering, one word per thread: consecutive lanes
// read consecutive words of a row and write consecutive words of the copy.
__global__ void k_gather_rows(const float *__restrict__ Q, const int32_t *__restrict__ perm, int64_t m, int d,
                              float *__restrict__ Qp)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * d) return;
    const int64_t i = e / d;
    Qp[e] = Q[(int64_t)perm[i] * d + (e - i * d)];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

static void check_launch()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BKD_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
}

void launch_init_state(int32_t *node, uint64_t *keys, uint32_t *kth, int64_t m, int K, hipStream_t s)
{
    if (m <= 0) return;
    k_init_state<<<grid_for(m, 256), 256, 0, s>>>(node, keys, kth, m, K);
    check_launch();
}

void launch_check_finite(const float *Q, int64_t count, int32_t *ctl, hipStream_t s)
{
    if (count <= 0) return;
    unsigned g = (unsigned)std::min<int64_t>(grid_for(count, 256), 4096);
    k_check_finite<<<g, 256, 0, s>>>(Q, count, ctl);
    check_launch();
}

void launch_fill_i32(int32_t *p, int32_t v, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    k_fill_i32<<<grid_for(count, 256), 256, 0, s>>>(p, v, count);
    check_launch();
}

void launch_find_leaf(const FetchSpec &f, const float *Q, int d, int32_t *node, const uint32_t *kth,
                      const float *split, int h, uint32_t *pend_leaf, int32_t *pend_q, int64_t pend_base,
                      int32_t *cnt, int32_t *ctl, hipStream_t s)
{
    int64_t total = f.ring_count + f.in_count;
    if (total <= 0) return;
    k_find_leaf<<<grid_for(total, 256), 256, 0, s>>>(f, Q, d, node, kth, split, h, pend_leaf, pend_q,
                                                     pend_base, cnt, ctl);
    check_launch();
}

size_t sort_hist_words(int64_t count)
{
    int64_t nblocks = (count + SORT_TILE - 1) / SORT_TILE;
    const size_t radix = (size_t)(std::max<int64_t>(nblocks, 1) + 1) * 256;  // histogram + column totals
    int64_t bblocks = (count + BK_TILE - 1) / BK_TILE;
    const size_t bucket = (size_t)(std::max<int64_t>(bblocks, 1) + 1) * BK_MAX;
    return std::max(radix, bucket);
}

int bucket_max_keys() { return BK_MAX; }

const int32_t *launch_bucket_count(const uint32_t *keys, int64_t count, int nb, uint32_t *hist,
                                   hipStream_t s, uint32_t key_base, const int32_t *dcount)
{
    const int nblocks = (int)((count + BK_TILE - 1) / BK_TILE);
    uint32_t *totals = hist + (size_t)nb * nblocks;
    if (nblocks > 0) k_bucket_hist<<<nblocks, BK_THREADS, 0, s>>>(keys, count, nb, hist, nblocks, key_base, dcount);
    k_scan_columns<<<nb, 256, 0, s>>>(hist, nblocks, totals);
    check_launch();
    return reinterpret_cast<const int32_t *>(totals);
}

void launch_bucket_scatter(const uint32_t *kin, const int32_t *vin, uint32_t *kout, int32_t *vout, int64_t count,
                           int nb, const uint32_t *hist, const int32_t *off, hipStream_t s, uint32_t key_base,
                           const int32_t *dcount)
{
    const int nblocks = (int)((count + BK_TILE - 1) / BK_TILE);
    if (nblocks == 0) return;
    k_bucket_scatter<<<nblocks, BK_THREADS, 0, s>>>(kin, vin, kout, vout, count, nb, hist, nblocks, off, key_base,
                                                    dcount);
    check_launch();
}

int launch_sort_pairs(uint32_t *key_a, int32_t *val_a, uint32_t *key_b, int32_t *val_b, int64_t count, int key_bits,
                      uint32_t *hist, hipStream_t s, const int32_t *dcount)
{
    if (count <= (dcount ? 0 : 1)) return 0;
    int nblocks = (int)((count + SORT_TILE - 1) / SORT_TILE);
    int passes = (key_bits + 7) / 8;
    uint32_t *kin = key_a, *kout = key_b;
    int32_t *vin = val_a, *vout = val_b;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        uint32_t *totals = hist + (size_t)nblocks * 256;
        k_radix_hist<<<nblocks, SORT_THREADS, 0, s>>>(kin, count, dcount, shift, hist, nblocks);
        k_scan_columns<<<256, 256, 0, s>>>(hist, nblocks, totals);
        k_radix_scatter<<<nblocks, SORT_THREADS, 0, s>>>(kin, vin, kout, vout, count, dcount, shift, hist, nblocks,
                                                         totals);
        check_launch();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return (passes & 1) ? 1 : 0;
}

void launch_leaf_offsets(const int32_t *cnt, const int32_t *start, const int32_t *leaf_off, int nleaf, int qt,
                         int dense_min, int32_t *off, int32_t *tiles, int32_t *sparse, int32_t *ctl, hipStream_t s,
                         bool count_work)
{
    k_leaf_offsets<<<1, 1024, 0, s>>>(cnt, start, leaf_off, nleaf, qt, dense_min, off, tiles, sparse, ctl,
                                      count_work ? 1 : 0);
    check_launch();
}

void launch_run_bounds(const uint32_t *leaf, int64_t count, int nleaf, int32_t *start, int32_t *end, hipStream_t s,
                       const int32_t *dcount)
{
    if (count <= 0) return;
    k_run_bounds<<<grid_for(count, 256), 256, 0, s>>>(leaf, count, dcount, (uint32_t)nleaf, start, end);
    check_launch();
}

void launch_count_work(const int32_t *off, const int32_t *leaf_off, int lf, int ll, int dense_min, int32_t *ctl,
                       hipStream_t s)
{
    k_count_work<<<1, 256, 0, s>>>(off, leaf_off, lf, ll, dense_min, ctl);
    check_launch();
}

void launch_distribute(const uint32_t *leaf, const int32_t *q, int64_t n, int nleaf, const int32_t *chunk_of, int c,
                       uint32_t *rleaf, int32_t *rq, int64_t rcap, int32_t *rcnt, uint32_t *sleaf, int32_t *sq,
                       int nchunks, hipStream_t s, const int32_t *dn)
{
    if (n <= 0) return;
    if (nchunks + 1 > DISTRIBUTE_MAX_TARGETS) fail(BKD_EINVAL, "chunk sweep: too many chunks");
    k_distribute<<<grid_for(n, 1024), 1024, 0, s>>>(leaf, q, n, dn, (uint32_t)nleaf, chunk_of, c, rleaf, rq, rcap, rcnt,
                                                    sleaf, sq, nchunks);
    check_launch();
}

void launch_restore(const uint32_t *sleaf, const int32_t *sq, int64_t n, uint32_t *rleaf, int32_t *rq, int32_t *rcnt,
                    int c, int nchunks, hipStream_t s)
{
    k_restore<<<grid_for(std::max<int64_t>(n, 1), 256), 256, 0, s>>>(sleaf, sq, n, rleaf, rq, rcnt, c, nchunks);
    check_launch();
}

void launch_ring_append(int32_t *ring, int64_t cap, int64_t tail, const int32_t *src, int64_t count, hipStream_t s)
{
    if (count <= 0) return;
    k_ring_append<<<grid_for(count, 256), 256, 0, s>>>(ring, cap, tail, src, count);
    check_launch();
}

void launch_finalize(const uint64_t *keys, int K, int k, int64_t m, const int32_t *perm, int64_t *idx, float *dist,
                     bool squared, hipStream_t s)
{
    if (m <= 0) return;
    k_finalize<<<grid_for(m * k, 256), 256, 0, s>>>(keys, K, k, m, perm, idx, dist, squared ? 1 : 0);
    check_launch();
}

void launch_localize(int32_t *ids, const uint32_t *leaf, int64_t m, int d, const float *Q, float *Qp, int32_t *perm,
                     int32_t *node, int h, hipStream_t s)
{
    if (m <= 0) return;
    k_localize<<<grid_for(m, 256), 256, 0, s>>>(ids, leaf, m, perm, node, (1 << h) - 1, 1u << h);
    k_gather_rows<<<grid_for(m * d, 256), 256, 0, s>>>(Q, perm, m, d, Qp);
    check_launch();
}

}  // namespace bkd
