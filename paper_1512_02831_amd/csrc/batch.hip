// batch.hip -- batched form: many independent instances in one persistent launch.
//
// Every instance runs the buffered search of Algorithm 1 in lock-step rounds
// (Section 2.4).  One persistent kernel serves all instances from a device
// task queue; a round of instance i is three phases of tasks:
//   FIND(i, j0, j1)  FindLeafBatch for a slice of i's active queries, with the
//                    buffer fills counted by per-leaf atomics;
//   ORGANIZE(i)      one workgroup: buffer offsets, the list of buffered
//                    leaves and the scatter of the queries into buffer order,
//                    then the list of pieces; an instance whose queries have
//                    all finished is done;
//   SCAN(i, e0, e1)  one wave per piece (at most SCAN_PIECE buffered queries
//                    of one leaf): the leaf's points sit in registers (lanes
//                    over points) while the wave walks the piece's queries;
//                    each query's k best keys are spread over the lanes and
//                    merged with ballots.
//   TAIL(i, j0, j1)  once an instance has at most solo_max active queries
//                    (or from the start, when it is that small): one wave per
//                    query walks that query's traversal to the end, lanes over
//                    each leaf's points, so the end of an instance is the
//                    longest single traversal rather than a chain of rounds.
// The last task of a phase enqueues the next phase of the same instance.
// Instances therefore advance independently; nothing waits for a global
// round.  Tasks are published with release stores of a per-slot sequence word
// and taken with acquire loads; every wait has a wall-clock guard that stops
// the whole launch with an error flag instead of spinning forever.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <map>
#include <tuple>
#include <memory>
#include <numeric>

#include "internal.h"
#include "traverse.h"

struct bkd_batch;

namespace bkd {

namespace {

constexpr int BT = 256;
constexpr int QCAP_LOG = 20;
constexpr unsigned long long QCAP = 1ull << QCAP_LOG;
constexpr int BATCH_MAX_LEAVES = 4096;  // height <= 12
constexpr int TASK_FIND = 1;
constexpr int TASK_ORGANIZE = 2;
constexpr int TASK_SCAN = 3;
constexpr int TASK_TAIL = 5;
constexpr int FIND_CHUNK = 2048;  // active queries per FIND task
// queries per TAIL task (32 per wave, one after another): fewer, longer tasks amortise the
// task claim and the split staging; 16, 64, 128 and 256 measured 616, 577, 569 and 569 ms
// on the 1024-instance batch
constexpr int TAIL_CHUNK = 128;
// A round's leaf scans are dealt out in pieces of at most this many buffered queries of one
// leaf (an instance with fewer than 2^26 queries; a piece is coded as the unsigned word
// leaf << 20 | index, leaf < 4096):
// a leaf holding thousands of queries then spreads over many waves instead of one wave
// walking them all.  Pieces of 16, 32, 64 and 128 measured 556, 538, 569 and 599 ms on the
// 1024-instance batch.
constexpr int SCAN_PIECE = 32;
constexpr int PIECE_M_MAX = 1 << 26;

struct BInst {
    int32_t d, k, h, nleaf, m, n;
    int64_t split_off, leaf_off_off, blk_off, pts_off, q_off, key_off, node_off, buf_off, tmp_off, loff_off, ne_off,
        cnt_off;
};

struct BState {
    int32_t round, V, E, pending;
};

struct BQueue {
    unsigned long long head, tail;
    int32_t done, error, active, pad;
    unsigned long long tasks, pairs, flops, rounds;
    unsigned long long wait_ticks;  // wall-clock ticks spent waiting for a task, summed over workgroups
};

struct BatchArgs {
    const BInst *inst;
    BState *state;
    BQueue *q;
    int4 *tasks;
    unsigned long long *seq;
    const float *split;
    const int32_t *leaf_off;
    const int32_t *blk;
    const float *pts;
    const float *Q;
    uint64_t *keys;
    int32_t *node;
    int32_t *buf;
    int32_t *tmp;
    int32_t *loff;
    int32_t *ne;
    int32_t *cnt;
    int32_t leaves_per_task;
    int32_t solo_max;  // instances with at most this many active queries finish per query (TAIL)
    int32_t count;
    unsigned long long spin_ticks;
};

__device__ inline unsigned long long ld_acq(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_rel(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int ld_flag(int32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// Polling load: coherent at agent scope but without the cache invalidation of
// an acquire (an acquire fence follows once the awaited value is seen), so
// idle workgroups do not flush the L1 of busy ones on the same CU.
__device__ inline unsigned long long ld_poll(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t rdlane64(uint64_t v, int lane)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Publish `count` tasks made by make(j); every thread of the workgroup calls it.
template <class F> __device__ __forceinline__ void push_tasks(const BatchArgs &a, int count, F make, unsigned long long *lds_base)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) *lds_base = atomicAdd(&a.q->tail, (unsigned long long)count);
    __syncthreads();
    const unsigned long long base = *lds_base;
    for (int j = threadIdx.x; j < count; j += BT) {
        const unsigned long long idx = base + j;
        const unsigned long long slot = idx & (QCAP - 1);
        const unsigned long long fr = 2 * (idx >> QCAP_LOG);
        const unsigned long long t0 = wall_clock64();
        bool ok = true;
        while (ld_poll(&a.seq[slot]) != fr) {  // slot still holds an older task (capacity exceeded)
            if (wall_clock64() - t0 > a.spin_ticks || ld_flag(&a.q->error)) {
                atomicOr(&a.q->error, 1);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        if (!ok) continue;
        a.tasks[slot] = make(j);
        st_rel(&a.seq[slot], fr + 1);
    }
    __syncthreads();
}

// Exclusive scan of lds[0..n) in place by one workgroup (segments of contiguous entries).
__device__ __forceinline__ int32_t block_scan_lds(int32_t *lds, int n, int32_t *part)
{
    const int tid = threadIdx.x;
    const int seg = (n + BT - 1) / BT;
    const int lo = min(n, tid * seg), hi = min(n, lo + seg);
    int32_t s = 0;
    for (int i = lo; i < hi; i++) s += lds[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < BT; o <<= 1) {
        int32_t add = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int32_t run = part[tid] - s;
    const int32_t total = part[BT - 1];
    for (int i = lo; i < hi; i++) {
        int32_t x = lds[i];
        lds[i] = run;
        run += x;
    }
    __syncthreads();
    return total;
}

struct RouteLds {
    int32_t hist[BATCH_MAX_LEAVES];
    int32_t cur[BATCH_MAX_LEAVES];
    int32_t part[BT];
    unsigned long long red[BT / 64];
    unsigned long long base;
    int32_t E;
};

// The instance's split values (at most 4095) in LDS for the walks of one task.
__device__ __forceinline__ const float *stage_split(const BatchArgs &a, const BInst &I, RouteLds &L)
{
    float *sl = reinterpret_cast<float *>(L.hist);
    const float *split = a.split + I.split_off;
    __syncthreads();  // the previous task may still read L
    for (int v = threadIdx.x; v < I.nleaf - 1; v += BT) sl[v] = split[v];
    __syncthreads();
    return sl;
}

// FindLeafBatch over active entries [j0, j1) of instance i's current round.
__device__ __forceinline__ void find_task(const BatchArgs &a, int i, int j0, int j1, RouteLds &L)
{
    const BInst I = a.inst[i];
    const int round = a.state[i].round;
    const int32_t *inb = a.buf + I.buf_off + (int64_t)(round & 1) * I.m;
    const float *split = a.split + I.split_off;
    int32_t *tmp = a.tmp + I.tmp_off;
    int32_t *node = a.node + I.node_off;
    int32_t *cnt = a.cnt + I.cnt_off;
    const uint64_t *keys = a.keys + I.key_off;
    const float *Q = a.Q + I.q_off;
    const int first = I.nleaf - 1;
    const float *sl = stage_split(a, I, L);
    for (int jb = j0; jb < j1; jb += BT) {
        const int j = jb + (int)threadIdx.x;
        int32_t lf = -1;
        if (j < j1) {
            const int32_t q = round == 0 ? j : inb[j];
            const int32_t v = next_leaf(node[q], Q + (int64_t)q * I.d, keys + (int64_t)q * I.k + (I.k - 1), split, sl,
                                        I.nleaf - 1, I.h, I.d);
            node[q] = v;
            lf = v >= 0 ? v - first : -1;
            tmp[j] = lf;
        }
        // one atomic per (wave, leaf): queries arrive grouped by their previous leaf
        uint64_t todo = __ballot(lf >= 0);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int32_t ll = __builtin_amdgcn_readlane(lf, leader);
            const uint64_t grp = __ballot(lf == ll);
            if ((int)__lane_id() == leader) atomicAdd(&cnt[ll], (int32_t)__popcll(grp));
            todo &= ~grp;
        }
    }
}

// Buffer offsets, buffered-leaf list and scatter of instance i's round, from
// the buffer fills in the global counters.  Returns the number of buffered
// queries V; an instance with V = 0 is finished.  On V > 0 the instance state
// moves to the next round.
__device__ __forceinline__ int organize_core(const BatchArgs &a, int i, RouteLds &L)
{
    const BInst I = a.inst[i];
    BState *st = a.state + i;
    const int tid = threadIdx.x;
    const int round = st->round;
    const int nleaf = I.nleaf;
    const int A = round == 0 ? I.m : st->V;
    const int32_t *inb = a.buf + I.buf_off + (int64_t)(round & 1) * I.m;
    int32_t *outb = a.buf + I.buf_off + (int64_t)((round + 1) & 1) * I.m;
    const int32_t *loffs = a.leaf_off + I.leaf_off_off;
    const int32_t *tmp = a.tmp + I.tmp_off;
    int32_t *cnt = a.cnt + I.cnt_off;
    int32_t *loff = a.loff + I.loff_off;
    int32_t *ne = a.ne + I.ne_off;

    unsigned long long pr = 0;
    constexpr int CU = 4;  // leaves per thread whose loads go out together
    for (int l0 = tid; l0 < nleaf; l0 += BT * CU) {
        int32_t c[CU], len[CU];
#pragma unroll
        for (int u = 0; u < CU; u++) {
            const int l = l0 + u * BT;
            c[u] = l < nleaf ? cnt[l] : 0;
            len[u] = l < nleaf ? loffs[l + 1] - loffs[l] : 0;
        }
#pragma unroll
        for (int u = 0; u < CU; u++) {
            const int l = l0 + u * BT;
            if (l < nleaf) {
                cnt[l] = 0;
                L.cur[l] = c[u];
                pr += (unsigned long long)c[u] * (unsigned)len[u];
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) pr += __shfl_xor(pr, o);
    if ((tid & 63) == 0) L.red[tid >> 6] = pr;
    __syncthreads();
    const int32_t V = block_scan_lds(L.cur, nleaf, L.part);
    for (int l = tid; l < nleaf; l += BT) loff[l] = L.cur[l];
    if (tid == 0) loff[nleaf] = V;
    // buffered leaves: positions by a scan of the "fill > 0" flags (each flag is re-derived
    // from the offsets, which stay in L.cur)
    for (int l = tid; l < nleaf; l += BT) L.hist[l] = ((l + 1 < nleaf ? L.cur[l + 1] : V) > L.cur[l]) ? 1 : 0;
    __syncthreads();
    const int32_t E = block_scan_lds(L.hist, nleaf, L.part);
    for (int l = tid; l < nleaf; l += BT)
        if ((l + 1 < nleaf ? L.cur[l + 1] : V) > L.cur[l]) ne[L.hist[l]] = l;
    __syncthreads();
    // eight entries per thread at a time: their loads are all issued before the first store
    // (which the compiler may not move a later load above), so the scatter waits for memory
    // once per eight entries instead of once per entry
    constexpr int SU = 8;
    for (int j0 = tid; j0 < A; j0 += BT * SU) {
        int32_t lf[SU], id[SU];
#pragma unroll
        for (int u = 0; u < SU; u++) {
            const int j = j0 + u * BT;
            lf[u] = j < A ? tmp[j] : -1;
            id[u] = (j < A && round != 0) ? inb[j] : j;
        }
#pragma unroll
        for (int u = 0; u < SU; u++)
            if (lf[u] >= 0) outb[atomicAdd(&L.cur[lf[u]], 1)] = id[u];
    }
    if (tid == 0) {
        unsigned long long p = 0;
        for (int w = 0; w < BT / 64; w++) p += L.red[w];
        if (p) {
            atomicAdd(&a.q->pairs, p);
            atomicAdd(&a.q->flops, p * 3ull * (unsigned)I.d);
        }
        L.E = E;
    }
    __threadfence();
    __syncthreads();
    if (V == 0) {
        if (tid == 0 && atomicSub(&a.q->active, 1) == 1)
            __hip_atomic_store(&a.q->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    if (tid == 0) {
        st->V = V;
        st->E = E;
        st->round = round + 1;
        atomicAdd(&a.q->rounds, 1ull);
    }
    __threadfence();
    __syncthreads();
    return V;
}

__device__ __forceinline__ void organize_task(const BatchArgs &a, int i, RouteLds &L)
{
    if (organize_core(a, i, L) == 0) return;
    const BInst I = a.inst[i];
    int E = L.E;
    if (I.m < PIECE_M_MAX) {
        // L.cur holds each leaf's end offset after the scatter (the next leaf's start)
        const int nleaf = I.nleaf;
        for (int l = threadIdx.x; l < nleaf; l += BT) {
            const int32_t c = L.cur[l] - (l ? L.cur[l - 1] : 0);
            L.hist[l] = (c + SCAN_PIECE - 1) / SCAN_PIECE;
        }
        __syncthreads();
        E = block_scan_lds(L.hist, nleaf, L.part);  // pieces in all; L.hist: each leaf's first
        int32_t *pieces = a.tmp + I.tmp_off;         // free until the next FindLeafBatch phase
        for (int l = threadIdx.x; l < nleaf; l += BT) {
            const int32_t c = L.cur[l] - (l ? L.cur[l - 1] : 0);
            const int np = (c + SCAN_PIECE - 1) / SCAN_PIECE;
            for (int x = 0; x < np; x++) pieces[L.hist[l] + x] = (int32_t)(((uint32_t)l << 20) | (uint32_t)x);
        }
    }
    const int lpt = a.leaves_per_task;
    const int T = (E + lpt - 1) / lpt;
    if (threadIdx.x == 0) a.state[i].pending = T;
    push_tasks(a, T, [&](int j) { return make_int4(TASK_SCAN, i, j * lpt, min(E, (j + 1) * lpt)); }, &L.base);
}


// One wave per piece (up to SCAN_PIECE buffered queries of one leaf; per buffered leaf for an
// instance of 2^26 queries or more); G groups of 64 points per pass held in registers.
template <int D, int G> __device__ __forceinline__ void scan_leaves(const BatchArgs &a, int i, int e0, int e1)
{
    const BInst I = a.inst[i];
    const int round = a.state[i].round;
    const int32_t *buf = a.buf + I.buf_off + (int64_t)(round & 1) * I.m;
    const int32_t *loff = a.loff + I.loff_off;
    const int32_t *ne = a.ne + I.ne_off;
    const int32_t *lo_pos = a.leaf_off + I.leaf_off_off;
    const int32_t *blk = a.blk + I.blk_off;
    const float *pts = a.pts + I.pts_off;
    const float *Q = a.Q + I.q_off;
    uint64_t *keys = a.keys + I.key_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = I.d, k = I.k;
    const bool by_piece = I.m < PIECE_M_MAX;
    const int32_t *pieces = a.tmp + I.tmp_off;
    for (int e = e0 + wave; e < e1; e += BT / 64) {
        int Lf, qs, qe;
        if (by_piece) {
            const uint32_t pc = (uint32_t)__builtin_amdgcn_readfirstlane(pieces[e]);
            Lf = (int)(pc >> 20);
            qs = loff[Lf] + (int)(pc & 0xfffffu) * SCAN_PIECE;
            qe = min(loff[Lf + 1], qs + SCAN_PIECE);
        } else {
            Lf = __builtin_amdgcn_readfirstlane(ne[e]);
            qs = loff[Lf];
            qe = loff[Lf + 1];
        }
        const int len = lo_pos[Lf + 1] - lo_pos[Lf];
        const float *X = pts + blk[Lf];
        const int32_t *orig = reinterpret_cast<const int32_t *>(X) + (int64_t)d * len;
        for (int gb = 0; gb < len; gb += 64 * G) {
            float x[G][D];
            uint32_t o[G];
            bool v[G];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int p = gb + 64 * g + lane;
                v[g] = p < len;
#pragma unroll
                for (int j = 0; j < D; j++) x[g][j] = (v[g] && j < d) ? X[(int64_t)j * len + p] : 0.0f;
                o[g] = v[g] ? (uint32_t)orig[p] : 0u;
            }
            // The leaf's buffered queries, 64 ids at a time in the lanes.  Each query's
            // coordinates (lane j: coordinate j) and key list are loaded four queries
            // ahead, so the loads of later queries overlap the merges of earlier ones.
            for (int jb = qs; jb < qe; jb += 64) {
                const int nq = min(64, qe - jb);
                const int32_t qid = lane < nq ? buf[jb + lane] : 0;
                auto fetch = [&](int t, float &qr, uint64_t &lr) {
                    if (t < nq) {
                        const int32_t qq = __builtin_amdgcn_readlane(qid, t);
                        qr = lane < d ? Q[(int64_t)qq * d + lane] : 0.0f;
                        lr = lane < k ? keys[(int64_t)qq * k + lane] : ~0ull;
                    }
                };
                auto merge = [&](int t, float ql, uint64_t li) {
                    const int32_t q = __builtin_amdgcn_readlane(qid, t);
                    float qv[D];
#pragma unroll
                    for (int j = 0; j < D; j++)
                        qv[j] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ql), j));
                    float acc[G];
#pragma unroll
                    for (int g = 0; g < G; g++) acc[g] = 0.0f;
#pragma unroll
                    for (int j = 0; j < D; j++) {
#pragma unroll
                        for (int g = 0; g < G; g++) {
                            const float tt = qv[j] - x[g][j];
                            acc[g] = fmaf(tt, tt, acc[g]);
                        }
                    }
                    uint64_t kth = rdlane64(li, k - 1);
                    bool dirty = false;
#pragma unroll
                    for (int g = 0; g < G; g++) {
                        const uint64_t key = v[g] ? (((uint64_t)__float_as_uint(acc[g]) << 32) | o[g]) : ~0ull;
                        uint64_t cand = __ballot(key < kth);
                        while (cand) {
                            const int c = __ffsll((unsigned long long)cand) - 1;
                            cand &= cand - 1;
                            const uint64_t ck = rdlane64(key, c);
                            if (ck < kth) {
                                const uint64_t moved = __ballot(li > ck);
                                const int pos = __ffsll((unsigned long long)moved) - 1;
                                const uint64_t up = __shfl_up(li, 1);
                                li = (lane < pos) ? li : (lane == pos ? ck : up);
                                if (lane >= k) li = ~0ull;
                                kth = rdlane64(li, k - 1);
                                dirty = true;
                            }
                        }
                    }
                    if (dirty && lane < k) keys[(int64_t)q * k + lane] = li;
                };
                float q0 = 0.0f, q1 = 0.0f, q2 = 0.0f, q3 = 0.0f;
                uint64_t l0 = ~0ull, l1 = ~0ull, l2 = ~0ull, l3 = ~0ull;
                fetch(0, q0, l0);
                fetch(1, q1, l1);
                fetch(2, q2, l2);
                fetch(3, q3, l3);
                for (int t = 0; t < nq; t += 4) {
                    merge(t, q0, l0);
                    fetch(t + 4, q0, l0);
                    if (t + 1 < nq) {
                        merge(t + 1, q1, l1);
                        fetch(t + 5, q1, l1);
                    }
                    if (t + 2 < nq) {
                        merge(t + 2, q2, l2);
                        fetch(t + 6, q2, l2);
                    }
                    if (t + 3 < nq) {
                        merge(t + 3, q3, l3);
                        fetch(t + 7, q3, l3);
                    }
                }
            }
        }
    }
}

// Queries [j0, j1) of instance i's active list (identity in round 0) finish their
// traversals, one wave per query; the last TAIL task of the instance retires it.
template <int D, int G>
__device__ __forceinline__ void tail_queries(const BatchArgs &a, int i, int j0, int j1, RouteLds &L)
{
    const BInst I = a.inst[i];
    const float *sl = stage_split(a, I, L);
    float *qs = reinterpret_cast<float *>(L.cur) + 32 * (threadIdx.x >> 6);  // this wave's query, for the walk
    const int round = a.state[i].round;
    const int32_t *list = a.buf + I.buf_off + (int64_t)(round & 1) * I.m;
    const int32_t *lo_pos = a.leaf_off + I.leaf_off_off;
    const int32_t *blk = a.blk + I.blk_off;
    const float *pts = a.pts + I.pts_off;
    const float *Q = a.Q + I.q_off;
    const float *split = a.split + I.split_off;
    int32_t *node = a.node + I.node_off;
    uint64_t *keys = a.keys + I.key_off;
    const int first = I.nleaf - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int d = I.d, k = I.k;
    unsigned long long pairs = 0;
    for (int j = j0 + wave; j < j1; j += BT / 64) {
        const int32_t q = round == 0 ? j : list[j];
        const float *qp = Q + (int64_t)q * d;
        const float ql = lane < d ? qp[lane] : 0.0f;
        if (lane < d) qs[lane] = ql;
        float qv[D];
#pragma unroll
        for (int c = 0; c < D; c++) qv[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ql), c));
        uint64_t li = lane < k ? keys[(int64_t)q * k + lane] : ~0ull;
        int32_t st = node[q];
        for (;;) {
            const uint64_t kth_key = rdlane64(li, k - 1);
            const int32_t v = next_leaf(st, qs, &kth_key, split, sl, I.nleaf - 1, I.h, d);
            if (v == NODE_DONE) break;
            st = v;
            const int Lf = v - first;
            const int len = lo_pos[Lf + 1] - lo_pos[Lf];
            const float *X = pts + blk[Lf];
            const int32_t *orig = reinterpret_cast<const int32_t *>(X) + (int64_t)d * len;
            pairs += (unsigned)len;
            uint64_t kth = kth_key;
            for (int gb = 0; gb < len; gb += 64 * G) {
                uint64_t key[G];
#pragma unroll
                for (int g = 0; g < G; g++) {
                    const int p = gb + 64 * g + lane;
                    const bool valid = p < len;
                    const int pi = valid ? p : 0;
                    float acc = 0.0f;
#pragma unroll
                    for (int c = 0; c < D; c++) {
                        const float x = X[(int64_t)(c < d ? c : 0) * len + pi];
                        const float tt = qv[c] - (c < d ? x : 0.0f);
                        acc = fmaf(tt, tt, acc);
                    }
                    key[g] = valid ? (((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)orig[pi]) : ~0ull;
                }
#pragma unroll
                for (int g = 0; g < G; g++) {
                    uint64_t cand = __ballot(key[g] < kth);
                    while (cand) {
                        const int c = __ffsll((unsigned long long)cand) - 1;
                        cand &= cand - 1;
                        const uint64_t ck = rdlane64(key[g], c);
                        if (ck < kth) {
                            const uint64_t moved = __ballot(li > ck);
                            const int pos = __ffsll((unsigned long long)moved) - 1;
                            const uint64_t up = __shfl_up(li, 1);
                            li = (lane < pos) ? li : (lane == pos ? ck : up);
                            if (lane >= k) li = ~0ull;
                            kth = rdlane64(li, k - 1);
                        }
                    }
                }
            }
        }
        node[q] = NODE_DONE;
        if (lane < k) keys[(int64_t)q * k + lane] = li;
    }
    if (lane == 0 && pairs) {
        atomicAdd(&a.q->pairs, pairs);
        atomicAdd(&a.q->flops, pairs * 3ull * (unsigned)d);
    }
}

__device__ __forceinline__ void tail_task(const BatchArgs &a, int i, int j0, int j1, RouteLds &L)
{
    switch (a.inst[i].d <= 2 ? 2 : a.inst[i].d <= 3 ? 3 : a.inst[i].d <= 4 ? 4 : a.inst[i].d <= 5 ? 5
            : a.inst[i].d <= 6 ? 6 : a.inst[i].d <= 8 ? 8 : a.inst[i].d <= 10 ? 10 : a.inst[i].d <= 12 ? 12
            : a.inst[i].d <= 15 ? 15 : a.inst[i].d <= 16 ? 16 : a.inst[i].d <= 20 ? 20 : a.inst[i].d <= 24 ? 24 : 32) {
    case 2: tail_queries<2, 2>(a, i, j0, j1, L); break;
    case 3: tail_queries<3, 2>(a, i, j0, j1, L); break;
    case 4: tail_queries<4, 2>(a, i, j0, j1, L); break;
    case 5: tail_queries<5, 2>(a, i, j0, j1, L); break;
    case 6: tail_queries<6, 2>(a, i, j0, j1, L); break;
    case 8: tail_queries<8, 2>(a, i, j0, j1, L); break;
    case 10: tail_queries<10, 2>(a, i, j0, j1, L); break;
    case 12: tail_queries<12, 2>(a, i, j0, j1, L); break;
    case 15: tail_queries<15, 2>(a, i, j0, j1, L); break;
    case 16: tail_queries<16, 2>(a, i, j0, j1, L); break;
    case 20: tail_queries<20, 1>(a, i, j0, j1, L); break;
    case 24: tail_queries<24, 1>(a, i, j0, j1, L); break;
    default: tail_queries<32, 1>(a, i, j0, j1, L); break;
    }
}

__device__ __forceinline__ void scan_task(const BatchArgs &a, int i, int e0, int e1)
{
    switch (a.inst[i].d <= 2 ? 2 : a.inst[i].d <= 3 ? 3 : a.inst[i].d <= 4 ? 4 : a.inst[i].d <= 5 ? 5
            : a.inst[i].d <= 6 ? 6 : a.inst[i].d <= 8 ? 8 : a.inst[i].d <= 10 ? 10 : a.inst[i].d <= 12 ? 12
            : a.inst[i].d <= 15 ? 15 : a.inst[i].d <= 16 ? 16 : a.inst[i].d <= 20 ? 20 : a.inst[i].d <= 24 ? 24 : 32) {
    case 2: scan_leaves<2, 2>(a, i, e0, e1); break;
    case 3: scan_leaves<3, 2>(a, i, e0, e1); break;
    case 4: scan_leaves<4, 2>(a, i, e0, e1); break;
    case 5: scan_leaves<5, 2>(a, i, e0, e1); break;
    case 6: scan_leaves<6, 2>(a, i, e0, e1); break;
    case 8: scan_leaves<8, 2>(a, i, e0, e1); break;
    case 10: scan_leaves<10, 2>(a, i, e0, e1); break;
    case 12: scan_leaves<12, 2>(a, i, e0, e1); break;
    case 15: scan_leaves<15, 2>(a, i, e0, e1); break;
    case 16: scan_leaves<16, 2>(a, i, e0, e1); break;
    case 20: scan_leaves<20, 1>(a, i, e0, e1); break;
    case 24: scan_leaves<24, 1>(a, i, e0, e1); break;
    default: scan_leaves<32, 1>(a, i, e0, e1); break;
    }
}

__global__ __launch_bounds__(BT) void k_batch(BatchArgs a)
{
    __shared__ RouteLds L;
    __shared__ int4 task;
    __shared__ int quit;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            quit = 0;
            const unsigned long long idx = atomicAdd(&a.q->head, 1ull);
            const unsigned long long slot = idx & (QCAP - 1);
            const unsigned long long want = 2 * (idx >> QCAP_LOG) + 1;
            const unsigned long long t0 = wall_clock64();
            while (ld_poll(&a.seq[slot]) != want) {
                if (ld_flag(&a.q->done) || ld_flag(&a.q->error)) {
                    quit = 1;
                    break;
                }
                if (wall_clock64() - t0 > a.spin_ticks) {
                    atomicOr(&a.q->error, 2);
                    quit = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
            if (!quit) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                task = a.tasks[slot];
                st_rel(&a.seq[slot], want + 1);
                atomicAdd(&a.q->tasks, 1ull);
                atomicAdd(&a.q->wait_ticks, wall_clock64() - t0);
            }
        }
        __syncthreads();
        if (quit) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int4 t = task;
        __syncthreads();
        if (t.x == TASK_ORGANIZE) {
            organize_task(a, t.y, L);
        } else if (t.x == TASK_TAIL) {
            tail_task(a, t.y, t.z, t.w, L);
            __threadfence();
            __syncthreads();
            // the last TAIL task retires the instance
            if (tid == 0 && atomicSub(&a.state[t.y].pending, 1) == 1 && atomicSub(&a.q->active, 1) == 1)
                __hip_atomic_store(&a.q->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (t.x == TASK_FIND) find_task(a, t.y, t.z, t.w, L);
            else scan_task(a, t.y, t.z, t.w);
            // the last task of the phase starts the next phase of this instance
            __threadfence();
            __syncthreads();
            if (tid == 0) quit = atomicSub(&a.state[t.y].pending, 1) == 1 ? 1 : 0;
            __syncthreads();
            if (quit) {
                if (t.x == TASK_FIND) {
                    push_tasks(a, 1, [&](int) { return make_int4(TASK_ORGANIZE, t.y, 0, 0); }, &L.base);
                } else {
                    const int V = a.state[t.y].V;
                    if (V <= a.solo_max) {
                        const int T = (V + TAIL_CHUNK - 1) / TAIL_CHUNK;
                        if (tid == 0) a.state[t.y].pending = T;
                        push_tasks(a, T, [&](int j) {
                            return make_int4(TASK_TAIL, t.y, j * TAIL_CHUNK, min(V, (j + 1) * TAIL_CHUNK));
                        }, &L.base);
                    } else {
                        const int F = (V + FIND_CHUNK - 1) / FIND_CHUNK;
                        if (tid == 0) a.state[t.y].pending = F;
                        push_tasks(a, F, [&](int j) {
                            return make_int4(TASK_FIND, t.y, j * FIND_CHUNK, min(V, (j + 1) * FIND_CHUNK));
                        }, &L.base);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Reset: keys EMPTY, queries FRESH, queue empty, one ROUTE task per instance with queries.
__global__ void k_batch_reset_u64(unsigned long long *p, unsigned long long v, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_batch_reset_i32(int32_t *p, int32_t v, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_batch_seed(BatchArgs a, const int4 *seed, int nseed, int nlive)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < a.count) {
        const int m = a.inst[j].m;
        const int chunk = m <= a.solo_max ? TAIL_CHUNK : FIND_CHUNK;  // the seed's task type
        a.state[j] = BState{0, 0, 0, (m + chunk - 1) / chunk};
    }
    if (j < nseed) {
        a.tasks[j] = seed[j];
        a.seq[j] = 1;
    }
    if (j == 0) {
        a.q->head = 0;
        a.q->tail = (unsigned long long)nseed;
        a.q->done = nlive == 0 ? 1 : 0;
        a.q->error = 0;
        a.q->active = nlive;
        a.q->tasks = a.q->pairs = a.q->flops = a.q->rounds = a.q->wait_ticks = 0;
    }
}
__global__ void k_batch_finalize(const uint64_t *keys, int64_t count, int64_t *idx, float *dist, int squared)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[i];
        const float d2 = __uint_as_float((uint32_t)(key >> 32));
        idx[i] = (int64_t)(uint32_t)key;
        dist[i] = squared ? d2 : sqrtf(d2);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side.

struct Batch {
    int device = 0;
    int count = 0;
    int flags = 0;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        DevBuf seed;
    };
    std::vector<bkd_instance> inst;
    std::vector<BInst> desc;
    std::vector<int32_t> live;
    int64_t keys_total = 0;
    DevBuf d_inst, d_state, d_q, d_tasks, d_seq, d_split, d_leaf_off, d_blk, d_pts, d_Q, d_keys, d_node, d_buf, d_tmp,
        d_loff, d_ne, d_cnt, d_oidx, d_odist;
    hipStream_t cap_stream = nullptr;
    std::map<std::tuple<int, int, int>, std::unique_ptr<Graph>> graphs;
    bkd_tuning tuned{};
    bool have_tuned = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t last_stream = nullptr;
    bool ran = false;
    int cus = 256;
    unsigned long long spin_ticks = 0;
    double wall_khz = 1.0;     // wall-clock counter rate
    int32_t last_workgroups = 0;
    ~Batch()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second->exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }
};

static void batch_validate(const bkd_instance *in, int32_t count)
{
    if (!in || count < 0) fail(BKD_EINVAL, "instances must be a non-NULL array and count >= 0");
    for (int i = 0; i < count; i++) {
        const bkd_instance &x = in[i];
        auto bad = [&](const char *what) { fail(BKD_EINVAL, "instance " + std::to_string(i) + ": " + what); };
        if (!x.P || x.n < 1 || x.n > INT32_MAX) bad("P must be non-NULL with 1 <= n <= 2^31-1");
        if (x.d < 1 || x.d > BKD_MAX_DIM) bad("d must be in [1, 32]");
        if (x.height < 0 || x.height > 12 || (int64_t(1) << x.height) > x.n) bad("height must be in [0, 12] with 2^h <= n");
        if (x.k < 1 || x.k > BKD_MAX_K || x.k > x.n) bad("k must be in [1, min(n, 64)]");
        if (x.m < 0 || x.m > INT32_MAX) bad("m must be in [0, 2^31-1]");
        if (x.m > 0 && (!x.Q || !x.out_idx || !x.out_dist)) bad("Q and outputs must be non-NULL");
        for (int64_t j = 0; j < x.n * x.d; j++)
            if (!std::isfinite(x.P[j])) bad("reference coordinates must be finite");
        for (int64_t j = 0; j < x.m * x.d; j++)
            if (!std::isfinite(x.Q[j])) bad("query coordinates must be finite");
    }
}

template <class T> static void upload(DevBuf &b, const std::vector<T> &v)
{
    b.ensure(sizeof(T) * std::max<size_t>(1, v.size()));
    if (!v.empty()) BKD_HIP(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
}

// Under BKD_FLAG_DEVICE_PTRS: every pointer of the instances must be device memory on `device`.
static void check_device_pointer(const void *p, int device, int i, const char *what)
{
    hipPointerAttribute_t at{};
    const hipError_t e = hipPointerGetAttributes(&at, p);
    if (e != hipSuccess || at.type != hipMemoryTypeDevice || at.device != device) {
        (void)hipGetLastError();
        fail(BKD_EINVAL, "instance " + std::to_string(i) + ": " + what + " is not device memory on the batch's device");
    }
}

Batch *batch_create(const bkd_instance *in_given, int32_t count, int32_t device, int32_t flags)
{
    if (!in_given || count < 0) fail(BKD_EINVAL, "instances must be a non-NULL array and count >= 0");
    int ndev = 0;
    BKD_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) fail(BKD_EINVAL, "device ordinal out of range");
    BKD_HIP(hipSetDevice(device));
    // device instances: P and Q read back into host copies for the host build and checks
    const bool dev_ptrs = (flags & BKD_FLAG_DEVICE_PTRS) != 0;
    std::vector<bkd_instance> hin;
    std::vector<std::vector<float>> hcopy;
    const bkd_instance *in = in_given;
    if (dev_ptrs) {
        hin.assign(in_given, in_given + count);
        hcopy.resize(2 * (size_t)count);
        for (int i = 0; i < count; i++) {
            bkd_instance &x = hin[(size_t)i];
            if (x.n < 1 || x.n > INT32_MAX || x.d < 1 || x.d > BKD_MAX_DIM || x.m < 0 || x.m > INT32_MAX) continue;
            if (x.P) {
                check_device_pointer(x.P, device, i, "P");
                hcopy[2 * (size_t)i].resize((size_t)(x.n * x.d));
                BKD_HIP(hipMemcpy(hcopy[2 * (size_t)i].data(), x.P, sizeof(float) * (size_t)(x.n * x.d),
                                  hipMemcpyDeviceToHost));
                x.P = hcopy[2 * (size_t)i].data();
            }
            if (x.m > 0 && x.Q) {
                check_device_pointer(x.Q, device, i, "Q");
                hcopy[2 * (size_t)i + 1].resize((size_t)(x.m * x.d));
                BKD_HIP(hipMemcpy(hcopy[2 * (size_t)i + 1].data(), x.Q, sizeof(float) * (size_t)(x.m * x.d),
                                  hipMemcpyDeviceToHost));
                x.Q = hcopy[2 * (size_t)i + 1].data();
            }
            if (x.m > 0 && x.out_idx) check_device_pointer(x.out_idx, device, i, "out_idx");
            if (x.m > 0 && x.out_dist) check_device_pointer(x.out_dist, device, i, "out_dist");
        }
        in = hin.data();
    }
    batch_validate(in, count);
    auto b = std::make_unique<Batch>();
    b->device = device;
    b->count = count;
    b->flags = flags;
    b->inst.assign(in_given, in_given + count);  // the caller's output pointers (host or device)
    // trees, built in parallel over instances
    std::vector<HostTree> trees((size_t)count);
    parallel_for(count, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; i++)
            build_canonical(in[i].P, in[i].n, in[i].d, in[i].height, trees[(size_t)i], false);
    });
    b->desc.resize((size_t)count);
    int64_t o_split = 0, o_lo = 0, o_blk = 0, o_pts = 0, o_q = 0, o_key = 0, o_m = 0, o_loff = 0, o_ne = 0, o_cnt = 0;
    for (int i = 0; i < count; i++) {
        const bkd_instance &x = in[i];
        BInst &D = b->desc[(size_t)i];
        const int nleaf = 1 << x.height;
        D.d = x.d;
        D.k = x.k;
        D.h = x.height;
        D.nleaf = nleaf;
        D.m = (int32_t)x.m;
        D.n = (int32_t)x.n;
        D.split_off = o_split;
        D.leaf_off_off = o_lo;
        D.blk_off = o_blk;
        D.pts_off = o_pts;
        D.q_off = o_q;
        D.key_off = o_key;
        D.node_off = o_m;
        D.buf_off = 2 * o_m;
        D.tmp_off = o_m;
        D.loff_off = o_loff;
        D.ne_off = o_ne;
        D.cnt_off = o_cnt;
        o_cnt += nleaf;
        o_split += nleaf - 1;
        o_lo += nleaf + 1;
        o_blk += nleaf + 1;
        o_pts += (int64_t)(x.d + 1) * x.n;
        o_q += x.m * x.d;
        o_key += x.m * x.k;
        o_m += x.m;
        o_loff += nleaf + 1;
        o_ne += nleaf;
        if (x.m > 0) b->live.push_back(i);
    }
    b->keys_total = o_key;
    std::vector<float> split((size_t)o_split), pts((size_t)o_pts), Q((size_t)o_q);
    std::vector<int32_t> leaf_off((size_t)o_lo), blk((size_t)o_blk);
    parallel_for(count, [&](int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; i++) {
            const bkd_instance &x = in[i];
            const BInst &D = b->desc[(size_t)i];
            const HostTree &H = trees[(size_t)i];
            std::copy(H.split.begin(), H.split.end(), split.begin() + D.split_off);
            int32_t w = 0;
            for (int l = 0; l <= D.nleaf; l++) {
                leaf_off[(size_t)(D.leaf_off_off + l)] = (int32_t)H.leaf_off[(size_t)l];
                blk[(size_t)(D.blk_off + l)] = w;
                if (l < D.nleaf) w += (int32_t)((x.d + 1) * (H.leaf_off[(size_t)l + 1] - H.leaf_off[(size_t)l]));
            }
            for (int l = 0; l < D.nleaf; l++) {
                const int64_t a0 = H.leaf_off[(size_t)l], len = H.leaf_off[(size_t)l + 1] - a0;
                float *X = pts.data() + D.pts_off + blk[(size_t)(D.blk_off + l)];
                int32_t *orig = reinterpret_cast<int32_t *>(X + (size_t)x.d * len);
                for (int64_t p = 0; p < len; p++) {
                    const int32_t o = H.perm[(size_t)(a0 + p)];
                    for (int j = 0; j < x.d; j++) X[(size_t)j * len + p] = x.P[(int64_t)o * x.d + j];
                    orig[p] = o;
                }
            }
            if (x.m > 0) std::copy(x.Q, x.Q + x.m * x.d, Q.begin() + D.q_off);
        }
    });
    upload(b->d_inst, b->desc);
    upload(b->d_split, split);
    upload(b->d_leaf_off, leaf_off);
    upload(b->d_blk, blk);
    upload(b->d_pts, pts);
    upload(b->d_Q, Q);
    b->d_state.ensure(sizeof(BState) * std::max(1, count));
    b->d_q.ensure(sizeof(BQueue));
    b->d_tasks.ensure(sizeof(int4) * QCAP);
    b->d_seq.ensure(sizeof(unsigned long long) * QCAP);
    b->d_keys.ensure(sizeof(uint64_t) * std::max<int64_t>(1, o_key));
    b->d_node.ensure(sizeof(int32_t) * std::max<int64_t>(1, o_m));
    b->d_buf.ensure(sizeof(int32_t) * std::max<int64_t>(1, 2 * o_m));
    b->d_tmp.ensure(sizeof(int32_t) * std::max<int64_t>(1, o_m));
    b->d_loff.ensure(sizeof(int32_t) * std::max<int64_t>(1, o_loff));
    b->d_ne.ensure(sizeof(int32_t) * std::max<int64_t>(1, o_ne));
    b->d_cnt.ensure(sizeof(int32_t) * std::max<int64_t>(1, o_cnt));
    b->d_oidx.ensure(sizeof(int64_t) * std::max<int64_t>(1, o_key));
    b->d_odist.ensure(sizeof(float) * std::max<int64_t>(1, o_key));
    BKD_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    BKD_HIP(hipEventCreate(&b->ev0));
    BKD_HIP(hipEventCreate(&b->ev1));
    hipDeviceProp_t prop;
    BKD_HIP(hipGetDeviceProperties(&prop, device));
    b->cus = prop.multiProcessorCount;
    int rate_khz = 0;
    BKD_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device));
    b->spin_ticks = (unsigned long long)std::max(rate_khz, 1) * 1000ull * 60ull;  // 60 s guard
    b->wall_khz = (double)std::max(rate_khz, 1);
    BKD_HIP(hipDeviceSynchronize());
    return b.release();
}

static BatchArgs batch_args(Batch &b, const bkd_tuning &tu)
{
    BatchArgs a{};
    a.inst = b.d_inst.as<BInst>();
    a.state = b.d_state.as<BState>();
    a.q = b.d_q.as<BQueue>();
    a.tasks = b.d_tasks.as<int4>();
    a.seq = b.d_seq.as<unsigned long long>();
    a.split = b.d_split.as<float>();
    a.leaf_off = b.d_leaf_off.as<int32_t>();
    a.blk = b.d_blk.as<int32_t>();
    a.pts = b.d_pts.as<float>();
    a.Q = b.d_Q.as<float>();
    a.keys = b.d_keys.as<uint64_t>();
    a.node = b.d_node.as<int32_t>();
    a.buf = b.d_buf.as<int32_t>();
    a.tmp = b.d_tmp.as<int32_t>();
    a.loff = b.d_loff.as<int32_t>();
    a.ne = b.d_ne.as<int32_t>();
    a.cnt = b.d_cnt.as<int32_t>();
    a.leaves_per_task = tu.leaves_per_task;
    a.solo_max = tu.solo_max;
    a.count = b.count;
    a.spin_ticks = b.spin_ticks;
    return a;
}

static bkd_tuning normalise(const bkd_tuning *t)
{
    bkd_tuning u{8, 4, 2048};
    if (t) {
        if (t->leaves_per_task) u.leaves_per_task = t->leaves_per_task;
        if (t->groups_per_cu) u.groups_per_cu = t->groups_per_cu;
        if (t->solo_max) u.solo_max = t->solo_max;
    }
    if (u.leaves_per_task < 1 || u.leaves_per_task > 256) fail(BKD_EINVAL, "leaves_per_task must be in [1, 256]");
    if (u.groups_per_cu < 1 || u.groups_per_cu > 16) fail(BKD_EINVAL, "groups_per_cu must be in [1, 16]");
    if (u.solo_max < 0) fail(BKD_EINVAL, "solo_max must be >= 0");
    return u;
}

void batch_run(Batch &b, const bkd_tuning *tune, hipStream_t s)
{
    BKD_HIP(hipSetDevice(b.device));
    const bkd_tuning tu = normalise(tune ? tune : (b.have_tuned ? &b.tuned : nullptr));
    b.last_workgroups = b.cus * tu.groups_per_cu;
    const auto key = std::make_tuple(tu.leaves_per_task, tu.groups_per_cu, tu.solo_max);
    auto it = b.graphs.find(key);
    if (it == b.graphs.end()) {
        auto G = std::make_unique<Batch::Graph>();
        // first tasks: per-query traversals (TAIL) for small instances, FIND slices otherwise
        std::vector<int4> seed;
        for (int i : b.live) {
            const int64_t m = b.inst[(size_t)i].m;
            if (m <= tu.solo_max) {
                for (int64_t j0 = 0; j0 < m; j0 += TAIL_CHUNK)
                    seed.push_back(make_int4(TASK_TAIL, i, (int)j0, (int)std::min<int64_t>(m, j0 + TAIL_CHUNK)));
            } else {
                for (int64_t j0 = 0; j0 < m; j0 += FIND_CHUNK)
                    seed.push_back(make_int4(TASK_FIND, i, (int)j0, (int)std::min<int64_t>(m, j0 + FIND_CHUNK)));
            }
        }
        if ((unsigned long long)seed.size() >= QCAP) fail(BKD_EINVAL, "too many queries for one batched launch");
        upload(G->seed, seed);
        // capture: reset state, persistent kernel, key -> (index, distance)
        const BatchArgs a = batch_args(b, tu);
        hipStream_t c = b.cap_stream;
        BKD_HIP(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        k_batch_reset_u64<<<1024, 256, 0, c>>>(b.d_keys.as<unsigned long long>(), EMPTY_KEY, b.keys_total);
        k_batch_reset_i32<<<1024, 256, 0, c>>>(b.d_node.as<int32_t>(), NODE_FRESH,
                                                (int64_t)(b.d_node.bytes / sizeof(int32_t)));
        k_batch_reset_i32<<<256, 256, 0, c>>>(b.d_cnt.as<int32_t>(), 0, (int64_t)(b.d_cnt.bytes / sizeof(int32_t)));
        k_batch_reset_u64<<<1024, 256, 0, c>>>(b.d_seq.as<unsigned long long>(), 0ull, (int64_t)QCAP);
        const int nseed = (int)seed.size(), nlive = (int)b.live.size();
        k_batch_seed<<<(std::max(b.count, nseed) + 255) / 256 + 1, 256, 0, c>>>(a, G->seed.as<int4>(), nseed, nlive);
        k_batch<<<b.cus * tu.groups_per_cu, BT, 0, c>>>(a);
        k_batch_finalize<<<1024, 256, 0, c>>>(b.d_keys.as<uint64_t>(), b.keys_total, b.d_oidx.as<int64_t>(),
                                              b.d_odist.as<float>(), (b.flags & BKD_FLAG_SQUARED) ? 1 : 0);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c, &g);
        if (e != hipSuccess) fail(BKD_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) fail(BKD_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        it = b.graphs.emplace(key, std::move(G)).first;
    }
    BKD_HIP(hipEventRecord(b.ev0, s));
    BKD_HIP(hipGraphLaunch(it->second->exec, s));
    BKD_HIP(hipEventRecord(b.ev1, s));
    b.last_stream = s;
    b.ran = true;
}

static BQueue read_queue(Batch &b)
{
    BKD_HIP(hipStreamSynchronize(b.last_stream));
    BQueue q;
    BKD_HIP(hipMemcpy(&q, b.d_q.p, sizeof(BQueue), hipMemcpyDeviceToHost));
    return q;
}

void batch_results(Batch &b)
{
    if (!b.ran) fail(BKD_EINVAL, "bkd_batch_run has not been called");
    BQueue q = read_queue(b);
    if (q.error) fail(BKD_EDEVICE, "batched launch stopped early (error flag " + std::to_string(q.error) + ")");
    if (b.flags & BKD_FLAG_DEVICE_PTRS) {
        // device outputs: one device-to-device copy per instance and array
        for (int i = 0; i < b.count; i++) {
            const bkd_instance &x = b.inst[(size_t)i];
            const int64_t o = b.desc[(size_t)i].key_off, c = x.m * x.k;
            if (!c) continue;
            BKD_HIP(hipMemcpyAsync(x.out_idx, b.d_oidx.as<int64_t>() + o, sizeof(int64_t) * c,
                                   hipMemcpyDeviceToDevice, b.cap_stream));
            BKD_HIP(hipMemcpyAsync(x.out_dist, b.d_odist.as<float>() + o, sizeof(float) * c,
                                   hipMemcpyDeviceToDevice, b.cap_stream));
        }
        BKD_HIP(hipStreamSynchronize(b.cap_stream));
        return;
    }
    std::vector<int64_t> idx((size_t)b.keys_total);
    std::vector<float> dist((size_t)b.keys_total);
    if (b.keys_total) {
        BKD_HIP(hipMemcpy(idx.data(), b.d_oidx.p, sizeof(int64_t) * idx.size(), hipMemcpyDeviceToHost));
        BKD_HIP(hipMemcpy(dist.data(), b.d_odist.p, sizeof(float) * dist.size(), hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < b.count; i++) {
        const bkd_instance &x = b.inst[(size_t)i];
        const int64_t o = b.desc[(size_t)i].key_off, c = x.m * x.k;
        if (c) {
            std::memcpy(x.out_idx, idx.data() + o, sizeof(int64_t) * c);
            std::memcpy(x.out_dist, dist.data() + o, sizeof(float) * c);
        }
    }
}

void batch_stats(Batch &b, bkd_batch_stats *out)
{
    *out = bkd_batch_stats{};
    out->instances = b.count;
    for (auto &x : b.inst) out->queries += x.m;
    if (!b.ran) return;
    BQueue q = read_queue(b);
    out->tasks = (int64_t)q.tasks;
    out->rounds = (int64_t)q.rounds;
    out->pairs = (int64_t)q.pairs;
    out->flops = (int64_t)q.flops;
    out->error = q.error;
    out->workgroups = b.last_workgroups;
    out->claim_wait_ms = (double)q.wait_ticks / b.wall_khz;
    float ms = 0;
    BKD_HIP(hipEventElapsedTime(&ms, b.ev0, b.ev1));
    out->run_ms = ms;
}

void batch_autotune(Batch &b, bkd_tuning *best, double *best_ms)
{
    const int lpts[] = {4, 16, 64};
    const int gpcs[] = {2, 4};
    const int solos[] = {2048, 8192, 16384, 32768};
    hipStream_t s = b.cap_stream;
    double bm = 1e300;
    bkd_tuning bt{8, 4, 2048};
    for (int g : gpcs)
        for (int l : lpts)
            for (int so : solos) {
            bkd_tuning t{l, g, so};
            batch_run(b, &t, s);  // warm-up (first run also captures the graph)
            batch_run(b, &t, s);
            BQueue q = read_queue(b);
            if (q.error) fail(BKD_EDEVICE, "batched launch stopped early during tuning");
            float ms = 0;
            BKD_HIP(hipEventElapsedTime(&ms, b.ev0, b.ev1));
            if (ms < bm) {
                bm = ms;
                bt = t;
            }
        }
    b.tuned = bt;
    b.have_tuned = true;
    if (best) *best = bt;
    if (best_ms) *best_ms = bm;
}

// Signature of a batch for the tuning cache: the device's name and compute-unit count, and every
// instance's (n, m, d, k, height), hashed with 64-bit FNV-1a.
static uint64_t batch_signature(const Batch &b)
{
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; i++) hsh = (hsh ^ c[i]) * 1099511628211ull;
    };
    hipDeviceProp_t prop;
    BKD_HIP(hipGetDeviceProperties(&prop, b.device));
    mix(prop.gcnArchName, std::strlen(prop.gcnArchName));
    mix(&b.cus, sizeof(b.cus));
    for (const bkd_instance &x : b.inst) {
        const int64_t v[5] = {x.n, x.m, x.d, x.k, x.height};
        mix(v, sizeof(v));
    }
    return hsh;
}

// The tuning cache: a text file of lines "signature leaves_per_task groups_per_cu solo_max ms".
void batch_tuning_save(const Batch &b, const char *path)
{
    if (!path) fail(BKD_EINVAL, "path is NULL");
    if (!b.have_tuned) fail(BKD_EINVAL, "the batch has not been tuned (bkd_batch_autotune)");
    const uint64_t sig = batch_signature(b);
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(path, "r")) {  // other batches' lines stay
        char line[256];
        while (std::fgets(line, sizeof line, f)) {
            unsigned long long s = 0;
            if (std::sscanf(line, "%llx", &s) == 1 && s != sig) keep.emplace_back(line);
        }
        std::fclose(f);
    }
    FILE *f = std::fopen(path, "w");
    if (!f) fail(BKD_EINVAL, std::string("cannot write the tuning cache ") + path);
    for (const std::string &l : keep) std::fputs(l.c_str(), f);
    std::fprintf(f, "%016llx %d %d %d\n", (unsigned long long)sig, b.tuned.leaves_per_task, b.tuned.groups_per_cu,
                 b.tuned.solo_max);
    const bool ok = std::fclose(f) == 0;
    if (!ok) fail(BKD_EINVAL, std::string("cannot write the tuning cache ") + path);
}

// Returns false (nothing changed) when the cache has no line for this batch.
bool batch_tuning_load(Batch &b, const char *path, bkd_tuning *out)
{
    if (!path) fail(BKD_EINVAL, "path is NULL");
    const uint64_t sig = batch_signature(b);
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    bkd_tuning t{};
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long s = 0;
        bkd_tuning u{};
        if (std::sscanf(line, "%llx %d %d %d", &s, &u.leaves_per_task, &u.groups_per_cu, &u.solo_max) == 4 && s == sig) {
            t = u;
            found = true;
        }
    }
    std::fclose(f);
    if (!found) return false;
    b.tuned = normalise(&t);
    b.have_tuned = true;
    if (out) *out = b.tuned;
    return true;
}

}  // namespace bkd

struct bkd_batch {
    bkd::Batch *b;
};

namespace bkd {
int guarded_call(const std::function<void()> &f);
}

extern "C" {

int bkd_batch_create(const bkd_instance *inst, int32_t count, int32_t device, int32_t flags, bkd_batch **out)
{
    return bkd::guarded_call([&] {
        if (!out) bkd::fail(BKD_EINVAL, "out is NULL");
        *out = nullptr;
        std::unique_ptr<bkd::Batch> b(bkd::batch_create(inst, count, device, flags));
        *out = new bkd_batch{b.release()};
    });
}

int bkd_batch_run(bkd_batch *batch, const bkd_tuning *tune, void *stream)
{
    return bkd::guarded_call([&] {
        if (!batch) bkd::fail(BKD_EINVAL, "batch is NULL");
        bkd::batch_run(*batch->b, tune, static_cast<hipStream_t>(stream));
    });
}

int bkd_batch_results(bkd_batch *batch)
{
    return bkd::guarded_call([&] {
        if (!batch) bkd::fail(BKD_EINVAL, "batch is NULL");
        bkd::batch_results(*batch->b);
    });
}

int bkd_batch_autotune(bkd_batch *batch, bkd_tuning *best, double *best_ms)
{
    return bkd::guarded_call([&] {
        if (!batch) bkd::fail(BKD_EINVAL, "batch is NULL");
        bkd::batch_autotune(*batch->b, best, best_ms);
    });
}

int bkd_batch_tuning_save(const bkd_batch *batch, const char *path)
{
    return bkd::guarded_call([&] {
        if (!batch) bkd::fail(BKD_EINVAL, "batch is NULL");
        bkd::batch_tuning_save(*batch->b, path);
    });
}

int bkd_batch_tuning_load(bkd_batch *batch, const char *path, bkd_tuning *tuning)
{
    return bkd::guarded_call([&] {
        if (!batch) bkd::fail(BKD_EINVAL, "batch is NULL");
        if (!bkd::batch_tuning_load(*batch->b, path, tuning))
            bkd::fail(BKD_ENOTFOUND, "no tuning for this batch in the cache");
    });
}

int bkd_batch_stats_get(const bkd_batch *batch, bkd_batch_stats *out)
{
    return bkd::guarded_call([&] {
        if (!batch || !out) bkd::fail(BKD_EINVAL, "NULL pointer");
        bkd::batch_stats(*batch->b, out);
    });
}

int bkd_batch_free(bkd_batch *batch)
{
    return bkd::guarded_call([&] {
        if (!batch) return;
        (void)hipSetDevice(batch->b->device);
        (void)hipDeviceSynchronize();
        delete batch->b;
        delete batch;
    });
}

}  // extern "C"
