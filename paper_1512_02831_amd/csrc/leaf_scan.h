// leaf_scan.h -- ProcessAllBuffers leaf scan (Section 2.4, Section 3.2), gfx950.
//
// Dense leaves (many buffered queries): one workgroup of 256 lanes takes one
// work item, up to 256 buffered queries of one leaf, one query per lane.  The
// leaf's points (the part held by the current chunk) stream through LDS in
// tiles, point-major with the coordinates padded to a multiple of four, so
// that every lane reads the same point with a broadcast ds_read_b128.  Each
// lane keeps its query in registers and its K best keys as a sorted register
// list; a point enters through a compare-exchange cascade only when its key
// beats the K-th best (a wave-uniform branch, skipped when no lane qualifies).
//
// Inner-product filter.  Once every query of a tile has K candidates, a point
// is first tested with the expansion |q-x|^2 = |q'|^2 + |x'|^2 - 2<q',x'> on
// coordinates relative to the leaf centre c (q' = q-c, x' = x-c, both rounded
// to float32): d fused multiply-adds per pair instead of d subtractions and d
// FMAs.  The test accepts every point whose exact float32 distance could reach
// the K-th best thr: with S = |q'|^2 + |x'|^2, the computed expansion differs
// from the float32 distance by at most (4d + 14) 2^-24 S (centring, the dot
// product, the norms, the final combination and the float32 distance itself;
// a borderline case has thr <= 2S, so the comparison's own rounding is of the
// same order), and the test  (1 - c(d)) S - 2<q',x'> <= thr  uses c(d) = 4
// times that bound.  Accepted points are re-checked with the exact float32
// distance, so keys and results are bit-identical to the exact path.
//
// Squared distances follow the float32 reading: t = q_j - x_j rounded, then
// acc = fma(t, t, acc) for j = 0..d-1 from +0.  Padding dimensions hold zero in
// both the query and the point and leave acc unchanged.  The key of a point
// is (bits of acc) << 32 | original index, so the sorted list breaks exact
// ties by smaller index.  Keys are merged into the query's list as a set:
// the result does not depend on tiling, chunking or processing order.
//
// Sparse leaves (few buffered queries, typical of the late rounds): one wave
// per buffered query.  The query sits in scalar registers, the 64 lanes walk
// the leaf's points 64 at a time with coalesced loads straight from the
// leaf structure, and the query's K best keys are spread over the lanes (lane
// i holds the i-th smallest).  A point whose key beats the K-th best is
// inserted with a ballot for its rank and a one-lane shift of the list.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"

namespace bkd {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PT = 256;  // points per LDS tile

template <int K> __device__ inline void key_insert(uint64_t (&lst)[K], uint64_t c)
{
#pragma unroll
    for (int s = 0; s < K; s++) {
        uint64_t a = lst[s];
        bool lt = c < a;
        lst[s] = lt ? c : a;
        c = lt ? a : c;
    }
}

__device__ inline int xcd_item(int b, int grid)
{
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of items so that a leaf's tiles share one L2.
    int per = grid >> 3;
    return (b & 7) * per + (b >> 3);
}

template <int D, int K> __global__ __launch_bounds__(SCAN_THREADS) void k_leaf_scan(ScanArgs a)
{
    constexpr int NQ = dense_queries_per_lane(D, K);  // queries per lane: each staged point feeds NQ queries
    constexpr int QT = SCAN_THREADS * NQ;
    constexpr int DS = (D + 3) & ~3;
    constexpr int PT = D > 16 ? SCAN_PT / 2 : SCAN_PT;  // points per LDS tile
    __shared__ float4 xs[PT * DS / 4];  // original coordinates, point-major
    __shared__ float4 xc[PT * DS / 4];  // coordinates minus the leaf centre
    __shared__ float bs[PT];            // (1 - c) |x - centre|^2 / 2
    __shared__ int32_t os[PT];

    int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= a.item_count) return;
    item += a.item_first;

    // leaf of the item: largest L in [leaf_first, leaf_last] with tiles[L] <= item
    int lo = a.leaf_first, hi = a.leaf_last;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.tiles[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    const int L = lo;
    const int qbase = a.off[L] + (item - a.tiles[L]) * QT;
    const int qcnt = min(QT, a.off[L + 1] - qbase);
    const int64_t l0 = a.leaf_off[L];
    const int len = a.leaf_off[L + 1] - a.leaf_off[L];
    const int64_t p0 = max(l0, a.chunk_lo);
    const int64_t p1 = min(l0 + len, a.chunk_hi);
    const float *X = a.base + (a.blk[L] + a.blk_shift);
    const int32_t *orig = reinterpret_cast<const int32_t *>(X) + (int64_t)a.d * len;
    const float *cen = a.centers + (int64_t)L * a.d;
    const float coef = a.filter_coef;

    const int tid = threadIdx.x;
    // lane tid holds queries tid and tid + 256 of the tile
    bool act[NQ];
    int32_t q[NQ];
    float qv[NQ][D], qc[NQ][D], Qn[NQ], thr[NQ], Aq[NQ];
    uint64_t lst[NQ][K];
    bool fresh = false;
#pragma unroll
    for (int u = 0; u < NQ; u++) {
        act[u] = tid + SCAN_THREADS * u < qcnt;
        q[u] = act[u] ? a.bufq[qbase + tid + SCAN_THREADS * u] : 0;
        Qn[u] = 0.0f;
#pragma unroll
        for (int j = 0; j < D; j++) {
            qv[u][j] = (act[u] && j < a.d) ? a.Q[(int64_t)q[u] * a.d + j] : 0.0f;
            qc[u][j] = (j < a.d) ? qv[u][j] - cen[j] : 0.0f;
            Qn[u] = fmaf(qc[u][j], qc[u][j], Qn[u]);
        }
#pragma unroll
        for (int s2 = 0; s2 < K; s2++) lst[u][s2] = act[u] ? a.keys[(int64_t)q[u] * K + s2] : 0ull;  // 0: nothing enters
        thr[u] = __uint_as_float((uint32_t)(lst[u][K - 1] >> 32));
        fresh |= act[u] && isinf(thr[u]);
        Aq[u] = act[u] ? 0.5f * (coef * Qn[u] - thr[u]) : INFINITY;
    }
    const bool wave_busy = (tid & ~63) < qcnt;
    const bool wave_dual = NQ > 1 && (tid & ~63) + SCAN_THREADS < qcnt;
    // A query whose list is not full yet (K-th key EMPTY) accepts every point; such
    // tiles take the exact path, all others the inner-product filter.
    const bool exact_path = __syncthreads_or(fresh) != 0;

    auto exact_points = [&](auto nq_tag, int np) {
        constexpr int N = decltype(nq_tag)::value;
#pragma unroll 2
        for (int i = 0; i < np; i++) {
            const float4 *xp = xs + i * (DS / 4);
            float acc[N];
#pragma unroll
            for (int u = 0; u < N; u++) acc[u] = 0.0f;
#pragma unroll
            for (int c = 0; c < DS / 4; c++) {
                float4 x4 = xp[c];
                float xe[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (4 * c + e < D) {
#pragma unroll
                        for (int u = 0; u < N; u++) {
                            float t = qv[u][4 * c + e] - xe[e];
                            acc[u] = fmaf(t, t, acc[u]);
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < N; u++) {
                uint64_t key = ((uint64_t)__float_as_uint(acc[u]) << 32) | (uint32_t)os[i];
                if (key < lst[u][K - 1]) key_insert<K>(lst[u], key);
            }
        }
    };
    auto filter_points = [&](auto nq_tag, int np) {
        constexpr int N = decltype(nq_tag)::value;
#pragma unroll 4
        for (int i = 0; i < np; i++) {
            const float4 *cp = xc + i * (DS / 4);
            float dot[N];
#pragma unroll
            for (int u = 0; u < N; u++) dot[u] = 0.0f;
#pragma unroll
            for (int c = 0; c < DS / 4; c++) {
                float4 x4 = cp[c];
                float xe[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
                for (int e = 0; e < 4; e++)
                    if (4 * c + e < D) {
#pragma unroll
                        for (int u = 0; u < N; u++) dot[u] = fmaf(qc[u][4 * c + e], xe[e], dot[u]);
                    }
            }
            const float b = bs[i];
            bool pass[N], any = false;
#pragma unroll
            for (int u = 0; u < N; u++) {
                pass[u] = Aq[u] + b <= dot[u];
                any |= pass[u];
            }
            if (any) {
                // inside the error band of the filter: decide with the exact float32 distance
                const float4 *xp = xs + i * (DS / 4);
#pragma unroll
                for (int u = 0; u < N; u++) {
                    if (pass[u]) {
                        float acc = 0.0f;
#pragma unroll
                        for (int c = 0; c < DS / 4; c++) {
                            float4 x4 = xp[c];
                            float xe[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
                            for (int e = 0; e < 4; e++) {
                                if (4 * c + e < D) {
                                    float t = qv[u][4 * c + e] - xe[e];
                                    acc = fmaf(t, t, acc);
                                }
                            }
                        }
                        uint64_t key = ((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)os[i];
                        if (key < lst[u][K - 1]) {
                            key_insert<K>(lst[u], key);
                            thr[u] = __uint_as_float((uint32_t)(lst[u][K - 1] >> 32));
                            Aq[u] = 0.5f * (coef * Qn[u] - thr[u]);
                        }
                    }
                }
            }
        }
    };

    for (int64_t pt = p0; pt < p1; pt += PT) {
        const int np = (int)min((int64_t)PT, p1 - pt);
        __syncthreads();
        for (int t = tid; t < np; t += SCAN_THREADS) {
            const int i = (int)(pt - l0) + t;
            float *ro = reinterpret_cast<float *>(xs) + t * DS;
            float *rc = reinterpret_cast<float *>(xc) + t * DS;
            float Xn = 0.0f;
#pragma unroll
            for (int j = 0; j < DS; j++) {
                const float x = (j < a.d) ? X[j * len + i] : 0.0f;
                const float c = (j < a.d) ? x - cen[j] : 0.0f;
                ro[j] = x;
                rc[j] = c;
                Xn = fmaf(c, c, Xn);
            }
            bs[t] = 0.5f * (coef * Xn);
            os[t] = orig[i];
        }
        __syncthreads();
        if (!wave_busy) continue;  // whole wave without queries: only helps staging
        if constexpr (NQ > 1) {
            if (wave_dual) {
                if (exact_path) exact_points(std::integral_constant<int, 2>{}, np);
                else filter_points(std::integral_constant<int, 2>{}, np);
                continue;
            }
        }
        if (exact_path) exact_points(std::integral_constant<int, 1>{}, np);
        else filter_points(std::integral_constant<int, 1>{}, np);
    }
#pragma unroll
    for (int u = 0; u < NQ; u++) {
        if (act[u]) {
#pragma unroll
            for (int s2 = 0; s2 < K; s2++) a.keys[(int64_t)q[u] * K + s2] = lst[u][s2];
        }
    }
}

__device__ inline uint64_t readlane_u64(uint64_t v, int lane)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

template <int D, int K> __global__ __launch_bounds__(SCAN_THREADS) void k_leaf_scan_sparse(ScanArgs a)
{
    const int lane = threadIdx.x & 63;
    int s = __builtin_amdgcn_readfirstlane(xcd_item(blockIdx.x, gridDim.x) * (SCAN_THREADS / 64) +
                                           (int)(threadIdx.x >> 6));
    if (s >= a.sitem_count) return;
    s += a.sitem_first;
    int lo = a.leaf_first, hi = a.leaf_last;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.sparse[mid] <= s) lo = mid;
        else hi = mid - 1;
    }
    const int L = lo;
    const int32_t q = __builtin_amdgcn_readfirstlane(a.bufq[a.off[L] + (s - a.sparse[L])]);
    const float *qp = a.Q + (int64_t)q * a.d;
    float qv[D];
#pragma unroll
    for (int j = 0; j < D; j++) qv[j] = (j < a.d) ? qp[j] : 0.0f;
    uint64_t *kp = a.keys + (int64_t)q * K;
    uint64_t li = (lane < K) ? kp[lane] : ~0ull;
    uint64_t kth = readlane_u64(li, K - 1);

    const int64_t l0 = a.leaf_off[L];
    const int len = a.leaf_off[L + 1] - a.leaf_off[L];
    const int64_t p0 = max(l0, a.chunk_lo);
    const int64_t p1 = min(l0 + len, a.chunk_hi);
    const float *X = a.base + (a.blk[L] + a.blk_shift);
    const int32_t *orig = reinterpret_cast<const int32_t *>(X) + (int64_t)a.d * len;
    for (int64_t pb = p0; pb < p1; pb += 64) {
        const int64_t p = pb + lane;
        const bool valid = p < p1;
        const int i = valid ? (int)(p - l0) : 0;
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < D; j++) {
            float x = (valid && j < a.d) ? X[j * len + i] : 0.0f;
            float t = qv[j] - x;
            acc = fmaf(t, t, acc);
        }
        const uint64_t key = valid ? (((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)orig[i]) : ~0ull;
        uint64_t cand = __ballot(key < kth);
        while (cand) {
            const int c = __ffsll((unsigned long long)cand) - 1;
            cand &= cand - 1;
            const uint64_t ck = readlane_u64(key, c);
            if (ck < kth) {
                const uint64_t moved = __ballot(li > ck);  // entries at and after the insertion rank
                const int pos = __ffsll((unsigned long long)moved) - 1;
                const uint64_t up = __shfl_up(li, 1);
                li = (lane < pos) ? li : (lane == pos ? ck : up);
                if (lane >= K) li = ~0ull;
                kth = readlane_u64(li, K - 1);
            }
        }
    }
    if (lane < K) kp[lane] = li;
}

template <int D> void launch_leaf_scan_d(const ScanArgs &a, int K, int sparse, hipStream_t s);

}  // namespace bkd
