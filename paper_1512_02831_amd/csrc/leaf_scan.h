// leaf_scan.h -- ProcessAllBuffers leaf scan (Section 2.4, Section 3.2), gfx950.
//
// Dense leaves (many buffered queries): one workgroup of 256 lanes takes one
// work item, up to 256 buffered queries of one leaf; lane i owns query i (its
// coordinates and its K best keys as a sorted register list).  The leaf's
// points (the part held by the current chunk) stream through LDS in tiles.
//
// Matrix-core filter.  Once every query of a wave has K candidates, a pair is
// first tested in the leaf's own frame: centred coordinates (relative to the
// leaf's bounding-box centre c, rounded to float32) times the leaf's scale s,
// a power of two that brings every centred point coordinate into [-1, 1], so
// u = fl32(x - c) s and p = fl32(q - c) s exactly.  Both are rounded to
// float16 (x~, q~), and G = <q~,x~> - |x~|^2/2 is formed on the matrix cores
// from d + 2 products (the norm term as a float16 hi and lo part against a
// one), one v_mfma_f32_32x32x16_f16 per step of sixteen and 32x32 tile (one
// step at d <= 14).  The vector unit then takes half a max per pair.  The
// rounding moves the scaled distance by at most
// delta = 2^-10 (1 + 2^-8)(|p| + sqrt d) + 2^-13 sqrt d (either rounding
// mode, float16 subnormals kept or flushed), so a pair whose float32 distance
// is within the query's K-th, thr, has |q~ - x~|^2 <= T = (sqrt(thr s^2) +
// delta)^2, and it passes G >= (|q~|^2 - T)/2 - 2^-18 (|q~|^2 + d + 1) - eta;
// the 2^-18 term covers the float32 accumulations (products of float16 are
// exact), eta = 2^-100 underflow; the square root in T is the hardware's
// (within 2^-21 relative, flushed below 2^-126), covered by delta's 1 + 2^-8.
// The band is relative to the leaf, not to |q'|^2 + |x'|^2: a query at
// distance r from the leaf centre moves its radius by about
// delta ~ 2^-10 (r + sqrt d) leaf radii.  A query with a scaled
// offset beyond 2^14 (far outside its leaf, or a leaf of tiny extent) takes
// the exact path.  Passing pairs go to the lane owning the query, which
// re-checks them with the exact float32 distance, so keys and results are
// bit-identical to the exact path.  A wave holding a query whose list is not
// full yet (a first visit) takes the exact path, every point through the
// float32 distance, 32 points at a time until all its lists are full.
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

#include "internal.h"
#include "traverse.h"

namespace bkd {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_PT = 256;  // points per LDS tile
constexpr int ROUTE_LDS_SPLITS = 1023;  // split values of the top ten levels, staged for the routing walk

// Insert key c into the sorted list: every entry above c moves down one place
// (the last one drops out) and c takes the first vacated place.
template <int K> __device__ inline void key_insert(uint64_t (&lst)[K], uint64_t c)
{
    bool lt[K];
#pragma unroll
    for (int s = 0; s < K; s++) lt[s] = c < lst[s];
#pragma unroll
    for (int s = K - 1; s > 0; s--) lst[s] = lt[s - 1] ? lst[s - 1] : (lt[s] ? c : lst[s]);
    lst[0] = lt[0] ? c : lst[0];
}

__device__ inline int xcd_item(int b, int count)
{
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous eighth of the count items so that a leaf's tiles share one
    // L2.  -1: a workgroup past the items (the grid may be an upper bound).
    const int per = (count + 7) >> 3;
    const int j = b >> 3;
    return j < per ? (b & 7) * per + j : -1;
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Absolute slack of the matrix-core filter (underflow of its float32 terms).
constexpr float FILTER_ABS_SLACK = 0x1p-100f;
// Scaled query offsets beyond this take the exact path (float16 range and band).
constexpr float FILTER_FAR = 0x1p14f;

// Two float32 values rounded to float16 in one word: a in the low half, b in
// the high half.
__device__ inline uint32_t pack_f16x2(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}
__device__ inline float f16_word_lo(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)); }
__device__ inline float f16_word_hi(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)); }

template <int D, int K>
__global__ __launch_bounds__(SCAN_THREADS, 4) void k_leaf_scan(ScanArgs a)
{
    constexpr int DS = (D + 3) & ~3;   // row of the exact copy, padded for float4 reads
    // Products of the filter's inner product, in operand order: x~_j q~_j for
    // every coordinate, then the two float16 parts of -|x~|^2/2 against 1.
    constexpr int NT = D + 2;
    constexpr int NS = (NT + 15) / 16;  // matrix-core steps of sixteen products
    constexpr int PT = D > 16 ? SCAN_PT / 2 : SCAN_PT;  // points per LDS tile
    constexpr int NB = PT / 32;        // 32-point blocks per tile
    __shared__ float4 xs[PT * DS / 4];  // original coordinates, point-major (exact distances)
    // point operands of the filter ([block][step][lane], 16 bytes per lane:
    // every read and write is one contiguous kilobyte)
    __shared__ f16x8 xa[NB * NS * 64];
    __shared__ int32_t os[PT];
    __shared__ float route_splits[ROUTE_LDS_SPLITS];

    // with dev_counts the item count is read on the device (the grid only bounds it)
    const int item_count = a.dev_counts ? a.dev_counts[CTL_T] : a.item_count;
    int item = xcd_item(blockIdx.x, item_count);
    if (item < 0 || item >= item_count) return;
    item += a.item_first;

    // leaf of the item: largest L in [leaf_first, leaf_last] with tiles[L] <= item
    int lo = a.leaf_first, hi = a.leaf_last;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.tiles[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    const int L = lo;
    const int qbase = a.off[L] + (item - a.tiles[L]) * SCAN_QT;
    const int qcnt = min(SCAN_QT, a.off[L + 1] - qbase);
    const int64_t l0 = a.leaf_off[L];
    const int len = a.leaf_off[L + 1] - a.leaf_off[L];
    const int64_t p0 = max(l0, a.chunk_lo);
    const int64_t p1 = min(l0 + len, a.chunk_hi);
    const float *X = a.base + (a.blk[L] + a.blk_shift);
    const int32_t *orig = reinterpret_cast<const int32_t *>(X) + (int64_t)a.d * len;
    const float *cen = a.centers + (int64_t)L * a.d;
    const float sc = a.scales[L];  // power of two: exact scaling

    const int tid = threadIdx.x;
    const int lane = tid & 63, half = lane >> 5, col = lane & 31;
    const bool act = tid < qcnt;
    const int32_t q = act ? a.bufq[qbase + tid] : 0;
    // qs: the scaled centred query p; Qn = |q~|^2 of its float16 rounding; Pn = |p|^2
    float qv[D], qs[D], Qn = 0.0f, Pn = 0.0f;
    bool far = false;
#pragma unroll
    for (int j = 0; j < D; j++) {
        qv[j] = (act && j < a.d) ? a.Q[(int64_t)q * a.d + j] : 0.0f;
        qs[j] = (act && j < a.d) ? (qv[j] - cen[j]) * sc : 0.0f;
        far |= !(fabsf(qs[j]) <= FILTER_FAR);
        const float r = (float)(_Float16)qs[j];
        Qn = fmaf(r, r, Qn);
        Pn = fmaf(qs[j], qs[j], Pn);
    }
    const float sqd = sqrtf((float)a.d);
    const float delta = 0x1.01p-10f * (sqrtf(Pn) + sqd) + 0x1p-13f * sqd;
    uint64_t lst[K];
#pragma unroll
    for (int s2 = 0; s2 < K; s2++) lst[s2] = act ? a.keys[(int64_t)q * K + s2] : 0ull;  // 0: nothing enters
    float thr = __uint_as_float((uint32_t)(lst[K - 1] >> 32));
    // filter threshold of this lane's query: a pair passes when G >= aq
    // (the hardware square root here: its error, at most 2^-21 relative and a
    // flush below 2^-126, is covered by the factor 1 + 2^-8 in delta)
    auto own_aq = [&]() {
        if (!act) return INFINITY;
        const float r = __builtin_amdgcn_sqrtf(thr * sc * sc) + delta;
        const float v = 0.5f * (Qn - r * r) - 0x1p-18f * (Qn + (float)(a.d + 1)) - FILTER_ABS_SLACK;
        return v == 0.0f ? -0x1p-149f : v;  // never zero: the mask test below reads a sign
    };

    const bool wave_busy = (tid & ~63) < qcnt;
    // A wave with a query whose list is not full yet (K-th key EMPTY, first
    // visit) accepts every point: it takes the exact path, 32 points at a time,
    // until every list is full, then the filter.  Coordinates beyond the
    // filter's range keep every wave on the exact path.
    const bool no_filter = a.exact_only || (a.wide_flag && *a.wide_flag);
    bool exact_wave = no_filter || __any(act && (isinf(thr) || far));

    // Matrix-core operands of the filter.  The wave's 64 queries form two
    // column tiles of 32; lane l supplies the query part of products
    // 16 s + 8 (l / 32) .. + 7 of step s for query (32 t + l % 32), and holds
    // that query's threshold.
    f16x8 qb[2][NS];
    float aq[2];
#pragma unroll
    for (int t = 0; t < 2; t++) {
        const int src = 32 * t + col;
        _Float16 g[D];
#pragma unroll
        for (int j = 0; j < D; j++) g[j] = (_Float16)__shfl(qs[j], src);
        auto part = [&](int u) -> _Float16 {  // query factor of product u
            if (u < D) return g[u];
            return (_Float16)(u < NT ? 1.0f : 0.0f);
        };
#pragma unroll
        for (int s2 = 0; s2 < NS; s2++) {
#pragma unroll
            for (int e = 0; e < 8; e++) qb[t][s2][e] = half ? part(16 * s2 + 8 + e) : part(16 * s2 + e);
        }
    }
    {
        const float o = own_aq();
        aq[0] = __shfl(o, col);
        aq[1] = __shfl(o, 32 + col);
    }

    auto exact_points = [&](int i0, int i1) {
#pragma unroll 2
        for (int i = i0; i < i1; i++) {
            const float4 *xp = xs + i * (DS / 4);
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < DS / 4; c++) {
                float4 x4 = xp[c];
                float xe[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (4 * c + e < D) {
                        float t = qv[4 * c + e] - xe[e];
                        acc = fmaf(t, t, acc);
                    }
                }
            }
            uint64_t key = ((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)os[i];
            if (key < lst[K - 1]) key_insert<K>(lst, key);
        }
    };

    // One 32-point block against the wave's 64 queries.  The accumulator
    // register r of lane l holds point 32 b + (r % 4) + 8 (r / 4) + 4 (l / 32)
    // against query (32 t + l % 32).
    auto filter_block = [&](int b, int np, const f16x8 *avs) {
        f32x16 c0 = {}, c1 = {};
#pragma unroll
        for (int s2 = 0; s2 < NS; s2++) {
            const f16x8 av = avs[s2];
            c0 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, qb[0][s2], c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, qb[1][s2], c1, 0, 0, 0);
        }
        float m0 = -INFINITY, m1 = -INFINITY;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            m0 = fmaxf(m0, c0[r]);
            m1 = fmaxf(m1, c1[r]);
        }
        if (!__any(m0 >= aq[0] || m1 >= aq[1])) return;
        // Some pair passed: hand each passing (point, query) to the lane that
        // owns the query (lane 32 t + j for column j of tile t), which
        // re-checks it with the exact float32 distance.  Bit r of a tile's
        // mask is accumulator register r (masks are built only for a tile that
        // has a passing pair): the sign of G - aq, shifted in by alignbit, is
        // clear exactly when G >= aq, since aq is never zero and float32
        // subtraction keeps subnormals (x - y is +0 only for x == y, and -0
        // never arises with y != 0).  The owner of tile t (lanes with l / 32 = t)
        // gets its partner's mask of the same column (lane l ^ 32), and bit
        // 16 h + r of the merged mask is point (r % 4) + 8 (r / 4) + 4 h.
        uint32_t f0 = 0, f1 = 0;
        if (__any(m0 >= aq[0])) {
            uint32_t nf = 0;
#pragma unroll
            for (int r = 15; r >= 0; r--) nf = __builtin_amdgcn_alignbit(nf, __float_as_uint(c0[r] - aq[0]), 31);
            f0 = ~nf & 0xffffu;
        }
        if (__any(m1 >= aq[1])) {
            uint32_t nf = 0;
#pragma unroll
            for (int r = 15; r >= 0; r--) nf = __builtin_amdgcn_alignbit(nf, __float_as_uint(c1[r] - aq[1]), 31);
            f1 = ~nf & 0xffffu;
        }
        const uint32_t recv = __shfl_xor(half ? f0 : f1, 32);
        uint32_t msk = half ? (recv | (f1 << 16)) : (f0 | (recv << 16));
        bool changed = false;
        while (msk) {
            const int i = __builtin_ctz(msk);
            msk &= msk - 1;
            const int p = 32 * b + (i & 3) + 8 * ((i >> 2) & 3) + 4 * (i >> 4);
            if (p >= np) continue;
            const float4 *xp = xs + p * (DS / 4);
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < DS / 4; c++) {
                float4 x4 = xp[c];
                float xe[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (4 * c + e < D) {
                        float t = qv[4 * c + e] - xe[e];
                        acc = fmaf(t, t, acc);
                    }
                }
            }
            const uint64_t key = ((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)os[p];
            if (key < lst[K - 1]) {
                key_insert<K>(lst, key);
                changed = true;
            }
        }
        if (__any(changed)) {
            thr = __uint_as_float((uint32_t)(lst[K - 1] >> 32));
            const float o = own_aq();
            aq[0] = __shfl(o, col);
            aq[1] = __shfl(o, 32 + col);
        }
    };

    // Staging: thread t brings point t of a tile; the next tile's coordinates
    // are loaded into registers while the current tile is scanned.
    const int first_pt = (int)(p0 - l0);  // a valid point of this item (clamped loads stay in the chunk)
    float pre[DS], cr[DS];
    int32_t pre_o = 0;
#pragma unroll
    for (int j = 0; j < DS; j++) cr[j] = (j < a.d) ? cen[j] : 0.0f;
    // A column base (uniform, 64-bit) plus one 32-bit byte offset per thread: the
    // loads take the scalar-base form, so the scan below never has to wait for
    // them before reusing an address register.  The offset 4 i stays below 2^32
    // because leaves of 2^30 points and more never reach this kernel (the host
    // scans them with the sparse and tail kernels).
    auto at = [](const void *base, uint32_t bo) {
        return reinterpret_cast<const char *>(base) + bo;
    };
    auto load_tile = [&](int64_t pt) {
        if (PT < SCAN_THREADS && tid >= PT) return;
        const int np = (int)min((int64_t)PT, p1 - pt);
        // rows past the tile load a valid point of the item; they are never read as points
        const int i = tid < np ? (int)(pt - l0) + tid : first_pt;
        if (a.d == D) {
            const uint32_t bo = (uint32_t)i * 4u;
#pragma unroll
            for (int j = 0; j < DS; j++)
                pre[j] = (j < D) ? *reinterpret_cast<const float *>(at(X + (int64_t)(j < D ? j : 0) * len, bo)) : 0.0f;
        } else {
            // a padded dimension: the plain indexed form (a common form for both branches
            // made the compiler give up the scalar-base loads above, 7% slower)
#pragma unroll
            for (int j = 0; j < DS; j++) {
                const float x = X[(int64_t)(j < a.d ? j : 0) * len + i];
                pre[j] = (j < a.d) ? x : 0.0f;
            }
        }
        pre_o = *reinterpret_cast<const int32_t *>(at(orig, (uint32_t)i * 4u));
    };
    // Every load issued so far (the query, its list) is complete here: without this
    // the compiler keeps a wait for them inside the re-check path, which then also
    // waits for the next tile's loads.
    __builtin_amdgcn_s_waitcnt(0);
    load_tile(p0);
    for (int64_t pt = p0; pt < p1; pt += PT) {
        const int np = (int)min((int64_t)PT, p1 - pt);
        const int npad = (np + 31) & ~31;
        __syncthreads();
        if (tid < npad) {
            const bool live = tid < np;
            float *ro = reinterpret_cast<float *>(xs) + tid * DS;
            const int ra = (tid >> 5) * NS * 64 + (tid & 31);
            // scaled centred coordinates (zero past d) rounded to float16, two to a word,
            // and |x~|^2 of the rounded values
            constexpr int DP = (D + 1) / 2;
            uint32_t H[DP];
            float Xn = 0.0f;
#pragma unroll
            for (int w = 0; w < DP; w++) {
                const int j0 = 2 * w, j1 = 2 * w + 1;
                const float u0 = (j0 < D) ? (pre[j0 < D ? j0 : 0] - cr[j0 < D ? j0 : 0]) * sc : 0.0f;
                const float u1 = (j1 < D) ? (pre[j1 < D ? j1 : 0] - cr[j1 < D ? j1 : 0]) * sc : 0.0f;
                H[w] = pack_f16x2(u0, u1);
                const float r0 = f16_word_lo(H[w]), r1 = f16_word_hi(H[w]);
                Xn = fmaf(r0, r0, Xn);
                Xn = fmaf(r1, r1, Xn);
            }
#pragma unroll
            for (int c4 = 0; c4 < DS / 4; c4++)
                reinterpret_cast<float4 *>(ro)[c4] = make_float4(pre[4 * c4], pre[4 * c4 + 1], pre[4 * c4 + 2], pre[4 * c4 + 3]);
            // -|x~|^2/2 as float16 hi + lo; padding rows take the most negative float16 in
            // both parts and never pass
            const float nb = -0.5f * Xn;
            const uint32_t t0 = pack_f16x2(nb, 0.0f);
            const uint32_t NBw = live ? pack_f16x2(nb, nb - f16_word_lo(t0)) : 0xfbfffbffu;
            auto part = [&](int u) -> uint32_t {  // point factor of product u, in the low 16 bits
                if (u < D) return (H[u >> 1] >> (16 * (u & 1))) & 0xffffu;
                if (u == D) return NBw & 0xffffu;
                if (u == D + 1) return NBw >> 16;
                return 0u;
            };
            auto word = [&](int w) -> uint32_t { return part(2 * w) | (part(2 * w + 1) << 16); };
            // products 16 s + 8 h .. + 7 of the point go to lane slot (tid % 32) + 32 h of step s
#pragma unroll
            for (int s2 = 0; s2 < NS; s2++) {
#pragma unroll
                for (int h2 = 0; h2 < 2; h2++) {
                    const int w0 = 8 * s2 + 4 * h2;
                    reinterpret_cast<uint4 *>(xa)[ra + s2 * 64 + 32 * h2] =
                        make_uint4(word(w0), word(w0 + 1), word(w0 + 2), word(w0 + 3));
                }
            }
            os[tid] = pre_o;
        }
        __syncthreads();
        if (pt + PT < p1) load_tile(pt + PT);
        if (!wave_busy) continue;  // whole wave without queries: only helps staging
        // the point operand of block b + 1 is read from LDS while block b is filtered
        const int nbl = npad / 32;
        f16x8 avn[NS];
        auto fetch_operand = [&](int b) {
            const int bn = min(b, nbl - 1);
#pragma unroll
            for (int s2 = 0; s2 < NS; s2++) avn[s2] = xa[(bn * NS + s2) * 64 + lane];
        };
        fetch_operand(0);
        for (int b = 0; b < nbl; b++) {
            if (!exact_wave) {
                f16x8 av[NS];
#pragma unroll
                for (int s2 = 0; s2 < NS; s2++) av[s2] = avn[s2];
                fetch_operand(b + 1);
                filter_block(b, np, av);
                continue;
            }
            exact_points(32 * b, min(32 * b + 32, np));
            thr = __uint_as_float((uint32_t)(lst[K - 1] >> 32));
            exact_wave = no_filter || __any(act && (isinf(thr) || far));
            if (!exact_wave) {
                fetch_operand(b + 1);
                const float o = own_aq();
                aq[0] = __shfl(o, col);
                aq[1] = __shfl(o, 32 + col);
            }
        }
    }
    uint32_t kb = 0;
    if (act) {
        const int kk = a.kq ? a.kq[q] : a.k;
#pragma unroll
        for (int s2 = 0; s2 < K; s2++) {
            a.keys[(int64_t)q * K + s2] = lst[s2];
            if (s2 == kk - 1) kb = (uint32_t)(lst[s2] >> 32);
        }
        a.kth[q] = kb;
    }
    if (a.route_leaf) {
        // next leaf of every query of the item (the FindLeafBatch step of the next round),
        // walked from LDS: the split values of the top levels and, in place of the point
        // tile, the lanes' query coordinates (coordinate-major)
        constexpr bool QL = SCAN_THREADS * D <= PT * DS;
        float *qlds = reinterpret_cast<float *>(xs);
        const int lds_nodes = min((1 << a.h) - 1, ROUTE_LDS_SPLITS);
        __syncthreads();  // every wave is done with the tile
        if constexpr (QL) {
#pragma unroll
            for (int j = 0; j < D; j++) qlds[j * SCAN_THREADS + tid] = qv[j];
        }
        for (int i = tid; i < lds_nodes; i += SCAN_THREADS) route_splits[i] = a.split[i];
        __syncthreads();
        if (act) {
            const int32_t first = (1 << a.h) - 1;
            // (only trees with the original rules route here: a variant tree's rounds route with
            // FindLeafBatch, which keeps this kernel's code and registers as they are)
            const int32_t v = QL ? next_leaf(first + L, qlds + tid, &kb, a.split, route_splits, lds_nodes, a.h, a.d,
                                             SCAN_THREADS)
                                 : next_leaf(first + L, a.Q + (int64_t)q * a.d, &kb, a.split, route_splits,
                                             lds_nodes, a.h, a.d);
            a.node[q] = v;
            a.route_leaf[qbase + tid] = v >= 0 ? (uint32_t)(v - first) : (uint32_t)(1 << a.h);
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
    constexpr int WPB = SCAN_THREADS / 64;
    const int blk = xcd_item(blockIdx.x, (a.sitem_count + WPB - 1) / WPB);
    if (blk < 0) return;
    int s = __builtin_amdgcn_readfirstlane(blk * WPB + (int)(threadIdx.x >> 6));
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
    // Four batches of 64 points per iteration: all their loads are issued before
    // the first distance, so a query's walk over the leaf waits on memory a
    // quarter as often.  Lanes past the end load a valid point and discard it.
    constexpr int U = 4;
    const int i_first = (int)(p0 - l0);
    for (int64_t pb = p0; pb < p1; pb += 64 * U) {
        float x[U][D];
        int32_t o[U];
        bool valid[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t p = pb + 64 * u + lane;
            valid[u] = p < p1;
            const int i = valid[u] ? (int)(p - l0) : i_first;
#pragma unroll
            for (int j = 0; j < D; j++) x[u][j] = X[(int64_t)(j < a.d ? j : 0) * len + i];
            o[u] = orig[i];
        }
        uint64_t key[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            float acc = 0.0f;
#pragma unroll
            for (int j = 0; j < D; j++) {
                const float t = qv[j] - ((j < a.d) ? x[u][j] : 0.0f);
                acc = fmaf(t, t, acc);
            }
            key[u] = valid[u] ? (((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)o[u]) : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            uint64_t cand = __ballot(key[u] < kth);
            while (cand) {
                const int c = __ffsll((unsigned long long)cand) - 1;
                cand &= cand - 1;
                const uint64_t ck = readlane_u64(key[u], c);
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
    }
    if (lane < K) kp[lane] = li;
    const int kk = a.kq ? a.kq[q] : a.k;
    if (lane == kk - 1) a.kth[q] = (uint32_t)(li >> 32);
    if (a.route_leaf) {
        // next leaf of the query (the FindLeafBatch step of the next round), walked by every lane alike
        const uint32_t kb = (uint32_t)(readlane_u64(li, kk - 1) >> 32);
        const int32_t first = (1 << a.h) - 1;
        const int32_t v = (a.dims || a.boxes) ? next_leaf_rules(first + L, qp, &kb, a.split, a.dims, a.boxes, a.h, a.d)
                                              : next_leaf(first + L, qp, &kb, a.split, a.split, 0, a.h, a.d);
        if (lane == 0) {
            a.node[q] = v;
            a.route_leaf[a.off[L] + (s - a.sparse[L])] = v >= 0 ? (uint32_t)(v - first) : (uint32_t)(1 << a.h);
        }
    }
}

// Tail of the lock-step schedule.  When only a few queries are pending, a
// round costs a dozen launches for little work, and the late rounds are
// spent on a handful of queries with long traversals.  Here each pending
// query finishes its whole traversal in one workgroup of four waves: the
// waves split each leaf's points, keep their new candidates (keys below the
// query's K-th) as lane-distributed lists, and merge them into the query's
// list in LDS order; then every lane walks to the next leaf with the same
// state (Sections 2.3, 2.4), so the walk is uniform.  Results do not depend
// on the schedule: a query's visits and its list are its own.  With
// route_leaf set (a streamed structure), only the leaves [leaf_first,
// leaf_last] of the resident chunk are available: a query stops at its first
// next leaf outside them and leaves that leaf (2^h when done) in its entry.
// TT lanes per entry: 256, or 512 for leaves of 2048 points and more, where
// twice the loads in flight per leaf visit pay for the wider merge.
constexpr int TAIL_THREADS = 256;
constexpr int TAIL_THREADS_WIDE = 512;
constexpr int TAIL_LDS_SPLITS = 2047;

template <int K> __device__ inline void lane_list_insert(uint64_t &li, uint64_t ck, int lane)
{
    const uint64_t moved = __ballot(li > ck);  // entries at and after the insertion rank
    const int pos = __ffsll((unsigned long long)moved) - 1;
    const uint64_t up = __shfl_up(li, 1);
    li = (lane < pos) ? li : (lane == pos ? ck : up);
    if (lane >= K) li = ~0ull;
}

template <int D, int K, int TT> __global__ __launch_bounds__(TT) void k_tail(ScanArgs a)
{
    constexpr int W = TT / 64;
    constexpr int U = 4;
    __shared__ float split_lds[TAIL_LDS_SPLITS];
    __shared__ uint64_t cand[W][K];
    __shared__ float q_lds[D];  // the query, read by every step of the walk
    const int h = a.h;
    const int lds_nodes = min((1 << h) - 1, TAIL_LDS_SPLITS);
    for (int i = threadIdx.x; i < lds_nodes; i += TT) split_lds[i] = a.split[i];

    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t q = a.tail_q[blockIdx.x];
    int32_t leaf = a.tail_from_node ? a.node[q] - ((1 << a.h) - 1) : (int32_t)a.tail_leaf[blockIdx.x];
    const float *qp = a.Q + (int64_t)q * a.d;
    if (threadIdx.x < D) q_lds[threadIdx.x] = (threadIdx.x < a.d) ? qp[threadIdx.x] : 0.0f;
    __syncthreads();
    float qv[D];
#pragma unroll
    for (int j = 0; j < D; j++) qv[j] = (j < a.d) ? qp[j] : 0.0f;
    uint64_t *kp = a.keys + (int64_t)q * K;
    uint64_t li = (lane < K) ? kp[lane] : ~0ull;  // the query's list, lane i holds the i-th smallest
    const int kk = a.kq ? a.kq[q] : a.k;
    const int32_t first = (1 << h) - 1;
    long long visits = 0, pairs = 0, visits_seen = 0;
    int32_t next = NODE_DONE;
    for (;;) {
        const int64_t l0 = a.leaf_off[leaf];
        const int len = a.leaf_off[leaf + 1] - (int32_t)l0;
        const float *X = a.base + (a.blk[leaf] + a.blk_shift);
        const int32_t *orig = reinterpret_cast<const int32_t *>(X) + (int64_t)a.d * len;
        const uint64_t kthK = readlane_u64(li, K - 1);
        // this wave's part of the leaf; its new candidates all lie below kthK
        const int part = (len + W - 1) / W;
        const int lo = min(len, w * part), hi = min(len, lo + part);
        uint64_t ni = ~0ull, nth = kthK;
        for (int pb = lo; pb < hi; pb += 64 * U) {
            float x[U][D];
            int32_t o[U];
            bool valid[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int p = pb + 64 * u + lane;
                valid[u] = p < hi;
                const int i = valid[u] ? p : lo;
#pragma unroll
                for (int j = 0; j < D; j++) x[u][j] = X[(int64_t)(j < a.d ? j : 0) * len + i];
                o[u] = orig[i];
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                float acc = 0.0f;
#pragma unroll
                for (int j = 0; j < D; j++) {
                    const float t = qv[j] - ((j < a.d) ? x[u][j] : 0.0f);
                    acc = fmaf(t, t, acc);
                }
                const uint64_t key = valid[u] ? (((uint64_t)__float_as_uint(acc) << 32) | (uint32_t)o[u]) : ~0ull;
                uint64_t cb = __ballot(key < nth);
                while (cb) {
                    const int c = __ffsll((unsigned long long)cb) - 1;
                    cb &= cb - 1;
                    const uint64_t ck = readlane_u64(key, c);
                    if (ck < nth) {
                        lane_list_insert<K>(ni, ck, lane);
                        const uint64_t nk = readlane_u64(ni, K - 1);
                        nth = nk < kthK ? nk : kthK;
                    }
                }
            }
        }
        if (lane < K) cand[w][lane] = ni;
        __syncthreads();
        // every wave merges the candidate lists in the same order, so all copies agree
#pragma unroll
        for (int w2 = 0; w2 < W; w2++) {
            const uint64_t cl = (lane < K) ? cand[w2][lane] : ~0ull;
            uint64_t cb = __ballot(cl < readlane_u64(li, K - 1));
            while (cb) {
                const int c = __ffsll((unsigned long long)cb) - 1;
                cb &= cb - 1;
                const uint64_t ck = readlane_u64(cl, c);
                if (ck < readlane_u64(li, K - 1)) lane_list_insert<K>(li, ck, lane);
            }
        }
        __syncthreads();  // cand is written again for the next leaf
        if (!(a.tail_counted && visits_seen == 0)) {
            visits++;
            pairs += len;
        }
        visits_seen++;
        const uint64_t kth_key = readlane_u64(li, kk - 1);
        const int32_t v = (a.dims || a.boxes)
                              ? next_leaf_rules(first + leaf, q_lds, &kth_key, a.split, a.dims, a.boxes, h, a.d)
                              : next_leaf(first + leaf, q_lds, &kth_key, a.split, split_lds, lds_nodes, h, a.d);
        if (v == NODE_DONE) break;
        leaf = v - first;
        if (a.route_leaf && (leaf < a.leaf_first || leaf > a.leaf_last)) {
            next = v;  // not resident: the query waits for that leaf's chunk
            break;
        }
    }
    if (w == 0 && lane < K) kp[lane] = li;
    if (w == 0 && lane == (a.kq ? a.kq[q] : a.k) - 1) a.kth[q] = (uint32_t)(li >> 32);
    if (threadIdx.x == 0) {
        a.node[q] = next;
        if (a.route_leaf) a.route_leaf[blockIdx.x] = next >= 0 ? (uint32_t)(next - first) : (uint32_t)(1 << h);
        if (a.req_left && next == NODE_DONE) {
            // last query of its request: record the request as complete
            const int32_t r = a.req_of[q];
            if (atomicSub(&a.req_left[r], 1) == 1) a.done_list[1 + atomicAdd(&a.done_list[0], 1)] = r;
        }
        atomicAdd((unsigned long long *)(a.ctl + CTL_VISITS_LO), (unsigned long long)visits);
        atomicAdd((unsigned long long *)(a.ctl + CTL_SPAIRS_LO), (unsigned long long)pairs);
        // each tail visit reads its leaf for one query: its points count as leaf reads
        atomicAdd((unsigned long long *)(a.ctl + CTL_LPS_LO), (unsigned long long)pairs);
    }
}

template <int D> void launch_leaf_scan_d(const ScanArgs &a, int K, int sparse, hipStream_t s);

}  // namespace bkd
