// traverse.h -- FindLeafBatch for one query on the device (Sections 2.3, 2.4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bkd {

constexpr int32_t NODE_FRESH = -2;
constexpr int32_t NODE_DONE = -1;
constexpr uint64_t EMPTY_KEY = 0x7F800000FFFFFFFFull;

// Next leaf (heap index) of a query, or NODE_DONE.  State: FRESH, DONE or the
// heap index of the last leaf visited.  A fresh query descends from the root:
// left iff q[dim] < split.  After a visit the walk goes back up; at a parent
// reached from its near child the far child is entered when the float32
// plane term (q[dim]-s)^2 does not exceed the current k-th squared distance
// (read through kth: the high word of a key, or those bits alone), and the
// walk descends from there to its nearest leaf; reaching the root from above
// ends the traversal.
//
// Every loop iteration is one step, up or down, reading one split value and
// one query coordinate, so that the lanes of a wave advance together whatever
// the level at which each turns around.  Splits of heap nodes below
// lds_nodes are read from split_lds (a copy in LDS), the others from split;
// coordinate j of the query is qp[j * qstride].
__device__ inline float kth_value(const uint64_t *key) { return __uint_as_float((uint32_t)(*key >> 32)); }
__device__ inline float kth_value(const uint32_t *bits) { return __uint_as_float(*bits); }

template <typename KthPtr>
__device__ inline int32_t next_leaf(int32_t st, const float *qp, KthPtr kth_ptr, const float *split,
                                    const float *split_lds, int lds_nodes, int h, int d, int qstride = 1)
{
    if (st == NODE_DONE) return NODE_DONE;
    int32_t node, from = -1;
    int lvl, dim;
    bool down;
    float kth = 0.0f;
    if (st == NODE_FRESH) {
        if (h == 0) return 0;  // the root is the only leaf
        node = 0;
        lvl = 0;
        dim = 0;
        down = true;
    } else {
        if (st == 0) return NODE_DONE;
        kth = kth_value(kth_ptr);
        from = st;
        node = (st - 1) >> 1;
        lvl = h - 1;
        dim = (h - 1) % d;
        down = false;
    }
    for (;;) {
        const float s = node < lds_nodes ? split_lds[node] : split[node];
        const float qd = qp[dim * qstride];
        const int32_t left = 2 * node + 1;
        const int32_t nearc = (qd < s) ? left : left + 1;
        if (down) {
            if (lvl + 1 == h) return nearc;
            node = nearc;
        } else {
            const float t = qd - s;
            if (from == nearc && t * t <= kth) {
                const int32_t farc = (nearc == left) ? left + 1 : left;
                if (lvl + 1 == h) return farc;
                node = farc;
                down = true;
            } else {
                if (node == 0) return NODE_DONE;
                from = node;
                node = (node - 1) >> 1;
                lvl--;
                dim = (dim == 0) ? d - 1 : dim - 1;
                continue;
            }
        }
        lvl++;
        dim = (dim + 1 == d) ? 0 : dim + 1;
    }
}

// Box term of query q against a box b (minima b[0..d), maxima b[d..2d)): g_j = the
// distance of q_j to [min_j, max_j] (0 inside), rounded to float32, accumulated as the
// distance is, acc = fma(g_j, g_j, acc) from +0.  For every point x in the box
// |fl32(q_j - x_j)| >= g_j, and rounding is monotone, so the term never exceeds the
// float32 squared distance of x: a subtree whose box term exceeds the k-th distance
// holds no closer point.
__device__ inline float box_term(const float *qp, int qstride, const float *b, int d)
{
    float acc = 0.0f;
    for (int j = 0; j < d; j++) {
        const float q = qp[j * qstride], lo = b[j], hi = b[d + j];
        const float g = q < lo ? lo - q : (q > hi ? q - hi : 0.0f);
        acc = fmaf(g, g, acc);
    }
    return acc;
}

// next_leaf for a variant tree (Section 2.3): node v splits dimension dims[v] (null:
// level mod d), and the far child is entered when its box term (boxes: 2d floats per
// heap node, null: the plane term of the split) does not exceed the current k-th
// squared distance.  Same walk and states as next_leaf, read from global memory.
template <typename KthPtr>
__device__ inline int32_t next_leaf_rules(int32_t st, const float *qp, KthPtr kth_ptr, const float *split,
                                          const uint8_t *dims, const float *boxes, int h, int d, int qstride = 1)
{
    if (st == NODE_DONE) return NODE_DONE;
    const int32_t first = (1 << h) - 1;
    auto dim_of = [&](int32_t v, int lvl) { return dims ? (int)dims[v] : lvl % d; };
    auto descend = [&](int32_t v, int lvl) {
        while (v < first) {
            const int dm = dim_of(v, lvl);
            v = (qp[dm * qstride] < split[v]) ? 2 * v + 1 : 2 * v + 2;
            lvl++;
        }
        return v;
    };
    if (st == NODE_FRESH) return descend(0, 0);
    if (st == 0) return NODE_DONE;
    const float kth = kth_value(kth_ptr);
    int32_t u = st;
    int lvl = h;  // level of u
    while (u != 0) {
        const int32_t p = (u - 1) >> 1;
        lvl--;
        const int dm = dim_of(p, lvl);
        const float qd = qp[dm * qstride], s = split[p];
        const int32_t left = 2 * p + 1;
        const int32_t nearc = (qd < s) ? left : left + 1;
        if (u == nearc) {
            const int32_t farc = (nearc == left) ? left + 1 : left;
            float bound;
            if (boxes) {
                bound = box_term(qp, qstride, boxes + (int64_t)farc * 2 * d, d);
            } else {
                const float t = qd - s;
                bound = t * t;
            }
            if (bound <= kth) return descend(farc, lvl + 1);
        }
        u = p;
    }
    return NODE_DONE;
}

}  // namespace bkd
