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

}  // namespace bkd
