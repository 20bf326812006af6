// traverse.h -- FindLeafBatch for one query on the device (Sections 2.3, 2.4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bkd {

constexpr int32_t NODE_FRESH = -2;
constexpr int32_t NODE_DONE = -1;
constexpr uint64_t EMPTY_KEY = 0x7F800000FFFFFFFFull;

// Descend from heap node v at the given level to a leaf: left iff q[dim] < split.
__device__ inline int32_t descend(const float *q, const float *split, int32_t v, int level, int h, int d)
{
    int dim = level % d;
    while (level < h) {
        v = (q[dim] < split[v]) ? 2 * v + 1 : 2 * v + 2;
        level++;
        dim = (dim + 1 == d) ? 0 : dim + 1;
    }
    return v;
}

// Next leaf (heap index) of a query, or NODE_DONE.  State: FRESH, DONE or the
// heap index of the last leaf visited.  After a visit the walk goes back up;
// at a parent reached from its near child the far child is entered when the
// float32 plane term (q[dim]-s)^2 does not exceed the current k-th squared
// distance (the high word of *kth_key); reaching the root from above ends
// the traversal.
__device__ inline int32_t next_leaf(int32_t st, const float *qp, const uint64_t *kth_key, const float *split, int h,
                                    int d)
{
    if (st == NODE_FRESH) return descend(qp, split, 0, 0, h, d);
    if (st == NODE_DONE) return NODE_DONE;
    const float kth = __uint_as_float((uint32_t)(*kth_key >> 32));
    int32_t u = st;
    int level = h;
    int dim = h % d;  // split dimension of the level, tracked on the way up
    while (u != 0) {
        const int32_t p = (u - 1) >> 1;
        level--;
        dim = (dim == 0) ? d - 1 : dim - 1;
        const float s = split[p];
        const float qd = qp[dim];
        const int32_t nearc = (qd < s) ? 2 * p + 1 : 2 * p + 2;
        if (u == nearc) {
            const float t = qd - s;
            const float h2 = t * t;
            if (h2 <= kth) return descend(qp, split, (nearc == 2 * p + 1) ? 2 * p + 2 : 2 * p + 1, level + 1, h, d);
        }
        u = p;
    }
    return NODE_DONE;
}

}  // namespace bkd
