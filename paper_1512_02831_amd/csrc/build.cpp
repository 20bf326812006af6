// build.cpp -- canonical top tree and leaf structure on the host (Section 2.3, Section 3.1).
//
// Level by level, every node holding c points is split in dimension
// (level mod d) at the point of rank floor(c/2) under the total order
// (coordinate, original index): the left child takes the floor(c/2) smallest
// points and the split value is the coordinate of the smallest point on the
// right.  Any exact selection gives the same tree; nth_element does the
// selection here (linear expected time per level, as with the linear-time
// median of Section 3.1).  Leaves keep their points in ascending index.
//
// Under the longest-side rule (the alternative named in Section 2.3) a node
// splits the dimension of the longest side of its points' bounding box: the j
// with the largest float32 fl32(max_j - min_j), the smaller j on ties.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace bkd {

namespace {
struct VI {
    float v;
    int32_t i;
};
inline bool vi_less(const VI &a, const VI &b) { return a.v < b.v || (!(b.v < a.v) && a.i < b.i); }
}  // namespace

void build_canonical(const float *P, int64_t n, int d, int h, HostTree &t, bool parallel, int rule)
{
    const int64_t nleaf = int64_t(1) << h;
    const int64_t nnodes = 2 * nleaf - 1;
    t.n = n;
    t.d = d;
    t.h = h;
    t.split.assign((size_t)(nleaf - 1), 0.0f);
    t.leaf_off.assign((size_t)(nleaf + 1), 0);
    t.perm.resize((size_t)n);
    if (rule == BKD_SPLIT_LONGEST) t.dims.assign((size_t)std::max<int64_t>(nleaf - 1, 0), 0);
    else t.dims.clear();
    std::iota(t.perm.begin(), t.perm.end(), 0);
    std::vector<int64_t> lo((size_t)nnodes), hi((size_t)nnodes);
    std::vector<VI> tmp((size_t)n);
    lo[0] = 0;
    hi[0] = n;
    int32_t *perm = t.perm.data();
    for (int l = 0; l < h; l++) {
        const int64_t first = (int64_t(1) << l) - 1, count = int64_t(1) << l;
        auto split_node = [&](int64_t v) {
            const int64_t a = lo[v], c = hi[v] - lo[v];
            int dim = l % d;
            if (rule == BKD_SPLIT_LONGEST) {
                float best = -1.0f;
                for (int j = 0; j < d; j++) {
                    float mn = INFINITY, mx = -INFINITY;
                    for (int64_t i = 0; i < c; i++) {
                        const float x = P[(int64_t)perm[a + i] * d + j];
                        mn = std::min(mn, x);
                        mx = std::max(mx, x);
                    }
                    const float side = mx - mn;
                    if (side > best) {
                        best = side;
                        dim = j;
                    }
                }
                t.dims[(size_t)v] = (uint8_t)dim;
            }
            VI *s = tmp.data() + a;
            for (int64_t i = 0; i < c; i++) {
                int32_t o = perm[a + i];
                s[i] = VI{P[(int64_t)o * d + dim], o};
            }
            std::nth_element(s, s + c / 2, s + c, vi_less);
            t.split[(size_t)v] = s[c / 2].v;
            for (int64_t i = 0; i < c; i++) perm[a + i] = s[i].i;
            lo[2 * v + 1] = a;
            hi[2 * v + 1] = a + c / 2;
            lo[2 * v + 2] = a + c / 2;
            hi[2 * v + 2] = a + c;
        };
        if (parallel && count >= 4) {
            parallel_for(count, [&](int64_t b, int64_t e) {
                for (int64_t x = b; x < e; x++) split_node(first + x);
            });
        } else {
            for (int64_t x = 0; x < count; x++) split_node(first + x);
        }
    }
    auto sort_leaves = [&](int64_t b, int64_t e) {
        for (int64_t x = b; x < e; x++) {
            int64_t v = nleaf - 1 + x;
            std::sort(perm + lo[v], perm + hi[v]);
        }
    };
    if (parallel) parallel_for(nleaf, sort_leaves);
    else sort_leaves(0, nleaf);
    for (int64_t x = 0; x < nleaf; x++) t.leaf_off[(size_t)x] = lo[nleaf - 1 + x];
    t.leaf_off[(size_t)nleaf] = n;
}

void build_boxes(const float *P, HostTree &t)
{
    const int d = t.d;
    const int64_t nleaf = int64_t(1) << t.h, first = nleaf - 1;
    t.box.assign((size_t)(2 * nleaf - 1) * 2 * d, 0.0f);
    float *box = t.box.data();
    parallel_for(nleaf, [&](int64_t b, int64_t e) {
        for (int64_t l = b; l < e; l++) {
            float *bx = box + (first + l) * 2 * d;
            for (int j = 0; j < d; j++) {
                bx[j] = INFINITY;
                bx[d + j] = -INFINITY;
            }
            for (int64_t p = t.leaf_off[(size_t)l]; p < t.leaf_off[(size_t)l + 1]; p++) {
                const float *x = P + (int64_t)t.perm[(size_t)p] * d;
                for (int j = 0; j < d; j++) {
                    bx[j] = std::min(bx[j], x[j]);
                    bx[d + j] = std::max(bx[d + j], x[j]);
                }
            }
        }
    });
    for (int64_t v = first - 1; v >= 0; v--) {
        float *bx = box + v * 2 * d;
        const float *lc = box + (2 * v + 1) * 2 * d, *rc = box + (2 * v + 2) * 2 * d;
        for (int j = 0; j < d; j++) {
            bx[j] = std::min(lc[j], rc[j]);
            bx[d + j] = std::max(lc[d + j], rc[d + j]);
        }
    }
}

}  // namespace bkd
