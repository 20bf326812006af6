// outliers.hip -- proximity-based outlier scores over the reference set
// (Section 4, large-scale outlier detection): every reference point is a
// query (the all-nearest-neighbours problem), its score is the mean distance
// to its k nearest other reference points, and the points are ranked by score.
#include <hipcub/hipcub.hpp>

#include <atomic>
#include <cmath>

#include "internal.h"

namespace bkd {
namespace {

// Rows of k + 1 neighbours in ascending key order.  A point's own entry is
// dropped once (it may be missing when more than k other points share its
// coordinates with smaller indices: then the first k entries are kept); the
// other k distances are summed in ascending order in float64.
__global__ void k_outlier_score(const int64_t *idx, const float *dist, int64_t n, int k, float *score,
                                int64_t *order)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t *ri = idx + i * (k + 1);
    const float *rd = dist + i * (k + 1);
    double s = 0.0;
    int taken = 0;
    bool self_seen = false;
    for (int j = 0; j <= k && taken < k; j++) {
        if (!self_seen && ri[j] == i) {
            self_seen = true;
            continue;
        }
        s += (double)rd[j];
        taken++;
    }
    score[i] = (float)(s / k);
    order[i] = i;
}

void require(bool ok, const char *msg)
{
    if (!ok) fail(BKD_EINVAL, msg);
}

// device memory owned by one call
struct Scratch {
    void *p = nullptr;
    explicit Scratch(size_t bytes)
    {
        if (bytes && hipMalloc(&p, bytes) != hipSuccess) fail(BKD_ENOMEM, "device allocation failed (outlier scores)");
    }
    ~Scratch() { if (p) (void)hipFree(p); }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

}  // namespace
}  // namespace bkd

extern "C" int bkd_outlier_scores(bkd_tree *tree, const float *P, int64_t n, int32_t k, float *out_score,
                                  int64_t *out_order)
{
    using namespace bkd;
    return guarded_call([&] {
        require(tree != nullptr, "tree is NULL");
        Tree &t = tree->t;
        require(n == t.host.n, "n must equal the tree's reference count");
        require(n <= INT32_MAX, "n must be below 2^31");
        require(k >= 1 && k + 1 <= BKD_MAX_K && (int64_t)k + 1 <= n, "k must be in [1, min(n - 1, 63)]");
        require(P && out_score && out_order, "NULL pointer");
        const int d = t.host.d;
        std::atomic<bool> finite{true};
        parallel_for(n * d, [&](int64_t b, int64_t e) {
            bool good = true;
            for (int64_t i = b; i < e; i++) good &= std::isfinite(P[i]);
            if (!good) finite = false;
        }, 1 << 16);
        require(finite, "reference coordinates must be finite");
        BKD_HIP(hipSetDevice(t.device));
        hipStream_t s = tree->stream;
        const int kq = k + 1;
        t.d_Q.ensure(sizeof(float) * (size_t)n * d);
        t.d_outi.ensure(sizeof(int64_t) * (size_t)n * kq);
        t.d_outd.ensure(sizeof(float) * (size_t)n * kq);
        BKD_HIP(hipMemcpyAsync(t.d_Q.p, P, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice, s));
        {
            // scores are means of distances, whatever the tree's output flag says
            struct FlagGuard {
                int32_t &f, saved;
                ~FlagGuard() { f = saved; }
            } guard{t.opt.flags, t.opt.flags};
            t.opt.flags &= ~BKD_FLAG_SQUARED;
            tree_query_device(t, t.d_Q.as<float>(), n, kq, t.d_outi.as<int64_t>(), t.d_outd.as<float>(), s);
        }

        Scratch score(sizeof(float) * n), score_sorted(sizeof(float) * n);
        Scratch order_in(sizeof(int64_t) * n), order(sizeof(int64_t) * n);
        const int threads = 256;
        k_outlier_score<<<(unsigned)((n + threads - 1) / threads), threads, 0, s>>>(
            t.d_outi.as<int64_t>(), t.d_outd.as<float>(), n, k, score.as<float>(), order_in.as<int64_t>());
        BKD_HIP(hipGetLastError());
        // rank: scores descending; the sort is stable, so equal scores keep ascending index
        size_t temp_bytes = 0;
        BKD_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, temp_bytes, score.as<float>(),
                                                             score_sorted.as<float>(), order_in.as<int64_t>(),
                                                             order.as<int64_t>(), (int)n, 0, 32, s));
        Scratch temp(temp_bytes);
        BKD_HIP(hipcub::DeviceRadixSort::SortPairsDescending(temp.p, temp_bytes, score.as<float>(),
                                                             score_sorted.as<float>(), order_in.as<int64_t>(),
                                                             order.as<int64_t>(), (int)n, 0, 32, s));
        BKD_HIP(hipMemcpyAsync(out_score, score.p, sizeof(float) * n, hipMemcpyDeviceToHost, s));
        BKD_HIP(hipMemcpyAsync(out_order, order.p, sizeof(int64_t) * n, hipMemcpyDeviceToHost, s));
        BKD_HIP(hipStreamSynchronize(s));
    });
}
