// build_device.hip -- the canonical top tree built on the device (Section 2.3;
// efficient construction is what Section 5 leaves open).  Same tree as the host
// build: level by level, each node of c points is split in dimension
// (level mod d) at rank floor(c/2) of the total order (coordinate, original
// index); the split value is the coordinate of the smallest point on the right,
// and every leaf keeps its points in ascending index.
//
// Every level is one segmented sort of all n points by the 64-bit key
// (ordered coordinate bits, index), one segment per node: the key is unique,
// so no stability is assumed of the sort.  The node ranges depend on n and h
// only and are computed on the host.  A last segmented sort by index orders
// the leaves.
#include <hipcub/hipcub.hpp>

#include <numeric>
#include <vector>

#include "internal.h"

namespace bkd {
namespace {

// float -> unsigned with the same order; -0 is taken as +0 (they compare equal)
__device__ inline uint32_t ordered_bits(float x)
{
    const uint32_t b = __float_as_uint(x == 0.0f ? 0.0f : x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__global__ void k_level_keys(const float *P, int64_t n, int d, int dim, const uint64_t *prev, uint64_t *keys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t o = prev ? (uint32_t)prev[i] : (uint32_t)i;
    keys[i] = ((uint64_t)ordered_bits(P[(int64_t)o * d + dim]) << 32) | o;
}

// split value of each node of a level: the coordinate of its point of rank floor(c/2)
__global__ void k_level_splits(const uint64_t *sorted, const int32_t *off, int count, const float *P, int d, int dim,
                               float *split)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= count) return;
    const int32_t a = off[x], c = off[x + 1] - a;
    const uint32_t o = (uint32_t)sorted[a + c / 2];
    split[x] = P[(int64_t)o * d + dim];
}

__global__ void k_low_words(const uint64_t *keys, int64_t n, uint32_t *idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) idx[i] = (uint32_t)keys[i];
}

struct Mem {
    void *p = nullptr;
    explicit Mem(size_t bytes)
    {
        if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) fail(BKD_ENOMEM, "device allocation failed (device build)");
    }
    ~Mem() { if (p) (void)hipFree(p); }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

unsigned blocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void build_canonical_device(const float *P, int64_t n, int d, int h, HostTree &t, hipStream_t s)
{
    if (n > INT32_MAX) fail(BKD_EINVAL, "the device build takes n below 2^31");
    const int64_t nleaf = int64_t(1) << h;
    t.n = n;
    t.d = d;
    t.h = h;
    t.split.assign((size_t)(nleaf - 1), 0.0f);
    t.leaf_off.assign((size_t)(nleaf + 1), 0);
    t.perm.resize((size_t)n);
    // node ranges, level by level (they depend on n and h only)
    std::vector<std::vector<int32_t>> off((size_t)h + 1);
    off[0] = {0, (int32_t)n};
    for (int l = 0; l < h; l++) {
        const std::vector<int32_t> &o = off[(size_t)l];
        std::vector<int32_t> &c = off[(size_t)l + 1];
        c.resize(o.size() * 2 - 1);
        for (size_t x = 0; x + 1 < o.size(); x++) {
            c[2 * x] = o[x];
            c[2 * x + 1] = o[x] + (o[x + 1] - o[x]) / 2;
        }
        c.back() = (int32_t)n;
    }
    for (int64_t x = 0; x <= nleaf; x++) t.leaf_off[(size_t)x] = off[(size_t)h][(size_t)x];
    if (h == 0) {
        std::iota(t.perm.begin(), t.perm.end(), 0);
        return;
    }

    Mem dP(sizeof(float) * (size_t)n * d), ka(sizeof(uint64_t) * n), kb(sizeof(uint64_t) * n);
    Mem doff(sizeof(int32_t) * (nleaf + 1)), dsplit(sizeof(float) * std::max<int64_t>(1, nleaf - 1));
    Mem ia(sizeof(uint32_t) * n), ib(sizeof(uint32_t) * n);
    BKD_HIP(hipMemcpyAsync(dP.p, P, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice, s));
    // temporary storage: the largest of every sort below
    size_t temp_bytes = 0;
    for (int l = 0; l < h; l++) {
        size_t b = 0;
        BKD_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, b, ka.as<uint64_t>(), kb.as<uint64_t>(), (int)n,
                                                             1 << l, doff.as<int32_t>(), doff.as<int32_t>() + 1, 0,
                                                             64, s));
        temp_bytes = std::max(temp_bytes, b);
    }
    {
        size_t b = 0;
        BKD_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, b, ia.as<uint32_t>(), ib.as<uint32_t>(), (int)n,
                                                             (int)nleaf, doff.as<int32_t>(), doff.as<int32_t>() + 1,
                                                             0, 32, s));
        temp_bytes = std::max(temp_bytes, b);
    }
    Mem temp(temp_bytes);
    const int T = 256;
    for (int l = 0; l < h; l++) {
        const int count = 1 << l, dim = l % d;
        BKD_HIP(hipMemcpyAsync(doff.p, off[(size_t)l].data(), sizeof(int32_t) * (count + 1), hipMemcpyHostToDevice, s));
        k_level_keys<<<blocks(n, T), T, 0, s>>>(dP.as<float>(), n, d, dim, l ? kb.as<uint64_t>() : nullptr,
                                                ka.as<uint64_t>());
        BKD_HIP(hipGetLastError());
        size_t b = temp_bytes;
        BKD_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(temp.p, b, ka.as<uint64_t>(), kb.as<uint64_t>(), (int)n,
                                                             count, doff.as<int32_t>(), doff.as<int32_t>() + 1, 0, 64,
                                                             s));
        k_level_splits<<<blocks(count, T), T, 0, s>>>(kb.as<uint64_t>(), doff.as<int32_t>(), count, dP.as<float>(),
                                                      d, dim, dsplit.as<float>() + (count - 1));
        BKD_HIP(hipGetLastError());
        // the host range array is reused by the next copy only after this level's kernels ran
        BKD_HIP(hipStreamSynchronize(s));
    }
    // leaves in ascending index
    k_low_words<<<blocks(n, T), T, 0, s>>>(kb.as<uint64_t>(), n, ia.as<uint32_t>());
    BKD_HIP(hipGetLastError());
    BKD_HIP(hipMemcpyAsync(doff.p, off[(size_t)h].data(), sizeof(int32_t) * (nleaf + 1), hipMemcpyHostToDevice, s));
    size_t b = temp_bytes;
    BKD_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(temp.p, b, ia.as<uint32_t>(), ib.as<uint32_t>(), (int)n,
                                                         (int)nleaf, doff.as<int32_t>(), doff.as<int32_t>() + 1, 0, 32,
                                                         s));
    BKD_HIP(hipMemcpyAsync(t.perm.data(), ib.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    BKD_HIP(hipMemcpyAsync(t.split.data(), dsplit.p, sizeof(float) * (nleaf - 1), hipMemcpyDeviceToHost, s));
    BKD_HIP(hipStreamSynchronize(s));
}

}  // namespace bkd
