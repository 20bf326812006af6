// build_device.hip -- the canonical top tree built on the device (Section 2.3;
// efficient construction is what Section 5 leaves open).  Same tree as the host
// build: level by level, each node of c points is split in dimension
// (level mod d) at rank floor(c/2) of the total order (coordinate, original
// index); the split value is the coordinate of the smallest point on the right,
// and every leaf keeps its points in ascending index.
//
// Each point carries the index of its node in the current level.  A level is
// one stable radix sort of all points, listed in index order, by the key
// (node, ordered coordinate bits): stability turns equal coordinates into
// ascending index, and the node ranges come out in place.  One pass over the
// sorted order then reads the split values and moves every point to its
// child.  A last stable sort by leaf, again over points in index order, gives
// each leaf its points in ascending index.  Coordinates are read from a
// column-major copy of P.
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

__global__ void k_columns(const float *P, int64_t n, int d, float *X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int j = 0; j < d; j++) X[(int64_t)j * n + i] = P[i * d + j];
}

// keys of the points in index order: (node in this level, ordered coordinate); values: the index
__global__ void k_node_keys(const float *col, const uint32_t *node, int64_t n, uint64_t *keys, uint32_t *vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = ((uint64_t)(node ? node[i] : 0u) << 32) | ordered_bits(col[i]);
    vals[i] = (uint32_t)i;
}

// Over the sorted order: node v holds positions [off[v], off[v+1]); its point of
// rank floor(c/2) gives the split value; the first floor(c/2) go to child 2v.
__global__ void k_split_children(const uint64_t *keys, const uint32_t *vals, int64_t n, const int32_t *off,
                                 const float *col, float *split, uint32_t *node)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t v = (uint32_t)(keys[p] >> 32);
    const int32_t a = off[v], half = (off[v + 1] - a) / 2;
    const uint32_t o = vals[p];
    node[o] = 2 * v + ((p - a) >= half ? 1u : 0u);
    if (p - a == half) split[v] = col[o];
}

__global__ void k_leaf_keys(const uint32_t *node, int64_t n, uint32_t *keys, uint32_t *vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = node[i];
    vals[i] = (uint32_t)i;
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

    const int T = 256;
    Mem dX(sizeof(float) * (size_t)n * d);
    {
        Mem dP(sizeof(float) * (size_t)n * d);
        BKD_HIP(hipMemcpyAsync(dP.p, P, sizeof(float) * (size_t)n * d, hipMemcpyHostToDevice, s));
        k_columns<<<blocks(n, T), T, 0, s>>>(dP.as<float>(), n, d, dX.as<float>());
        BKD_HIP(hipGetLastError());
        BKD_HIP(hipStreamSynchronize(s));
    }
    Mem ka(sizeof(uint64_t) * n), kb(sizeof(uint64_t) * n), va(sizeof(uint32_t) * n), vb(sizeof(uint32_t) * n);
    Mem node(sizeof(uint32_t) * n), doff(sizeof(int32_t) * (nleaf + 1));
    Mem dsplit(sizeof(float) * std::max<int64_t>(1, nleaf - 1));
    // temporary storage: the larger of the two sorts' needs
    size_t temp_bytes = 0, leaf_bytes = 0;
    BKD_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, ka.as<uint64_t>(), kb.as<uint64_t>(),
                                               va.as<uint32_t>(), vb.as<uint32_t>(), (int)n, 0, 64, s));
    BKD_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, leaf_bytes, reinterpret_cast<uint32_t *>(ka.p),
                                               reinterpret_cast<uint32_t *>(kb.p), va.as<uint32_t>(),
                                               vb.as<uint32_t>(), (int)n, 0, 32, s));
    temp_bytes = std::max(temp_bytes, leaf_bytes);
    Mem temp(temp_bytes);
    for (int l = 0; l < h; l++) {
        const int count = 1 << l, dim = l % d;
        const float *col = dX.as<float>() + (int64_t)dim * n;
        BKD_HIP(hipMemcpyAsync(doff.p, off[(size_t)l].data(), sizeof(int32_t) * (count + 1), hipMemcpyHostToDevice, s));
        k_node_keys<<<blocks(n, T), T, 0, s>>>(col, l ? node.as<uint32_t>() : nullptr, n, ka.as<uint64_t>(),
                                              va.as<uint32_t>());
        BKD_HIP(hipGetLastError());
        size_t b = temp_bytes;
        BKD_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, b, ka.as<uint64_t>(), kb.as<uint64_t>(), va.as<uint32_t>(),
                                                   vb.as<uint32_t>(), (int)n, 0, 32 + l, s));
        k_split_children<<<blocks(n, T), T, 0, s>>>(kb.as<uint64_t>(), vb.as<uint32_t>(), n, doff.as<int32_t>(), col,
                                                     dsplit.as<float>() + (count - 1), node.as<uint32_t>());
        BKD_HIP(hipGetLastError());
        // the host range array of this level is read by the copy above until the stream gets here
        BKD_HIP(hipStreamSynchronize(s));
    }
    // leaves in ascending index: a stable sort by leaf of the points in index order
    {
        uint32_t *keys = reinterpret_cast<uint32_t *>(ka.p), *keys_out = reinterpret_cast<uint32_t *>(kb.p);
        k_leaf_keys<<<blocks(n, T), T, 0, s>>>(node.as<uint32_t>(), n, keys, va.as<uint32_t>());
        BKD_HIP(hipGetLastError());
        size_t b = temp_bytes;
        BKD_HIP(hipcub::DeviceRadixSort::SortPairs(temp.p, b, keys, keys_out, va.as<uint32_t>(), vb.as<uint32_t>(),
                                                   (int)n, 0, std::max(1, h), s));
    }
    BKD_HIP(hipMemcpyAsync(t.perm.data(), vb.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    BKD_HIP(hipMemcpyAsync(t.split.data(), dsplit.p, sizeof(float) * (nleaf - 1), hipMemcpyDeviceToHost, s));
    BKD_HIP(hipStreamSynchronize(s));
}

}  // namespace bkd
