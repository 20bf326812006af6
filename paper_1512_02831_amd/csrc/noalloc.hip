// noalloc.hip -- bkd_query_async_noalloc: the device-pointer query with no allocation.
//
// The call's workspace (key lists, traversal state, pending pairs, grouping
// scratch, per-leaf offsets) lives in a fixed device array of this file rather
// than in buffers the library grows on demand, so the call itself makes no
// hipMalloc or hipFree.  The array exists once per device (each GPU the
// library runs on holds it until the process ends); its device address is
// looked up once per device and kept.  Calls on one device share the array,
// so calls that overlap on one device race; every part of it that must start
// at zero is cleared by the call's own fill kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace bkd {

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's copy of the array (the current device is `dev`).
void *scratch_on(int dev)
{
    if (dev < 0 || dev >= MAX_DEVICES) fail(BKD_EINVAL, "device ordinal out of range for the fixed workspace");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(BKD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

}  // namespace bkd

extern "C" int bkd_query_async_noalloc(bkd_tree *tree, const float *dQ, int64_t m, int32_t k, int64_t *d_idx,
                                       float *d_dist, void *stream)
{
    return bkd::guarded_call([&] {
        if (!tree) bkd::fail(BKD_EINVAL, "tree is NULL");
        if (m < 0 || m > INT32_MAX) bkd::fail(BKD_EINVAL, "m must be in [0, 2^31-1]");
        if (k < 1 || k > BKD_MAX_K || k > tree->t.host.n) bkd::fail(BKD_EINVAL, "k must be in [1, min(n, 64)]");
        if (m == 0) return;
        if (!dQ || !d_idx || !d_dist) bkd::fail(BKD_EINVAL, "NULL pointer");
        bkd::Tree &t = tree->t;
        if (!t.resident) bkd::fail(BKD_EINVAL, "the fixed workspace serves resident trees only");
        if (t.opt.flags & BKD_FLAG_TRACE) bkd::fail(BKD_EINVAL, "the fixed workspace records no trace");
        const size_t need = bkd::workspace_bytes(t, m, k);
        if (need > bkd::SCRATCH_BYTES)
            bkd::fail(BKD_EINVAL, "query needs " + std::to_string(need) + " workspace bytes; the fixed workspace holds " +
                                      std::to_string(bkd::SCRATCH_BYTES));
        BKD_HIP(hipSetDevice(t.device));
        void *region = bkd::scratch_on(t.device);
        bkd::tree_query_device(t, dQ, m, k, d_idx, d_dist, static_cast<hipStream_t>(stream), region);
    });
}
