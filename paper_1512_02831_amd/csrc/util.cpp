// util.cpp -- errors, host thread pool, device and pinned buffers.
#include <algorithm>
#include <thread>

#include "internal.h"

namespace bkd {

static thread_local std::string g_error;
static thread_local int g_code = 0;

void fail(int code, const std::string &msg) { throw BkdError{code, msg}; }

void set_error(int code, const std::string &msg)
{
    g_code = code;
    g_error = msg;
}

void clear_error()
{
    g_code = 0;
    g_error.clear();
}

const char *last_error_cstr() { return g_error.c_str(); }

int host_threads()
{
    unsigned n = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(n, 64u));
}

void parallel_for(int64_t count, const std::function<void(int64_t, int64_t)> &body, int64_t grain)
{
    if (count <= 0) return;
    int nt = (int)std::min<int64_t>(host_threads(), (count + grain - 1) / grain);
    if (nt <= 1) {
        body(0, count);
        return;
    }
    std::atomic<int64_t> next{0};
    int64_t step = std::max<int64_t>(grain, count / (nt * 8));
    auto worker = [&]() {
        for (;;) {
            int64_t a = next.fetch_add(step);
            if (a >= count) break;
            body(a, std::min(count, a + step));
        }
    };
    std::vector<std::thread> th;
    th.reserve(nt - 1);
    for (int i = 0; i < nt - 1; i++) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

void DevBuf::ensure(size_t need)
{
    if (need <= bytes && p) return;
    release();
    size_t b = std::max<size_t>(need, 256);
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(BKD_ENOMEM, std::string("hipMalloc(") + std::to_string(b) + "): " + hipGetErrorString(e));
    }
    bytes = b;
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

void PinnedBuf::ensure(size_t need)
{
    if (need <= bytes && p) return;
    release();
    size_t b = std::max<size_t>(need, 256);
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(BKD_ENOMEM, std::string("hipHostMalloc(") + std::to_string(b) + "): " + hipGetErrorString(e));
    }
    bytes = b;
}

void PinnedBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

}  // namespace bkd
