// api.cpp -- the extern "C" boundary: argument checks, error codes, no exceptions escape.
#include <cmath>
#include <new>

#include "internal.h"

namespace bkd {
const char *last_error_cstr();
}

namespace bkd {
// The boundary's exception guard, shared with the batched and served forms.
int guarded_call(const std::function<void()> &f);
}

namespace {

template <class F> int guarded(F &&f)
{
    bkd::clear_error();
    try {
        f();
        return BKD_OK;
    } catch (const bkd::BkdError &e) {
        bkd::set_error(e.code, e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        bkd::set_error(BKD_ENOMEM, "host allocation failed");
        return BKD_ENOMEM;
    } catch (const std::exception &e) {
        bkd::set_error(BKD_EDEVICE, e.what());
        return BKD_EDEVICE;
    } catch (...) {
        bkd::set_error(BKD_EDEVICE, "unknown failure");
        return BKD_EDEVICE;
    }
}

}  // namespace

int bkd::guarded_call(const std::function<void()> &f) { return guarded(f); }

namespace {

void require(bool ok, const char *msg)
{
    if (!ok) bkd::fail(BKD_EINVAL, msg);
}

bool all_finite(const float *p, int64_t count)
{
    std::atomic<bool> ok{true};
    bkd::parallel_for(count, [&](int64_t b, int64_t e) {
        bool good = true;
        for (int64_t i = b; i < e; i++) good &= std::isfinite(p[i]);
        if (!good) ok = false;
    }, 1 << 16);
    return ok;
}

void check_query_args(const bkd_tree *tree, int64_t m, int32_t k)
{
    require(tree != nullptr, "tree is NULL");
    require(m >= 0 && m <= INT32_MAX, "m must be in [0, 2^31-1]");
    require(k >= 1 && k <= BKD_MAX_K && k <= tree->t.host.n, "k must be in [1, min(n, 64)]");
}

}  // namespace

extern "C" {

const char *bkd_last_error(void) { return bkd::last_error_cstr(); }

const char *bkd_version(void) { return "bkd-mi355x 0.1 (gfx950)"; }

int bkd_default_options(int32_t height, bkd_options *out)
{
    return guarded([&] {
        require(out != nullptr, "out is NULL");
        require(height >= 0 && height <= BKD_MAX_HEIGHT, "height out of range");
        *out = bkd_options{};
        out->buffer_size = int64_t(1) << (height < 24 ? 24 - height : 0);
        out->fetch_size = 10 * out->buffer_size;
        out->chunk_mode = BKD_CHUNK_LEAF;
    });
}

int bkd_build(const float *P, int64_t n, int32_t d, int32_t height, const bkd_options *opt, bkd_tree **out)
{
    bkd_tree *tree = nullptr;
    int rc = guarded([&] {
        require(out != nullptr, "out is NULL");
        *out = nullptr;
        require(P != nullptr, "P is NULL");
        require(n >= 1 && n <= INT32_MAX, "n must be in [1, 2^31-1]");
        require(d >= 1 && d <= BKD_MAX_DIM, "d must be in [1, 32]");
        require(height >= 0 && height <= BKD_MAX_HEIGHT, "height must be in [0, 24]");
        require((int64_t(1) << height) <= n, "2^height must not exceed n");
        bkd_options o{};
        if (opt) o = *opt;
        else bkd_default_options(height, &o);
        require(o.device >= 0, "device must be >= 0");
        require(all_finite(P, n * d), "reference coordinates must be finite");
        int ndev = 0;
        BKD_HIP(hipGetDeviceCount(&ndev));
        require(o.device < ndev, "device ordinal out of range");
        tree = new bkd_tree();
        bkd::tree_build(tree->t, P, n, d, height, o);
        BKD_HIP(hipStreamCreateWithFlags(&tree->stream, hipStreamNonBlocking));
        *out = tree;
    });
    if (rc != BKD_OK) {
        if (tree) {
            bkd::leaffile_destroy(tree->t);
            if (tree->stream) (void)hipStreamDestroy(tree->stream);
            if (tree->t.copy_stream) (void)hipStreamDestroy(tree->t.copy_stream);
            delete tree;
        }
    }
    return rc;
}

int bkd_free(bkd_tree *tree)
{
    return guarded([&] {
        if (!tree) return;
        (void)hipSetDevice(tree->t.device);
        (void)hipDeviceSynchronize();
        bkd::leaffile_destroy(tree->t);
        if (tree->stream) (void)hipStreamDestroy(tree->stream);
        if (tree->t.copy_stream) (void)hipStreamDestroy(tree->t.copy_stream);
        for (int b = 0; b < 2; b++) {
            if (tree->t.ev_copied[b]) (void)hipEventDestroy(tree->t.ev_copied[b]);
            if (tree->t.ev_used[b]) (void)hipEventDestroy(tree->t.ev_used[b]);
        }
        if (tree->t.ev_rb) (void)hipEventDestroy(tree->t.ev_rb);
        delete tree;
    });
}

int bkd_query(bkd_tree *tree, const float *Q, int64_t m, int32_t k, int64_t *out_idx, float *out_dist)
{
    return guarded([&] {
        check_query_args(tree, m, k);
        if (m == 0) return;
        require(Q && out_idx && out_dist, "NULL pointer");
        const int d = tree->t.host.d;
        require(all_finite(Q, m * d), "query coordinates must be finite");
        bkd::Tree &t = tree->t;
        BKD_HIP(hipSetDevice(t.device));
        t.d_Q.ensure(sizeof(float) * (size_t)m * d);
        t.d_outi.ensure(sizeof(int64_t) * (size_t)m * k);
        t.d_outd.ensure(sizeof(float) * (size_t)m * k);
        BKD_HIP(hipMemcpyAsync(t.d_Q.p, Q, sizeof(float) * (size_t)m * d, hipMemcpyHostToDevice, tree->stream));
        bkd::tree_query_device(t, t.d_Q.as<float>(), m, k, t.d_outi.as<int64_t>(), t.d_outd.as<float>(),
                               tree->stream);
        BKD_HIP(hipMemcpyAsync(out_idx, t.d_outi.p, sizeof(int64_t) * (size_t)m * k, hipMemcpyDeviceToHost,
                               tree->stream));
        BKD_HIP(hipMemcpyAsync(out_dist, t.d_outd.p, sizeof(float) * (size_t)m * k, hipMemcpyDeviceToHost,
                               tree->stream));
        BKD_HIP(hipStreamSynchronize(tree->stream));
    });
}

int bkd_query_async(bkd_tree *tree, const float *dQ, int64_t m, int32_t k, int64_t *d_idx, float *d_dist,
                    void *stream)
{
    return guarded([&] {
        check_query_args(tree, m, k);
        if (m == 0) return;
        require(dQ && d_idx && d_dist, "NULL pointer");
        bkd::tree_query_device(tree->t, dQ, m, k, d_idx, d_dist, static_cast<hipStream_t>(stream));
    });
}

int bkd_tree_info_get(const bkd_tree *tree, bkd_tree_info *out)
{
    return guarded([&] {
        require(tree && out, "NULL pointer");
        const bkd::Tree &t = tree->t;
        out->n = t.host.n;
        out->d = t.host.d;
        out->height = t.host.h;
        out->buffer_size = t.B;
        out->fetch_size = t.M;
        out->num_chunks = (int32_t)t.chunks.size();
        out->resident = t.resident ? 1 : 0;
        out->leaf_bytes = t.host.n * (int64_t)(4 * t.host.d + 4);
        out->chunk_capacity_bytes = (int64_t)t.chunk_cap_bytes;
        out->on_disk = t.leaf_file ? 1 : 0;
        out->direct_io = bkd::leaffile_direct(t) ? 1 : 0;
    });
}

int bkd_tree_export(const bkd_tree *tree, float *split, int64_t *leaf_off, int32_t *perm)
{
    return guarded([&] {
        require(tree != nullptr, "tree is NULL");
        const bkd::HostTree &H = tree->t.host;
        if (split && !H.split.empty()) std::memcpy(split, H.split.data(), sizeof(float) * H.split.size());
        if (leaf_off) std::memcpy(leaf_off, H.leaf_off.data(), sizeof(int64_t) * H.leaf_off.size());
        if (perm) std::memcpy(perm, H.perm.data(), sizeof(int32_t) * H.perm.size());
    });
}

int bkd_tree_rules_export(const bkd_tree *tree, int32_t *dims, float *box)
{
    return guarded([&] {
        require(tree != nullptr, "tree is NULL");
        const bkd::HostTree &H = tree->t.host;
        if (dims) {
            for (size_t v = 0; v < H.split.size(); v++) {
                int level = 0;
                while ((size_t(2) << level) <= v + 1) level++;
                dims[v] = H.dims.empty() ? level % H.d : (int32_t)H.dims[v];
            }
        }
        if (box) {
            require(!H.box.empty(), "the tree was built without BKD_PRUNE_BOX (no node boxes)");
            std::memcpy(box, H.box.data(), sizeof(float) * H.box.size());
        }
    });
}

int bkd_chunk_plan(const bkd_tree *tree, int64_t *lo, int64_t *hi)
{
    return guarded([&] {
        require(tree && lo && hi, "NULL pointer");
        for (size_t j = 0; j < tree->t.chunks.size(); j++) {
            lo[j] = tree->t.chunks[j].lo;
            hi[j] = tree->t.chunks[j].hi;
        }
    });
}

int bkd_last_stats(const bkd_tree *tree, bkd_stats *out)
{
    return guarded([&] {
        require(tree && out, "NULL pointer");
        *out = tree->t.stats;
    });
}

int bkd_trace_size(const bkd_tree *tree, int64_t *ncalls, int64_t *length)
{
    return guarded([&] {
        require(tree && ncalls && length, "NULL pointer");
        *ncalls = (int64_t)tree->t.trace_off.size() - 1;
        *length = (int64_t)tree->t.trace_q.size();
    });
}

int bkd_trace_get(const bkd_tree *tree, int64_t *call_off, int32_t *query, int32_t *leaf)
{
    return guarded([&] {
        require(tree && call_off && query && leaf, "NULL pointer");
        const bkd::Tree &t = tree->t;
        std::memcpy(call_off, t.trace_off.data(), sizeof(int64_t) * t.trace_off.size());
        if (!t.trace_q.empty()) {
            std::memcpy(query, t.trace_q.data(), sizeof(int32_t) * t.trace_q.size());
            std::memcpy(leaf, t.trace_leaf.data(), sizeof(int32_t) * t.trace_leaf.size());
        }
    });
}

}  // extern "C"
