// query.cpp -- tree upload, streaming plan and the two query schedules.
//
// Algorithm 1 schedule (fetch_size >= 0).  The paper's queues live on the
// device: `input` is the range of not yet fetched query ids, `reinsert` a
// FIFO ring.  Each iteration fetches up to M ids (reinsert first), runs
// FindLeafBatch, appends the (leaf, query) pairs to the pending list (the
// pooled buffers, in fetch order) and reads back the largest buffer fill.
// When a buffer is half-full or both queues are empty, ProcessAllBuffers
// runs: a stable sort groups the pending pairs by leaf (the buffers' contents
// in insertion order), the leaf scans update every buffered query's list and
// the buffered ids are appended to reinsert in ascending leaf order.  With a
// streamed leaf structure every call walks the chunks holding a buffered leaf
// in order (Section 3.2): the copy of the next chunk runs on a second stream
// while the scan of the current chunk runs on the caller's stream, events
// order each copy after the last scan that read its buffer and each scan after
// its copy (Brute / Copy / Wait on two queues, without blocking the host), and
// after the last chunk of a call the first chunk is prefetched for the next.
//
// Lock-step schedule (fetch_size < 0).  Every iteration is one round over all
// active queries: sort the pending pairs by leaf, scan, FindLeafBatch on the
// scanned queries.  With a leaf-aligned streamed structure a round covers one
// resident chunk at a time: the chunk is drained (its queries scanned and
// routed again, round after round, while their next leaf stays inside it)
// before the sweep moves on to the next chunk holding pending queries, whose
// copy was prefetched meanwhile.  A query's leaf sequence depends only on its
// own data, so both schedules visit the same (query, leaf) pairs and give the
// same results; the sweep copies each chunk once per pass instead of once per
// round.
#include <atomic>
#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"

namespace bkd {

static int key_bits_for(int nleaf)
{
    // keys are leaf ids 0..nleaf-1 plus the sentinel nleaf
    int b = 1;
    while ((1ll << b) <= nleaf) b++;
    return b;
}

static void plan_chunks(Tree &t)
{
    const HostTree &H = t.host;
    const int64_t n = H.n;
    const int d = H.d;
    t.leaf_blk.assign((size_t)t.nleaf + 1, 0);
    int64_t maxleaf = 0;
    for (int l = 0; l < t.nleaf; l++) {
        const int64_t len = H.leaf_off[l + 1] - H.leaf_off[l];
        t.leaf_blk[(size_t)l + 1] = t.leaf_blk[(size_t)l] + (int64_t)(d + 1) * len;
        maxleaf = std::max(maxleaf, len);
    }
    const size_t bpp = (size_t)(4 * d + 4);
    const size_t total = (size_t)n * bpp;
    const int64_t budget = t.opt.leaf_budget_bytes;
    if (budget < 0) fail(BKD_EINVAL, "leaf_budget_bytes must be >= 0");
    if (t.opt.num_chunks < 0) fail(BKD_EINVAL, "num_chunks must be >= 0");
    if (t.opt.chunk_mode != BKD_CHUNK_LEAF && t.opt.chunk_mode != BKD_CHUNK_POSITION)
        fail(BKD_EINVAL, "unknown chunk_mode");
    t.chunks.clear();
    t.resident = (t.opt.num_chunks == 0) && (budget == 0 || (size_t)budget >= total);
    if (t.resident) {
        t.chunks.push_back(Chunk{0, n, 0, t.nleaf - 1, 0, t.leaf_blk.back()});
        t.chunk_cap_bytes = total;
        return;
    }
    if (budget > 0 && (size_t)budget < 2 * (size_t)maxleaf * bpp)
        fail(BKD_EBUDGET, "leaf budget of " + std::to_string(budget) + " bytes is below two leaves (" +
                              std::to_string(2 * (size_t)maxleaf * bpp) + " bytes)");
    const size_t cap_bytes = budget > 0 ? (size_t)budget / 2 : total;
    std::vector<std::pair<int64_t, int64_t>> ranges;  // positions
    if (t.opt.chunk_mode == BKD_CHUNK_POSITION) {
        // chunk j of N: positions [ceil((j-1) n / N), ceil(j n / N)); a leaf crossing a bound is
        // held whole by both chunks, each scanning only its own positions
        int64_t N = t.opt.num_chunks;
        if (N == 0) {
            N = (int64_t)((total + cap_bytes - 1) / cap_bytes);
            for (;; N++) {  // the leaf blocks a chunk holds may exceed its positions
                bool fits = true;
                for (int64_t j = 1; j <= N && fits; j++) {
                    int64_t lo = ((j - 1) * n + N - 1) / N, hi = (j * n + N - 1) / N;
                    int64_t a = std::upper_bound(H.leaf_off.begin(), H.leaf_off.end(), lo) - H.leaf_off.begin() - 1;
                    int64_t b = std::upper_bound(H.leaf_off.begin(), H.leaf_off.end(), hi - 1) - H.leaf_off.begin();
                    fits = (size_t)(H.leaf_off[b] - H.leaf_off[a]) * bpp <= cap_bytes;
                }
                if (fits || N >= n) break;
            }
        }
        N = std::max<int64_t>(1, std::min<int64_t>(N, n));
        for (int64_t j = 1; j <= N; j++) ranges.emplace_back(((j - 1) * n + N - 1) / N, (j * n + N - 1) / N);
    } else if (t.opt.num_chunks > 0) {
        // whole leaves, the leaf index range split by the same ceiling rule
        int64_t N = std::min<int64_t>(t.opt.num_chunks, t.nleaf);
        for (int64_t j = 1; j <= N; j++) {
            int64_t a = ((j - 1) * t.nleaf + N - 1) / N, b = (j * t.nleaf + N - 1) / N;
            ranges.emplace_back(H.leaf_off[a], H.leaf_off[b]);
        }
    } else {
        // greedy: as many whole leaves as fit the chunk capacity
        int l = 0;
        while (l < t.nleaf) {
            int e = l;
            while (e < t.nleaf && (size_t)(H.leaf_off[e + 1] - H.leaf_off[l]) * bpp <= cap_bytes) e++;
            ranges.emplace_back(H.leaf_off[l], H.leaf_off[e]);
            l = e;
        }
    }
    size_t cap = 0;
    for (auto &r : ranges) {
        Chunk c;
        c.lo = r.first;
        c.hi = r.second;
        c.leaf_first = (int32_t)(std::upper_bound(H.leaf_off.begin(), H.leaf_off.end(), c.lo) - H.leaf_off.begin() - 1);
        c.leaf_last =
            (int32_t)(std::upper_bound(H.leaf_off.begin(), H.leaf_off.end(), c.hi - 1) - H.leaf_off.begin() - 1);
        c.word_lo = t.leaf_blk[(size_t)c.leaf_first];
        c.word_hi = t.leaf_blk[(size_t)c.leaf_last + 1];
        cap = std::max(cap, (size_t)(c.word_hi - c.word_lo) * 4);
        t.chunks.push_back(c);
    }
    if (budget > 0 && cap > cap_bytes) fail(BKD_EBUDGET, "chunk count too small for the leaf budget");
    t.chunk_cap_bytes = cap;
}

// Write the blocks of leaves [lf, ll] to dst (word 0 = first word of leaf lf).
void gather_leaves(const float *P, const Tree &t, int lf, int ll, void *dst)
{
    const HostTree &H = t.host;
    const int d = H.d;
    float *out = static_cast<float *>(dst) - t.leaf_blk[(size_t)lf];
    parallel_for(ll - lf + 1, [&](int64_t b, int64_t e) {
        for (int64_t x = b; x < e; x++) {
            const int l = lf + (int)x;
            const int64_t a = H.leaf_off[(size_t)l], len = H.leaf_off[(size_t)l + 1] - a;
            float *X = out + t.leaf_blk[(size_t)l];
            int32_t *orig = reinterpret_cast<int32_t *>(X + (size_t)d * len);
            for (int64_t i = 0; i < len; i++) {
                const int32_t o = H.perm[(size_t)(a + i)];
                const float *p = P + (int64_t)o * d;
                for (int j = 0; j < d; j++) X[(size_t)j * len + i] = p[j];
                orig[i] = o;
            }
        }
    });
}

void tree_build(Tree &t, const float *P, int64_t n, int d, int h, const bkd_options &opt)
{
    t.opt = opt;
    t.device = opt.device;
    BKD_HIP(hipSetDevice(t.device));
    t.nleaf = 1 << h;
    t.B = opt.buffer_size == 0 ? (int64_t(1) << std::max(0, 24 - h)) : (opt.buffer_size < 0 ? -1 : opt.buffer_size);
    if (opt.fetch_size == 0) t.M = t.B > 0 ? 10 * t.B : -1;
    else t.M = opt.fetch_size < 0 ? -1 : opt.fetch_size;

    if (opt.split_rule != BKD_SPLIT_CYCLIC && opt.split_rule != BKD_SPLIT_LONGEST)
        fail(BKD_EINVAL, "split_rule must be BKD_SPLIT_CYCLIC or BKD_SPLIT_LONGEST");
    if (opt.prune != BKD_PRUNE_PLANE && opt.prune != BKD_PRUNE_BOX)
        fail(BKD_EINVAL, "prune must be BKD_PRUNE_PLANE or BKD_PRUNE_BOX");
    if ((opt.flags & BKD_FLAG_DEVICE_BUILD) && opt.split_rule != BKD_SPLIT_CYCLIC)
        fail(BKD_EINVAL, "the device build supports the cyclic splitting rule only");
    if (opt.flags & BKD_FLAG_DEVICE_BUILD) build_canonical_device(P, n, d, h, t.host, nullptr);
    else build_canonical(P, n, d, h, t.host, true, opt.split_rule);
    if (opt.prune == BKD_PRUNE_BOX) build_boxes(P, t.host);
    plan_chunks(t);
    t.sweep = !t.resident && t.opt.chunk_mode == BKD_CHUNK_LEAF &&
              (int64_t)t.chunks.size() < DISTRIBUTE_MAX_TARGETS;
    for (int l = 0; l < t.nleaf; l++)
        if (t.host.leaf_off[(size_t)l + 1] - t.host.leaf_off[(size_t)l] >= (int64_t(1) << 30)) t.dense_min = INT32_MAX;

    const HostTree &H = t.host;
    t.d_split.ensure(sizeof(float) * std::max<size_t>(1, H.split.size()));
    if (!H.split.empty())
        BKD_HIP(hipMemcpy(t.d_split.p, H.split.data(), sizeof(float) * H.split.size(), hipMemcpyHostToDevice));
    std::vector<int32_t> lo32(H.leaf_off.size());
    for (size_t i = 0; i < lo32.size(); i++) lo32[i] = (int32_t)H.leaf_off[i];
    t.d_leaf_off.ensure(sizeof(int32_t) * lo32.size());
    BKD_HIP(hipMemcpy(t.d_leaf_off.p, lo32.data(), sizeof(int32_t) * lo32.size(), hipMemcpyHostToDevice));
    if (!H.dims.empty()) {
        t.d_dims.ensure(H.dims.size());
        BKD_HIP(hipMemcpy(t.d_dims.p, H.dims.data(), H.dims.size(), hipMemcpyHostToDevice));
    }
    if (!H.box.empty()) {
        t.d_box.ensure(sizeof(float) * H.box.size());
        BKD_HIP(hipMemcpy(t.d_box.p, H.box.data(), sizeof(float) * H.box.size(), hipMemcpyHostToDevice));
    }
    t.d_leaf_blk.ensure(sizeof(int64_t) * t.leaf_blk.size());
    BKD_HIP(hipMemcpy(t.d_leaf_blk.p, t.leaf_blk.data(), sizeof(int64_t) * t.leaf_blk.size(), hipMemcpyHostToDevice));
    {
        // leaf centres (bounding-box midpoints) for the inner-product filter of the dense scan
        // leaf centres, then each leaf's scale: the power of two 2^-e with 2^e at least its
        // largest centred coordinate |fl32(x - c)| (attained at the box's lo or hi, since
        // rounding is monotone), so that scaled centred coordinates lie in [-1, 1]
        std::vector<float> cen((size_t)t.nleaf * d + t.nleaf);
        std::atomic<bool> wide{false};
        parallel_for(t.nleaf, [&](int64_t b, int64_t e) {
            bool w = false;
            for (int64_t l = b; l < e; l++) {
                float mx = 0.0f;
                for (int j = 0; j < d; j++) {
                    float lo = INFINITY, hi = -INFINITY;
                    for (int64_t p = H.leaf_off[(size_t)l]; p < H.leaf_off[(size_t)l + 1]; p++) {
                        const float v = P[(int64_t)H.perm[(size_t)p] * d + j];
                        lo = std::min(lo, v);
                        hi = std::max(hi, v);
                    }
                    const float c = 0.5f * lo + 0.5f * hi;
                    cen[(size_t)l * d + j] = c;
                    mx = std::max(mx, std::max(std::fabs(lo - c), std::fabs(hi - c)));
                    w |= -lo > FILTER_RANGE || hi > FILTER_RANGE;
                }
                int ex = 0;
                const float m = std::frexp(mx, &ex);  // mx = m 2^ex, m in [0.5, 1)
                int pe = (mx == 0.0f) ? 0 : (m == 0.5f ? ex - 1 : ex);
                pe = std::min(126, std::max(-126, pe));
                cen[(size_t)t.nleaf * d + l] = std::ldexp(1.0f, -pe);
            }
            if (w) wide = true;
        });
        t.wide = wide;
        t.d_centers.ensure(sizeof(float) * cen.size());
        BKD_HIP(hipMemcpy(t.d_centers.p, cen.data(), sizeof(float) * cen.size(), hipMemcpyHostToDevice));
    }

    const size_t total_bytes = (size_t)t.leaf_blk.back() * 4;
    if (t.resident) {
        std::vector<float> blk((size_t)t.leaf_blk.back());
        gather_leaves(P, t, 0, t.nleaf - 1, blk.data());
        t.d_chunk[0].ensure(total_bytes);
        BKD_HIP(hipMemcpy(t.d_chunk[0].p, blk.data(), total_bytes, hipMemcpyHostToDevice));
        t.chunk_in[0] = 0;
    } else {
        if (opt.leaf_path) {
            leaffile_create(t, P, opt.leaf_path);
        } else {
            t.h_leaf.ensure(total_bytes);
            gather_leaves(P, t, 0, t.nleaf - 1, t.h_leaf.p);
        }
        t.d_chunk[0].ensure(t.chunk_cap_bytes);
        t.d_chunk[1].ensure(t.chunk_cap_bytes);
        BKD_HIP(hipStreamCreateWithFlags(&t.copy_stream, hipStreamNonBlocking));
        for (int b = 0; b < 2; b++) {
            BKD_HIP(hipEventCreateWithFlags(&t.ev_copied[b], hipEventDisableTiming));
            BKD_HIP(hipEventCreateWithFlags(&t.ev_used[b], hipEventDisableTiming));
            BKD_HIP(hipEventRecord(t.ev_copied[b], t.copy_stream));
            BKD_HIP(hipEventRecord(t.ev_used[b], t.copy_stream));
        }
        t.chunk_in[0] = t.chunk_in[1] = -1;
        std::vector<int32_t> chunk_of((size_t)t.nleaf, 0);
        for (int j = 0; j < (int)t.chunks.size(); j++)
            for (int l = t.chunks[(size_t)j].leaf_first; l <= t.chunks[(size_t)j].leaf_last; l++) chunk_of[(size_t)l] = j;
        t.d_chunk_of.ensure(sizeof(int32_t) * chunk_of.size());
        BKD_HIP(hipMemcpy(t.d_chunk_of.p, chunk_of.data(), sizeof(int32_t) * chunk_of.size(), hipMemcpyHostToDevice));
    }
    t.d_ctl.ensure(sizeof(int32_t) * CTL_WORDS);
    t.h_ctl.ensure(sizeof(int32_t) * CTL_WORDS);
    BKD_HIP(hipEventCreateWithFlags(&t.ev_rb, hipEventDisableTiming));
    BKD_HIP(hipDeviceSynchronize());
}

namespace {

struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    bool on = false;
    void begin(hipStream_t s)
    {
        if (!on) return;
        hipEvent_t a, b;
        BKD_HIP(hipEventCreate(&a));
        BKD_HIP(hipEventCreate(&b));
        BKD_HIP(hipEventRecord(a, s));
        ev.emplace_back(a, b);
    }
    void end(hipStream_t s)
    {
        if (!on) return;
        BKD_HIP(hipEventRecord(ev.back().second, s));
    }
    double total_ms()
    {
        double t = 0;
        for (auto &p : ev) {
            float ms = 0;
            BKD_HIP(hipEventSynchronize(p.second));
            BKD_HIP(hipEventElapsedTime(&ms, p.first, p.second));
            t += ms;
        }
        return t;
    }
    ~Timer()
    {
        for (auto &p : ev) {
            (void)hipEventDestroy(p.first);
            (void)hipEventDestroy(p.second);
        }
    }
};

// Per-query-call state shared by both schedules.
struct Run {
    Tree &t;
    hipStream_t s;
    const float *dQ;               // query coordinates as numbered inside the call
    const int32_t *perm = nullptr;  // internal number -> caller's query (null: identity)
    int64_t m;
    int k, K, d, h, nleaf, kbits;
    bool counted = false;  // the last sort_and_offsets already counted a full scan's work
    bool tracing;
    int32_t *ctl, *hctl, *cnt;
    uint32_t *leafbuf[2];
    int32_t *qbuf[2];
    int cur = 0;  // pair holding the pending list
    const int32_t *bufq_override = nullptr;  // scan input other than the pending pair (chunk sweep)
    uint32_t *route_override = nullptr;     // chunk sweep: the scans route into this list
    Timer tdense, tsparse, tfind, tgroup, tcopy;
    double wait_ms = 0;  // host time spent waiting for the device
    std::vector<int32_t> tr_q, tr_l;
    Workspace ws;

    Run(Tree &t_, hipStream_t s_, const float *dQ_, int64_t m_, int k_, const Workspace &ws_, bool timing)
        : t(t_), s(s_), dQ(dQ_), m(m_), k(k_), K(key_capacity(k_)), d(t_.host.d), h(t_.host.h), nleaf(t_.nleaf),
          kbits(key_bits_for(t_.nleaf)), tracing((t_.opt.flags & BKD_FLAG_TRACE) != 0), ws(ws_)
    {
        if (!t.resident) t.h_tiles.ensure(sizeof(int32_t) * 3 * (size_t)(nleaf + 1));
        ctl = t.d_ctl.as<int32_t>();
        hctl = t.h_ctl.as<int32_t>();
        cnt = ws.cnt;
        leafbuf[0] = ws.pleaf;
        leafbuf[1] = ws.tleaf;
        qbuf[0] = ws.pq;
        qbuf[1] = ws.tq;
        tdense.on = tsparse.on = tfind.on = tgroup.on = tcopy.on = timing;
    }

    const int32_t *htiles() const { return t.h_tiles.as<int32_t>(); }
    const int32_t *hsparse() const { return t.h_tiles.as<int32_t>() + nleaf + 1; }
    const int32_t *hoff() const { return t.h_tiles.as<int32_t>() + 2 * (nleaf + 1); }

    void readback()
    {
        readback_issue();
        readback_wait();
    }

    void readback_issue()
    {
        BKD_HIP(hipMemcpyAsync(hctl, ctl, sizeof(int32_t) * CTL_WORDS, hipMemcpyDeviceToHost, s));
        BKD_HIP(hipEventRecord(t.ev_rb, s));
    }

    // Host-side wait for the device, counted in wait_ms.
    template <class F> void waiting(F &&f)
    {
        const auto w0 = std::chrono::steady_clock::now();
        f();
        wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
    }

    void readback_wait()
    {
        waiting([&] {
            for (;;) {
                const hipError_t e = hipEventQuery(t.ev_rb);
                if (e == hipSuccess) break;
                if (e != hipErrorNotReady) BKD_HIP(e);
            }
        });
        if (hctl[CTL_BAD]) fail(BKD_EINVAL, "query coordinates must be finite");
    }

    void find_leaf(const FetchSpec &f, int64_t base) { find_leaf_into(f, leafbuf[cur], qbuf[cur], base); }

    void find_leaf_into(const FetchSpec &f0, uint32_t *out_leaf, int32_t *out_q, int64_t base)
    {
        FetchSpec f = f0;
        f.dims = t.dims_dev();
        f.boxes = t.boxes_dev();
        tfind.begin(s);
        launch_find_leaf(f, dQ, d, ws.node, ws.kth, t.d_split.as<float>(), h,
                         out_leaf, out_q, base, cnt, ctl, s);
        tfind.end(s);
        t.stats.fetches++;
        const int64_t F = f.ring_count + f.in_count;
        if (tracing && F > 0) {
            tr_q.resize((size_t)F);
            tr_l.resize((size_t)F);
            BKD_HIP(hipMemcpyAsync(tr_q.data(), out_q + base, sizeof(int32_t) * F, hipMemcpyDeviceToHost, s));
            BKD_HIP(hipMemcpyAsync(tr_l.data(), out_leaf + base, sizeof(int32_t) * F, hipMemcpyDeviceToHost, s));
            waiting([&] { BKD_HIP(hipStreamSynchronize(s)); });
            for (int64_t j = 0; j < F; j++) {
                t.trace_q.push_back(tr_q[(size_t)j]);
                t.trace_leaf.push_back(tr_l[(size_t)j] == (uint32_t)nleaf ? -1 : (int32_t)tr_l[(size_t)j]);
            }
        }
    }

    // Sort the pending list, compute buffer offsets and work items, read the counters back.
    // With runs, the per-leaf counts come from the runs of the sorted list (the fetch
    // did not count); otherwise from the fetch's counters.
    // wait: read the control words back before returning (else the copy is only issued)
    // count_full: a resident round's grouping counts the work of scanning every buffer (false when
    // the round goes to the tail, which counts its own visits)
    void sort_and_offsets(int64_t count, bool runs = false, bool wait = true, bool count_full = true)
    {
        tgroup.begin(s);
        if (runs && !tracing && nleaf + 1 <= bucket_max_keys()) {
            // lock-step rounds: group by leaf in one pass (order within a buffer is free)
            const int nb = nleaf + 1;
            uint32_t *hist = ws.hist;
            const int32_t *counts = launch_bucket_count(leafbuf[cur], count, nb, hist, s);
            // a resident round scans every buffer: its work is counted here
            counted = t.resident && count_full;
            offsets(counts, nullptr, counted);
            launch_bucket_scatter(leafbuf[cur], qbuf[cur], leafbuf[1 - cur], qbuf[1 - cur], count, nb, hist,
                                  ws.off, s);
            cur = 1 - cur;
        } else {
            int which = launch_sort_pairs(leafbuf[cur], qbuf[cur], leafbuf[1 - cur], qbuf[1 - cur], count, kbits,
                                          ws.hist, s);
            if (which) cur = 1 - cur;
            int32_t *start = nullptr;
            if (runs) {
                start = ws.cnt0;
                launch_fill_i32(cnt, 0, nleaf, s);
                launch_fill_i32(start, 0, nleaf, s);
                launch_run_bounds(leafbuf[cur], count, nleaf, start, cnt, s);
            }
            counted = false;
            offsets(cnt, start, false);
        }
        tgroup.end(s);
        if (!t.resident) {
            BKD_HIP(hipMemcpyAsync(t.h_tiles.p, ws.tiles, sizeof(int32_t) * 2 * (size_t)(nleaf + 1),
                                   hipMemcpyDeviceToHost, s));
            BKD_HIP(hipMemcpyAsync(t.h_tiles.as<int32_t>() + 2 * (nleaf + 1), ws.off,
                                   sizeof(int32_t) * (size_t)(nleaf + 1), hipMemcpyDeviceToHost, s));
        }
        if (wait) readback();
        else readback_issue();
    }

    // Buffer offsets, work items and the pending count from per-leaf counts
    // (cnt, or end - start of each run when start is given).
    void offsets(const int32_t *counts, const int32_t *start, bool count_work)
    {
        launch_leaf_offsets(counts, start, t.d_leaf_off.as<int32_t>(), nleaf, SCAN_QT, t.dense_min,
                            ws.off, ws.tiles, ws.tiles + nleaf + 1, ctl,
                            s, count_work);
    }

    ScanArgs scan_args(const float *base, int64_t shift) const
    {
        ScanArgs a{};
        a.tiles = ws.tiles;
        a.sparse = a.tiles + nleaf + 1;
        a.off = ws.off;
        a.bufq = bufq_override ? bufq_override : qbuf[cur];
        a.leaf_off = t.d_leaf_off.as<int32_t>();
        a.base = base;
        a.blk = t.d_leaf_blk.as<int64_t>();
        a.blk_shift = shift;
        a.Q = dQ;
        a.d = d;
        a.keys = ws.keys;
        a.kth = ws.kth;
        a.k = k;
        a.centers = t.d_centers.as<float>();
        a.scales = a.centers + (size_t)nleaf * d;
        a.exact_only = t.wide ? 1 : 0;
        a.wide_flag = ctl + CTL_WIDE;
        a.dims = t.dims_dev();
        a.boxes = t.boxes_dev();
        return a;
    }

    void run_scan(const ScanArgs &a)
    {
        if (a.item_count > 0) {
            tdense.begin(s);
            launch_leaf_scan(a, K, 0, s);
            tdense.end(s);
            t.stats.dense_launches++;
        }
        if (a.sitem_count > 0) {
            tsparse.begin(s);
            launch_leaf_scan(a, K, 1, s);
            tsparse.end(s);
            t.stats.sparse_launches++;
        }
    }

    void count_work(int lf, int ll)
    {
        launch_count_work(ws.off, t.d_leaf_off.as<int32_t>(), lf, ll, t.dense_min, ctl, s);
    }

    // Scan every buffered query of a resident structure.
    void scan_resident()
    {
        if (!counted) count_work(0, nleaf - 1);
        ScanArgs a = scan_args(t.d_chunk[0].as<float>(), 0);
        a.chunk_lo = 0;
        a.chunk_hi = t.host.n;
        a.item_first = 0;
        a.item_count = hctl[CTL_T];
        a.sitem_first = 0;
        a.sitem_count = hctl[CTL_S];
        a.leaf_first = 0;
        a.leaf_last = nleaf - 1;
        run_scan(a);
    }

    // Scans of the pipelined rounds also route their queries (the next FindLeafBatch
    // step), in place in the sorted list, which the next round sorts again.
    void route_args(ScanArgs &a) const
    {
        a.route_leaf = leafbuf[cur];
        a.node = ws.node;
        a.split = t.d_split.as<float>();
        a.h = h;
    }

    // Dense scan of a resident round queued before its counts reach the host:
    // the item count is read on the device, the grid is bounded by the list
    // length (a dense leaf holds at least dense_min queries).
    void scan_resident_dense_ahead(int64_t list)
    {
        if (!counted) count_work(0, nleaf - 1);
        ScanArgs a = scan_args(t.d_chunk[0].as<float>(), 0);
        a.chunk_lo = 0;
        a.chunk_hi = t.host.n;
        a.item_first = 0;
        const int64_t bound = list / SCAN_QT + std::min<int64_t>(nleaf, list / std::max(1, t.dense_min)) + 1;
        a.item_count = (int32_t)std::min<int64_t>(bound, INT32_MAX);
        a.dev_counts = ctl;
        route_args(a);
        a.sitem_first = 0;
        a.sitem_count = 0;
        a.leaf_first = 0;
        a.leaf_last = nleaf - 1;
        run_scan(a);
    }

    // The sparse items of the same round, once their count is on the host.
    void scan_resident_sparse()
    {
        ScanArgs a = scan_args(t.d_chunk[0].as<float>(), 0);
        a.chunk_lo = 0;
        a.chunk_hi = t.host.n;
        a.item_first = 0;
        a.item_count = 0;
        route_args(a);
        a.sitem_first = 0;
        a.sitem_count = hctl[CTL_S];
        a.leaf_first = 0;
        a.leaf_last = nleaf - 1;
        run_scan(a);
    }

    int64_t chunk_items(int j) const
    {
        const Chunk &c = t.chunks[(size_t)j];
        return (htiles()[c.leaf_last + 1] - htiles()[c.leaf_first]) + (hsparse()[c.leaf_last + 1] - hsparse()[c.leaf_first]);
    }

    // Leaf file: start reading chunk j unless a device buffer already holds it.
    void prefetch(int j)
    {
        if (t.leaf_file && j >= 0 && t.chunk_in[0] != j && t.chunk_in[1] != j) leaffile_prefetch(t, j);
    }

    void issue_copy(int b, int j)
    {
        const Chunk &c = t.chunks[(size_t)j];
        const size_t bytes = (size_t)(c.word_hi - c.word_lo) * 4;
        BKD_HIP(hipStreamWaitEvent(t.copy_stream, t.ev_used[b], 0));
        tcopy.begin(t.copy_stream);
        if (t.leaf_file) {
            // disk -> staging (reader thread, usually prefetched) -> device
            wait_ms += leaffile_copy(t, j, t.d_chunk[b].p, t.copy_stream);
        } else {
            BKD_HIP(hipMemcpyAsync(t.d_chunk[b].p, t.h_leaf.as<float>() + c.word_lo, bytes, hipMemcpyHostToDevice,
                                   t.copy_stream));
        }
        tcopy.end(t.copy_stream);
        BKD_HIP(hipEventRecord(t.ev_copied[b], t.copy_stream));
        t.chunk_in[b] = j;
        t.stats.chunk_copies++;
        t.stats.bytes_h2d += (int64_t)bytes;
    }

    // Scan the buffered queries of chunk j's leaves; prefetch chunk nj (-1: none) into the other buffer.
    // Make chunk j resident (copy it unless a buffer holds it) and order the query stream
    // after its copy; returns the buffer.
    int chunk_buffer(int j, int nj)
    {
        int b = (t.chunk_in[0] == j) ? 0 : (t.chunk_in[1] == j) ? 1 : -1;
        if (b < 0) {
            b = (t.chunk_in[0] == nj) ? 1 : 0;
            issue_copy(b, j);
        }
        BKD_HIP(hipStreamWaitEvent(s, t.ev_copied[b], 0));
        return b;
    }

    // After the work on buffer b: record its use and prefetch chunk nj into the other buffer.
    void chunk_done(int b, int j, int nj)
    {
        BKD_HIP(hipEventRecord(t.ev_used[b], s));
        if (nj >= 0 && nj != j && t.chunk_in[1 - b] != nj) issue_copy(1 - b, nj);
    }

    // Drain the n pending entries (Rl, Rq) of resident chunk j with the tail kernel: each query
    // walks on while its next leaf lies in j and leaves in its entry the first leaf outside j
    // (or the finished sentinel).
    void tail_chunk(int j, int nj, uint32_t *Rl, int32_t *Rq, int64_t n)
    {
        const int b = chunk_buffer(j, nj);
        const Chunk &c = t.chunks[(size_t)j];
        ScanArgs a = scan_args(t.d_chunk[b].as<float>(), -c.word_lo);
        a.leaf_first = c.leaf_first;
        a.leaf_last = c.leaf_last;
        a.tail_leaf = Rl;
        a.tail_q = Rq;
        a.tail_count = (int32_t)n;
        a.tail_wide = (t.host.n >> h) >= TAIL_WIDE_LEAF;
        a.route_leaf = Rl;
        a.node = ws.node;
        a.split = t.d_split.as<float>();
        a.h = h;
        a.ctl = ctl;
        tsparse.begin(s);
        launch_leaf_scan(a, K, 2, s);
        tsparse.end(s);
        t.stats.sparse_launches++;
        chunk_done(b, j, nj);
    }

    void scan_chunk(int j, int nj)
    {
        const int b = chunk_buffer(j, nj);
        const Chunk &c = t.chunks[(size_t)j];
        ScanArgs a = scan_args(t.d_chunk[b].as<float>(), -c.word_lo);
        a.chunk_lo = c.lo;
        a.chunk_hi = c.hi;
        a.leaf_first = c.leaf_first;
        a.leaf_last = c.leaf_last;
        a.item_first = htiles()[c.leaf_first];
        a.item_count = htiles()[c.leaf_last + 1] - htiles()[c.leaf_first];
        a.sitem_first = hsparse()[c.leaf_first];
        a.sitem_count = hsparse()[c.leaf_last + 1] - hsparse()[c.leaf_first];
        if (route_override) {
            // every query of the chunk's region is scanned once here and takes its next
            // FindLeafBatch step at the end of its scan, written into its list position
            a.route_leaf = route_override;
            a.node = ws.node;
            a.split = t.d_split.as<float>();
            a.h = h;
        }
        run_scan(a);
        chunk_done(b, j, nj);
    }

    // ProcessAllBuffers over a streamed structure: every chunk holding a buffered leaf, in order.
    void scan_all_chunks()
    {
        count_work(0, nleaf - 1);
        std::vector<int> active;
        for (int j = 0; j < (int)t.chunks.size(); j++)
            if (chunk_items(j) > 0) active.push_back(j);
        for (size_t ai = 0; ai < active.size(); ai++) {
            // read ahead from the leaf file: the next chunks of the walk
            for (size_t x = ai + 1; x < std::min(active.size(), ai + 3); x++) prefetch(active[x]);
            scan_chunk(active[ai], ai + 1 < active.size() ? active[ai + 1] : 0);
        }
    }

    void end_call()
    {
        t.stats.calls++;
        if (tracing) t.trace_off.push_back((int64_t)t.trace_q.size());
    }

    // ---------------------------------------------------------------- Algorithm 1
    void algorithm1()
    {
        const int64_t M = t.M < 0 ? INT64_MAX : t.M;
        const int64_t half = t.B > 0 ? (t.B + 1) / 2 : INT64_MAX;
        int64_t in_head = 0, re_head = 0, re_len = 0, pend = 0;
        while (in_head < m || re_len > 0) {
            const int64_t take_re = std::min(M, re_len);
            const int64_t take_in = std::min(M - take_re, m - in_head);
            FetchSpec f{ws.ring, re_head, take_re, m, in_head, take_in};
            f.track_fill = true;
            find_leaf(f, pend);
            pend += take_re + take_in;
            re_head = (re_head + take_re) % m;
            re_len -= take_re;
            in_head += take_in;
            const bool queues_empty = (in_head == m && re_len == 0);
            bool trigger = queues_empty;
            if (!trigger) {
                readback();
                trigger = hctl[CTL_MAXCNT] >= half;
            }
            if (!trigger) continue;
            // ---- ProcessAllBuffers ----
            sort_and_offsets(pend);
            const int64_t V = hctl[CTL_V];
            if (hctl[CTL_T] + hctl[CTL_S] > 0) {
                if (t.resident) scan_resident();
                else scan_all_chunks();
            }
            launch_ring_append(ws.ring, m, (re_head + re_len) % m, qbuf[cur], V, s);
            re_len += V;
            launch_fill_i32(cnt, 0, nleaf, s);
            launch_fill_i32(ctl + CTL_MAXCNT, 0, 2, s);
            pend = 0;
            end_call();
        }
    }

    // ---------------------------------------------------------------- lock-step rounds
    void lockstep()
    {
        // first round: every query descends from the root
        FetchSpec f0{nullptr, 0, 0, 1, 0, m};
        f0.count_leaves = false;  // per-leaf counts come from the sorted runs
        find_leaf(f0, 0);
        if (t.sweep) {
            sweep();
            return;
        }
        int64_t P = m;  // pending entries (leaf order after each sort; finished ones sort last)
        bool first = true;
        const int64_t tail_max = t.opt.tail_max == 0 ? TAIL_MAX : t.opt.tail_max;
        const bool use_tail = !(t.opt.flags & BKD_FLAG_NO_TAIL);
        if (t.resident && !tracing && !t.dims_dev() && !t.boxes_dev()) {
            // Resident rounds without a host wait before the scan: the dense scan of a round is
            // queued behind its sort and reads its item count on the device, and the host reads
            // the round's counts back meanwhile.  The tail takes over once a round's list (the
            // pending entries routed in the previous round) is at most tail_max long.
            for (;;) {
                const int64_t list = P;
                const bool tail_now = use_tail && list <= tail_max;
                sort_and_offsets(list, true, false, !tail_now);
                if (first) localize();
                first = false;
                if (!tail_now) scan_resident_dense_ahead(list);
                readback_wait();
                P = hctl[CTL_V];
                if (P == 0) {
                    end_call();
                    break;
                }
                if (tail_now) {
                    tail(P);
                    end_call();
                    break;
                }
                if (hctl[CTL_S] > 0) scan_resident_sparse();
                end_call();
                t.stats.fetches++;  // the scans routed every pending query
            }
            return;
        }
        for (;;) {
            sort_and_offsets(P, true);
            P = hctl[CTL_V];
            if (P == 0) {
                end_call();
                break;
            }
            if (first && !tracing) localize();
            first = false;
            if (t.resident && !tracing && use_tail && P <= tail_max) {
                tail(P);
                end_call();
                break;
            }
            if (t.resident) scan_resident();
            else scan_all_chunks();
            end_call();
            FetchSpec f{qbuf[cur], 0, P, std::max<int64_t>(P, 1), 0, 0};
            f.count_leaves = false;
            find_leaf(f, 0);
        }
    }

    // The P pending entries (sorted, all live) finish their traversals in the tail kernel.
    void tail(int64_t P)
    {
        ScanArgs a = scan_args(t.d_chunk[0].as<float>(), 0);
        a.tail_leaf = leafbuf[cur];
        a.tail_q = qbuf[cur];
        a.tail_count = (int32_t)P;
        a.tail_wide = (t.host.n >> h) >= TAIL_WIDE_LEAF;
        a.tail_counted = counted ? 1 : 0;
        a.node = ws.node;
        a.split = t.d_split.as<float>();
        a.h = h;
        a.k = k;
        a.ctl = ctl;
        tsparse.begin(s);
        launch_leaf_scan(a, K, 2, s);
        tsparse.end(s);
        t.stats.sparse_launches++;
    }

    // Renumber the queries in first-leaf order (the pending list right after the
    // first sort), so that the queries of one buffer have neighbouring numbers.
    // Results are independent of numbering; traces keep the caller's numbers.
    void localize()
    {
        launch_localize(qbuf[cur], leafbuf[cur], m, d, dQ, ws.Qp, ws.perm,
                        ws.node, h, s);
        dQ = ws.Qp;
        perm = ws.perm;
    }

    // Chunk sweep over a streamed, leaf-aligned structure.  Pending entries live in one
    // region per chunk; a step sorts only the region of the resident chunk c, scans it,
    // routes its queries again and moves each entry to the region of its next chunk.
    // The sweep stays on c while c holds at least a quarter of the average pending
    // share, then moves on (cyclically) to the next chunk above that mark, whose copy
    // was prefetched meanwhile.
    void sweep()
    {
        const int N = (int)t.chunks.size();
        t.d_rleaf.ensure(sizeof(uint32_t) * (size_t)N * m);
        t.d_rq.ensure(sizeof(int32_t) * (size_t)N * m);
        t.d_rcnt.ensure(sizeof(int32_t) * (N + 1));
        t.h_rcnt.ensure(sizeof(int32_t) * (N + 1));
        uint32_t *rleaf = t.d_rleaf.as<uint32_t>();
        int32_t *rq = t.d_rq.as<int32_t>();
        int32_t *rcnt = t.d_rcnt.as<int32_t>();
        int32_t *hr = t.h_rcnt.as<int32_t>();
        const int32_t *chunk_of = t.d_chunk_of.as<int32_t>();
        // a chunk's pending queries go to the tail kernel at the chunk's share of tail_max: a tail
        // query reads each of its leaves alone, which pays only for a few queries per chunk
        const int64_t tail_max = std::max<int64_t>(1, (t.opt.tail_max == 0 ? TAIL_MAX : t.opt.tail_max) / N);
        const bool use_tail = !tracing && !(t.opt.flags & BKD_FLAG_NO_TAIL) && t.opt.tail_max >= 0;
        uint32_t *sleaf = leafbuf[1 - cur];
        int32_t *sq = qbuf[1 - cur];
        // the scans route their queries themselves (original splitting rule, untraced)
        const bool scan_routes = !tracing && !t.dims_dev() && !t.boxes_dev();
        auto read_counts = [&]() {
            BKD_HIP(hipMemcpyAsync(hr, rcnt, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost, s));
            readback();
        };
        tgroup.begin(s);
        launch_fill_i32(rcnt, 0, N + 1, s);
        launch_distribute(leafbuf[cur], qbuf[cur], m, nleaf, chunk_of, -1, rleaf, rq, m, rcnt, sleaf, sq, N, s);
        tgroup.end(s);
        read_counts();
        int c = -1;
        for (;;) {
            int64_t total = 0, best = -1;
            for (int j = 0; j < N; j++) {
                total += hr[j];
                if (best < 0 || hr[j] > hr[best]) best = j;
            }
            if (total == 0) {
                end_call();
                break;
            }
            const int64_t mark = std::max<int64_t>(1, total / N / 4);
            auto next_from = [&](int from, int skip) {
                for (int x = 1; x <= N; x++) {
                    const int j = ((from < 0 ? -1 : from) + x + N) % N;
                    if (j != skip && hr[j] >= mark) return j;
                }
                int b = -1;
                for (int j = 0; j < N; j++)
                    if (j != skip && hr[j] > 0 && (b < 0 || hr[j] > hr[b])) b = j;
                return b;
            };
            if (c < 0 || hr[c] < mark) c = next_from(c, -1);
            const int nc = next_from(c, c);
            // from a leaf file: read c (if not on the device) and the chunk after it while c is
            // sorted, scanned and routed
            prefetch(c);
            prefetch(nc);
            const Chunk &C = t.chunks[(size_t)c];
            const int lf = C.leaf_first, ll = C.leaf_last, nl = ll - lf + 1;
            const int64_t n = hr[c];
            uint32_t *Rl = rleaf + (int64_t)c * m;
            int32_t *Rq = rq + (int64_t)c * m;
            if (use_tail && n <= tail_max) {
                // few queries left in c: the tail kernel drains the chunk in one launch
                tail_chunk(c, nc, Rl, Rq, n);
                end_call();
                tgroup.begin(s);
                launch_distribute(Rl, Rq, n, nleaf, chunk_of, c, rleaf, rq, m, rcnt, sleaf, sq, N, s);
                launch_restore(sleaf, sq, n, Rl, Rq, rcnt, c, N, s);
                launch_fill_i32(rcnt + N, 0, 1, s);
                tgroup.end(s);
                read_counts();
                continue;
            }
            // Steps on c, pipelined: a step's grouping and its dense scan are queued before the
            // host has its counts (read back ahead of the dense scan), and from the second step
            // on they take the region's size on the device (the previous step's distribution),
            // so the host queues a step's sparse scan and distribution, and the next step, while
            // the dense scan runs.  The host sees a region's size one step late, so it may stay
            // on c for one step more than the mark asks.
            int64_t nstep = n;               // bound on the size of the step being queued
            const int32_t *dstep = nullptr;  // its size on the device (from the second step on)
            for (;;) {
                tgroup.begin(s);
                int32_t *dtiles = ws.tiles;
                if (!tracing && nl <= bucket_max_keys()) {
                    // one pass: per-leaf counts of the region (keys relative to the chunk's
                    // first leaf), the offsets, a scatter by leaf (order within a leaf free, as
                    // in resident rounds), copied back into the region
                    const int32_t *counts = launch_bucket_count(Rl, nstep, nl, ws.hist, s, (uint32_t)lf, dstep);
                    launch_leaf_offsets(counts, nullptr, t.d_leaf_off.as<int32_t>() + lf, nl, SCAN_QT, t.dense_min,
                                        ws.off + lf, dtiles + lf, dtiles + nleaf + 1 + lf, ctl, s);
                    launch_bucket_scatter(Rl, Rq, sleaf, sq, nstep, nl, ws.hist, ws.off + lf, s, (uint32_t)lf, dstep);
                    BKD_HIP(hipMemcpyAsync(Rl, sleaf, sizeof(uint32_t) * nstep, hipMemcpyDeviceToDevice, s));
                    BKD_HIP(hipMemcpyAsync(Rq, sq, sizeof(int32_t) * nstep, hipMemcpyDeviceToDevice, s));
                } else {
                    if (launch_sort_pairs(Rl, Rq, sleaf, sq, nstep, kbits, ws.hist, s, dstep)) {
                        BKD_HIP(hipMemcpyAsync(Rl, sleaf, sizeof(uint32_t) * nstep, hipMemcpyDeviceToDevice, s));
                        BKD_HIP(hipMemcpyAsync(Rq, sq, sizeof(int32_t) * nstep, hipMemcpyDeviceToDevice, s));
                    }
                    int32_t *start = ws.cnt0;
                    launch_fill_i32(cnt + lf, 0, nl, s);
                    launch_fill_i32(start + lf, 0, nl, s);
                    launch_run_bounds(Rl, nstep, nleaf, start, cnt, s, dstep);
                    launch_leaf_offsets(cnt + lf, start + lf, t.d_leaf_off.as<int32_t>() + lf, nl, SCAN_QT,
                                        t.dense_min, ws.off + lf, dtiles + lf, dtiles + nleaf + 1 + lf, ctl, s);
                }
                tgroup.end(s);
                count_work(lf, ll);
                // this step's counts, and every region's size before its distribution: read back
                // while the dense scan (queued next) runs
                BKD_HIP(hipMemcpyAsync(hr, rcnt, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost, s));
                readback_issue();
                const int bb = chunk_buffer(c, nc);
                ScanArgs a = scan_args(t.d_chunk[bb].as<float>(), -C.word_lo);
                a.bufq = Rq;
                a.chunk_lo = C.lo;
                a.chunk_hi = C.hi;
                a.leaf_first = lf;
                a.leaf_last = ll;
                a.item_first = 0;  // the chunk's work items are numbered from its first leaf
                a.item_count = (int32_t)std::min<int64_t>(
                    nstep / SCAN_QT + std::min<int64_t>(nl, nstep / std::max(1, t.dense_min)) + 1, INT32_MAX);
                a.dev_counts = ctl;
                a.sitem_first = 0;
                a.sitem_count = 0;
                if (scan_routes) {
                    // every query of the region is scanned once in this step and takes its next
                    // FindLeafBatch step at the end of its scan, written into its list position
                    a.route_leaf = Rl;
                    a.node = ws.node;
                    a.split = t.d_split.as<float>();
                    a.h = h;
                }
                run_scan(a);
                readback_wait();
                const int64_t nthis = hr[c];
                a.dev_counts = nullptr;
                a.item_count = 0;
                a.sitem_count = hctl[CTL_S];
                run_scan(a);
                chunk_done(bb, c, nc);
                end_call();
                if (!scan_routes) {
                    FetchSpec f{Rq, 0, nthis, std::max<int64_t>(nthis, 1), 0, 0};
                    f.count_leaves = false;
                    find_leaf_into(f, Rl, Rq, 0);
                } else {
                    t.stats.fetches++;
                }
                // move every entry to the region of its next chunk
                tgroup.begin(s);
                launch_distribute(Rl, Rq, nthis, nleaf, chunk_of, c, rleaf, rq, m, rcnt, sleaf, sq, N, s);
                launch_restore(sleaf, sq, nthis, Rl, Rq, rcnt, c, N, s);
                launch_fill_i32(rcnt + N, 0, 1, s);
                tgroup.end(s);
                int64_t tot = 0;
                for (int j = 0; j < N; j++) tot += hr[j];
                if (nthis < std::max<int64_t>(1, tot / N / 4) || (use_tail && nthis <= tail_max)) break;
                nstep = nthis;
                dstep = rcnt + c;
            }
            read_counts();
        }
    }
};

}  // namespace

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The workspace's arrays in order, with their sizes for m queries of key capacity K.
template <class F> static void workspace_layout(const Tree &t, int64_t m, int k, F &&place)
{
    const size_t M = (size_t)m, L = (size_t)t.nleaf;
    const size_t K = (size_t)key_capacity(k), d = (size_t)t.host.d;
    place(0, sizeof(uint64_t) * M * K);                  // keys
    place(1, sizeof(uint32_t) * M);                      // kth
    place(2, sizeof(int32_t) * M);                       // node
    place(3, sizeof(int32_t) * M);                       // ring
    place(4, sizeof(uint32_t) * M);                      // pleaf
    place(5, sizeof(uint32_t) * M);                      // tleaf
    place(6, sizeof(int32_t) * M);                       // pq
    place(7, sizeof(int32_t) * M);                       // tq
    place(8, sizeof(uint32_t) * sort_hist_words(m));     // hist
    place(9, sizeof(int32_t) * L);                       // cnt
    place(10, sizeof(int32_t) * L);                      // cnt0
    place(11, sizeof(int32_t) * (L + 1));                // off
    place(12, sizeof(int32_t) * 2 * (L + 1));            // tiles
    place(13, sizeof(float) * M * d);                    // Qp
    place(14, sizeof(int32_t) * M);                      // perm
}

static Workspace workspace_from(void *const (&p)[15])
{
    Workspace w;
    w.keys = static_cast<uint64_t *>(p[0]);
    w.kth = static_cast<uint32_t *>(p[1]);
    w.node = static_cast<int32_t *>(p[2]);
    w.ring = static_cast<int32_t *>(p[3]);
    w.pleaf = static_cast<uint32_t *>(p[4]);
    w.tleaf = static_cast<uint32_t *>(p[5]);
    w.pq = static_cast<int32_t *>(p[6]);
    w.tq = static_cast<int32_t *>(p[7]);
    w.hist = static_cast<uint32_t *>(p[8]);
    w.cnt = static_cast<int32_t *>(p[9]);
    w.cnt0 = static_cast<int32_t *>(p[10]);
    w.off = static_cast<int32_t *>(p[11]);
    w.tiles = static_cast<int32_t *>(p[12]);
    w.Qp = static_cast<float *>(p[13]);
    w.perm = static_cast<int32_t *>(p[14]);
    return w;
}

size_t workspace_bytes(const Tree &t, int64_t m, int k)
{
    size_t total = 0;
    workspace_layout(t, m, k, [&](int, size_t b) { total += align256(b); });
    return total;
}

Workspace workspace_in(const Tree &t, int64_t m, int k, void *region)
{
    void *p[15];
    size_t off = 0;
    workspace_layout(t, m, k, [&](int i, size_t b) {
        p[i] = static_cast<char *>(region) + off;
        off += align256(b);
    });
    return workspace_from(p);
}

// The tree's own workspace: one device buffer per array, grown on demand.
static Workspace tree_workspace(Tree &t, int64_t m, int k)
{
    DevBuf *bufs[15] = {&t.d_keys, &t.d_kth, &t.d_node, &t.d_ring, &t.d_pleaf, &t.d_tleaf, &t.d_pq, &t.d_tq,
                        &t.d_hist, &t.d_cnt, &t.d_cnt0, &t.d_off, &t.d_tiles, &t.d_Qp, &t.d_perm};
    void *p[15];
    workspace_layout(t, m, k, [&](int i, size_t b) {
        bufs[i]->ensure(b);
        p[i] = bufs[i]->p;
    });
    return workspace_from(p);
}

void tree_query_device(Tree &t, const float *dQ, int64_t m, int k, int64_t *d_idx, float *d_dist, hipStream_t s,
                       void *region)
{
    auto t0 = std::chrono::steady_clock::now();
    BKD_HIP(hipSetDevice(t.device));
    t.stats = bkd_stats{};
    t.stats.queries = m;
    t.trace_off.assign(1, 0);
    t.trace_q.clear();
    t.trace_leaf.clear();
    if (m == 0) return;
    if (region && (!t.resident || (t.opt.flags & BKD_FLAG_TRACE)))
        fail(BKD_EINVAL, "a query in a caller-provided workspace needs a resident structure and no trace");

    const Workspace ws = region ? workspace_in(t, m, k, region) : tree_workspace(t, m, k);
    Run r(t, s, dQ, m, k, ws, !region && (t.opt.flags & BKD_FLAG_TIMING) != 0);
    launch_fill_i32(r.ctl, 0, CTL_WORDS, s);
    launch_fill_i32(r.cnt, 0, t.nleaf, s);
    launch_check_finite(dQ, m * t.host.d, r.ctl, s);
    launch_init_state(ws.node, ws.keys, ws.kth, m, r.K, s);
    if (t.M < 0) r.lockstep();
    else r.algorithm1();
    launch_finalize(ws.keys, r.K, k, m, r.perm, d_idx, d_dist, (t.opt.flags & BKD_FLAG_SQUARED) != 0, s);
    r.readback();
    std::memcpy(&t.stats.visits, r.hctl + CTL_VISITS_LO, 8);
    std::memcpy(&t.stats.dense_pairs, r.hctl + CTL_DPAIRS_LO, 8);
    std::memcpy(&t.stats.sparse_pairs, r.hctl + CTL_SPAIRS_LO, 8);
    t.stats.pairs = t.stats.dense_pairs + t.stats.sparse_pairs;
    std::memcpy(&t.stats.dense_visits, r.hctl + CTL_DVISITS_LO, 8);
    std::memcpy(&t.stats.leaf_points_dense, r.hctl + CTL_LPD_LO, 8);
    std::memcpy(&t.stats.leaf_points_other, r.hctl + CTL_LPS_LO, 8);
    {
        // algorithmic bytes: every buffered leaf once per call, and per visit the query, its
        // key list (read and written) and its buffer entry
        const int64_t per_point = 4 * (int64_t)t.host.d + 4, per_visit = 4 * (int64_t)t.host.d + 16 * (int64_t)k + 4;
        t.stats.alg_bytes = (t.stats.leaf_points_dense + t.stats.leaf_points_other) * per_point +
                            t.stats.visits * per_visit;
        t.stats.alg_bytes_dense = t.stats.leaf_points_dense * per_point + t.stats.dense_visits * per_visit;
    }
    if (r.tdense.on) {
        t.stats.dense_ms = r.tdense.total_ms();
        t.stats.sparse_ms = r.tsparse.total_ms();
        t.stats.find_ms = r.tfind.total_ms();
        t.stats.group_ms = r.tgroup.total_ms();
        t.stats.copy_ms = r.tcopy.total_ms();
    }
    t.stats.wait_ms = r.wait_ms;
    if (t.leaf_file) leaffile_take_stats(t, &t.stats.bytes_disk, &t.stats.disk_ms);
    t.stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace bkd
