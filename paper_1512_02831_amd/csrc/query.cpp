// query.cpp -- tree upload, streaming plan and the query loop of Algorithm 1.
//
// The loop keeps the paper's queues on the device: `input` is the range of
// not yet fetched query ids, `reinsert` a FIFO ring.  Each iteration fetches
// up to M ids (reinsert first), runs FindLeafBatch, appends the (leaf, query)
// pairs to the pending list (the pooled buffers, in fetch order), and reads
// back the largest buffer fill.  When a buffer is half-full or both queues are
// empty, ProcessAllBuffers runs: a stable sort groups the pending pairs by
// leaf (the buffers' contents in insertion order), one leaf-scan launch per
// needed chunk updates every buffered query's list, and the buffered ids are
// appended to reinsert in ascending leaf order.
//
// Streaming (Section 3.2): with a leaf budget, the leaf structure stays in
// pinned host memory in chunk-major blocks and passes through two device
// chunk buffers.  The copy of the next chunk runs on a second stream while
// the scan of the current chunk runs on the caller's stream; events order
// each copy after the last scan that read its buffer and each scan after its
// copy (the paper's Brute / Copy / Wait with two command queues, without
// blocking the host).  Chunks holding no buffered leaf are skipped, and after
// the last chunk of a call the first chunk is prefetched for the next call.
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
    const size_t bpp = (size_t)(4 * H.d + 4);
    const size_t total = (size_t)n * bpp;
    int64_t maxleaf = 0;
    for (int l = 0; l < t.nleaf; l++) maxleaf = std::max(maxleaf, H.leaf_off[l + 1] - H.leaf_off[l]);
    const int64_t budget = t.opt.leaf_budget_bytes;
    if (budget < 0) fail(BKD_EINVAL, "leaf_budget_bytes must be >= 0");
    if (t.opt.num_chunks < 0) fail(BKD_EINVAL, "num_chunks must be >= 0");
    if (t.opt.chunk_mode != BKD_CHUNK_LEAF && t.opt.chunk_mode != BKD_CHUNK_POSITION)
        fail(BKD_EINVAL, "unknown chunk_mode");
    t.chunks.clear();
    t.resident = (t.opt.num_chunks == 0) && (budget == 0 || (size_t)budget >= total);
    if (t.resident) {
        t.chunks.push_back(Chunk{0, n, 0, t.nleaf - 1, 0, total});
        t.chunk_cap_points = n;
        t.chunk_cap_bytes = total;
        return;
    }
    if (budget > 0 && (size_t)budget < 2 * (size_t)maxleaf * bpp)
        fail(BKD_EBUDGET, "leaf budget of " + std::to_string(budget) + " bytes is below two leaves (" +
                              std::to_string(2 * (size_t)maxleaf * bpp) + " bytes)");
    const size_t cap_bytes = budget > 0 ? (size_t)budget / 2 : total;
    std::vector<std::pair<int64_t, int64_t>> ranges;  // positions
    if (t.opt.chunk_mode == BKD_CHUNK_POSITION) {
        int64_t N = t.opt.num_chunks > 0 ? t.opt.num_chunks
                                         : (int64_t)((total + cap_bytes - 1) / cap_bytes);
        N = std::max<int64_t>(1, std::min<int64_t>(N, n));
        for (int64_t j = 1; j <= N; j++) ranges.emplace_back(((j - 1) * n + N - 1) / N, (j * n + N - 1) / N);
        if (budget > 0) {
            for (auto &r : ranges)
                if ((size_t)(r.second - r.first) * bpp > cap_bytes)
                    fail(BKD_EBUDGET, "forced chunk count exceeds the leaf budget");
        }
    } else if (t.opt.num_chunks > 0) {
        // whole leaves, the leaf index range split by the same ceiling rule
        int64_t N = std::min<int64_t>(t.opt.num_chunks, t.nleaf);
        for (int64_t j = 1; j <= N; j++) {
            int64_t a = ((j - 1) * t.nleaf + N - 1) / N, b = (j * t.nleaf + N - 1) / N;
            ranges.emplace_back(H.leaf_off[a], H.leaf_off[b]);
            if (budget > 0 && (size_t)(H.leaf_off[b] - H.leaf_off[a]) * bpp > cap_bytes)
                fail(BKD_EBUDGET, "forced chunk count exceeds the leaf budget");
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
    size_t off = 0;
    int64_t cap = 0;
    for (auto &r : ranges) {
        Chunk c;
        c.lo = r.first;
        c.hi = r.second;
        // leaves overlapping [lo, hi)
        c.leaf_first = (int32_t)(std::upper_bound(H.leaf_off.begin(), H.leaf_off.end(), c.lo) - H.leaf_off.begin() - 1);
        c.leaf_last = (int32_t)(std::upper_bound(H.leaf_off.begin(), H.leaf_off.end(), c.hi - 1) - H.leaf_off.begin() - 1);
        c.host_offset = off;
        c.bytes = (size_t)(c.hi - c.lo) * bpp;
        off += (c.bytes + 255) & ~(size_t)255;
        cap = std::max(cap, c.hi - c.lo);
        t.chunks.push_back(c);
    }
    t.chunk_cap_points = cap;
    t.chunk_cap_bytes = (size_t)cap * bpp;
}

// Write positions [lo, hi) of the leaf structure as [d][hi-lo] floats then [hi-lo] int32.
static void gather_block(const float *P, const HostTree &H, int64_t lo, int64_t hi, void *dst)
{
    const int d = H.d;
    const int64_t len = hi - lo;
    float *X = static_cast<float *>(dst);
    int32_t *orig = reinterpret_cast<int32_t *>(X + (size_t)d * len);
    parallel_for(len, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; i++) {
            int32_t o = H.perm[(size_t)(lo + i)];
            const float *p = P + (int64_t)o * d;
            for (int j = 0; j < d; j++) X[(size_t)j * len + i] = p[j];
            orig[i] = o;
        }
    }, 4096);
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

    build_canonical(P, n, d, h, t.host);
    plan_chunks(t);

    const HostTree &H = t.host;
    t.d_split.ensure(sizeof(float) * std::max<size_t>(1, H.split.size()));
    if (!H.split.empty())
        BKD_HIP(hipMemcpy(t.d_split.p, H.split.data(), sizeof(float) * H.split.size(), hipMemcpyHostToDevice));
    std::vector<int32_t> lo32(H.leaf_off.size());
    for (size_t i = 0; i < lo32.size(); i++) lo32[i] = (int32_t)H.leaf_off[i];
    t.d_leaf_off.ensure(sizeof(int32_t) * lo32.size());
    BKD_HIP(hipMemcpy(t.d_leaf_off.p, lo32.data(), sizeof(int32_t) * lo32.size(), hipMemcpyHostToDevice));

    if (t.resident) {
        std::vector<char> blk(t.chunks[0].bytes);
        gather_block(P, H, 0, n, blk.data());
        t.d_chunk[0].ensure(blk.size());
        BKD_HIP(hipMemcpy(t.d_chunk[0].p, blk.data(), blk.size(), hipMemcpyHostToDevice));
        t.chunk_in[0] = 0;
    } else {
        const Chunk &lastc = t.chunks.back();
        t.h_leaf.ensure(lastc.host_offset + lastc.bytes);
        for (const Chunk &c : t.chunks) gather_block(P, H, c.lo, c.hi, static_cast<char *>(t.h_leaf.p) + c.host_offset);
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
    }
    t.d_ctl.ensure(sizeof(int32_t) * CTL_WORDS);
    t.h_ctl.ensure(sizeof(int32_t) * CTL_WORDS);
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

// Copy chunk j into device buffer b on the copy stream, after the last scan that read b.
void issue_copy(Tree &t, int b, int j)
{
    const Chunk &c = t.chunks[(size_t)j];
    BKD_HIP(hipStreamWaitEvent(t.copy_stream, t.ev_used[b], 0));
    BKD_HIP(hipMemcpyAsync(t.d_chunk[b].p, static_cast<char *>(t.h_leaf.p) + c.host_offset, c.bytes,
                           hipMemcpyHostToDevice, t.copy_stream));
    BKD_HIP(hipEventRecord(t.ev_copied[b], t.copy_stream));
    t.chunk_in[b] = j;
    t.stats.chunk_copies++;
    t.stats.bytes_h2d += (int64_t)c.bytes;
}

}  // namespace

void tree_query_device(Tree &t, const float *dQ, int64_t m, int k, int64_t *d_idx, float *d_dist, hipStream_t s)
{
    auto t0 = std::chrono::steady_clock::now();
    BKD_HIP(hipSetDevice(t.device));
    t.stats = bkd_stats{};
    t.stats.queries = m;
    t.trace_off.assign(1, 0);
    t.trace_q.clear();
    t.trace_leaf.clear();
    const bool tracing = (t.opt.flags & BKD_FLAG_TRACE) != 0;
    if (m == 0) return;

    const HostTree &H = t.host;
    const int d = H.d, h = H.h, nleaf = t.nleaf;
    const int K = key_capacity(k);
    t.d_keys.ensure(sizeof(uint64_t) * (size_t)m * K);
    t.d_node.ensure(sizeof(int32_t) * (size_t)m);
    t.d_ring.ensure(sizeof(int32_t) * (size_t)m);
    t.d_pleaf.ensure(sizeof(uint32_t) * (size_t)m);
    t.d_pq.ensure(sizeof(int32_t) * (size_t)m);
    t.d_tleaf.ensure(sizeof(uint32_t) * (size_t)m);
    t.d_tq.ensure(sizeof(int32_t) * (size_t)m);
    t.d_hist.ensure(sizeof(uint32_t) * sort_hist_words(m));
    t.d_cnt.ensure(sizeof(int32_t) * (size_t)nleaf);
    t.d_off.ensure(sizeof(int32_t) * (size_t)(nleaf + 1));
    t.d_tiles.ensure(sizeof(int32_t) * 2 * (size_t)(nleaf + 1));
    if (!t.resident) t.h_tiles.ensure(sizeof(int32_t) * 2 * (size_t)(nleaf + 1));

    int32_t *ctl = t.d_ctl.as<int32_t>();
    int32_t *hctl = t.h_ctl.as<int32_t>();
    int32_t *cnt = t.d_cnt.as<int32_t>();
    launch_fill_i32(ctl, 0, CTL_WORDS, s);
    launch_fill_i32(cnt, 0, nleaf, s);
    launch_check_finite(dQ, m * d, ctl, s);
    launch_init_state(t.d_node.as<int32_t>(), t.d_keys.as<uint64_t>(), m, K, s);

    Timer timer;
    timer.on = (t.opt.flags & BKD_FLAG_TIMING) != 0;
    const int64_t M = t.M < 0 ? INT64_MAX : t.M;
    const int64_t half = t.B > 0 ? (t.B + 1) / 2 : INT64_MAX;
    const int kbits = key_bits_for(nleaf);
    const size_t bpp = (size_t)(4 * d + 4);

    auto readback = [&](size_t words) {
        BKD_HIP(hipMemcpyAsync(hctl, ctl, sizeof(int32_t) * words, hipMemcpyDeviceToHost, s));
        BKD_HIP(hipStreamSynchronize(s));
        if (hctl[CTL_BAD]) fail(BKD_EINVAL, "query coordinates must be finite");
    };

    int64_t in_head = 0, re_head = 0, re_len = 0, pend = 0;
    std::vector<int32_t> tr_q, tr_l;
    while (in_head < m || re_len > 0) {
        const int64_t take_re = std::min(M, re_len);
        const int64_t take_in = std::min(M - take_re, m - in_head);
        const int64_t F = take_re + take_in;
        FetchSpec f{t.d_ring.as<int32_t>(), re_head, take_re, m, in_head, take_in};
        launch_find_leaf(f, dQ, d, t.d_node.as<int32_t>(), t.d_keys.as<uint64_t>(), K, k, t.d_split.as<float>(), h,
                         t.d_pleaf.as<uint32_t>(), t.d_pq.as<int32_t>(), pend, cnt, ctl, s);
        t.stats.fetches++;
        if (tracing && F > 0) {
            tr_q.resize((size_t)F);
            tr_l.resize((size_t)F);
            BKD_HIP(hipMemcpyAsync(tr_q.data(), t.d_pq.as<int32_t>() + pend, sizeof(int32_t) * F,
                                   hipMemcpyDeviceToHost, s));
            BKD_HIP(hipMemcpyAsync(tr_l.data(), t.d_pleaf.as<uint32_t>() + pend, sizeof(int32_t) * F,
                                   hipMemcpyDeviceToHost, s));
            BKD_HIP(hipStreamSynchronize(s));
            for (int64_t j = 0; j < F; j++) {
                t.trace_q.push_back(tr_q[(size_t)j]);
                t.trace_leaf.push_back(tr_l[(size_t)j] == (uint32_t)nleaf ? -1 : tr_l[(size_t)j]);
            }
        }
        pend += F;
        re_head = (re_head + take_re) % m;
        re_len -= take_re;
        in_head += take_in;
        const bool queues_empty = (in_head == m && re_len == 0);
        bool trigger = queues_empty;
        if (!trigger) {
            readback(CTL_WORDS);
            trigger = hctl[CTL_MAXCNT] >= half;
        }
        if (!trigger) continue;

        // ---- ProcessAllBuffers ----
        int which = launch_sort_pairs(t.d_pleaf.as<uint32_t>(), t.d_pq.as<int32_t>(), t.d_tleaf.as<uint32_t>(),
                                      t.d_tq.as<int32_t>(), pend, kbits, t.d_hist.as<uint32_t>(), s);
        const int32_t *bufq = which ? t.d_tq.as<int32_t>() : t.d_pq.as<int32_t>();
        launch_leaf_offsets(cnt, t.d_leaf_off.as<int32_t>(), nleaf, SCAN_QT, SCAN_DENSE_MIN, t.d_off.as<int32_t>(),
                            t.d_tiles.as<int32_t>(), ctl, s);
        if (!t.resident)
            BKD_HIP(hipMemcpyAsync(t.h_tiles.p, t.d_tiles.p, sizeof(int32_t) * 2 * (size_t)(nleaf + 1),
                                   hipMemcpyDeviceToHost, s));
        readback(CTL_WORDS);
        const int64_t V = hctl[CTL_V];
        const int64_t T = hctl[CTL_T];
        const int64_t S = hctl[CTL_S];
        if (T + S > 0) {
            ScanArgs a{};
            a.tiles = t.d_tiles.as<int32_t>();
            a.sparse = a.tiles + nleaf + 1;
            a.off = t.d_off.as<int32_t>();
            a.bufq = bufq;
            a.leaf_off = t.d_leaf_off.as<int32_t>();
            a.Q = dQ;
            a.d = d;
            a.keys = t.d_keys.as<uint64_t>();
            if (t.resident) {
                a.X = t.d_chunk[0].as<float>();
                a.orig = reinterpret_cast<const int32_t *>(a.X + (size_t)d * H.n);
                a.pitch = H.n;
                a.chunk_lo = 0;
                a.chunk_hi = H.n;
                a.item_first = 0;
                a.item_count = (int32_t)T;
                a.sitem_first = 0;
                a.sitem_count = (int32_t)S;
                a.leaf_first = 0;
                a.leaf_last = nleaf - 1;
                timer.begin(s);
                launch_leaf_scan(a, K, s);
                timer.end(s);
                t.stats.scan_launches++;
            } else {
                const int32_t *tiles = t.h_tiles.as<int32_t>();
                const int32_t *sparse = tiles + nleaf + 1;
                std::vector<int> active;
                for (int j = 0; j < (int)t.chunks.size(); j++) {
                    const Chunk &c = t.chunks[(size_t)j];
                    if (tiles[c.leaf_last + 1] > tiles[c.leaf_first] || sparse[c.leaf_last + 1] > sparse[c.leaf_first])
                        active.push_back(j);
                }
                for (size_t ai = 0; ai < active.size(); ai++) {
                    const int j = active[ai];
                    const Chunk &c = t.chunks[(size_t)j];
                    int b = (t.chunk_in[0] == j) ? 0 : (t.chunk_in[1] == j) ? 1 : -1;
                    if (b < 0) {
                        // not prefetched: take the buffer that the next chunk does not need
                        int nj = ai + 1 < active.size() ? active[ai + 1] : -1;
                        b = (t.chunk_in[0] == nj) ? 1 : 0;
                        issue_copy(t, b, j);
                    }
                    BKD_HIP(hipStreamWaitEvent(s, t.ev_copied[b], 0));
                    a.X = t.d_chunk[b].as<float>();
                    const int64_t len = c.hi - c.lo;
                    a.orig = reinterpret_cast<const int32_t *>(a.X + (size_t)d * len);
                    a.pitch = len;
                    a.chunk_lo = c.lo;
                    a.chunk_hi = c.hi;
                    a.leaf_first = c.leaf_first;
                    a.leaf_last = c.leaf_last;
                    a.item_first = tiles[c.leaf_first];
                    a.item_count = tiles[c.leaf_last + 1] - tiles[c.leaf_first];
                    a.sitem_first = sparse[c.leaf_first];
                    a.sitem_count = sparse[c.leaf_last + 1] - sparse[c.leaf_first];
                    timer.begin(s);
                    launch_leaf_scan(a, K, s);
                    timer.end(s);
                    t.stats.scan_launches++;
                    BKD_HIP(hipEventRecord(t.ev_used[b], s));
                    // prefetch: the next active chunk, or chunk 0 for the next call
                    const int nj = ai + 1 < active.size() ? active[ai + 1] : 0;
                    const int nb = 1 - b;
                    if (t.chunk_in[nb] != nj && t.chunk_in[b] != nj) issue_copy(t, nb, nj);
                }
            }
        }
        (void)bpp;
        // reinsert the processed ids (ascending leaf, buffer order)
        launch_ring_append(t.d_ring.as<int32_t>(), m, (re_head + re_len) % m, bufq, V, s);
        re_len += V;
        launch_fill_i32(cnt, 0, nleaf, s);
        launch_fill_i32(ctl + CTL_MAXCNT, 0, 2, s);
        pend = 0;
        t.stats.calls++;
        if (tracing) t.trace_off.push_back((int64_t)t.trace_q.size());
    }
    launch_finalize(t.d_keys.as<uint64_t>(), K, k, m, d_idx, d_dist, (t.opt.flags & BKD_FLAG_SQUARED) != 0, s);
    readback(CTL_WORDS);
    int64_t pairs, visits;
    std::memcpy(&pairs, hctl + CTL_PAIRS_LO, 8);
    std::memcpy(&visits, hctl + CTL_VISITS_LO, 8);
    t.stats.pairs = pairs;
    t.stats.visits = visits;
    if (timer.on) t.stats.scan_ms = timer.total_ms();
    t.stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace bkd
