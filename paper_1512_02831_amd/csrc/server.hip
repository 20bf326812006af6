// server.hip -- served form: resident trees, continuous batching of query requests.
//
// A session serves one (tree, key capacity) pair on its own stream and host
// thread.  It runs lock-step rounds (Algorithm 1 with every active query
// fetched each round, Section 2.4) without stopping: between two rounds it
// admits waiting requests whose queries fit into its free query slots (the
// memory reserved for query coordinates, key lists and buffers), so new
// queries join the same leaf buffers as the queries already in flight
// (on-the-fly admission, Section 3.2 "Multi-Many-Core Querying").  A request
// completes when FindLeafBatch finishes its last query; its keys are then
// converted, copied to the caller and its slots freed.  Every query's result
// depends only on its own data, so a result is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.h"
#include "traverse.h"

namespace bkd {

int guarded_call(const std::function<void()> &f);

namespace {

__global__ void k_admit(const float *__restrict__ stage, const int32_t *__restrict__ slots, int64_t m, int d, int K,
                        int k, int32_t table, float *__restrict__ Qpool, uint64_t *__restrict__ keys,
                        uint32_t *__restrict__ kth, int32_t *__restrict__ node, int32_t *__restrict__ kq,
                        int32_t *__restrict__ req_of, int32_t *__restrict__ age)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t s = slots[i];
    for (int j = 0; j < d; j++) Qpool[(int64_t)s * d + j] = stage[i * d + j];
    for (int j = 0; j < K; j++) keys[(int64_t)s * K + j] = EMPTY_KEY;
    kth[s] = (uint32_t)(EMPTY_KEY >> 32);
    node[s] = NODE_FRESH;
    kq[s] = k;
    req_of[s] = table;
    age[s] = 0;
}

__global__ void k_gather(const uint64_t *__restrict__ keys, const int32_t *__restrict__ slots, int64_t m, int K, int k,
                         int64_t *__restrict__ idx, float *__restrict__ dist, int squared)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m * k) return;
    const int64_t q = i / k;
    const int r = (int)(i - q * k);
    const uint64_t key = keys[(int64_t)slots[q] * K + r];
    const float d2 = __uint_as_float((uint32_t)(key >> 32));
    idx[i] = (int64_t)(uint32_t)key;
    dist[i] = squared ? d2 : sqrtf(d2);
}

__global__ void k_set_i32(int32_t *p, int64_t i, int32_t v) { p[i] = v; }

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Pending queries at or below which a session's round hands them all to the tail kernel
// (bkd_server_opts.tail_max).  Lower than the single call's default: a session keeps
// admitting work, and its rounds share leaf reads among the queries in flight.  Measured on
// the two-tree workload: 2048 gave 0.79 M queries/s saturated and p99 8.0 s at half load,
// 16384 gave 0.81 M and 4.7 s, 65536 gave 0.66 M and 10.6 s.
constexpr int64_t SERVED_TAIL_MAX = 16384;

struct Request {
    int64_t id = 0;
    int tree = 0, k = 0, K = 0;
    int64_t m = 0;
    std::vector<float> Q;
    int64_t *out_idx = nullptr;
    float *out_dist = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;  // 0 waiting, 1 running, 2 done, 3 cancelled
    int32_t table = -1;
    std::vector<int32_t> slots;
    bool cancel = false;
    bool wide = false;  // a coordinate beyond +-FILTER_RANGE
};

struct Server;

struct Session {
    Server *srv = nullptr;
    bkd_tree *tree = nullptr;
    int tree_id = 0, K = 0;
    int64_t cap = 0;  // query slots
    int max_req = 0;
    int age_max = 0;  // rounds after which a query leaves the rounds for the tail (0: never)
    int strag_max = 0;  // a request's travelling queries at or below which they leave likewise (0: never)
    int64_t tail_max = 0;  // pending queries at or below which a round hands them all to the tail
    hipStream_t s = nullptr;
    // device state
    DevBuf Qpool, keys, kth, node, kq, req_of, req_left, done, pleaf, pq, tleaf, tq, hist, cnt, cnt0, off, tiles, ctl, newslots,
        stage, oidx, odist, gslots, fleaf, fq, age;
    PinnedBuf hctl, hdone, hstage, hout, hgslots;
    hipEvent_t ev_stage = nullptr;  // after the last admission's staging copies
    hipEvent_t ev_sync = nullptr;   // the round's readback
    hipEvent_t ev_out = nullptr;    // the delivered requests' results on the host
    bool stage_pending = false;
    bool wide = false;  // a request with coordinates beyond +-FILTER_RANGE was admitted: exact scans from then on
    // host state
    std::vector<int32_t> free_slots, free_tables;
    std::deque<Request *> waiting;
    std::map<int32_t, Request *> running;  // by table index
    int64_t P = 0;  // pending entries in flight (sorted list of the last round)
    int64_t nfast = 0;  // admitted queries of small requests (at the front of newslots), this round
    int cur = 0;
    std::thread th;
    int64_t rounds = 0, scans = 0, tails = 0, directs = 0, admitted = 0, aged = 0;
    double busy_s = 0, admit_s = 0, complete_s = 0;
};

struct Server {
    int device = 0;
    int64_t slots_per_session = 0;
    int32_t max_requests = 0;
    int32_t flags = 0;
    int32_t age_max = 0;
    int32_t strag_max = 0;
    int64_t tail_max = SERVED_TAIL_MAX;
    std::mutex mu;
    std::condition_variable cv;       // wakes sessions (new work, stop)
    std::condition_variable done_cv;  // wakes waiters
    bool stop = false;
    std::vector<bkd_tree *> trees;
    std::vector<std::unique_ptr<Session>> sessions;
    std::map<int64_t, std::unique_ptr<Request>> requests;
    int64_t next_id = 1;
    std::string error;
};

static void session_init(Session &S)
{
    const HostTree &H = S.tree->t.host;
    const int64_t cap = S.cap;
    const int nleaf = S.tree->t.nleaf;
    S.Qpool.ensure(sizeof(float) * cap * H.d);
    S.keys.ensure(sizeof(uint64_t) * cap * S.K);
    S.kth.ensure(sizeof(uint32_t) * cap);
    S.node.ensure(sizeof(int32_t) * cap);
    S.kq.ensure(sizeof(int32_t) * cap);
    S.req_of.ensure(sizeof(int32_t) * cap);
    S.req_left.ensure(sizeof(int32_t) * S.max_req);
    S.done.ensure(sizeof(int32_t) * (S.max_req + 1));
    S.pleaf.ensure(sizeof(uint32_t) * cap);
    S.pq.ensure(sizeof(int32_t) * cap);
    S.tleaf.ensure(sizeof(uint32_t) * cap);
    S.tq.ensure(sizeof(int32_t) * cap);
    S.hist.ensure(sizeof(uint32_t) * sort_hist_words(cap));
    S.cnt.ensure(sizeof(int32_t) * nleaf);
    S.cnt0.ensure(sizeof(int32_t) * nleaf);
    S.off.ensure(sizeof(int32_t) * (nleaf + 1));
    S.tiles.ensure(sizeof(int32_t) * 2 * (nleaf + 1));
    S.ctl.ensure(sizeof(int32_t) * CTL_WORDS);
    S.newslots.ensure(sizeof(int32_t) * cap);
    S.fleaf.ensure(sizeof(uint32_t) * cap);
    S.fq.ensure(sizeof(int32_t) * cap);
    S.age.ensure(sizeof(int32_t) * cap);
    S.hctl.ensure(sizeof(int32_t) * CTL_WORDS);
    S.hdone.ensure(sizeof(int32_t) * (S.max_req + 1));
    S.free_slots.resize((size_t)cap);
    for (int64_t i = 0; i < cap; i++) S.free_slots[(size_t)i] = (int32_t)(cap - 1 - i);
    S.free_tables.resize((size_t)S.max_req);
    for (int i = 0; i < S.max_req; i++) S.free_tables[(size_t)i] = S.max_req - 1 - i;
    BKD_HIP(hipStreamCreateWithFlags(&S.s, hipStreamNonBlocking));
    BKD_HIP(hipEventCreateWithFlags(&S.ev_stage, hipEventDisableTiming));
    BKD_HIP(hipEventCreateWithFlags(&S.ev_sync, hipEventDisableTiming));
    BKD_HIP(hipEventCreateWithFlags(&S.ev_out, hipEventDisableTiming));
    launch_fill_i32(S.cnt.as<int32_t>(), 0, nleaf, S.s);
    launch_fill_i32(S.ctl.as<int32_t>(), 0, CTL_WORDS, S.s);
    launch_fill_i32(S.done.as<int32_t>(), 0, 1, S.s);
    BKD_HIP(hipStreamSynchronize(S.s));
}

// Requests of at most this many queries skip the rounds: each of their queries is routed to its
// first leaf and finishes its whole traversal in one tail workgroup, right after admission, so
// their latency is one launch instead of the session's round count (Section 2.3 search phases,
// the same visits and results as the rounds).
constexpr int64_t SERVED_DIRECT_MAX = 2048;

// Admit waiting requests that fit (FIFO); called with the server lock held for the bookkeeping.
static int64_t session_admit(Session &S, std::unique_lock<std::mutex> &lk)
{
    const int d = S.tree->t.host.d;
    int64_t nnew = 0;
    std::vector<Request *> adm;
    while (!S.waiting.empty()) {
        Request *r = S.waiting.front();
        if (r->cancel) {
            S.waiting.pop_front();
            r->state = 3;
            S.srv->done_cv.notify_all();
            continue;
        }
        if ((int64_t)S.free_slots.size() < r->m || S.free_tables.empty()) break;
        S.waiting.pop_front();
        r->table = S.free_tables.back();
        S.free_tables.pop_back();
        r->slots.assign(S.free_slots.end() - r->m, S.free_slots.end());
        S.free_slots.resize(S.free_slots.size() - (size_t)r->m);
        r->state = 1;
        r->t_admit = now_s();
        S.running[r->table] = r;
        adm.push_back(r);
    }
    lk.unlock();
    // small requests first: their queries take the direct path (one traversal per query, no rounds)
    std::stable_partition(adm.begin(), adm.end(), [](const Request *r) { return r->m <= SERVED_DIRECT_MAX; });
    S.nfast = 0;
    for (Request *r : adm)
        if (r->m <= SERVED_DIRECT_MAX) S.nfast += r->m;
    if (!adm.empty()) {
        // all admitted requests in one staging pass: host -> pinned stage -> device stage -> slots
        int64_t total = 0;
        for (Request *r : adm) total += r->m;
        const size_t qb = sizeof(float) * (size_t)total * d;
        if (S.stage_pending) BKD_HIP(hipEventSynchronize(S.ev_stage));  // the stage buffers are free again
        S.hstage.ensure(qb + sizeof(int32_t) * (size_t)total);
        S.stage.ensure(qb);
        char *hs = static_cast<char *>(S.hstage.p);
        int64_t off = 0;
        for (Request *r : adm) {
            std::memcpy(hs + sizeof(float) * (size_t)off * d, r->Q.data(), sizeof(float) * (size_t)r->m * d);
            std::memcpy(hs + qb + sizeof(int32_t) * (size_t)off, r->slots.data(), sizeof(int32_t) * (size_t)r->m);
            off += r->m;
        }
        BKD_HIP(hipMemcpyAsync(S.stage.p, hs, qb, hipMemcpyHostToDevice, S.s));
        BKD_HIP(hipMemcpyAsync(S.newslots.p, hs + qb, sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, S.s));
        for (Request *r : adm) {
            S.wide |= r->wide;
            k_admit<<<(unsigned)((r->m + 255) / 256), 256, 0, S.s>>>(
                S.stage.as<float>() + nnew * d, S.newslots.as<int32_t>() + nnew, r->m, d, S.K, r->k, r->table,
                S.Qpool.as<float>(), S.keys.as<uint64_t>(), S.kth.as<uint32_t>(), S.node.as<int32_t>(),
                S.kq.as<int32_t>(),
                S.req_of.as<int32_t>(), S.age.as<int32_t>());
            k_set_i32<<<1, 1, 0, S.s>>>(S.req_left.as<int32_t>(), r->table, (int32_t)r->m);
            nnew += r->m;
        }
        BKD_HIP(hipEventRecord(S.ev_stage, S.s));
        S.stage_pending = true;
    }
    S.admitted += nnew;
    lk.lock();
    return nnew;
}

// Buffers of at least this many queries take the dense scan in a session round (8 against 32:
// a session's rounds hold few queries per leaf, and reading a leaf once for eight queries beats
// eight walks of it; saturated throughput 0.70 -> 0.77 M queries/s on the two-tree workload).
constexpr int SERVED_DENSE_MIN = 8;


// Wait for an event recorded on the session's stream, spinning (a blocking wait can sleep
// well past the event on a busy host, and every round waits once).
static void session_wait_event(hipEvent_t ev)
{
    for (int spins = 0;; spins++) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) BKD_HIP(e);
        if ((spins & 63) == 63) std::this_thread::yield();
    }
}

// Delivery of finished requests, part one (no server lock): every finished request's slot
// list up, one gather per request, the results down, then an event; queued before the
// round's scans, so the wait for it does not cover them.
static void session_deliver_begin(Session &S, const std::vector<Request *> &fin)
{
    int64_t nslots = 0, nout = 0;
    for (Request *r : fin) {
        nslots += r->m;
        nout += r->m * r->k;
    }
    S.hgslots.ensure(sizeof(int32_t) * (size_t)nslots);
    S.gslots.ensure(sizeof(int32_t) * (size_t)nslots);
    S.oidx.ensure(sizeof(int64_t) * (size_t)nout);
    S.odist.ensure(sizeof(float) * (size_t)nout);
    S.hout.ensure((sizeof(int64_t) + sizeof(float)) * (size_t)nout);
    int64_t so = 0;
    for (Request *r : fin) {
        std::memcpy(S.hgslots.as<int32_t>() + so, r->slots.data(), sizeof(int32_t) * (size_t)r->m);
        so += r->m;
    }
    BKD_HIP(hipMemcpyAsync(S.gslots.p, S.hgslots.p, sizeof(int32_t) * (size_t)nslots, hipMemcpyHostToDevice, S.s));
    so = 0;
    int64_t oo = 0;
    for (Request *r : fin) {
        const int64_t cnt = r->m * r->k;
        k_gather<<<(unsigned)((cnt + 255) / 256), 256, 0, S.s>>>(
            S.keys.as<uint64_t>(), S.gslots.as<int32_t>() + so, r->m, S.K, r->k, S.oidx.as<int64_t>() + oo,
            S.odist.as<float>() + oo, (S.srv->flags & BKD_FLAG_SQUARED) ? 1 : 0);
        so += r->m;
        oo += cnt;
    }
    int64_t *hidx = S.hout.as<int64_t>();
    float *hdist = reinterpret_cast<float *>(hidx + nout);
    BKD_HIP(hipMemcpyAsync(hidx, S.oidx.p, sizeof(int64_t) * (size_t)nout, hipMemcpyDeviceToHost, S.s));
    BKD_HIP(hipMemcpyAsync(hdist, S.odist.p, sizeof(float) * (size_t)nout, hipMemcpyDeviceToHost, S.s));
    BKD_HIP(hipEventRecord(S.ev_out, S.s));
}

// Part two: once the results are on the host, copy them to the callers' arrays, then (under
// the server lock) free the requests' slots and tables and wake the waiters.
static void session_deliver_end(Session &S, std::unique_lock<std::mutex> &lk, const std::vector<Request *> &fin)
{
    session_wait_event(S.ev_out);
    int64_t nout = 0;
    for (Request *r : fin) nout += r->m * r->k;
    const int64_t *hidx = S.hout.as<int64_t>();
    const float *hdist = reinterpret_cast<const float *>(hidx + nout);
    int64_t oo = 0;
    for (Request *r : fin) {
        const int64_t cnt = r->m * r->k;
        std::memcpy(r->out_idx, hidx + oo, sizeof(int64_t) * (size_t)cnt);
        std::memcpy(r->out_dist, hdist + oo, sizeof(float) * (size_t)cnt);
        oo += cnt;
        r->t_done = now_s();
    }
    lk.lock();
    for (Request *r : fin) {
        S.running.erase(r->table);
        S.free_tables.push_back(r->table);
        S.free_slots.insert(S.free_slots.end(), r->slots.begin(), r->slots.end());
        r->slots.clear();
        r->slots.shrink_to_fit();
        r->state = r->cancel ? 3 : 2;
    }
    S.srv->done_cv.notify_all();
    lk.unlock();
}

// One round: route the last round's queries and the new ones, buffer them, read the counts
// and the completion list back (the round's one wait, which also covers the last round's
// scans), hand the finished requests' results down, scan.  Called without the server lock.
static void session_round(Session &S, int64_t nnew, std::unique_lock<std::mutex> &lk)
{
    Tree &T = S.tree->t;
    const HostTree &H = T.host;
    const int nleaf = T.nleaf;
    uint32_t *leafbuf[2] = {S.pleaf.as<uint32_t>(), S.tleaf.as<uint32_t>()};
    int32_t *qbuf[2] = {S.pq.as<int32_t>(), S.tq.as<int32_t>()};
    int32_t *ctl = S.ctl.as<int32_t>();
    int32_t *hctl = S.hctl.as<int32_t>();
    if (S.nfast > 0) {
        // small requests: first leaf of each query, then its whole traversal in one workgroup
        FetchSpec g{nullptr, 0, 0, 1, 0, S.nfast};
        g.count_leaves = false;
        g.in_list = S.newslots.as<int32_t>();
        g.req_of = S.req_of.as<int32_t>();
        g.req_left = S.req_left.as<int32_t>();
        g.done_list = S.done.as<int32_t>();
        g.dims = T.dims_dev();
        g.boxes = T.boxes_dev();
        launch_find_leaf(g, S.Qpool.as<float>(), H.d, S.node.as<int32_t>(), S.kth.as<uint32_t>(),
                         T.d_split.as<float>(), H.h, S.fleaf.as<uint32_t>(), S.fq.as<int32_t>(), 0,
                         S.cnt.as<int32_t>(), ctl, S.s);
        ScanArgs a{};
        a.leaf_off = T.d_leaf_off.as<int32_t>();
        a.base = T.d_chunk[0].as<float>();
        a.blk = T.d_leaf_blk.as<int64_t>();
        a.Q = S.Qpool.as<float>();
        a.d = H.d;
        a.keys = S.keys.as<uint64_t>();
        a.kth = S.kth.as<uint32_t>();
        a.tail_leaf = S.fleaf.as<uint32_t>();
        a.tail_q = S.fq.as<int32_t>();
        a.tail_count = (int32_t)S.nfast;
        a.tail_wide = (H.n >> H.h) >= TAIL_WIDE_LEAF;
        a.node = S.node.as<int32_t>();
        a.split = T.d_split.as<float>();
        a.h = H.h;
        a.k = S.K;
        a.ctl = ctl;
        a.kq = S.kq.as<int32_t>();
        a.req_of = S.req_of.as<int32_t>();
        a.req_left = S.req_left.as<int32_t>();
        a.done_list = S.done.as<int32_t>();
        a.dims = T.dims_dev();
        a.boxes = T.boxes_dev();
        launch_leaf_scan(a, S.K, 2, S.s);
        S.directs++;
    }
    nnew -= S.nfast;
    // route in place: the previous sorted list, then the other admitted slots appended
    FetchSpec f{qbuf[S.cur], 0, S.P, std::max<int64_t>(S.P, 1), 0, nnew};
    f.count_leaves = false;  // per-leaf counts come from the runs of the sorted list
    f.in_list = S.newslots.as<int32_t>() + S.nfast;
    f.req_of = S.req_of.as<int32_t>();
    f.req_left = S.req_left.as<int32_t>();
    f.done_list = S.done.as<int32_t>();
    f.dims = T.dims_dev();
    f.boxes = T.boxes_dev();
    if (S.age_max > 0) {
        f.age = S.age.as<int32_t>();
        f.age_max = S.age_max;
    }
    f.strag_max = S.strag_max;
    if (S.age_max > 0 || S.strag_max > 0) launch_fill_i32(ctl + CTL_AGED, 0, 1, S.s);
    launch_find_leaf(f, S.Qpool.as<float>(), H.d, S.node.as<int32_t>(), S.kth.as<uint32_t>(),
                     T.d_split.as<float>(), H.h, leafbuf[S.cur], qbuf[S.cur], 0, S.cnt.as<int32_t>(), ctl, S.s);
    const int64_t total = S.P + nnew;
    // keys: leaves 0 .. 2^h - 1, 2^h for a finished query, 2^h + 1 for one handed to the tail
    int which = launch_sort_pairs(leafbuf[S.cur], qbuf[S.cur], leafbuf[1 - S.cur], qbuf[1 - S.cur], total,
                                  [&] { int b = 1; while ((1ll << b) <= nleaf + 1) b++; return b; }(),
                                  S.hist.as<uint32_t>(), S.s);
    if (which) S.cur = 1 - S.cur;
    launch_fill_i32(S.cnt.as<int32_t>(), 0, nleaf, S.s);
    launch_fill_i32(S.cnt0.as<int32_t>(), 0, nleaf, S.s);
    launch_run_bounds(leafbuf[S.cur], total, nleaf, S.cnt0.as<int32_t>(), S.cnt.as<int32_t>(), S.s);
    launch_leaf_offsets(S.cnt.as<int32_t>(), S.cnt0.as<int32_t>(), T.d_leaf_off.as<int32_t>(), nleaf, SCAN_QT,
                        T.dense_min == INT32_MAX ? INT32_MAX : SERVED_DENSE_MIN,
                        S.off.as<int32_t>(), S.tiles.as<int32_t>(), S.tiles.as<int32_t>() + nleaf + 1, ctl, S.s);
    BKD_HIP(hipMemcpyAsync(hctl, ctl, sizeof(int32_t) * CTL_WORDS, hipMemcpyDeviceToHost, S.s));
    // the completion list (its count and every entry, at most max_req): requests whose last
    // query finished in this round's routing or in the last round's tail launches
    BKD_HIP(hipMemcpyAsync(S.hdone.p, S.done.p, sizeof(int32_t) * (size_t)(1 + S.max_req), hipMemcpyDeviceToHost,
                           S.s));
    BKD_HIP(hipEventRecord(S.ev_sync, S.s));
    session_wait_event(S.ev_sync);
    S.P = hctl[CTL_V];
    std::vector<Request *> fin;
    const double tc = now_s();
    if (const int nd = S.hdone.as<int32_t>()[0]) {
        launch_fill_i32(S.done.as<int32_t>(), 0, 1, S.s);  // before any launch that appends to it
        lk.lock();
        for (int x = 0; x < nd; x++) {
            auto it = S.running.find(S.hdone.as<int32_t>()[1 + x]);
            if (it != S.running.end()) fin.push_back(it->second);
        }
        lk.unlock();
        if (!fin.empty()) session_deliver_begin(S, fin);
    }
    S.complete_s += now_s() - tc;
    const int64_t aged = (S.age_max > 0 || S.strag_max > 0) ? hctl[CTL_AGED] : 0;
    if (aged > 0) {
        // queries routed more than age_max times, or among their request's last strag_max
        // travelling ones, sort last: each walks the rest of its traversal in one workgroup
        // from the leaf in node[q], so a request is not held by its longest walks
        ScanArgs a{};
        a.leaf_off = T.d_leaf_off.as<int32_t>();
        a.base = T.d_chunk[0].as<float>();
        a.blk = T.d_leaf_blk.as<int64_t>();
        a.Q = S.Qpool.as<float>();
        a.d = H.d;
        a.keys = S.keys.as<uint64_t>();
        a.kth = S.kth.as<uint32_t>();
        a.tail_q = qbuf[S.cur] + (total - aged);
        a.tail_count = (int32_t)aged;
        a.tail_from_node = 1;
        a.tail_wide = (H.n >> H.h) >= TAIL_WIDE_LEAF;
        a.node = S.node.as<int32_t>();
        a.split = T.d_split.as<float>();
        a.h = H.h;
        a.k = S.K;
        a.ctl = ctl;
        a.kq = S.kq.as<int32_t>();
        a.req_of = S.req_of.as<int32_t>();
        a.req_left = S.req_left.as<int32_t>();
        a.done_list = S.done.as<int32_t>();
        a.dims = T.dims_dev();
        a.boxes = T.boxes_dev();
        launch_leaf_scan(a, S.K, 2, S.s);
        S.aged += aged;
    }
    if (S.P > 0 && S.P <= S.tail_max) {
        // few queries in flight: each finishes its traversal in one workgroup, and its request
        // completes as its last query does
        ScanArgs a{};
        a.leaf_off = T.d_leaf_off.as<int32_t>();
        a.base = T.d_chunk[0].as<float>();
        a.blk = T.d_leaf_blk.as<int64_t>();
        a.Q = S.Qpool.as<float>();
        a.d = H.d;
        a.keys = S.keys.as<uint64_t>();
        a.kth = S.kth.as<uint32_t>();
        a.tail_leaf = leafbuf[S.cur];
        a.tail_q = qbuf[S.cur];
        a.tail_count = (int32_t)S.P;
        a.tail_wide = (H.n >> H.h) >= TAIL_WIDE_LEAF;
        a.node = S.node.as<int32_t>();
        a.split = T.d_split.as<float>();
        a.h = H.h;
        a.k = S.K;
        a.ctl = ctl;
        a.kq = S.kq.as<int32_t>();
        a.req_of = S.req_of.as<int32_t>();
        a.req_left = S.req_left.as<int32_t>();
        a.done_list = S.done.as<int32_t>();
        a.dims = T.dims_dev();
        a.boxes = T.boxes_dev();
        launch_leaf_scan(a, S.K, 2, S.s);
        S.P = 0;
        S.tails++;
    } else if (hctl[CTL_T] + hctl[CTL_S] > 0) {
        ScanArgs a{};
        a.tiles = S.tiles.as<int32_t>();
        a.sparse = a.tiles + nleaf + 1;
        a.off = S.off.as<int32_t>();
        a.bufq = qbuf[S.cur];
        a.leaf_off = T.d_leaf_off.as<int32_t>();
        a.base = T.d_chunk[0].as<float>();
        a.blk = T.d_leaf_blk.as<int64_t>();
        a.blk_shift = 0;
        a.chunk_lo = 0;
        a.chunk_hi = H.n;
        a.item_first = 0;
        a.item_count = hctl[CTL_T];
        a.sitem_first = 0;
        a.sitem_count = hctl[CTL_S];
        a.leaf_first = 0;
        a.leaf_last = nleaf - 1;
        a.Q = S.Qpool.as<float>();
        a.d = H.d;
        a.keys = S.keys.as<uint64_t>();
        a.kth = S.kth.as<uint32_t>();
        a.k = S.K;
        a.kq = S.kq.as<int32_t>();
        a.exact_only = (T.wide || S.wide) ? 1 : 0;
        a.centers = T.d_centers.as<float>();
        a.scales = a.centers + (size_t)nleaf * H.d;
        a.dims = T.dims_dev();
        a.boxes = T.boxes_dev();
        launch_leaf_scan(a, S.K, 0, S.s);
        launch_leaf_scan(a, S.K, 1, S.s);
        S.scans++;
    }
    S.rounds++;
    if (!fin.empty()) {
        const double td = now_s();
        session_deliver_end(S, lk, fin);
        S.complete_s += now_s() - td;
    }
}

static void session_loop(Session *Sp)
{
    Session &S = *Sp;
    Server &V = *S.srv;
    try {
        BKD_HIP(hipSetDevice(V.device));
        std::unique_lock<std::mutex> lk(V.mu);
        for (;;) {
            if (V.stop) break;
            const double ta = now_s();
            const int64_t nnew = session_admit(S, lk);
            S.admit_s += now_s() - ta;
            if (S.P == 0 && nnew == 0 && S.running.empty()) {
                V.cv.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
            lk.unlock();
            const double t0 = now_s(), c0 = S.complete_s;
            session_round(S, nnew, lk);
            S.busy_s += now_s() - t0 - (S.complete_s - c0);  // the delivery inside is counted apart
            lk.lock();
        }
    } catch (const BkdError &e) {
        std::lock_guard<std::mutex> g(V.mu);
        V.error = e.msg;
        V.stop = true;
        V.done_cv.notify_all();
    }
}

static Session &session_for(Server &V, int tree_id, int K)
{
    for (auto &s : V.sessions)
        if (s->tree_id == tree_id && s->K == K) return *s;
    auto S = std::make_unique<Session>();
    S->srv = &V;
    S->tree = V.trees[(size_t)tree_id];
    S->tree_id = tree_id;
    S->K = K;
    S->cap = V.slots_per_session;
    S->max_req = V.max_requests;
    S->age_max = V.age_max;
    S->strag_max = V.strag_max;
    S->tail_max = V.tail_max;
    session_init(*S);
    S->th = std::thread(session_loop, S.get());
    V.sessions.push_back(std::move(S));
    return *V.sessions.back();
}

}  // namespace bkd

struct bkd_server {
    bkd::Server v;
};

extern "C" {

int bkd_server_create(const bkd_server_opts *opts, bkd_server **out)
{
    return bkd::guarded_call([&] {
        if (!out) bkd::fail(BKD_EINVAL, "out is NULL");
        *out = nullptr;
        bkd_server_opts o{};
        if (opts) o = *opts;
        if (o.slots_per_session == 0) o.slots_per_session = 1 << 20;
        if (o.max_requests == 0) o.max_requests = 4096;
        if (o.slots_per_session < 1 || o.slots_per_session > INT32_MAX || o.max_requests < 1 || o.device < 0 ||
            o.age_max < 0 || o.straggle_max < 0)
            bkd::fail(BKD_EINVAL, "invalid server options");
        int ndev = 0;
        BKD_HIP(hipGetDeviceCount(&ndev));
        if (o.device >= ndev) bkd::fail(BKD_EINVAL, "device ordinal out of range");
        auto s = std::make_unique<bkd_server>();
        s->v.device = o.device;
        s->v.slots_per_session = o.slots_per_session;
        s->v.max_requests = o.max_requests;
        s->v.flags = o.flags;
        s->v.age_max = o.age_max;
        s->v.strag_max = o.straggle_max;
        s->v.tail_max = o.tail_max == 0 ? bkd::SERVED_TAIL_MAX : (o.tail_max < 0 ? 0 : o.tail_max);
        *out = s.release();
    });
}

int bkd_server_add_tree(bkd_server *srv, bkd_tree *tree, int32_t *tree_id)
{
    return bkd::guarded_call([&] {
        if (!srv || !tree || !tree_id) bkd::fail(BKD_EINVAL, "NULL pointer");
        if (!tree->t.resident) bkd::fail(BKD_EINVAL, "served trees must be resident (no leaf budget)");
        if (tree->t.opt.device != srv->v.device) bkd::fail(BKD_EINVAL, "tree lives on another device");
        std::lock_guard<std::mutex> g(srv->v.mu);
        srv->v.trees.push_back(tree);
        *tree_id = (int32_t)srv->v.trees.size() - 1;
    });
}

int bkd_submit(bkd_server *srv, int32_t tree_id, const float *Q, int64_t m, int32_t k, int64_t *out_idx,
               float *out_dist, int64_t *req_id)
{
    return bkd::guarded_call([&] {
        if (!srv || !req_id) bkd::fail(BKD_EINVAL, "NULL pointer");
        bkd::Server &V = srv->v;
        std::unique_lock<std::mutex> lk(V.mu);
        if (!V.error.empty()) bkd::fail(BKD_EDEVICE, "server stopped: " + V.error);
        if (tree_id < 0 || tree_id >= (int32_t)V.trees.size()) bkd::fail(BKD_ENOTFOUND, "unknown tree id");
        bkd_tree *t = V.trees[(size_t)tree_id];
        const int d = t->t.host.d;
        if (m < 1 || !Q || !out_idx || !out_dist) bkd::fail(BKD_EINVAL, "need m >= 1 and non-NULL Q and outputs");
        if (k < 1 || k > BKD_MAX_K || k > t->t.host.n) bkd::fail(BKD_EINVAL, "k must be in [1, min(n, 64)]");
        if (m > V.slots_per_session) bkd::fail(BKD_EBUSY, "request larger than a session's query slots");
        bool wide = false;
        for (int64_t i = 0; i < m * d; i++) {
            if (!std::isfinite(Q[i])) bkd::fail(BKD_EINVAL, "query coordinates must be finite");
            wide |= std::fabs(Q[i]) > bkd::FILTER_RANGE;
        }
        const int K = bkd::key_capacity(k);
        auto r = std::make_unique<bkd::Request>();
        r->id = V.next_id++;
        r->tree = tree_id;
        r->k = k;
        r->K = K;
        r->m = m;
        r->wide = wide;
        r->Q.assign(Q, Q + m * d);
        r->out_idx = out_idx;
        r->out_dist = out_dist;
        r->t_submit = bkd::now_s();
        bkd::Session &S = bkd::session_for(V, tree_id, K);
        S.waiting.push_back(r.get());
        *req_id = r->id;
        V.requests[r->id] = std::move(r);
        V.cv.notify_all();
    });
}

int bkd_poll(bkd_server *srv, int64_t req_id, int32_t *state)
{
    return bkd::guarded_call([&] {
        if (!srv || !state) bkd::fail(BKD_EINVAL, "NULL pointer");
        std::lock_guard<std::mutex> g(srv->v.mu);
        auto it = srv->v.requests.find(req_id);
        if (it == srv->v.requests.end()) bkd::fail(BKD_ENOTFOUND, "unknown request id");
        *state = it->second->state;
    });
}

int bkd_wait(bkd_server *srv, int64_t req_id, int64_t timeout_us)
{
    return bkd::guarded_call([&] {
        if (!srv) bkd::fail(BKD_EINVAL, "NULL pointer");
        bkd::Server &V = srv->v;
        std::unique_lock<std::mutex> lk(V.mu);
        auto it = V.requests.find(req_id);
        if (it == V.requests.end()) bkd::fail(BKD_ENOTFOUND, "unknown request id");
        bkd::Request *r = it->second.get();
        auto pred = [&] { return r->state >= 2 || !V.error.empty(); };
        if (timeout_us < 0) V.done_cv.wait(lk, pred);
        else if (!V.done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
            bkd::fail(BKD_ETIMEOUT, "request not finished");
        if (!V.error.empty()) bkd::fail(BKD_EDEVICE, "server stopped: " + V.error);
    });
}

int bkd_cancel(bkd_server *srv, int64_t req_id)
{
    return bkd::guarded_call([&] {
        if (!srv) bkd::fail(BKD_EINVAL, "NULL pointer");
        std::lock_guard<std::mutex> g(srv->v.mu);
        auto it = srv->v.requests.find(req_id);
        if (it == srv->v.requests.end()) bkd::fail(BKD_ENOTFOUND, "unknown request id");
        it->second->cancel = true;
        srv->v.cv.notify_all();
    });
}

int bkd_request_times(bkd_server *srv, int64_t req_id, double *submit_s, double *admit_s, double *done_s)
{
    return bkd::guarded_call([&] {
        if (!srv || !submit_s || !admit_s || !done_s) bkd::fail(BKD_EINVAL, "NULL pointer");
        std::lock_guard<std::mutex> g(srv->v.mu);
        auto it = srv->v.requests.find(req_id);
        if (it == srv->v.requests.end()) bkd::fail(BKD_ENOTFOUND, "unknown request id");
        *submit_s = it->second->t_submit;
        *admit_s = it->second->t_admit;
        *done_s = it->second->t_done;
    });
}

int bkd_server_stats_get(bkd_server *srv, bkd_server_stats *out)
{
    return bkd::guarded_call([&] {
        if (!srv || !out) bkd::fail(BKD_EINVAL, "NULL pointer");
        std::lock_guard<std::mutex> g(srv->v.mu);
        *out = bkd_server_stats{};
        for (auto &s : srv->v.sessions) {
            out->sessions++;
            out->rounds += s->rounds;
            out->scan_rounds += s->scans;
            out->tail_rounds += s->tails;
            out->direct_launches += s->directs;
            out->aged_queries += s->aged;
            out->queries += s->admitted;
            out->busy_s += s->busy_s;
            out->admit_s += s->admit_s;
            out->complete_s += s->complete_s;
        }
    });
}

int bkd_release(bkd_server *srv, int64_t req_id)
{
    return bkd::guarded_call([&] {
        if (!srv) bkd::fail(BKD_EINVAL, "NULL pointer");
        std::lock_guard<std::mutex> g(srv->v.mu);
        auto it = srv->v.requests.find(req_id);
        if (it == srv->v.requests.end()) bkd::fail(BKD_ENOTFOUND, "unknown request id");
        if (it->second->state < 2) bkd::fail(BKD_EBUSY, "request still in flight");
        srv->v.requests.erase(it);
    });
}

int bkd_server_destroy(bkd_server *srv)
{
    return bkd::guarded_call([&] {
        if (!srv) return;
        {
            std::lock_guard<std::mutex> g(srv->v.mu);
            srv->v.stop = true;
            srv->v.cv.notify_all();
        }
        for (auto &s : srv->v.sessions)
            if (s->th.joinable()) s->th.join();
        (void)hipSetDevice(srv->v.device);
        (void)hipDeviceSynchronize();
        for (auto &s : srv->v.sessions) {
            if (s->ev_stage) (void)hipEventDestroy(s->ev_stage);
            if (s->ev_sync) (void)hipEventDestroy(s->ev_sync);
            if (s->ev_out) (void)hipEventDestroy(s->ev_out);
            if (s->s) (void)hipStreamDestroy(s->s);
        }
        delete srv;
    });
}

}  // extern "C"
