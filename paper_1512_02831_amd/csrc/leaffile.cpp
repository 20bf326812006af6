// leaffile.cpp -- disk-backed leaf structure (Section 3.2: when host memory cannot hold
// the leaf structure, it is kept on disk and every chunk travels disk -> host -> device).
//
// The file holds the whole structure in leaf-block layout, so chunk j is the byte range
// [4 word_lo, 4 word_hi) of the file.  Three stages overlap: a reader thread reads one
// chunk into one of two pinned staging buffers (with O_DIRECT where the file system
// allows it, through a small aligned bounce buffer, so reads come from the drive and
// not from the page cache), the copy
// stream moves the other staging buffer to a device chunk buffer, and the scans run on
// the chunk already resident.  A staging buffer is reused only after the copy out of it
// has completed (an event recorded behind the copy).
#include <fcntl.h>
#include <unistd.h>

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.h"

namespace bkd {

namespace {
constexpr size_t IO_ALIGN = 4096;  // direct I/O: offsets, sizes and buffers aligned to this
constexpr int SLOTS = 2;
// Direct I/O cannot target pinned (device-mapped) host memory here (the kernel cannot pin
// its pages for the transfer), so direct reads go through an aligned bounce buffer of
// this size and a host copy into the staging buffer.
constexpr size_t BOUNCE_BYTES = size_t(32) << 20;

size_t align_down(size_t x) { return x / IO_ALIGN * IO_ALIGN; }
size_t align_up(size_t x) { return (x + IO_ALIGN - 1) / IO_ALIGN * IO_ALIGN; }
}  // namespace

struct LeafFile {
    std::string path;
    int fd = -1;
    bool direct = false;
    int device = 0;
    // staging slots: chunk held or being read (-1: none), ready flag, event after the copy out
    PinnedBuf stage[SLOTS];
    int chunk[SLOTS] = {-1, -1};
    bool ready[SLOTS] = {false, false};
    bool copy_pending[SLOTS] = {false, false};
    hipEvent_t ev_free[SLOTS] = {nullptr, nullptr};
    size_t stage_off[SLOTS] = {0, 0};  // offset of the chunk's first byte inside the slot
    // reader thread
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<int> queue;  // slots to read
    bool stop = false;
    std::string error;
    int64_t bytes = 0;
    double ms = 0;
    const std::vector<Chunk> *chunks = nullptr;
    void *bounce = nullptr;  // aligned host buffer of direct reads (reader thread only)
};

static void read_range(LeafFile &F, int slot, const Chunk &c)
{
    const size_t b0 = (size_t)c.word_lo * 4, b1 = (size_t)c.word_hi * 4;
    const size_t a0 = F.direct ? align_down(b0) : b0;
    const size_t a1 = F.direct ? align_up(b1) : b1;
    char *dst = static_cast<char *>(F.stage[slot].p);
    size_t done = 0;
    while (a0 + done < a1) {
        const size_t want = F.direct ? std::min(BOUNCE_BYTES, a1 - a0 - done) : a1 - a0 - done;
        const ssize_t r = pread(F.fd, F.direct ? F.bounce : dst + done, want, (off_t)(a0 + done));
        if (r < 0) fail(BKD_EDEVICE, std::string("reading the leaf file: ") + std::strerror(errno));
        if (r == 0) {
            if (a0 + done >= b1) break;  // the aligned tail past the end of the file
            fail(BKD_EDEVICE, "leaf file shorter than the leaf structure");
        }
        if (F.direct) std::memcpy(dst + done, F.bounce, (size_t)r);
        done += (size_t)r;
    }
    F.stage_off[slot] = b0 - a0;
    F.bytes += (int64_t)done;
}

static void reader_loop(LeafFile *Fp)
{
    LeafFile &F = *Fp;
    (void)hipSetDevice(F.device);
    std::unique_lock<std::mutex> lk(F.mu);
    for (;;) {
        F.cv.wait(lk, [&] { return F.stop || !F.queue.empty(); });
        if (F.stop) return;
        const int slot = F.queue.front();
        F.queue.pop_front();
        const int j = F.chunk[slot];
        const bool pending = F.copy_pending[slot];
        lk.unlock();
        try {
            // the slot's previous contents must have left for the device
            if (pending) BKD_HIP(hipEventSynchronize(F.ev_free[slot]));
            const auto t0 = std::chrono::steady_clock::now();
            read_range(F, slot, (*F.chunks)[(size_t)j]);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            lk.lock();
            F.ms += ms;
            F.copy_pending[slot] = false;
            F.ready[slot] = true;
        } catch (const BkdError &e) {
            lk.lock();
            F.error = e.msg;
            F.ready[slot] = true;
        }
        F.done_cv.notify_all();
    }
}

void leaffile_create(Tree &t, const float *P, const char *path)
{
    auto F = std::make_unique<LeafFile>();
    F->path = path;
    F->device = t.device;
    F->chunks = &t.chunks;
    {
        // write the structure leaf range by leaf range (at most about 256 MiB of host memory at a time)
        const int fd = open(path, O_WRONLY | O_CREAT | O_TRUNC, 0600);
        if (fd < 0) fail(BKD_EINVAL, std::string("cannot create the leaf file ") + path + ": " + std::strerror(errno));
        std::vector<float> buf;
        int l = 0;
        try {
            while (l < t.nleaf) {
                int e = l + 1;
                while (e < t.nleaf && (t.leaf_blk[(size_t)e + 1] - t.leaf_blk[(size_t)l]) * 4 <= (int64_t(256) << 20)) e++;
                buf.resize((size_t)(t.leaf_blk[(size_t)e] - t.leaf_blk[(size_t)l]));
                gather_leaves(P, t, l, e - 1, buf.data());
                const char *src = reinterpret_cast<const char *>(buf.data());
                size_t left = buf.size() * 4, off = (size_t)t.leaf_blk[(size_t)l] * 4;
                while (left > 0) {
                    const ssize_t w = pwrite(fd, src, left, (off_t)off);
                    if (w <= 0) fail(BKD_ENOMEM, std::string("writing the leaf file: ") + std::strerror(errno));
                    src += w;
                    off += (size_t)w;
                    left -= (size_t)w;
                }
                l = e;
            }
        } catch (...) {
            close(fd);
            unlink(path);
            throw;
        }
        if (fsync(fd) != 0 || close(fd) != 0) {
            unlink(path);
            fail(BKD_ENOMEM, std::string("writing the leaf file: ") + std::strerror(errno));
        }
    }
    F->fd = open(path, O_RDONLY | O_DIRECT);
    F->direct = F->fd >= 0 && posix_memalign(&F->bounce, IO_ALIGN, BOUNCE_BYTES) == 0;
    if (!F->direct) {
        if (F->fd >= 0) close(F->fd);
        F->fd = open(path, O_RDONLY);
    }
    if (F->fd < 0) {
        unlink(path);
        fail(BKD_EINVAL, std::string("cannot open the leaf file ") + path + ": " + std::strerror(errno));
    }
    try {
        for (int s = 0; s < SLOTS; s++) {
            F->stage[s].ensure(t.chunk_cap_bytes + 2 * IO_ALIGN);  // page-aligned pinned memory
            BKD_HIP(hipEventCreateWithFlags(&F->ev_free[s], hipEventDisableTiming));
        }
    } catch (...) {
        for (int s = 0; s < SLOTS; s++)
            if (F->ev_free[s]) (void)hipEventDestroy(F->ev_free[s]);
        close(F->fd);
        free(F->bounce);
        unlink(path);
        throw;
    }
    F->th = std::thread(reader_loop, F.get());
    t.leaf_file = F.release();
}

void leaffile_destroy(Tree &t)
{
    LeafFile *F = t.leaf_file;
    if (!F) return;
    {
        std::lock_guard<std::mutex> g(F->mu);
        F->stop = true;
    }
    F->cv.notify_all();
    if (F->th.joinable()) F->th.join();
    for (int s = 0; s < SLOTS; s++)
        if (F->ev_free[s]) (void)hipEventDestroy(F->ev_free[s]);
    if (F->fd >= 0) close(F->fd);
    free(F->bounce);
    unlink(F->path.c_str());
    delete F;
    t.leaf_file = nullptr;
}

// With the lock held: the slot holding or reading chunk j, else -1.
static int slot_of(LeafFile &F, int j)
{
    for (int s = 0; s < SLOTS; s++)
        if (F.chunk[s] == j) return s;
    return -1;
}

// With the lock held: start reading chunk j into a slot that is not waited for (the slot
// whose copy out was queued longest ago); -1 if both hold chunks not yet copied.
static int start_read(LeafFile &F, int j, bool must)
{
    int s = -1;
    for (int x = 0; x < SLOTS; x++)
        if (F.chunk[x] < 0 || (F.ready[x] && F.copy_pending[x])) {
            s = x;
            break;
        }
    if (s < 0) {
        if (!must) return -1;
        // both slots hold ready chunks nobody has copied yet: drop the older request
        for (int x = 0; x < SLOTS; x++)
            if (F.ready[x]) {
                s = x;
                break;
            }
        if (s < 0) return -1;
    }
    F.chunk[s] = j;
    F.ready[s] = false;
    F.queue.push_back(s);
    F.cv.notify_all();
    return s;
}

void leaffile_prefetch(Tree &t, int j)
{
    LeafFile &F = *t.leaf_file;
    if (j < 0) return;
    std::lock_guard<std::mutex> g(F.mu);
    if (slot_of(F, j) >= 0) return;
    start_read(F, j, false);
}

double leaffile_copy(Tree &t, int j, void *dst, hipStream_t s)
{
    LeafFile &F = *t.leaf_file;
    const auto t0 = std::chrono::steady_clock::now();
    std::unique_lock<std::mutex> lk(F.mu);
    int slot = slot_of(F, j);
    while (slot < 0) {
        slot = start_read(F, j, true);
        if (slot < 0) F.done_cv.wait(lk);  // both slots are being read: wait for one
    }
    F.done_cv.wait(lk, [&] { return F.ready[slot] || !F.error.empty(); });
    if (!F.error.empty()) fail(BKD_EDEVICE, F.error);
    const Chunk &c = t.chunks[(size_t)j];
    const size_t bytes = (size_t)(c.word_hi - c.word_lo) * 4;
    BKD_HIP(hipMemcpyAsync(dst, static_cast<char *>(F.stage[slot].p) + F.stage_off[slot], bytes,
                           hipMemcpyHostToDevice, s));
    BKD_HIP(hipEventRecord(F.ev_free[slot], s));
    F.copy_pending[slot] = true;  // ready and copied: reusable once ev_free completes
    // the slot keeps chunk j until it is refilled, so a repeated request re-copies it
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

bool leaffile_direct(const Tree &t) { return t.leaf_file && t.leaf_file->direct; }

void leaffile_take_stats(Tree &t, int64_t *bytes, double *ms)
{
    LeafFile &F = *t.leaf_file;
    std::lock_guard<std::mutex> g(F.mu);
    *bytes = F.bytes;
    *ms = F.ms;
    F.bytes = 0;
    F.ms = 0;
}

}  // namespace bkd
