// Streaming server of libcfar2d: frames from many streams are admitted to
// the device as memory and in-flight slots free up, grouped into batches,
// and run as TILED batched launches rotating over several HIP streams, so
// frames that arrive while others are on the device overlap with them.
//
// One scheduler thread per server owns all device work.  Per round it
//   1. reaps batches whose completion event has fired (frees their pool
//      memory, posts completions),
//   2. admits queued frames in submission order while the in-flight frame
//      limit and the device pool allow (a frame that does not fit waits, and
//      so do the frames behind it),
//   3. launches the admitted frames as one batch on the least busy stream:
//      host-to-device copies of host frames, cfar2d_batched, device-to-host
//      copies of their masks, an event,
// and sleeps on a condition variable when there is nothing to do.
//
// Device memory: one pool of device_budget_bytes (clamped to the free device
// memory) allocated at creation; frames from host memory take their map and
// mask from it (first fit, coalescing free list), and each HIP stream the
// workspace of its batches (grown on demand).
#include "cfar2d.h"
#include "internal.h"

#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include <time.h>

namespace cfar {
namespace {

int64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

constexpr size_t kAlign = 256;

// First-fit allocator over [0, size) with coalescing free list.
class Pool {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), kAlign);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

struct Frame {
    cfar_map map;       // as submitted (host or device pointers)
    bool on_host;
    bool packed;        // the host mask takes the bit-packed mask (rows x ld_mask words)
    uint64_t ticket, tag;
    int64_t t_submit, t_start;
    size_t off_x = 0, off_m = 0, bytes_x = 0, bytes_m = 0;  // pool blocks of host frames
};

struct Batch {
    std::vector<Frame> frames;
    int stream = 0;
    hipEvent_t done = nullptr;
    int status = CFAR_OK;
};

// Workspace of one HIP stream's batches (a pool block, grown on demand).
struct StreamWs {
    size_t off = 0, bytes = 0;
};

}  // namespace
}  // namespace cfar

struct cfar_server {
    cfar_server_opts opts;
    char *pool_base = nullptr;
    size_t pool_bytes = 0;
    cfar::Pool pool;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;  // batches in flight per stream
    std::vector<cfar::StreamWs> stream_ws;
    std::vector<hipEvent_t> spare_events;

    std::mutex mu;
    std::condition_variable cv_sched;  // work for the scheduler
    std::condition_variable cv_poll;   // completions or state changes
    std::deque<cfar::Frame> queue;
    std::vector<cfar::Batch> inflight;
    std::deque<cfar_completion> done;
    bool accepting = true;
    bool stop = false;
    uint64_t next_ticket = 1;
    cfar_server_stats st{};
    int device = 0;
    // CFAR2D_SERVER_FAIL_TAG (read at creation): every batch holding a frame
    // with this user tag reports failure, after its device work ran, so the
    // failure path can be tested without a device fault
    bool fail_tag_set = false;
    uint64_t fail_tag = 0;
    // CFAR2D_SERVER_GRAPH=1 (read at creation): batches launch with
    // CFAR_BATCH_GRAPH (a replay where a stream's previous batch had the same
    // layout, else a capture)
    int batch_flags = 0;
    std::thread thr;
};

namespace cfar {
namespace {

void post(cfar_server *s, const Frame &f, int status, int64_t t_done)
{
    cfar_completion c;
    std::memset(&c, 0, sizeof c);
    c.ticket = f.ticket;
    c.user_tag = f.tag;
    c.status = status;
    c.t_submit_ns = f.t_submit;
    c.t_start_ns = f.t_start;
    c.t_done_ns = t_done;
    s->done.push_back(c);
    s->st.completed++;
    if (status != CFAR_OK) s->st.failed++;
}

size_t frame_es(const cfar_map &m) { return m.dtype == CFAR_F32 ? 4 : 8; }

// Words per row of a packed mask.
int64_t packed_words(const cfar_map &m) { return (m.cols + 31) / 32; }

// Pool bytes a frame holds while in flight: its map and its mask (and the
// packed mask after the mask, 256-byte aligned, for packed frames).
void frame_bytes(const Frame &f, size_t *bx, size_t *bm)
{
    if (!f.on_host) { *bx = *bm = 0; return; }
    *bx = (size_t)f.map.rows * (size_t)f.map.cols * frame_es(f.map);
    *bm = (size_t)f.map.rows * (size_t)f.map.cols;
    if (f.packed) *bm = align_up(*bm, 256) + (size_t)f.map.rows * (size_t)packed_words(f.map) * 4;
}

// Reap finished batches (lock held).
void reap(cfar_server *s)
{
    for (size_t i = 0; i < s->inflight.size();) {
        Batch &b = s->inflight[i];
        hipError_t q = hipEventQuery(b.done);
        if (q == hipErrorNotReady) { ++i; continue; }
        const int64_t t = now_ns();
        const int status = (q == hipSuccess && b.status == CFAR_OK) ? CFAR_OK : CFAR_EDEVICE;
        for (const Frame &f : b.frames) {
            if (f.bytes_x) s->pool.release(f.off_x, f.bytes_x);
            if (f.bytes_m) s->pool.release(f.off_m, f.bytes_m);
            post(s, f, status, t);
        }
        s->st.inflight_frames -= (int32_t)b.frames.size();
        s->stream_load[b.stream]--;
        s->spare_events.push_back(b.done);
        s->inflight[i] = std::move(s->inflight.back());
        s->inflight.pop_back();
        s->cv_poll.notify_all();
    }
    s->st.device_bytes_in_use = s->pool.used();
}

// Enqueue one batch on its stream (HIP calls are asynchronous; the lock
// is not held: only the scheduler thread touches batches, streams and the
// pool's blocks).
int launch(cfar_server *s, Batch &b)
{
    hipStream_t st = s->streams[b.stream];
    const StreamWs &ws = s->stream_ws[b.stream];
    std::vector<cfar_map> maps;
    maps.reserve(b.frames.size());
    for (Frame &f : b.frames) {
        cfar_map m = f.map;
        if (f.on_host) {
            char *dx = s->pool_base + f.off_x;
            uint8_t *dm = (uint8_t *)(s->pool_base + f.off_m);
            const size_t es = frame_es(m);
            // contiguous frames as one copy (a 2D copy may go row by row)
            hipError_t e = m.ld == m.cols
                               ? hipMemcpyAsync(dx, m.x, (size_t)m.rows * (size_t)m.cols * es, hipMemcpyHostToDevice, st)
                               : hipMemcpy2DAsync(dx, (size_t)m.cols * es, m.x, (size_t)m.ld * es,
                                                  (size_t)m.cols * es, (size_t)m.rows, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return hip_error(e, "hipMemcpy2DAsync(frame in)");
            m.x = dx;
            m.ld = m.cols;
            m.mask = dm;
            m.ld_mask = m.cols;
        }
        maps.push_back(m);
    }
    int rc = cfar2d_batched(maps.data(), (int32_t)maps.size(), CFAR_FORM_TILED, s->batch_flags, s->pool_base + ws.off,
                            ws.bytes, st);
    if (rc != CFAR_OK) return rc;
    for (size_t i = 0; i < b.frames.size(); ++i) {
        const Frame &f = b.frames[i];
        if (!f.on_host) continue;
        if (f.packed) {  // pack on the device, copy the words back
            const int64_t words = packed_words(f.map);
            uint32_t *dp = (uint32_t *)(s->pool_base + f.off_m +
                                        align_up((size_t)f.map.rows * (size_t)f.map.cols, 256));
            int prc = cfar_mask_pack(&maps[i], dp, words, st);
            if (prc != CFAR_OK) return prc;
            hipError_t e = f.map.ld_mask == words
                               ? hipMemcpyAsync(f.map.mask, dp, (size_t)f.map.rows * (size_t)words * 4,
                                                hipMemcpyDeviceToHost, st)
                               : hipMemcpy2DAsync(f.map.mask, (size_t)f.map.ld_mask * 4, dp, (size_t)words * 4,
                                                  (size_t)words * 4, (size_t)f.map.rows, hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return hip_error(e, "hipMemcpy2DAsync(packed mask out)");
            continue;
        }
        hipError_t e = f.map.ld_mask == f.map.cols
                           ? hipMemcpyAsync(f.map.mask, maps[i].mask, (size_t)f.map.rows * (size_t)f.map.cols,
                                            hipMemcpyDeviceToHost, st)
                           : hipMemcpy2DAsync(f.map.mask, (size_t)f.map.ld_mask, maps[i].mask, (size_t)f.map.cols,
                                              (size_t)f.map.cols, (size_t)f.map.rows, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_error(e, "hipMemcpy2DAsync(mask out)");
    }
    hipError_t e = hipEventRecord(b.done, st);
    if (e != hipSuccess) return hip_error(e, "hipEventRecord(batch)");
    return CFAR_OK;
}

// Give a frame's pool blocks back and requeue it at the head (lock held).
void requeue(cfar_server *s, Frame f)
{
    if (f.bytes_x) s->pool.release(f.off_x, f.bytes_x);
    if (f.bytes_m) s->pool.release(f.off_m, f.bytes_m);
    f.bytes_x = f.bytes_m = 0;
    s->queue.push_front(f);
}

// Workspace bytes of a batch of frames.
size_t batch_ws_bytes(cfar_server *s, const std::vector<Frame> &frames)
{
    std::vector<cfar_map> probe;
    for (const Frame &f : frames) {
        cfar_map m = f.map;
        if (f.on_host) {  // sizing only: any device pointers with the pool's layout
            m.x = s->pool_base;
            m.mask = (uint8_t *)s->pool_base;
            m.ld = m.cols;
            m.ld_mask = m.cols;
        }
        probe.push_back(m);
    }
    return cfar_workspace_bytes(probe.data(), (int32_t)probe.size(), CFAR_FORM_TILED);
}

// Admit queued frames into one batch on the least busy stream (lock held).
// Returns false if nothing could be admitted.
bool admit(cfar_server *s, Batch &b)
{
    if (s->queue.empty()) return false;
    const int max_batch = std::max(1, std::min(s->opts.max_batch_frames, s->opts.max_inflight_frames));
    int si = 0;
    for (int i = 1; i < (int)s->streams.size(); ++i)
        if (s->stream_load[i] < s->stream_load[si]) si = i;
    b = Batch();
    b.stream = si;
    while (!s->queue.empty() && (int)b.frames.size() < max_batch &&
           s->st.inflight_frames + (int)b.frames.size() < s->opts.max_inflight_frames) {
        Frame f = s->queue.front();
        size_t bx, bm, ox = 0, om = 0;
        frame_bytes(f, &bx, &bm);
        if (bx && !s->pool.alloc(bx, &ox)) break;
        if (bm && !s->pool.alloc(bm, &om)) {
            if (bx) s->pool.release(ox, bx);
            break;
        }
        f.off_x = ox;
        f.off_m = om;
        f.bytes_x = bx;
        f.bytes_m = bm;
        b.frames.push_back(f);
        s->queue.pop_front();
    }
    // the stream's workspace must hold the batch; grow it (after the stream's
    // earlier batches, which use it, have finished) or give frames back
    StreamWs &ws = s->stream_ws[si];
    while (!b.frames.empty()) {
        const size_t need = batch_ws_bytes(s, b.frames);
        if (need && need <= ws.bytes) break;
        if (need) {
            const size_t want = align_up(need + need / 2, kAlign);
            if (s->stream_load[si] == 0) {
                if (ws.bytes) {
                    drop_batch_ctx(s->streams[si], s->pool_base + ws.off);
                    s->pool.release(ws.off, ws.bytes);
                    ws.bytes = 0;
                }
                size_t off;
                if (s->pool.alloc(want, &off)) {
                    ws.off = off;
                    ws.bytes = want;
                    continue;
                }
            }
        }
        Frame f = b.frames.back();
        b.frames.pop_back();
        requeue(s, f);
    }
    return !b.frames.empty();
}

// Launch an admitted batch (lock held on entry and exit, released around
// the HIP calls).
void launch_admitted(cfar_server *s, std::unique_lock<std::mutex> &lk, Batch &b)
{
    if (s->spare_events.empty()) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
        s->spare_events.push_back(ev);
    }
    b.done = s->spare_events.back();
    s->spare_events.pop_back();
    const int64_t t = now_ns();
    for (Frame &f : b.frames) f.t_start = t;
    s->st.inflight_frames += (int32_t)b.frames.size();
    s->stream_load[b.stream]++;
    s->st.device_bytes_in_use = s->pool.used();
    s->st.device_bytes_peak = std::max(s->st.device_bytes_peak, s->pool.used());
    lk.unlock();
    int rc = b.done ? launch(s, b) : CFAR_EDEVICE;
    if (rc == CFAR_OK && s->fail_tag_set) {  // forced failure of a batch (tests of the failure path)
        for (const Frame &f : b.frames)
            if (f.tag == s->fail_tag) rc = set_error(CFAR_EDEVICE, "batch failed (forced for tag %llu)",
                                                     (unsigned long long)f.tag);
    }
    if (rc != CFAR_OK) (void)hipStreamSynchronize(s->streams[b.stream]);  // let what was enqueued finish
    lk.lock();
    b.status = rc;
    if (rc != CFAR_OK && !b.done) {
        // no event to wait for: complete the frames now
        for (const Frame &f : b.frames) {
            if (f.bytes_x) s->pool.release(f.off_x, f.bytes_x);
            if (f.bytes_m) s->pool.release(f.off_m, f.bytes_m);
            post(s, f, CFAR_EDEVICE, now_ns());
        }
        s->st.inflight_frames -= (int32_t)b.frames.size();
        s->stream_load[b.stream]--;
        s->cv_poll.notify_all();
        return;
    }
    if (rc != CFAR_OK) (void)hipEventRecord(b.done, s->streams[b.stream]);  // reaped with status EDEVICE
    s->st.batches++;
    s->inflight.push_back(std::move(b));
}

void scheduler(cfar_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        reap(s);
        bool launched = false;
        Batch b;
        while (admit(s, b)) {
            launch_admitted(s, lk, b);
            launched = true;
            reap(s);
        }
        s->st.queued_frames = (int32_t)s->queue.size();
        if (s->stop && s->inflight.empty()) break;
        if (launched) continue;
        // device work in flight: poll its events often; else sleep until a
        // submit or a state change
        if (!s->inflight.empty())
            s->cv_sched.wait_for(lk, std::chrono::microseconds(50));
        else if (!s->stop && s->queue.empty())
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(5));
        else if (!s->queue.empty())
            s->cv_sched.wait_for(lk, std::chrono::microseconds(200));
    }
    s->cv_poll.notify_all();
}

}  // namespace
}  // namespace cfar

using namespace cfar;

extern "C" {

int cfar_host_alloc(size_t bytes, void **out)
{
    if (!out || bytes == 0) return set_error(CFAR_EINVAL, "bytes is 0 or out is NULL");
    *out = nullptr;
    hipError_t e = hipHostMalloc(out, bytes, hipHostMallocDefault);
    if (e != hipSuccess) return hip_error(e, "hipHostMalloc");
    return CFAR_OK;
}

int cfar_host_free(void *p)
{
    if (!p) return CFAR_OK;
    hipError_t e = hipHostFree(p);
    if (e != hipSuccess) return hip_error(e, "hipHostFree");
    return CFAR_OK;
}

int cfar_server_create(const cfar_server_opts *opts, cfar_server **out)
{
    if (!opts || !out) return set_error(CFAR_EINVAL, "opts or out is NULL");
    *out = nullptr;
    cfar_server_opts o = *opts;
    if (o.device_budget_bytes < (1u << 20)) return set_error(CFAR_EINVAL, "device_budget_bytes below 1 MiB");
    if (o.max_inflight_frames < 1) return set_error(CFAR_EINVAL, "max_inflight_frames must be >= 1");
    if (o.n_hip_streams < 1 || o.n_hip_streams > 16) return set_error(CFAR_EINVAL, "n_hip_streams must be 1..16");
    if (o.queue_depth < 1) return set_error(CFAR_EINVAL, "queue_depth must be >= 1");
    if (o.max_batch_frames < 1) return set_error(CFAR_EINVAL, "max_batch_frames must be >= 1");
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return hip_error(e, "hipMemGetInfo");
    // keep a margin for the HIP runtime and other users of the device
    const size_t cap = free_b > (size_t(256) << 20) ? free_b - (size_t(256) << 20) : free_b / 2;
    o.device_budget_bytes = align_up(std::min(o.device_budget_bytes, cap), kAlign);
    std::unique_ptr<cfar_server> s(new cfar_server());
    s->opts = o;
    (void)hipGetDevice(&s->device);
    if (const char *ft = std::getenv("CFAR2D_SERVER_FAIL_TAG")) {
        s->fail_tag_set = true;
        s->fail_tag = std::strtoull(ft, nullptr, 10);
    }
    if (const char *g = std::getenv("CFAR2D_SERVER_GRAPH"))
        if (std::atoi(g) == 1) s->batch_flags = CFAR_BATCH_GRAPH;
    e = hipMalloc((void **)&s->pool_base, o.device_budget_bytes);
    if (e != hipSuccess) return hip_error(e, "hipMalloc(server pool)");
    s->pool_bytes = o.device_budget_bytes;
    s->pool.reset(s->pool_bytes);
    for (int i = 0; i < o.n_hip_streams; ++i) {
        hipStream_t st;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            (void)hipFree(s->pool_base);
            return hip_error(e, "hipStreamCreate(server)");
        }
        s->streams.push_back(st);
        s->stream_load.push_back(0);
        s->stream_ws.push_back(StreamWs());
    }
    cfar_server *raw = s.release();
    raw->thr = std::thread(scheduler, raw);
    *out = raw;
    return CFAR_OK;
}

int cfar_submit(cfar_server *s, const cfar_map *frame, int32_t flags, uint64_t user_tag, uint64_t *ticket_out)
{
    if (!s || !frame || !ticket_out) return set_error(CFAR_EINVAL, "server, frame or ticket_out is NULL");
    if (flags & ~(CFAR_SUBMIT_HOST | CFAR_SUBMIT_PACKED_MASK)) return set_error(CFAR_EINVAL, "unknown flags 0x%x", flags);
    const bool on_host = (flags & CFAR_SUBMIT_HOST) != 0, packed = (flags & CFAR_SUBMIT_PACKED_MASK) != 0;
    if (packed && !on_host) return set_error(CFAR_EINVAL, "CFAR_SUBMIT_PACKED_MASK needs CFAR_SUBMIT_HOST");
    cfar_map v = *frame;
    if (packed) {  // ld_mask counts 32-bit words; the device-side mask is dense
        if (frame->ld_mask < packed_words(*frame) || frame->ld_mask < 1)
            return set_error(CFAR_EINVAL, "packed mask: ld_mask (words) < ceil(cols / 32)");
        v.ld_mask = v.cols;
    }
    int rc = validate_map(&v, 0, CFAR_FORM_TILED);
    if (rc != CFAR_OK) return rc;
    if (on_host && (frame->train_sum || frame->threshold))
        return set_error(CFAR_EINVAL, "frames from host memory take no training-sum or threshold output");
    Frame f;
    f.map = *frame;
    f.on_host = on_host;
    f.packed = packed;
    f.tag = user_tag;
    size_t bx, bm;
    frame_bytes(f, &bx, &bm);
    const size_t ws = cfar_workspace_bytes(&v, 1, CFAR_FORM_TILED);
    if (!ws) return CFAR_EINVAL;
    if (align_up(bx, kAlign) + align_up(bm, kAlign) + align_up(ws + ws / 2, kAlign) > s->pool_bytes)
        return set_error(CFAR_EINVAL, "frame needs more device memory than the server's budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->accepting) return set_error(CFAR_ESHUTDOWN, "server is shutting down");
    if ((int)s->queue.size() >= s->opts.queue_depth) return set_error(CFAR_EAGAIN, "queue full");
    f.ticket = s->next_ticket++;
    f.t_submit = now_ns();
    f.t_start = 0;
    s->queue.push_back(f);
    s->st.submitted++;
    s->st.queued_frames = (int32_t)s->queue.size();
    *ticket_out = f.ticket;
    s->cv_sched.notify_one();
    return CFAR_OK;
}

int cfar_poll(cfar_server *s, cfar_completion *out, int32_t max, int32_t timeout_us, int32_t *n_out)
{
    if (!s || !n_out || (max > 0 && !out)) return set_error(CFAR_EINVAL, "server, out or n_out is NULL");
    *n_out = 0;
    if (max <= 0) return CFAR_OK;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return !s->done.empty() || s->stop; };
    // (frames being launched have left the queue but are not yet in
    // `inflight`; inflight_frames counts them from admission on)
    if (timeout_us < 0)
        s->cv_poll.wait(lk, [&] {
            return !s->done.empty() || (s->queue.empty() && s->st.inflight_frames == 0 && !s->accepting) ||
                   s->stop;
        });
    else if (timeout_us > 0)
        s->cv_poll.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
    int n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return CFAR_OK;
}

int cfar_server_stats_get(cfar_server *s, cfar_server_stats *out)
{
    if (!s || !out) return set_error(CFAR_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued_frames = (int32_t)s->queue.size();
    return CFAR_OK;
}

int cfar_server_shutdown(cfar_server *s, int32_t drain_queued)
{
    if (!s) return set_error(CFAR_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->accepting = false;
    if (!drain_queued) {
        const int64_t t = now_ns();
        while (!s->queue.empty()) {
            post(s, s->queue.front(), CFAR_ESHUTDOWN, t);
            s->queue.pop_front();
        }
        s->st.queued_frames = 0;
        s->cv_poll.notify_all();
    }
    s->cv_sched.notify_one();
    // the scheduler keeps running until the queue and the device are empty
    // (inflight_frames also counts admitted frames whose batch is being
    // launched, which are in neither list)
    while (!s->queue.empty() || s->st.inflight_frames > 0) {
        s->cv_poll.wait_for(lk, std::chrono::milliseconds(1));
        s->cv_sched.notify_one();
    }
    return CFAR_OK;
}

int cfar_server_destroy(cfar_server *s)
{
    if (!s) return set_error(CFAR_EINVAL, "server is NULL");
    cfar_server_shutdown(s, 0);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_sched.notify_one();
    }
    if (s->thr.joinable()) s->thr.join();
    for (size_t i = 0; i < s->streams.size(); ++i) {
        (void)hipStreamSynchronize(s->streams[i]);
        if (s->stream_ws[i].bytes) drop_batch_ctx(s->streams[i], s->pool_base + s->stream_ws[i].off);
        (void)hipStreamDestroy(s->streams[i]);
    }
    for (hipEvent_t ev : s->spare_events)
        if (ev) (void)hipEventDestroy(ev);
    if (s->pool_base) (void)hipFree(s->pool_base);
    delete s;
    return CFAR_OK;
}

}  // extern "C"
