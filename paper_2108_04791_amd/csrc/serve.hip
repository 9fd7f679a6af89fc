// serve.hip -- request server with continuous batching (host code).
//
// A client submits a request (host arrays n[len] -> out[len]) and gets a
// ticket.  Admission reserves 9 bytes per element (8 in, 1 out) from the
// memory budget; a request that does not fit waits (or is refused with
// ISP_EBUSY) until earlier requests complete.  Admitted requests are split
// into pieces of at most max_batch_elems and queued.
//
// The dispatcher thread keeps up to max_inflight batches on the device: as
// soon as a slot is free it packs the queued pieces (in arrival order) into
// that slot's batch and hands it to the slot's own worker thread.  The
// worker stages the inputs into the slot's pinned buffer, enqueues on the
// slot's own stream the isprime_u64 kernels over the whole packed buffer
// (elements are independent, so one call classifies every piece) and an
// event, waits for the event, scatters the results to the requests' output
// arrays and completes each request whose last piece has arrived.  The
// pinned buffers are mapped and coherent: the kernels read the values and
// write the verdicts there directly, so no copy engine is on the path
// (asynchronous copies from pinned memory were measured to stall every
// slot for 7-9 ms now and then, a few times a second).  Requests that
// arrive while other batches run are packed into the next batch as
// capacity frees up, batches on different streams overlap on the device,
// and staging, launching and completing run in parallel across slots.  A
// failed batch fails exactly the requests that had pieces in it.
//
// Test mode (cfg.test_mode = 1): no device at all; a batch "runs" on its
// slot's worker thread and writes n & 1 for every element, optionally after a
// delay and with every k-th batch failing, so the queueing, admission,
// splitting and error paths can be checked on a machine without a GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    const uint64_t *n = nullptr;
    uint8_t *out = nullptr;
    size_t len = 0;
    size_t pieces_left = 0;
    size_t bytes = 0;
    int status = ISP_OK;
    bool done = false;
};

struct Piece {
    Request *req;
    size_t off;  // in the request
    size_t len;
};

// Host copies of one batch (dst, src, bytes) split over a few persistent
// threads and the calling thread.  One host thread copies about 10 GB/s into
// pinned memory, well below what the host memory system and the PCIe link
// carry, and staging each batch's inputs is the serving path's bottleneck.
class CopyPool {
public:
    struct Seg {
        void *dst;
        const void *src;
        size_t bytes;
    };

    explicit CopyPool(int workers)
    {
        for (int i = 0; i < workers; ++i)
            th_.emplace_back([this, i] { loop(i + 1); });
    }
    ~CopyPool()
    {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_)
            t.join();
    }
    // Every segment copied when it returns.  Batches below a few hundred KB
    // are copied by the caller alone.
    void run(const std::vector<Seg> &segs)
    {
        size_t total = 0;
        for (const Seg &x : segs)
            total += x.bytes;
        if (th_.empty() || total < ((size_t)256 << 10)) {
            copy_range(segs, 0, total);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            job_ = &segs;
            total_ = total;
            parts_ = th_.size() + 1;
            left_ = th_.size();
            ++gen_;
        }
        cv_.notify_all();
        copy_part(segs, total, 0, th_.size() + 1);
        std::unique_lock<std::mutex> g(mu_);
        cv_done_.wait(g, [&] { return left_ == 0; });
        job_ = nullptr;
    }

private:
    static void copy_range(const std::vector<Seg> &segs, size_t b0, size_t b1)
    {
        size_t at = 0;  // byte offset of the current segment in the batch
        for (const Seg &x : segs) {
            const size_t s0 = std::max(b0, at), s1 = std::min(b1, at + x.bytes);
            if (s0 < s1)
                std::memcpy(static_cast<char *>(x.dst) + (s0 - at),
                            static_cast<const char *>(x.src) + (s0 - at), s1 - s0);
            at += x.bytes;
            if (at >= b1)
                break;
        }
    }
    static void copy_part(const std::vector<Seg> &segs, size_t total, size_t part, size_t parts)
    {
        // 4 KB-aligned cut points
        auto cut = [&](size_t k) { return k >= parts ? total : std::min(total, (total / parts * k) & ~(size_t)4095); };
        copy_range(segs, cut(part), cut(part + 1));
    }
    void loop(size_t part)
    {
        uint64_t seen = 0;
        for (;;) {
            const std::vector<Seg> *job;
            size_t total, parts;
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return stop_ || gen_ != seen; });
                if (stop_)
                    return;
                seen = gen_;
                job = job_;
                total = total_;
                parts = parts_;
            }
            copy_part(*job, total, part, parts);
            {
                std::lock_guard<std::mutex> g(mu_);
                if (--left_ == 0)
                    cv_done_.notify_all();
            }
        }
    }

    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, cv_done_;
    const std::vector<Seg> *job_ = nullptr;
    size_t total_ = 0, parts_ = 0, left_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t *h_n = nullptr;  // pinned, mapped, coherent (plain heap in test mode)
    uint8_t *h_out = nullptr;
    const uint64_t *dev_n = nullptr;  // the device's addresses of h_n and h_out
    uint8_t *dev_out = nullptr;
    std::vector<Piece> pieces;
    size_t elems = 0;
    int status = ISP_OK;
    bool busy = false;  // a batch is assigned (until it completes)
    std::thread worker;
};

}  // namespace

struct isp_server {
    isp_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_dispatch;  // queued work or a free slot
    std::condition_variable cv_work;      // a batch assigned to a slot, or the end
    std::condition_variable cv_space;     // budget freed
    std::condition_variable cv_done;      // a request completed
    std::deque<Piece> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
    std::vector<std::unique_ptr<Slot>> slots;
    uint64_t next_ticket = 1;
    uint64_t bytes_in_use = 0;
    uint64_t batches = 0;  // batches run (test mode counts failures by it)
    uint64_t device_bytes = 0;  // the slots' device workspaces, reserved at creation
    uint64_t pinned_bytes = 0;  // the slots' pinned staging buffers
    bool stop = false;
    bool dispatcher_done = false;
    std::mutex stage_mu;  // one batch staged at a time, with all the copy threads
    std::unique_ptr<CopyPool> stage_pool;
    std::thread dispatcher;
};

namespace {

constexpr size_t BYTES_PER_ELEM = sizeof(uint64_t) + sizeof(uint8_t);
constexpr int SERVER_COPY_THREADS = 3;  // staging helpers next to the staging worker

void free_slot_resources(isp_server *s, Slot &sl)
{
    if (s->cfg.test_mode) {
        delete[] sl.h_n;
        delete[] sl.h_out;
    } else {
        if (sl.h_n)
            (void)hipHostFree(sl.h_n);
        if (sl.h_out)
            (void)hipHostFree(sl.h_out);
        if (sl.done)
            (void)hipEventDestroy(sl.done);
        if (sl.stream) {
            isp::release_stream_ws(s->cfg.device, sl.stream);
            (void)hipStreamDestroy(sl.stream);
        }
    }
    sl = Slot();
}

// Caller holds s->mu.  Marks the pieces of a finished batch.
void finish_batch(isp_server *s, Slot &sl)
{
    for (const Piece &p : sl.pieces) {
        Request *r = p.req;
        if (sl.status != ISP_OK && r->status == ISP_OK)
            r->status = sl.status;
        if (--r->pieces_left == 0) {
            r->done = true;
            s->bytes_in_use -= r->bytes;
        }
    }
    sl.pieces.clear();
    sl.elems = 0;
    sl.status = ISP_OK;
    sl.busy = false;
}

void dispatcher_main(isp_server *s)
{
    const size_t cap = s->cfg.max_batch_elems;
    for (;;) {
        Slot *sl = nullptr;
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_dispatch.wait(g, [&] {
                if (s->stop && s->queue.empty())
                    return true;
                if (s->queue.empty())
                    return false;
                for (auto &x : s->slots)
                    if (!x->busy)
                        return true;
                return false;
            });
            if (s->queue.empty()) {  // stopping and drained
                s->dispatcher_done = true;
                break;
            }
            for (auto &x : s->slots)
                if (!x->busy) {
                    sl = x.get();
                    break;
                }
            // pack queued pieces in arrival order
            while (!s->queue.empty() && (int)sl->pieces.size() < s->cfg.max_batch_reqs &&
                   sl->elems + s->queue.front().len <= cap) {
                sl->pieces.push_back(s->queue.front());
                sl->elems += s->queue.front().len;
                s->queue.pop_front();
            }
            sl->busy = true;
        }
        s->cv_work.notify_all();
    }
    s->cv_work.notify_all();
}

// One slot's worker: runs each batch the dispatcher assigns to the slot,
// from staging to completion.
void slot_main(isp_server *s, Slot *sl)
{
    if (!s->cfg.test_mode)
        (void)hipSetDevice(s->cfg.device);
    for (;;) {
        {
            std::unique_lock<std::mutex> g(s->mu);
            s->cv_work.wait(g, [&] { return sl->busy || s->dispatcher_done; });
            if (!sl->busy)
                return;  // the dispatcher finished and nothing is assigned
        }
        // stage the inputs (outside the server lock: the host arrays belong
        // to the requests until they complete)
        {
            std::vector<CopyPool::Seg> segs;
            segs.reserve(sl->pieces.size());
            size_t off = 0;
            for (const Piece &p : sl->pieces) {
                segs.push_back({sl->h_n + off, p.req->n + p.off, p.len * sizeof(uint64_t)});
                off += p.len;
            }
            std::lock_guard<std::mutex> sg(s->stage_mu);
            s->stage_pool->run(segs);
        }
        uint64_t seq;
        {
            std::lock_guard<std::mutex> g(s->mu);
            seq = ++s->batches;
        }
        int st = ISP_OK;
        if (s->cfg.test_mode) {
            if (s->cfg.test_delay_us > 0)
                std::this_thread::sleep_for(std::chrono::microseconds(s->cfg.test_delay_us));
            if (s->cfg.test_fail_every > 0 && seq % (uint64_t)s->cfg.test_fail_every == 0)
                st = ISP_EDEVICE;
            else
                for (size_t i = 0; i < sl->elems; ++i)
                    sl->h_out[i] = (uint8_t)(sl->h_n[i] & 1);
        } else {
            st = isprime_u64(sl->dev_n, sl->dev_out, sl->elems, sl->stream);
            hipError_t e = st == ISP_OK ? hipEventRecord(sl->done, sl->stream) : hipSuccess;
            if (st == ISP_OK && e == hipSuccess)
                e = hipEventSynchronize(sl->done);
            else
                (void)hipStreamSynchronize(sl->stream);  // whatever was enqueued
            if (e != hipSuccess && st == ISP_OK)
                st = ISP_EDEVICE;
        }
        if (st == ISP_OK) {
            size_t off = 0;
            for (const Piece &p : sl->pieces) {
                std::memcpy(p.req->out + p.off, sl->h_out + off, p.len);
                off += p.len;
            }
        }
        {
            std::lock_guard<std::mutex> g(s->mu);
            sl->status = st;
            finish_batch(s, *sl);
        }
        s->cv_done.notify_all();
        s->cv_space.notify_all();
        s->cv_dispatch.notify_one();
    }
}

}  // namespace

extern "C" {

int isp_server_create(const isp_server_config *cfg, isp_server **srv)
{
    if (!cfg || !srv)
        return ISP_EINVAL;
    std::unique_ptr<isp_server> s(new isp_server());
    s->cfg = *cfg;
    isp_server_config &c = s->cfg;
    // 8 slots of 2^18 elements: a request of up to 2^20 elements is split
    // over several slots that run it in parallel (measured on the C5 stream
    // at 42 k requests/s: p50 0.33 / p99 1.08 ms, against 0.45 / 1.55 ms
    // for 6 slots of 2^20, at the same capacity of about 60 k requests/s;
    // 2^17-element slots lost capacity, 2^16 lost half of it)
    if (!c.max_inflight)
        c.max_inflight = 8;
    if (!c.mem_budget_bytes)
        c.mem_budget_bytes = (uint64_t)1 << 30;
    if (!c.max_batch_elems)
        c.max_batch_elems = (uint64_t)1 << 18;
    if (!c.max_batch_reqs)
        c.max_batch_reqs = 1024;
    if (c.max_inflight < 1 || c.max_inflight > 8 || c.max_batch_reqs < 1 ||
        c.max_batch_elems > ((uint64_t)1 << 28) || c.test_mode < 0 || c.test_mode > 1)
        return ISP_EINVAL;
    if (!c.test_mode) {
        int st = isp_init(c.device);
        if (st != ISP_OK)
            return st;
    }
    int prev = 0;
    if (!c.test_mode && hipGetDevice(&prev) != hipSuccess)
        return ISP_EDEVICE;
    if (!c.test_mode && hipSetDevice(c.device) != hipSuccess)
        return ISP_EDEVICE;
    int st = ISP_OK;
    for (int k = 0; k < c.max_inflight && st == ISP_OK; ++k) {
        std::unique_ptr<Slot> sl(new Slot());
        const size_t cap = c.max_batch_elems;
        if (c.test_mode) {
            sl->h_n = new uint64_t[cap];
            sl->h_out = new uint8_t[cap];
        } else {
            hipError_t e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&sl->done, hipEventDisableTiming);
            const unsigned fl = hipHostMallocMapped | hipHostMallocCoherent;
            if (e == hipSuccess)
                e = hipHostMalloc(&sl->h_n, cap * sizeof(uint64_t), fl);
            if (e == hipSuccess)
                e = hipHostMalloc(&sl->h_out, cap, fl);
            void *dn = nullptr, *dout = nullptr;
            if (e == hipSuccess)
                e = hipHostGetDevicePointer(&dn, sl->h_n, 0);
            if (e == hipSuccess)
                e = hipHostGetDevicePointer(&dout, sl->h_out, 0);
            sl->dev_n = static_cast<const uint64_t *>(dn);
            sl->dev_out = static_cast<uint8_t *>(dout);
            // the workspace of the slot's stream, at its largest batch now,
            // so that serving never allocates device memory
            uint64_t wb = 0;
            if (e == hipSuccess) {
                st = isp::reserve_stream_ws(c.device, sl->stream, cap, &wb);
                s->device_bytes += wb;
                s->pinned_bytes += cap * BYTES_PER_ELEM;
            }
            if (e != hipSuccess && st == ISP_OK)
                st = e == hipErrorOutOfMemory ? ISP_ENOMEM : ISP_EDEVICE;
        }
        s->slots.push_back(std::move(sl));
    }
    if (!c.test_mode)
        (void)hipSetDevice(prev);
    if (st != ISP_OK) {
        for (auto &sl : s->slots)
            free_slot_resources(s.get(), *sl);
        return st;
    }
    isp_server *raw = s.release();
    raw->stage_pool.reset(new CopyPool(SERVER_COPY_THREADS));
    for (auto &sl : raw->slots)
        sl->worker = std::thread(slot_main, raw, sl.get());
    raw->dispatcher = std::thread(dispatcher_main, raw);
    *srv = raw;
    return ISP_OK;
}

int isp_submit(isp_server *s, const uint64_t *host_n, uint8_t *host_out, size_t len,
               uint64_t *ticket)
{
    if (!s || !ticket || (len && (!host_n || !host_out)))
        return ISP_EINVAL;
    if (len > UINT64_MAX / BYTES_PER_ELEM)  // no such host array; keeps bytes exact
        return ISP_EINVAL;
    const uint64_t bytes = (uint64_t)len * BYTES_PER_ELEM;
    std::unique_lock<std::mutex> g(s->mu);
    if (s->stop)
        return ISP_EINVAL;
    // admit when it fits the budget, or when nothing else holds any of it
    auto fits = [&] { return s->bytes_in_use == 0 || s->bytes_in_use + bytes <= s->cfg.mem_budget_bytes; };
    if (!fits()) {
        if (!s->cfg.block_on_full)
            return ISP_EBUSY;
        s->cv_space.wait(g, fits);
    }
    std::unique_ptr<Request> r(new Request());
    r->ticket = s->next_ticket++;
    r->n = host_n;
    r->out = host_out;
    r->len = len;
    r->bytes = bytes;
    const size_t cap = s->cfg.max_batch_elems;
    r->pieces_left = len ? (len + cap - 1) / cap : 0;
    if (len == 0) {
        r->done = true;
    } else {
        s->bytes_in_use += bytes;
        for (size_t off = 0; off < len; off += cap)
            s->queue.push_back(Piece{r.get(), off, std::min(cap, len - off)});
    }
    *ticket = r->ticket;
    s->reqs[r->ticket] = std::move(r);
    g.unlock();
    s->cv_dispatch.notify_one();
    if (len == 0)
        s->cv_done.notify_all();
    return ISP_OK;
}

int isp_poll(isp_server *s, uint64_t ticket)
{
    if (!s)
        return ISP_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return ISP_ENOENT;
    if (!it->second->done)
        return 0;
    return it->second->status == ISP_OK ? 1 : it->second->status;
}

int isp_wait(isp_server *s, uint64_t ticket, int64_t timeout_us)
{
    if (!s)
        return ISP_EINVAL;
    std::unique_lock<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return ISP_ENOENT;
    Request *r = it->second.get();
    if (timeout_us < 0) {
        s->cv_done.wait(g, [&] { return r->done; });
    } else if (!s->cv_done.wait_for(g, std::chrono::microseconds(timeout_us),
                                    [&] { return r->done; })) {
        return ISP_ETIMEDOUT;
    }
    const int st = r->status;
    s->reqs.erase(ticket);
    return st;
}

int isp_server_footprint(const isp_server *s, uint64_t *device_bytes, uint64_t *pinned_bytes)
{
    if (!s || !device_bytes || !pinned_bytes)
        return ISP_EINVAL;
    *device_bytes = s->device_bytes;
    *pinned_bytes = s->pinned_bytes;
    return ISP_OK;
}

int isp_server_destroy(isp_server *s)
{
    if (!s)
        return ISP_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv_dispatch.notify_all();
    if (s->dispatcher.joinable())
        s->dispatcher.join();  // the queue is drained into the slots
    for (auto &sl : s->slots)
        if (sl->worker.joinable())
            sl->worker.join();  // each finishes its batch, then sees the end
    if (!s->cfg.test_mode)
        (void)hipSetDevice(s->cfg.device);
    for (auto &sl : s->slots)
        free_slot_resources(s, *sl);
    delete s;
    return ISP_OK;
}

}  // extern "C"
