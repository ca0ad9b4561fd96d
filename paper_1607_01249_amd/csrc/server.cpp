// Serving: a request loop with continuous batching.
//
// Clients submit transpositions (Eqn. 1 each) at any time.  A dispatcher
// thread admits them in arrival order while their HBM footprint fits the
// budget (a fraction of the device memory free when the server starts),
// gives each admitted request an output region in a server-owned arena,
// and groups whatever is ready into a micro-batch whenever one of K device
// slots is free.  A slot owns a stream, a descriptor ring entry in device
// memory and a completion event; the micro-batch is one launch of the
// persistent batched kernel.  Requests that arrive while other micro-batches
// run are admitted and launched as soon as a slot and memory free up, so
// their work overlaps on the device.  Completion is observed by polling the
// slots' events; latency is completion minus arrival.
//
// The arithmetic is the batched kernel's, which is the per-call kernels'
// tile code: a request's result does not depend on what it was batched with.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "ttx_internal.h"

using Clock = std::chrono::steady_clock;

static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

namespace ttx {

// First-fit allocator over [0, size) with coalescing free ranges.
class Arena {
   public:
    void reset(int64_t size) {
        free_.clear();
        if (size > 0) free_[0] = size;
        size_ = size;
    }
    int64_t alloc(int64_t bytes) {
        bytes = (bytes + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes) {
        bytes = (bytes + 255) & ~int64_t(255);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    int64_t size() const { return size_; }

   private:
    std::map<int64_t, int64_t> free_;
    int64_t size_ = 0;
};

enum ReqState { WAITING = 0, READY = 1, RUNNING = 2, DONE = 3 };

// Requests of at least this many algorithmic bytes run alone.
static constexpr int64_t kDirectBytes = int64_t(32) << 20;

struct Request {
    Problem p;
    ttx_config cfg;          // batched-menu config, chosen at submission
    ttx_config direct;       // per-call config, for requests large enough to run alone
    BatchDesc desc;          // described at submission; an arena output is filled in at launch
    bool large = false;      // runs alone with the per-call kernels (large, complex or mixed)
    bool beta0;
    Scalar alpha, beta;
    const void* A;
    const void* Bin;
    void* Bout;
    bool arena_out;
    int64_t arena_off = -1;
    int64_t out_bytes;
    int64_t footprint;
    int64_t bytes;          // algorithmic
    int64_t t_arrival, t_done = 0;
    int state = WAITING;
    bool keep;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // work block of one micro-batch: count descriptors followed directly by
    // the count + 1 chunk prefix entries (one host-to-device copy), and the
    // claim counter at a fixed offset after room for max_batch descriptors
    unsigned char* d_blk = nullptr;
    unsigned char* h_blk = nullptr;  // pinned staging (host memory with the fake executor)
    uint32_t* d_counter = nullptr;
    std::vector<uint64_t> tickets;
    bool busy = false;
    bool finished = false;   // seen complete by the dispatcher's lock-free poll
    int64_t fake_done_at = 0;
};

}  // namespace ttx

using namespace ttx;

struct ttx_server {
    ttx_server_opts opts;
    int device = 0;
    char* arena_base = nullptr;
    Arena arena;
    int64_t budget = 0;
    int64_t in_use = 0;
    int64_t peak_in_use = 0;
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work;   // wakes the dispatcher
    std::atomic<uint64_t> work_seq{0};  // bumped on submission, release and stop
    std::condition_variable cv_done;   // wakes waiters
    std::deque<uint64_t> waiting;      // submitted, not admitted yet
    std::deque<uint64_t> ready;        // admitted, not launched yet
    std::unordered_map<uint64_t, Request> reqs;
    std::unordered_set<uint64_t> cancelled;   // tickets withdrawn before launch
    uint64_t next_ticket = 1;
    int64_t running = 0;
    bool stop = false;
    std::string worker_error;
    std::thread worker;

    // statistics
    int64_t submitted = 0, rejected = 0, completed = 0, batches = 0, batched_requests = 0;
    int64_t bytes_done = 0, first_arrival = 0, last_done = 0;
    std::vector<double> latencies_us;
};

static void release_locked(ttx_server* s, Request& r) {
    if (r.arena_out && r.arena_off >= 0) r.arena_off = (s->arena.release(r.arena_off, r.out_bytes), -1);
    s->in_use -= r.footprint;
}

// Completion: requests of finished slots become DONE.
// Whether a busy slot's work is complete (dispatcher thread only; no lock).
static bool slot_complete(const ttx_server* s, Slot& slot) {
    if (!slot.finished)
        slot.finished = s->opts.fake_device ? now_ns() >= slot.fake_done_at
                                            : hipEventQuery(slot.done) == hipSuccess;
    return slot.finished;
}

static void reap_locked(ttx_server* s) {
    for (auto& slot : s->slots) {
        if (!slot.busy || !slot_complete(s, slot)) continue;
        const int64_t t = now_ns();
        for (uint64_t tk : slot.tickets) {
            auto it = s->reqs.find(tk);
            if (it == s->reqs.end()) continue;
            Request& r = it->second;
            r.state = DONE;
            r.t_done = t;
            ++s->completed;
            s->bytes_done += r.bytes;
            s->last_done = std::max(s->last_done, t);
            s->latencies_us.push_back((t - r.t_arrival) * 1e-3);
            --s->running;
            if (!r.keep) {
                release_locked(s, r);
                s->reqs.erase(it);
            }
        }
        slot.tickets.clear();
        slot.busy = false;
        slot.finished = false;
        s->cv_done.notify_all();
    }
}

// Admission in arrival order: the head waits until its footprint fits.
static void admit_locked(ttx_server* s) {
    while (!s->waiting.empty()) {
        Request& r = s->reqs[s->waiting.front()];
        if (s->in_use + r.footprint > s->budget) break;
        if (r.arena_out) {
            const int64_t off = s->arena.alloc(r.out_bytes);
            if (off < 0) break;
            r.arena_off = off;
            r.Bout = s->opts.fake_device ? reinterpret_cast<void*>(uintptr_t(1) << 44 | uintptr_t(off))
                                         : static_cast<void*>(s->arena_base + off);
        }
        s->in_use += r.footprint;
        s->peak_in_use = std::max(s->peak_in_use, s->in_use);
        r.state = READY;
        s->ready.push_back(s->waiting.front());
        s->waiting.pop_front();
    }
}

// Forms and launches one micro-batch into a free slot.
static bool launch_locked(ttx_server* s) {
    if (s->ready.empty()) return false;
    Slot* slot = nullptr;
    for (auto& sl : s->slots)
        if (!sl.busy) {
            slot = &sl;
            break;
        }
    if (!slot) return false;
    int count = 0;
    int64_t bytes = 0;
    BatchDesc* h_desc = reinterpret_cast<BatchDesc*>(slot->h_blk);
    while (!s->ready.empty() && count < s->opts.max_batch) {
        Request& r = s->reqs[s->ready.front()];
        if (count > 0 && (r.large || bytes + r.bytes > s->opts.max_batch_bytes)) break;
        if (r.large) {   // alone, with the per-call kernels
            slot->tickets.push_back(s->ready.front());
            s->ready.pop_front();
            r.state = RUNNING;
            slot->busy = true;
            s->running += 1;
            ++s->batches;
            s->batched_requests += 1;
            if (s->opts.fake_device) {
                slot->fake_done_at = now_ns() + int64_t(double(r.bytes) / 4e12 * 1e9) + 2000;
                return true;
            }
            hipError_t e = launch_tiles(r.p, r.direct, r.beta0, r.A, r.beta0 ? nullptr : r.Bin, r.Bout, r.alpha,
                                        r.beta, slot->stream);
            if (e == hipSuccess) e = hipEventRecord(slot->done, slot->stream);
            if (e != hipSuccess) s->worker_error = std::string("server launch: ") + hipGetErrorString(e);
            return true;
        }
        BatchDesc& d = h_desc[count];
        d = r.desc;
        if (r.arena_out) batch_set_output(&d, r.Bout);
        bytes += r.bytes;
        r.state = RUNNING;
        slot->tickets.push_back(s->ready.front());
        s->ready.pop_front();
        ++count;
    }
    uint32_t* h_prefix = reinterpret_cast<uint32_t*>(slot->h_blk + sizeof(BatchDesc) * count);
    int grid = 0;
    const uint32_t chunks = s->opts.fake_device ? 0 : batch_layout(h_desc, count, h_prefix, &grid);
    slot->busy = true;
    s->running += count;
    ++s->batches;
    s->batched_requests += count;
    if (s->opts.fake_device) {
        // test executor: completes after the time the bytes would take at 4 TB/s
        slot->fake_done_at = now_ns() + int64_t(double(bytes) / 4e12 * 1e9) + 2000;
        return true;
    }
    const size_t nbytes = sizeof(BatchDesc) * count + sizeof(uint32_t) * (count + 1);
    hipError_t e = hipMemcpyAsync(slot->d_blk, slot->h_blk, nbytes, hipMemcpyHostToDevice, slot->stream);
    if (e == hipSuccess)
        e = launch_batch(reinterpret_cast<const BatchDesc*>(slot->d_blk),
                         reinterpret_cast<const uint32_t*>(slot->d_blk + sizeof(BatchDesc) * count), count, chunks,
                         grid, slot->d_counter, slot->stream);
    if (e == hipSuccess) e = hipEventRecord(slot->done, slot->stream);
    if (e != hipSuccess) s->worker_error = std::string("server launch: ") + hipGetErrorString(e);
    return true;
}

static void worker_main(ttx_server* s) {
    if (!s->opts.fake_device) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        reap_locked(s);
        admit_locked(s);
        while (launch_locked(s)) {
        }
        const bool busy = s->running > 0;
        if (s->stop && !busy) break;   // requests never launched are dropped
        if (busy) {
            // device work in flight: poll its completion without sleeping (a
            // sleep would add the scheduler's timer slack to every latency)
            // and without the lock, so that submissions are not held up;
            // return to the locked part when a slot finishes or work arrives
            const uint64_t seq = s->work_seq.load(std::memory_order_acquire);
            lock.unlock();
            while (true) {
                bool done = false;
                for (auto& slot : s->slots)
                    if (slot.busy && slot_complete(s, slot)) done = true;
                if (done || s->work_seq.load(std::memory_order_acquire) != seq) break;
                std::this_thread::yield();
            }
            lock.lock();
        } else {
            s->cv_work.wait_for(lock, std::chrono::milliseconds(2));
        }
    }
}

static void free_slots(ttx_server* s) {
    for (auto& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.d_blk) (void)hipFree(sl.d_blk);
        if (!s->opts.fake_device) {
            if (sl.h_blk) (void)hipHostFree(sl.h_blk);
        } else {
            delete[] sl.h_blk;
        }
    }
    s->slots.clear();
}

static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    const double pos = q * double(v.size() - 1);
    const size_t i = size_t(pos);
    const double f = pos - double(i);
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

static ttx_status submit_one(ttx_server* s, const ttx_request* rq, uint64_t* ticket) {
    const ttx_problem& q = rq->problem;
    Request r;
    ttx_status st = make_problem(q.dtype, q.n, q.perm, q.size, q.has_outer_a ? q.outer_a : nullptr,
                                 q.has_outer_b ? q.outer_b : nullptr, &r.p);
    if (st != TTX_OK) return st;
    if (!dtype_complex(r.p.dtype) && (q.alpha_im != 0.0 || q.beta_im != 0.0))
        return fail(TTX_EINVAL, "complex alpha or beta for a real element type");
    r.alpha = Scalar(q.alpha, q.alpha_im);
    r.beta = Scalar(q.beta, q.beta_im);
    r.beta0 = beta_is_zero(r.p.dtype, r.beta);
    r.A = q.A;
    r.arena_out = q.B == nullptr;
    r.Bout = q.B;
    r.Bin = q.B_in ? q.B_in : q.B;
    if (r.arena_out && !r.beta0 && !q.B_in) return fail(TTX_EINVAL, "beta != 0 needs B_in when B is server-allocated");
    if (!r.arena_out) {
        st = check_pointers(r.p, r.A, r.Bin, r.Bout, r.beta0);
        if (st != TTX_OK) return st;
    } else if (r.p.family != TTX_FAMILY_EMPTY && (!r.A || reinterpret_cast<uintptr_t>(r.A) % elem_bytes(r.p.dtype_a))) {
        return fail(TTX_EINVAL, "A must be a non-NULL, element-aligned device pointer");
    }
    r.out_bytes = r.p.family == TTX_FAMILY_EMPTY ? 0 : r.p.extent_b;
    r.bytes = r.p.elements * (elem_bytes(r.p.dtype_a) + elem_bytes(r.p.dtype) * (r.beta0 ? 1 : 2));
    // HBM the request occupies while admitted: its output region plus the
    // tensors it reads (inputs may be shared with other requests; counting
    // them keeps the bound conservative)
    r.footprint = r.p.extent_a + r.out_bytes + (r.beta0 ? 0 : r.p.extent_b);
    r.keep = rq->keep_result != 0;
    if (r.p.family != TTX_FAMILY_EMPTY) {
        // plan outside the lock; arena outputs are 256-byte aligned, like the
        // probe pointer used here for the vector decision
        const void* out_probe = r.arena_out ? reinterpret_cast<void*>(uintptr_t(1) << 44) : r.Bout;
        // a large request fills the device by itself: it runs alone with the
        // per-call kernels (whole tile menu, tuned configs); so do complex and
        // mixed-precision requests, which the persistent kernel does not take
        const bool per_call_type = dtype_complex(r.p.dtype) || r.p.dtype_a != r.p.dtype;
        if (!per_call_type) {
            st = batch_describe(r.p, nullptr, r.beta0, r.A, r.Bin, const_cast<void*>(out_probe), r.alpha.re,
                                r.beta.re, &r.desc, &r.cfg);
            if (st != TTX_OK) return st;
        }
        r.large = r.bytes >= kDirectBytes || per_call_type;
        if (r.large && !table_lookup(r.p, r.beta0, &r.direct)) r.direct = default_config(r.p);
    }
    r.t_arrival = rq->arrival_ns > 0 ? rq->arrival_ns : now_ns();
    std::lock_guard<std::mutex> lock(s->mu);
    if (!s->worker_error.empty()) return fail(TTX_EHIP, s->worker_error);
    if (r.footprint > s->budget || (r.arena_out && r.out_bytes > s->arena.size())) {
        ++s->rejected;
        return fail(TTX_EBUSY, "request footprint exceeds the admission budget");
    }
    if (int64_t(s->waiting.size() + s->ready.size()) >= s->opts.max_queue) {
        ++s->rejected;
        return fail(TTX_EBUSY, "request queue full");
    }
    const uint64_t tk = s->next_ticket++;
    if (s->submitted == 0) s->first_arrival = r.t_arrival;
    ++s->submitted;
    if (r.p.family == TTX_FAMILY_EMPTY) {
        r.state = DONE;
        r.t_done = r.t_arrival;
        r.footprint = 0;
        ++s->completed;
        if (r.keep) s->reqs[tk] = r;
    } else {
        s->reqs[tk] = r;
        s->waiting.push_back(tk);
        s->work_seq.fetch_add(1, std::memory_order_release);
        s->cv_work.notify_one();
    }
    *ticket = tk;
    return TTX_OK;
}

extern "C" {

ttx_status ttx_server_create(ttx_server** out, const ttx_server_opts* opts) {
    if (!out) return fail(TTX_EINVAL, "NULL server");
    ttx_server_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.hbm_fraction <= 0) o.hbm_fraction = 0.8;
    if (o.hbm_fraction > 1) return fail(TTX_EINVAL, "hbm_fraction must be in (0, 1]");
    if (o.slots <= 0) o.slots = 4;
    if (o.max_batch <= 0) o.max_batch = 256;
    if (o.max_batch_bytes <= 0) o.max_batch_bytes = int64_t(256) << 20;
    if (o.max_queue <= 0) o.max_queue = 1 << 16;
    ttx_server* s = new (std::nothrow) ttx_server;
    if (!s) return fail(TTX_ENOMEM, "out of host memory");
    s->opts = o;
    if (!o.fake_device) {
        size_t free_b = 0, total_b = 0;
        if (hipGetDevice(&s->device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return fail(TTX_EHIP, "cannot query device memory");
        }
        s->budget = int64_t(o.hbm_fraction * double(free_b));
    } else {
        s->budget = o.fake_free_bytes > 0 ? int64_t(o.hbm_fraction * double(o.fake_free_bytes)) : (int64_t(1) << 34);
    }
    const int64_t arena = o.arena_bytes > 0 ? std::min(o.arena_bytes, s->budget) : s->budget;
    s->arena.reset(arena);
    if (!o.fake_device && hipMalloc(reinterpret_cast<void**>(&s->arena_base), size_t(arena)) != hipSuccess) {
        delete s;
        return fail(TTX_ENOMEM, "arena allocation failed");
    }
    s->slots.resize(o.slots);
    const size_t staged = sizeof(BatchDesc) * o.max_batch + sizeof(uint32_t) * (o.max_batch + 1);
    const size_t counter_at = (staged + 255) & ~size_t(255);
    for (auto& sl : s->slots) {
        if (o.fake_device) {
            sl.h_blk = new unsigned char[staged];
            continue;
        }
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&sl.d_blk), counter_at + 2 * sizeof(uint32_t)) != hipSuccess ||
            hipMemset(sl.d_blk + counter_at, 0, 2 * sizeof(uint32_t)) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.h_blk), staged, 0) != hipSuccess) {
            free_slots(s);
            if (s->arena_base) (void)hipFree(s->arena_base);
            delete s;
            return fail(TTX_ENOMEM, "server slot allocation failed");
        }
        sl.d_counter = reinterpret_cast<uint32_t*>(sl.d_blk + counter_at);
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return TTX_OK;
}

ttx_status ttx_server_submit(ttx_server* s, const ttx_request* request, uint64_t* ticket) {
    if (!s || !request || !ticket) return fail(TTX_EINVAL, "NULL argument");
    return submit_one(s, request, ticket);
}

ttx_status ttx_server_poll(ttx_server* s, uint64_t ticket, int* done) {
    if (!s || !done) return fail(TTX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) {
        if (ticket == 0 || ticket >= s->next_ticket) return fail(TTX_ENOTFOUND, "unknown ticket");
        if (s->cancelled.count(ticket)) return fail(TTX_ENOTFOUND, "request was cancelled");
        *done = 1;   // completed and already released
        return TTX_OK;
    }
    *done = it->second.state == DONE;
    return TTX_OK;
}

ttx_status ttx_server_wait(ttx_server* s, uint64_t ticket) {
    if (!s) return fail(TTX_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lock(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return fail(TTX_ENOTFOUND, "unknown ticket");
    if (s->cancelled.count(ticket)) return fail(TTX_ENOTFOUND, "request was cancelled");
    while (true) {
        if (!s->worker_error.empty()) return fail(TTX_EHIP, s->worker_error);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end() || it->second.state == DONE) return TTX_OK;
        s->cv_done.wait_for(lock, std::chrono::milliseconds(1));
    }
}

ttx_status ttx_server_result(ttx_server* s, uint64_t ticket, void** B, double* latency_us) {
    if (!s) return fail(TTX_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(TTX_ENOTFOUND, "unknown or released ticket");
    if (it->second.state != DONE) return fail(TTX_EBUSY, "request not finished");
    if (B) *B = it->second.Bout;
    if (latency_us) *latency_us = (it->second.t_done - it->second.t_arrival) * 1e-3;
    return TTX_OK;
}

ttx_status ttx_server_release(ttx_server* s, uint64_t ticket) {
    if (!s) return fail(TTX_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(TTX_ENOTFOUND, "unknown or released ticket");
    if (it->second.state != DONE) return fail(TTX_EBUSY, "request not finished");
    release_locked(s, it->second);
    s->reqs.erase(it);
    s->work_seq.fetch_add(1, std::memory_order_release);
    s->cv_work.notify_one();
    return TTX_OK;
}

ttx_status ttx_server_cancel(ttx_server* s, uint64_t ticket) {
    if (!s) return fail(TTX_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(TTX_ENOTFOUND, "unknown, released or cancelled ticket");
    Request& r = it->second;
    if (r.state == RUNNING) return fail(TTX_EBUSY, "request already launched");
    if (r.state == DONE) return fail(TTX_EBUSY, "request finished: release it instead");
    auto& q = r.state == WAITING ? s->waiting : s->ready;
    q.erase(std::find(q.begin(), q.end(), ticket));
    if (r.state == READY) release_locked(s, r);   // admitted: its arena region and budget
    s->reqs.erase(it);
    s->cancelled.insert(ticket);
    s->work_seq.fetch_add(1, std::memory_order_release);   // freed budget may admit the next request
    s->cv_work.notify_one();
    s->cv_done.notify_all();
    return TTX_OK;
}

ttx_status ttx_server_drain(ttx_server* s) {
    if (!s) return fail(TTX_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lock(s->mu);
    int idle_checks = 0;
    while (!(s->waiting.empty() && s->ready.empty() && s->running == 0)) {
        if (!s->worker_error.empty()) return fail(TTX_EHIP, s->worker_error);
        if (s->running == 0 && s->ready.empty() && !s->waiting.empty()) {
            // nothing on the device and the head of the queue still waiting:
            // results the caller has not released hold the budget
            if (++idle_checks > 50)
                return fail(TTX_EBUSY, "admission blocked by results that were not released");
        } else {
            idle_checks = 0;
        }
        s->cv_done.wait_for(lock, std::chrono::milliseconds(1));
    }
    return s->worker_error.empty() ? TTX_OK : fail(TTX_EHIP, s->worker_error);
}

ttx_status ttx_server_replay_clients(ttx_server* s, int64_t count, const ttx_request* requests,
                                     const int64_t* offsets_ns, int clients, uint64_t* tickets) {
    if (!s || count < 0 || clients < 1 || clients > 64 || (count > 0 && (!requests || !offsets_ns || !tickets)))
        return fail(TTX_EINVAL, "bad replay arguments");
    const int64_t t0 = now_ns();
    std::vector<ttx_status> status(clients, TTX_OK);
    std::vector<std::string> errors(clients);
    auto client = [&](int c) {
        for (int64_t i = c; i < count; i += clients) {
            const int64_t due = t0 + offsets_ns[i];
            while (now_ns() < due) {
                const int64_t wait = due - now_ns();
                if (wait > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(wait - 100000));
            }
            ttx_request r = requests[i];
            r.arrival_ns = due;
            ttx_status st;
            // a full queue is back-pressure: retry; a request too large for the
            // budget can never be admitted and is reported as ticket 0
            while ((st = submit_one(s, &r, &tickets[i])) == TTX_EBUSY) {
                std::string why = ttx_last_error();
                if (why.find("queue full") == std::string::npos) {
                    tickets[i] = 0;
                    break;
                }
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
            if (st != TTX_OK && st != TTX_EBUSY) {
                status[c] = st;
                errors[c] = ttx_last_error();
                return;
            }
        }
    };
    if (clients == 1) {
        client(0);
    } else {
        std::vector<std::thread> pool;
        for (int c = 0; c < clients; ++c) pool.emplace_back(client, c);
        for (auto& t : pool) t.join();
    }
    for (int c = 0; c < clients; ++c)
        if (status[c] != TTX_OK) return fail(status[c], errors[c]);
    return TTX_OK;
}

ttx_status ttx_server_replay(ttx_server* s, int64_t count, const ttx_request* requests,
                             const int64_t* offsets_ns, uint64_t* tickets) {
    return ttx_server_replay_clients(s, count, requests, offsets_ns, 1, tickets);
}

ttx_status ttx_server_get_stats(ttx_server* s, ttx_server_stats* out) {
    if (!s || !out) return fail(TTX_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->rejected = s->rejected;
    out->completed = s->completed;
    out->queued = int64_t(s->waiting.size() + s->ready.size());
    out->running = s->running;
    out->batches = s->batches;
    out->mean_batch = s->batches ? double(s->batched_requests) / double(s->batches) : 0;
    out->algorithmic_bytes = s->bytes_done;
    out->budget_bytes = s->budget;
    out->in_use_bytes = s->in_use;
    out->peak_in_use_bytes = s->peak_in_use;
    out->span_s = s->last_done > s->first_arrival ? (s->last_done - s->first_arrival) * 1e-9 : 0;
    out->throughput_gbps = out->span_s > 0 ? double(s->bytes_done) / out->span_s / 1e9 : 0;
    out->p50_us = percentile(s->latencies_us, 0.50);
    out->p99_us = percentile(s->latencies_us, 0.99);
    out->max_us = s->latencies_us.empty() ? 0 : *std::max_element(s->latencies_us.begin(), s->latencies_us.end());
    return TTX_OK;
}

ttx_status ttx_replay_sequential(int64_t count, const ttx_request* requests, const int64_t* offsets_ns,
                                 void* scratch, int64_t scratch_bytes, hipStream_t stream,
                                 double* latencies_us) {
    if (count < 0 || (count > 0 && (!requests || !offsets_ns || !latencies_us)))
        return fail(TTX_EINVAL, "bad replay arguments");
    const int64_t t0 = now_ns();
    for (int64_t i = 0; i < count; ++i) {
        const int64_t due = t0 + offsets_ns[i];
        while (now_ns() < due) {
            const int64_t wait = due - now_ns();
            if (wait > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(wait - 100000));
        }
        const ttx_problem& q = requests[i].problem;
        Problem p;
        ttx_status st = make_problem(q.dtype, q.n, q.perm, q.size, q.has_outer_a ? q.outer_a : nullptr,
                                     q.has_outer_b ? q.outer_b : nullptr, &p);
        if (st != TTX_OK) return st;
        void* out = q.B ? q.B : scratch;   // (planning here is repeated by the cached path: cheap)
        if (!q.B && p.extent_b > scratch_bytes) return fail(TTX_EINVAL, "scratch too small");
        const bool beta0 = beta_is_zero(p.dtype, Scalar(q.beta, q.beta_im));
        const void* Bin = q.B_in ? q.B_in : out;
        st = transpose_cached(q.dtype, q.n, q.perm, q.size, q.has_outer_a ? q.outer_a : nullptr,
                              q.has_outer_b ? q.outer_b : nullptr, Scalar(q.alpha, q.alpha_im), q.A,
                              Scalar(q.beta, q.beta_im), beta0 ? nullptr : Bin, out, stream);
        if (st != TTX_OK) return st;
        if (hipStreamSynchronize(stream) != hipSuccess) return fail(TTX_EHIP, "sync failed");
        latencies_us[i] = (now_ns() - due) * 1e-3;
    }
    return TTX_OK;
}

ttx_status ttx_server_destroy(ttx_server* s) {
    if (!s) return TTX_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->work_seq.fetch_add(1, std::memory_order_release);
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    free_slots(s);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
    return TTX_OK;
}

}  // extern "C"
