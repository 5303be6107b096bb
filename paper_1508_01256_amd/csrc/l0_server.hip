// Decoding server (C-ABI l0_server_*): continuous batching of independent
// decoding requests on top of l0_decode_batched, under a fixed budget of
// device memory.
//
// Host side only.  Requests wait in a first-come-first-served queue (a batch
// gathers the waiting small requests past any large ones).  Every
// poll first collects finished requests: a batch writes its results into
// host memory the device can write, each outcome last (behind a system-scope
// fence), so a request completes when its own outcome appears there, not
// when its whole batch ends.  A batch's slot (and its part of the budget) is
// released once all its requests are done and its completion event has
// fired.  Then the poll fills free slots: a new batch takes waiting
// requests in order while their workspace bound fits a free range of the
// budget.  Each slot has a stream and an event of its own (default
// priority), so a new batch can start while an earlier one drains its last,
// largest instances.
//
// Batches that may run together are planned within an equal share of the
// device's resident workgroups (one share per slot), so that all of them fit
// on the device at once and no team waits for members that cannot be
// scheduled.  A batch of at most kExclusiveMax requests launched while the
// server is idle gets the whole device instead (lowest latency at low load).
// A large request (at least kSoloIndices column indices) is decoded alone by
// the single-instance decoder (l0_decode_ex), which streams at the device's
// full rate.  Work that must run alone (a large request, a whole-device
// batch) is ordered on the device, not by the host: its stream waits for
// the events of everything launched before it, and work launched while it
// is in flight waits for its event.  So the device never idles for a host
// round trip between them, and nothing ever runs beside them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <deque>
#include <mutex>
#include <vector>

#include "l0_batch.h"
#include "l0_internal.h"
#include "l0decode.h"

namespace {

constexpr int kMaxSlots = 4;
constexpr size_t kExclusiveMax = 2;
constexpr int64_t kSoloIndices = int64_t(1) << 21;

bool is_large(const l0_problem& p) { return p.n * p.d >= kSoloIndices; }

struct Request {
    l0_problem p;
    int64_t id;
    double submit_s;
    size_t bound;  // workspace bound of the request alone
};

// Outcome stored in a result record before its batch is launched: no
// decode produces it, so a different value means the record is written.
constexpr int32_t kPending = -1;

struct Slot {
    bool busy = false;
    std::vector<Request> reqs;
    std::vector<char> done;    // request completed
    size_t remaining = 0;
    size_t off = 0, size = 0;  // range of the budget
    double launch_s = 0.0;
    hipStream_t stream = nullptr;
    hipEvent_t done_event = nullptr;
    l0_result* host_res = nullptr;  // host memory the device writes, max_batch records
    l0_status status = L0_OK;
    bool exclusive = false;    // planned for the whole device
    bool solo = false;         // one request on the single-instance decoder
};


}  // namespace

struct l0_server_s {
    int device = 0;
    l0_server_opts opts{};
    char* arena = nullptr;
    std::deque<Request> waiting;
    std::vector<Slot> slots;
    std::deque<l0_completion> ready;
    int64_t outstanding = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

bool server_opts_ok(const l0_server_opts* o) {
    if (!o || o->budget_bytes < 256) return false;
    if (o->max_batch < 0 || o->max_inflight < 0 || o->max_inflight > kMaxSlots) return false;
    const l0_batch_opts& b = o->batch;
    if (b.timing) return false;
    if ((b.rule < L0_RULE_L0DEC || b.rule > L0_RULE_SHIFTED_MODE)) return false;
    if (b.tol_mode != L0_TOL_RELATIVE && b.tol_mode != L0_TOL_ABSOLUTE) return false;
    if (b.block_threads != 0 && b.block_threads != 256 && b.block_threads != 512) return false;
    return b.words_cap == 0 || (b.words_cap >= 64 && b.words_cap <= 32768);
}

// Largest free range of the budget not used by a busy slot: first fit of
// `need` bytes, returned as an offset, or SIZE_MAX.
size_t find_range(const l0_server_s* s, size_t need) {
    std::vector<std::pair<size_t, size_t>> used;
    for (const Slot& sl : s->slots)
        if (sl.busy) used.emplace_back(sl.off, sl.off + sl.size);
    std::sort(used.begin(), used.end());
    size_t at = 0;
    for (const auto& u : used) {
        if (u.first >= at + need) return at;
        at = std::max(at, u.second);
    }
    return at + need <= s->opts.budget_bytes ? at : SIZE_MAX;
}

void complete_one(l0_server_s* s, Slot& sl, size_t q, l0_status status, double t) {
    l0_completion c{};
    c.id = sl.reqs[q].id;
    c.status = status;
    if (status == L0_OK) c.result = sl.host_res[q];
    c.submit_s = sl.reqs[q].submit_s;
    c.launch_s = sl.launch_s;
    c.done_s = t;
    s->ready.push_back(c);
    sl.done[q] = 1;
    --sl.remaining;
}

void release_slot(Slot& sl) {
    sl.reqs.clear();
    sl.done.clear();
    sl.remaining = 0;
    sl.busy = false;
    sl.exclusive = false;
    sl.solo = false;
}

// Fail every request of the slot that has not completed.
void fail_rest(l0_server_s* s, Slot& sl, l0_status status) {
    const double t = s->now();
    for (size_t q = 0; q < sl.reqs.size(); ++q)
        if (!sl.done[q]) complete_one(s, sl, q, status, t);
}

// Collect finished requests and batches (blocking on each busy slot's
// event when `wait`).
void collect(l0_server_s* s, bool wait) {
    for (Slot& sl : s->slots) {
        if (!sl.busy) continue;
        const double t = s->now();
        // a batch writes each outcome last; the single-instance decoder does
        // not, so its request completes with its event
        for (size_t q = 0; q < sl.reqs.size() && sl.remaining && !sl.solo; ++q) {
            if (sl.done[q]) continue;
            const int32_t oc = __atomic_load_n(&sl.host_res[q].outcome, __ATOMIC_ACQUIRE);
            if (oc != kPending) complete_one(s, sl, q, L0_OK, t);
        }
        const hipError_t e = wait ? hipEventSynchronize(sl.done_event) : hipEventQuery(sl.done_event);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail_rest(s, sl, L0_ERR_HIP);
        } else if (sl.remaining) {
            // the batch has ended: every outcome is written; read them again
            const double t2 = s->now();
            for (size_t q = 0; q < sl.reqs.size(); ++q) {
                if (sl.done[q]) continue;
                const int32_t oc = __atomic_load_n(&sl.host_res[q].outcome, __ATOMIC_ACQUIRE);
                complete_one(s, sl, q, oc != kPending ? L0_OK : L0_ERR_HIP, t2);
            }
        }
        release_slot(sl);
    }
}

// Make this slot's stream wait for the events of the busy slots: all of them
// (`all`), or those whose work must run alone.
hipError_t wait_for_busy(l0_server_s* s, Slot& sl, bool all) {
    for (Slot& o : s->slots) {
        if (&o == &sl || !o.busy || !(all || o.exclusive)) continue;
        const hipError_t e = hipStreamWaitEvent(sl.stream, o.done_event, 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Decode the first waiting request alone with the single-instance decoder on
// this (free) slot, after everything launched before it.  Returns false,
// launching nothing, while its workspace does not fit beside the work in
// flight.
bool launch_solo(l0_server_s* s, Slot& sl) {
    const l0_problem& P0 = s->waiting.front().p;
    const size_t ws = l0_workspace_bytes(P0.n, P0.m, P0.d, P0.max_iter);
    const size_t at = ws ? find_range(s, ws) : SIZE_MAX;
    if (at == SIZE_MAX && ws != 0)
        for (const Slot& o : s->slots)
            if (o.busy) return false;
    const Request r = s->waiting.front();
    s->waiting.pop_front();
    const l0_problem& P = r.p;
    sl.reqs.assign(1, r);
    sl.done.assign(1, 0);
    sl.remaining = 1;
    sl.off = at == SIZE_MAX ? 0 : at;
    sl.size = at == SIZE_MAX ? 0 : ws;
    sl.busy = true;
    sl.exclusive = true;
    sl.solo = true;
    sl.launch_s = s->now();
    std::memset(&sl.host_res[0], 0, sizeof(l0_result));
    sl.host_res[0].outcome = kPending;
    l0_opts o{};
    o.rule = s->opts.batch.rule;
    o.tol_mode = s->opts.batch.tol_mode;
    o.weights = P.weights;
    l0_status st = at == SIZE_MAX ? L0_ERR_WORKSPACE : L0_OK;
    if (st == L0_OK && wait_for_busy(s, sl, true) != hipSuccess) st = L0_ERR_HIP;
    if (st == L0_OK)
        st = l0_decode_ex(P.col_idx, P.n, P.m, P.d, P.y, P.alpha, P.max_iter, P.tol, P.x_out, &o, sl.host_res,
                          s->arena + at, ws, sl.stream);
    if (st == L0_OK && hipEventRecord(sl.done_event, sl.stream) != hipSuccess) st = L0_ERR_HIP;
    if (st != L0_OK) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(sl.stream);
        fail_rest(s, sl, st);
        release_slot(sl);
    }
    return true;
}

// Launch batches into free slots while requests wait.
l0_status launch(l0_server_s* s) {
    const int32_t max_batch = s->opts.max_batch ? s->opts.max_batch : 1024;
    const int nslots = static_cast<int>(s->slots.size());
    for (Slot& sl : s->slots) {
        if (s->waiting.empty()) break;
        if (sl.busy) continue;
        int busy = 0;
        for (const Slot& o : s->slots) busy += o.busy;
        if (is_large(s->waiting.front().p)) {
            if (!launch_solo(s, sl)) break;  // after everything in flight
            continue;
        }
        // take the waiting small requests in arrival order (past waiting
        // large ones, which are queued one at a time as slots free) while
        // their bound fits a free range
        size_t bound = 0;
        std::vector<size_t> pick;
        for (size_t q = 0; q < s->waiting.size() && pick.size() < static_cast<size_t>(max_batch); ++q) {
            if (is_large(s->waiting[q].p)) continue;
            const size_t next = bound + s->waiting[q].bound;
            if (find_range(s, next) == SIZE_MAX) break;
            bound = next;
            pick.push_back(q);
        }
        const size_t take = pick.size();
        if (take == 0) break;  // wait for a running batch to free its range
        std::vector<l0_problem> probs(take);
        for (size_t q = 0; q < take; ++q) probs[q] = s->waiting[pick[q]].p;
        const size_t ws = l0_batch_workspace_bytes(probs.data(), static_cast<int32_t>(take), &s->opts.batch);
        const size_t at = ws ? find_range(s, ws) : SIZE_MAX;
        if (at == SIZE_MAX) return L0_ERR_WORKSPACE;  // the bounds are conservative; not expected
        sl.reqs.clear();
        for (size_t q : pick) sl.reqs.push_back(s->waiting[q]);
        for (size_t q = take; q-- > 0;) s->waiting.erase(s->waiting.begin() + static_cast<std::ptrdiff_t>(pick[q]));
        sl.done.assign(take, 0);
        sl.remaining = take;
        sl.off = at;
        sl.size = ws;
        sl.busy = true;
        sl.launch_s = s->now();
        for (size_t q = 0; q < take; ++q) {
            std::memset(&sl.host_res[q], 0, sizeof(l0_result));
            sl.host_res[q].outcome = kPending;
        }
        std::atomic_thread_fence(std::memory_order_seq_cst);
        // the whole device when idle and the batch is small, else one share;
        // after any work in flight that must run alone
        sl.exclusive = busy == 0 && take <= kExclusiveMax;
        l0_status st = wait_for_busy(s, sl, false) == hipSuccess ? L0_OK : L0_ERR_HIP;
        if (st == L0_OK)
            st = l0::decode_batched_share(probs.data(), static_cast<int32_t>(take), &s->opts.batch, sl.host_res,
                                          s->arena + at, ws, sl.stream, sl.exclusive ? 1 : nslots);
        if (st == L0_OK && hipEventRecord(sl.done_event, sl.stream) != hipSuccess) st = L0_ERR_HIP;
        if (st != L0_OK) {
            (void)hipGetLastError();
            // wait for whatever was enqueued on this slot's stream, then fail
            // the batch's requests
            (void)hipStreamSynchronize(sl.stream);
            fail_rest(s, sl, st);
            release_slot(sl);
        }
    }
    return L0_OK;
}

void release(l0_server_s* s) {
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done_event) (void)hipEventDestroy(sl.done_event);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.host_res) (void)hipHostFree(sl.host_res);
    }
    if (s->arena) (void)hipFree(s->arena);
}

}  // namespace

extern "C" {

l0_status l0_server_create(const l0_server_opts* opts, l0_server* out) {
    if (!out || !server_opts_ok(opts)) return L0_ERR_ARG;
    *out = nullptr;
    l0_server_s* s = new l0_server_s();
    s->opts = *opts;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return L0_ERR_HIP;
    }
    const int nslots = opts->max_inflight ? opts->max_inflight : 2;
    const size_t max_batch = opts->max_batch ? static_cast<size_t>(opts->max_batch) : 1024;
    s->slots.resize(nslots);
    l0_status st = L0_OK;
    if (hipMalloc(&s->arena, opts->budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        s->arena = nullptr;
        st = L0_ERR_OOM;
    }
    for (Slot& sl : s->slots) {
        if (st != L0_OK) break;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done_event, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.host_res), max_batch * sizeof(l0_result),
                          hipHostMallocCoherent) != hipSuccess)
            st = L0_ERR_HIP;
    }
    if (st != L0_OK) {
        (void)hipGetLastError();
        release(s);
        delete s;
        return st;
    }
    *out = s;
    return L0_OK;
}

l0_status l0_server_submit(l0_server s, const l0_problem* prob, int64_t id) {
    if (!s || !prob) return L0_ERR_ARG;
    // host checks of sizes and scalars (a one-instance batch that cannot be
    // planned is invalid), then the buffers
    size_t one = l0_batch_workspace_bytes(prob, 1, &s->opts.batch);
    if (one == 0) return L0_ERR_ARG;
    if (is_large(*prob)) one = std::max(one, l0_workspace_bytes(prob->n, prob->m, prob->d, prob->max_iter));
    if (!l0::device_buffer_ok(prob->col_idx, static_cast<size_t>(prob->n) * prob->d * sizeof(int32_t)) ||
        !l0::device_buffer_ok(prob->y, static_cast<size_t>(prob->m) * sizeof(double)) ||
        !l0::device_buffer_ok(prob->x_out, static_cast<size_t>(prob->n) * sizeof(double)) ||
        (prob->weights && !l0::device_buffer_ok(prob->weights, static_cast<size_t>(prob->n) * sizeof(double))))
        return L0_ERR_ARG;
    if (one > s->opts.budget_bytes) return L0_ERR_WORKSPACE;
    std::lock_guard<std::mutex> lock(s->mu);
    Request r{};
    r.p = *prob;
    r.id = id;
    r.submit_s = s->now();
    r.bound = one;
    s->waiting.push_back(r);
    ++s->outstanding;
    return L0_OK;
}

int32_t l0_server_poll(l0_server s, l0_completion* out, int32_t cap) {
    if (!s || cap < 0 || (cap > 0 && !out)) return -static_cast<int32_t>(L0_ERR_ARG);
    std::lock_guard<std::mutex> lock(s->mu);
    collect(s, false);
    const l0_status st = launch(s);
    if (st != L0_OK) return -static_cast<int32_t>(st);
    int32_t n = 0;
    while (n < cap && !s->ready.empty()) {
        out[n++] = s->ready.front();
        s->ready.pop_front();
        --s->outstanding;
    }
    return n;
}

l0_status l0_server_drain(l0_server s) {
    if (!s) return L0_ERR_ARG;
    std::lock_guard<std::mutex> lock(s->mu);
    for (;;) {
        collect(s, false);
        const l0_status st = launch(s);
        if (st != L0_OK) return st;
        bool busy = false;
        for (const Slot& sl : s->slots) busy |= sl.busy;
        if (!busy && s->waiting.empty()) return L0_OK;
        // block on the oldest running batch
        for (Slot& sl : s->slots)
            if (sl.busy) {
                (void)hipEventSynchronize(sl.done_event);
                break;
            }
    }
}

int64_t l0_server_outstanding(l0_server s) {
    if (!s) return 0;
    std::lock_guard<std::mutex> lock(s->mu);
    return s->outstanding;
}

l0_status l0_server_destroy(l0_server s) {
    if (!s) return L0_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        collect(s, true);
        release(s);
    }
    delete s;
    return L0_OK;
}

}  // extern "C"
