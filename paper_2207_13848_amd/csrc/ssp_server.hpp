// Request serving with continuous batching (included by ssp_lib.hip, which
// defines the planner and the launch sequence it uses).
//
// A worker thread owns `nslots` slots, each a stream with its own workspace
// and pinned staging buffer.  Submitted requests wait in a FIFO queue; as soon
// as a slot is free the worker takes the oldest requests whose combined
// workspace fits the slot (and at most max_batch of them), plans them as one
// batch and launches it on the slot's stream.  Batches on different slots
// overlap on the device; requests that arrive while batches run join the
// next free slot.  The worker polls the slots' completion events and records,
// for every request, the time from its submission to the moment the worker
// saw its batch finish.  Every result equals the per-matrix call on the same
// inputs, whatever the batch it travelled in (the batch path is bit-exact).
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

namespace {

using ServerClock = std::chrono::steady_clock;

struct ServerReq {
    uint64_t ticket;
    CaseIn in;
    size_t need;  // workspace of the request planned alone, less the shared part
    ServerClock::time_point t_submit;
};

struct ServerSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* ws = nullptr;
    void* pin = nullptr;
    size_t pin_bytes = 0;
    bool busy = false;
    std::vector<ServerReq> reqs;
};

// Workspace every plan holds once whatever its cases (control block and the
// part scratch: server plans keep kPartWindowsBase windows whatever their
// size); a batch needs it once plus each request's own part.
size_t plan_shared_bytes()
{
    return align256(sizeof(Ctl)) + align256((size_t)kPartWindowsBase * kWinWords * sizeof(uint32_t));
}

} // namespace

struct ssp_server_s {
    ssp_context ctx;          // the worker's own context (device, CU count, errors)
    int device = 0;
    size_t slot_bytes = 0;
    int max_batch = 0;
    std::vector<ssp_csr> mats;
    std::vector<ServerSlot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<ServerReq> pending;
    // ticket -> 0 queued, 1 running, 2 done, < 0 failed (status)
    std::unordered_map<uint64_t, int> state;
    std::vector<double> latency_ms;
    uint64_t next_ticket = 1, submitted = 0, completed = 0, batches = 0, max_seen = 0;
    uint64_t max_busy = 0;
    ServerClock::time_point t0;
    bool stop = false;
    std::thread worker;
};

namespace {

ssp_status server_launch(ssp_server_s* S, ServerSlot& slot, std::vector<ServerReq>& reqs)
{
    std::vector<CaseIn> in;
    in.reserve(reqs.size());
    for (auto& r : reqs) in.push_back(r.in);
    Plan P = make_plan(&S->ctx, in, PLAN_PREDICT, kPartWindowsBase);
    if (P.total > S->slot_bytes) return SSP_ERR_BUDGET;
    const Bound b = bind_plan(P, slot.ws);
    const bool small = P.n <= kArgCases;
    if (!small) {
        const size_t bytes = (size_t)P.n * sizeof(CaseDesc);
        if (bytes > slot.pin_bytes) {
            if (slot.pin) (void)hipHostFree(slot.pin);
            slot.pin = nullptr;
            slot.pin_bytes = 0;
            if (hipHostMalloc(&slot.pin, bytes, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return SSP_ERR_OOM;
            }
            slot.pin_bytes = bytes;
        }
        std::memcpy(slot.pin, P.cs.data(), bytes);  // the slot is idle: its last copy is done
        if (hipMemcpyAsync(b.cs, slot.pin, bytes, hipMemcpyHostToDevice, slot.stream) != hipSuccess)
            return SSP_ERR_HIP;
    }
    const ssp_status st = launch_plan(&S->ctx, P, b, slot.stream, !small, false);
    if (st != SSP_OK) return st;
    if (hipEventRecord(slot.done, slot.stream) != hipSuccess) return SSP_ERR_HIP;
    return SSP_OK;
}

void server_loop(ssp_server_s* S)
{
    DeviceGuard g(S->device);
    std::unique_lock<std::mutex> lock(S->mu);
    for (;;) {
        bool progressed = false, any_busy = false;
        // completions
        for (auto& slot : S->slots) {
            if (!slot.busy) continue;
            const hipError_t q = hipEventQuery(slot.done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                continue;
            }
            const auto now = ServerClock::now();
            for (auto& r : slot.reqs) {
                S->state[r.ticket] = q == hipSuccess ? 2 : (int)SSP_ERR_HIP;
                S->latency_ms.push_back(
                    std::chrono::duration<double, std::milli>(now - r.t_submit).count());
                ++S->completed;
            }
            slot.reqs.clear();
            slot.busy = false;
            progressed = true;
        }
        // admissions: the oldest requests that fit a free slot
        for (auto& slot : S->slots) {
            if (slot.busy || S->pending.empty()) continue;
            std::vector<ServerReq> batch;
            size_t bytes = plan_shared_bytes();
            while (!S->pending.empty() && (int)batch.size() < S->max_batch &&
                   bytes + S->pending.front().need <= S->slot_bytes) {
                bytes += S->pending.front().need;
                batch.push_back(S->pending.front());
                S->pending.pop_front();
            }
            if (batch.empty()) continue;
            for (auto& r : batch) S->state[r.ticket] = 1;
            lock.unlock();
            ssp_status st = server_launch(S, slot, batch);
            lock.lock();
            if (st == SSP_ERR_BUDGET && batch.size() > 1) {
                // the joint plan came out larger than the sum estimate: put the
                // newest request back and launch the rest (never on one request,
                // which fits alone by admission)
                S->pending.push_front(batch.back());
                S->state[batch.back().ticket] = 0;
                batch.pop_back();
                lock.unlock();
                st = server_launch(S, slot, batch);
                lock.lock();
            }
            if (st != SSP_OK) {
                for (auto& r : batch) {
                    S->state[r.ticket] = (int)st;
                    ++S->completed;
                }
                continue;
            }
            S->max_seen = std::max<uint64_t>(S->max_seen, batch.size());
            ++S->batches;
            slot.reqs = std::move(batch);
            slot.busy = true;
            uint64_t nbusy = 0;
            for (auto& o : S->slots) nbusy += o.busy ? 1 : 0;
            S->max_busy = std::max(S->max_busy, nbusy);
            any_busy = true;
            progressed = true;
        }
        if (S->stop && S->pending.empty() && !any_busy) break;
        if (progressed) {
            S->cv.notify_all();
            continue;
        }
        // nothing to do now: poll the running batches at a short interval,
        // or sleep until a submission when the device is idle
        if (any_busy) S->cv.wait_for(lock, std::chrono::microseconds(20));
        else S->cv.wait(lock, [S] { return S->stop || !S->pending.empty(); });
    }
    S->cv.notify_all();
}

} // namespace

extern "C" {

ssp_status ssp_server_create(ssp_handle h, int nslots, size_t slot_bytes, int max_batch,
                             ssp_server* out)
{
    if (!h || !out || nslots < 1 || nslots > 64 || max_batch < 1) return SSP_ERR_INVALID_ARG;
    *out = nullptr;
    if (slot_bytes == 0) slot_bytes = (size_t)1 << 30;
    if (slot_bytes < plan_shared_bytes() + 4096) return SSP_ERR_INVALID_ARG;
    if (h->budget && (size_t)nslots * slot_bytes > h->budget) {
        h->last_error = "server slots exceed the handle's budget";
        return SSP_ERR_BUDGET;
    }
    DeviceGuard g(h->device);
    if (!g.ok()) return SSP_ERR_NO_DEVICE;
    prepare_kernels();
    ssp_server_s* S = new (std::nothrow) ssp_server_s();
    if (!S) return SSP_ERR_OOM;
    S->ctx.device = h->device;
    S->ctx.num_cus = h->num_cus;
    S->ctx.tuning = h->tuning;
    S->device = h->device;
    S->slot_bytes = slot_bytes;
    S->max_batch = max_batch;
    S->slots.resize((size_t)nslots);
    auto fail = [&](ssp_status st, hipError_t e, const char* what) {
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->last_error = std::string(what) + ": " + hipGetErrorString(e);
        }
        for (auto& sl : S->slots) {
            if (sl.ws) (void)hipFree(sl.ws);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete S;
        return st;
    };
    for (auto& sl : S->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(SSP_ERR_HIP, e, "hipStreamCreate");
        e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e != hipSuccess) return fail(SSP_ERR_HIP, e, "hipEventCreate");
        e = hipMalloc(&sl.ws, slot_bytes);
        if (e != hipSuccess) return fail(SSP_ERR_OOM, e, "hipMalloc");
    }
    S->t0 = ServerClock::now();
    S->worker = std::thread(server_loop, S);
    *out = S;
    return SSP_OK;
}

ssp_status ssp_server_register_matrix(ssp_server S, const ssp_csr* m, int32_t* id)
{
    if (!S || !id) return SSP_ERR_INVALID_ARG;
    const ssp_status st = check_csr(m);
    if (st != SSP_OK) return st;
    std::lock_guard<std::mutex> lock(S->mu);
    *id = (int32_t)S->mats.size();
    S->mats.push_back(*m);
    return SSP_OK;
}

ssp_status ssp_server_submit(ssp_server S, const ssp_request* r, uint64_t* ticket)
{
    if (!S || !r || !ticket) return SSP_ERR_INVALID_ARG;
    ServerReq q;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        if (r->a < 0 || r->b < 0 || r->a >= (int32_t)S->mats.size() ||
            r->b >= (int32_t)S->mats.size())
            return SSP_ERR_INVALID_ARG;
        const ssp_csr A = S->mats[(size_t)r->a], B = S->mats[(size_t)r->b];
        const ssp_sampler smp = (ssp_sampler)r->sampler;
        ssp_status st = common_checks(&S->ctx, &A, &B, smp, r->sample_rate, r->nnz_pred);
        if (st != SSP_OK) return st;
        q.in = case_in(&A, &B, smp, r->sample_rate, r->seed, r->nnz_pred, nullptr, r->stats);
    }
    const Plan alone = make_plan(&S->ctx, {q.in}, PLAN_PREDICT, kPartWindowsBase);
    if (alone.total > S->slot_bytes) return SSP_ERR_BUDGET;
    q.need = alone.total - plan_shared_bytes();
    {
        std::lock_guard<std::mutex> lock(S->mu);
        if (S->stop) return SSP_ERR_INVALID_ARG;
        q.ticket = S->next_ticket++;
        q.t_submit = ServerClock::now();
        S->state[q.ticket] = 0;
        S->pending.push_back(q);
        ++S->submitted;
        *ticket = q.ticket;
    }
    S->cv.notify_all();
    return SSP_OK;
}

ssp_status ssp_server_poll(ssp_server S, uint64_t ticket)
{
    if (!S) return SSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->state.find(ticket);
    if (it == S->state.end()) return SSP_ERR_INVALID_ARG;
    if (it->second == 2) return SSP_OK;
    if (it->second < 0) return (ssp_status)it->second;
    return SSP_ERR_NOT_READY;
}

ssp_status ssp_server_wait(ssp_server S, uint64_t ticket, double timeout_s)
{
    if (!S) return SSP_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lock(S->mu);
    const auto until = ServerClock::now() + std::chrono::duration_cast<ServerClock::duration>(
                                                std::chrono::duration<double>(timeout_s));
    for (;;) {
        auto it = S->state.find(ticket);
        if (it == S->state.end()) return SSP_ERR_INVALID_ARG;
        if (it->second == 2) return SSP_OK;
        if (it->second < 0) return (ssp_status)it->second;
        if (timeout_s >= 0 && ServerClock::now() >= until) return SSP_ERR_NOT_READY;
        S->cv.wait_for(lock, std::chrono::milliseconds(1));
    }
}

ssp_status ssp_server_info(ssp_server S, ssp_server_stats* out)
{
    if (!S || !out) return SSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(S->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->batches = S->batches;
    out->max_batch_seen = S->max_seen;
    out->max_slots_busy = S->max_busy;
    out->queued = S->pending.size();
    out->elapsed_s = std::chrono::duration<double>(ServerClock::now() - S->t0).count();
    std::vector<double> v = S->latency_ms;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            const size_t k = (size_t)std::min<double>((double)v.size() - 1,
                                                      std::ceil(p * (double)v.size()) - 1);
            return v[k];
        };
        double sum = 0;
        for (double x : v) sum += x;
        out->latency_p50_ms = pct(0.50);
        out->latency_p99_ms = pct(0.99);
        out->latency_mean_ms = sum / (double)v.size();
        out->latency_max_ms = v.back();
    }
    return SSP_OK;
}

ssp_status ssp_server_reset_stats(ssp_server S)
{
    if (!S) return SSP_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(S->mu);
    S->latency_ms.clear();
    S->submitted = S->completed = S->batches = S->max_seen = S->max_busy = 0;
    S->t0 = ServerClock::now();
    return SSP_OK;
}

ssp_status ssp_server_destroy(ssp_server S)
{
    if (!S) return SSP_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    DeviceGuard g(S->device);
    ssp_status st = SSP_OK;
    for (auto& sl : S->slots) {
        if (sl.stream && hipStreamSynchronize(sl.stream) != hipSuccess) st = SSP_ERR_HIP;
        if (sl.ws) (void)hipFree(sl.ws);
        if (sl.pin) (void)hipHostFree(sl.pin);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete S;
    return st;
}

} // extern "C"
