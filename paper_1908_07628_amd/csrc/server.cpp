// Serving of EELS-map requests on one GPU (eels_server_*, eels_admission_*).
//
// Requests arrive at any time.  A dispatcher thread admits them first-fit in arrival order
// while a slot (one HIP stream) is free and the plan's workspace fits the HBM budget; each
// admitted request runs eels_execute_ex on its own stream, so work of requests that arrive
// while others are on the GPU overlaps on the device.  Completion is detected with an event
// per request.  The map of each request is computed by the same kernels, in the same order,
// as a lone eels_execute: it is bitwise the same alone and in the mix.
//
// S-matrix residency: plans are made with resident_s, and a finished request's workspace stays
// allocated, keyed by the content of V and H (a device hash) and the plan's S signature.  A
// later request with the same key runs with EELS_EXEC_SKIP_SWEEPS on that workspace (only the
// set-up and the contractions for its probes).  Resident workspaces count against the budget
// and are freed least-recently-used when an admission needs the memory.
//
// The memory model of the footprint is that of the paper's memory discussion (Sec. 3:
// transmission stack, both S-matrices, the multislice arrays), extended by the plan to its
// whole workspace (windows, contraction buffers, tables).
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "eels.h"
#include "internal.h"

namespace eels {
// content hash of device memory (kernels_misc.hip): synchronous on `stream`
eels_status device_hash64(const void* d_ptr, size_t bytes, uint64_t* d_scratch, uint64_t* out, hipStream_t stream);
}

// ------------------------------------------------------------------------------ admission

struct eels_admission {
    struct Pending {
        uint64_t ticket;
        size_t footprint;
        double arrival;
        int skipped;
    };
    size_t budget;
    int max_slots, max_overtake;
    std::deque<Pending> queue;
    std::map<uint64_t, size_t> running;
    size_t used = 0;

    // First fit in arrival order while a slot is free and used + footprint <= capacity.  Once
    // the oldest queued request has been overtaken max_overtake times, nothing behind it is
    // admitted until it fits (no starvation of large requests).
    int admit(size_t capacity, uint64_t* out, int max_out) {
        int n = 0;
        bool head_blocked = false;
        for (size_t i = 0; i < queue.size() && n < max_out;) {
            if ((int)running.size() >= max_slots) break;
            Pending p = queue[i];
            const bool fits = used + p.footprint <= capacity;
            if (fits && !head_blocked) {
                queue.erase(queue.begin() + (long)i);
                running[p.ticket] = p.footprint;
                used += p.footprint;
                out[n++] = p.ticket;
                for (auto& q : queue)
                    if (q.arrival < p.arrival) ++q.skipped;
                continue;   // same index: the next request moved into it
            }
            if (!fits && i == 0 && p.skipped >= max_overtake) head_blocked = true;
            ++i;
        }
        return n;
    }
    bool cancel(uint64_t t) {
        for (auto it = queue.begin(); it != queue.end(); ++it)
            if (it->ticket == t) {
                queue.erase(it);
                return true;
            }
        return false;
    }
    void finish(uint64_t t) {
        auto it = running.find(t);
        if (it == running.end()) return;
        used -= it->second;
        running.erase(it);
    }
    void set_footprint(uint64_t t, size_t bytes) {
        auto it = running.find(t);
        if (it == running.end()) return;
        used = used - it->second + bytes;
        it->second = bytes;
    }
};

extern "C" {

eels_status eels_admission_create(eels_admission** out, size_t budget_bytes, int max_slots, int max_overtake) {
    if (!out || max_slots < 1 || max_overtake < 0) return EELS_ERR_INVALID_ARG;
    try {
        eels_admission* a = new eels_admission{};
        a->budget = budget_bytes;
        a->max_slots = max_slots;
        a->max_overtake = max_overtake;
        *out = a;
        return EELS_OK;
    } catch (...) {
        return EELS_ERR_INTERNAL;
    }
}

eels_status eels_admission_offer(eels_admission* a, uint64_t ticket, size_t footprint, double arrival) {
    if (!a) return EELS_ERR_INVALID_ARG;
    if (footprint > a->budget) {
        eels::set_error("request footprint exceeds the memory budget");
        return EELS_ERR_OOM;
    }
    a->queue.push_back({ticket, footprint, arrival, 0});
    return EELS_OK;
}

int eels_admission_admit(eels_admission* a, size_t capacity, uint64_t* tickets, int max_out) {
    if (!a || !tickets || max_out < 1) return 0;
    return a->admit(capacity, tickets, max_out);
}

eels_status eels_admission_finish(eels_admission* a, uint64_t ticket) {
    if (!a) return EELS_ERR_INVALID_ARG;
    a->finish(ticket);
    return EELS_OK;
}

eels_status eels_admission_cancel(eels_admission* a, uint64_t ticket) {
    if (!a) return EELS_ERR_INVALID_ARG;
    return a->cancel(ticket) ? EELS_OK : EELS_ERR_INVALID_ARG;
}

size_t eels_admission_used(const eels_admission* a) { return a ? a->used : 0; }

eels_status eels_admission_destroy(eels_admission* a) {
    delete a;
    return EELS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------ server

namespace {

enum { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
    uint64_t ticket = 0;
    eels_plan* plan = nullptr;
    const float* dV = nullptr;
    const void* dH = nullptr;
    double* dmap = nullptr;
    uint64_t content = 0, sig = 0;
    size_t ws_bytes = 0;
    int state = Q_QUEUED;
    eels_status status = EELS_OK;
    int hit = 0, slot = -1;
    void* ws = nullptr;
    hipEvent_t ev = nullptr;
    double arrival = 0, start = 0, finish = 0;
};

struct Resident {
    uint64_t content, sig;
    void* ws;
    size_t bytes;
    bool busy;
};

}  // namespace

struct eels_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 0;
    std::vector<hipStream_t> streams;
    std::vector<int> free_slots;
    eels_admission policy{};
    std::mutex mu, hash_mu;
    std::condition_variable wake, done_cv;
    std::map<uint64_t, Request> reqs;
    std::list<Resident> resident;        // front = least recently used
    size_t held = 0;                     // bytes of resident workspaces (busy or not)
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    hipStream_t hash_stream = nullptr;
    uint64_t* d_hash = nullptr;          // device word of the content hash
    std::chrono::steady_clock::time_point t0;
    eels_server_stats stats{};

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

    size_t held_busy() const {
        size_t b = 0;
        for (auto& r : resident) b += r.busy ? r.bytes : 0;
        return b;
    }
    // free idle resident workspaces, least recently used first, until used + held <= budget
    void evict_to_budget(hipStream_t st) {
        for (auto it = resident.begin(); it != resident.end() && policy.used + held > budget;) {
            if (it->busy) { ++it; continue; }
            hipFreeAsync(it->ws, st);
            held -= it->bytes;
            ++stats.evictions;
            it = resident.erase(it);
        }
    }
    void fail(Request& r, eels_status s) {
        r.state = Q_DONE;
        r.status = s;
        r.finish = now();
        ++stats.failed;
    }

    // start an admitted request on a free slot; on any failure the slot, the footprint and a
    // borrowed resident workspace are given back and the request ends with the error
    void start(Request& r) {
        const int slot = free_slots.back();
        free_slots.pop_back();
        hipStream_t st = streams[slot];
        r.slot = slot;
        r.start = now();
        Resident* hit = nullptr;
        for (auto it = resident.begin(); it != resident.end(); ++it)
            if (it->content == r.content && it->sig == r.sig && !it->busy && it->bytes >= r.ws_bytes) {
                resident.splice(resident.end(), resident, it);   // most recently used
                hit = &resident.back();
                break;
            }
        unsigned flags = 0;
        if (hit) {
            hit->busy = true;
            r.ws = hit->ws;
            r.hit = 1;
            policy.set_footprint(r.ticket, 0);       // no new memory
            flags = EELS_EXEC_SKIP_SWEEPS;
        } else {
            evict_to_budget(st);
            if (hipMallocAsync(&r.ws, r.ws_bytes, st) != hipSuccess) {
                r.ws = nullptr;
                (void)hipGetLastError();
                free_slots.push_back(slot);
                policy.finish(r.ticket);
                eels::set_error("workspace allocation failed");
                fail(r, EELS_ERR_OOM);
                return;
            }
        }
        eels_status s = eels_execute_ex(r.plan, r.dV, r.dH, r.dmap, r.ws, r.ws_bytes, st, flags);
        if (s == EELS_OK && hipEventRecord(r.ev, st) != hipSuccess) s = EELS_ERR_DEVICE;
        if (s != EELS_OK) {
            if (hit) hit->busy = false;
            else if (r.ws) hipFreeAsync(r.ws, st);
            r.ws = nullptr;
            free_slots.push_back(slot);
            policy.finish(r.ticket);
            fail(r, s);
            return;
        }
        r.state = Q_RUNNING;
        if (r.hit) ++stats.resident_hits;
    }

    void complete(Request& r, hipError_t e) {
        r.finish = now();
        r.state = Q_DONE;
        r.status = e == hipSuccess ? EELS_OK : EELS_ERR_DEVICE;
        policy.finish(r.ticket);
        free_slots.push_back(r.slot);
        if (r.hit) {
            for (auto& x : resident)
                if (x.ws == r.ws) x.busy = false;
        } else if (r.status == EELS_OK) {
            resident.push_back({r.content, r.sig, r.ws, r.ws_bytes, false});
            held += r.ws_bytes;
        } else {
            hipFreeAsync(r.ws, streams[r.slot]);
        }
        r.ws = nullptr;
        eels_plan_destroy(r.plan);
        r.plan = nullptr;
        if (r.status == EELS_OK) ++stats.completed;
        else ++stats.failed;
    }

    void loop() {
        hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        std::vector<uint64_t> adm((size_t)max_slots);
        for (;;) {
            bool running = false;
            for (auto& kv : reqs) {
                Request& r = kv.second;
                if (r.state != Q_RUNNING) continue;
                hipError_t e = hipEventQuery(r.ev);
                if (e == hipErrorNotReady) { running = true; continue; }
                complete(r, e);
                done_cv.notify_all();
            }
            if (stop && !running && policy.queue.empty()) break;
            // capacity for fresh workspaces: the budget less what busy residents hold (idle
            // ones can be freed on demand)
            const size_t busy = held_busy();
            const size_t cap = budget > busy ? budget - busy : 0;
            int n = stop ? 0 : policy.admit(cap, adm.data(), max_slots);
            for (int i = 0; i < n; ++i) {
                Request& r = reqs[adm[(size_t)i]];
                start(r);
                if (r.state == Q_DONE) done_cv.notify_all();
            }
            wake.wait_for(lk, std::chrono::microseconds(200));
        }
    }
};

extern "C" {

eels_status eels_server_create(eels_server** out, int device, size_t hbm_budget_bytes, int max_slots) {
    if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes == 0) return EELS_ERR_INVALID_ARG;
    eels_server* s = nullptr;
    try {
        s = new eels_server();
    } catch (...) {
        return EELS_ERR_INTERNAL;
    }
    s->device = device;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->policy.budget = hbm_budget_bytes;
    s->policy.max_slots = max_slots;
    s->policy.max_overtake = 4;
    s->t0 = std::chrono::steady_clock::now();
    if (hipSetDevice(device) != hipSuccess) {
        delete s;
        eels::set_error("hipSetDevice failed");
        return EELS_ERR_DEVICE;
    }
    for (int i = 0; i < max_slots; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) hipStreamDestroy(x);
            delete s;
            eels::set_error("hipStreamCreate failed");
            return EELS_ERR_DEVICE;
        }
        s->streams.push_back(st);
        s->free_slots.push_back(max_slots - 1 - i);
    }
    if (hipStreamCreateWithFlags(&s->hash_stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void**)&s->d_hash, 256) != hipSuccess) {
        for (auto x : s->streams) hipStreamDestroy(x);
        if (s->hash_stream) hipStreamDestroy(s->hash_stream);
        delete s;
        eels::set_error("server set-up failed");
        return EELS_ERR_DEVICE;
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return EELS_OK;
}

eels_status eels_server_submit(eels_server* s, const eels_problem* prob, const float* d_V, const void* d_H,
                               double* d_map, uint64_t* ticket) {
    if (!s || !prob || !d_V || !d_H || !d_map || !ticket) return EELS_ERR_INVALID_ARG;
    eels_problem q = *prob;
    q.resident_s = 1;               // every served workspace can be reused
    q.s1_mode = EELS_S1_STORED;
    q.max_workspace_bytes = 0;      // one slice group (residency)
    eels_plan* plan = nullptr;
    eels_status st = eels_plan_create(&plan, &q);
    if (st != EELS_OK) return st;
    Request r;
    r.plan = plan;
    r.dV = d_V;
    r.dH = d_H;
    r.dmap = d_map;
    eels_plan_workspace_bytes(plan, &r.ws_bytes);
    eels_plan_s_signature(plan, &r.sig);
    // content key: hash of V and H as they are now (the caller has finished writing them)
    const size_t vbytes = (size_t)prob->n_slices * prob->ny * prob->nx * sizeof(float);
    size_t hbytes = (size_t)prob->n_trans_total * 8;
    {
        eels_plan_info info;
        eels_plan_info_get(plan, &info);
        hbytes *= (size_t)info.window_nx * info.window_ny;
    }
    uint64_t hv = 0, hh = 0;
    hipSetDevice(s->device);
    std::unique_lock<std::mutex> hash_lk(s->hash_mu);   // one device word for the hash
    if ((st = eels::device_hash64(d_V, vbytes, s->d_hash, &hv, s->hash_stream)) != EELS_OK ||
        (st = eels::device_hash64(d_H, hbytes, s->d_hash, &hh, s->hash_stream)) != EELS_OK) {
        eels_plan_destroy(plan);
        return st;
    }
    hash_lk.unlock();
    r.content = hv * 0x9E3779B97F4A7C15ull ^ hh;
    if (hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess) {
        eels_plan_destroy(plan);
        eels::set_error("hipEventCreate failed");
        return EELS_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        eels_plan_destroy(plan);
        hipEventDestroy(r.ev);
        return EELS_ERR_INVALID_ARG;
    }
    r.ticket = s->next_ticket++;
    r.arrival = s->now();
    st = eels_admission_offer(&s->policy, r.ticket, r.ws_bytes, r.arrival);
    if (st != EELS_OK) {
        eels_plan_destroy(plan);
        hipEventDestroy(r.ev);
        return st;
    }
    ++s->stats.submitted;
    *ticket = r.ticket;
    s->reqs.emplace(r.ticket, r);
    s->wake.notify_all();
    return EELS_OK;
}

static void fill_timing(const Request& r, eels_request_timing* t) {
    if (!t) return;
    t->arrival_s = r.arrival;
    t->start_s = r.start;
    t->finish_s = r.finish;
    t->resident_hit = r.hit;
    t->status = r.status;
    t->workspace_bytes = r.ws_bytes;
}

eels_status eels_server_poll(eels_server* s, uint64_t ticket, int* done, eels_request_timing* t) {
    if (!s || !done) return EELS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return EELS_ERR_INVALID_ARG;
    *done = it->second.state == Q_DONE;
    fill_timing(it->second, t);
    return EELS_OK;
}

eels_status eels_server_wait(eels_server* s, uint64_t ticket, double timeout_s, int* done, eels_request_timing* t) {
    if (!s || !done) return EELS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return EELS_ERR_INVALID_ARG;
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(timeout_s, 0.0));
    s->done_cv.wait_until(lk, until, [&] { return it->second.state == Q_DONE; });
    *done = it->second.state == Q_DONE;
    fill_timing(it->second, t);
    return EELS_OK;
}

eels_status eels_server_cancel(eels_server* s, uint64_t ticket) {
    if (!s) return EELS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != Q_QUEUED || !s->policy.cancel(ticket)) {
        eels::set_error("only a queued request can be cancelled");
        return EELS_ERR_INVALID_ARG;
    }
    Request& r = it->second;
    r.state = Q_DONE;
    r.status = EELS_ERR_CANCELLED;
    r.finish = s->now();
    eels_plan_destroy(r.plan);
    r.plan = nullptr;
    ++s->stats.cancelled;
    s->done_cv.notify_all();
    return EELS_OK;
}

eels_status eels_server_release(eels_server* s, uint64_t ticket) {
    if (!s) return EELS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second.state != Q_DONE) return EELS_ERR_INVALID_ARG;
    if (it->second.ev) hipEventDestroy(it->second.ev);
    s->reqs.erase(it);
    return EELS_OK;
}

eels_status eels_server_get_stats(eels_server* s, eels_server_stats* out) {
    if (!s || !out) return EELS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->resident_bytes = s->held;
    out->resident_entries = (int64_t)s->resident.size();
    out->running_bytes = s->policy.used;
    return EELS_OK;
}

eels_status eels_server_destroy(eels_server* s) {
    if (!s) return EELS_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        // queued requests end as cancelled; running ones finish
        for (auto& kv : s->reqs) {
            Request& r = kv.second;
            if (r.state == Q_QUEUED && s->policy.cancel(r.ticket)) {
                r.state = Q_DONE;
                r.status = EELS_ERR_CANCELLED;
                eels_plan_destroy(r.plan);
                r.plan = nullptr;
                ++s->stats.cancelled;
            }
        }
        s->wake.notify_all();
    }
    s->th.join();
    hipSetDevice(s->device);
    for (auto& r : s->resident) hipFreeAsync(r.ws, s->streams[0]);
    for (auto& st : s->streams) hipStreamSynchronize(st);
    hipFree(s->d_hash);
    for (auto& kv : s->reqs)
        if (kv.second.ev) hipEventDestroy(kv.second.ev);
    for (auto st : s->streams) hipStreamDestroy(st);
    hipStreamDestroy(s->hash_stream);
    delete s;
    return EELS_OK;
}

}  // extern "C"
