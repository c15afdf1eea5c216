// Serving loop: requests (one pscl_job each) decoded as they arrive.  Two
// modes:
//  - launches: a dispatcher thread keeps up to S mixed launches in flight,
//    one per stream, and whenever a stream is free launches every pending
//    request as one batch (continuous batching at launch granularity).
//    Built on the public group API; each stream owns a group with one call
//    in flight, so no two launches share a workspace.
//  - persistent: the dispatcher publishes requests into a ring in coherent
//    host memory (ring.h) that a persistent kernel consumes frame by frame
//    (continuous batching at frame granularity, no launch per batch); the
//    kernel leaves after a spell without work and is relaunched when
//    requests are held and no launch runs.  A replay driver submits a request trace at given arrival times
// through a server, or as plain per-request pscl_decode launches (the
// baseline), and reports per-request latencies.

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pscl.h"
#include "ring.h"

namespace {

double now_us() {
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() *
           1e-3;
}

struct Req {
    pscl_job job;
    uint64_t ticket;
    double t_arrive;     // latency reference
    double* sink;        // if set, the latency goes here and the ticket is not kept
    hipEvent_t ready;    // recorded on the submitter's stream (NULL: inputs resident)
    int64_t footprint;   // device bytes charged to the admission budget
};

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    const size_t k = std::min(v.size() - 1, (size_t)(q * (double)(v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + (ptrdiff_t)k, v.end());
    return v[k];
}

}  // namespace

struct pscl_server {
    int device = 0;
    int S = 2;
    int max_requests = 4096, max_batch_requests = 1024;
    int64_t max_pending_frames = 0, max_batch_frames = 0;
    std::vector<const pscl_plan*> plans;
    std::vector<pscl_group*> groups;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> ev;
    std::vector<std::vector<Req>> inflight;
    std::vector<int64_t> frame_bytes;  // pscl_plan_footprint of each plan
    int64_t max_footprint = 0;         // 0 = no limit

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req> pending;
    int64_t pending_frames = 0;
    int64_t held = 0;            // pending + in flight
    int64_t held_footprint = 0;  // their device bytes
    std::vector<hipEvent_t> free_events;  // readiness events to reuse
    std::unordered_map<uint64_t, double> done;
    uint64_t next_ticket = 1;
    bool stop = false;
    pscl_status error = PSCL_OK;  // first launch failure, reported by later calls

    std::vector<double> lat;
    int64_t n_req = 0, n_frames = 0, n_launch = 0;
    std::thread th;

    // persistent mode
    bool ring = false;
    pscl_group* rgroup = nullptr;
    hipStream_t rstream = nullptr;
    hipEvent_t rev = nullptr;  // end of the current launch
    bool rlaunched = false;
    pscl_ring::Ctl* ctl = nullptr;
    pscl_ring::Rec* rec = nullptr;
    uint64_t* rdone = nullptr;
    uint32_t* rcount = nullptr;
    pscl_ring::Dev* rdev = nullptr;
    unsigned long long* rorphans = nullptr;
    uint32_t* rcu = nullptr;
    pscl_ring::Args rargs{};
    int64_t rec_size = 0;
    std::vector<int64_t> row_in, row_out;  // LLR row bytes and K per plan
    int64_t ring_frames = 0;  // published and not finished
    uint64_t published = 0;
    uint32_t idle_us = 2000;
    int cus = 1;
    int active_cfg = 0;      // fixed workgroups per CU taking frames (0: adaptive)
    uint32_t active_set = 0;  // value last written to the ring
    std::vector<int> free_slots;
    std::vector<Req> slot_req;
    std::vector<int> busy_slots;

    void run();
    void run_ring();
    pscl_status submit(const pscl_job& job, hipStream_t ready_on, bool order, double t_arrive,
                       double* sink, uint64_t* ticket);
};

void pscl_server::run() {
    (void)hipSetDevice(device);
    if (ring) {
        run_ring();
        return;
    }
    std::vector<pscl_job> jobs;
    for (;;) {
        bool progress = false;
        // completions
        for (int s = 0; s < S; ++s) {
            if (inflight[s].empty()) continue;
            const hipError_t q = hipEventQuery(ev[s]);
            if (q == hipErrorNotReady) continue;
            const double t = now_us();
            std::lock_guard<std::mutex> lk(mu);
            if (q != hipSuccess && error == PSCL_OK) error = PSCL_E_HIP;
            for (const Req& r : inflight[s]) {
                const double l = t - r.t_arrive;
                if (r.sink) *r.sink = l;
                else done[r.ticket] = l;
                lat.push_back(l);
                n_req += 1;
                n_frames += r.job.F;
                held -= 1;
                held_footprint -= r.footprint;
                if (r.ready) free_events.push_back(r.ready);
            }
            inflight[s].clear();
            progress = true;
            cv_done.notify_all();
        }
        // launches: every free stream takes what is pending
        for (int s = 0; s < S; ++s) {
            if (!inflight[s].empty()) continue;
            std::vector<Req>& batch = inflight[s];
            {
                std::lock_guard<std::mutex> lk(mu);
                int64_t fr = 0;
                while (!pending.empty() && (int)batch.size() < max_batch_requests) {
                    const Req& r = pending.front();
                    if (!batch.empty() && max_batch_frames > 0 && fr + r.job.F > max_batch_frames)
                        break;
                    fr += r.job.F;
                    pending_frames -= r.job.F;
                    batch.push_back(r);
                    pending.pop_front();
                }
            }
            if (batch.empty()) continue;
            jobs.clear();
            pscl_status st = PSCL_OK;
            for (const Req& r : batch) {
                jobs.push_back(r.job);
                // the launch runs after the work that produced the inputs
                if (r.ready && hipStreamWaitEvent(streams[s], r.ready, 0) != hipSuccess)
                    st = PSCL_E_HIP;
            }
            if (st == PSCL_OK)
                st = pscl_group_decode(groups[s], jobs.data(), (int)jobs.size(), streams[s]);
            if (st == PSCL_OK && hipEventRecord(ev[s], streams[s]) != hipSuccess) st = PSCL_E_HIP;
            if (st != PSCL_OK) {
                // the requests complete as failed; later calls report it
                std::lock_guard<std::mutex> lk(mu);
                if (error == PSCL_OK) error = st;
                (void)hipStreamSynchronize(streams[s]);
                (void)hipEventRecord(ev[s], streams[s]);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                n_launch += 1;
            }
            progress = true;
        }
        if (progress) continue;
        std::unique_lock<std::mutex> lk(mu);
        bool busy = false;
        for (int s = 0; s < S; ++s) busy = busy || !inflight[s].empty();
        if (!busy && pending.empty()) {
            if (stop) return;
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        } else {
            lk.unlock();
            std::this_thread::yield();
        }
    }
}

// Persistent mode: completions are read from the ring's completion words;
// pending requests whose inputs are ready are published in order while ring
// slots and frame-map entries are free; a launch is started whenever
// requests are held and none runs.
void pscl_server::run_ring() {
    for (;;) {
        bool progress = false;
        // completions
        for (size_t i = 0; i < busy_slots.size();) {
            const int sl = busy_slots[i];
            const Req& r = slot_req[sl];
            if (__atomic_load_n(&rdone[sl], __ATOMIC_ACQUIRE) != r.ticket) {
                ++i;
                continue;
            }
            const double t = now_us();
            std::lock_guard<std::mutex> lk(mu);
            const double l = t - r.t_arrive;
            if (r.sink) *r.sink = l;
            else done[r.ticket] = l;
            lat.push_back(l);
            n_req += 1;
            n_frames += r.job.F;
            held -= 1;
            held_footprint -= r.footprint;
            ring_frames -= r.job.F;
            if (r.ready) free_events.push_back(r.ready);
            free_slots.push_back(sl);
            busy_slots[i] = busy_slots.back();
            busy_slots.pop_back();
            progress = true;
            cv_done.notify_all();
        }
        // publication
        {
            std::lock_guard<std::mutex> lk(mu);
            while (!pending.empty() && !free_slots.empty()) {
                const Req& r = pending.front();
                if (ring_frames + r.job.F > rec_size) break;
                if (r.ready) {
                    const hipError_t q = hipEventQuery(r.ready);
                    if (q == hipErrorNotReady) break;
                    if (q != hipSuccess && error == PSCL_OK) error = PSCL_E_HIP;
                }
                const int sl = free_slots.back();
                free_slots.pop_back();
                slot_req[sl] = r;
                const pscl_job& J = r.job;
                const int64_t in = row_in[J.plan], out = row_out[J.plan];
                for (int64_t f = 0; f < J.F; ++f) {
                    pscl_ring::Rec& d = rec[(published + (uint64_t)f) & (uint64_t)(rec_size - 1)];
                    d.llr = (const uint8_t*)J.llr + f * in;
                    d.u_hat = J.u_hat + f * out;
                    d.crc_ok = J.crc_ok ? J.crc_ok + f : nullptr;
                    d.pm = J.pm ? (void*)((uint8_t*)J.pm + f * 4) : nullptr;
                    d.ticket = r.ticket;
                    d.slot = (uint32_t)sl;
                    d.plan = J.plan;
                    d.F = J.F;
                    d.pad = 0;
                }
                published += (uint64_t)J.F;
                // the records before the count that publishes them
                __atomic_store_n(&ctl->published, published, __ATOMIC_RELEASE);
                ring_frames += r.job.F;
                pending_frames -= r.job.F;
                busy_slots.push_back(sl);
                pending.pop_front();
                progress = true;
            }
        }
        // workgroups per CU taking frames: a fixed count, or 0 (the kernel
        // admits workgroups by the frames outstanding on the device)
        {
            const uint32_t want = active_cfg > 0 ? (uint32_t)active_cfg : 0u;
            if (want != active_set) {
                __atomic_store_n(&ctl->active, want, __ATOMIC_RELEASE);
                active_set = want;
            }
        }
        // a launch while requests are held
        if (!busy_slots.empty()) {
            bool running = rlaunched && hipEventQuery(rev) == hipErrorNotReady;
            if (!running) {
                rargs.parity = (uint32_t)(n_launch & 1);
                pscl_status st = pscl_ring::launch(rgroup, rargs, rstream);
                if (st == PSCL_OK && hipEventRecord(rev, rstream) != hipSuccess) st = PSCL_E_HIP;
                std::lock_guard<std::mutex> lk(mu);
                if (st != PSCL_OK) {
                    if (error == PSCL_OK) error = st;
                } else {
                    rlaunched = true;
                    n_launch += 1;
                }
                progress = true;
            }
        }
        std::unique_lock<std::mutex> lk(mu);
        if (error != PSCL_OK) {
            // nothing more can complete: release the waiters
            cv_done.notify_all();
            if (stop) return;
        }
        if (busy_slots.empty() && pending.empty()) {
            if (stop) return;
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        } else if (!progress) {
            lk.unlock();
            std::this_thread::yield();
        }
    }
}

pscl_status pscl_server::submit(const pscl_job& job, hipStream_t ready_on, bool order,
                                 double t_arrive, double* sink, uint64_t* ticket) {
    if (job.plan < 0 || job.plan >= (int)plans.size() || job.F < 0) return PSCL_E_INVALID;
    if (job.F > 0 && (!job.llr || !job.u_hat || ((uintptr_t)job.llr & 15u) != 0))
        return PSCL_E_INVALID;
    if (max_pending_frames > 0 && job.F > max_pending_frames) return PSCL_E_INVALID;  // never fits
    const int64_t fp = job.F * frame_bytes[job.plan];
    if (max_footprint > 0 && fp > max_footprint) return PSCL_E_INVALID;  // never fits
    if (ring && job.F > rec_size) return PSCL_E_INVALID;  // never fits the frame records
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (error != PSCL_OK) return error;
        if (held >= max_requests) return PSCL_E_BUSY;
        if (max_pending_frames > 0 && pending_frames + job.F > max_pending_frames)
            return PSCL_E_BUSY;
        if (max_footprint > 0 && held_footprint + fp > max_footprint) return PSCL_E_BUSY;
        if (order && job.F > 0 && !free_events.empty()) {
            ev = free_events.back();
            free_events.pop_back();
        }
    }
    if (order && job.F > 0) {
        // readiness of the inputs: an event on the submitter's stream
        if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return PSCL_E_HIP;
        if (hipEventRecord(ev, ready_on) != hipSuccess) {
            std::lock_guard<std::mutex> lk(mu);
            free_events.push_back(ev);
            return PSCL_E_HIP;
        }
    }
    std::lock_guard<std::mutex> lk(mu);
    // admission is re-checked: another thread may have submitted meanwhile
    if (held >= max_requests ||
        (max_pending_frames > 0 && pending_frames + job.F > max_pending_frames) ||
        (max_footprint > 0 && held_footprint + fp > max_footprint)) {
        if (ev) free_events.push_back(ev);
        return PSCL_E_BUSY;
    }
    const uint64_t t = next_ticket++;
    if (ticket) *ticket = t;
    if (job.F == 0) {  // nothing to decode: done at once
        if (sink) *sink = 0.0;
        else done[t] = 0.0;
        cv_done.notify_all();
        return PSCL_OK;
    }
    pending.push_back(Req{job, t, t_arrive, sink, ev, fp});
    pending_frames += job.F;
    held += 1;
    held_footprint += fp;
    cv_work.notify_one();
    return PSCL_OK;
}

// Persistent mode: one group for the workspace and plan tables, a stream
// and an end event for the launches, the ring in coherent host memory
// (frame records, completion words per slot, the control block) and the
// device counters.
static pscl_status ring_setup(pscl_server* sv, const pscl_server_cfg* cfg) {
    pscl_status st = pscl_group_create(cfg->plans, cfg->n_plans, 1, 1, nullptr, &sv->rgroup);
    if (st != PSCL_OK) return st;
    const int R = sv->max_requests;
    sv->rec_size = int64_t(1) << 18;
    for (int i = 0; i < cfg->n_plans; ++i) {
        int N = 0, K = 0, dt = 0;
        st = pscl_plan_code(cfg->plans[i], &N, &K, nullptr, nullptr, &dt);
        if (st != PSCL_OK) return st;
        sv->row_in.push_back((int64_t)N * (dt == PSCL_F32 ? 4 : (dt == PSCL_I16 ? 2 : 1)));
        sv->row_out.push_back(K);
    }
    auto hmalloc = [&](void** p, size_t bytes) {
        if (st != PSCL_OK) return;
        if (hipHostMalloc(p, bytes, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            *p = nullptr;
            st = PSCL_E_NOMEM;
            return;
        }
        memset(*p, 0, bytes);
    };
    hmalloc((void**)&sv->ctl, sizeof(pscl_ring::Ctl));
    hmalloc((void**)&sv->rec, sizeof(pscl_ring::Rec) * (size_t)sv->rec_size);
    hmalloc((void**)&sv->rdone, sizeof(uint64_t) * (size_t)R);
    if (st != PSCL_OK) return st;
    if (hipMalloc((void**)&sv->rcount, sizeof(uint32_t) * (size_t)R) != hipSuccess ||
        hipMalloc((void**)&sv->rdev, sizeof(pscl_ring::Dev)) != hipSuccess)
        return PSCL_E_NOMEM;
    // orphan lists: at most one ticket per workgroup per launch
    const uint32_t cap = 1u << 16;
    if (hipMalloc((void**)&sv->rorphans, sizeof(unsigned long long) * 2 * cap) != hipSuccess ||
        hipMalloc((void**)&sv->rcu, sizeof(uint32_t) * pscl_ring::kCuSlots) != hipSuccess)
        return PSCL_E_NOMEM;
    if (hipMemset(sv->rcount, 0, sizeof(uint32_t) * (size_t)R) != hipSuccess ||
        hipMemset(sv->rdev, 0, sizeof(pscl_ring::Dev)) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->rstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sv->rev, hipEventDisableTiming) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
        return PSCL_E_HIP;
    pscl_ring::Args& a = sv->rargs;
    void* dp = nullptr;
    auto dev_ptr = [&](void* h) {
        if (st == PSCL_OK && hipHostGetDevicePointer(&dp, h, 0) != hipSuccess) st = PSCL_E_HIP;
        return dp;
    };
    a.ctl = (pscl_ring::Ctl*)dev_ptr(sv->ctl);
    a.rec = (const pscl_ring::Rec*)dev_ptr(sv->rec);
    a.done = (uint64_t*)dev_ptr(sv->rdone);
    a.count = sv->rcount;
    a.dev = sv->rdev;
    a.orphans = sv->rorphans;
    a.cu_rank = sv->rcu;
    a.orphan_cap = cap;
    a.parity = 0;
    a.rec_mask = (uint32_t)(sv->rec_size - 1);
    a.idle_us = sv->idle_us;
    a.wg_per_cu = (uint32_t)cfg->wg_per_cu;
    a.cus = 1;  // set by each launch
    sv->active_cfg = cfg->active_per_cu;
    if (hipDeviceGetAttribute(&sv->cus, hipDeviceAttributeMultiprocessorCount, sv->device) != hipSuccess ||
        sv->cus < 1)
        return PSCL_E_HIP;
    sv->slot_req.resize((size_t)R);
    for (int i = R - 1; i >= 0; --i) sv->free_slots.push_back(i);
    return st;
}

extern "C" {

void pscl_server_destroy(pscl_server* sv) {
    if (!sv) return;
    if (sv->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        sv->th.join();
    }
    if (sv->ctl) __atomic_store_n(&sv->ctl->stop, 1u, __ATOMIC_RELEASE);
    if (sv->rlaunched) (void)hipEventSynchronize(sv->rev);
    if (sv->rstream) (void)hipStreamSynchronize(sv->rstream);
    pscl_group_destroy(sv->rgroup);
    if (sv->rev) (void)hipEventDestroy(sv->rev);
    if (sv->rstream) (void)hipStreamDestroy(sv->rstream);
    for (void* h : {(void*)sv->ctl, (void*)sv->rec, (void*)sv->rdone})
        if (h) (void)hipHostFree(h);
    (void)hipFree(sv->rcount);
    (void)hipFree(sv->rdev);
    (void)hipFree(sv->rorphans);
    (void)hipFree(sv->rcu);
    for (pscl_group* g : sv->groups) pscl_group_destroy(g);
    for (hipEvent_t e : sv->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : sv->free_events) (void)hipEventDestroy(e);
    for (hipStream_t s : sv->streams)
        if (s) (void)hipStreamDestroy(s);
    delete sv;
}

pscl_status pscl_server_create(const pscl_server_cfg* cfg, pscl_server** out) {
    if (!cfg || !out || !cfg->plans || cfg->n_plans < 1) return PSCL_E_INVALID;
    if (cfg->streams < 0 || cfg->streams > 8 || cfg->max_requests < 0 ||
        cfg->max_pending_frames < 0 || cfg->max_batch_frames < 0 || cfg->max_batch_requests < 0 ||
        cfg->max_footprint_bytes < 0 || cfg->persistent < 0 || cfg->persistent > 1 ||
        cfg->idle_us < 0 || cfg->wg_per_cu < 0 || cfg->active_per_cu < 0)
        return PSCL_E_INVALID;
    for (int i = 0; i < cfg->n_plans; ++i)
        if (!cfg->plans[i]) return PSCL_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    pscl_server* sv = new pscl_server();
    sv->device = dev;
    sv->S = cfg->streams ? cfg->streams : 2;
    if (cfg->max_requests) sv->max_requests = cfg->max_requests;
    if (cfg->max_batch_requests) sv->max_batch_requests = cfg->max_batch_requests;
    sv->max_pending_frames = cfg->max_pending_frames;
    sv->max_batch_frames = cfg->max_batch_frames;
    sv->plans.assign(cfg->plans, cfg->plans + cfg->n_plans);
    sv->inflight.resize(sv->S);
    sv->max_footprint = cfg->max_footprint_bytes;
    pscl_status st = PSCL_OK;
    for (int i = 0; i < cfg->n_plans && st == PSCL_OK; ++i) {
        int64_t b = 0;
        st = pscl_plan_footprint(cfg->plans[i], &b);
        sv->frame_bytes.push_back(b);
    }
    sv->ring = cfg->persistent == 1;
    if (sv->ring) {
        if (cfg->idle_us) sv->idle_us = (uint32_t)cfg->idle_us;
        st = ring_setup(sv, cfg);
        if (st != PSCL_OK) {
            pscl_server_destroy(sv);
            return st;
        }
        sv->th = std::thread([sv] { sv->run(); });
        *out = sv;
        return PSCL_OK;
    }
    for (int s = 0; s < sv->S && st == PSCL_OK; ++s) {
        pscl_group* g = nullptr;
        st = pscl_group_create(cfg->plans, cfg->n_plans, sv->max_batch_requests, 1, nullptr, &g);
        if (st != PSCL_OK) break;
        sv->groups.push_back(g);
        hipStream_t str = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&str, hipStreamNonBlocking) != hipSuccess) st = PSCL_E_HIP;
        sv->streams.push_back(str);
        if (st == PSCL_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            st = PSCL_E_HIP;
        sv->ev.push_back(e);
    }
    if (st != PSCL_OK) {
        pscl_server_destroy(sv);
        return st;
    }
    sv->th = std::thread([sv] { sv->run(); });
    *out = sv;
    return PSCL_OK;
}

pscl_status pscl_server_submit(pscl_server* sv, const pscl_job* job, void* stream,
                               uint64_t* ticket) {
    if (!sv || !job) return PSCL_E_INVALID;
    return sv->submit(*job, (hipStream_t)stream, true, now_us(), nullptr, ticket);
}

pscl_status pscl_server_poll(pscl_server* sv, uint64_t ticket, int* is_done, double* latency_us) {
    if (!sv || !is_done) return PSCL_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        if (ticket == 0 || ticket >= sv->next_ticket) return PSCL_E_INVALID;
        *is_done = 0;
        return sv->error;
    }
    *is_done = 1;
    if (latency_us) *latency_us = it->second;
    sv->done.erase(it);
    return sv->error;
}

pscl_status pscl_server_wait(pscl_server* sv, uint64_t ticket, double timeout_ms,
                             double* latency_us) {
    if (!sv) return PSCL_E_INVALID;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (ticket == 0 || ticket >= sv->next_ticket) return PSCL_E_INVALID;
    auto ready = [&] { return sv->done.count(ticket) > 0 || sv->error != PSCL_OK; };
    if (timeout_ms < 0) {
        sv->cv_done.wait(lk, ready);
    } else {
        const auto limit = std::chrono::steady_clock::now() +
                           std::chrono::microseconds((int64_t)(timeout_ms * 1e3));
        if (!sv->cv_done.wait_until(lk, limit, ready)) return PSCL_E_TIMEOUT;
    }
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) return sv->error;
    if (latency_us) *latency_us = it->second;
    sv->done.erase(it);
    return sv->error;
}

pscl_status pscl_server_stats(pscl_server* sv, int64_t* requests, int64_t* frames,
                              int64_t* launches, double* p50_us, double* p99_us, int reset) {
    if (!sv) return PSCL_E_INVALID;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (requests) *requests = sv->n_req;
    if (frames) *frames = sv->n_frames;
    if (launches) *launches = sv->n_launch;
    if (p50_us) *p50_us = percentile(sv->lat, 0.50);
    if (p99_us) *p99_us = percentile(sv->lat, 0.99);
    if (reset) {
        sv->lat.clear();
        sv->n_req = sv->n_frames = sv->n_launch = 0;
    }
    return sv->error;
}

pscl_status pscl_replay(pscl_server* sv, const pscl_plan* const* plans, int n_plans, int streams,
                        const pscl_job* jobs, const double* arrival_us, int n,
                        double* latency_us, double* elapsed_us) {
    if (n < 0 || (n > 0 && (!jobs || !arrival_us || !latency_us))) return PSCL_E_INVALID;
    if (!sv && (!plans || n_plans < 1 || streams < 1 || streams > 8)) return PSCL_E_INVALID;
    for (int i = 0; i < n; ++i) {
        if (i > 0 && arrival_us[i] < arrival_us[i - 1]) return PSCL_E_INVALID;
        if (!sv && (jobs[i].plan < 0 || jobs[i].plan >= n_plans)) return PSCL_E_INVALID;
    }
    if (!sv)
        for (int i = 0; i < n_plans * streams; ++i)
            if (!plans[i]) return PSCL_E_INVALID;
    if (sv) {
        const double t0 = now_us();
        for (int i = 0; i < n; ++i) {
            const double ta = t0 + arrival_us[i];
            while (now_us() < ta) {
            }
            for (;;) {
                const pscl_status st =
                    sv->submit(jobs[i], nullptr, false, ta, &latency_us[i], nullptr);
                if (st == PSCL_OK) break;
                if (st != PSCL_E_BUSY) return st;
                std::this_thread::yield();
            }
        }
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [&] { return sv->held == 0 || sv->error != PSCL_OK; });
        if (elapsed_us) *elapsed_us = now_us() - t0;
        return sv->error;
    }
    // baseline: one pscl_decode per request, issued in arrival order
    // round-robin over `streams` streams, request i with plan set i % streams
    // (so that no two streams share a plan's workspace); each stream
    // completes in order, observed by a poller
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PSCL_E_NODEV;
    const int S = streams;
    const int RING = 1024;  // events per stream
    std::vector<hipStream_t> str(S, nullptr);
    std::vector<hipEvent_t> evs((size_t)S * RING, nullptr);
    pscl_status st = PSCL_OK;
    for (int s = 0; s < S && st == PSCL_OK; ++s)
        if (hipStreamCreateWithFlags(&str[s], hipStreamNonBlocking) != hipSuccess) st = PSCL_E_HIP;
    for (size_t i = 0; i < evs.size() && st == PSCL_OK; ++i)
        if (hipEventCreateWithFlags(&evs[i], hipEventDisableTiming) != hipSuccess) st = PSCL_E_HIP;
    // per stream: requests issued and completed (request i is the
    // (i / S)-th of stream i % S)
    std::mutex mu;
    std::condition_variable cv;
    std::vector<int> issued(S, 0), completed(S, 0);
    int n_issued = 0, n_completed = 0;
    bool failed = false;
    std::vector<double> t_arr(n > 0 ? n : 1);
    std::thread poller;
    const double t0 = now_us();
    if (st == PSCL_OK) {
        poller = std::thread([&] {
            (void)hipSetDevice(dev);
            for (;;) {
                {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait(lk, [&] { return n_completed < n_issued || failed || n_completed == n; });
                    if (n_completed == n || (failed && n_completed == n_issued)) return;
                }
                bool any = false;
                for (int s = 0; s < S; ++s) {
                    int head;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        if (completed[s] >= issued[s]) continue;
                        head = completed[s];
                    }
                    const hipError_t q = hipEventQuery(evs[(size_t)s * RING + head % RING]);
                    if (q == hipErrorNotReady) continue;
                    const double t = now_us();
                    std::lock_guard<std::mutex> lk(mu);
                    const int req = head * S + s;
                    latency_us[req] = t - t_arr[req];
                    if (q != hipSuccess) failed = true;
                    completed[s] += 1;
                    n_completed += 1;
                    any = true;
                    cv.notify_all();
                }
                if (!any) std::this_thread::yield();
            }
        });
    }
    for (int i = 0; i < n && st == PSCL_OK; ++i) {
        const int s = i % S;
        const double ta = t0 + arrival_us[i];
        while (now_us() < ta) {
        }
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return issued[s] - completed[s] < RING || failed; });
            if (failed) {
                st = PSCL_E_HIP;
                break;
            }
        }
        const pscl_job& J = jobs[i];
        t_arr[i] = ta;
        st = pscl_decode(plans[s * n_plans + J.plan], J.llr, J.F, J.u_hat, J.crc_ok, J.pm, str[s]);
        if (st == PSCL_OK &&
            hipEventRecord(evs[(size_t)s * RING + issued[s] % RING], str[s]) != hipSuccess)
            st = PSCL_E_HIP;
        std::lock_guard<std::mutex> lk(mu);
        if (st != PSCL_OK) {
            failed = true;
        } else {
            issued[s] += 1;
            n_issued += 1;
        }
        cv.notify_all();
    }
    if (poller.joinable()) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (st != PSCL_OK) failed = true;
            cv.notify_all();
        }
        poller.join();
    }
    if (elapsed_us) *elapsed_us = now_us() - t0;
    for (hipStream_t x : str)
        if (x) (void)hipStreamSynchronize(x);
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t x : str)
        if (x) (void)hipStreamDestroy(x);
    if (st == PSCL_OK && failed) st = PSCL_E_HIP;
    return st;
}

}  // extern "C"
