// Serving layer of libkarl (include/karl.h, "serving"): a request queue, admission by device
// memory (first-fit sub-allocation of a caller-owned arena) and rounds of batched transport
// over the admitted jobs, run either by the caller (karl_server_step) or by worker threads
// that each own a batch and a stream, so that one worker's round tail overlaps the others'
// work.  Uses only the public C ABI of the job and batch entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "karl.h"

extern "C" __attribute__((visibility("hidden"))) karl_status karl_internal_set_error(karl_status code,
                                                                                     const char* msg);

namespace {

karl_status sfail(karl_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return karl_internal_set_error(code, buf);
}

constexpr uint64_t kArenaAlign = 256;
constexpr double kDefaultRoundMs = 50.0;
constexpr int64_t kDefaultMinQuantum = 64;
constexpr int64_t kDefaultMaxQuantum = int64_t(1) << 22;
constexpr int kDefaultWorkers = 2;
constexpr int kMaxWorkers = 4;
constexpr int kFloorWindow = 8;

// A job descriptor together with copies of every host array it points to.
struct OwnedDesc {
    karl_job_desc d{};
    std::vector<double> n_gas, n_field[KARL_MAX_SPECIES], edges[KARL_MAX_SPECIES],
        dens_edges[KARL_MAX_SPECIES], xs[KARL_MAX_PROC], e_field, b_field;
    std::vector<double> ang_edges[KARL_MAX_PROC], ang_theta[KARL_MAX_PROC], ang_pdf[KARL_MAX_PROC];
    std::vector<int32_t> planes;

    void copy_from(const karl_job_desc& s) {
        d = s;
        n_gas.assign(s.n_gas, s.n_gas + s.n_z);
        d.n_gas = n_gas.data();
        // an out-of-range species count is rejected by validation; copy no more than fits
        const int ns = (s.n_species >= 2 && s.n_species <= KARL_MAX_SPECIES) ? s.n_species : 2;
        for (int k = 0; k < ns; ++k) {
            if (s.n_field[k]) {
                n_field[k].assign(s.n_field[k], s.n_field[k] + (size_t)s.n_r * s.n_z);
                d.n_field[k] = n_field[k].data();
            }
            edges[k].assign(s.species[k].edges, s.species[k].edges + s.n_bins + 1);
            d.species[k].edges = edges[k].data();
            if (s.n_dens_bins > 0 && s.species[k].dens_edges) {
                dens_edges[k].assign(s.species[k].dens_edges, s.species[k].dens_edges + s.n_dens_bins + 1);
                d.species[k].dens_edges = dens_edges[k].data();
            }
        }
        for (int i = 0; i < s.n_proc; ++i) {
            xs[i].assign(s.proc[i].xs, s.proc[i].xs + s.n_e);
            d.proc[i].xs = xs[i].data();
            const karl_process_desc& p = s.proc[i];
            if (p.ang_bins > 0) {
                ang_edges[i].assign(p.ang_edges, p.ang_edges + p.ang_bins + 1);
                ang_theta[i].assign(p.ang_theta, p.ang_theta + p.ang_nodes);
                ang_pdf[i].assign(p.ang_pdf, p.ang_pdf + (size_t)p.ang_bins * p.ang_nodes);
                d.proc[i].ang_edges = ang_edges[i].data();
                d.proc[i].ang_theta = ang_theta[i].data();
                d.proc[i].ang_pdf = ang_pdf[i].data();
            }
        }
        if (s.n_planes > 0) {
            planes.assign(s.planes, s.planes + s.n_planes);
            d.planes = planes.data();
        }
        const size_t fb = (size_t)std::max(s.field_nr, 0) * (size_t)std::max(s.field_nz, 0) * 3;
        if (s.e_field) {
            e_field.assign(s.e_field, s.e_field + fb);
            d.e_field = e_field.data();
        }
        if (s.b_field) {
            b_field.assign(s.b_field, s.b_field + fb);
            d.b_field = b_field.data();
        }
        d.workspace = nullptr;
        d.workspace_bytes = 0;
    }
};

// First-fit allocator over [0, size): free blocks by offset, merged with their neighbours.
struct Arena {
    uint64_t size = 0, used = 0, peak = 0;
    std::map<uint64_t, uint64_t> free_blocks;   // offset -> bytes

    void init(uint64_t bytes) {
        size = bytes;
        free_blocks.clear();
        if (bytes) free_blocks[0] = bytes;
    }
    static uint64_t round(uint64_t b) { return (b + kArenaAlign - 1) & ~(kArenaAlign - 1); }
    bool alloc(uint64_t bytes, uint64_t* off) {
        const uint64_t need = round(bytes);
        for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const uint64_t rest = it->second - need;
                const uint64_t start = it->first + need;
                free_blocks.erase(it);
                if (rest) free_blocks[start] = rest;
                used += need;
                peak = std::max(peak, used);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        const uint64_t len = round(bytes);
        used -= len;
        auto next = free_blocks.lower_bound(off);
        uint64_t start = off, end = off + len;
        if (next != free_blocks.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                free_blocks.erase(prev);
            }
        }
        if (next != free_blocks.end() && next->first == end) {
            end += next->second;
            free_blocks.erase(next);
        }
        free_blocks[start] = end - start;
    }
};

enum State { PENDING, ACTIVE, DONE };

struct Served {
    int64_t ticket = 0;
    OwnedDesc desc;
    uint64_t bytes = 0, off = 0;
    void* job = nullptr;
    int64_t next = 0, n = 0;
    int worker = 0;
    State state = PENDING;
};

// One batch, its stream and its round-size control.  The quantum (primaries per job per round)
// starts at its maximum and follows a target round time: the larger of the requested one and
// twice the shortest recent round.  A round lasts at least as long as the longest chain of
// histories in it, whatever its size, so rounds shorter than that floor only waste the device.
struct Worker {
    void* batch = nullptr;
    hipStream_t stream = nullptr;   // created by the server for worker threads
    int64_t quantum = 0;
    double recent[kFloorWindow] = {};
    int n_recent = 0;
    std::thread thread;
};

struct Server {
    int32_t max_jobs = 0;
    int32_t precision = KARL_FP64;
    char* arena_base = nullptr;
    Arena arena;
    double round_ms = kDefaultRoundMs;
    int64_t min_q = kDefaultMinQuantum, max_q = kDefaultMaxQuantum;
    int device = 0;
    int n_workers = 1;
    Worker workers[kMaxWorkers];
    int64_t next_ticket = 1;
    std::deque<Served*> pending;
    std::vector<Served*> active;
    std::deque<int64_t> completed;
    std::unordered_map<int64_t, std::unique_ptr<Served>> all;
    karl_server_stats st{};
    // worker threads
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool running = false, stopping = false;
    karl_status worker_status = KARL_OK;
    std::string worker_error;
};

karl_status server_layout(const karl_server_desc* d, uint64_t* batch_bytes, uint64_t* total) {
    if (!d) return sfail(KARL_EINVAL, "server descriptor is NULL");
    if (d->max_jobs < 1) return sfail(KARL_EINVAL, "max_jobs must be >= 1");
    if (d->precision != KARL_FP64 && d->precision != KARL_FP32)
        return sfail(KARL_EINVAL, "precision must be KARL_FP64 or KARL_FP32");
    if (d->queue_capacity < 0 || d->min_quantum < 0 || d->max_quantum < 0)
        return sfail(KARL_EINVAL, "negative queue or quantum size");
    if (d->min_quantum && d->max_quantum && d->min_quantum > d->max_quantum)
        return sfail(KARL_EINVAL, "min_quantum exceeds max_quantum");
    if (d->n_workers < 0 || d->n_workers > kMaxWorkers)
        return sfail(KARL_EINVAL, "n_workers must be in 0..%d", kMaxWorkers);
    if (!std::isfinite(d->round_ms)) return sfail(KARL_EINVAL, "round_ms must be finite");
    karl_status s = karl_batch_workspace_bytes(d->max_jobs, d->queue_capacity, batch_bytes);
    if (s != KARL_OK) return s;
    *batch_bytes = Arena::round(*batch_bytes);
    const int nw = d->n_workers ? d->n_workers : kDefaultWorkers;
    *total = (uint64_t)nw * *batch_bytes + Arena::round(d->arena_bytes);
    return KARL_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Admit queued jobs in arrival order while a slot is free and the head of the queue fits; each
// goes to the worker with the fewest primaries still to run.  Caller holds the lock.
karl_status admit(Server* S) {
    while (!S->pending.empty() && (int32_t)S->active.size() < S->max_jobs) {
        Served* j = S->pending.front();
        uint64_t off = 0;
        if (!S->arena.alloc(j->bytes, &off)) break;
        karl_job_desc d = j->desc.d;
        d.workspace = S->arena_base + off;
        d.workspace_bytes = j->bytes;
        void* h = nullptr;
        karl_status s = karl_create_job(&d, &h);
        if (s != KARL_OK) {
            S->arena.release(off, j->bytes);
            return s;
        }
        S->pending.pop_front();
        j->off = off;
        j->job = h;
        S->st.admitted += 1;
        if (j->n == 0) {
            j->state = DONE;
            S->completed.push_back(j->ticket);
            S->st.completed += 1;
            continue;
        }
        int64_t load[kMaxWorkers] = {};
        for (Served* a : S->active) load[a->worker] += a->n - a->next;
        int best = 0;
        for (int w = 1; w < S->n_workers; ++w)
            if (load[w] < load[best]) best = w;
        j->worker = best;
        j->state = ACTIVE;
        S->active.push_back(j);
    }
    return KARL_OK;
}

// The jobs of worker w and their ranges for the next round.  Caller holds the lock.
void plan_round(Server* S, int w, std::vector<Served*>& jobs, std::vector<void*>& handles,
                std::vector<int64_t>& ranges) {
    jobs.clear();
    handles.clear();
    ranges.clear();
    const int64_t q = S->workers[w].quantum;
    for (Served* j : S->active) {
        if (j->worker != w) continue;
        jobs.push_back(j);
        handles.push_back(j->job);
        ranges.push_back(j->next);
        ranges.push_back(std::min(j->n, j->next + q));
    }
}

// Book a finished round: advance the jobs, move finished ones to the completed list, update the
// statistics and the worker's quantum.  Caller holds the lock.
void finish_round(Server* S, int w, const std::vector<Served*>& jobs, const std::vector<int64_t>& ranges,
                  double dt, double kernel_ms) {
    int64_t prim = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        Served* j = jobs[i];
        prim += ranges[2 * i + 1] - ranges[2 * i];
        j->next = ranges[2 * i + 1];
        if (j->next >= j->n) {
            j->state = DONE;
            S->completed.push_back(j->ticket);
            S->st.completed += 1;
        }
    }
    S->active.erase(std::remove_if(S->active.begin(), S->active.end(),
                                   [](const Served* j) { return j->state == DONE; }),
                    S->active.end());
    S->st.rounds += 1;
    S->st.primaries += prim;
    S->st.busy_ms += dt;
    S->st.kernel_ms += kernel_ms;
    Worker& W = S->workers[w];
    W.recent[W.n_recent % kFloorWindow] = dt;
    W.n_recent += 1;
    double floor_ms = dt;
    for (int k = 0; k < std::min(W.n_recent, kFloorWindow); ++k) floor_ms = std::min(floor_ms, W.recent[k]);
    const double target = std::max(S->round_ms, 2.0 * floor_ms);
    const double f = std::min(2.0, std::max(0.5, target / std::max(dt, 1e-3)));
    W.quantum = std::min(S->max_q, std::max(S->min_q, (int64_t)std::llround((double)W.quantum * f)));
    S->st.quantum = W.quantum;
}

// One round on worker w's batch (no lock held: the jobs are this worker's alone).
karl_status run_round(Server* S, int w, std::vector<void*>& handles, std::vector<int64_t>& ranges,
                      hipStream_t stream, double* dt, double* kernel_ms) {
    Worker& W = S->workers[w];
    double k0 = 0.0, k1 = 0.0;
    karl_batch_stats(W.batch, &k0, nullptr, nullptr, nullptr);
    const double t0 = now_ms();
    karl_status s = karl_transport_batch(W.batch, handles.data(), ranges.data(), (int32_t)handles.size(), stream);
    *dt = now_ms() - t0;
    karl_batch_stats(W.batch, &k1, nullptr, nullptr, nullptr);
    *kernel_ms = k1 - k0;
    return s;
}

void worker_main(Server* S, int w) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto record = [&](karl_status s) {
        if (S->worker_status == KARL_OK) {
            S->worker_status = s;
            S->worker_error = karl_last_error();
        }
        S->cv_done.notify_all();
    };
    if (hipSetDevice(S->device) != hipSuccess) {
        record(sfail(KARL_EDEVICE, "worker %d: hipSetDevice failed", w));
        return;
    }
    std::vector<Served*> jobs;
    std::vector<void*> handles;
    std::vector<int64_t> ranges;
    while (!S->stopping && S->worker_status == KARL_OK) {
        karl_status s = admit(S);
        if (s != KARL_OK) {
            record(s);
            break;
        }
        plan_round(S, w, jobs, handles, ranges);
        if (jobs.empty()) {
            S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        lk.unlock();
        double dt = 0.0, kms = 0.0;
        s = run_round(S, w, handles, ranges, S->workers[w].stream, &dt, &kms);
        lk.lock();
        if (s != KARL_OK) {
            record(s);
            break;
        }
        finish_round(S, w, jobs, ranges, dt, kms);
        S->cv_done.notify_all();
        S->cv_work.notify_all();
    }
}

}  // namespace

extern "C" {

karl_status karl_server_workspace_bytes(const karl_server_desc* desc, uint64_t* bytes) {
    if (!bytes) return sfail(KARL_EINVAL, "bytes is NULL");
    uint64_t b = 0;
    return server_layout(desc, &b, bytes);
}

karl_status karl_create_server(const karl_server_desc* d, void** out) {
    if (!out) return sfail(KARL_EINVAL, "out is NULL");
    *out = nullptr;
    uint64_t batch_bytes = 0, total = 0;
    karl_status s = server_layout(d, &batch_bytes, &total);
    if (s != KARL_OK) return s;
    if (!d->workspace) return sfail(KARL_EINVAL, "workspace is NULL");
    if (d->workspace_bytes < total)
        return sfail(KARL_ENOMEM, "workspace has %llu bytes, server needs %llu",
                     (unsigned long long)d->workspace_bytes, (unsigned long long)total);
    auto S = std::make_unique<Server>();
    S->max_jobs = d->max_jobs;
    S->precision = d->precision;
    S->round_ms = d->round_ms > 0.0 ? d->round_ms : kDefaultRoundMs;
    S->min_q = d->min_quantum ? d->min_quantum : kDefaultMinQuantum;
    S->max_q = d->max_quantum ? d->max_quantum : std::max(kDefaultMaxQuantum, S->min_q);
    S->n_workers = d->n_workers ? d->n_workers : kDefaultWorkers;
    if (hipGetDevice(&S->device) != hipSuccess) return sfail(KARL_EDEVICE, "hipGetDevice failed");
    for (int w = 0; w < S->n_workers; ++w) {
        Worker& W = S->workers[w];
        W.quantum = S->max_q;
        s = karl_create_batch(d->max_jobs, d->queue_capacity, (char*)d->workspace + (size_t)w * batch_bytes,
                              batch_bytes, &W.batch);
        if (s == KARL_OK && hipStreamCreateWithFlags(&W.stream, hipStreamNonBlocking) != hipSuccess)
            s = sfail(KARL_EDEVICE, "hipStreamCreateWithFlags failed");
        if (s != KARL_OK) {
            for (int k = 0; k <= w; ++k) {
                if (S->workers[k].batch) karl_destroy_batch(S->workers[k].batch);
                if (S->workers[k].stream) (void)hipStreamDestroy(S->workers[k].stream);
            }
            return s;
        }
    }
    S->arena_base = (char*)d->workspace + (size_t)S->n_workers * batch_bytes;
    S->arena.init(d->workspace_bytes - (uint64_t)S->n_workers * batch_bytes);
    S->st.quantum = S->max_q;
    *out = S.release();
    return KARL_OK;
}

karl_status karl_server_submit(void* server, const karl_job_desc* desc, int64_t* ticket) {
    Server* S = (Server*)server;
    if (!S || !desc || !ticket) return sfail(KARL_EINVAL, "server, desc or ticket is NULL");
    uint64_t bytes = 0;
    karl_status s = karl_workspace_bytes(desc, &bytes);
    if (s != KARL_OK) return s;
    if (desc->precision != S->precision)
        return sfail(KARL_EINVAL, "job precision %d differs from the server's %d", desc->precision,
                     S->precision);
    if (Arena::round(bytes) > S->arena.size)
        return sfail(KARL_EINVAL, "job needs %llu bytes, the whole arena has %llu",
                     (unsigned long long)bytes, (unsigned long long)S->arena.size);
    auto j = std::make_unique<Served>();
    j->desc.copy_from(*desc);
    j->bytes = bytes;
    j->n = desc->n_primaries;
    std::lock_guard<std::mutex> lk(S->mu);
    j->ticket = S->next_ticket++;
    *ticket = j->ticket;
    S->pending.push_back(j.get());
    S->all[j->ticket] = std::move(j);
    S->st.submitted += 1;
    S->cv_work.notify_all();
    return KARL_OK;
}

karl_status karl_server_step(void* server, void* hip_stream, int32_t* n_active, int32_t* n_pending) {
    Server* S = (Server*)server;
    if (!S) return sfail(KARL_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->running) return sfail(KARL_ESTATE, "worker threads run the rounds: use karl_server_wait");
    if (hipSetDevice(S->device) != hipSuccess) return sfail(KARL_EDEVICE, "hipSetDevice failed");
    karl_status s = admit(S);
    if (s != KARL_OK) return s;
    std::vector<Served*> jobs;
    std::vector<void*> handles;
    std::vector<int64_t> ranges;
    for (int w = 0; w < S->n_workers; ++w) {
        plan_round(S, w, jobs, handles, ranges);
        if (jobs.empty()) continue;
        double dt = 0.0, kms = 0.0;
        s = run_round(S, w, handles, ranges, (hipStream_t)hip_stream, &dt, &kms);
        if (s != KARL_OK) return s;
        finish_round(S, w, jobs, ranges, dt, kms);
    }
    // jobs that finished free slots (not memory) for the next admission
    if ((s = admit(S)) != KARL_OK) return s;
    if (n_active) *n_active = (int32_t)S->active.size();
    if (n_pending) *n_pending = (int32_t)S->pending.size();
    return KARL_OK;
}

karl_status karl_server_start(void* server) {
    Server* S = (Server*)server;
    if (!S) return sfail(KARL_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->running) return sfail(KARL_ESTATE, "server already started");
    S->stopping = false;
    S->running = true;
    for (int w = 0; w < S->n_workers; ++w) S->workers[w].thread = std::thread(worker_main, S, w);
    return KARL_OK;
}

karl_status karl_server_wait(void* server, double timeout_ms, int32_t* n_active, int32_t* n_pending) {
    Server* S = (Server*)server;
    if (!S) return sfail(KARL_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->running) return sfail(KARL_ESTATE, "server not started");
    if (S->completed.empty() && S->worker_status == KARL_OK && timeout_ms > 0.0)
        S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), [&] {
            return !S->completed.empty() || S->worker_status != KARL_OK;
        });
    if (n_active) *n_active = (int32_t)S->active.size();
    if (n_pending) *n_pending = (int32_t)S->pending.size();
    if (S->worker_status != KARL_OK)
        return karl_internal_set_error(S->worker_status, S->worker_error.c_str());
    return KARL_OK;
}

karl_status karl_server_stop(void* server) {
    Server* S = (Server*)server;
    if (!S) return sfail(KARL_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (!S->running) return KARL_OK;
        S->stopping = true;
        S->cv_work.notify_all();
    }
    for (int w = 0; w < S->n_workers; ++w)
        if (S->workers[w].thread.joinable()) S->workers[w].thread.join();
    std::lock_guard<std::mutex> lk(S->mu);
    S->running = false;
    if (S->worker_status != KARL_OK)
        return karl_internal_set_error(S->worker_status, S->worker_error.c_str());
    return KARL_OK;
}

karl_status karl_server_poll(void* server, int64_t* tickets, int32_t capacity, int32_t* n) {
    Server* S = (Server*)server;
    if (!S || !n || (capacity > 0 && !tickets)) return sfail(KARL_EINVAL, "server, tickets or n is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    int32_t k = 0;
    while (k < capacity && !S->completed.empty()) {
        tickets[k++] = S->completed.front();
        S->completed.pop_front();
    }
    *n = k;
    return KARL_OK;
}

karl_status karl_server_job(void* server, int64_t ticket, void** job) {
    Server* S = (Server*)server;
    if (!S || !job) return sfail(KARL_EINVAL, "server or job is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return sfail(KARL_EINVAL, "unknown ticket %lld", (long long)ticket);
    if (it->second->state == PENDING) return sfail(KARL_ESTATE, "ticket %lld is not admitted yet", (long long)ticket);
    *job = it->second->job;
    return KARL_OK;
}

karl_status karl_server_release(void* server, int64_t ticket) {
    Server* S = (Server*)server;
    if (!S) return sfail(KARL_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return sfail(KARL_EINVAL, "unknown ticket %lld", (long long)ticket);
    Served* j = it->second.get();
    if (j->state != DONE) return sfail(KARL_ESTATE, "ticket %lld has not completed", (long long)ticket);
    karl_status s = karl_destroy_job(j->job);
    S->arena.release(j->off, j->bytes);
    S->completed.erase(std::remove(S->completed.begin(), S->completed.end(), ticket), S->completed.end());
    S->all.erase(it);
    S->st.released += 1;
    S->cv_work.notify_all();
    return s;
}

karl_status karl_server_stats_get(void* server, karl_server_stats* out) {
    Server* S = (Server*)server;
    if (!S || !out) return sfail(KARL_EINVAL, "server or out is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->arena_used = S->arena.used;
    out->arena_peak = S->arena.peak;
    return KARL_OK;
}

karl_status karl_destroy_server(void* server) {
    Server* S = (Server*)server;
    if (!S) return sfail(KARL_EINVAL, "server is NULL");
    karl_server_stop(S);
    karl_status s = KARL_OK;
    for (auto& kv : S->all)
        if (kv.second->job) karl_destroy_job(kv.second->job);
    for (int w = 0; w < S->n_workers; ++w) {
        if (S->workers[w].stream) (void)hipStreamSynchronize(S->workers[w].stream);
        karl_status b = karl_destroy_batch(S->workers[w].batch);
        if (s == KARL_OK) s = b;
        if (S->workers[w].stream) (void)hipStreamDestroy(S->workers[w].stream);
    }
    delete S;
    return s;
}

}  // extern "C"
