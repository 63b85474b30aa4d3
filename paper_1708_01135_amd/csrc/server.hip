// Request loop serving many independent Ewald systems on one GPU (C ABI in
// include/ewald_server.h).  Built only on the public plan ABI of ewald.h:
// every evaluation is one ewald_energy_forces() call on the system's plan,
// enqueued by a dispatcher thread on one of the server's streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <ctime>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ewald_server.h"

namespace {

constexpr int kMaxStreams = 16;

double now_s()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct System {
    ewald_plan_t plan = nullptr;
    size_t bytes = 0;
    int64_t n_max = 0;
    double cost_per_particle = 0.0;  // relative work estimate of one request per particle
    int stream = -1;                 // stream of its requests in flight (dispatcher)
    int queued = 0;                  // submitted, not yet enqueued      (under the lock)
    int in_flight = 0;               // enqueued, not yet completed      (under the lock)
    bool removing = false;           // no further submissions           (under the lock)
};

struct Request {
    int64_t ticket = 0;
    System *sys = nullptr;
    int64_t n = 0;
    const double *pos = nullptr, *q = nullptr;
    double *energy = nullptr, *forces = nullptr, *dEdq = nullptr;
    double t_submit = 0.0, t_done = 0.0;
    double cost = 0.0;
    int stream = -1;
    hipEvent_t ev = nullptr;
    ewald_status status = EWALD_OK;
    bool done = false, waited = false;
};

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev)
    {
        ok_ = hipGetDevice(&prev_) == hipSuccess;
        if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
        restore_ = ok_ && prev_ != dev;
    }
    ~DeviceGuard()
    {
        if (restore_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = 0;
    bool ok_ = false, restore_ = false;
};

}  // namespace

struct ewald_server_s {
    ewald_server_params prm{};
    std::vector<hipStream_t> streams;
    hipStream_t setup = nullptr;  // plan creation
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<System *> systems;  // by id, nullptr once removed
    std::unordered_map<int64_t, Request *> requests;
    std::deque<Request *> queue;  // submitted, not yet enqueued
    int64_t next_ticket = 0, submitted = 0, completed = 0, in_flight = 0;
    uint64_t budget = 0, used = 0;
    bool stop = false;
    // dispatcher-only state
    std::vector<Request *> flight;
    std::vector<double> load;
    std::vector<hipEvent_t> events;
    std::thread worker;
};

namespace {

hipEvent_t take_event(ewald_server_s *s)
{
    if (!s->events.empty()) {
        hipEvent_t e = s->events.back();
        s->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Enqueue one request: its system's stream while the system has work in
// flight (requests of a system share its workspace), else the stream with
// the least outstanding estimated work.
void enqueue(ewald_server_s *s, Request *r)
{
    System *y = r->sys;
    int st = 0;
    if (y->in_flight > 0) {
        st = y->stream;
    } else {
        for (int i = 1; i < (int)s->streams.size(); ++i)
            if (s->load[i] < s->load[st]) st = i;
    }
    hipEvent_t ev = take_event(s);
    ewald_status rc = ev ? EWALD_OK : EWALD_ERR_DEVICE;
    if (rc == EWALD_OK) rc = ewald_plan_set_stream(y->plan, s->streams[st]);
    if (rc == EWALD_OK) rc = ewald_energy_forces(y->plan, r->n, r->pos, r->q, r->energy, r->forces, r->dEdq);
    if (rc == EWALD_OK && hipEventRecord(ev, s->streams[st]) != hipSuccess) {
        (void)hipGetLastError();
        rc = EWALD_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    y->queued -= 1;
    if (rc != EWALD_OK) {
        if (ev) s->events.push_back(ev);
        r->status = rc;
        r->t_done = now_s();
        r->done = true;
        s->completed += 1;
        s->cv_done.notify_all();
        return;
    }
    r->ev = ev;
    r->stream = st;
    y->stream = st;
    y->in_flight += 1;
    s->in_flight += 1;
    s->load[st] += r->cost;
    s->flight.push_back(r);
}

// Completion of requests in flight; returns whether any completed.
bool poll_flight(ewald_server_s *s)
{
    bool any = false;
    for (size_t i = 0; i < s->flight.size();) {
        Request *r = s->flight[i];
        const hipError_t e = hipEventQuery(r->ev);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        const double t = now_s();
        if (e != hipSuccess) (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->events.push_back(r->ev);
            r->ev = nullptr;
            s->load[r->stream] = std::max(0.0, s->load[r->stream] - r->cost);
            r->t_done = t;
            if (e != hipSuccess) r->status = EWALD_ERR_DEVICE;
            r->done = true;
            r->sys->in_flight -= 1;
            s->in_flight -= 1;
            s->completed += 1;
        }
        s->flight[i] = s->flight.back();
        s->flight.pop_back();
        any = true;
    }
    if (any) s->cv_done.notify_all();
    return any;
}

void dispatcher(ewald_server_s *s)
{
    (void)hipSetDevice(s->prm.device);
    std::vector<Request *> batch;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->queue.empty() && s->flight.empty()) {
                s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
                if (s->queue.empty()) break;  // stopped and drained
            }
            batch.assign(s->queue.begin(), s->queue.end());
            s->queue.clear();
        }
        bool progress = !batch.empty();
        for (Request *r : batch) enqueue(s, r);
        batch.clear();
        progress = poll_flight(s) || progress;
        if (!progress) std::this_thread::yield();
    }
}

System *find_system(ewald_server_s *s, int32_t id)
{
    if (id < 0 || id >= (int32_t)s->systems.size()) return nullptr;
    return s->systems[id];
}

}  // namespace

extern "C" {

double ewald_server_clock(void) { return now_s(); }

ewald_status ewald_server_create(const ewald_server_params *params, ewald_server_t *out)
{
    if (!out) return EWALD_ERR_INVALID_ARG;
    *out = nullptr;
    if (!params || params->n_streams < 1 || params->n_streams > kMaxStreams || params->flags != 0 ||
        params->device < 0 ||
        (params->precision != EWALD_PRECISION_FP64 && params->precision != EWALD_PRECISION_MIXED))
        return EWALD_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return EWALD_ERR_DEVICE;
    }
    if (params->device >= ndev) return EWALD_ERR_INVALID_ARG;
    DeviceGuard dg(params->device);
    if (!dg.ok()) return EWALD_ERR_DEVICE;
    ewald_server_s *s = new (std::nothrow) ewald_server_s();
    if (!s) return EWALD_ERR_OUT_OF_MEMORY;
    s->prm = *params;
    s->budget = params->hbm_budget;
    if (s->budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return EWALD_ERR_DEVICE;
        }
        s->budget = (uint64_t)(0.9 * (double)free_b);
    }
    bool ok = hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < params->n_streams; ++i) {
        hipStream_t st = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->streams.push_back(st);
    }
    s->load.assign(s->streams.size(), 0.0);
    if (ok) {
        try {
            s->worker = std::thread(dispatcher, s);
        } catch (...) {
            ok = false;
        }
    }
    if (!ok) {
        (void)hipGetLastError();
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->setup) (void)hipStreamDestroy(s->setup);
        delete s;
        return EWALD_ERR_DEVICE;
    }
    *out = s;
    return EWALD_OK;
}

ewald_status ewald_server_add_system(ewald_server_t s, const ewald_params *params, int32_t *system_id)
{
    if (!s || !params || !system_id) return EWALD_ERR_INVALID_ARG;
    *system_id = -1;
    ewald_params p = *params;
    p.precision = s->prm.precision;
    p.device = s->prm.device;
    p.stream = s->setup;
    if (ewald_params_validate(&p) != EWALD_OK) return EWALD_ERR_INVALID_ARG;
    const size_t bytes = ewald_plan_workspace_bytes(&p);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->used + bytes > s->budget) return EWALD_ERR_ADMISSION;
        s->used += bytes;  // reserved while the plan is built
    }
    System *y = new (std::nothrow) System();
    ewald_status rc = y ? ewald_plan(&p, &y->plan) : EWALD_ERR_OUT_OF_MEMORY;
    if (rc != EWALD_OK) {
        delete y;
        std::lock_guard<std::mutex> lk(s->mu);
        s->used -= bytes;
        return rc;
    }
    y->bytes = bytes;
    y->n_max = p.n_max;
    // work of one request per particle: the two reciprocal sweeps (structure
    // factor and gather, ~30 flops per k vector) and the pairs inside r_c
    // (~40 flops each), plus a fixed launch cost expressed in the same units
    const double rho = (double)p.n_max / (p.box_L * p.box_L * p.box_L);
    const double pairs = 4.0 / 3.0 * 3.14159265358979323846 * p.r_c * p.r_c * p.r_c * rho;
    y->cost_per_particle = 30.0 * (double)ewald_plan_kcount(y->plan) + 40.0 * pairs;
    std::lock_guard<std::mutex> lk(s->mu);
    *system_id = (int32_t)s->systems.size();
    s->systems.push_back(y);
    return EWALD_OK;
}

ewald_status ewald_server_remove_system(ewald_server_t s, int32_t id)
{
    if (!s) return EWALD_ERR_INVALID_ARG;
    System *y = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        y = find_system(s, id);
        if (!y || y->removing) return EWALD_ERR_INVALID_ARG;
        y->removing = true;
        s->cv_done.wait(lk, [y] { return y->queued == 0 && y->in_flight == 0; });
        s->systems[id] = nullptr;
        s->used -= y->bytes;
    }
    ewald_release(y->plan);
    delete y;
    return EWALD_OK;
}

ewald_status ewald_server_submit(ewald_server_t s, int32_t id, int64_t n, const double *pos, const double *q,
                                 double *energy, double *forces, double *dEdq, int64_t *ticket)
{
    if (!s || !pos || !q || !energy || !ticket || n < 1) return EWALD_ERR_INVALID_ARG;
    Request *r = new (std::nothrow) Request();
    if (!r) return EWALD_ERR_OUT_OF_MEMORY;
    r->n = n;
    r->pos = pos;
    r->q = q;
    r->energy = energy;
    r->forces = forces;
    r->dEdq = dEdq;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        System *y = find_system(s, id);
        if (!y || y->removing) {
            delete r;
            return EWALD_ERR_INVALID_ARG;
        }
        if (n > y->n_max) {
            delete r;
            return EWALD_ERR_CAPACITY;
        }
        r->sys = y;
        r->cost = y->cost_per_particle * (double)n + 2.0e6;
        r->ticket = s->next_ticket++;
        r->t_submit = now_s();
        y->queued += 1;
        s->submitted += 1;
        s->requests.emplace(r->ticket, r);
        s->queue.push_back(r);
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return EWALD_OK;
}

ewald_status ewald_server_wait(ewald_server_t s, int64_t ticket, double *t_submit, double *t_done)
{
    if (!s) return EWALD_ERR_INVALID_ARG;
    Request *r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->requests.find(ticket);
        if (it == s->requests.end() || it->second->waited) return EWALD_ERR_INVALID_ARG;
        r = it->second;
        r->waited = true;
        s->cv_done.wait(lk, [r] { return r->done; });
        s->requests.erase(ticket);
    }
    if (t_submit) *t_submit = r->t_submit;
    if (t_done) *t_done = r->t_done;
    const ewald_status st = r->status;
    delete r;
    return st;
}

ewald_status ewald_server_poll(ewald_server_t s, int64_t ticket, int32_t *done)
{
    if (!s || !done) return EWALD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return EWALD_ERR_INVALID_ARG;
    *done = it->second->done ? 1 : 0;
    return EWALD_OK;
}

ewald_status ewald_server_drain(ewald_server_t s)
{
    if (!s) return EWALD_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [s] { return s->completed == s->submitted; });
    return EWALD_OK;
}

ewald_status ewald_server_system_status(ewald_server_t s, int32_t id)
{
    if (!s) return EWALD_ERR_INVALID_ARG;
    System *y = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        y = find_system(s, id);
        if (!y) return EWALD_ERR_INVALID_ARG;
        s->cv_done.wait(lk, [y] { return y->queued == 0 && y->in_flight == 0; });
    }
    return ewald_plan_status(y->plan);
}

ewald_status ewald_server_get_stats(ewald_server_t s, ewald_server_stats *out)
{
    if (!s || !out) return EWALD_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    int64_t nsys = 0;
    for (System *y : s->systems) nsys += y != nullptr;
    out->systems = nsys;
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->in_flight = s->in_flight;
    out->budget = s->budget;
    out->used = s->used;
    return EWALD_OK;
}

void ewald_server_destroy(ewald_server_t s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();  // the dispatcher drains before it stops
    DeviceGuard dg(s->prm.device);
    for (System *y : s->systems) {
        if (!y) continue;
        ewald_release(y->plan);
        delete y;
    }
    for (auto &kv : s->requests) delete kv.second;
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->setup) (void)hipStreamDestroy(s->setup);
    delete s;
}

}  // extern "C"
