// Request loop serving many independent Ewald systems on one GPU (C ABI in
// include/ewald_server.h).  Built only on the public plan ABI of ewald.h:
// every evaluation is one ewald_energy_forces_ws() call on the system's plan,
// with its per-evaluation buffers in a block of the server's device arena,
// enqueued by a dispatcher thread on one of the server's streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <ctime>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ewald_server.h"

namespace {

constexpr int kMaxStreams = 16;
// Requests whose estimated work is below this go to the express stream
// (stream 0, when the server has more than one), so that they never queue
// behind a large request: about a 5,000-ion electrolyte at the serving mix's
// density and cutoffs (30 flops per particle and k vector, 40 per pair).
constexpr double kExpressCost = 3.0e9;
// A held request (its workspace did not fit) that has waited this long stops
// later requests of its class (express or bulk) from taking arena memory
// before it.
constexpr double kMaxHoldBypass = 0.020;
// Launch sequences in flight per stream: two on the express stream, one on
// each bulk stream (enough queued work to keep the GPU busy); the rest wait in
// the dispatcher's pending list, where a small request that arrives later can
// still pass them (and their workspace is not yet taken).  Fewer large
// requests in flight leave small ones fewer busy compute units to wait for:
// on the serving mix, p99 latency at 0.5 / 0.7 load of arrival rate 4.4-4.7 /
// 4.9-5.2 ms against 5.0-5.6 / 5.9-6.6 ms with two per bulk stream, at the
// same saturation rate (three runs each).
constexpr int kMaxInFlightExpress = 2;
constexpr int kMaxInFlightBulk = 1;
// Express requests that can start together go out as one batched launch
// sequence (ewald_energy_forces_batch), at most this many at a time.
constexpr int kMaxBatch = 64;
constexpr size_t kArenaAlign = 256;
// With EWALD_SERVER_FLAG_EXPRESS_CUS: compute units of the express stream, two
// on each of the 8 XCDs of a 256-CU part, bits 32 g + g and 32 g + g + 8 for
// g = 0..7, which fall two on every XCD whether the mask numbers CUs XCD by
// XCD (32 each) or interleaves them over the XCDs.  The bulk streams get the
// other CUs, so neither class waits for the other's workgroups.
constexpr int kCusExpected = 256;
inline bool reserved_cu(int i)
{
    const int g = i / 32, h = i % 32;
    return h == g || h == g + 8;
}
constexpr uint64_t kDefaultArenaCap = (uint64_t)8 << 30;

double now_s()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct System {
    ewald_plan_t plan = nullptr;
    size_t bytes = 0;  // workspace of a request of n_max particles
    int64_t n_max = 0;
    double cost_per_particle = 0.0;  // relative work estimate of one request per particle
    int stream = -1;                 // stream of its requests in flight (dispatcher)
    int queued = 0;                  // submitted, not yet enqueued      (under the lock)
    int in_flight = 0;               // enqueued, not yet completed      (under the lock)
    bool removing = false;           // no further submissions           (under the lock)
    int64_t hold_pass = -1;          // pass of start_pending that held one of its requests
};

struct Request {
    int64_t ticket = 0;
    System *sys = nullptr;
    int64_t n = 0;
    const double *pos = nullptr, *q = nullptr;
    double *energy = nullptr, *forces = nullptr, *dEdq = nullptr;
    double t_submit = 0.0, t_done = 0.0;
    double cost = 0.0;
    size_t ws_bytes = 0, ws_off = 0;  // its block of the arena
    int stream = -1;
    ewald_status status = EWALD_OK;
    bool done = false, waited = false, held = false;
};

// One enqueued launch sequence (one request, or a batch of express requests)
// and the event recorded after it.
struct Launch {
    hipEvent_t ev = nullptr;
    int stream = -1;
    std::vector<Request *> reqs;
};

// First-fit allocator over one device allocation (host bookkeeping only; used
// by the dispatcher thread alone).
class Arena {
  public:
    void reset(char *base, size_t size)
    {
        base_ = base;
        size_ = size;
        free_.clear();
        if (size) free_[0] = size;
        used_ = peak_ = 0;
    }
    char *base() const { return base_; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    static size_t round(size_t b) { return (b + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = round(bytes);
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

  private:
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length
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
    std::deque<Request *> queue;  // submitted, not yet seen by the dispatcher
    int64_t next_ticket = 0, submitted = 0, completed = 0, in_flight = 0;
    int64_t held = 0, held_total = 0;  // waiting for arena memory now / ever
    uint64_t budget = 0, used = 0, peak_used = 0;
    bool stop = false;
    void *arena_mem = nullptr;
    // dispatcher-only state
    Arena arena;
    std::list<Request *> pending;  // seen, not yet enqueued (in submission order)
    int64_t pass = 0;              // start_pending passes
    int masked = 0;                // bulk streams created with the CU mask
    std::vector<Launch *> flight;
    bool batching = true;
    int64_t batches = 0, batched = 0;  // batched launch sequences, and the requests they carried
    std::vector<double> load;
    std::vector<int> stream_flight;  // launch sequences in flight per stream
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

bool is_express(const ewald_server_s *s, const Request *r)
{
    return s->streams.size() > 1 && r->cost < kExpressCost;
}

// The stream a request would go to now, or -1 if it has to wait for a slot:
// its system's stream while the system has work in flight (the plan is not
// re-entrant), the express stream for a small request, else the bulk stream
// with the least outstanding estimated work; a stream takes at most
// kMaxInFlightExpress (stream 0, also the only stream of a one-stream
// server) or kMaxInFlightBulk launch sequences at a time.
int pick_stream(const ewald_server_s *s, const Request *r)
{
    const int ns = (int)s->streams.size();
    auto open = [&](int i) {
        return s->stream_flight[i] < (i == 0 ? kMaxInFlightExpress : kMaxInFlightBulk);
    };
    if (r->sys->in_flight > 0) return open(r->sys->stream) ? r->sys->stream : -1;
    if (is_express(s, r)) return open(0) ? 0 : -1;
    int st = -1;
    for (int i = ns > 1 ? 1 : 0; i < ns; ++i)
        if (open(i) && (st < 0 || s->load[i] < s->load[st])) st = i;
    return st;
}

// Enqueue requests whose workspace blocks are reserved, on stream st: one
// request alone, or several as one batched launch sequence.
void enqueue(ewald_server_s *s, const std::vector<Request *> &rs, int st)
{
    hipEvent_t ev = take_event(s);
    ewald_status rc = ev ? EWALD_OK : EWALD_ERR_DEVICE;
    const hipStream_t stream = s->streams[st];
    if (rc == EWALD_OK && rs.size() == 1) {
        Request *r = rs[0];
        rc = ewald_plan_set_stream(r->sys->plan, stream);
        if (rc == EWALD_OK)
            rc = ewald_energy_forces_ws(r->sys->plan, r->n, r->pos, r->q, r->energy, r->forces, r->dEdq,
                                        s->arena.base() + r->ws_off, r->ws_bytes);
    } else if (rc == EWALD_OK) {
        const size_t k = rs.size();
        std::vector<ewald_plan_t> plans(k);
        std::vector<int64_t> n(k);
        std::vector<const double *> pos(k), q(k);
        std::vector<double *> energy(k), forces(k), dEdq(k);
        std::vector<void *> ws(k);
        std::vector<size_t> wsb(k);
        for (size_t i = 0; i < k; ++i) {
            const Request *r = rs[i];
            plans[i] = r->sys->plan;
            n[i] = r->n;
            pos[i] = r->pos;
            q[i] = r->q;
            energy[i] = r->energy;
            forces[i] = r->forces;
            dEdq[i] = r->dEdq;
            ws[i] = s->arena.base() + r->ws_off;
            wsb[i] = r->ws_bytes;
        }
        rc = ewald_energy_forces_batch((int32_t)k, plans.data(), n.data(), pos.data(), q.data(), energy.data(),
                                       forces.data(), dEdq.data(), ws.data(), wsb.data(), stream);
    }
    if (rc == EWALD_OK && hipEventRecord(ev, stream) != hipSuccess) {
        (void)hipGetLastError();
        rc = EWALD_ERR_DEVICE;
    }
    if (rc == EWALD_ERR_DEVICE) {
        // part of the sequence may have been enqueued: let it finish before the
        // workspace blocks return to the arena
        (void)hipStreamSynchronize(stream);
        (void)hipGetLastError();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc != EWALD_OK) {
        if (ev) s->events.push_back(ev);
        for (Request *r : rs) {
            r->sys->queued -= 1;
            s->arena.release(r->ws_off, r->ws_bytes);
            r->status = rc;
            r->t_done = now_s();
            r->done = true;
            s->completed += 1;
        }
        s->used = s->arena.used();
        s->cv_done.notify_all();
        return;
    }
    Launch *l = new Launch();
    l->ev = ev;
    l->stream = st;
    l->reqs = rs;
    for (Request *r : rs) {
        System *y = r->sys;
        y->queued -= 1;
        r->stream = st;
        y->stream = st;
        y->in_flight += 1;
        s->in_flight += 1;
        s->load[st] += r->cost;
    }
    if (rs.size() > 1) {
        s->batches += 1;
        s->batched += (int64_t)rs.size();
    }
    s->stream_flight[st] += 1;
    s->flight.push_back(l);
}

// Starts pending requests, in submission order, when their stream has a slot
// and their workspace fits the arena.  One that does not fit is held (it stays
// pending) and later ones may go ahead, until it has waited kMaxHoldBypass:
// then nothing of its class (express or bulk) behind it starts before it does.
// A system's requests start in submission order.  The express requests that
// can start in one pass go out together as one batched launch sequence (one
// slot of the express stream), unless batching is off.  Returns whether any
// started.
bool start_pending(ewald_server_s *s)
{
    bool any = false, blocked[2] = {false, false};
    const double now = now_s();
    const int64_t pass = ++s->pass;
    std::vector<Request *> batch;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Request *r = *it;
        const int cls = is_express(s, r) ? 0 : 1;
        if (r->sys->hold_pass == pass || blocked[cls]) {
            r->sys->hold_pass = pass;
            ++it;
            continue;
        }
        const int st = pick_stream(s, r);
        const bool joins = s->batching && cls == 0 && st == 0;
        if (st < 0 || (joins && (int)batch.size() >= kMaxBatch)) {
            // no slot now; later requests of other systems may have one
            r->sys->hold_pass = pass;
            ++it;
            continue;
        }
        size_t off = 0;
        if (s->arena.alloc(r->ws_bytes, off)) {
            r->ws_off = off;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (r->held) s->held -= 1;
                s->used = s->arena.used();
                s->peak_used = s->arena.peak();
            }
            it = s->pending.erase(it);
            if (joins)
                batch.push_back(r);
            else
                enqueue(s, {r}, st);
            any = true;
            continue;
        }
        r->sys->hold_pass = pass;
        if (!r->held) {
            std::lock_guard<std::mutex> lk(s->mu);
            r->held = true;
            s->held += 1;
            s->held_total += 1;
        }
        if (now - r->t_submit > kMaxHoldBypass) blocked[cls] = true;
        ++it;
    }
    if (!batch.empty()) enqueue(s, batch, 0);
    return any;
}

// Completion of launch sequences in flight; returns whether any completed.
bool poll_flight(ewald_server_s *s)
{
    bool any = false;
    for (size_t i = 0; i < s->flight.size();) {
        Launch *l = s->flight[i];
        const hipError_t e = hipEventQuery(l->ev);
        if (e == hipErrorNotReady) {
            ++i;
            continue;
        }
        const double t = now_s();
        if (e != hipSuccess) (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->events.push_back(l->ev);
            for (Request *r : l->reqs) {
                s->arena.release(r->ws_off, r->ws_bytes);
                s->load[l->stream] = std::max(0.0, s->load[l->stream] - r->cost);
                r->t_done = t;
                if (e != hipSuccess) r->status = EWALD_ERR_DEVICE;
                r->done = true;
                r->sys->in_flight -= 1;
                s->in_flight -= 1;
                s->completed += 1;
            }
            s->used = s->arena.used();
            s->stream_flight[l->stream] -= 1;
        }
        delete l;
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
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->queue.empty() && s->flight.empty() && s->pending.empty()) {
                s->cv_work.wait(lk, [s] { return s->stop || !s->queue.empty(); });
                if (s->queue.empty()) break;  // stopped and drained
            }
            s->pending.insert(s->pending.end(), s->queue.begin(), s->queue.end());
            s->queue.clear();
        }
        // completions first: they return arena memory to held requests
        bool progress = poll_flight(s);
        progress = start_pending(s) || progress;
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
    if (!params || params->n_streams < 1 || params->n_streams > kMaxStreams ||
        (params->flags & ~(EWALD_SERVER_FLAG_EXPRESS_CUS | EWALD_SERVER_FLAG_NO_BATCH)) != 0 ||
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
    s->batching = (params->flags & EWALD_SERVER_FLAG_NO_BATCH) == 0;
    s->budget = params->hbm_budget;
    if (s->budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return EWALD_ERR_DEVICE;
        }
        s->budget = std::min<uint64_t>((uint64_t)(0.9 * (double)free_b), kDefaultArenaCap);
    }
    s->budget = s->budget / kArenaAlign * kArenaAlign;
    if (s->budget == 0 || hipMalloc(&s->arena_mem, s->budget) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return EWALD_ERR_OUT_OF_MEMORY;
    }
    s->arena.reset(static_cast<char *>(s->arena_mem), s->budget);
    bool ok = hipStreamCreateWithFlags(&s->setup, hipStreamNonBlocking) == hipSuccess;
    // with EWALD_SERVER_FLAG_EXPRESS_CUS and more than one stream, the express
    // stream (0) runs on the reserved CUs and the bulk streams on the others,
    // so that a small request always finds free CUs beside large ones
    int n_cus = 0;
    if (hipDeviceGetAttribute(&n_cus, hipDeviceAttributeMultiprocessorCount, params->device) != hipSuccess) {
        (void)hipGetLastError();
        n_cus = 0;
    }
    const bool reserve = params->n_streams > 1 && n_cus == kCusExpected && (params->flags & EWALD_SERVER_FLAG_EXPRESS_CUS);
    std::vector<uint32_t> bulk_mask((size_t)(kCusExpected + 31) / 32, 0u), express_mask(bulk_mask.size(), 0u);
    for (int i = 0; i < kCusExpected; ++i) {
        if (reserved_cu(i))
            express_mask[(size_t)i / 32] |= 1u << (i % 32);
        else
            bulk_mask[(size_t)i / 32] |= 1u << (i % 32);
    }
    for (int i = 0; ok && i < params->n_streams; ++i) {
        hipStream_t st = nullptr;
        const std::vector<uint32_t> &mask = i == 0 ? express_mask : bulk_mask;
        if (reserve && hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()) == hipSuccess) {
            s->masked += 1;
        } else {
            (void)hipGetLastError();
            ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        }
        if (ok) s->streams.push_back(st);
    }
    s->load.assign(s->streams.size(), 0.0);
    s->stream_flight.assign(s->streams.size(), 0);
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
        (void)hipFree(s->arena_mem);
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
    // requests take their buffers from the arena, and run wholly on the stream
    // the dispatcher gives them (so that its CU mask covers every kernel)
    p.flags = EWALD_FLAG_NO_WORKSPACE | EWALD_FLAG_ONE_STREAM;
    if (ewald_params_validate(&p) != EWALD_OK) return EWALD_ERR_INVALID_ARG;
    System *y = new (std::nothrow) System();
    ewald_status rc = y ? ewald_plan(&p, &y->plan) : EWALD_ERR_OUT_OF_MEMORY;
    if (rc != EWALD_OK) {
        delete y;
        return rc;
    }
    y->bytes = ewald_eval_workspace_bytes(y->plan, p.n_max);
    if (Arena::round(y->bytes) > s->budget) {  // a request of n_max could never run
        ewald_release(y->plan);
        delete y;
        return EWALD_ERR_ADMISSION;
    }
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
        r->ws_bytes = ewald_eval_workspace_bytes(y->plan, n);
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
    out->peak_used = s->peak_used;
    out->held = s->held;
    out->held_total = s->held_total;
    out->masked_streams = s->masked;
    out->batches = s->batches;
    out->batched = s->batched;
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
    (void)hipFree(s->arena_mem);
    delete s;
}

}  // extern "C"
