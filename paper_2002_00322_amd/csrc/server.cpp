// Serving loop of libesmf.  Sessions (one molecule each, an ESMF optimisation
// that asks for a grouped J/K build per iteration, Sec. "Shell-Pair
// Screening") are admitted against an HBM budget by the footprint of their
// screened integral store, which then stays resident until the session is
// closed.  Requests are grouped continuously: a dispatcher thread takes the
// pending requests in arrival order, forms a group bounded by a request count
// and the free space of a workspace arena allocated once at creation, and
// enqueues it as one grouped launch on the least loaded of several streams,
// so that groups overlap on the device; a completion thread polls the groups'
// events, stamps completion times and returns their workspace to the arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace esmf;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    int32_t session = 0;
    int32_t m = 0;
    const double* d = nullptr;
    double* j = nullptr;
    double* k = nullptr;
    size_t ws_bytes = 0;
    // recorded on the caller's (producer) stream at submit: the build waits
    // for it, so it sees the density written and the outputs free there
    hipEvent_t ready = nullptr;
    Clock::time_point t_submit, t_done;
    bool done = false;
    esmf_status status = ESMF_OK;
    std::string error;
};

struct Session {
    esmf_eri_t h = nullptr;
    int64_t footprint = 0;
    int64_t outstanding = 0;  // submitted, not yet completed
};

struct Group {
    std::vector<int64_t> ids;
    std::vector<hipEvent_t> ready;  // the requests' producer events, destroyed at completion
    hipEvent_t ev = nullptr;
    int stream = 0;
    size_t off = 0, ws = 0;  // workspace range in the arena
};

// First-fit allocator over the server's workspace arena (one device
// allocation made at creation), 256-byte granularity, coalescing frees.
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(char* b, size_t n) {
        base = b;
        size = n / 256 * 256;
        free_.clear();
        if (size) free_[0] = size;
    }
    static size_t round(size_t n) { return (n + 255) / 256 * 256; }
    size_t largest() const {
        size_t m = 0;
        for (const auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    size_t alloc(size_t n) {  // returns SIZE_MAX if no block fits
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t n) {
        n = round(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && off + it->second == nx->first) {
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
};

struct Server {
    esmf_server_config cfg{};
    int device = 0;
    std::vector<hipStream_t> streams;
    hipStream_t prep_stream = nullptr;
    std::vector<int> load;  // groups in flight per stream
    std::mutex mu;
    std::mutex admit_mu;    // serialises admissions
    std::condition_variable cv_work, cv_done, cv_flight;
    std::deque<int64_t> pending;
    std::unordered_map<int64_t, Request> reqs;
    std::map<int32_t, Session> sessions;
    std::vector<Group> flight;
    int64_t next_req = 1;
    int32_t next_session = 1;
    int64_t resident = 0;
    Arena arena;             // workspace of the groups being enqueued or in flight
    bool stopping = false;
    bool dispatcher_done = false;
    esmf_server_stats stats{};
    std::thread dispatcher, completer;
};

// The next group may start if a stream has room and the first pending request's
// workspace fits next to the workspace in flight (or nothing is in flight).
bool can_start(const Server& S);
int free_stream(const Server& S) {
    int best = -1;
    for (int x = 0; x < (int)S.load.size(); ++x)
        if (S.load[x] < S.cfg.max_inflight && (best < 0 || S.load[x] < S.load[best])) best = x;
    return best;
}

bool can_start(const Server& S) {
    if (S.pending.empty() || free_stream(S) < 0) return false;
    const Request& r = S.reqs.at(S.pending.front());
    return S.arena.largest() >= Arena::round(r.ws_bytes);
}

void finish(Server& S, int64_t id, esmf_status st, const std::string& err, Clock::time_point now) {
    Request& r = S.reqs[id];
    r.done = true;
    r.t_done = now;
    r.status = st;
    r.error = err;
    auto it = S.sessions.find(r.session);
    if (it != S.sessions.end()) --it->second.outstanding;
    ++S.stats.requests_completed;
}

void dispatch_loop(Server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_work.wait(lk, [&] {
            return (S->stopping && S->pending.empty()) || can_start(*S);
        });
        if (S->pending.empty()) break;  // stopping and drained
        const int si = free_stream(*S);
        std::vector<int64_t> ids;
        std::vector<GroupEntry> es;
        std::vector<hipEvent_t> ready;
        size_t ws = 0;
        const size_t room = S->arena.largest();
        while (!S->pending.empty() && (int)ids.size() < S->cfg.max_group) {
            const int64_t id = S->pending.front();
            const Request& r = S->reqs[id];
            if (ws + Arena::round(r.ws_bytes) > room) break;
            ws += Arena::round(r.ws_bytes);
            ids.push_back(id);
            ready.push_back(r.ready);
            es.push_back(GroupEntry{(const Handle*)S->sessions[r.session].h, r.m, r.d, r.j, r.k});
            S->pending.pop_front();
        }
        ++S->load[si];
        const size_t off = S->arena.alloc(ws);  // fits: ws <= the largest free block
        lk.unlock();
        // sessions with outstanding requests cannot be closed, so the
        // handles stay valid while the group is enqueued without the lock.
        // The group's stream first waits for every request's producer event.
        esmf_status st = ESMF_OK;
        for (hipEvent_t e : ready) {
            const hipError_t we = hipStreamWaitEvent(S->streams[si], e, 0);
            if (we != hipSuccess) {
                st = device_fail(we, "wait for the producer stream");
                break;
            }
        }
        if (st == ESMF_OK)
            st = enqueue_group(es, build_mode(*es[0].h, S->cfg.prec), S->streams[si], S->arena.base + off, ws);
        hipEvent_t ev = nullptr;
        if (st == ESMF_OK) {
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                hipEventRecord(ev, S->streams[si]) != hipSuccess) {
                st = device_fail(hipGetLastError(), "group event");
            }
        }
        const std::string err = st == ESMF_OK ? std::string() : std::string(esmf_last_error());
        lk.lock();
        if (st != ESMF_OK) {
            if (ev) (void)hipEventDestroy(ev);
            for (hipEvent_t e : ready) (void)hipEventDestroy(e);
            --S->load[si];
            S->arena.release(off, ws);
            const auto now = Clock::now();
            for (int64_t id : ids) finish(*S, id, st, err, now);
            S->cv_done.notify_all();
            continue;
        }
        S->flight.push_back(Group{ids, ready, ev, si, off, ws});
        ++S->stats.groups_launched;
        S->stats.max_group_size = std::max<int64_t>(S->stats.max_group_size, (int64_t)ids.size());
        S->cv_flight.notify_one();
    }
    S->dispatcher_done = true;
    S->cv_flight.notify_one();
}

void complete_loop(Server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_flight.wait(lk, [&] { return !S->flight.empty() || S->dispatcher_done; });
        if (S->flight.empty()) break;  // dispatcher done and nothing in flight
        bool any = false;
        for (size_t x = 0; x < S->flight.size();) {
            const hipError_t q = hipEventQuery(S->flight[x].ev);
            if (q == hipErrorNotReady) {
                ++x;
                continue;
            }
            const auto now = Clock::now();
            const esmf_status st = q == hipSuccess ? ESMF_OK : ESMF_ERR_DEVICE;
            const std::string err = q == hipSuccess ? std::string()
                                                    : std::string("grouped build: ") + hipGetErrorString(q);
            for (int64_t id : S->flight[x].ids) finish(*S, id, st, err, now);
            (void)hipEventDestroy(S->flight[x].ev);
            for (hipEvent_t e : S->flight[x].ready) (void)hipEventDestroy(e);
            --S->load[S->flight[x].stream];
            S->arena.release(S->flight[x].off, S->flight[x].ws);
            S->flight.erase(S->flight.begin() + x);
            any = true;
        }
        if (any) {
            S->cv_done.notify_all();
            S->cv_work.notify_one();
        } else {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        }
    }
}

void destroy_streams(Server* S) {
    for (hipStream_t s : S->streams)
        if (s) (void)hipStreamDestroy(s);
    if (S->prep_stream) (void)hipStreamDestroy(S->prep_stream);
    if (S->arena.base) (void)hipFree(S->arena.base);
}

}  // namespace

namespace {
esmf_status open_session_impl(esmf_server_t srv, int32_t nbf, const double* centers, const double* exponents,
                              double schwarz_tau, int32_t* session, int64_t* footprint_bytes,
                              const int32_t* lmn, const int32_t* poff, const double* pexp, const double* pcoef);
}  // namespace

extern "C" {

esmf_status esmf_server_create(const esmf_server_config* cfg, esmf_server_t* out) {
    clear_error();
    if (!out) return fail(ESMF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(ESMF_ERR_INVALID_ARG, "cfg is NULL");
    if (cfg->nstreams < 1 || cfg->nstreams > 16) return fail(ESMF_ERR_INVALID_ARG, "nstreams must be 1..16");
    if (cfg->max_group < 1) return fail(ESMF_ERR_INVALID_ARG, "max_group must be >= 1");
    if (cfg->max_inflight < 1) return fail(ESMF_ERR_INVALID_ARG, "max_inflight must be >= 1");
    if (cfg->prec != ESMF_PREC_FP64 && cfg->prec != ESMF_PREC_MIXED && cfg->prec != ESMF_PREC_STORE32)
        return fail(ESMF_ERR_INVALID_ARG, "bad precision");
    if (cfg->storage != ESMF_STORE_FP64 && cfg->storage != ESMF_STORE_FP32 && cfg->storage != ESMF_STORE_DIRECT)
        return fail(ESMF_ERR_INVALID_ARG, "bad storage");
    if (!precision_reads(cfg->prec, cfg->storage))
        return fail(ESMF_ERR_INVALID_ARG,
                    "FP64 builds need FP64 or integral-direct storage, STORE32 builds FP32 storage, "
                    "mixed builds FP32 or FP64 storage");
    if (cfg->hbm_budget_bytes < 0 || cfg->workspace_limit_bytes < 0)
        return fail(ESMF_ERR_INVALID_ARG, "budgets must be >= 0");
    Server* S = new (std::nothrow) Server;
    if (!S) return fail(ESMF_ERR_OUT_OF_MEMORY, "server");
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return device_fail(hipGetLastError(), "hipGetDevice");
    }
    S->streams.assign(cfg->nstreams, nullptr);
    S->load.assign(cfg->nstreams, 0);
    for (auto& s : S->streams) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            destroy_streams(S);
            delete S;
            return device_fail(hipGetLastError(), "hipStreamCreate");
        }
    }
    if (hipStreamCreateWithFlags(&S->prep_stream, hipStreamNonBlocking) != hipSuccess) {
        destroy_streams(S);
        delete S;
        return device_fail(hipGetLastError(), "hipStreamCreate");
    }
    if (cfg->workspace_limit_bytes >= 256) {
        void* a = nullptr;
        if (hipMalloc(&a, (size_t)cfg->workspace_limit_bytes) != hipSuccess) {
            (void)hipGetLastError();
            destroy_streams(S);
            delete S;
            return fail(ESMF_ERR_OUT_OF_MEMORY, "server workspace arena");
        }
        S->arena.init((char*)a, (size_t)cfg->workspace_limit_bytes);
    }
    S->stats.budget_bytes = cfg->hbm_budget_bytes;
    S->dispatcher = std::thread(dispatch_loop, S);
    S->completer = std::thread(complete_loop, S);
    *out = (esmf_server_t)S;
    return ESMF_OK;
}

esmf_status esmf_server_destroy(esmf_server_t srv) {
    clear_error();
    if (!srv) return ESMF_OK;
    Server* S = (Server*)srv;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_work.notify_all();
    S->dispatcher.join();
    S->cv_flight.notify_all();
    S->completer.join();
    for (auto& kv : S->sessions) (void)esmf_eri_release(kv.second.h);
    destroy_streams(S);
    delete S;
    return ESMF_OK;
}

esmf_status esmf_server_open_session(esmf_server_t srv, int32_t nbf, const double* centers,
                                     const double* exponents, double schwarz_tau,
                                     int32_t* session, int64_t* footprint_bytes) {
    clear_error();
    return open_session_impl(srv, nbf, centers, exponents, schwarz_tau, session, footprint_bytes, nullptr,
                             nullptr, nullptr, nullptr);
}

esmf_status esmf_server_open_session_contracted(esmf_server_t srv, int32_t nbf, const double* centers,
                                                const int32_t* lmn, const int32_t* prim_offset,
                                                const double* prim_exp, const double* prim_coef,
                                                double schwarz_tau, int32_t* session, int64_t* footprint_bytes) {
    clear_error();
    std::vector<double> emin;
    const esmf_status st = check_contraction(nbf, lmn, prim_offset, prim_exp, prim_coef, emin);
    if (st != ESMF_OK) return st;
    return open_session_impl(srv, nbf, centers, emin.data(), schwarz_tau, session, footprint_bytes, lmn,
                             prim_offset, prim_exp, prim_coef);
}

}  // extern "C"

namespace {
esmf_status open_session_impl(esmf_server_t srv, int32_t nbf, const double* centers, const double* exponents,
                              double schwarz_tau, int32_t* session, int64_t* footprint_bytes,
                              const int32_t* lmn, const int32_t* poff, const double* pexp, const double* pcoef) {
    if (!srv || !session) return fail(ESMF_ERR_INVALID_ARG, "NULL argument");
    Server* S = (Server*)srv;
    std::lock_guard<std::mutex> adm(S->admit_mu);
    int64_t left;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        left = S->cfg.hbm_budget_bytes - S->resident;
    }
    // give cached, unused workspace back so that the store can be allocated
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, S->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    (void)hipGetLastError();
    int64_t fp = 0;
    esmf_eri_t h = nullptr;
    esmf_status st = prepare_impl(nbf, centers, exponents, schwarz_tau, S->cfg.storage, S->prep_stream,
                                  std::max<int64_t>(left, 0), &fp, &h, lmn, poff, pexp, pcoef);
    if (footprint_bytes) *footprint_bytes = fp;
    std::lock_guard<std::mutex> lk(S->mu);
    if (st != ESMF_OK) {
        if (st == ESMF_ERR_OUT_OF_MEMORY) ++S->stats.sessions_rejected;
        return st;
    }
    const int32_t id = S->next_session++;
    S->sessions[id] = Session{h, fp, 0};
    S->resident += fp;
    S->stats.resident_bytes = S->resident;
    S->stats.sessions_open = (int32_t)S->sessions.size();
    *session = id;
    return ESMF_OK;
}
}  // namespace

extern "C" {

esmf_status esmf_server_close_session(esmf_server_t srv, int32_t session) {
    clear_error();
    if (!srv) return fail(ESMF_ERR_INVALID_ARG, "srv is NULL");
    Server* S = (Server*)srv;
    esmf_eri_t h = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->sessions.find(session);
        if (it == S->sessions.end()) return fail(ESMF_ERR_INVALID_ARG, "unknown session");
        S->cv_done.wait(lk, [&] {
            auto f = S->sessions.find(session);
            return f == S->sessions.end() || f->second.outstanding == 0;
        });
        it = S->sessions.find(session);
        if (it == S->sessions.end()) return fail(ESMF_ERR_INVALID_ARG, "session closed concurrently");
        h = it->second.h;
        S->resident -= it->second.footprint;
        S->sessions.erase(it);
        S->stats.resident_bytes = S->resident;
        S->stats.sessions_open = (int32_t)S->sessions.size();
    }
    return esmf_eri_release(h);
}

esmf_status esmf_server_submit(esmf_server_t srv, int32_t session, int32_t m, const double* d,
                               double* j, double* k, void* hip_stream, int64_t* request) {
    clear_error();
    if (!srv || !request) return fail(ESMF_ERR_INVALID_ARG, "NULL argument");
    Server* S = (Server*)srv;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->sessions.find(session);
    if (it == S->sessions.end()) return fail(ESMF_ERR_INVALID_ARG, "unknown session");
    const Handle* h = (const Handle*)it->second.h;
    esmf_status st = check_build_args(h, m, d, j, k, S->cfg.prec);
    if (st != ESMF_OK) return st;
    Request r;
    r.session = session;
    r.m = m;
    r.d = d;
    r.j = j;
    r.k = k;
    r.ws_bytes = group_workspace_bytes(*h, m, default_variant(build_mode(*h, S->cfg.prec)).plan);
    if (Arena::round(r.ws_bytes) > S->arena.size) {
        char msg[160];
        snprintf(msg, sizeof msg, "request needs %.3f GB of workspace, the server has %.3f GB",
                 r.ws_bytes / 1e9, S->arena.size / 1e9);
        return fail(ESMF_ERR_OUT_OF_MEMORY, msg);
    }
    // the producer event is recorded now, in submission order on the
    // caller's stream, so the build follows everything enqueued there before
    if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
        return device_fail(hipGetLastError(), "producer event");
    const hipError_t re = hipEventRecord(r.ready, (hipStream_t)hip_stream);
    if (re != hipSuccess) {
        (void)hipEventDestroy(r.ready);
        return device_fail(re, "producer event record");
    }
    r.t_submit = Clock::now();
    const int64_t id = S->next_req++;
    S->reqs.emplace(id, r);
    S->pending.push_back(id);
    ++it->second.outstanding;
    ++S->stats.requests_submitted;
    *request = id;
    S->cv_work.notify_one();
    return ESMF_OK;
}

esmf_status esmf_server_wait(esmf_server_t srv, int64_t request, double* latency_ms) {
    clear_error();
    if (!srv) return fail(ESMF_ERR_INVALID_ARG, "srv is NULL");
    Server* S = (Server*)srv;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(request);
    if (it == S->reqs.end()) return fail(ESMF_ERR_INVALID_ARG, "unknown request");
    S->cv_done.wait(lk, [&] {
        auto f = S->reqs.find(request);
        return f == S->reqs.end() || f->second.done;
    });
    it = S->reqs.find(request);
    if (it == S->reqs.end()) return fail(ESMF_ERR_INVALID_ARG, "request waited for concurrently");
    const Request r = it->second;
    S->reqs.erase(it);
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
    if (r.status != ESMF_OK) return fail(r.status, r.error);
    return ESMF_OK;
}

esmf_status esmf_server_stats_get(esmf_server_t srv, esmf_server_stats* out) {
    clear_error();
    if (!srv || !out) return fail(ESMF_ERR_INVALID_ARG, "NULL argument");
    Server* S = (Server*)srv;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    return ESMF_OK;
}

}  // extern "C"
