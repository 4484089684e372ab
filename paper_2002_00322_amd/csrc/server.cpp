// Serving loop of libesmf.  Sessions (one molecule each, an ESMF optimisation
// that asks for a grouped J/K build per iteration, Sec. "Shell-Pair
// Screening") are admitted against an HBM budget by the footprint of their
// screened integral store, which then stays resident until the session is
// closed.  Requests are grouped continuously: a dispatcher thread takes the
// pending requests in arrival order, forms a group bounded by a request count
// and a workspace cap, and enqueues it as one grouped launch on the least
// loaded of several streams, so that groups overlap on the device; a
// completion thread polls the groups' events and stamps completion times.
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
    hipEvent_t ev = nullptr;
    int stream = 0;
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
    bool stopping = false;
    bool dispatcher_done = false;
    esmf_server_stats stats{};
    std::thread dispatcher, completer;
};

int free_stream(const Server& S) {
    int best = -1;
    for (int x = 0; x < (int)S.load.size(); ++x)
        if (S.load[x] < S.cfg.max_inflight && (best < 0 || S.load[x] < S.load[best])) best = x;
    return best;
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
            return (S->stopping && S->pending.empty()) || (!S->pending.empty() && free_stream(*S) >= 0);
        });
        if (S->pending.empty()) break;  // stopping and drained
        const int si = free_stream(*S);
        std::vector<int64_t> ids;
        std::vector<GroupEntry> es;
        size_t ws = 0;
        while (!S->pending.empty() && (int)ids.size() < S->cfg.max_group) {
            const int64_t id = S->pending.front();
            const Request& r = S->reqs[id];
            if (!ids.empty() && ws + r.ws_bytes > (size_t)S->cfg.workspace_limit_bytes) break;
            ws += r.ws_bytes;
            ids.push_back(id);
            es.push_back(GroupEntry{(const Handle*)S->sessions[r.session].h, r.m, r.d, r.j, r.k});
            S->pending.pop_front();
        }
        ++S->load[si];
        lk.unlock();
        // sessions with outstanding requests cannot be closed, so the
        // handles stay valid while the group is enqueued without the lock
        esmf_status st = enqueue_group(es, S->cfg.prec == ESMF_PREC_MIXED, S->streams[si]);
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
            --S->load[si];
            const auto now = Clock::now();
            for (int64_t id : ids) finish(*S, id, st, err, now);
            S->cv_done.notify_all();
            continue;
        }
        S->flight.push_back(Group{ids, ev, si});
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
            --S->load[S->flight[x].stream];
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
}

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
    if (cfg->prec != ESMF_PREC_FP64 && cfg->prec != ESMF_PREC_MIXED)
        return fail(ESMF_ERR_INVALID_ARG, "bad precision");
    if (cfg->storage != ESMF_STORE_FP64 && cfg->storage != ESMF_STORE_FP32)
        return fail(ESMF_ERR_INVALID_ARG, "bad storage");
    if ((cfg->prec == ESMF_PREC_FP64) != (cfg->storage == ESMF_STORE_FP64))
        return fail(ESMF_ERR_INVALID_ARG, "FP64 builds need FP64 storage, mixed builds FP32 storage");
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
    if (!srv || !session) return fail(ESMF_ERR_INVALID_ARG, "NULL argument");
    Server* S = (Server*)srv;
    std::lock_guard<std::mutex> adm(S->admit_mu);
    int64_t left;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        left = S->cfg.hbm_budget_bytes - S->resident;
    }
    int64_t fp = 0;
    esmf_eri_t h = nullptr;
    esmf_status st = prepare_impl(nbf, centers, exponents, schwarz_tau, S->cfg.storage, S->prep_stream,
                                  std::max<int64_t>(left, 0), &fp, &h);
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
                               double* j, double* k, int64_t* request) {
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
    r.ws_bytes = group_workspace_bytes(*h, m);
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
