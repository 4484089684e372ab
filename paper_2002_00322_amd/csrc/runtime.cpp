// Host runtime of libesmf: argument checking, the tile plan of a molecule,
// the screened block list, HBM ownership and the launch sequence of a build.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <thread>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

using namespace esmf;

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace esmf {

esmf_status fail(esmf_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

esmf_status device_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return ESMF_ERR_DEVICE;
}

void clear_error() { g_last_error.clear(); }

}  // namespace esmf

namespace esmf {

// per-thread instrumentation of the main contraction kernel
struct TimedLaunch {
    hipEvent_t start, stop;
};
thread_local bool g_timing = false;
// Default launch variant; ESMF_OCCUPANCY=2|3 (4: STORE32) and ESMF_SKIP_ZERO_FRAGMENTS=0|1
// override it (tuning comparisons), ESMF_XCD_ORDER=0 disables the per-XCD
// grouping of work items at prepare time.
int env_int(const char* name, int dflt) {
    const char* v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}
KernelVariant default_variant(int mode) {
    KernelVariant v;
    // measured on MI355X (1000-function slab): FP64 and both mixed forms at
    // 3 workgroups per CU (FP64: the LDS bound; FP64 runs as fast at 2),
    // STORE32 at 4; MIXED on an FP64 store spills ~20 bytes at 3 and still
    // runs 13 % faster than at 2.  Mixed: FP32 chains of 2 steps (8
    // products) between FP64 drains of the K views; on the 64-chain batch
    // the largest K error against the oracle was 8.6e-9 and 9.4e-9 with
    // chains of 2 and 4 steps (J runs in FP64 and does not depend on it)
    v.occupancy = env_int("ESMF_OCCUPANCY", mode == 2 ? 4 : 3);
    v.skip_zero_fragments = env_int("ESMF_SKIP_ZERO_FRAGMENTS", 1) != 0;
    v.chain = env_int("ESMF_CHAIN", 2);
    // work plan: integral-direct builds evaluate each integral once in the
    // fused plan against twice in two visits (slab1000, FP64: 150 ms against
    // 290 ms); stored builds run faster on the two-visit plan at 3
    // workgroups per CU than fused at 2, the fused kernel's LDS bound (67 ms
    // against 83 ms FP64, 57 against 82 STORE32, 63 against 90 mixed)
    const int plan_default = mode == 3 ? kPlanFused : kPlanTwoVisit;
    v.plan = env_int("ESMF_PLAN", plan_default) == kPlanTwoVisit ? kPlanTwoVisit : kPlanFused;
    if (v.plan == kPlanFused) v.occupancy = 2;
    v.band = fused_band();
    return v;
}
int fused_band() { return env_int("ESMF_BAND", kFusedBand) == 2 ? 2 : kFusedBand; }
thread_local std::vector<TimedLaunch> g_timed;

#define ESMF_HIP(call, what)                                 \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return device_fail(e_, what);  \
    } while (0)

template <typename T>
struct DevBuf {
    T* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) { return hipMalloc((void**)&p, sizeof(T) * std::max<size_t>(count, 1)); }
};

bool finite_all(const double* x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// Narrow group g of a build of m densities without symmetric ones:
// densities 8g .. 8g+mg-1, columns D_0..D_{mg-1} | D_0^T..D_{mg-1}^T packed
// at the front (2 mg of the 16), so that a small group's K views can run on
// fewer products (k_products).
DensityGroup narrow_group(int m, int g) {
    DensityGroup G;
    G.c0 = 8 * g;
    G.mg = std::min(8, m - 8 * g);
    G.jw = 8;
    for (int c = 0; c < 16; ++c) G.xsrc[c] = G.kf[c] = G.kt[c] = -1;
    for (int p = 0; p < G.mg; ++p) {
        G.kf[p] = (int8_t)p;
        G.kt[p] = (int8_t)(G.mg + p);
        G.xsrc[p] = (int8_t)p;
        G.xsrc[G.mg + p] = (int8_t)(p | kXsrcTransposed);
    }
    return G;
}

// 4-column matrix-core products of a group's K views: the groups of 4 its
// used K columns span, where that is 1 or 2 and the build runs an FP64
// matrix-core mode (0, 2, 3) on the two-visit plan with 8 J columns; else
// 0, the 16-column product.  The operand prep and the contraction both read
// it from the unit.
int k_products(const DensityGroup& G, int mode, int plan) {
    if ((mode != 0 && mode != 2 && mode != 3) || plan != kPlanTwoVisit || G.jw != 8) return 0;
    int ncol = 0;
    for (int c = 0; c < 16; ++c)
        if (G.xsrc[c] >= 0) ncol = c + 1;
    const int q = (ncol + 3) / 4;
    return q >= 3 ? 0 : q;
}

// Descriptor of density group G of molecule h under work plan `plan`; the
// launch-range offsets and workspace pointers are set by the caller.
void fill_unit(UnitDesc& u, const Handle& h, int plan, int mode, const double* d, double* j, double* k,
               const DensityGroup& G) {
    const DevPlan& P = h.plan[plan];
    std::memset(&u, 0, sizeof u);
    u.vals = h.d_vals;
    u.rec = P.d_rec;
    u.slot_fn = h.d_slot_fn;
    u.kptr = P.d_kptr;
    u.jptr = P.d_jptr;
    u.used = h.d_used;
    u.nused = h.nused;
    u.red = P.d_red;
    u.nred = P.nred;
    u.d = d;
    u.j = j;
    u.k = k;
    u.nbf = h.nbf;
    u.ntiles = h.ntiles;
    u.c0 = G.c0;
    u.mg = G.mg;
    u.jw = G.jw;
    u.kq = k_products(G, mode, plan);
    for (int c = 0; c < 16; ++c) {
        u.xsrc[c] = G.xsrc[c];
        u.kf[c] = G.kf[c];
        u.kt[c] = G.kt[c];
    }
    u.nslots = h.nslots;
    u.tau = h.tau;
}

void fill_unit(UnitDesc& u, const Handle& h, int plan, int mode, int m, const double* d, double* j, double* k,
               int g) {
    fill_unit(u, h, plan, mode, d, j, k, narrow_group(m, g));
}

int64_t DevPlan::device_bytes() const {
    return (int64_t)(sizeof(WorkItem) * items.size() + sizeof(EntryRecord) * (size_t)nentries +
                     sizeof(int64_t) * 2 * (size_t)(ntargets + 1) + sizeof(int32_t) * (size_t)nred);
}

void DevPlan::release() {
    if (d_items) (void)hipFree(d_items);
    if (d_rec) (void)hipFree(d_rec);
    if (d_kptr) (void)hipFree(d_kptr);
    if (d_jptr) (void)hipFree(d_jptr);
    if (d_red) (void)hipFree(d_red);
    *this = DevPlan();
}

std::vector<DensityGroup> plan_density_groups(int m, const uint8_t* sym) {
    std::vector<DensityGroup> out;
    bool any = false;
    for (int p = 0; sym && p < m; ++p) any = any || sym[p] != 0;
    if (!any) {
        for (int g = 0; g < (m + 7) / 8; ++g) out.push_back(narrow_group(m, g));
        return out;
    }
    int c0 = 0;
    while (c0 < m) {
        // as many densities as 16 K columns and 16 J columns hold
        int mg = 0, cols = 0;
        while (c0 + mg < m && mg < 16) {
            const int need = sym[c0 + mg] ? 1 : 2;
            if (cols + need > 16) break;
            cols += need;
            ++mg;
        }
        DensityGroup G;
        G.c0 = c0;
        G.mg = mg;
        G.jw = mg > 8 ? 16 : 8;
        for (int c = 0; c < 16; ++c) G.xsrc[c] = G.kf[c] = G.kt[c] = -1;
        int col = 0;
        for (int p = 0; p < mg; ++p) {  // forward columns first
            G.kf[p] = (int8_t)col;
            G.xsrc[col++] = (int8_t)p;
        }
        for (int p = 0; p < mg; ++p) {  // then the transposed ones
            if (sym[c0 + p]) {
                G.kt[p] = G.kf[p];
            } else {
                G.kt[p] = (int8_t)col;
                G.xsrc[col++] = (int8_t)(p | kXsrcTransposed);
            }
        }
        out.push_back(G);
        c0 += mg;
    }
    return out;
}

// Per-build workspace comes from the device's stream-ordered pool, kept
// cached between builds (release threshold raised once per device).
void ensure_pool_cached(int device) {
    static thread_local int done_device = -1;
    if (done_device == device) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    done_device = device;
}

// Scratch of the ESMF terms (densities, energy, gradient: megabytes) comes
// from a pool of its own, so that it never splits the cached build
// workspace (tens of GB) of the device's default pool: a split block forces
// the next build to map fresh memory.
hipError_t small_scratch_alloc(void** p, size_t bytes, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::vector<hipMemPool_t> pools;
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        if ((int)pools.size() <= dev) pools.resize(dev + 1, nullptr);
        if (!pools[dev]) {
            hipMemPoolProps props;
            std::memset(&props, 0, sizeof props);
            props.allocType = hipMemAllocationTypePinned;
            props.location.type = hipMemLocationTypeDevice;
            props.location.id = dev;
            e = hipMemPoolCreate(&pools[dev], &props);
            if (e != hipSuccess) {
                pools[dev] = nullptr;
                return e;
            }
            uint64_t keep = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pools[dev], hipMemPoolAttrReleaseThreshold, &keep);
        }
        pool = pools[dev];
    }
    return hipMallocFromPoolAsync(p, bytes, pool, s);
}

void free_handle(Handle* h) {
    if (!h) return;
    for (DevPlan& p : h->plan) p.release();
    if (h->d_used) (void)hipFree(h->d_used);
    if (h->d_vals) (void)hipFree(h->d_vals);
    if (h->d_blk_mask) (void)hipFree(h->d_blk_mask);
    if (h->d_blk_off) (void)hipFree(h->d_blk_off);
    if (h->d_blk_tiles) (void)hipFree(h->d_blk_tiles);
    if (h->d_slot_fn) (void)hipFree(h->d_slot_fn);
    if (h->ws_done) {
        (void)hipEventSynchronize(h->ws_done);
        (void)hipEventDestroy(h->ws_done);
    }
    if (h->ws) (void)hipFree(h->ws);
    delete h;
}

// ---- batched builds --------------------------------------------------------
// A batched plan serves one combination of molecules, density counts,
// precision and stream: one unit per molecule and density group with its own
// workspace, and for each work-plan kind (two visits, fused) a unit table and
// the concatenated work items (each molecule's list padded to a multiple of 8
// so that its per-XCD grouping is kept).  On its first call it times the
// contraction variants on itself and keeps the fastest; on a non-NULL stream
// the build (pointer-table copy, operand prep, contraction, reduction) is
// then captured once as a HIP graph and replayed.  A call refreshes the
// density/output pointers in the pinned host table, which the copy node reads
// at replay time.
struct BatchPlan {
    std::vector<const Handle*> hs;
    std::vector<int32_t> ms;
    int mode = 0;  // arithmetic mode = esmf_precision
    int kind = kPlanTwoVisit;  // work plan of every unit (the default of the mode)
    hipStream_t stream = nullptr;
    int nunits = 0, nitems = 0, red_total = 0;
    int64_t prep_total = 0, zero_total = 0;
    std::vector<int> unit_mol;       // molecule of each unit
    UnitDesc* d_units = nullptr;
    UnitDesc* h_units = nullptr;     // pinned
    WorkItem* d_items = nullptr;
    void* ws = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
    bool tuned = false;
    bool graph = false;              // replays run the captured graph
    KernelVariant variant;
    std::vector<KernelVariant> cand; // tuner candidates and their best times
    std::vector<double> cand_ms;
    double best_ms = 0.0;
    // work-item length stage: factors applied to every molecule's cut, times
    std::vector<double> item_factor, item_ms;
    double item_factor_chosen = 1.0;
    ~BatchPlan() {
        if (launched && done) (void)hipEventSynchronize(done);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (done) (void)hipEventDestroy(done);
        if (d_units) (void)hipFree(d_units);
        if (h_units) (void)hipHostFree(h_units);
        if (d_items) (void)hipFree(d_items);
        if (ws) (void)hipFree(ws);
    }
};

std::mutex g_plan_mu;
std::vector<std::unique_ptr<BatchPlan>> g_plans;  // most recently used last
constexpr size_t kMaxPlans = 4;
// what the last batched build of the calling thread ran
thread_local esmf_batch_report g_batch_report{};

esmf_status make_plan(const std::vector<const Handle*>& hs, const std::vector<int32_t>& ms,
                      int mode, hipStream_t stream, std::unique_ptr<BatchPlan>& out) {
    std::unique_ptr<BatchPlan> p(new (std::nothrow) BatchPlan);
    if (!p) return fail(ESMF_ERR_OUT_OF_MEMORY, "plan");
    p->hs = hs;
    p->ms = ms;
    p->mode = mode;
    p->kind = default_variant(mode).plan;
    p->stream = stream;
    const int kind = p->kind;
    std::vector<UnitDesc> units;
    std::vector<WorkItem> items;
    std::vector<size_t> ws_off;
    size_t ws_total = 0;
    for (size_t i = 0; i < hs.size(); ++i) {
        const Handle& h = *hs[i];
        const int G = (ms[i] + 7) / 8;
        for (int g = 0; g < G; ++g) {
            UnitDesc u;
            fill_unit(u, h, kind, mode, ms[i], nullptr, nullptr, nullptr, g);
            u.prep_begin = p->prep_total;
            u.red_begin = p->red_total;
            u.zero_begin = p->zero_total;
            p->prep_total += unit_prep_size(u);
            p->red_total += h.plan[kind].nred;
            p->zero_total += unit_zero_size(u);
            const int uid = (int)units.size();
            units.push_back(u);
            p->unit_mol.push_back((int)i);
            ws_off.push_back(ws_total);
            ws_total += group_unit_bytes(h, kind);
            for (WorkItem it : h.plan[kind].items) {
                it.unit = uid;
                items.push_back(it);
            }
            while (items.size() % 8) items.push_back(WorkItem{0, 0, 0, 0, 0, 0, 0, uid});
        }
    }
    if ((int64_t)items.size() > INT32_MAX || p->red_total < 0) return fail(ESMF_ERR_OUT_OF_MEMORY, "batch too large");
    p->nunits = (int)units.size();
    p->nitems = (int)items.size();
    if (hipMalloc(&p->ws, std::max<size_t>(ws_total, 1)) != hipSuccess ||
        hipMalloc((void**)&p->d_units, sizeof(UnitDesc) * std::max<size_t>(units.size(), 1)) != hipSuccess ||
        hipMalloc((void**)&p->d_items, sizeof(WorkItem) * std::max<size_t>(items.size(), 1)) != hipSuccess ||
        hipHostMalloc((void**)&p->h_units, sizeof(UnitDesc) * std::max<size_t>(units.size(), 1),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ESMF_ERR_OUT_OF_MEMORY, "batch workspace");
    }
    for (size_t u = 0; u < units.size(); ++u) {
        const Handle& h = *hs[p->unit_mol[u]];
        double* base = (double*)((char*)p->ws + ws_off[u]);
        unit_set_workspace(units[u], base, (double*)((char*)base + operand_bytes(h.ntiles)), h.plan[kind].nkslots);
        p->h_units[u] = units[u];
    }
    if (!items.empty())
        ESMF_HIP(hipMemcpy(p->d_items, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice),
                 "copy batch items");
    ESMF_HIP(hipEventCreateWithFlags(&p->done, hipEventDisableTiming), "batch event");
    out = std::move(p);
    return ESMF_OK;
}

// The plan's launch sequence with variant v (table copy, prep, contraction
// bracketed by e0/e1, reduction) on stream s.
hipError_t enqueue_plan(BatchPlan& p, hipStream_t s, const KernelVariant& v, hipEvent_t e0, hipEvent_t e1) {
    hipError_t e = hipMemcpyAsync(p.d_units, p.h_units, sizeof(UnitDesc) * p.nunits, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return launch_units(p.d_units, 0, p.nunits, p.prep_total, p.zero_total, p.red_total, p.d_items, p.nitems, p.mode,
                        v, s, e0, e1);
}

void set_plan_pointers(BatchPlan& p, const double* const* d, double* const* j, double* const* k) {
    for (int u = 0; u < p.nunits; ++u) {
        const int i = p.unit_mol[u];
        p.h_units[u].d = d[i];
        p.h_units[u].j = j[i];
        p.h_units[u].k = k[i];
    }
}

// Best of two timed runs of the plan's variant (ms of contraction).
esmf_status time_plan(BatchPlan& p, const double* const* d, double* const* j, double* const* k, double* ms) {
    if (p.launched) ESMF_HIP(hipEventSynchronize(p.done), "previous batch");
    set_plan_pointers(p, d, j, k);
    hipEvent_t e0, e1;
    ESMF_HIP(hipEventCreate(&e0), "hipEventCreate");
    ESMF_HIP(hipEventCreate(&e1), "hipEventCreate");
    hipError_t err = hipSuccess;
    float t = 0.0f, tmin = 3.4e38f;
    for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
        err = enqueue_plan(p, p.stream, p.variant, e0, e1);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        tmin = std::min(tmin, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return device_fail(err, "batched tuner");
    *ms = tmin;
    return ESMF_OK;
}

esmf_status run_plan(BatchPlan& p, const double* const* d, double* const* j, double* const* k) {
    if (p.launched) ESMF_HIP(hipEventSynchronize(p.done), "previous batch");
    set_plan_pointers(p, d, j, k);
    auto enqueue_v = [&](hipStream_t s, const KernelVariant& v, hipEvent_t e0,
                         hipEvent_t e1) -> hipError_t { return enqueue_plan(p, s, v, e0, e1); };
    if (!p.tuned) {
        // first call: time every variant on the plan itself (the last run
        // leaves valid results; all variants agree to rounding), keep the fastest
        p.variant = default_variant(p.mode);
        if (env_int("ESMF_TUNE", 1) && p.nunits > 0) {
            hipEvent_t e0, e1;
            ESMF_HIP(hipEventCreate(&e0), "hipEventCreate");
            ESMF_HIP(hipEventCreate(&e1), "hipEventCreate");
            double best = 1e300;
            hipError_t err = hipSuccess;
            // within the plan's work plan (the mode's default), so that a
            // batch equals, bitwise, the single builds of its molecules
            for (const KernelVariant& v : tune_candidates(p.mode))
                if (v.plan == p.kind) p.cand.push_back(v);
            p.cand_ms.assign(p.cand.size(), 0.0);
            for (size_t c = 0; c < p.cand.size() && err == hipSuccess; ++c) {
                const KernelVariant& v = p.cand[c];
                float t = 0.0f, tmin = 3.4e38f;
                const bool big = p.nitems > (1 << 16);
                for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
                    err = enqueue_v(p.stream, v, e0, e1);
                    if (err == hipSuccess) err = hipEventSynchronize(e1);
                    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
                    if (rep > 0 || big) tmin = std::min(tmin, t);
                }
                p.cand_ms[c] = tmin;
                if (tmin < best) {
                    best = tmin;
                    p.variant = v;
                }
            }
            p.best_ms = best;
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            if (err != hipSuccess) return device_fail(err, "batched tuner");
        }
        p.tuned = true;
    }
    auto enqueue = [&](hipStream_t s) -> hipError_t { return enqueue_v(s, p.variant, nullptr, nullptr); };
    TimedLaunch tl{nullptr, nullptr};
    if (g_timing) {
        ESMF_HIP(hipEventCreate(&tl.start), "hipEventCreate");
        ESMF_HIP(hipEventCreate(&tl.stop), "hipEventCreate");
        ESMF_HIP(hipEventRecord(tl.start, p.stream), "hipEventRecord");
    }
    if (!p.exec && p.stream != nullptr) {
        // capture once; a stream that cannot capture falls back to plain
        // launches (reported by esmf_fock_batched_report)
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(p.stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            hipError_t e = enqueue(p.stream);
            hipError_t ec = hipStreamEndCapture(p.stream, &graph);
            if (e == hipSuccess && ec == hipSuccess && graph) {
                if (hipGraphInstantiate(&p.exec, graph, nullptr, nullptr, 0) != hipSuccess) p.exec = nullptr;
            }
            if (graph) (void)hipGraphDestroy(graph);
        }
        (void)hipGetLastError();
    }
    p.graph = p.exec != nullptr;
    if (p.exec) {
        ESMF_HIP(hipGraphLaunch(p.exec, p.stream), "hipGraphLaunch");
    } else {
        ESMF_HIP(enqueue(p.stream), "batched build");
    }
    ESMF_HIP(hipEventRecord(p.done, p.stream), "batch event");
    p.launched = true;
    if (g_timing) {
        ESMF_HIP(hipEventRecord(tl.stop, p.stream), "hipEventRecord");
        g_timed.push_back(tl);
    }
    esmf_batch_report& r = g_batch_report;
    std::memset(&r, 0, sizeof r);
    r.graph = p.graph ? 1 : 0;
    r.units = p.nunits;
    r.items = p.nitems;
    r.plan = p.variant.plan;
    r.occupancy = p.variant.occupancy;
    r.skip_zero = p.variant.skip_zero_fragments ? 1 : 0;
    r.item_factor = p.item_factor_chosen;
    r.item_candidates = (int32_t)std::min<size_t>(p.item_factor.size(), 4);
    for (int32_t c = 0; c < r.item_candidates; ++c) {
        r.item_factors[c] = p.item_factor[c];
        r.item_ms[c] = p.item_ms[c];
    }
    r.candidates = (int32_t)std::min<size_t>(p.cand.size(), 16);
    for (int32_t c = 0; c < r.candidates; ++c) {
        r.cand_plan[c] = p.cand[c].plan;
        r.cand_occupancy[c] = p.cand[c].occupancy;
        r.cand_skip_zero[c] = p.cand[c].skip_zero_fragments ? 1 : 0;
        r.cand_ms[c] = p.cand_ms[c];
    }
    return ESMF_OK;
}

// drop every cached plan that uses handle h (called on release)
void drop_plans_using(const Handle* h) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    drop_plans_using_locked(h);
}

// the same with g_plan_mu held by the caller
void drop_plans_using_locked(const Handle* h) {
    for (size_t x = 0; x < g_plans.size();) {
        const auto& hs = g_plans[x]->hs;
        if (std::find(hs.begin(), hs.end(), h) != hs.end())
            g_plans.erase(g_plans.begin() + x);
        else
            ++x;
    }
}

esmf_status check_build_args(const Handle* h, int32_t m, const double* d, double* j, double* k,
                             esmf_precision prec) {
    if (!h) return fail(ESMF_ERR_INVALID_ARG, "eri is NULL");
    if (m < 1) return fail(ESMF_ERR_INVALID_ARG, "m must be >= 1");
    if (!d || !j || !k) return fail(ESMF_ERR_INVALID_ARG, "NULL density/output pointer");
    const size_t bytes = sizeof(double) * (size_t)m * h->nbf * h->nbf;
    auto overlap = [bytes](const void* a, const void* b) {
        const char* x = (const char*)a;
        const char* y = (const char*)b;
        return x < y + bytes && y < x + bytes;
    };
    if (overlap(d, j) || overlap(d, k) || overlap(j, k))
        return fail(ESMF_ERR_INVALID_ARG, "d, j and k must not overlap");
    if (prec != ESMF_PREC_FP64 && prec != ESMF_PREC_MIXED && prec != ESMF_PREC_STORE32)
        return fail(ESMF_ERR_INVALID_ARG, "bad precision");
    if (!precision_reads(prec, h->storage))
        return fail(ESMF_ERR_INVALID_ARG,
                    prec == ESMF_PREC_FP64    ? "FP64 builds need ESMF_STORE_FP64 or ESMF_STORE_DIRECT"
                    : prec == ESMF_PREC_MIXED ? "mixed builds read an FP32 or FP64 store (not integral-direct)"
                                              : "STORE32 builds read FP32 storage (prepare with ESMF_STORE_FP32)");
    return ESMF_OK;
}

size_t group_unit_bytes(const Handle& h, int kind) {
    return (operand_bytes(h.ntiles) + partial_bytes(h.plan[kind].nkslots, h.plan[kind].njslots) + 255) / 256 * 256;
}

size_t group_workspace_bytes(const Handle& h, int m, int kind) {
    const size_t G = (size_t)((m + 7) / 8);
    const size_t table = (sizeof(UnitDesc) * G + 255) / 256 * 256;
    const size_t nit = (size_t)h.plan[kind].nitems;
    const size_t items = (sizeof(WorkItem) * G * ((nit + 7) / 8 * 8) + 255) / 256 * 256;
    return table + items + group_unit_bytes(h, kind) * G;
}

// Several builds (any molecules, each with its own m) as one launch sequence
// on one stream: one operand prep over all their density groups, one
// contraction over the concatenation of their work lists (each padded to a
// multiple of 8 items so that every list keeps its XCD grouping), one
// reduction.  Workspace (unit table, item list, per-group operand and
// partial areas) is ws_ext when given (at least group_workspace_bytes summed
// over the entries; the caller keeps it until the sequence has run), else it
// comes from the stream-ordered pool and goes back to it at the end of the
// sequence.  Arguments must have been checked.
esmf_status enqueue_group(const std::vector<GroupEntry>& es, int mode, hipStream_t s, void* ws_ext,
                          size_t ws_ext_bytes) {
    std::vector<UnitDesc> units;
    std::vector<const Handle*> unit_h;
    int64_t prep_total = 0, zero_total = 0, red_total = 0, nitems = 0;
    size_t ws_units = 0;
    const KernelVariant v = default_variant(mode);
    const int kind = v.plan;
    for (const GroupEntry& e : es) {
        const Handle& h = *e.h;
        for (int g = 0; g < (e.m + 7) / 8; ++g) {
            UnitDesc u;
            fill_unit(u, h, kind, mode, e.m, e.d, e.j, e.k, g);
            u.prep_begin = prep_total;
            u.red_begin = (int32_t)red_total;
            u.zero_begin = zero_total;
            prep_total += unit_prep_size(u);
            red_total += h.plan[kind].nred;
            zero_total += unit_zero_size(u);
            nitems += (h.plan[kind].nitems + 7) / 8 * 8;
            ws_units += group_unit_bytes(h, kind);
            units.push_back(u);
            unit_h.push_back(&h);
        }
    }
    if (units.empty()) return ESMF_OK;
    if (nitems > INT32_MAX || red_total > INT32_MAX) return fail(ESMF_ERR_OUT_OF_MEMORY, "group too large");
    const size_t table_bytes = (sizeof(UnitDesc) * units.size() + 255) / 256 * 256;
    const size_t items_bytes = (sizeof(WorkItem) * (size_t)nitems + 255) / 256 * 256;
    const size_t need = table_bytes + items_bytes + ws_units;
    void* ws = ws_ext;
    if (ws_ext) {
        if (ws_ext_bytes < need) return fail(ESMF_ERR_INVALID_ARG, "group workspace too small");
    } else {
        ensure_pool_cached(es[0].h->device);
        if (hipMallocAsync(&ws, need, s) != hipSuccess) {
            // the pool keeps what earlier groups freed: hand that back to the
            // device (once their frees have run) and try once more
            (void)hipGetLastError();
            hipMemPool_t pool;
            if (hipStreamSynchronize(s) != hipSuccess ||
                hipDeviceGetDefaultMemPool(&pool, es[0].h->device) != hipSuccess ||
                hipMemPoolTrimTo(pool, 0) != hipSuccess || hipMallocAsync(&ws, need, s) != hipSuccess) {
                (void)hipGetLastError();
                return fail(ESMF_ERR_OUT_OF_MEMORY, "group workspace");
            }
        }
    }
    UnitDesc* d_units = (UnitDesc*)ws;
    WorkItem* d_items = (WorkItem*)((char*)ws + table_bytes);
    char* area = (char*)ws + table_bytes + items_bytes;
    for (size_t u = 0; u < units.size(); ++u) {
        const Handle& h = *unit_h[u];
        unit_set_workspace(units[u], (double*)area, (double*)(area + operand_bytes(h.ntiles)), h.plan[kind].nkslots);
        area += group_unit_bytes(h, kind);
    }
    hipError_t le = launch_store_units(units.data(), (int)units.size(), d_units, s);
    int64_t at = 0;
    for (size_t u = 0; u < units.size() && le == hipSuccess; ++u) {
        const DevPlan& P = unit_h[u]->plan[kind];
        const int npad = (P.nitems + 7) / 8 * 8;
        le = launch_copy_items((const WorkItem*)P.d_items, P.nitems, d_items + at, npad, (int)u, s);
        at += npad;
    }
    if (le == hipSuccess)
        le = launch_units(d_units, 0, (int)units.size(), prep_total, zero_total, (int)red_total, d_items, (int)nitems,
                          mode, v, s);
    hipError_t fe = ws_ext ? hipSuccess : hipFreeAsync(ws, s);
    if (le != hipSuccess) return device_fail(le, "grouped build");
    if (fe != hipSuccess) return device_fail(fe, "workspace release");
    return ESMF_OK;
}

}  // namespace esmf

extern "C" {

const char* esmf_status_string(esmf_status s) {
    switch (s) {
        case ESMF_OK: return "ESMF_OK";
        case ESMF_ERR_INVALID_ARG: return "ESMF_ERR_INVALID_ARG";
        case ESMF_ERR_OUT_OF_MEMORY: return "ESMF_ERR_OUT_OF_MEMORY";
        case ESMF_ERR_DEVICE: return "ESMF_ERR_DEVICE";
        case ESMF_ERR_NOT_SUPPORTED: return "ESMF_ERR_NOT_SUPPORTED";
    }
    return "ESMF_ERR_UNKNOWN";
}

const char* esmf_last_error(void) { return g_last_error.c_str(); }

esmf_status esmf_nine_densities(int32_t nbf, int32_t n_occ, int32_t n_virt, const double* theta,
                                const double* gamma, const double* sigma, const double* mu,
                                const double* r, const double* phi, double* d, void* hip_stream) {
    g_last_error.clear();
    if (nbf < 1 || n_occ < 1 || n_virt < 1) return fail(ESMF_ERR_INVALID_ARG, "nbf, n_occ and n_virt must be >= 1");
    if (nbf > (1 << 15) || n_occ > (1 << 15) || n_virt > (1 << 15))
        return fail(ESMF_ERR_INVALID_ARG, "sizes too large (max 32768)");
    if (!theta || !gamma || !sigma || !mu || !r || !phi || !d) return fail(ESMF_ERR_INVALID_ARG, "NULL pointer");
    const size_t dbytes = sizeof(double) * 9 * (size_t)nbf * nbf;
    const size_t ins[6] = {(size_t)n_occ * nbf, (size_t)n_virt * nbf, (size_t)n_occ * n_virt,
                           (size_t)n_occ * n_virt, (size_t)n_occ * nbf, (size_t)n_virt * nbf};
    const double* inp[6] = {theta, gamma, sigma, mu, r, phi};
    for (int x = 0; x < 6; ++x) {
        const char* a = (const char*)inp[x];
        const char* b = (const char*)d;
        if (a < b + dbytes && b < a + sizeof(double) * ins[x])
            return fail(ESMF_ERR_INVALID_ARG, "d must not overlap the inputs");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    void* work = nullptr;
    const size_t wbytes = sizeof(double) * nine_densities_work_doubles(nbf, n_occ);
    if (small_scratch_alloc(&work, wbytes, s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ESMF_ERR_OUT_OF_MEMORY, "density scratch");
    }
    const hipError_t le = launch_nine_densities(nbf, n_occ, n_virt, theta, gamma, sigma, mu, r, phi, d,
                                                (double*)work, s);
    const hipError_t fe = hipFreeAsync(work, s);
    if (le != hipSuccess) return device_fail(le, "nine densities");
    if (fe != hipSuccess) return device_fail(fe, "density scratch release");
    return ESMF_OK;
}

esmf_status esmf_energy_two_body(int32_t nbf, double n2, double c0, const double* d, const double* j,
                                 const double* k, double* e2, void* hip_stream) {
    g_last_error.clear();
    if (nbf < 1 || nbf > (1 << 15)) return fail(ESMF_ERR_INVALID_ARG, "nbf must be in 1..32768");
    if (!d || !j || !k || !e2) return fail(ESMF_ERR_INVALID_ARG, "NULL pointer");
    if (!std::isfinite(n2) || !std::isfinite(c0)) return fail(ESMF_ERR_INVALID_ARG, "n2 and c0 must be finite");
    {
        const size_t nn = sizeof(double) * (size_t)nbf * nbf;
        const char* o = (const char*)e2;
        const char* in[3] = {(const char*)d, (const char*)j, (const char*)k};
        const size_t len[3] = {3 * nn, 2 * nn, 2 * nn};
        for (int x = 0; x < 3; ++x)
            if (o < in[x] + len[x] && in[x] < o + sizeof(double))
                return fail(ESMF_ERR_INVALID_ARG, "e2 must not overlap d, j or k");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    void* part = nullptr;
    if (small_scratch_alloc(&part, sizeof(double) * energy_partial_doubles(), s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ESMF_ERR_OUT_OF_MEMORY, "energy scratch");
    }
    const hipError_t le = launch_energy_two_body(nbf, n2, c0, d, j, k, e2, (double*)part, s);
    const hipError_t fe = hipFreeAsync(part, s);
    if (le != hipSuccess) return device_fail(le, "two-body energy");
    if (fe != hipSuccess) return device_fail(fe, "energy scratch release");
    return ESMF_OK;
}

esmf_status esmf_energy_gradient(int32_t nbf, int32_t n_occ, int32_t n_virt, double c0, double n2,
                                 const double* theta, const double* gamma, const double* sigma, const double* g,
                                 const double* d, const double* j, const double* k, double* energy,
                                 double* d_sigma, double* d_theta, double* d_gamma, void* hip_stream) {
    g_last_error.clear();
    if (nbf < 1 || n_occ < 1 || n_virt < 1) return fail(ESMF_ERR_INVALID_ARG, "nbf, n_occ and n_virt must be >= 1");
    if (nbf > (1 << 15) || n_occ > (1 << 15) || n_virt > (1 << 15))
        return fail(ESMF_ERR_INVALID_ARG, "sizes too large (max 32768)");
    if (!theta || !gamma || !sigma || !g || !d || !j || !k || !energy || !d_sigma || !d_theta || !d_gamma)
        return fail(ESMF_ERR_INVALID_ARG, "NULL pointer");
    if (!std::isfinite(c0) || !std::isfinite(n2) || !(n2 > 0.0))
        return fail(ESMF_ERR_INVALID_ARG, "c0 must be finite and n2 finite and > 0");
    // the outputs must not overlap each other or the inputs
    const size_t nn = (size_t)nbf * nbf;
    struct R {
        const char* p;
        size_t n;
    };
    const R outs[4] = {{(const char*)energy, 4 * sizeof(double)},
                       {(const char*)d_sigma, sizeof(double) * n_occ * n_virt},
                       {(const char*)d_theta, sizeof(double) * n_occ * nbf},
                       {(const char*)d_gamma, sizeof(double) * n_virt * nbf}};
    const R all[11] = {outs[0], outs[1], outs[2], outs[3],
                       {(const char*)theta, sizeof(double) * n_occ * nbf},
                       {(const char*)gamma, sizeof(double) * n_virt * nbf},
                       {(const char*)sigma, sizeof(double) * n_occ * n_virt},
                       {(const char*)g, sizeof(double) * nn},
                       {(const char*)d, 3 * sizeof(double) * nn},
                       {(const char*)j, 3 * sizeof(double) * nn},
                       {(const char*)k, 3 * sizeof(double) * nn}};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 11; ++b)
            if (a != b && all[a].p < all[b].p + all[b].n && all[b].p < all[a].p + all[a].n)
                return fail(ESMF_ERR_INVALID_ARG, "outputs must not overlap each other or the inputs");
    hipStream_t s = (hipStream_t)hip_stream;
    void* work = nullptr;
    if (small_scratch_alloc(&work, sizeof(double) * gradient_work_doubles(nbf, n_occ), s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ESMF_ERR_OUT_OF_MEMORY, "gradient scratch");
    }
    const hipError_t le = launch_energy_gradient(nbf, n_occ, n_virt, c0, n2, theta, gamma, sigma, g, d, j, k,
                                                 energy, d_sigma, d_theta, d_gamma, (double*)work, s);
    const hipError_t fe = hipFreeAsync(work, s);
    if (le != hipSuccess) return device_fail(le, "energy gradient");
    if (fe != hipSuccess) return device_fail(fe, "gradient scratch release");
    return ESMF_OK;
}

esmf_status esmf_timing_enable(int32_t enable) {
    g_last_error.clear();
    g_timing = enable != 0;
    return ESMF_OK;
}

esmf_status esmf_timing_collect(double* total_ms, int64_t* launches) {
    g_last_error.clear();
    if (!total_ms || !launches) return fail(ESMF_ERR_INVALID_ARG, "NULL argument");
    double tot = 0.0;
    esmf_status st = ESMF_OK;
    for (auto& t : g_timed) {
        float ms = 0.0f;
        if (st == ESMF_OK) {
            hipError_t e = hipEventSynchronize(t.stop);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
            if (e != hipSuccess) st = device_fail(e, "timing events");
        }
        tot += ms;
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    *total_ms = tot;
    *launches = (int64_t)g_timed.size();
    g_timed.clear();
    return st;
}

esmf_status esmf_eri_prepare(int32_t nbf, const double* centers, const double* exponents,
                             double schwarz_tau, esmf_storage storage, void* hip_stream,
                             esmf_eri_t* out) {
    g_last_error.clear();
    return prepare_impl(nbf, centers, exponents, schwarz_tau, storage, hip_stream, -1, nullptr, out);
}

esmf_status esmf_eri_prepare_cart(int32_t nbf, const double* centers, const double* exponents,
                                  const int32_t* lmn, double schwarz_tau, esmf_storage storage,
                                  void* hip_stream, esmf_eri_t* out) {
    g_last_error.clear();
    if (!lmn) return fail(ESMF_ERR_INVALID_ARG, "lmn is NULL");
    return prepare_impl(nbf, centers, exponents, schwarz_tau, storage, hip_stream, -1, nullptr, out, lmn);
}

esmf_status esmf_eri_prepare_contracted(int32_t nbf, const double* centers, const int32_t* lmn,
                                        const int32_t* prim_offset, const double* prim_exp,
                                        const double* prim_coef, double schwarz_tau, esmf_storage storage,
                                        void* hip_stream, esmf_eri_t* out) {
    g_last_error.clear();
    if (!out) return fail(ESMF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::vector<double> emin;
    const esmf_status st = check_contraction(nbf, lmn, prim_offset, prim_exp, prim_coef, emin);
    if (st != ESMF_OK) return st;
    return prepare_impl(nbf, centers, emin.data(), schwarz_tau, storage, hip_stream, -1, nullptr, out, lmn,
                        prim_offset, prim_exp, prim_coef);
}

}  // extern "C"

// Arguments of a contracted basis; emin receives each function's most
// diffuse exponent (by which the tile plan groups functions).
esmf_status esmf::check_contraction(int32_t nbf, const int32_t* lmn, const int32_t* prim_offset,
                                    const double* prim_exp, const double* prim_coef, std::vector<double>& emin) {
    if (nbf < 1 || nbf > (1 << 15)) return fail(ESMF_ERR_INVALID_ARG, "nbf must be in 1..32768");
    if (!lmn || !prim_offset || !prim_exp || !prim_coef) return fail(ESMF_ERR_INVALID_ARG, "NULL array");
    if (prim_offset[0] != 0) return fail(ESMF_ERR_INVALID_ARG, "prim_offset[0] must be 0");
    for (int f = 0; f < nbf; ++f) {
        const int k = prim_offset[f + 1] - prim_offset[f];
        if (k < 1 || k > kMaxPrimitives)
            return fail(ESMF_ERR_INVALID_ARG, "each function needs 1..16 primitives");
    }
    emin.assign(nbf, 0.0);
    for (int f = 0; f < nbf; ++f) {
        double e = 1e300;
        for (int k = prim_offset[f]; k < prim_offset[f + 1]; ++k) {
            if (!std::isfinite(prim_exp[k]) || !(prim_exp[k] > 0.0) || !std::isfinite(prim_coef[k]))
                return fail(ESMF_ERR_INVALID_ARG, "primitive exponents must be finite and > 0, coefficients finite");
            e = std::min(e, prim_exp[k]);
        }
        emin[f] = e;
    }
    return ESMF_OK;
}

// Device arrays of a work plan (items, slot ranges, reduction pairs; the
// entry records are sized here and filled by fill_plan_records).
esmf_status esmf::alloc_plan(DevPlan& P, const WorkPlan& w, int64_t ntargets, hipStream_t s) {
    P.kind = w.kind;
    P.seg = w.seg;
    P.band = w.band;
    P.nitems = (int32_t)w.items.size();
    P.items = w.items;
    P.nentries = (int64_t)w.entries.size();
    P.ntargets = ntargets;
    P.nkslots = w.nkslots;
    P.njslots = w.njslots;
    P.nred = (int32_t)w.red.size();
    auto dalloc = [](void** p, size_t bytes) {
        if (hipMalloc(p, std::max<size_t>(bytes, 1)) != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return false;
        }
        return true;
    };
    if (!dalloc(&P.d_items, sizeof(WorkItem) * std::max<size_t>(w.items.size(), 1)) ||
        !dalloc((void**)&P.d_rec, sizeof(EntryRecord) * std::max<size_t>(w.entries.size(), 1)) ||
        !dalloc((void**)&P.d_kptr, sizeof(int64_t) * w.kptr.size()) ||
        !dalloc((void**)&P.d_jptr, sizeof(int64_t) * w.jptr.size()) ||
        !dalloc((void**)&P.d_red, sizeof(int32_t) * std::max<size_t>(w.red.size(), 1)))
        return fail(ESMF_ERR_OUT_OF_MEMORY, "work plan allocation");
    if (!w.items.empty())
        ESMF_HIP(hipMemcpyAsync(P.d_items, w.items.data(), sizeof(WorkItem) * w.items.size(), hipMemcpyHostToDevice, s),
                 "copy items");
    ESMF_HIP(hipMemcpyAsync(P.d_kptr, w.kptr.data(), sizeof(int64_t) * w.kptr.size(), hipMemcpyHostToDevice, s),
             "copy kptr");
    ESMF_HIP(hipMemcpyAsync(P.d_jptr, w.jptr.data(), sizeof(int64_t) * w.jptr.size(), hipMemcpyHostToDevice, s),
             "copy jptr");
    if (!w.red.empty())
        ESMF_HIP(hipMemcpyAsync(P.d_red, w.red.data(), sizeof(int32_t) * w.red.size(), hipMemcpyHostToDevice, s),
                 "copy reduction pairs");
    return ESMF_OK;
}

// Entry records of a plan from its entries' blocks and partial slots (the
// block arrays and granule offsets of the handle must be on the device).
esmf_status esmf::fill_plan_records(const Handle& h, DevPlan& P, const WorkPlan& w, hipStream_t s) {
    if (w.entries.empty()) return ESMF_OK;
    DevBuf<int32_t> des, den;
    if (des.alloc(w.eslot.size()) || den.alloc(w.entries.size())) return fail(ESMF_ERR_OUT_OF_MEMORY, "entry slots");
    ESMF_HIP(hipMemcpyAsync(des.p, w.eslot.data(), sizeof(int32_t) * w.eslot.size(), hipMemcpyHostToDevice, s),
             "copy entry slots");
    ESMF_HIP(hipMemcpyAsync(den.p, w.entries.data(), sizeof(int32_t) * w.entries.size(), hipMemcpyHostToDevice, s),
             "copy entries");
    ESMF_HIP(launch_build_records((int64_t)w.entries.size(), den.p, h.d_blk_tiles, h.d_blk_mask, h.d_blk_off, des.p,
                                  P.d_rec, s), "build_records");
    ESMF_HIP(hipStreamSynchronize(s), "sync build_records");
    return ESMF_OK;
}

// Cut the handle's work plan of `kind` again with items of `seg` blocks
// (the tuners' work-item length).  Waits for the handle's builds, drops the
// batched plans that use the handle, and replaces the plan's device arrays;
// must not run while builds of the handle are being enqueued.
esmf_status esmf::recut_plan(Handle& h, int kind, int seg, hipStream_t s, bool plans_locked) {
    if (h.plan[kind].seg == seg) return ESMF_OK;
    BlockList bl;
    bl.nbf = h.nbf;
    bl.nslots = h.nslots;
    bl.ntiles = h.ntiles;
    bl.slot_fn = h.slot_fn;
    bl.blk_tiles = h.blk_tiles;
    bl.weight = h.weight;
    WorkPlan w;
    const int xcd = env_int("ESMF_XCD_ORDER", 1) ? 8 : 1;
    const int band = h.plan[kind].band > 0 ? h.plan[kind].band : fused_band();
    if (plan_work(bl, kind, seg, band, xcd, w) != 0)
        return fail(ESMF_ERR_OUT_OF_MEMORY, "too many partial slots");
    DevPlan fresh;
    esmf_status st = alloc_plan(fresh, w, (int64_t)h.ntiles * h.ntiles, s);
    if (st == ESMF_OK) st = fill_plan_records(h, fresh, w, s);
    if (st != ESMF_OK) {
        fresh.release();
        return st;
    }
    // nothing may still read the old arrays
    {
        std::lock_guard<std::mutex> lk(h.ws_mu);
        if (h.ws_done && h.ws_used) ESMF_HIP(hipEventSynchronize(h.ws_done), "previous builds");
    }
    if (plans_locked)
        drop_plans_using_locked(&h);
    else
        drop_plans_using(&h);
    ESMF_HIP(hipStreamSynchronize(s), "plan cut");
    h.plan[kind].release();
    h.plan[kind] = std::move(fresh);
    return ESMF_OK;
}

// Prepare with an optional cap on the handle's device footprint: when
// byte_limit >= 0 and the store would need more, nothing stays allocated and
// ESMF_ERR_OUT_OF_MEMORY is returned; *footprint (if given) receives the
// footprint either way once it is known (0 if it never was).
esmf_status esmf::prepare_impl(int32_t nbf, const double* centers, const double* exponents,
                               double schwarz_tau, esmf_storage storage, void* hip_stream,
                               int64_t byte_limit, int64_t* footprint, esmf_eri_t* out,
                               const int32_t* lmn, const int32_t* poff, const double* pexp,
                               const double* pcoef) {
    if (footprint) *footprint = 0;
    if (!out) return fail(ESMF_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nbf < 1) return fail(ESMF_ERR_INVALID_ARG, "nbf must be >= 1");
    if (nbf > (1 << 15)) return fail(ESMF_ERR_INVALID_ARG, "nbf too large (max 32768)");
    if (!centers || !exponents) return fail(ESMF_ERR_INVALID_ARG, "centers/exponents NULL");
    if (!finite_all(centers, 3 * (size_t)nbf)) return fail(ESMF_ERR_INVALID_ARG, "non-finite centre");
    for (int i = 0; i < nbf; ++i)
        if (!std::isfinite(exponents[i]) || !(exponents[i] > 0.0))
            return fail(ESMF_ERR_INVALID_ARG, "exponents must be finite and > 0");
    if (!std::isfinite(schwarz_tau) || schwarz_tau < 0.0)
        return fail(ESMF_ERR_INVALID_ARG, "schwarz_tau must be finite and >= 0");
    if (storage != ESMF_STORE_FP64 && storage != ESMF_STORE_FP32 && storage != ESMF_STORE_DIRECT)
        return fail(ESMF_ERR_INVALID_ARG, "bad storage");
    const bool direct = storage == ESMF_STORE_DIRECT;
    // Cartesian functions: (l, m, n) >= 0 with l + m + n <= 2 (s, p, d), each
    // a contraction of primitives (one primitive of coefficient 1 unless
    // poff / pexp / pcoef are given)
    bool cart = false;
    std::vector<int32_t> c_off;
    std::vector<double> c_exp, c_coef;
    if (lmn) {
        for (int i = 0; i < nbf; ++i) {
            const int32_t* l = lmn + 3 * (size_t)i;
            if (l[0] < 0 || l[1] < 0 || l[2] < 0 || l[0] + l[1] + l[2] > 2)
                return fail(ESMF_ERR_INVALID_ARG, "lmn: each function needs l, m, n >= 0 and l + m + n <= 2");
            cart = cart || (l[0] | l[1] | l[2]) != 0;
        }
        c_off.resize(nbf + 1);
        if (poff) {
            for (int i = 0; i <= nbf; ++i) c_off[i] = poff[i];
            for (int i = 0; i < nbf; ++i) {
                cart = cart || c_off[i + 1] - c_off[i] > 1;
                // normalisation of the contraction over normalised primitives:
                // <g_a|g_b> = (2 sqrt(ab) / (a + b))^(L + 3/2) for one centre
                // and one set of powers
                const int32_t* l = lmn + 3 * (size_t)i;
                const double Lh = l[0] + l[1] + l[2] + 1.5;
                double ss = 0.0;
                for (int a = c_off[i]; a < c_off[i + 1]; ++a)
                    for (int b = c_off[i]; b < c_off[i + 1]; ++b)
                        ss += pcoef[a] * pcoef[b] *
                              std::pow(2.0 * std::sqrt(pexp[a] * pexp[b]) / (pexp[a] + pexp[b]), Lh);
                if (!(ss > 0.0) || !std::isfinite(ss))
                    return fail(ESMF_ERR_INVALID_ARG, "a contraction has zero or non-finite norm");
                const double nf = 1.0 / std::sqrt(ss);
                for (int a = c_off[i]; a < c_off[i + 1]; ++a) {
                    c_exp.push_back(pexp[a]);
                    c_coef.push_back(nf * pcoef[a]);
                    // a single normalised primitive has coefficient c / |c|,
                    // +-1 up to rounding; the s-type fill takes it as +1, so
                    // a negative one needs the general fill
                    cart = cart || c_coef.back() < 0.0;
                }
            }
        } else {
            for (int i = 0; i <= nbf; ++i) c_off[i] = i;
            c_exp.assign(exponents, exponents + nbf);
            c_coef.assign(nbf, 1.0);
        }
    }
    if (cart && direct)
        return fail(ESMF_ERR_NOT_SUPPORTED, "integral-direct builds take one-primitive s functions of positive coefficient only");
    hipStream_t s = (hipStream_t)hip_stream;

    std::unique_ptr<Handle, void (*)(Handle*)> h(new (std::nothrow) Handle, free_handle);
    if (!h) return fail(ESMF_ERR_OUT_OF_MEMORY, "host allocation");
    ESMF_HIP(hipGetDevice(&h->device), "hipGetDevice");
    h->nbf = nbf;
    h->tau = schwarz_tau;
    h->storage = storage;
    h->slot_fn = make_tile_plan(nbf, centers, exponents);
    h->nslots = (int32_t)h->slot_fn.size();
    h->ntiles = h->nslots / kTile;
    if (h->ntiles > kMaxTiles) return fail(ESMF_ERR_INVALID_ARG, "too many tiles (the limit is 8191)");
    h->fn_slot.assign(nbf, -1);
    for (int s2 = 0; s2 < h->nslots; ++s2)
        if (h->slot_fn[s2] >= 0) h->fn_slot[h->slot_fn[s2]] = s2;

    const int ns = h->nslots;
    const size_t nss = (size_t)ns * ns;
    // device inputs and pair quantities (temporary)
    DevBuf<double> dc, da, pz, px, py, pzc, pe, pq;
    DevBuf<int32_t> dsf;
    if (dc.alloc(3 * (size_t)nbf) || da.alloc(nbf) || dsf.alloc(ns) || pz.alloc(nss) ||
        px.alloc(nss) || py.alloc(nss) || pzc.alloc(nss) || pe.alloc(nss) || pq.alloc(nss))
        return fail(ESMF_ERR_OUT_OF_MEMORY, "pair buffers");
    ESMF_HIP(hipMemcpyAsync(dc.p, centers, sizeof(double) * 3 * nbf, hipMemcpyHostToDevice, s), "copy centers");
    ESMF_HIP(hipMemcpyAsync(da.p, exponents, sizeof(double) * nbf, hipMemcpyHostToDevice, s), "copy exponents");
    ESMF_HIP(hipMemcpyAsync(dsf.p, h->slot_fn.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s), "copy slots");
    ESMF_HIP(launch_pair_build(ns, dsf.p, dc.p, da.p, pz.p, px.p, py.p, pzc.p, pe.p, pq.p, s), "pair_build");
    DevBuf<int8_t> dl;
    DevBuf<int32_t> dpo;
    DevBuf<double> dpe, dpc;
    if (cart) {
        std::vector<int8_t> l8(3 * (size_t)nbf);
        for (size_t i = 0; i < l8.size(); ++i) l8[i] = (int8_t)lmn[i];
        if (dl.alloc(l8.size()) || dpo.alloc(c_off.size()) || dpe.alloc(c_exp.size()) || dpc.alloc(c_coef.size()))
            return fail(ESMF_ERR_OUT_OF_MEMORY, "basis buffers");
        ESMF_HIP(hipMemcpy(dl.p, l8.data(), l8.size(), hipMemcpyHostToDevice), "copy lmn");
        ESMF_HIP(hipMemcpy(dpo.p, c_off.data(), sizeof(int32_t) * c_off.size(), hipMemcpyHostToDevice), "copy offsets");
        ESMF_HIP(hipMemcpy(dpe.p, c_exp.data(), sizeof(double) * c_exp.size(), hipMemcpyHostToDevice), "copy exponents");
        ESMF_HIP(hipMemcpy(dpc.p, c_coef.data(), sizeof(double) * c_coef.size(), hipMemcpyHostToDevice), "copy coefficients");
        ESMF_HIP(launch_cart_pair_q(ns, dsf.p, dc.p, dl.p, dpo.p, dpe.p, dpc.p, pq.p, s), "cart Schwarz factors");
    }
    std::vector<double> Q(nss);
    ESMF_HIP(hipMemcpyAsync(Q.data(), pq.p, sizeof(double) * nss, hipMemcpyDeviceToHost, s), "copy Q");
    ESMF_HIP(hipStreamSynchronize(s), "sync pair_build");

    // pair and quartet statistics (exact, over function pairs)
    double qmax = 0.0;
    for (size_t i = 0; i < nss; ++i) qmax = std::max(qmax, Q[i]);
    h->q_max = qmax;
    std::vector<double> qp;
    qp.reserve((size_t)nbf * (nbf + 1) / 2);
    for (int a = 0; a < ns; ++a) {
        if (h->slot_fn[a] < 0) continue;
        for (int b = 0; b < ns; ++b) {
            if (h->slot_fn[b] < 0) continue;
            if (h->slot_fn[b] > h->slot_fn[a]) continue;  // p >= q once
            qp.push_back(Q[(size_t)a * ns + b]);
        }
    }
    int64_t kept = 0;
    for (double v : qp)
        if (v * qmax > schwarz_tau) ++kept;
    h->npairs_kept = kept;
    {
        std::vector<double> sq(qp);
        std::sort(sq.begin(), sq.end());
        int64_t ordered = 0, diag = 0;
        for (double v : sq) {
            if (v * v > schwarz_tau) ++diag;
            // partners w with v * w > tau: the sorted suffix above tau / v
            // (found by the predicate itself, so decisions match exactly)
            size_t lo = 0, hi = sq.size();
            while (lo < hi) {
                size_t mid = (lo + hi) / 2;
                if (v * sq[mid] > schwarz_tau) hi = mid; else lo = mid + 1;
            }
            ordered += (int64_t)(sq.size() - lo);
        }
        h->nquartets_kept = (ordered + diag) / 2;
    }

    // the block list and the two work plans (host, plan.cpp)
    BlockList bl;
    plan_blocks(Q, h->slot_fn, schwarz_tau, bl);
    h->nblocks = bl.nblocks();
    if (h->nblocks > INT32_MAX / 2) return fail(ESMF_ERR_OUT_OF_MEMORY, "too many blocks");
    const int xcd = env_int("ESMF_XCD_ORDER", 1) ? 8 : 1;
    const int seg_env = env_int("ESMF_ITEM_BLOCKS", 0);  // override of the item length, for comparisons
    WorkPlan wp[2];
    {
        // the two plans are independent: the fused one on a second thread
        int rc[2] = {0, 0};
        const int band = fused_band();
        auto make = [&](int kind) {
            const int seg = seg_env > 0 ? seg_env : default_item_blocks(kind, h->nblocks);
            rc[kind] = plan_work(bl, kind, seg, band, xcd, wp[kind]);
        };
        std::thread other;
        try {
            other = std::thread(make, 1);
        } catch (const std::exception&) {
            make(1);  // no thread available: one after the other
        }
        make(0);
        if (other.joinable()) other.join();
        for (int kind = 0; kind < 2; ++kind) {
            if (rc[kind] != 0) return fail(ESMF_ERR_OUT_OF_MEMORY, "too many partial slots");
            if ((int64_t)wp[kind].items.size() > INT32_MAX / 2)
                return fail(ESMF_ERR_OUT_OF_MEMORY, "too many work items");
        }
    }
    h->blk_tiles = std::move(bl.blk_tiles);
    h->weight = std::move(bl.weight);
    const std::vector<int32_t>& bt = h->blk_tiles;
    const std::vector<int32_t>& used = wp[0].used;   // the same for both plans
    h->nused = (int32_t)used.size();
    const int64_t ntargets = (int64_t)h->ntiles * h->ntiles;
    const size_t esz = storage == ESMF_STORE_FP64 ? sizeof(double) : sizeof(float);
    const size_t nb = (size_t)std::max<int64_t>(h->nblocks, 1);
    auto dalloc = [](void** p, size_t bytes) {
        if (hipMalloc(p, std::max<size_t>(bytes, 1)) != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return false;
        }
        return true;
    };
    if (!dalloc((void**)&h->d_blk_tiles, sizeof(int32_t) * std::max<size_t>(bt.size(), 1)) ||
        !dalloc((void**)&h->d_slot_fn, sizeof(int32_t) * ns) ||
        !dalloc((void**)&h->d_blk_mask, sizeof(uint64_t) * 4 * nb) ||
        !dalloc((void**)&h->d_blk_off, sizeof(int64_t) * nb) ||
        !dalloc((void**)&h->d_used, sizeof(int32_t) * std::max<size_t>(used.size(), 1)))
        return fail(ESMF_ERR_OUT_OF_MEMORY, "block list allocation");
    for (int kind = 0; kind < 2; ++kind) {
        const esmf_status st = alloc_plan(h->plan[kind], wp[kind], ntargets, s);
        if (st != ESMF_OK) return st;
    }
    ESMF_HIP(hipMemcpyAsync(h->d_blk_tiles, bt.data(), sizeof(int32_t) * bt.size(), hipMemcpyHostToDevice, s), "copy blocks");
    ESMF_HIP(hipMemcpyAsync(h->d_slot_fn, h->slot_fn.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, s), "copy slots");
    if (!used.empty())
        ESMF_HIP(hipMemcpyAsync(h->d_used, used.data(), sizeof(int32_t) * used.size(), hipMemcpyHostToDevice, s), "copy used pairs");
    // granule presence and per-block counts, then offsets by a host prefix sum
    std::vector<int64_t> off(nb, 0);
    if (h->nblocks > 0) {
        DevBuf<int32_t> dcnt;
        if (dcnt.alloc(nb)) return fail(ESMF_ERR_OUT_OF_MEMORY, "granule counts");
        ESMF_HIP(launch_granule_mask(h->nblocks, h->d_blk_tiles, ns, pq.p, schwarz_tau, h->d_blk_mask,
                                     dcnt.p, s), "granule_mask");
        std::vector<int32_t> cnt(nb);
        ESMF_HIP(hipMemcpyAsync(cnt.data(), dcnt.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s), "copy counts");
        ESMF_HIP(hipStreamSynchronize(s), "sync granule_mask");
        // each block's granules are padded with zero granules to a multiple
        // of 16 (rows of 256 values), so the contraction loads whole rows;
        // integral-direct handles store nothing and record the block index
        int64_t acc = 0;
        for (size_t b = 0; b < (size_t)h->nblocks; ++b) {
            off[b] = direct ? (int64_t)b : acc;
            acc += (cnt[b] + kGranuleRow - 1) / kGranuleRow * kGranuleRow;
        }
        h->ngranules = direct ? 0 : acc;
        h->ngranules_fp64 = acc;
    }
    const size_t store_bytes = direct ? sizeof(double) * (kDirectArrays * nss + nb)
                                      : (size_t)h->ngranules * kGranule * esz;
    h->device_bytes = (int64_t)(store_bytes + sizeof(int32_t) * (bt.size() + ns + used.size()) +
                                (sizeof(uint64_t) * 4 + sizeof(int64_t)) * nb) +
                      h->plan[0].device_bytes() + h->plan[1].device_bytes();
    if (footprint) *footprint = h->device_bytes;
    if (byte_limit >= 0 && h->device_bytes > byte_limit) {
        char msg[160];
        snprintf(msg, sizeof msg, "integral store needs %.3f GB, budget left %.3f GB",
                 h->device_bytes / 1e9, byte_limit / 1e9);
        return fail(ESMF_ERR_OUT_OF_MEMORY, msg);
    }
    size_t free_b = 0, total_b = 0;
    ESMF_HIP(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if (store_bytes + ((size_t)64 << 20) > free_b) {
        char msg[160];
        snprintf(msg, sizeof msg, "block store needs %.2f GB, %.2f GB free", store_bytes / 1e9,
                 free_b / 1e9);
        return fail(ESMF_ERR_OUT_OF_MEMORY, msg);
    }
    if (!dalloc(&h->d_vals, store_bytes)) return fail(ESMF_ERR_OUT_OF_MEMORY, "block store allocation");
    // the s-type fill writes every slot of the store, row padding included;
    // the Cartesian fill writes the kept granules only
    if (store_bytes > 0 && cart) ESMF_HIP(hipMemsetAsync(h->d_vals, 0, store_bytes, s), "clear block store");
    ESMF_HIP(hipMemcpyAsync(h->d_blk_off, off.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, s), "copy offsets");
    for (int kind = 0; kind < 2; ++kind) {
        const esmf_status st = fill_plan_records(*h, h->plan[kind], wp[kind], s);
        if (st != ESMF_OK) return st;
    }
    if (direct) {
        // integral-direct data: the pair arrays and the block weights
        double* dd = (double*)h->d_vals;
        const double* src[kDirectArrays] = {pz.p, px.p, py.p, pzc.p, pe.p, pq.p};
        for (int a = 0; a < kDirectArrays; ++a)
            ESMF_HIP(hipMemcpyAsync(dd + a * nss, src[a], sizeof(double) * nss, hipMemcpyDeviceToDevice, s),
                     "copy pair data");
        if (!h->weight.empty())
            ESMF_HIP(hipMemcpyAsync(dd + kDirectArrays * nss, h->weight.data(), sizeof(double) * h->weight.size(),
                                    hipMemcpyHostToDevice, s), "copy weights");
        ESMF_HIP(hipStreamSynchronize(s), "sync direct data");
        *out = (esmf_eri_t)h.release();
        return ESMF_OK;
    }
    DevBuf<double> dw;
    if (dw.alloc(h->weight.size())) return fail(ESMF_ERR_OUT_OF_MEMORY, "weights");
    ESMF_HIP(hipMemcpyAsync(dw.p, h->weight.data(), sizeof(double) * h->weight.size(), hipMemcpyHostToDevice, s), "copy weights");
    if (h->nblocks > 0 && cart)
        ESMF_HIP(launch_eri_fill_cart(h->nblocks, h->d_blk_tiles, dw.p, h->d_blk_mask, h->d_blk_off, ns,
                                      pz.p, px.p, py.p, pzc.p, pe.p, pq.p, schwarz_tau, dsf.p, dc.p, dl.p, dpo.p,
                                      dpe.p, dpc.p, h->d_vals, storage == ESMF_STORE_FP32, s),
                 "eri_fill_cart");
    else if (h->nblocks > 0)
        ESMF_HIP(launch_eri_fill(h->nblocks, h->d_blk_tiles, dw.p, h->d_blk_mask, h->d_blk_off, ns,
                                 pz.p, px.p, py.p, pzc.p, pe.p, pq.p, schwarz_tau, h->d_vals,
                                 storage == ESMF_STORE_FP32, s),
                 "eri_fill");
    ESMF_HIP(hipStreamSynchronize(s), "sync eri_fill");
    *out = (esmf_eri_t)h.release();
    return ESMF_OK;
}

extern "C" {

esmf_status esmf_eri_info_get(esmf_eri_t eri, esmf_eri_info* out) {
    g_last_error.clear();
    if (!eri || !out) return fail(ESMF_ERR_INVALID_ARG, "NULL argument");
    const Handle* h = (const Handle*)eri;
    std::memset(out, 0, sizeof *out);
    out->nbf = h->nbf;
    out->tile = kTile;
    out->npairs = (int64_t)h->nbf * (h->nbf + 1) / 2;
    out->npairs_kept = h->npairs_kept;
    out->nquartets_kept = h->nquartets_kept;
    out->nblocks = h->nblocks;
    out->nelements_stored = h->ngranules * (int64_t)kGranule;
    out->device_bytes = h->device_bytes;
    {
        // a group of up to 8 densities on the default plan of the store's FP64
        // or (FP32 store) STORE32 builds
        const int kind = default_variant(h->storage == ESMF_STORE_DIRECT ? 3 : h->storage == ESMF_STORE_FP32 ? 2 : 0)
                             .plan;
        for (int x = 0; x < 2; ++x)
            out->workspace_bytes_plan[x] =
                (int64_t)(operand_bytes(h->ntiles) + partial_bytes(h->plan[x].nkslots, h->plan[x].njslots));
        out->workspace_bytes = out->workspace_bytes_plan[kind];
    }
    out->fp64_store_bytes = h->ngranules_fp64 * (int64_t)kGranule * (int64_t)sizeof(double);
    out->q_max = h->q_max;
    out->tau = h->tau;
    out->storage = h->storage;
    return ESMF_OK;
}

esmf_status esmf_eri_release(esmf_eri_t eri) {
    g_last_error.clear();
    if (eri) drop_plans_using((const Handle*)eri);
    free_handle((Handle*)eri);
    return ESMF_OK;
}

esmf_status esmf_eri_lookup(esmf_eri_t eri, int64_t count, const int32_t* p, const int32_t* q,
                            const int32_t* r, const int32_t* s, double* out) {
    g_last_error.clear();
    if (!eri) return fail(ESMF_ERR_INVALID_ARG, "eri is NULL");
    if (count < 0) return fail(ESMF_ERR_INVALID_ARG, "count < 0");
    if (count == 0) return ESMF_OK;
    if (!p || !q || !r || !s || !out) return fail(ESMF_ERR_INVALID_ARG, "NULL array");
    const Handle* h = (const Handle*)eri;
    for (int64_t t = 0; t < count; ++t) {
        int32_t f[4] = {p[t], q[t], r[t], s[t]};
        for (int x = 0; x < 4; ++x)
            if (f[x] < 0 || f[x] >= h->nbf) return fail(ESMF_ERR_INVALID_ARG, "index out of range");
    }
    if (h->storage == ESMF_STORE_DIRECT)
        return fail(ESMF_ERR_NOT_SUPPORTED, "an integral-direct handle stores no integrals");
    // canonical tile-pair index of (I, J), I >= J
    auto tp_index = [](int I, int J) { return (int64_t)I * (I + 1) / 2 + J; };
    std::vector<int64_t> blk_key(h->nblocks);
    for (int64_t b = 0; b < h->nblocks; ++b) {
        const int32_t* bt = &h->blk_tiles[4 * b];
        blk_key[b] = tp_index(bt[0], bt[1]) * ((int64_t)1 << 32) + tp_index(bt[2], bt[3]);
    }
    ESMF_HIP(hipSetDevice(h->device), "hipSetDevice");
    const size_t esz = h->storage == ESMF_STORE_FP64 ? sizeof(double) : sizeof(float);
    for (int64_t t = 0; t < count; ++t) {
        int sl[4];
        int32_t f[4] = {p[t], q[t], r[t], s[t]};
        for (int x = 0; x < 4; ++x) sl[x] = h->fn_slot[f[x]];
        // order each pair so its first tile is the larger, then the bra pair first
        if (sl[0] / kTile < sl[1] / kTile) std::swap(sl[0], sl[1]);
        if (sl[2] / kTile < sl[3] / kTile) std::swap(sl[2], sl[3]);
        int64_t x1 = tp_index(sl[0] / kTile, sl[1] / kTile), x2 = tp_index(sl[2] / kTile, sl[3] / kTile);
        if (x1 < x2) {
            std::swap(sl[0], sl[2]);
            std::swap(sl[1], sl[3]);
            std::swap(x1, x2);
        }
        // block keys are generated in increasing tile-pair order of the bra,
        // then of the ket, but tile pairs were enumerated in (I, J) order which
        // is the same as the tp_index order, so the keys are sorted
        int64_t key = x1 * ((int64_t)1 << 32) + x2;
        auto it = std::lower_bound(blk_key.begin(), blk_key.end(), key);
        if (it == blk_key.end() || *it != key) {
            out[t] = 0.0;
            continue;
        }
        int64_t b = it - blk_key.begin();
        int e = (((sl[0] % kTile) * kTile + (sl[1] % kTile)) * kTile + (sl[2] % kTile)) * kTile + (sl[3] % kTile);
        const int g = e / kGranule, u = e % kGranule;
        uint64_t mk[4];
        int64_t boff = 0;
        ESMF_HIP(hipMemcpy(mk, h->d_blk_mask + 4 * b, sizeof mk, hipMemcpyDeviceToHost), "lookup mask");
        ESMF_HIP(hipMemcpy(&boff, h->d_blk_off + b, sizeof boff, hipMemcpyDeviceToHost), "lookup offset");
        if (!((mk[g / 64] >> (g % 64)) & 1)) {
            out[t] = 0.0;
            continue;
        }
        int64_t rank = 0;
        for (int x = 0; x < g / 64; ++x) rank += __builtin_popcountll(mk[x]);
        if (g % 64) rank += __builtin_popcountll(mk[g / 64] & (~0ull >> (64 - g % 64)));
        const size_t pos = (size_t)(boff + rank) * kGranule + u;
        double v = 0.0;
        if (h->storage == ESMF_STORE_FP64) {
            ESMF_HIP(hipMemcpy(&v, (const char*)h->d_vals + pos * esz, esz, hipMemcpyDeviceToHost), "lookup copy");
        } else {
            float fv = 0.0f;
            ESMF_HIP(hipMemcpy(&fv, (const char*)h->d_vals + pos * esz, esz, hipMemcpyDeviceToHost), "lookup copy");
            v = fv;
        }
        out[t] = v / h->weight[b];
    }
    return ESMF_OK;
}

esmf_status esmf_fock_build(esmf_eri_t eri, int32_t m, const double* d, double* j, double* k,
                            esmf_precision prec, void* hip_stream) {
    return esmf_fock_build_sym(eri, m, d, j, k, prec, nullptr, hip_stream);
}

esmf_status esmf_fock_build_sym(esmf_eri_t eri, int32_t m, const double* d, double* j, double* k,
                                esmf_precision prec, const uint8_t* symmetric, void* hip_stream) {
    g_last_error.clear();
    const Handle* h = (const Handle*)eri;
    esmf_status st = check_build_args(h, m, d, j, k, prec);
    if (st != ESMF_OK) return st;
    const int pi = (int)prec;
    const int mode = build_mode(*h, prec);
    KernelVariant v = default_variant(mode);
    {
        // the tuner publishes its choice under the same lock
        std::lock_guard<std::mutex> lk(h->ws_mu);
        if (h->has_tuned[pi]) v = h->tuned[pi];
    }
    TimedLaunch tl{nullptr, nullptr};
    if (g_timing) {
        ESMF_HIP(hipEventCreate(&tl.start), "hipEventCreate");
        ESMF_HIP(hipEventCreate(&tl.stop), "hipEventCreate");
    }
    st = build_impl(*h, m, d, j, k, mode, v, (hipStream_t)hip_stream, tl.start, tl.stop, symmetric);
    if (st != ESMF_OK) return st;
    if (g_timing) g_timed.push_back(tl);
    return ESMF_OK;
}

}  // extern "C"

// Partial slots a build needs: those of the plan of its narrow groups (the
// variant's) and, with a wide group, of the two-visit plan.
static void build_slots(const Handle& h, const std::vector<DensityGroup>& groups, const KernelVariant& v,
                        int64_t& nk, int64_t& nj) {
    nk = nj = 0;
    for (const DensityGroup& g : groups) {
        const DevPlan& P = h.plan[g.jw == 16 ? kPlanTwoVisit : v.plan];
        nk = std::max(nk, P.nkslots);
        nj = std::max(nj, P.njslots);
    }
}

size_t esmf::build_workspace_bytes(const Handle& h, int32_t m, const uint8_t* sym, const KernelVariant& v) {
    const std::vector<DensityGroup> groups = plan_density_groups(m, sym);
    int jw = 8;
    for (const DensityGroup& g : groups) jw = std::max(jw, g.jw);
    int64_t nk, nj;
    build_slots(h, groups, v, nk, nj);
    const size_t table_bytes = (sizeof(UnitDesc) * groups.size() + 255) / 256 * 256;
    return table_bytes + operand_bytes(h.ntiles, jw) + partial_bytes(nk, nj, jw);
}

// The launches of one build into a workspace of build_workspace_bytes (unit
// table, operand tiles, partial tiles), shared by the density groups (their
// launches are stream-ordered).  A narrow group runs the variant's work plan;
// a wide group (16 J columns) always the two-visit plan, whose contraction
// holds the 16-column J operand in LDS.
esmf_status esmf::enqueue_build(const Handle& h, int32_t m, const double* d, double* j, double* k, int mode,
                                const KernelVariant& v, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop,
                                const uint8_t* sym, void* ws) {
    const std::vector<DensityGroup> groups = plan_density_groups(m, sym);
    const int G = (int)groups.size();
    int jw = 8;
    for (const DensityGroup& g : groups) jw = std::max(jw, g.jw);
    const size_t table_bytes = (sizeof(UnitDesc) * G + 255) / 256 * 256;
    std::vector<UnitDesc> units(G);
    std::vector<int> kinds(G);
    double* operands = (double*)((char*)ws + table_bytes);
    double* partials = (double*)((char*)operands + operand_bytes(h.ntiles, jw));
    int64_t nk, nj;
    build_slots(h, groups, v, nk, nj);
    for (int g = 0; g < G; ++g) {
        kinds[g] = groups[g].jw == 16 ? kPlanTwoVisit : v.plan;
        fill_unit(units[g], h, kinds[g], mode, d, j, k, groups[g]);
        unit_set_workspace(units[g], operands, partials, nk);
    }
    UnitDesc* d_units = (UnitDesc*)ws;
    hipError_t le = launch_store_units(units.data(), G, d_units, s);
    for (int g = 0; g < G && le == hipSuccess; ++g) {
        const DevPlan& P = h.plan[kinds[g]];
        KernelVariant vg = v;
        vg.plan = kinds[g];
        vg.band = P.band;
        le = launch_units(d_units, g, 1, unit_prep_size(units[g]), unit_zero_size(units[g]), P.nred,
                          (const WorkItem*)P.d_items, P.nitems, mode, vg, s, g == 0 ? ev_start : nullptr,
                          g == G - 1 ? ev_stop : nullptr, groups[g].jw);
    }
    if (le != hipSuccess) return device_fail(le, "fock");
    return ESMF_OK;
}

// One build with an explicit variant; ev_start/ev_stop (optional) bracket the
// contraction kernels.  The workspace is the handle's own, allocated with
// its first build and grown on demand (a stream-ordered pool block of this
// size is at times released and mapped again, which stalls the stream for
// hundreds of milliseconds).
esmf_status esmf::build_impl(const Handle& hr, int32_t m, const double* d, double* j, double* k,
                             int mode, const KernelVariant& v, hipStream_t s, hipEvent_t ev_start,
                             hipEvent_t ev_stop, const uint8_t* sym) {
    const Handle* h = &hr;
    const size_t ws_bytes = build_workspace_bytes(*h, m, sym, v);
    std::lock_guard<std::mutex> lk(h->ws_mu);
    if (!h->ws_done) ESMF_HIP(hipEventCreateWithFlags(&h->ws_done, hipEventDisableTiming), "workspace event");
    if (h->ws_bytes < ws_bytes) {
        if (h->ws) {
            ESMF_HIP(hipEventSynchronize(h->ws_done), "workspace release");
            ESMF_HIP(hipFree(h->ws), "workspace release");
            h->ws = nullptr;
            h->ws_bytes = 0;
        }
        if (hipMalloc(&h->ws, ws_bytes) != hipSuccess) {
            (void)hipGetLastError();
            h->ws = nullptr;
            return fail(ESMF_ERR_OUT_OF_MEMORY, "build workspace");
        }
        h->ws_bytes = ws_bytes;
        h->ws_used = false;
    }
    if (h->ws_used && h->ws_stream != s) ESMF_HIP(hipStreamWaitEvent(s, h->ws_done, 0), "workspace order");
    const esmf_status st = enqueue_build(*h, m, d, j, k, mode, v, s, ev_start, ev_stop, sym, h->ws);
    hipError_t fe = hipEventRecord(h->ws_done, s);
    h->ws_stream = s;
    h->ws_used = true;
    if (st != ESMF_OK) return st;
    if (fe != hipSuccess) return device_fail(fe, "workspace order");
    return ESMF_OK;
}

// Candidate variants of the tuner: the fused plan (two workgroups per CU,
// the LDS bound) with and without the zero-fragment skip, and the two-visit
// plan at 2 and 3 workgroups per CU (4 too for STORE32) with the skip.
std::vector<KernelVariant> esmf::tune_candidates(int mode) {
    std::vector<KernelVariant> c;
    const KernelVariant base = default_variant(mode);
    for (int skip : {1, 0}) {
        KernelVariant v = base;
        v.plan = kPlanFused;
        v.occupancy = 2;
        v.skip_zero_fragments = skip != 0;
        c.push_back(v);
    }
    for (int occ : {2, 3}) {
        KernelVariant v = base;
        v.plan = kPlanTwoVisit;
        v.occupancy = occ;
        v.skip_zero_fragments = true;
        c.push_back(v);
    }
    if (mode == 2) {  // STORE32's register budget also fits 4 workgroups per CU
        KernelVariant v = base;
        v.plan = kPlanTwoVisit;
        v.occupancy = 4;
        v.skip_zero_fragments = true;
        c.push_back(v);
    }
    return c;
}

extern "C" {

esmf_status esmf_fock_tune(esmf_eri_t eri, int32_t m, esmf_precision prec, void* hip_stream,
                           esmf_tune_report* out) {
    g_last_error.clear();
    Handle* h = (Handle*)eri;
    if (!h) return fail(ESMF_ERR_INVALID_ARG, "eri is NULL");
    if (m < 1) return fail(ESMF_ERR_INVALID_ARG, "m must be >= 1");
    if (prec != ESMF_PREC_FP64 && prec != ESMF_PREC_MIXED && prec != ESMF_PREC_STORE32)
        return fail(ESMF_ERR_INVALID_ARG, "bad precision");
    if (!precision_reads(prec, h->storage))
        return fail(ESMF_ERR_INVALID_ARG, "the precision does not read this handle's storage");
    const int mode = build_mode(*h, prec);
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t bytes = sizeof(double) * (size_t)m * h->nbf * h->nbf;
    DevBuf<double> buf;
    if (buf.alloc(3 * bytes / sizeof(double))) return fail(ESMF_ERR_OUT_OF_MEMORY, "tuner buffers");
    ESMF_HIP(hipMemsetAsync(buf.p, 0, bytes, s), "tuner density");
    double* d = buf.p;
    double* j = (double*)((char*)buf.p + bytes);
    double* k = (double*)((char*)buf.p + 2 * bytes);
    // stage 1: every variant on the current cuts of the plans; stage 2: the
    // best variant's plan cut again at half and twice its work-item length
    std::vector<KernelVariant> cand = tune_candidates(mode);
    std::vector<int> segs;
    for (const KernelVariant& v : cand) segs.push_back(h->plan[v.plan].seg);
    hipEvent_t e0, e1;
    ESMF_HIP(hipEventCreate(&e0), "hipEventCreate");
    ESMF_HIP(hipEventCreate(&e1), "hipEventCreate");
    std::vector<double> ms;
    esmf_status st = ESMF_OK;
    auto time_variant = [&](const KernelVariant& v) {
        double best = 1e300;
        for (int rep = 0; rep < 3 && st == ESMF_OK; ++rep) {  // first run is a warm-up
            st = build_impl(*h, m, d, j, k, mode, v, s, e0, e1);
            float t = 0.0f;
            if (st == ESMF_OK && (hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                st = device_fail(hipGetLastError(), "tuner timing");
            if (rep > 0) best = std::min(best, (double)t);
        }
        return best;
    };
    for (size_t c = 0; c < cand.size() && st == ESMF_OK; ++c) ms.push_back(time_variant(cand[c]));
    size_t bi = ms.empty() ? 0 : (size_t)(std::min_element(ms.begin(), ms.end()) - ms.begin());
    if (st == ESMF_OK && !cand.empty() && env_int("ESMF_TUNE_ITEMS", 1)) {
        const KernelVariant vb = cand[bi];
        const int seg0 = h->plan[vb.plan].seg;
        int best_seg = seg0;
        double best_ms = ms[bi];
        for (int sg : {seg0 / 2, seg0 * 2}) {
            if (sg < 4 || sg > 512 || st != ESMF_OK) continue;
            st = recut_plan(*h, vb.plan, sg, s);
            if (st != ESMF_OK) break;
            const double t = time_variant(vb);
            cand.push_back(vb);
            segs.push_back(sg);
            ms.push_back(t);
            if (t < best_ms) {
                best_ms = t;
                best_seg = sg;
                bi = ms.size() - 1;
            }
        }
        if (st == ESMF_OK) st = recut_plan(*h, vb.plan, best_seg, s);
        if (st == ESMF_OK) h->cut_tuned = true;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ESMF_HIP(hipStreamSynchronize(s), "tuner");
    if (st != ESMF_OK) return st;
    const int pi = (int)prec;   // tuned variants are kept per precision
    {
        std::lock_guard<std::mutex> lk(h->ws_mu);
        h->tuned[pi] = cand[bi];
        h->has_tuned[pi] = true;
    }
    if (out) {
        std::memset(out, 0, sizeof *out);
        out->candidates = (int32_t)std::min<size_t>(cand.size(), 16);
        out->chosen = (int32_t)bi;
        for (size_t c = 0; c < cand.size() && c < 16; ++c) {
            out->plan[c] = cand[c].plan;
            out->occupancy[c] = cand[c].occupancy;
            out->skip_zero[c] = cand[c].skip_zero_fragments ? 1 : 0;
            out->item_blocks[c] = segs[c];
            out->ms[c] = ms[c];
        }
    }
    return ESMF_OK;
}

esmf_status esmf_fock_batched_report(esmf_batch_report* out) {
    g_last_error.clear();
    if (!out) return fail(ESMF_ERR_INVALID_ARG, "out is NULL");
    if (g_batch_report.units == 0) return fail(ESMF_ERR_NOT_SUPPORTED, "no batched build on this thread yet");
    *out = g_batch_report;
    return ESMF_OK;
}

esmf_status esmf_fock_build_batched(int32_t nmol, const esmf_eri_t* eri, const int32_t* m,
                                    const double* const* d, double* const* j,
                                    double* const* k, esmf_precision prec, void* hip_stream) {
    g_last_error.clear();
    if (nmol < 0) return fail(ESMF_ERR_INVALID_ARG, "nmol < 0");
    if (nmol == 0) return ESMF_OK;
    if (!eri || !m || !d || !j || !k) return fail(ESMF_ERR_INVALID_ARG, "NULL array");
    std::vector<const Handle*> hs(nmol);
    std::vector<int32_t> ms(m, m + nmol);
    for (int32_t i = 0; i < nmol; ++i) {
        hs[i] = (const Handle*)eri[i];
        esmf_status st = check_build_args(hs[i], m[i], d[i], j[i], k[i], prec);
        if (st != ESMF_OK) {
            g_last_error = "molecule " + std::to_string(i) + ": " + g_last_error;
            return st;
        }
        if (hs[i]->device != hs[0]->device) return fail(ESMF_ERR_INVALID_ARG, "molecules on different devices");
        if (build_mode(*hs[i], prec) != build_mode(*hs[0], prec))
            return fail(ESMF_ERR_INVALID_ARG, "molecule " + std::to_string(i) +
                                                  ": integral-direct and stored handles in one batch");
    }
    const int mode = build_mode(*hs[0], prec);
    hipStream_t s = (hipStream_t)hip_stream;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    BatchPlan* plan = nullptr;
    for (size_t x = 0; x < g_plans.size(); ++x) {
        BatchPlan& p = *g_plans[x];
        if (p.hs == hs && p.ms == ms && p.mode == mode && p.stream == s) {
            std::unique_ptr<BatchPlan> keep = std::move(g_plans[x]);
            g_plans.erase(g_plans.begin() + x);
            g_plans.push_back(std::move(keep));
            plan = g_plans.back().get();
            break;
        }
    }
    if (!plan) {
        if (g_plans.size() >= kMaxPlans) g_plans.erase(g_plans.begin());
        std::unique_ptr<BatchPlan> p;
        esmf_status st = make_plan(hs, ms, mode, s, p);
        if (st != ESMF_OK) return st;
        // the work-item stage runs only while no member's cut has been
        // chosen yet (by esmf_fock_tune or an earlier batched plan): later
        // plans over the same handles then keep their cuts, and their
        // results equal the members' single builds bitwise
        bool cuts_free = true;
        for (const Handle* x : hs) cuts_free = cuts_free && !x->cut_tuned;
        if (env_int("ESMF_TUNE", 1) && env_int("ESMF_TUNE_ITEMS", 1) && p->nunits > 0 && cuts_free) {
            // first call: tune the variant on the molecules' current cuts (this
            // run leaves valid results), then every molecule's plan cut again
            // at half and twice its work-item length, each timed as a whole
            // batch; the fastest cut stays (the handles keep it)
            st = run_plan(*p, d, j, k);
            if (st != ESMF_OK) return st;
            ESMF_HIP(hipEventSynchronize(p->done), "batched tuner");
            const KernelVariant v0 = p->variant;
            const int kind = v0.plan;
            std::vector<int> seg0(nmol);
            for (int32_t i = 0; i < nmol; ++i) seg0[i] = hs[i]->plan[kind].seg;
            auto recut_all = [&](double f) -> esmf_status {
                for (int32_t i = 0; i < nmol; ++i) {
                    const int sg = std::max(4, std::min(512, (int)(seg0[i] * f)));
                    const esmf_status r = recut_plan(*const_cast<Handle*>(hs[i]), kind, sg, s, true);
                    if (r != ESMF_OK) return r;
                }
                return ESMF_OK;
            };
            std::vector<double> fs = {1.0}, ts = {p->best_ms};
            double best_f = 1.0, best_t = p->best_ms;
            for (double f : {0.5, 2.0}) {
                st = recut_all(f);
                std::unique_ptr<BatchPlan> q;
                if (st == ESMF_OK) st = make_plan(hs, ms, mode, s, q);
                double t = 0.0;
                if (st == ESMF_OK) {
                    q->variant = v0;
                    q->tuned = true;
                    st = time_plan(*q, d, j, k, &t);
                }
                if (st != ESMF_OK) return st;
                fs.push_back(f);
                ts.push_back(t);
                if (t < best_t) {
                    best_t = t;
                    best_f = f;
                }
            }
            st = recut_all(best_f);
            std::unique_ptr<BatchPlan> fin;
            if (st == ESMF_OK) st = make_plan(hs, ms, mode, s, fin);
            if (st != ESMF_OK) return st;
            for (const Handle* x : hs) const_cast<Handle*>(x)->cut_tuned = true;
            fin->variant = v0;
            fin->tuned = true;
            fin->cand = p->cand;
            fin->cand_ms = p->cand_ms;
            fin->best_ms = best_t;
            fin->item_factor = fs;
            fin->item_ms = ts;
            fin->item_factor_chosen = best_f;
            p = std::move(fin);
        }
        g_plans.push_back(std::move(p));
        plan = g_plans.back().get();
    }
    return run_plan(*plan, d, j, k);
}

}  // extern "C"
