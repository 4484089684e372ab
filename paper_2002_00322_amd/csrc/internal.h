// Host-side internals of libesmf shared by the runtime and the kernel launch
// wrappers.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/esmf.h"
#include "plan.h"

namespace esmf {

// A block is stored compressed by granules: granule g (0..255) holds the 16
// values with natural index 16g .. 16g+15, i.e. fixed (i, j, k/2) and all
// (k%2, l), natural index ((i*8 + j)*8 + k)*8 + l.  Only granules with at least
// one retained integral are stored, in increasing g, starting at granule
// offset blk_off[b] of the packed array; bit g of blk_mask[b] marks them.
constexpr int kGranule = 16;
constexpr int kGranules = kBlockElems / kGranule;
constexpr int kGranuleRow = 16;   // a block's granules are stored in rows of 16 (zero-padded)

// Device-side description of one molecule's block store, passed by value to
// the kernels.
struct StoreView {
    const void* vals;          // packed granules, FP64 or FP32
    const uint64_t* blk_mask;  // nblocks * 4 words: granule presence
    const int64_t* blk_off;    // nblocks: first granule of the block
    const int32_t* blk_tiles;  // nblocks * 4: tile indices I, J, K, L
    const int32_t* slot_fn;    // ntiles * kTile: caller's function index of a slot, -1 = ghost
    int64_t nblocks;
    int32_t nbf;
    int32_t ntiles;
};

// Per work entry (block in work-list order) of the contraction: the block's
// granule mask and packed offset, its ket tiles and band position (kl =
// K | L << 13 | bpos << 26), and the partial slots it feeds: the K slots of
// its run (targets (I, key) and (J, key)), its own J slot (target (K, L):
// visit 1 and fused) and, fused, the L slots of its band position (targets
// (I, L) and (J, L)).  64 bytes, read by the kernel two entries ahead.
struct alignas(16) EntryRecord {
    uint64_t mask[4];
    int64_t off;
    uint32_t kl;
    int32_t kslot_a, kslot_b;
    int32_t jslot;
    int32_t lslot_a, lslot_b;
};
static_assert(sizeof(EntryRecord) == 64, "entry record of 16 dwords");

// Partial slots are numbered by target: the slots of ordered tile pair
// t = A * ntiles + B are [kptr[t], kptr[t + 1]) (K) and [jptr[t], jptr[t + 1])
// (J, canonical pairs A >= B only), each range in the fixed order in which
// the slots were created, so the reduction streams them.

// Everything a launch needs about one (molecule, density group): the store,
// the partial plan, the group's densities and outputs, and its workspace.
struct UnitDesc {
    const void* vals;
    const EntryRecord* rec;
    const int32_t* slot_fn;
    const int64_t* kptr;
    const int64_t* jptr;
    void* X;            // operand tiles [T][T][64][16]
    void* S;            // S tiles [T][T][64][8]
    double* PK;         // K partials
    double* PJ;         // J partials
    const double* d;    // densities [m][N][N] (whole molecule)
    double* j;          // outputs [m][N][N]
    double* k;
    int32_t nbf, ntiles;
    int32_t mg, c0;     // densities c0 .. c0+mg-1 of the molecule (mg <= jw)
    int32_t jw;         // J columns of the group: 8, or 16 for a wide group
    int32_t kq;         // 4-column products of its K views (1, 2), 0: the 16-column product
    // Column map of the group (see DensityGroup): source of each matrix-core
    // column of the K operands, and each density's forward / transposed
    // K column.
    int8_t xsrc[16];
    int8_t kf[16], kt[16];
    const int32_t* used; // tile pairs A * ntiles + B that blocks read as operands
    const int32_t* red;  // unordered tile pairs X * ntiles + Y, X >= Y, with partials
    int64_t prep_begin; // first index of the unit in a launch's operand-prep range
    int64_t zero_begin; // first index of the unit in a launch's output-clearing range
    int32_t red_begin;  // first pair of the unit in a launch's reduction range
    int32_t nused;
    int32_t nred;
    int32_t nslots;     // integral-direct: slots per side of the pair arrays
    double tau;         // integral-direct: screening threshold
};

// Integral-direct data (one allocation, doubles): the six pair arrays
// 1/z, Px, Py, Pz, E', Q over nslots^2 slot pairs, then the block weights
// [nblocks].  Entry records then carry the block index in `off`.
constexpr int kDirectArrays = 6;

// Most primitives per contracted function (esmf_eri_prepare_contracted).
constexpr int kMaxPrimitives = 16;

// Launch variant of the contraction (the tuner picks one per handle and
// precision, or per batched plan):
// workgroups per CU the kernel is compiled for, and whether matrix-core
// fragments whose integrals are all zero are skipped by a wave-uniform test.
// The work plan the variant runs (kPlanTwoVisit or kPlanFused) is part of it.
struct KernelVariant {
    int occupancy = 3;
    bool skip_zero_fragments = true;
    int chain = 4;   // mode 1: reduction steps per FP32 chain (1, 2, 4 or 8)
    int plan = kPlanFused;
    int band = kFusedBand;  // fused plan: L values per band (2 or 4), as the plan was cut
};
// band of the fused plans cut at prepare time (ESMF_BAND=2 for comparisons)
int fused_band();

// A work plan on the device: work items (host copy too, batched plans
// replicate it), entry records, partial-slot ranges per target and the
// reduction's tile-pair list.
struct DevPlan {
    int kind = kPlanTwoVisit;
    int seg = 0, band = 0;
    int32_t nitems = 0;
    std::vector<WorkItem> items;
    void* d_items = nullptr;
    EntryRecord* d_rec = nullptr;
    int64_t nentries = 0;
    int64_t ntargets = 0;            // ordered tile pairs: kptr, jptr hold ntargets + 1 each
    int64_t nkslots = 0, njslots = 0;
    int64_t* d_kptr = nullptr;
    int64_t* d_jptr = nullptr;
    int32_t nred = 0;
    int32_t* d_red = nullptr;
    int64_t device_bytes() const;
    void release();
};

struct Handle {
    int32_t nbf = 0;
    int32_t ntiles = 0;
    int32_t nslots = 0;
    int device = 0;
    double tau = 0.0;
    double q_max = 0.0;
    esmf_storage storage = ESMF_STORE_FP64;
    int64_t npairs_kept = 0;
    int64_t nquartets_kept = 0;
    int64_t nblocks = 0;
    int64_t device_bytes = 0;
    // variant chosen by esmf_fock_tune, per precision (esmf_precision value)
    bool has_tuned[3] = {false, false, false};
    KernelVariant tuned[3];
    // host copies
    std::vector<int32_t> slot_fn;     // [nslots]
    std::vector<int32_t> fn_slot;     // [nbf]
    std::vector<int32_t> blk_tiles;   // [nblocks*4]
    std::vector<double> weight;       // [nblocks]
    // the two work plans: two visits per block, and fused (one visit)
    DevPlan plan[2];
    // tile pairs read as operand tiles (X or S) by some block, ascending
    int32_t nused = 0;
    int32_t* d_used = nullptr;
    // device memory
    void* d_vals = nullptr;          // integral store, or integral-direct data
    uint64_t* d_blk_mask = nullptr;
    int64_t* d_blk_off = nullptr;
    int64_t ngranules = 0;
    int64_t ngranules_fp64 = 0;
    // a work-item cut was chosen by a tuner (esmf_fock_tune or a batched
    // plan's first call); batched plans then keep it
    bool cut_tuned = false;  // granules an FP64 store of the block list holds (direct handles too)
    int32_t* d_blk_tiles = nullptr;
    int32_t* d_slot_fn = nullptr;
    // Workspace of single builds (unit table, operand and partial tiles),
    // kept with the handle and grown on demand: builds on one stream reuse it
    // in stream order; a build on another stream first waits for the event
    // recorded after the last use.
    mutable std::mutex ws_mu;
    mutable void* ws = nullptr;
    mutable size_t ws_bytes = 0;
    mutable hipEvent_t ws_done = nullptr;
    mutable hipStream_t ws_stream = nullptr;
    mutable bool ws_used = false;

    StoreView view() const {
        StoreView v;
        v.vals = d_vals;
        v.blk_mask = d_blk_mask;
        v.blk_off = d_blk_off;
        v.blk_tiles = d_blk_tiles;
        v.slot_fn = d_slot_fn;
        v.nblocks = nblocks;
        v.nbf = nbf;
        v.ntiles = ntiles;
        return v;
    }
};

// Arithmetic mode of the contraction for a precision on a handle: the
// esmf_precision value, 3 for FP64 on an integral-direct handle, 4 for
// MIXED on an FP64 store (integrals rounded to FP32 as they are loaded).
inline int build_mode(const Handle& h, esmf_precision prec) {
    if (h.storage == ESMF_STORE_DIRECT) return 3;
    if (prec == ESMF_PREC_MIXED && h.storage == ESMF_STORE_FP64) return 4;
    return (int)prec;
}

// Storage a precision reads: FP64 builds an FP64 or integral-direct store,
// STORE32 builds an FP32 store, MIXED builds an FP32 or FP64 store.
inline bool precision_reads(esmf_precision prec, int storage) {
    switch (prec) {
        case ESMF_PREC_FP64: return storage == ESMF_STORE_FP64 || storage == ESMF_STORE_DIRECT;
        case ESMF_PREC_MIXED: return storage == ESMF_STORE_FP32 || storage == ESMF_STORE_FP64;
        case ESMF_PREC_STORE32: return storage == ESMF_STORE_FP32;
    }
    return false;
}

// ---- ESMF terms around the build (esmf_terms.hip) ----
// The nine densities [9][n][n] from Theta [no][n], Gamma [nv][n], sigma and
// mu [no][nv], R [no][n], Phi [nv][n] (device, row-major); `work` holds
// nine_densities_work_doubles(n, no) doubles.
hipError_t launch_nine_densities(int n, int no, int nv, const double* theta, const double* gamma,
                                 const double* sigma, const double* mu, const double* r,
                                 const double* phi, double* d, double* work, hipStream_t s);
size_t nine_densities_work_doubles(int n, int no);
// E_2 of Eq. esmf_energy_2b into the device scalar e2; `partial` holds
// energy_partial_doubles() doubles.
hipError_t launch_energy_two_body(int n, double n2, double c0, const double* d, const double* j,
                                  const double* k, double* e2, double* partial, hipStream_t s);
size_t energy_partial_doubles();
// energy and first derivatives (esmf_energy_gradient); work: gradient_work_doubles
hipError_t launch_energy_gradient(int n, int no, int nv, double c0, double n2, const double* theta,
                                  const double* gamma, const double* sigma, const double* g, const double* d,
                                  const double* j, const double* k, double* energy, double* dsigma,
                                  double* dtheta, double* dgamma, double* work, hipStream_t s);
size_t gradient_work_doubles(int n, int no);

// ---- launch wrappers (kernels.hip) ----
// Pair quantities in slot order for all slot pairs (a, b): 1/zeta, P,
// E' = E (pi/zeta)^(3/2) and the Schwarz factor Q = sqrt((ab|ab)); ghost
// slots give E' = Q = 0.
hipError_t launch_pair_build(int nslots, const int32_t* d_slot_fn, const double* d_centers,
                             const double* d_alpha, double* d_pz, double* d_px, double* d_py,
                             double* d_pzc, double* d_pe, double* d_pq, hipStream_t s);
// Granule presence of every block (a granule is kept if one of its integrals
// passes Q_ij Q_kl > tau) and the number of kept granules per block.
hipError_t launch_granule_mask(int64_t nblocks, const int32_t* d_blk_tiles, int nslots,
                               const double* d_pq, double tau, uint64_t* d_mask,
                               int32_t* d_count, hipStream_t s);
// Fill the kept granules: w * (ij|kl) where Q_ij Q_kl > tau, else 0.
hipError_t launch_eri_fill(int64_t nblocks, const int32_t* d_blk_tiles, const double* d_w,
                           const uint64_t* d_mask, const int64_t* d_off, int nslots,
                           const double* d_pz, const double* d_px, const double* d_py,
                           const double* d_pzc, const double* d_pe, const double* d_pq,
                           double tau, void* d_vals, int fp32, hipStream_t s);

// Cartesian basis (lmn: int8 [nbf][3], l + m + n <= 2; function f is the sum
// of primitives [poff[f], poff[f+1]) with exponents pexp and coefficients
// pcoef, normalisation included): Schwarz factors of the slot pairs with a
// function other than a one-primitive s function (overwriting pq), and the
// fill with the Cartesian integral where a quartet has one.
hipError_t launch_cart_pair_q(int nslots, const int32_t* d_slot_fn, const double* d_centers, const int8_t* d_lmn,
                              const int32_t* d_off, const double* d_pexp, const double* d_pcoef, double* d_pq,
                              hipStream_t s);
hipError_t launch_eri_fill_cart(int64_t nblocks, const int32_t* d_blk_tiles, const double* d_w,
                                const uint64_t* d_mask, const int64_t* d_off, int nslots, const double* d_pz,
                                const double* d_px, const double* d_py, const double* d_pzc, const double* d_pe,
                                const double* d_pq, double tau, const int32_t* d_slot_fn, const double* d_centers,
                                const int8_t* d_lmn, const int32_t* d_poff, const double* d_pexp,
                                const double* d_pcoef, void* d_vals, int fp32, hipStream_t s);

// entry records from the block arrays and the per-entry slots (kSlotFields
// per entry, plan.h)
hipError_t launch_build_records(int64_t n, const int32_t* d_entries, const int32_t* d_blk_tiles,
                                const uint64_t* d_mask, const int64_t* d_off, const int32_t* d_eslot,
                                EntryRecord* d_rec, hipStream_t s);


// A density group: densities c0 .. c0+mg-1 of a build, contracted in one
// pass over the integrals.  The K operands have 16 matrix-core columns; a
// density takes a forward column (D) and a transposed one (D^T), or, when it
// is symmetric, one column serving both (its transposed partials equal its
// forward ones).  J takes one column per density: 8 in a narrow group, 16 in
// a wide one (whose contraction holds a 16-column J operand in LDS).
//   xsrc[c]: -1 unused, else density p | kXsrcTransposed for the D^T column
//   kf[p], kt[p]: forward and transposed K columns of density p
constexpr int kXsrcTransposed = 0x20;
struct DensityGroup {
    int c0 = 0, mg = 0, jw = 8;
    int8_t xsrc[16];
    int8_t kf[16], kt[16];
};
// Groups of a build of m densities (sym: m flags, nonzero = symmetric, or
// NULL): in order, each as large as 16 K columns and 16 J columns allow; a
// group of at most 8 densities is narrow.  Without symmetric densities this
// is groups of 8 with the columns D_0..D_7 | D_0^T..D_7^T.
std::vector<DensityGroup> plan_density_groups(int m, const uint8_t* sym);

// tuned FP64 build (fock_mfma.hip)
hipError_t launch_store_units(const UnitDesc* h, int n, UnitDesc* d, hipStream_t s);
// workspace of one density group of J width jw (8 or 16)
size_t operand_bytes(int ntiles, int jw = 8);
size_t partial_bytes(int64_t nkslots, int64_t njslots, int jw = 8);
void unit_set_workspace(UnitDesc& u, double* operands, double* partials, int64_t nkslots);
int64_t unit_prep_size(const UnitDesc& u);
int64_t unit_zero_size(const UnitDesc& u);  // output elements cleared per matrix
// Operand prep over units [unit_base, unit_base + nunits) (prep_total
// indices), clearing of their outputs (zero_total elements per matrix), the
// contraction over `nitems` items, and the reduction over red_total tile
// pairs; ev_start/ev_stop (optional) bracket the contraction.
// mode: arithmetic mode of the contraction (0 FP64, 1 FP32 hi/lo split on
// FP32 matrix cores, 2 FP32 integrals on FP64 matrix cores, 3 integral-direct).
// jw: J width of every unit of the launch (8; 16 runs the wide contraction,
// which has its own fixed variant).
hipError_t launch_units(const UnitDesc* d_units, int unit_base, int nunits, int64_t prep_total,
                        int64_t zero_total, int red_total, const WorkItem* d_items, int nitems, int mode,
                        const KernelVariant& variant, hipStream_t s, hipEvent_t ev_start = nullptr,
                        hipEvent_t ev_stop = nullptr, int jw = 8);

// copy n work items into a launch's list at dst, unit index set to `unit`,
// padded with empty items to npad
hipError_t launch_copy_items(const WorkItem* src, int n, WorkItem* dst, int npad, int unit,
                             hipStream_t s);

// ---- runtime (runtime.cpp) ----
// error reporting through esmf_last_error (thread-local)
esmf_status fail(esmf_status s, const std::string& msg);
esmf_status device_fail(hipError_t e, const char* what);
void clear_error();
KernelVariant default_variant(int mode);
void ensure_pool_cached(int device);
void fill_unit(UnitDesc& u, const Handle& h, int plan, int mode, int m, const double* d, double* j, double* k,
               int g);
esmf_status check_build_args(const Handle* h, int32_t m, const double* d, double* j, double* k,
                             esmf_precision prec);
esmf_status prepare_impl(int32_t nbf, const double* centers, const double* exponents,
                         double schwarz_tau, esmf_storage storage, void* hip_stream,
                         int64_t byte_limit, int64_t* footprint, esmf_eri_t* out,
                         const int32_t* lmn = nullptr, const int32_t* poff = nullptr,
                         const double* pexp = nullptr, const double* pcoef = nullptr);

esmf_status check_contraction(int32_t nbf, const int32_t* lmn, const int32_t* prim_offset,
                              const double* prim_exp, const double* prim_coef, std::vector<double>& emin);

// one build with an explicit variant (events bracket the contraction)
// (sym: m symmetry flags or NULL, see plan_density_groups)
esmf_status build_impl(const Handle& h, int32_t m, const double* d, double* j, double* k, int mode,
                       const KernelVariant& v, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop,
                       const uint8_t* sym = nullptr);
// the launches of one build into a caller-provided workspace of
// build_workspace_bytes (no allocation)
size_t build_workspace_bytes(const Handle& h, int32_t m, const uint8_t* sym, const KernelVariant& v);
esmf_status enqueue_build(const Handle& h, int32_t m, const double* d, double* j, double* k, int mode,
                          const KernelVariant& v, hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop,
                          const uint8_t* sym, void* ws);
std::vector<KernelVariant> tune_candidates(int mode);
// device arrays of a work plan, its entry records, and a new cut of a
// handle's plan with items of `seg` blocks (tuning)
esmf_status alloc_plan(DevPlan& P, const WorkPlan& w, int64_t ntargets, hipStream_t s);
esmf_status fill_plan_records(const Handle& h, DevPlan& P, const WorkPlan& w, hipStream_t s);
esmf_status recut_plan(Handle& h, int kind, int seg, hipStream_t s, bool plans_locked = false);
// drop the cached batched plans that use h (the second form with the plan
// cache's lock held by the caller)
void drop_plans_using(const Handle* h);
void drop_plans_using_locked(const Handle* h);
int env_int(const char* name, int dflt);

// one build of a grouped launch
struct GroupEntry {
    const Handle* h;
    int32_t m;
    const double* d;
    double* j;
    double* k;
};
// workspace of one density group / of a build of m densities in a grouped
// launch (table, items and group areas; the sum over a group's entries bounds
// the group's need)
size_t group_unit_bytes(const Handle& h, int kind);
size_t group_workspace_bytes(const Handle& h, int m, int kind);
esmf_status enqueue_group(const std::vector<GroupEntry>& es, int mode, hipStream_t s,
                          void* ws_ext = nullptr, size_t ws_ext_bytes = 0);

}  // namespace esmf
