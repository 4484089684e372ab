// Host-side internals of libesmf shared by the runtime and the kernel launch
// wrappers.  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/esmf.h"

namespace esmf {

// Functions per tile of the block store: a stored block holds the integrals
// (ij|kl) for i in tile I, j in J, k in K, l in L, i.e. kTile^4 values.
constexpr int kTile = 8;
constexpr int kBlockElems = kTile * kTile * kTile * kTile;

// Device-side description of one molecule's block store, passed by value to
// the kernels.
struct StoreView {
    const void* vals;          // nblocks * kBlockElems, FP64 or FP32
    const int32_t* blk_tiles;  // nblocks * 4: tile indices I, J, K, L
    const int32_t* slot_fn;    // ntiles * kTile: caller's function index of a slot, -1 = ghost
    int64_t nblocks;
    int32_t nbf;
    int32_t ntiles;
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
    // host copies
    std::vector<int32_t> slot_fn;     // [nslots]
    std::vector<int32_t> fn_slot;     // [nbf]
    std::vector<int32_t> blk_tiles;   // [nblocks*4]
    std::vector<double> weight;       // [nblocks]
    // work lists of the tuned build: entries (block indices in visit order)
    // and work items (24-byte records, see fock_mfma.hip)
    int32_t nitems = 0;
    int32_t* d_entries = nullptr;
    void* d_items = nullptr;
    // device memory
    void* d_vals = nullptr;
    int32_t* d_blk_tiles = nullptr;
    int32_t* d_slot_fn = nullptr;

    StoreView view() const {
        StoreView v;
        v.vals = d_vals;
        v.blk_tiles = d_blk_tiles;
        v.slot_fn = d_slot_fn;
        v.nblocks = nblocks;
        v.nbf = nbf;
        v.ntiles = ntiles;
        return v;
    }
};

// ---- launch wrappers (kernels.hip) ----
// Pair quantities in slot order for all slot pairs (a, b): zeta, P, E and the
// Schwarz factor Q = sqrt((ab|ab)); ghost slots give E = Q = 0.
hipError_t launch_pair_build(int nslots, const int32_t* d_slot_fn, const double* d_centers,
                             const double* d_alpha, double* d_pz, double* d_px, double* d_py,
                             double* d_pzc, double* d_pe, double* d_pq, hipStream_t s);
// Fill the block store: w * (ij|kl) where Q_ij Q_kl > tau, else 0.
hipError_t launch_eri_fill(int64_t nblocks, const int32_t* d_blk_tiles, const double* d_w,
                           int nslots, const double* d_pz, const double* d_px,
                           const double* d_py, const double* d_pzc, const double* d_pe,
                           const double* d_pq, double tau, void* d_vals, int fp32,
                           hipStream_t s);
hipError_t launch_zero(double* p, int64_t n, hipStream_t s);
hipError_t launch_fock_fp64_simple(const StoreView& sv, int m, const double* d, double* j,
                                   double* k, hipStream_t s);
hipError_t launch_symmetrize_j(int nbf, int m, double* j, hipStream_t s);

// tuned FP64 build (fock_mfma.hip)
size_t fock_mfma_workspace_bytes(int ntiles);
size_t fock_mfma_item_bytes();
hipError_t launch_fock_mfma_f64(const StoreView& sv, const int32_t* d_entries,
                                const void* d_items, int nitems, int m, const double* d,
                                double* j, double* k, double* workspace, hipStream_t s);

}  // namespace esmf
