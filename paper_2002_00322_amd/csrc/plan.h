// Host planning of the grouped J/K build: the tile plan of a molecule, the
// screened list of canonical tile-quartet blocks with their degeneracy
// weights, and the work plans of the contraction (work items, entry order and
// the numbering of partial slots).  Plain C++ with no device calls, so that it
// can be built and checked on a CPU (and under sanitizers) on its own.
#pragma once

#include <cstdint>
#include <vector>

namespace esmf {

// Functions per tile of the block store: a stored block holds the integrals
// (ij|kl) for i in tile I, j in J, k in K, l in L, i.e. kTile^4 values.
constexpr int kTile = 8;
constexpr int kBlockElems = kTile * kTile * kTile * kTile;
// Tile indices are packed into 13 bits of an entry record.
constexpr int kMaxTiles = 8191;
// L values of a fused item's band (one accumulator pair each in registers):
// the most a plan may use, and the contraction kernel's band.
constexpr int kMaxBand = 8;
constexpr int kFusedBand = 4;

// One work item of the contraction: block entries [e0, e1) of bra (I, J),
// walked as `visit` 0 (runs of equal K), 1 (runs of equal L) or 2 (fused: both
// visits' products on one read of each block, over a band of L values), with
// its J slot of target (I, J) (visit 0 and fused; -1 in visit 1); `unit`
// selects the molecule / density group of a launch.  Items with e1 <= e0 are
// padding.
struct WorkItem {
    int32_t e0, e1;
    int32_t I, J;
    int32_t visit;
    int32_t reserved;
    int32_t jslot0;
    int32_t unit;
};

// The screened block list of one molecule.
struct BlockList {
    int32_t nbf = 0, nslots = 0, ntiles = 0;
    std::vector<int32_t> slot_fn;     // [nslots]: function of a slot, -1 = ghost
    std::vector<int32_t> blk_tiles;   // [nblocks][4]: I, J, K, L
    std::vector<double> weight;       // [nblocks]: degeneracy weight of the block's slots
    int64_t nblocks() const { return (int64_t)weight.size(); }
};

// Partial-slot fields of an entry (block in work order).
enum { kSlotKA = 0, kSlotKB, kSlotJ, kSlotLA, kSlotLB, kSlotBpos, kSlotFields };

// Plan kinds.
enum { kPlanTwoVisit = 0, kPlanFused = 1 };

// A work plan of the contraction over a block list.
//   entries  block index of each entry, in work order (two entries per block
//            for a two-visit plan, one for a fused plan)
//   items    work items over the entries
//   eslot    [entries][kSlotFields]: per entry, the K slots of its run
//            (targets (I, key), (J, key)), its own J slot (target (K, L):
//            visit 1 and fused), and in a fused plan the L slots of its band
//            position in its item (targets (I, L), (J, L)) and that position
//   kptr, jptr  slot ranges per ordered tile pair t = A * ntiles + B: the K
//            slots of target t are [kptr[t], kptr[t+1]), the J slots
//            [jptr[t], jptr[t+1]), each in creation order
//   used     tile pairs A * ntiles + B read as operand tiles, ascending
//   red      unordered tile pairs X * ntiles + Y (X >= Y) with any partial
struct WorkPlan {
    int kind = kPlanTwoVisit;
    int seg = 0, band = 0;
    std::vector<int32_t> entries;
    std::vector<WorkItem> items;
    std::vector<int32_t> eslot;
    std::vector<int64_t> kptr, jptr;
    int64_t nkslots = 0, njslots = 0;
    std::vector<int32_t> used, red;
};

// Slots of the functions: grouped by exponent (classes smaller than a tile
// merged with their neighbours), each group cut into tiles of kTile by
// recursive coordinate bisection, the last tile of a group padded with ghost
// slots (-1).
std::vector<int32_t> make_tile_plan(int n, const double* centers, const double* alpha);

// Canonical blocks (IJ|KL), I >= J, K >= L, (IJ) >= (KL) in tile-pair order,
// whose largest Schwarz product exceeds tau, from the Schwarz factors of the
// slot pairs q[a * nslots + b] (0 for ghost slots), bra-major with the kets
// in (K, L) order, each with the weight 1/2 per coincidence I = J, K = L,
// IJ = KL.
void plan_blocks(const std::vector<double>& q, const std::vector<int32_t>& slot_fn, double tau, BlockList& bl);

// Blocks per work item when none is given: about four items per workgroup
// slot of the device (512 slots), between 8 and 64 blocks.
int default_item_blocks(int kind, int64_t nblocks);

// The work plan of `kind` with items of at most `seg` blocks (fused: bands of
// `band` distinct L values, 1..kMaxBand).  Items are interleaved over `xcd`
// queues (bra rows spread over the queues by size) so that item i of the
// list runs on XCD i % xcd.  Returns 0, or -1 when a slot count exceeds the
// 31-bit range.
int plan_work(const BlockList& bl, int kind, int seg, int band, int xcd, WorkPlan& wp);

}  // namespace esmf
