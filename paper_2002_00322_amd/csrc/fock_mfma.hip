// Tuned grouped J/K build for gfx950 on matrix cores, FP64 and mixed precision.
//
// The store holds canonical tile-quartet blocks (IJ|KL), I>=J, K>=L,
// (I,J)>=(K,L), each kTile^4 = 4096 weighted, screened integrals v[i][j][k][l].
// With the 2m-column trick (columns 0..7 carry D_c, columns 8..15 carry D_c^T)
// every K update of Eq. J_and_K for a block is one of four GEMM "views":
//
//   target (I,K): C[(i,k)][c] += sum_(j,l) v X_JL[(j,l)][c]      (view V2)
//   target (J,K): C[(j,k)][c] += sum_(i,l) v X_IL[(i,l)][c]      (view V3^T)
//   target (I,L): C[(i,l)][c] += sum_(j,k) v X_JK[(j,k)][c]      (view V3)
//   target (J,L): C[(j,l)][c] += sum_(i,k) v X_IK[(i,k)][c]      (view V2^T)
//
// where X_AB[(a,b)][c] = D_c[A_a][B_b] for c < 8 and D_{c-8}[B_b][A_a] for
// c >= 8; a column c >= 8 of a target (A,B) lands at K[B_b][A_a].  J uses
// S = D + D^T: J_IJ[(i,j)][c] += sum_(k,l) v S_KL[(k,l)][c] (view V1) and
// J_KL[(k,l)][c] += sum_(i,j) v S_IJ[(i,j)][c] (view V1^T), the two symmetric
// positions of J being summed by the reduction.
// That is the layout of a narrow group of 8 densities; a smaller one packs
// its m forward and m transposed columns at the front (D_c at c, D_c^T at
// m + c).  In general a density group carries a column map: each X
// column's source density and orientation, and each density's forward and
// transposed column.  A symmetric density uses one column for both (its
// transposed partials equal its forward ones), so up to 16 densities fit
// the 16 columns; a group of more than 8 is wide and runs with JW = 16 J
// columns.
//
// Every block is visited twice, both times from its bra tile pair IJ:
//   visit 0: blocks of bra IJ in runs of equal K  -> (I,K), (J,K) and J_IJ
//   visit 1: blocks of bra IJ in runs of equal L  -> (I,L), (J,L) and J_KL
// so the K targets of a visit stay in matrix-core accumulators for a whole run
// and J_IJ for the whole work item.  Run ends, work-item ends and J_KL (per
// block) store their accumulators as partial tiles (plain coalesced stores)
// into slots fixed at prepare time; a reduction kernel then sums, for every
// output tile, its list of partial slots in a fixed order and writes J and K.
// No atomics: a build is bitwise reproducible.
//
// Precision.  FP64: FP64 integrals and v_mfma_f64_16x16x4 (K views) and
// v_mfma_f64_4x4x4 (J views of a narrow group).  Mixed: FP32 integrals; the
// four K views split each density D = D_hi + D_lo (D_hi = fp32(D),
// D_lo = fp32(D - D_hi)); the hi product on v_mfma_f32_16x16x4 into an FP32
// chain added into the FP64 accumulator every CHAIN reduction steps (4 CHAIN
// products per chain), the lo product, a correction of relative size 2^-24,
// on BF16 matrix cores (v_mfma_f32_16x16x16_bf16, four steps per product)
// into an FP32 sum added into FP64 when the accumulator is stored.  The two
// J views (a fifth of the products) run in FP64 on the FP32 integrals, which
// convert exactly.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "eri_device.h"
#include "internal.h"

namespace esmf {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
static_assert(sizeof(u4) == 16, "16-byte chunk");

constexpr int kW = 4;                      // waves per workgroup
constexpr int kThreads = 64 * kW;
constexpr int kCols = 16;                  // matrix-core N: the group's K columns
constexpr int kOpElems = 64 * kCols;       // one operand tile [64][16]
// a J operand tile / J partial slot of J width JW: [64][JW]
template <int JW>
constexpr int kSE = 64 * JW;

// LDS position of v[i][j][k][l]: the natural index ((i*8+j)*8+k)*8+l with its
// low bank bits replaced by a bank function, linear over GF(2) in the index
// bits, chosen so that every lane group the LDS serves at once (16 lanes for
// 8-byte, 32 lanes for 4-byte elements) reads distinct banks in all six views,
// and so that the map is a bijection inside each group of 2^bits positions.
//   8-byte (4 bits): b0 = l0^k0^j1, b1 = l1^k1^j0, b2 = l2^k2^j2, b3 = i0^j0^k0.
//   4-byte (5 bits): b = XOR of the columns i0:15 j0:21 j1:1 j2:28 k0:1 k1:10
//                    k2:17 l0:13 l1:27 l2:18 over the set bits.
template <bool F32>
struct Swz;

template <>
struct Swz<false> {
    static constexpr int kBits = 4;
    __device__ __forceinline__ static constexpr int pos(int i, int j, int k, int l) {
        int nat = ((i * 8 + j) * 8 + k) * 8 + l;
        int b0 = (l ^ k ^ (j >> 1)) & 1;
        int b1 = ((l >> 1) ^ (k >> 1) ^ j) & 1;
        int b2 = ((l >> 2) ^ (k >> 2) ^ (j >> 2)) & 1;
        int b3 = (i ^ j ^ k) & 1;
        return (nat & ~15) | (b3 << 3) | (b2 << 2) | (b1 << 1) | b0;
    }
};

template <>
struct Swz<true> {
    static constexpr int kBits = 5;
    __device__ __forceinline__ static constexpr int pos(int i, int j, int k, int l) {
        int nat = ((i * 8 + j) * 8 + k) * 8 + l;
        int b = 0;
        b ^= (i & 1) ? 15 : 0;
        b ^= (j & 1) ? 21 : 0;
        b ^= (j & 2) ? 1 : 0;
        b ^= (j & 4) ? 28 : 0;
        b ^= (k & 1) ? 1 : 0;
        b ^= (k & 2) ? 10 : 0;
        b ^= (k & 4) ? 17 : 0;
        b ^= (l & 1) ? 13 : 0;
        b ^= (l & 2) ? 27 : 0;
        b ^= (l & 4) ? 18 : 0;
        return (nat & ~31) | b;
    }
};

// Granule g holds natural indices 16 g + u (i = g/32, j = (g/4)%8,
// k = 2 (g%4) + u/8, l = u%8).  The swizzle only rewrites the bank bits, which
// lie inside the granule's own aligned group, and is linear in the index bits,
// so pos = gran_base(g) XOR gran_bits(u): one XOR per element of a granule.
template <bool F32>
__device__ __forceinline__ constexpr int gran_base(int g) {
    return Swz<F32>::pos(g >> 5, (g >> 2) & 7, 2 * (g & 3), 0);
}
template <bool F32>
__device__ __forceinline__ constexpr int gran_bits(int u) {
    return Swz<F32>::pos(0, 0, u >> 3, u & 7);
}
template <bool F32>
constexpr bool gran_split_holds() {
    for (int g = 0; g < kGranules; ++g)
        for (int u = 0; u < kGranule; ++u)
            if (Swz<F32>::pos(g >> 5, (g >> 2) & 7, 2 * (g & 3) + (u >> 3), u & 7) !=
                (gran_base<F32>(g) ^ gran_bits<F32>(u)))
                return false;
    return true;
}
static_assert(gran_split_holds<false>() && gran_split_holds<true>(),
              "swizzle is not a per-granule XOR");

// Arithmetic modes P:
//   0  FP64 integrals, FP64 matrix cores;
//   1  FP32 integrals, densities split hi/lo, both parts on FP32 matrix cores
//      into FP32 chains that are summed in FP64 every CHAIN steps;
//   2  FP32 integrals converted exactly to FP64 at the matrix-core input,
//      FP64 matrix cores (error: only the FP32 rounding of the stored values);
//   3  integral-direct FP64: no store, each block's kept integrals are
//      computed in the fetch from the resident pair data (FP64 matrix cores);
//   4  the arithmetic of mode 1 on an FP64 store: each integral is rounded
//      to FP32 as the block goes into LDS (the value an FP32 store holds).
// Element types: the store holds GT, LDS holds ET; an operand value is one
// FP64 number, or the FP32 pair (hi, lo) of the split (8 bytes either way).
template <int P>
struct Prec {
    using ET = double;
    using GT = double;
    using OT = double;
};
template <>
struct Prec<1> {
    using ET = float;
    using GT = float;
    using OT = f2;
};
template <>
struct Prec<2> {
    using ET = float;
    using GT = float;
    using OT = double;
};
template <>
struct Prec<4> {
    using ET = float;
    using GT = double;
    using OT = f2;
};

// Modes with the hi/lo split on FP32 matrix cores, and modes with 4-byte
// integrals in LDS.
template <int P>
constexpr bool kMixed = P == 1 || P == 4;
template <int P>
constexpr bool kLds32 = P == 1 || P == 2 || P == 4;
// The J views run on the FP64 matrix cores in every mode: J is a fifth of a
// quartet's products, and the mixed modes' FP32 integrals convert exactly.
// Those of a narrow group (8 columns) run as two v_mfma_f64_4x4x4f64
// products (four 4x4 blocks each, columns 0..3 and 4..7) instead of one
// 16x16x4 product whose columns 8..15 are discarded: the same 16x4 A
// fragment, half the matrix-core time, and on this chip the same bits as the
// 16-column product.
template <int P, int JW>
constexpr bool kJ4 = JW == 8;
// K views of a narrow column set.  A density group's K columns (forward and
// transposed, packed at the front of the 16) may fit KQ = 1 or 2 groups of
// 4; its four K views then run KQ v_mfma_f64_4x4x4f64 products per step
// (columns 4h..4h+3, h < KQ) instead of the 16-column product: the same bits
// (as for J), a quarter of the matrix-core time saved per unused group of 4.
// The operand prep interleaves such a group's X tile rows (column c at
// 4 (c % 4) + c / 4), so that a lane's KQ values lie side by side.  FP64
// matrix-core modes on the two-visit plan (the unit's kq); KQ = 0 is the
// 16-column product, also for 9..12 columns: a third path's operands would
// raise the register use of every kernel that holds it.
template <int P>
constexpr bool kNarrowK = P == 0 || P == 2 || P == 3;

// Pointers read from a unit descriptor are generic; marking them global lets
// the compiler use global (saddr + offset) loads and stores instead of flat
// ones, which need 64-bit per-lane addresses and the LDS counter as well.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

// Matrix-core fragment layouts (lane l of a wave), both 16x16x4:
//   A[16][4]: l holds A[l % 16][l / 16];  B[4][16]: l holds B[l / 16][l % 16];
//   C[16][16] element r (0..3) of lane l holds column l % 16 of row
//     4 r + l / 16       for v_mfma_f64_16x16x4f64,
//     4 (l / 16) + r     for v_mfma_f32_16x16x4f32.
// v_mfma_f64_4x4x4f64 (block b = (l / 4) % 4 of four): A_b[l % 4][l / 16],
// B_b[l / 16][l % 4], C_b[l / 16][l % 4].  With block b = rows 4b..4b+3 of a
// 16-row tile, its A operand is the 16x16x4 fragment above (row l % 16,
// k = l / 16); lane l holds C[4 ((l / 4) % 4) + l / 16][l % 4].
template <int P>
__device__ __forceinline__ int c_row(int r, int lane) {
    return kMixed<P> ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4);
}

// Store the row-tile rt of a 64x16 K accumulator as part of partial slot
// `slot` ([64][16], row = (a, b) of the target tile pair).
template <int P>
__device__ __forceinline__ void store_partial_k(const UnitDesc& a, int slot, int rt, d4 acc,
                                                int lane) {
    gptr<double> dst = (gptr<double>)a.PK + (int64_t)slot * kOpElems + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(16 * rt + c_row<P>(r, lane)) * kCols] = acc[r];
}

// The K accumulator of a narrow column set (KQ 4x4x4 products): lane l holds
// row 4 ((l / 4) % 4) + l / 16 of the row tile, columns 4h + l % 4, h < KQ.
template <int KQ>
__device__ __forceinline__ void store_partial_kq(const UnitDesc& a, int slot, int rt, d4 acc, int lane) {
    gptr<double> dst = (gptr<double>)a.PK + (int64_t)slot * kOpElems +
                       (16 * rt + 4 * ((lane >> 2) & 3) + (lane >> 4)) * kCols + (lane & 3);
#pragma unroll
    for (int h = 0; h < KQ; ++h) dst[4 * h] = acc[h];
}

// J accumulators (FP64 matrix-core outputs in every mode): a narrow group
// holds the two 4x4x4 products' columns l % 4 and 4 + l % 4 of partial slot
// [64][8] (see kJ4), a wide group a 16x16x4 tile of slot [64][16].
template <int P, int JW>
__device__ __forceinline__ void store_partial_j(const UnitDesc& a, int slot, int rt, d2 acc,
                                                int lane) {
    static_assert(kJ4<P, JW>, "two-column J accumulators are the narrow form");
    gptr<double> dst = (gptr<double>)a.PJ + (int64_t)slot * kSE<8> +
                       (16 * rt + 4 * ((lane >> 2) & 3) + (lane >> 4)) * 8 + (lane & 3);
    dst[0] = acc[0];
    dst[4] = acc[1];
}
template <int P, int JW>
__device__ __forceinline__ void store_partial_j(const UnitDesc& a, int slot, int rt, d4 acc,
                                                int lane) {
    static_assert(!kJ4<P, JW>, "a narrow group stores two-column J accumulators");
    gptr<double> dst = (gptr<double>)a.PJ + (int64_t)slot * kSE<JW> + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[(16 * rt + c_row<0>(r, lane)) * JW] = acc[r];
}

// LDS position of the element a lane reads in view WHICH of visit VIS, with
// (x1, x2) its row indices and (y1, y2) its reduction indices.
template <int P, int VIS, int WHICH>
__device__ __forceinline__ constexpr int view_pos(int x1, int x2, int y1, int y2) {
    using W = Swz<kLds32<P>>;
    if constexpr (VIS == 0) {
        if constexpr (WHICH == 0) return W::pos(x1, y1, x2, y2);       // V2:   rows (i,k), red (j,l)
        else if constexpr (WHICH == 1) return W::pos(y1, x1, x2, y2);  // V3^T: rows (j,k), red (i,l)
        else return W::pos(x1, x2, y1, y2);                            // V1:   rows (i,j), red (k,l)
    } else {
        if constexpr (WHICH == 0) return W::pos(x1, y1, y2, x2);       // V3:   rows (i,l), red (j,k)
        else if constexpr (WHICH == 1) return W::pos(y1, x1, y2, x2);  // V2^T: rows (j,l), red (i,k)
        else return W::pos(y1, y2, x1, x2);                            // V1^T: rows (k,l), red (i,j)
    }
}

// Element read at reduction step s: the reduction index q = 4s + fk has
// y1 = s/2 and y2 = 4(s%2) + fk, so every index bit belongs either to the lane
// or to s.  As the swizzle is linear over GF(2) in the bits and the bits above
// the bank are a sum, the position is (lane base XOR C_s[bank]) + C_s[above]
// with lane base = the position at s = 0 and C_s = the position of lane 0.
// Lane bases are kept in bytes, so that each read costs one XOR.
template <int P, int VIS, int WHICH, int S, typename ET>
__device__ __forceinline__ ET read_a(const ET* sV, int lanebase_bytes) {
    constexpr int C = view_pos<P, VIS, WHICH>(0, 0, S >> 1, 4 * (S & 1));
    constexpr int M = (1 << Swz<kLds32<P>>::kBits) - 1;
    constexpr int Z = (int)sizeof(ET);
    return *(const ET*)((const char*)sV + ((lanebase_bytes ^ ((C & M) * Z)) + (C & ~M) * Z));
}

// Accumulators of one view: FP64, plus in modes 1 and 4 the FP32 chain of the hi
// product (drained into FP64 every CHAIN steps) and the FP32 sum of the lo
// products (a correction of relative size 2^-24, so its own FP32 rounding is
// of relative size 2^-48: drained only when the accumulator is stored).
template <int P>
struct Acc {
    d4 d;
    f4 hi, lo;
    __device__ __forceinline__ void zero() {
        d = d4{0, 0, 0, 0};
        hi = f4{0, 0, 0, 0};
        lo = f4{0, 0, 0, 0};
    }
    __device__ __forceinline__ void drain() {
        if constexpr (kMixed<P>) {
#pragma unroll
            for (int r = 0; r < 4; ++r) d[r] += (double)hi[r];
            hi = f4{0, 0, 0, 0};
            // The next chain starts from zero and would not depend on this
            // drain; an opaque read-modify of the accumulators ties them, so
            // chains are drained in order instead of all products being formed
            // first (which holds every chain's result live at once).
            asm volatile("" : "+v"(d), "+v"(hi));
        }
    }
    __device__ __forceinline__ void drain_all() {
        if constexpr (kMixed<P>) {
#pragma unroll
            for (int r = 0; r < 4; ++r) d[r] += (double)hi[r] + (double)lo[r];
            hi = f4{0, 0, 0, 0};
            lo = f4{0, 0, 0, 0};
            asm volatile("" : "+v"(d), "+v"(hi), "+v"(lo));
        }
    }
};

template <int P, typename ET, typename OT>
__device__ __forceinline__ void mma(ET a, OT b, Acc<P>& c) {
    if constexpr (kMixed<P>) {
        c.hi = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b.x, c.hi, 0, 0, 0);
    } else {
        c.d = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, b, c.d, 0, 0, 0);
    }
}

// The J accumulator of a narrow group: columns l % 4 and 4 + l % 4 of the
// two 4x4x4 products.  A wide group's is the FP64 form of Acc.
struct AccJ4 {
    d2 d;
    __device__ __forceinline__ void zero() { d = d2{0, 0}; }
    __device__ __forceinline__ void drain() {}
    __device__ __forceinline__ void drain_all() {}
};
template <int P, int JW>
using AccJ = typename std::conditional<kJ4<P, JW>, AccJ4, Acc<0>>::type;
// its value between blocks, and the J operand a lane holds at one step
template <int P, int JW>
using JVal = typename std::conditional<kJ4<P, JW>, d2, d4>::type;
template <int P, int JW>
using JOp = typename std::conditional<kJ4<P, JW>, d2, double>::type;

// The K accumulators of a narrow column set: element h of d is product h's
// (h < KQ); no FP32 chain.
struct AccK4 {
    d4 d;
    __device__ __forceinline__ void zero() { d = d4{0, 0, 0, 0}; }
    __device__ __forceinline__ void drain() {}
    __device__ __forceinline__ void drain_all() {}
};
template <int P, int KQ>
using AccK = typename std::conditional<(KQ > 0), AccK4, Acc<P>>::type;
// the K operand a lane holds at one step: KQ values (columns 4h + l % 4)
template <int P, int KQ>
using KOp = typename std::conditional<KQ == 0, typename Prec<P>::OT,
                                      typename std::conditional<KQ == 1, double, d2>::type>::type;

template <int P, int KQ, typename ET, typename BT, typename AK>
__device__ __forceinline__ void mma_k(ET a, BT b, AK& c) {
    static_assert(KQ >= 0 && KQ <= 2, "K column sets of 4 or 8 columns, or the 16-column product");
    if constexpr (KQ == 0) {
        mma<P>(a, b, c);
    } else if constexpr (KQ == 1) {
        c.d[0] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)a, b, c.d[0], 0, 0, 0);
    } else {
#pragma unroll
        for (int h = 0; h < KQ; ++h)
            c.d[h] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)a, b[h], c.d[h], 0, 0, 0);
    }
}

template <int P, int JW, typename ET, typename BT, typename AJ>
__device__ __forceinline__ void mma_j(ET a, BT b, AJ& c) {
    if constexpr (kJ4<P, JW>) {
        c.d[0] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)a, b[0], c.d[0], 0, 0, 0);
        c.d[1] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)a, b[1], c.d[1], 0, 0, 0);
    } else {
        c.d = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, b, c.d, 0, 0, 0);
    }
}

// Modes 1 and 4, the lo products v * D_lo on BF16 matrix cores.  Over four reduction
// steps 4t..4t+3 lane l holds A[row][4S + l/16] and B[4S + l/16][col] in its
// FP32 fragments; for v_mfma_f32_16x16x16_bf16 the same lane supplies A and B
// at the reduction positions 4 (l/16) + e, e = 0..3, so element e of its
// packed operands is taken from step 4t + e: the product is the sum of the
// four steps' lo products.  The operands are truncated to bf16 (their upper
// 16 bits, 8 significant bits: relative error below 2^-7 each), so a lo
// product is off by less than 2^-6 of a term of relative size 2^-24, i.e.
// 2^-30 of |v D|, against the 2^-24 rounding of the hi chain.
typedef short s4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));
struct LoView {
    u2v a, b;      // bf16 pairs of v and D_lo
    float pa, pb;  // the even step's values, until paired
    bool any;      // a fragment of the four steps is present
};
struct LoPack {
    LoView v0, v1;
};

// The upper halves of x (low 16 bits of the result) and y (high 16 bits): one
// v_perm_b32.  (Rounding to nearest even took four instructions through
// v_cvt_pk_bf16_f32 and ran 6 % slower overall; one v_cvt_pk_bf16_f32 of both
// values ran at half speed.)
__device__ __forceinline__ uint32_t pack_bf16(float x, float y) {
    return __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, y), __builtin_bit_cast(uint32_t, x), 0x07060302u);
}

__device__ __forceinline__ f4 mfma_lo(u2v a, u2v b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4v, a), __builtin_bit_cast(s4v, b), c, 0,
                                                      0, 0);
}

// Step S of a view's lo operands: pair the even step's values with the odd
// step's, and after the fourth step issue the BF16 product.
template <int S>
__device__ __forceinline__ void lo_step(LoView& lv, float av, float bl, bool present, f4& lo) {
    if constexpr (S % 2 == 0) {
        lv.pa = av;
        lv.pb = bl;
    } else if constexpr ((S % 4) / 2 == 0) {
        lv.a.x = pack_bf16(lv.pa, av);
        lv.b.x = pack_bf16(lv.pb, bl);
    } else {
        lv.a.y = pack_bf16(lv.pa, av);
        lv.b.y = pack_bf16(lv.pb, bl);
    }
    lv.any = (S % 4 == 0) ? present : (lv.any || present);
    if constexpr (S % 4 == 3) {
        if (lv.any) lo = mfma_lo(lv.a, lv.b, lo);
    }
}

// The fragments of one reduction step: A values of the three views and their
// B operands.
template <int P, int JW, int KQ>
struct Frag {
    typename Prec<P>::ET v0, v1, vj;
    KOp<P, KQ> b0, b1;
    JOp<P, JW> bj;
};

template <int P, int VIS, int JW, int KQ, int S>
__device__ __forceinline__ Frag<P, JW, KQ> load_frag(const typename Prec<P>::ET* sV,
                                             const typename Prec<P>::OT* sB0,
                                             const typename Prec<P>::OT* sB1,
                                             const double* sBJ, int lane, int lb0,
                                             int lb1, int lbj) {
    Frag<P, JW, KQ> f;
    f.v0 = read_a<P, VIS, 0, S>(sV, lb0);
    f.v1 = read_a<P, VIS, 1, S>(sV, lb1);
    f.vj = read_a<P, VIS, 2, S>(sV, lbj);
    // B fragment: lane holds B[4s + l/16][l%16] = operand[(4s + l/16) * 16 + l%16].
    // The J operand is FP64 in every mode.  A narrow one (8 columns) is read
    // as columns l%4 and 4 + l%4, which its tile holds side by side (column c
    // at 2 (c % 4) + c / 4).
    // A narrow K column set reads columns 4h + l%4, h < KQ, of its
    // interleaved tile row: KQ adjacent values.
    if constexpr (KQ == 0) {
        f.b0 = sB0[64 * S + lane];
        f.b1 = sB1[64 * S + lane];
    } else {
        const int kb = 64 * S + 16 * (lane >> 4) + 4 * (lane & 3);
        f.b0 = *(const KOp<P, KQ>*)(sB0 + kb);
        f.b1 = *(const KOp<P, KQ>*)(sB1 + kb);
    }
    if constexpr (kJ4<P, JW>)
        f.bj = *(const d2*)(sBJ + 32 * S + 8 * (lane >> 4) + 2 * (lane & 3));
    else
        f.bj = sBJ[64 * S + lane];
    return f;
}

// Which granules a matrix-core fragment reads, as scalar tests on the block's
// 256-bit granule mask (dword q = granules 32 q .. 32 q + 31, i.e. i = q).  A
// fragment of view WHICH at step S in row tile w covers:
//   visit 0  V2   i in {2w, 2w+1}, j = S/2, all k      -> (d[2w]|d[2w+1]) & 0xF << 4j
//            V3^T i = S/2, j in {2w, 2w+1}, all k      -> d[i] & 0xFF << 8w
//            V1   i in {2w, 2w+1}, all j, k = S/2      -> (d[2w]|d[2w+1]) & 0x11111111 << k/2
//   visit 1  V3   i in {2w, 2w+1}, j = S/2, k/2 in 2(S%2) + {0, 1}
//                                                    -> (d[2w]|d[2w+1]) & 0x3 << (4j + 2(S%2))
//            V2^T i = S/2, j in {2w, 2w+1}, k/2 in 2(S%2) + {0, 1}
//                                                    -> d[i] & (0x33 << 8w) << 2(S%2)
//            V1^T i = S/2, j in 4(S%2) + 0..3, k/2 = w -> d[i] & (0x1111 << w) << 16(S%2)
// A fragment whose granules are all absent is zero and its product is
// skipped; the decision is uniform and needs no data.
struct SkipMask {
    uint32_t d[8];   // mask dwords of the block
    uint32_t orw;    // d[2w] | d[2w+1]
    uint32_t m8;     // 0xFF << 8w
    uint32_t m33;    // 0x33 << 8w
    uint32_t m1;     // 0x1111 << w
};

template <int VIS, int WHICH, int S>
__device__ __forceinline__ bool frag_present(const SkipMask& k) {
    if constexpr (VIS == 0) {
        if constexpr (WHICH == 0) return (k.orw & (0xFu << (4 * (S >> 1)))) != 0;
        else if constexpr (WHICH == 1) return (k.d[S >> 1] & k.m8) != 0;
        else return (k.orw & (0x11111111u << (S >> 2))) != 0;
    } else {
        if constexpr (WHICH == 0) return (k.orw & (0x3u << (4 * (S >> 1) + 2 * (S & 1)))) != 0;
        else if constexpr (WHICH == 1) return (k.d[S >> 1] & (k.m33 << (2 * (S & 1)))) != 0;
        else return (k.d[S >> 1] & (k.m1 << (16 * (S & 1)))) != 0;
    }
}

// SKIP: 0 every product; 1 only products of fragments with a present
// granule (scalar mask tests: no wait on the fragment values, no vector work).
template <int P, int VIS, int SKIP, int CHAIN, int JW, int KQ, int S>
__device__ __forceinline__ void k_step(const Frag<P, JW, KQ>& f, const SkipMask& sk, AccK<P, KQ>& acc0,
                                       AccK<P, KQ>& acc1, AccJ<P, JW>& accJ, LoPack& lp) {
    bool n0 = true, n1 = true, nj = true;
    if constexpr (SKIP == 1) {
        n0 = frag_present<VIS, 0, S>(sk);
        n1 = frag_present<VIS, 1, S>(sk);
        nj = frag_present<VIS, 2, S>(sk);
    }
    if (n0) mma_k<P, KQ>(f.v0, f.b0, acc0);
    if (n1) mma_k<P, KQ>(f.v1, f.b1, acc1);
    if (nj) mma_j<P, JW>(f.vj, f.bj, accJ);
    if constexpr (kMixed<P>) {
        lo_step<S>(lp.v0, (float)f.v0, f.b0.y, n0, acc0.lo);
        lo_step<S>(lp.v1, (float)f.v1, f.b1.y, n1, acc1.lo);
        if constexpr ((S + 1) % CHAIN == 0) {
            acc0.drain();
            acc1.drain();
        }
    }
}

// The 16 reduction steps of a block, software-pipelined: the fragments of
// step S + 1 are read from LDS before the (conditional) matrix-core
// issues of step S, so the LDS latency of a step hides behind the previous
// step's products.
template <int P, int VIS, int SKIP, int CHAIN, int JW, int KQ, int S = 0>
__device__ __forceinline__ void k_steps(const typename Prec<P>::ET* sV,
                                        const typename Prec<P>::OT* sB0,
                                        const typename Prec<P>::OT* sB1,
                                        const double* sBJ, int lane, int lb0,
                                        int lb1, int lbj, const SkipMask& sk, AccK<P, KQ>& acc0,
                                        AccK<P, KQ>& acc1, AccJ<P, JW>& accJ, const Frag<P, JW, KQ>& cur,
                                        LoPack& lp) {
    if constexpr (S < 16) {
        Frag<P, JW, KQ> nxt;
        if constexpr (S + 1 < 16)
            nxt = load_frag<P, VIS, JW, KQ, S + 1>(sV, sB0, sB1, sBJ, lane, lb0, lb1, lbj);
        k_step<P, VIS, SKIP, CHAIN, JW, KQ, S>(cur, sk, acc0, acc1, accJ, lp);
        k_steps<P, VIS, SKIP, CHAIN, JW, KQ, S + 1>(sV, sB0, sB1, sBJ, lane, lb0, lb1, lbj, sk, acc0,
                                                        acc1, accJ, nxt, lp);
    }
}

// An entry record as the kernel uses it: the packed tile and band fields
// unpacked (see EntryRecord).
struct Rec {
    uint64_t mask[4];
    int64_t off;
    int K, L, bpos;
    int kslot_a, kslot_b, jslot, lslot_a, lslot_b;
};

__device__ __forceinline__ void unpack_kl(uint32_t kl, Rec& r) {
    r.K = (int)(kl & 0x1FFFu);
    r.L = (int)((kl >> 13) & 0x1FFFu);
    r.bpos = (int)(kl >> 26);
}

// A record in flight: lane l holds dword l % 16 of the record (one VGPR), so
// the load is a vector load, counted with the block loads in issue order; its
// fields are read out into scalars when the record is used.
__device__ __forceinline__ uint32_t load_rec_word(gptr<const EntryRecord> p, int lane) {
    return ((gptr<const uint32_t>)p)[lane & 15];
}
__device__ __forceinline__ Rec unpack_rec(uint32_t wd) {
    auto rl = [&](int i) { return (uint32_t)__builtin_amdgcn_readlane((int)wd, i); };
    Rec r;
#pragma unroll
    for (int x = 0; x < 4; ++x) r.mask[x] = (uint64_t)rl(2 * x) | ((uint64_t)rl(2 * x + 1) << 32);
    r.off = (int64_t)((uint64_t)rl(8) | ((uint64_t)rl(9) << 32));
    unpack_kl(rl(10), r);
    r.kslot_a = (int32_t)rl(11);
    r.kslot_b = (int32_t)rl(12);
    r.jslot = (int32_t)rl(13);
    r.lslot_a = (int32_t)rl(14);
    r.lslot_b = (int32_t)rl(15);
    return r;
}

__device__ __forceinline__ Rec load_rec(gptr<const EntryRecord> p) {
    Rec r;
#pragma unroll
    for (int x = 0; x < 4; ++x) r.mask[x] = p->mask[x];
    r.off = p->off;
    unpack_kl(p->kl, r);
    r.kslot_a = p->kslot_a;
    r.kslot_b = p->kslot_b;
    r.jslot = p->jslot;
    r.lslot_a = p->lslot_a;
    r.lslot_b = p->lslot_b;
    return r;
}

// Integral-direct: the 16 integrals of granule g (i, j, k/2 of the granule;
// u = (k%2, l)) of block `blk` = (I J | K L), computed from the pair data with
// the store fill's formula and screen and stored into the block's LDS image
// (FP64 layout).  Not inlined: the Boys function's constants then stay in the
// callee instead of being hoisted into the contraction loop's registers.
__device__ __attribute__((noinline)) void direct_granule(double* sV, const double* pairs, int ns,
                                                         double tau, int64_t blk, int I, int J, int K,
                                                         int L, int g) {
    const int64_t nss = (int64_t)ns * ns;
    const gptr<const double> dd = (gptr<const double>)pairs;
    auto pair = [&](int64_t x) {
        return PairData{dd[x], dd[nss + x], dd[2 * nss + x], dd[3 * nss + x], dd[4 * nss + x],
                        dd[5 * nss + x]};
    };
    const double wb = dd[kDirectArrays * nss + blk];
    const int gi = g >> 5, gj = (g >> 2) & 7, kp = g & 3;
    const PairData pab = pair((int64_t)(I * kTile + gi) * ns + (J * kTile + gj));
    const int gbase = gran_base<false>(g);
    for (int u = 0; u < 16; ++u) {
        const int k = 2 * kp + (u >> 3), l = u & 7;
        sV[gbase ^ gran_bits<false>(u)] =
            screened_eri(wb, pab, pair((int64_t)(K * kTile + k) * ns + (L * kTile + l)), tau);
    }
}

// Integral-direct in the fused kernel: the pair data of the item's bra tile
// pair and of the block's ket tile pair are staged in LDS as
// sPair[side][array][a * 8 + b] (side 0 bra, 1 ket; the six arrays of
// PairData), so the 16 integrals of a granule read their pair quantities
// from LDS (the threads of one k/2 read the same 16 ket pairs: broadcasts).
constexpr int kPairLds = 2 * kDirectArrays * 64;

// Load of one side's 64 pairs x 6 arrays from the pair arrays into the
// registers of threads 0..383 of a 256-thread group (two values per thread
// for threads < 128): value v = t or t + 256 is array v / 64, pair v % 64.
__device__ __forceinline__ void load_pairs(const double* pairs, int ns, int A, int B, int tid, double& x0,
                                           double& x1) {
    const int64_t nss = (int64_t)ns * ns;
    const gptr<const double> dd = (gptr<const double>)pairs;
    auto at = [&](int v) {
        const int arr = v >> 6, ab = v & 63;
        return dd[arr * nss + (int64_t)(A * kTile + (ab >> 3)) * ns + (B * kTile + (ab & 7))];
    };
    x0 = at(tid);
    x1 = tid < 128 ? at(tid + 256) : 0.0;
}

__device__ __forceinline__ void store_pairs(double* sSide, int tid, double x0, double x1) {
    sSide[tid] = x0;
    if (tid < 128) sSide[tid + 256] = x1;
}

__device__ __attribute__((noinline)) void direct_granule_lds(double* sV, const double* sPair, double wb,
                                                             double tau, int g) {
    const int gi = g >> 5, gj = (g >> 2) & 7, kp = g & 3;
    auto pair = [&](int side, int ab) {
        const double* p = sPair + side * (kDirectArrays * 64) + ab;
        return PairData{p[0], p[64], p[128], p[192], p[256], p[320]};
    };
    const PairData pab = pair(0, gi * 8 + gj);
    const int gbase = gran_base<false>(g);
    for (int u = 0; u < 16; ++u) {
        const int k = 2 * kp + (u >> 3), l = u & 7;
        sV[gbase ^ gran_bits<false>(u)] = screened_eri(wb, pab, pair(1, k * 8 + l), tau);
    }
}

// A K accumulator's partial tile, in the layout of its products.
template <int P, int KQ>
__device__ __forceinline__ void store_k(const UnitDesc& a, int slot, int rt, d4 acc, int lane) {
    if constexpr (KQ == 0)
        store_partial_k<P>(a, slot, rt, acc, lane);
    else
        store_partial_kq<KQ>(a, slot, rt, acc, lane);
}

// One work item of visit VIS: bra (I, J), block entries [e0, e1); JW is the
// J width of the item's density group, KQ its K column set (see kNarrowK).
template <int P, int VIS, int SKIP, int CHAIN, int JW, int KQ>
__device__ __forceinline__ void run_item(const UnitDesc& a, const WorkItem& it,
                                         typename Prec<P>::ET* sV,
                                         typename Prec<P>::OT* sB0,
                                         typename Prec<P>::OT* sB1,
                                         double* sBJ, uint16_t* sSel) {
    using ET = typename Prec<P>::ET;
    using GT = typename Prec<P>::GT;
    using OT = typename Prec<P>::OT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave = row-tile of every view
    const int I = it.I, J = it.J;
    const int T = a.ntiles;
    const int fr = lane & 15, fk = lane >> 4;
    // row indices of this lane in row-tile w: rows 16w + fr = (x1, x2)
    const int x1 = (16 * w + fr) >> 3, x2 = fr & 7;
    constexpr int kZ = (int)sizeof(typename Prec<P>::ET);
    constexpr bool kF32 = kLds32<P>;   // 4-byte integrals in LDS
    int lb0 = view_pos<P, VIS, 0>(x1, x2, 0, fk) * kZ;   // lane bases in bytes
    int lb1 = view_pos<P, VIS, 1>(x1, x2, 0, fk) * kZ;
    int lbj = view_pos<P, VIS, 2>(x1, x2, 0, fk) * kZ;
    SkipMask sk;
    sk.m8 = 0xFFu << (8 * w);
    sk.m33 = 0x33u << (8 * w);
    sk.m1 = 0x1111u << w;
    const gptr<const GT> vals = (gptr<const GT>)a.vals;
    const gptr<const OT> Xo = (gptr<const OT>)a.X;
    const gptr<const double> So = (gptr<const double>)a.S;
    const gptr<const EntryRecord> rec = (gptr<const EntryRecord>)a.rec;

    AccK<P, KQ> acc0, acc1;
    AccJ<P, JW> accJ;
    acc0.zero();
    acc1.zero();
    accJ.zero();
    int run_key = -1;
    int run_ka = 0, run_kb = 0;  // K slots of the current run
    GT pv[16];   // the block's values in flight (store precision)
    constexpr int kVW = 16 / (int)sizeof(GT);   // values per 16-byte load
    typedef GT VT __attribute__((ext_vector_type(kVW)));
    // operand tiles staged as 16-byte chunks: X tiles 2 per thread, S tile
    // JW / 8
    constexpr int kSC = JW / 8;
    static_assert(sizeof(OT) * kOpElems == 2 * kThreads * 16 && sizeof(double) * kSE<JW> == kSC * kThreads * 16,
                  "operand tile chunking");
    u4 pb0[2], pb1[2], pbj[kSC];

    // Entry records are read two entries ahead (vector loads, see
    // load_rec_word), the block data one entry ahead: no load of the data path
    // waits on another, and no LDS wait waits on a scalar load.
    // The block's present granules are contiguous in the packed array; they are
    // loaded flat (coalesced): packed value x*256 + tid is element u = tid % 16
    // of the present granule of rank r = 16 x + tid / 16.  Granule tid itself
    // is present iff bit tid of the mask; `myrank` is its rank among them.
    int cnt = 0, myrank = -1;
    int64_t blk_off = 0;       // integral-direct: block index of the fetched entry
    int blk_K = 0, blk_L = 0;  // and its ket tiles
    bool was_present = true;  // granule tid present in the previous block (LDS group not zero)
    // Visit 1's J operand S_IJ is the item's own bra pair: loaded with the
    // first block only, it then stays in LDS for the whole item.
    auto fetch = [&](const Rec& r, bool first) {
        const uint64_t m0 = r.mask[0], m1 = r.mask[1], m2 = r.mask[2], m3 = r.mask[3];
        const uint64_t mw = w == 0 ? m0 : w == 1 ? m1 : w == 2 ? m2 : m3;
        int rank = (w > 0 ? __popcll(m0) : 0) + (w > 1 ? __popcll(m1) : 0) + (w > 2 ? __popcll(m2) : 0);
        // set bits of mw below this lane
        rank += __builtin_amdgcn_mbcnt_hi((uint32_t)(mw >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mw, 0u));
        myrank = ((mw >> lane) & 1) ? rank : -1;
        cnt = __popcll(m0) + __popcll(m1) + __popcll(m2) + __popcll(m3);
        const int K = r.K, L = r.L;
        if constexpr (P == 3) {
            blk_off = r.off;  // integral-direct: the block index (values are computed in the scatter)
            blk_K = K;
            blk_L = L;
        } else {
            // rank -> LDS base of the granule, read by the scatter of this
            // block after the next barrier.  The packed granules of a block
            // are zero-padded to whole rows of 16 (256 values), so rows load
            // without per-lane tests.  Ranks >= cnt, whose padding zeros the
            // last row also stores, point at an absent granule: its LDS group
            // holds zeros, or gets them in this phase.
            if (myrank >= 0) sSel[myrank] = (uint16_t)(gran_base<kF32>(tid) * kZ);
            if (tid >= cnt) {
                const int q = ~m0 ? 0 : ~m1 ? 1 : ~m2 ? 2 : 3;
                const uint64_t mq = q == 0 ? m0 : q == 1 ? m1 : q == 2 ? m2 : m3;
                const int gabs = 64 * q + __builtin_ctzll(~mq | (1ull << 63));
                sSel[tid] = (uint16_t)(gran_base<kF32>(gabs) * kZ);
            }
            // 16-byte loads: lane tid of load x takes values
            // kVW (kThreads x + tid) .. + kVW - 1 of the block, kVW
            // consecutive elements of one granule; rows of 16 granules are
            // loaded while they hold a present granule (the store pads the
            // last row with zeros)
            const gptr<const VT> src = (gptr<const VT>)(vals + r.off * 16);
            const int npad = (cnt + 15) / 16 * 256;   // values in the padded rows
#pragma unroll
            for (int x = 0; x < 16 / kVW; ++x)
                if (kVW * (x * kThreads + tid) < npad) {
                    const VT t = __builtin_nontemporal_load(src + x * kThreads + tid);
#pragma unroll
                    for (int w = 0; w < kVW; ++w) pv[kVW * x + w] = t[w];
                }
        }
        gptr<const OT> X0, X1;
        gptr<const double> Sp;
        if constexpr (VIS == 0) {  // X_JL, X_IL, S_KL
            X0 = Xo + ((int64_t)J * T + L) * kOpElems;
            X1 = Xo + ((int64_t)I * T + L) * kOpElems;
            Sp = So + ((int64_t)K * T + L) * kSE<JW>;
        } else {                   // X_JK, X_IK, S_IJ
            X0 = Xo + ((int64_t)J * T + K) * kOpElems;
            X1 = Xo + ((int64_t)I * T + K) * kOpElems;
            Sp = So + ((int64_t)I * T + J) * kSE<JW>;
        }
        const gptr<const u4> X0c = (gptr<const u4>)X0, X1c = (gptr<const u4>)X1;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            pb0[x] = X0c[x * kThreads + tid];
            pb1[x] = X1c[x * kThreads + tid];
        }
        if (VIS == 0 || first) {
#pragma unroll
            for (int x = 0; x < kSC; ++x) pbj[x] = ((gptr<const u4>)Sp)[x * kThreads + tid];
        }
    };

    if (it.e1 <= it.e0) return;  // padding item
    Rec rc = load_rec(rec + it.e0);                                              // entry e
    uint32_t wn = load_rec_word(rec + (it.e0 + 1 < it.e1 ? it.e0 + 1 : it.e0), lane);  // e + 1
    fetch(rc, true);
    __syncthreads();
    // Visit 1: the J_KL partial of the previous block, stored one iteration
    // late (after this iteration's wait for its block data), so that no wait
    // for block data ever waits for a store issued just before it.
    JVal<P, JW> jk_prev = {};
    int jslot_prev = -1;
    LoPack lp;  // modes 1 and 4: packed lo operands of the current four steps
    for (int e = it.e0; e < it.e1; ++e) {
        const int key = VIS == 0 ? rc.K : rc.L;
        const bool run_ends = key != run_key && run_key >= 0;
        const int jslot = rc.jslot;  // visit 1: this block's J_KL slot
        if constexpr (SKIP == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sk.d[2 * q] = (uint32_t)rc.mask[q];
                sk.d[2 * q + 1] = (uint32_t)(rc.mask[q] >> 32);
            }
            const uint64_t mw = w == 0 ? rc.mask[0] : w == 1 ? rc.mask[1] : w == 2 ? rc.mask[2] : rc.mask[3];
            sk.orw = (uint32_t)mw | (uint32_t)(mw >> 32);
        }
        // Absent granules must read as zero.  A granule's LDS group is written
        // only by the scatter of blocks where it is present, so it needs
        // zeroing (by its own thread) only where it is absent now and was
        // present in the previous block of the item (or this is the item's
        // first block).  The rank table of this block was written by its
        // fetch, before the last barrier.
        char* const sVb = (char*)sV;
        const bool refill = myrank < 0 && was_present;
        was_present = myrank >= 0;
        if (refill) {
            int gbase = gran_base<kF32>(tid) * kZ;
            asm("" : "+v"(gbase) : "s"(e));  // addresses formed here, not kept live
#pragma unroll
            for (int u = 0; u < 16; ++u) *(ET*)(sVb + (gbase ^ (gran_bits<kF32>(u) * kZ))) = (ET)0;
        }
        if constexpr (P == 3) {
            // Integral-direct: the thread of a present granule computes its 16
            // integrals (i, j, k/2 of the granule; u = (k%2, l)) from the pair
            // data, with the store fill's formula and screen, and stores each
            // into the block's LDS image (lanes of 16 consecutive granules hit
            // distinct banks).
            if (myrank >= 0)
                direct_granule((double*)sV, (const double*)a.vals, a.nslots, a.tau, blk_off, I, J,
                               blk_K, blk_L, tid);
        } else {
            // all rank-table reads first (r < kGranules always), then the
            // stores: load x of lane tid holds elements uq .. uq + kVW - 1,
            // uq = kVW (tid % (16 / kVW)), of the granule of rank
            // 16 kVW x + tid / (16 / kVW)
            constexpr int kLanesPerGranule = 16 / kVW;
            const int ub = gran_bits<kF32>(kVW * (tid % kLanesPerGranule)) * kZ;
            const int npad = (cnt + 15) / 16 * 256;
            int gsel[16 / kVW];
#pragma unroll
            for (int x = 0; x < 16 / kVW; ++x) gsel[x] = sSel[16 * kVW * x + tid / kLanesPerGranule];
#pragma unroll
            for (int x = 0; x < 16 / kVW; ++x)
                if (kVW * (x * kThreads + tid) < npad) {
#pragma unroll
                    for (int w = 0; w < kVW; ++w)
                        *(ET*)(sVb + (gsel[x] ^ ub ^ (gran_bits<kF32>(w) * kZ))) = (ET)pv[kVW * x + w];
                }
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            ((u4*)sB0)[x * kThreads + tid] = pb0[x];
            ((u4*)sB1)[x * kThreads + tid] = pb1[x];
        }
        if (VIS == 0 || e == it.e0) {
#pragma unroll
            for (int x = 0; x < kSC; ++x) ((u4*)sBJ)[x * kThreads + tid] = pbj[x];
        }
        // Stores of finished accumulators, after the block data were waited for.
        if (run_ends) {
            acc0.drain_all();
            acc1.drain_all();
            store_k<P, KQ>(a, run_ka, w, acc0.d, lane);
            store_k<P, KQ>(a, run_kb, w, acc1.d, lane);
            acc0.zero();
            acc1.zero();
        }
        if (key != run_key) {
            run_ka = rc.kslot_a;
            run_kb = rc.kslot_b;
        }
        run_key = key;
        if constexpr (VIS == 1) {
            if (jslot_prev >= 0) store_partial_j<P, JW>(a, jslot_prev, w, jk_prev, lane);
        }
        __syncthreads();
        // The per-step LDS addresses are (lane base XOR constant); made opaque
        // per entry (an empty, memory-free asm that depends on e), they are
        // formed next to their reads in every iteration instead of being
        // hoisted out of the loop as ~30 live registers.
        asm("" : "+v"(lb0), "+v"(lb1), "+v"(lbj) : "s"(e));
        const Frag<P, JW, KQ> f0 = load_frag<P, VIS, JW, KQ, 0>(sV, sB0, sB1, sBJ, lane, lb0, lb1, lbj);
        if (e + 1 < it.e1) {
            const Rec rn = unpack_rec(wn);
            wn = load_rec_word(rec + (e + 2 < it.e1 ? e + 2 : e + 1), lane);
            fetch(rn, false);
            rc = rn;
        }
        if constexpr (VIS == 0) {
            k_steps<P, VIS, SKIP, CHAIN, JW, KQ>(sV, sB0, sB1, sBJ, lane, lb0, lb1, lbj, sk, acc0,
                                             acc1, accJ, f0, lp);
        } else {
            AccJ<P, JW> accK;  // J_KL of this block
            accK.zero();
            k_steps<P, VIS, SKIP, CHAIN, JW, KQ>(sV, sB0, sB1, sBJ, lane, lb0, lb1, lbj, sk, acc0,
                                             acc1, accK, f0, lp);
            accK.drain_all();
            jk_prev = accK.d;
            jslot_prev = jslot;
        }
        __syncthreads();
    }
    if constexpr (VIS == 1) {
        if (jslot_prev >= 0) store_partial_j<P, JW>(a, jslot_prev, w, jk_prev, lane);
    }
    acc0.drain_all();
    acc1.drain_all();
    accJ.drain_all();
    if (run_key >= 0) {
        store_k<P, KQ>(a, run_ka, w, acc0.d, lane);
        store_k<P, KQ>(a, run_kb, w, acc1.d, lane);
    }
    if constexpr (VIS == 0) store_partial_j<P, JW>(a, it.jslot0, w, accJ.d, lane);
}

// Fused work item: bra (I, J), the blocks of one band of at most NB distinct
// L values in (K, L) order.  Each block is read and scattered into LDS once
// and all six views run on it:
//   visit-0 views V2, V3^T, V1 -> (I,K), (J,K) [run-stationary over a K-run],
//                                  J_IJ [item-stationary], operands X_JL, X_IL, S_KL;
//   visit-1 views V3, V2^T, V1^T -> (I,L), (J,L) [item-stationary, one pair of
//                                  accumulators per band position],
//                                  J_KL [per block], operands X_JK, X_IK, S_IJ.
// The L accumulators live as FP64 values between blocks (NB pairs); each
// block's visit-1 products continue the pair of its band position.  Partial
// stores: K-run ends, J_KL one block late, and at the item's end J_IJ and
// every band position's L pair.
template <int P, int SKIP, int CHAIN, int NB>
__device__ __forceinline__ void run_item_fused(const UnitDesc& a, const WorkItem& it,
                                               typename Prec<P>::ET* sV, typename Prec<P>::OT* sX0,
                                               typename Prec<P>::OT* sX1, typename Prec<P>::OT* sX2,
                                               typename Prec<P>::OT* sX3, double* sS0, double* sS1,
                                               uint16_t* sSel, double* sPair) {
    using ET = typename Prec<P>::ET;
    using GT = typename Prec<P>::GT;
    using OT = typename Prec<P>::OT;
    constexpr int JW = 8;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave = row-tile of every view
    const int I = it.I, J = it.J;
    const int T = a.ntiles;
    const int fr = lane & 15, fk = lane >> 4;
    const int x1 = (16 * w + fr) >> 3, x2 = fr & 7;
    constexpr int kZ = (int)sizeof(ET);
    constexpr bool kF32 = kLds32<P>;
    int lb0 = view_pos<P, 0, 0>(x1, x2, 0, fk) * kZ;   // visit-0 lane bases (bytes)
    int lb1 = view_pos<P, 0, 1>(x1, x2, 0, fk) * kZ;
    int lbj = view_pos<P, 0, 2>(x1, x2, 0, fk) * kZ;
    int mb0 = view_pos<P, 1, 0>(x1, x2, 0, fk) * kZ;   // visit-1 lane bases
    int mb1 = view_pos<P, 1, 1>(x1, x2, 0, fk) * kZ;
    int mbj = view_pos<P, 1, 2>(x1, x2, 0, fk) * kZ;
    SkipMask sk;
    sk.m8 = 0xFFu << (8 * w);
    sk.m33 = 0x33u << (8 * w);
    sk.m1 = 0x1111u << w;
    const gptr<const GT> vals = (gptr<const GT>)a.vals;
    const gptr<const OT> Xo = (gptr<const OT>)a.X;
    const gptr<const double> So = (gptr<const double>)a.S;
    const gptr<const EntryRecord> rec = (gptr<const EntryRecord>)a.rec;
    if (it.e1 <= it.e0) return;  // padding item

    // persistent FP64 sums: the K-run pair, J_IJ, and the L pairs
    d4 pK0 = d4{0, 0, 0, 0}, pK1 = d4{0, 0, 0, 0};
    JVal<P, JW> pJ = {};
    d4 hA[NB], hB[NB];
    int lsa[NB], lsb[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        hA[p] = d4{0, 0, 0, 0};
        hB[p] = d4{0, 0, 0, 0};
        lsa[p] = -1;
        lsb[p] = -1;
    }
    int run_key = -1, run_ka = 0, run_kb = 0;
    GT pv[16];   // the block's values in flight (store precision)
    static_assert(sizeof(OT) * kOpElems == 2 * kThreads * 16 && sizeof(double) * kSE<JW> == kThreads * 16,
                  "operand tile chunking");
    u4 pb0[2], pb1[2], pbs, pc0[2], pc1[2];
    int cnt = 0, myrank = -1;
    int64_t blk_off = 0;
    int blk_K = 0, blk_L = 0;
    bool was_present = true;
    int fetched_K = -1;   // K of the last fetched block: X_JK, X_IK are reloaded when it changes
    bool newK = false;    // the fetched block starts a new K (its X_JK, X_IK are in pc0, pc1)
    double kp0 = 0.0, kp1 = 0.0;   // integral-direct: the fetched block's ket pair data
    double blk_w = 0.0;            // integral-direct: its weight
    auto fetch = [&](const Rec& r) {
        const uint64_t m0 = r.mask[0], m1 = r.mask[1], m2 = r.mask[2], m3 = r.mask[3];
        const uint64_t mw = w == 0 ? m0 : w == 1 ? m1 : w == 2 ? m2 : m3;
        int rank = (w > 0 ? __popcll(m0) : 0) + (w > 1 ? __popcll(m1) : 0) + (w > 2 ? __popcll(m2) : 0);
        rank += __builtin_amdgcn_mbcnt_hi((uint32_t)(mw >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mw, 0u));
        myrank = ((mw >> lane) & 1) ? rank : -1;
        cnt = __popcll(m0) + __popcll(m1) + __popcll(m2) + __popcll(m3);
        const int K = r.K, L = r.L;
        if constexpr (P == 3) {
            blk_off = r.off;
            blk_K = K;
            blk_L = L;
            load_pairs((const double*)a.vals, a.nslots, K, L, tid, kp0, kp1);
            const int64_t nss = (int64_t)a.nslots * a.nslots;
            blk_w = ((gptr<const double>)a.vals)[kDirectArrays * nss + r.off];
        } else {
            if (myrank >= 0) sSel[myrank] = (uint16_t)(gran_base<kF32>(tid) * kZ);
            if (tid >= cnt) {
                const int q = ~m0 ? 0 : ~m1 ? 1 : ~m2 ? 2 : 3;
                const uint64_t mq = q == 0 ? m0 : q == 1 ? m1 : q == 2 ? m2 : m3;
                const int gabs = 64 * q + __builtin_ctzll(~mq | (1ull << 63));
                sSel[tid] = (uint16_t)(gran_base<kF32>(gabs) * kZ);
            }
            const gptr<const GT> src = vals + r.off * 16;
            const int nval = cnt * 16;
#pragma unroll
            for (int x = 0; x < 16; ++x)
                if (x * kThreads < nval) pv[x] = __builtin_nontemporal_load(src + x * kThreads + tid);
        }
        // visit-0 operands of every block: X_JL, X_IL, S_KL
        const gptr<const u4> X0c = (gptr<const u4>)(Xo + ((int64_t)J * T + L) * kOpElems);
        const gptr<const u4> X1c = (gptr<const u4>)(Xo + ((int64_t)I * T + L) * kOpElems);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            pb0[x] = X0c[x * kThreads + tid];
            pb1[x] = X1c[x * kThreads + tid];
        }
        pbs = ((gptr<const u4>)(So + ((int64_t)K * T + L) * kSE<JW>))[tid];
        // visit-1 K operands X_JK, X_IK when K changes
        newK = K != fetched_K;
        if (newK) {
            const gptr<const u4> X2c = (gptr<const u4>)(Xo + ((int64_t)J * T + K) * kOpElems);
            const gptr<const u4> X3c = (gptr<const u4>)(Xo + ((int64_t)I * T + K) * kOpElems);
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                pc0[x] = X2c[x * kThreads + tid];
                pc1[x] = X3c[x * kThreads + tid];
            }
            fetched_K = K;
        }
    };

    Rec rc = load_rec(rec + it.e0);
    uint32_t wn = load_rec_word(rec + (it.e0 + 1 < it.e1 ? it.e0 + 1 : it.e0), lane);
    // S_IJ, the operand of J_KL, is the item's own bra pair: staged once
    ((u4*)sS1)[tid] = ((gptr<const u4>)(So + ((int64_t)I * T + J) * kSE<JW>))[tid];
    if constexpr (P == 3) {  // and so are the bra's pair data
        double b0, b1;
        load_pairs((const double*)a.vals, a.nslots, I, J, tid, b0, b1);
        store_pairs(sPair, tid, b0, b1);
    }
    fetch(rc);
    __syncthreads();
    JVal<P, JW> jk_prev = {};
    int jslot_prev = -1;
    LoPack lp;  // modes 1 and 4: packed lo operands of the current four steps
    for (int e = it.e0; e < it.e1; ++e) {
        const int key = rc.K;
        const bool run_ends = key != run_key && run_key >= 0;
        const int jslot = rc.jslot;
        const int bpos = rc.bpos;
        if constexpr (SKIP == 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                sk.d[2 * q] = (uint32_t)rc.mask[q];
                sk.d[2 * q + 1] = (uint32_t)(rc.mask[q] >> 32);
            }
            const uint64_t mw = w == 0 ? rc.mask[0] : w == 1 ? rc.mask[1] : w == 2 ? rc.mask[2] : rc.mask[3];
            sk.orw = (uint32_t)mw | (uint32_t)(mw >> 32);
        }
        char* const sVb = (char*)sV;
        const bool refill = myrank < 0 && was_present;
        was_present = myrank >= 0;
        if (refill) {
            int gbase = gran_base<kF32>(tid) * kZ;
            asm("" : "+v"(gbase) : "s"(e));
#pragma unroll
            for (int u = 0; u < 16; ++u) *(ET*)(sVb + (gbase ^ (gran_bits<kF32>(u) * kZ))) = (ET)0;
        }
        if constexpr (P == 3) {
            // the block's ket pair data into LDS, then each present granule's
            // 16 integrals (a barrier between: threads read all 64 pairs)
            store_pairs(sPair + kDirectArrays * 64, tid, kp0, kp1);
            __syncthreads();
            if (myrank >= 0) direct_granule_lds((double*)sV, sPair, blk_w, a.tau, tid);
        } else {
            const int ub = gran_bits<kF32>(tid & 15) * kZ;
            int gsel[16];
#pragma unroll
            for (int x = 0; x < 16; ++x) gsel[x] = sSel[16 * x + (tid >> 4)];
#pragma unroll
            for (int x = 0; x < 16; ++x)
                if (16 * x < cnt) *(ET*)(sVb + (gsel[x] ^ ub)) = (ET)pv[x];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            ((u4*)sX0)[x * kThreads + tid] = pb0[x];
            ((u4*)sX1)[x * kThreads + tid] = pb1[x];
        }
        ((u4*)sS0)[tid] = pbs;
        if (newK) {
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                ((u4*)sX2)[x * kThreads + tid] = pc0[x];
                ((u4*)sX3)[x * kThreads + tid] = pc1[x];
            }
        }
        if (run_ends) {
            store_partial_k<P>(a, run_ka, w, pK0, lane);
            store_partial_k<P>(a, run_kb, w, pK1, lane);
            pK0 = d4{0, 0, 0, 0};
            pK1 = d4{0, 0, 0, 0};
        }
        if (key != run_key) {
            run_ka = rc.kslot_a;
            run_kb = rc.kslot_b;
        }
        run_key = key;
        if (jslot_prev >= 0) store_partial_j<P, JW>(a, jslot_prev, w, jk_prev, lane);
        // the L slots of this block's band position (the same for every block
        // of the item at that position)
#pragma unroll
        for (int p = 0; p < NB; ++p)
            if (p == bpos) {
                lsa[p] = rc.lslot_a;
                lsb[p] = rc.lslot_b;
            }
        __syncthreads();
        asm("" : "+v"(lb0), "+v"(lb1), "+v"(lbj), "+v"(mb0), "+v"(mb1), "+v"(mbj) : "s"(e));
        const Frag<P, JW, 0> f0 = load_frag<P, 0, JW, 0, 0>(sV, sX0, sX1, sS0, lane, lb0, lb1, lbj);
        if (e + 1 < it.e1) {
            const Rec rn = unpack_rec(wn);
            wn = load_rec_word(rec + (e + 2 < it.e1 ? e + 2 : e + 1), lane);
            fetch(rn);
            rc = rn;
        }
        {   // visit-0 views into the K-run pair and J_IJ
            Acc<P> c0, c1;
            AccJ<P, JW> cj;
            c0.zero();
            c1.zero();
            cj.zero();
            c0.d = pK0;
            c1.d = pK1;
            cj.d = pJ;
            k_steps<P, 0, SKIP, CHAIN, JW, 0>(sV, sX0, sX1, sS0, lane, lb0, lb1, lbj, sk, c0, c1, cj, f0, lp);
            c0.drain_all();
            c1.drain_all();
            cj.drain_all();
            pK0 = c0.d;
            pK1 = c1.d;
            pJ = cj.d;
        }
        {   // visit-1 views into the band position's L pair and this block's J_KL
            Acc<P> c0, c1;
            AccJ<P, JW> cj;
            c0.zero();
            c1.zero();
            cj.zero();
#pragma unroll
            for (int p = 0; p < NB; ++p)
                if (p == bpos) {
                    c0.d = hA[p];
                    c1.d = hB[p];
                }
            const Frag<P, JW, 0> g0 = load_frag<P, 1, JW, 0, 0>(sV, sX2, sX3, sS1, lane, mb0, mb1, mbj);
            k_steps<P, 1, SKIP, CHAIN, JW, 0>(sV, sX2, sX3, sS1, lane, mb0, mb1, mbj, sk, c0, c1, cj, g0, lp);
            c0.drain_all();
            c1.drain_all();
            cj.drain_all();
#pragma unroll
            for (int p = 0; p < NB; ++p)
                if (p == bpos) {
                    hA[p] = c0.d;
                    hB[p] = c1.d;
                }
            jk_prev = cj.d;
            jslot_prev = jslot;
        }
        __syncthreads();
    }
    if (jslot_prev >= 0) store_partial_j<P, JW>(a, jslot_prev, w, jk_prev, lane);
    if (run_key >= 0) {
        store_partial_k<P>(a, run_ka, w, pK0, lane);
        store_partial_k<P>(a, run_kb, w, pK1, lane);
    }
    store_partial_j<P, JW>(a, it.jslot0, w, pJ, lane);
#pragma unroll
    for (int p = 0; p < NB; ++p)
        if (lsa[p] >= 0) {
            store_partial_k<P>(a, lsa[p], w, hA[p], lane);
            store_partial_k<P>(a, lsb[p], w, hB[p], lane);
        }
}

// The fused contraction: one workgroup per fused work item (same grid and
// XCD mapping as fock_mfma_kernel), LDS for the block and six operand tiles.
template <int P, int SKIP, int OCC, int CHAIN, int NB>
__global__ void __launch_bounds__(kThreads, OCC)
fock_fused_kernel(const UnitDesc* __restrict__ units, int unit_base, const WorkItem* __restrict__ items,
                  int item_base) {
    using ET = typename Prec<P>::ET;
    using OT = typename Prec<P>::OT;
    __shared__ ET sV[4096];
    __shared__ __attribute__((aligned(16))) OT sX0[kOpElems];   // X_JL
    __shared__ __attribute__((aligned(16))) OT sX1[kOpElems];   // X_IL
    __shared__ __attribute__((aligned(16))) OT sX2[kOpElems];   // X_JK
    __shared__ __attribute__((aligned(16))) OT sX3[kOpElems];   // X_IK
    __shared__ __attribute__((aligned(16))) double sS0[kSE<8>];   // S_KL
    __shared__ __attribute__((aligned(16))) double sS1[kSE<8>];   // S_IJ
    __shared__ uint16_t sSel[kGranules];
    __shared__ double sPair[P == 3 ? kPairLds : 1];   // integral-direct: bra and ket pair data
    const WorkItem it = items[item_base + blockIdx.x];
    const UnitDesc* up = units + unit_base + it.unit;
    UnitDesc u;
    u.vals = up->vals;
    u.rec = up->rec;
    u.X = up->X;
    u.S = up->S;
    u.PK = up->PK;
    u.PJ = up->PJ;
    u.ntiles = up->ntiles;
    if constexpr (P == 3) {
        u.nslots = up->nslots;
        u.tau = up->tau;
    }
    run_item_fused<P, SKIP, CHAIN, NB>(u, it, sV, sX0, sX1, sX2, sX3, sS0, sS1, sSel, sPair);
}

// One workgroup per work item: item item_base + b on workgroup b (item_base
// a multiple of 8, so item i runs on XCD i % 8).  Item `unit` selects the
// molecule and density group; `unit_base` offsets it.  (A persistent loop
// over items keeps the per-lane LDS addressing live across items and spills.)
// JW: J width of every unit of the launch (8 narrow, 16 wide).
template <int P, int SKIP, int OCC, int CHAIN, int JW>
__global__ void __launch_bounds__(kThreads, OCC)
fock_mfma_kernel(const UnitDesc* __restrict__ units, int unit_base,
                 const WorkItem* __restrict__ items, int item_base) {
    using ET = typename Prec<P>::ET;
    using OT = typename Prec<P>::OT;
    __shared__ ET sV[4096];
    __shared__ __attribute__((aligned(32))) OT sB0[kOpElems];   // operand of the first K view
    __shared__ __attribute__((aligned(32))) OT sB1[kOpElems];   // operand of the second K view
    __shared__ __attribute__((aligned(16))) double sBJ[kSE<JW>];  // operand of the J view
    __shared__ uint16_t sSel[kGranules];  // rank of a present granule -> its LDS byte offset
    {
        const WorkItem it = items[item_base + blockIdx.x];
        const UnitDesc* up = units + unit_base + it.unit;
        UnitDesc u;
        u.vals = up->vals;
        u.rec = up->rec;
        u.X = up->X;
        u.S = up->S;
        u.PK = up->PK;
        u.PJ = up->PJ;
        u.ntiles = up->ntiles;
        if constexpr (P == 3) {
            u.nslots = up->nslots;
            u.tau = up->tau;
        }
        // the unit's K column set (uniform over the workgroup)
        if constexpr (kNarrowK<P> && JW == 8) {
            const int kq = up->kq;
            if (kq == 1) {
                if (it.visit == 0) run_item<P, 0, SKIP, CHAIN, JW, 1>(u, it, sV, sB0, sB1, sBJ, sSel);
                else run_item<P, 1, SKIP, CHAIN, JW, 1>(u, it, sV, sB0, sB1, sBJ, sSel);
                return;
            }
            if (kq == 2) {
                if (it.visit == 0) run_item<P, 0, SKIP, CHAIN, JW, 2>(u, it, sV, sB0, sB1, sBJ, sSel);
                else run_item<P, 1, SKIP, CHAIN, JW, 2>(u, it, sV, sB0, sB1, sBJ, sSel);
                return;
            }
        }
        if (it.visit == 0)
            run_item<P, 0, SKIP, CHAIN, JW, 0>(u, it, sV, sB0, sB1, sBJ, sSel);
        else
            run_item<P, 1, SKIP, CHAIN, JW, 0>(u, it, sV, sB0, sB1, sBJ, sSel);
    }
}

// Up to four unit descriptors passed by value (kernel arguments are copied at
// launch, so the host array may go away right after) into device memory.
struct UnitChunk {
    UnitDesc u[4];
    int n;
};
__global__ void store_units_kernel(UnitChunk c, UnitDesc* dst) {
    if ((int)threadIdx.x < c.n) dst[threadIdx.x] = c.u[threadIdx.x];
}

__global__ void copy_items_kernel(const WorkItem* __restrict__ src, int n, WorkItem* __restrict__ dst,
                                  int npad, int unit) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    WorkItem it;
    if (i < n) {
        it = src[i];
    } else {
        it.e0 = it.e1 = 0;   // empty: the contraction skips it
        it.I = it.J = it.visit = it.reserved = it.jslot0 = 0;
    }
    it.unit = unit;
    dst[i] = it;
}

// unit of a launch-wide index: the last unit whose start is <= idx
template <typename F>
__device__ __forceinline__ int find_unit(int n, int64_t idx, F start) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (start(mid) <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Operand tiles of a density group: for every used tile pair (A, B),
//   X[A][B][(a,b)][c] = D_{c0+p}[A_a][B_b], or D_{c0+p}[B_b][A_a] for a
//                       transposed column, p = the column's source density
//   S[A][B][(a,b)][c] = D_{c0+c}[A_a][B_b] + D_{c0+c}[B_b][A_a]  (c < jw)
// with zeros for ghost slots, unused columns and densities beyond the group.
// (Narrow groups without symmetric densities: X columns D_0..D_7 | D_0^T..D_7^T.)
// Mixed: each value x is stored as the FP32 pair (hi, lo), hi = fp32(x),
// lo = fp32(x - hi).
template <bool SPLIT>
__global__ void prep_operands_kernel(const UnitDesc* __restrict__ units, int unit_base, int nunits,
                                     int64_t total, int64_t base) {
    using OT = typename Prec<SPLIT ? 1 : 0>::OT;
    const int64_t bidx = base + blockIdx.x;
    const int64_t gidx = bidx * blockDim.x + threadIdx.x;
    if (gidx >= total) return;
    // Every unit's range starts at a multiple of kOpElems (nused * kOpElems
    // indices each), so the 256 threads of a block lie in one unit: the
    // search takes the block's first index, a uniform value.
    static_assert(kOpElems % 256 == 0, "a prep block must not straddle two units");
    const UnitDesc& u = units[unit_base + find_unit(nunits, bidx * 256, [&](int x) {
        return units[unit_base + x].prep_begin;
    })];
    const int64_t li = gidx - u.prep_begin;
    const int ntiles = u.ntiles, nbf = u.nbf, mg = u.mg, c0 = u.c0;
    const gptr<const int32_t> slot_fn = (gptr<const int32_t>)u.slot_fn;
    const gptr<const double> d = (gptr<const double>)u.d;
    const gptr<OT> X = (gptr<OT>)u.X;
    const gptr<double> S = (gptr<double>)u.S;
    if (li >= (int64_t)u.nused * kOpElems) return;
    // only tile pairs some block reads are prepared (the others are never read)
    const int64_t tp = ((gptr<const int32_t>)u.used)[li / kOpElems];
    const int64_t idx = tp * kOpElems + li % kOpElems;
    const int c = (int)(idx % kCols);
    // X column at this position: a narrow K column set (kq > 0) interleaves
    // its rows (column cx at 4 (cx % 4) + cx / 4, an involution)
    const int cx = u.kq > 0 ? 4 * (c & 3) + (c >> 2) : c;
    const int ab = (int)((idx / kCols) % 64);
    const int A = (int)(tp / ntiles), B = (int)(tp % ntiles);
    const int fa = slot_fn[A * 8 + (ab >> 3)], fb = slot_fn[B * 8 + (ab & 7)];
    const int jw = u.jw;
    const int xs = u.xsrc[cx];
    const int64_t nn = (int64_t)nbf * nbf;
    double x = 0.0, s = 0.0;
    if (fa >= 0 && fb >= 0) {
        if (xs >= 0) {
            const gptr<const double> Dp = d + (int64_t)(c0 + (xs & 31)) * nn;
            x = (xs & kXsrcTransposed) ? Dp[(int64_t)fb * nbf + fa] : Dp[(int64_t)fa * nbf + fb];
        }
        if (c < mg) {
            const gptr<const double> Dc = d + (int64_t)(c0 + c) * nn;
            s = Dc[(int64_t)fa * nbf + fb] + Dc[(int64_t)fb * nbf + fa];
        }
    }
    if constexpr (SPLIT) {
        const float xh = (float)x;
        X[idx] = f2{xh, (float)(x - (double)xh)};
    } else {
        X[idx] = x;
    }
    // the J operand is FP64 in every mode; a narrow one holds column c at
    // 2 (c % 4) + c / 4, so that the two 4x4x4 products' columns l % 4 and
    // 4 + l % 4 are adjacent
    if (c < jw) S[tp * 64 * jw + ab * jw + (jw == 8 ? 2 * (c & 3) + (c >> 2) : c)] = s;
}

// Reduction of the partial tiles of one density group.  One workgroup per
// unordered tile pair X >= Y that receives any partial (the unit's pair
// list); it owns the output tiles (X, Y) and (Y, X), whose other elements a
// clearing pass has zeroed.  The partial slots of a target are contiguous, so each list is read
// as a stream of whole slots: a [64][16] K slot of target (A, B) holds, for
// density c, K[A][B] rows (a, b) in its forward column f = kf[c] and K[B][A]
// transposed in its transposed column t = kt[c] (f = t for a symmetric
// density: its transposed partials equal the forward ones); a [64][jw] J slot
// of canonical (A, B) holds J[A][B] rows (a, b) in column c.  Then
//   K[X][Y]_xy,c = sum_{kl(X,Y)} P[(x,y)][f]   + sum_{kl(Y,X)} P[(y,x)][t]
//   K[Y][X]_yx,c = sum_{kl(Y,X)} P[(y,x)][f]   + sum_{kl(X,Y)} P[(x,y)][t]
//   J[X][Y]_xy,c = J[Y][X]_yx,c = sum_{jl(X,Y)} PJ[(x,y)][c]                (X > Y)
//   J[X][X]_xy,c = sum_{jl(X,X)} PJ[(x,y)][c] + sum_{jl(X,X)} PJ[(y,x)][c]
// each list summed in slot order, the two sums added last: fixed order.
__device__ __forceinline__ void sum_slots(gptr<const double> P, int64_t stride, int64_t q0, int64_t q1,
                                          int nvec, d2* acc) {
    for (int v = 0; v < nvec; ++v) acc[v] = d2{0.0, 0.0};
    int64_t q = q0;
    for (; q + 4 <= q1; q += 4) {
        d2 t[4][2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
                if (v < nvec) t[u][v] = *(gptr<const d2>)(P + (q + u) * stride + 2 * v);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v)
                if (v < nvec) acc[v] += t[u][v];
    }
    for (; q < q1; ++q)
#pragma unroll
        for (int v = 0; v < 2; ++v)
            if (v < nvec) acc[v] += *(gptr<const d2>)(P + q * stride + 2 * v);
}

__global__ void __launch_bounds__(256)
reduce_partials_kernel(const UnitDesc* __restrict__ units, int unit_base, int nunits, int base) {
    const int bidx = base + (int)blockIdx.x;
    const UnitDesc& u = units[unit_base + find_unit(nunits, bidx, [&](int x) {
        return (int64_t)units[unit_base + x].red_begin;
    })];
    const int pr = bidx - u.red_begin;
    const int ntiles = u.ntiles, nbf = u.nbf, mg = u.mg, c0 = u.c0;
    if (pr >= u.nred) return;
    const int tile = ((gptr<const int32_t>)u.red)[pr];
    const int X = tile / ntiles, Y = tile % ntiles;
    const gptr<const double> PK = (gptr<const double>)u.PK;
    const gptr<const double> PJ = (gptr<const double>)u.PJ;
    const gptr<const int64_t> kptr = (gptr<const int64_t>)u.kptr;
    const gptr<const int64_t> jptr = (gptr<const int64_t>)u.jptr;
    const gptr<const int32_t> slot_fn = (gptr<const int32_t>)u.slot_fn;
    const gptr<double> J = (gptr<double>)u.j;
    const gptr<double> K = (gptr<double>)u.k;
    __shared__ __attribute__((aligned(16))) double sA[64 * 16];  // sum over kl(X, Y)
    __shared__ __attribute__((aligned(16))) double sB[64 * 16];  // sum over kl(Y, X)
    __shared__ __attribute__((aligned(16))) double sJ[64 * 16];  // sum over jl(X, Y)
    const int t = threadIdx.x;
    const int row = t >> 2, q4 = t & 3;
    const int tp = X * ntiles + Y, tq = Y * ntiles + X;
    {
        d2 acc[2];
        // K: thread (row, q4) streams columns 4 q4 .. 4 q4 + 3 of its row
        sum_slots(PK + row * kCols + 4 * q4, kOpElems, kptr[tp], kptr[tp + 1], 2, acc);
        *(d2*)(sA + row * 16 + 4 * q4) = acc[0];
        *(d2*)(sA + row * 16 + 4 * q4 + 2) = acc[1];
        if (X != Y) {
            sum_slots(PK + row * kCols + 4 * q4, kOpElems, kptr[tq], kptr[tq + 1], 2, acc);
            *(d2*)(sB + row * 16 + 4 * q4) = acc[0];
            *(d2*)(sB + row * 16 + 4 * q4 + 2) = acc[1];
        }
        // J: columns jw/4 q4 .. jw/4 q4 + jw/4 - 1 of its row
        const int jw = u.jw;
        sum_slots(PJ + row * jw + (jw / 4) * q4, 64 * jw, jptr[tp], jptr[tp + 1], jw / 8, acc);
        *(d2*)(sJ + row * 16 + (jw / 4) * q4) = acc[0];
        if (jw == 16) *(d2*)(sJ + row * 16 + 4 * q4 + 2) = acc[1];
    }
    __syncthreads();
    const double* sBX = X != Y ? sB : sA;
    const int x = row >> 3, y = row & 7;
    const int64_t nn = (int64_t)nbf * nbf;
    const int fx = slot_fn[X * 8 + x], fy = slot_fn[Y * 8 + y];
    if (fx < 0 || fy < 0) return;
    const int per = u.jw / 4;  // densities per thread
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        const int c = per * q4 + cc;
        if (cc >= per || c >= mg) continue;
        const int yx = y * 8 + x;
        const int f = u.kf[c], t = u.kt[c];
        const double kxy = sA[row * 16 + f] + sBX[yx * 16 + t];
        const double jxy = X != Y ? sJ[row * 16 + c] : sJ[row * 16 + c] + sJ[yx * 16 + c];
        K[(int64_t)(c0 + c) * nn + (int64_t)fx * nbf + fy] = kxy;
        J[(int64_t)(c0 + c) * nn + (int64_t)fx * nbf + fy] = jxy;
        if (X != Y) {
            const double kyx = sB[yx * 16 + f] + sA[row * 16 + t];
            K[(int64_t)(c0 + c) * nn + (int64_t)fy * nbf + fx] = kyx;
            J[(int64_t)(c0 + c) * nn + (int64_t)fy * nbf + fx] = jxy;
        }
    }
}

// Clearing of the unit's outputs (densities c0 .. c0 + mg - 1 of J and K);
// the reduction then writes the tile pairs that received partials.
__global__ void zero_outputs_kernel(const UnitDesc* __restrict__ units, int unit_base, int nunits,
                                    int64_t total, int64_t base) {
    const int64_t gidx = (base + blockIdx.x) * blockDim.x + threadIdx.x;
    if (gidx >= total) return;
    const UnitDesc& u = units[unit_base + find_unit(nunits, gidx, [&](int x) {
        return units[unit_base + x].zero_begin;
    })];
    const int64_t i = gidx - u.zero_begin;
    const int64_t off = (int64_t)u.c0 * u.nbf * u.nbf + i;
    ((gptr<double>)u.j)[off] = 0.0;
    ((gptr<double>)u.k)[off] = 0.0;
}

__global__ void build_records_kernel(int64_t n, const int32_t* __restrict__ entries,
                                     const int32_t* __restrict__ blk_tiles,
                                     const uint64_t* __restrict__ mask,
                                     const int64_t* __restrict__ off,
                                     const int32_t* __restrict__ eslot, EntryRecord* rec) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t b = entries[e];
    const int32_t* es = eslot + (int64_t)kSlotFields * e;
    EntryRecord r;
    for (int x = 0; x < 4; ++x) r.mask[x] = mask[4 * b + x];
    r.off = off[b];
    const uint32_t bpos = es[kSlotBpos] < 0 ? 0u : (uint32_t)es[kSlotBpos];
    r.kl = (uint32_t)blk_tiles[4 * b + 2] | ((uint32_t)blk_tiles[4 * b + 3] << 13) | (bpos << 26);
    r.kslot_a = es[kSlotKA];
    r.kslot_b = es[kSlotKB];
    r.jslot = es[kSlotJ];
    r.lslot_a = es[kSlotLA];
    r.lslot_b = es[kSlotLB];
    rec[e] = r;
}

template <int P, int SKIP, int OCC>
void launch_main(const UnitDesc* units, int unit_base, const WorkItem* items, int item_base,
                 int chain, int grid, hipStream_t s) {
    if constexpr (!kMixed<P>) {
        (void)chain;
        fock_mfma_kernel<P, SKIP, OCC, 4, 8><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base);
    } else {
        switch (chain) {
            case 1: fock_mfma_kernel<P, SKIP, OCC, 1, 8><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base); break;
            case 2: fock_mfma_kernel<P, SKIP, OCC, 2, 8><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base); break;
            case 8: fock_mfma_kernel<P, SKIP, OCC, 8, 8><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base); break;
            default: fock_mfma_kernel<P, SKIP, OCC, 4, 8><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base); break;
        }
    }
}

// The fused contraction; modes 1 and 4 with FP32 chains of 2 or 4 steps.
template <int P, int SKIP, int NB>
void launch_fused(const UnitDesc* units, int unit_base, const WorkItem* items, int item_base, int chain, int grid,
                  hipStream_t s) {
    if constexpr (kMixed<P>) {
        if (chain <= 2) {
            fock_fused_kernel<P, SKIP, 2, 2, NB><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base);
            return;
        }
    }
    (void)chain;
    fock_fused_kernel<P, SKIP, 2, 4, NB><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base);
}

// Wide groups (16 J columns) run one fixed variant: zero-fragment skip, the
// variant's FP32 chain length in modes 1 and 4 (2 or 4, so that a wide group rounds
// as a narrow one does), and as many workgroups per CU as their LDS allows
// (the J operand takes 8 KB instead of 4): 2 with FP64 integrals in LDS
// (56.5 KB), 3 with FP32 ones (40.5 KB).
template <int P>
constexpr int kWideOcc = kLds32<P> ? 3 : 2;

template <int P>
void launch_variant(const UnitDesc* units, int unit_base, const WorkItem* items, int item_base,
                    const KernelVariant& v, int jw, int grid, hipStream_t s) {
    if (jw == 16) {
        if constexpr (kMixed<P>) {
            if (v.chain <= 2) {
                fock_mfma_kernel<P, 1, kWideOcc<P>, 2, 16><<<grid, kThreads, 0, s>>>(units, unit_base, items,
                                                                                    item_base);
                return;
            }
        }
        fock_mfma_kernel<P, 1, kWideOcc<P>, 4, 16><<<grid, kThreads, 0, s>>>(units, unit_base, items, item_base);
        return;
    }
    if (v.plan == kPlanFused) {
        // the block and six operand tiles take 56.5-72.5 KB of LDS: two
        // workgroups per CU
        if (v.band <= 2) {
            if (v.skip_zero_fragments)
                launch_fused<P, 1, 2>(units, unit_base, items, item_base, v.chain, grid, s);
            else
                launch_fused<P, 0, 2>(units, unit_base, items, item_base, v.chain, grid, s);
        } else {
            if (v.skip_zero_fragments)
                launch_fused<P, 1, kFusedBand>(units, unit_base, items, item_base, v.chain, grid, s);
            else
                launch_fused<P, 0, kFusedBand>(units, unit_base, items, item_base, v.chain, grid, s);
        }
        return;
    }
    if constexpr (P == 2) {  // STORE32 fits 4 workgroups per CU in registers and LDS
        if (v.skip_zero_fragments && v.occupancy >= 4) {
            launch_main<P, 1, 4>(units, unit_base, items, item_base, v.chain, grid, s);
            return;
        }
    }
    if (v.skip_zero_fragments) {
        if (v.occupancy >= 3)
            launch_main<P, 1, 3>(units, unit_base, items, item_base, v.chain, grid, s);
        else
            launch_main<P, 1, 2>(units, unit_base, items, item_base, v.chain, grid, s);
    } else {
        if (v.occupancy >= 3)
            launch_main<P, 0, 3>(units, unit_base, items, item_base, v.chain, grid, s);
        else
            launch_main<P, 0, 2>(units, unit_base, items, item_base, v.chain, grid, s);
    }
}

}  // namespace

hipError_t launch_build_records(int64_t n, const int32_t* d_entries, const int32_t* d_blk_tiles,
                                const uint64_t* d_mask, const int64_t* d_off, const int32_t* d_eslot,
                                EntryRecord* d_rec, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    build_records_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, d_entries, d_blk_tiles,
                                                                    d_mask, d_off, d_eslot, d_rec);
    return hipGetLastError();
}

hipError_t launch_copy_items(const WorkItem* src, int n, WorkItem* dst, int npad, int unit,
                             hipStream_t s) {
    if (npad <= 0) return hipSuccess;
    copy_items_kernel<<<(npad + 255) / 256, 256, 0, s>>>(src, n, dst, npad, unit);
    return hipGetLastError();
}

hipError_t launch_store_units(const UnitDesc* h, int n, UnitDesc* d, hipStream_t s) {
    for (int x = 0; x < n; x += 4) {
        UnitChunk c;
        c.n = n - x < 4 ? n - x : 4;
        for (int y = 0; y < c.n; ++y) c.u[y] = h[x + y];
        store_units_kernel<<<1, 64, 0, s>>>(c, d + x);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t operand_bytes(int ntiles, int jw) {
    return sizeof(double) * (size_t)ntiles * ntiles * (kOpElems + 64 * (size_t)jw);
}

size_t partial_bytes(int64_t nkslots, int64_t njslots, int jw) {
    return sizeof(double) * ((size_t)nkslots * kOpElems + (size_t)njslots * 64 * (size_t)jw);
}

void unit_set_workspace(UnitDesc& u, double* operands, double* partials, int64_t nkslots) {
    const size_t T = (size_t)u.ntiles;
    u.X = operands;
    u.S = operands + T * T * kOpElems;
    u.PK = partials;
    u.PJ = partials + (size_t)nkslots * kOpElems;
}

int64_t unit_prep_size(const UnitDesc& u) { return (int64_t)u.nused * kOpElems; }

int64_t unit_zero_size(const UnitDesc& u) { return (int64_t)u.mg * u.nbf * u.nbf; }

constexpr int64_t kGridChunk = (int64_t)1 << 22;

hipError_t launch_units(const UnitDesc* d_units, int unit_base, int nunits, int64_t prep_total,
                        int64_t zero_total, int red_total, const WorkItem* d_items, int nitems, int mode,
                        const KernelVariant& variant, hipStream_t s, hipEvent_t ev_start,
                        hipEvent_t ev_stop, int jw) {
    // A launch holds fewer than 2^32 work items: grids of 256-thread
    // workgroups go in chunks of kGridChunk workgroups.
    const int64_t pgrid = (prep_total + 255) / 256;
    for (int64_t b0 = 0; b0 < pgrid; b0 += kGridChunk) {
        const unsigned g = (unsigned)std::min<int64_t>(kGridChunk, pgrid - b0);
        if (mode == 1 || mode == 4)
            prep_operands_kernel<true><<<g, 256, 0, s>>>(d_units, unit_base, nunits, prep_total, b0);
        else
            prep_operands_kernel<false><<<g, 256, 0, s>>>(d_units, unit_base, nunits, prep_total, b0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_start) {
        e = hipEventRecord(ev_start, s);
        if (e != hipSuccess) return e;
    }
    // chunks of at most 8M workgroups (a multiple of 8)
    constexpr int kChunk = 1 << 23;
    for (int base = 0; base < nitems; base += kChunk) {
        const int grid = nitems - base < kChunk ? nitems - base : kChunk;
        if (mode == 1)
            launch_variant<1>(d_units, unit_base, d_items, base, variant, jw, grid, s);
        else if (mode == 2)
            launch_variant<2>(d_units, unit_base, d_items, base, variant, jw, grid, s);
        else if (mode == 3)
            launch_variant<3>(d_units, unit_base, d_items, base, variant, jw, grid, s);
        else if (mode == 4)
            launch_variant<4>(d_units, unit_base, d_items, base, variant, jw, grid, s);
        else
            launch_variant<0>(d_units, unit_base, d_items, base, variant, jw, grid, s);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (ev_stop) {
        e = hipEventRecord(ev_stop, s);
        if (e != hipSuccess) return e;
    }
    const int64_t zgrid = (zero_total + 255) / 256;
    for (int64_t b0 = 0; b0 < zgrid; b0 += kGridChunk)
        zero_outputs_kernel<<<(unsigned)std::min<int64_t>(kGridChunk, zgrid - b0), 256, 0, s>>>(
            d_units, unit_base, nunits, zero_total, b0);
    for (int b0 = 0; b0 < red_total; b0 += (int)kGridChunk)
        reduce_partials_kernel<<<(unsigned)std::min<int64_t>(kGridChunk, red_total - b0), 256, 0, s>>>(
            d_units, unit_base, nunits, b0);
    return hipGetLastError();
}

}  // namespace esmf
