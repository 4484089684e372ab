// Tuned grouped J/K build for gfx950: FP64 matrix cores (v_mfma_f64_16x16x4).
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
// J_KL[(k,l)][c] += sum_(i,j) v S_IJ[(i,j)][c] (view V1^T), J being
// symmetrised afterwards.
//
// Every block is visited twice, both times from its bra tile pair IJ:
//   visit 0: blocks of bra IJ in runs of equal K  -> (I,K), (J,K) and J_IJ
//   visit 1: blocks of bra IJ in runs of equal L  -> (I,L), (J,L) and J_KL
// so the K targets of a visit stay in matrix-core accumulators for a whole run
// and J_IJ for the whole work item; only run ends, work-item ends and J_KL
// (per block) are added to global memory, with FP64 atomics.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace esmf {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kW = 4;                      // waves per workgroup
constexpr int kThreads = 64 * kW;
constexpr int kCols = 16;                  // matrix-core N: 8 densities + 8 transposed
constexpr int kOpElems = 64 * kCols;       // one operand tile [64][16]

// LDS position of v[i][j][k][l]: the natural index with its low four bits
// replaced by a bank function (over GF(2)) chosen so that the 16 lanes of every
// fragment column of all six views hit 16 distinct 8-byte banks:
//   b0 = l0^k0^j1, b1 = l1^k1^j0, b2 = l2^k2^j2, b3 = i0^j0^k0.
__device__ __forceinline__ int vpos(int i, int j, int k, int l) {
    int nat = ((i * 8 + j) * 8 + k) * 8 + l;
    int b0 = (l ^ k ^ (j >> 1)) & 1;
    int b1 = ((l >> 1) ^ (k >> 1) ^ j) & 1;
    int b2 = ((l >> 2) ^ (k >> 2) ^ (j >> 2)) & 1;
    int b3 = (i ^ j ^ k) & 1;
    return (nat & ~15) | (b3 << 3) | (b2 << 2) | (b1 << 1) | b0;
}

// one work item: entries [e0, e1) of the entry list, all with bra (I, J)
struct WorkItem {
    int32_t e0, e1;
    int32_t I, J;
    int32_t visit;
    int32_t pad;
};

struct FockArgs {
    const double* vals;        // block store
    const int32_t* blk_tiles;  // [nblocks][4]
    const int32_t* slot_fn;    // [ntiles*8]
    const int32_t* entries;    // block indices in work order
    const WorkItem* items;
    const double* X;           // [T][T][64][16] operand tiles (D | D^T)
    const double* S;           // [T][T][64][16] S = D + D^T (cols >= mg are 0)
    double* J;                 // [m][N][N] (accumulated at canonical positions)
    double* K;                 // [m][N][N]
    int nbf;
    int ntiles;
    int mg;                    // densities in this group (<= 8)
    int c0;                    // first density of this group
    int nitems;
};

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Matrix-core fragment layout of v_mfma_f64_16x16x4 (lane l of a wave):
//   A[16][4]: l holds A[l % 16][l / 16];  B[4][16]: l holds B[l / 16][l % 16];
//   C[16][16]: element r (0..3) of l holds C[4 r + l / 16][l % 16].
// add a 64x16 accumulator tile held as one row-tile per wave to K:
// rows (a, b) = (row / 8, row % 8) of target tiles (A, B); column c < 8 goes
// to K_c[A_a][B_b], c >= 8 to K_{c-8}[B_b][A_a].
__device__ __forceinline__ void flush_k(const FockArgs& a, int A, int B, int rt, d4 acc,
                                        int lane) {
    const int c = lane & 15;
    const int dens = c & 7;
    if (dens >= a.mg) return;
    const int64_t nn = (int64_t)a.nbf * a.nbf;
    double* Kc = a.K + (int64_t)(a.c0 + dens) * nn;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * r + (lane >> 4);
        const int fa = a.slot_fn[A * 8 + (row >> 3)];
        const int fb = a.slot_fn[B * 8 + (row & 7)];
        if (fa < 0 || fb < 0) continue;
        const double v = acc[r];
        if (v == 0.0) continue;
        if (c < 8)
            unsafeAtomicAdd(Kc + (int64_t)fa * a.nbf + fb, v);
        else
            unsafeAtomicAdd(Kc + (int64_t)fb * a.nbf + fa, v);
    }
}

__device__ __forceinline__ void flush_j(const FockArgs& a, int A, int B, int rt, d4 acc,
                                        int lane) {
    const int c = lane & 15;
    if (c >= a.mg) return;
    const int64_t nn = (int64_t)a.nbf * a.nbf;
    double* Jc = a.J + (int64_t)(a.c0 + c) * nn;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * r + (lane >> 4);
        const int fa = a.slot_fn[A * 8 + (row >> 3)];
        const int fb = a.slot_fn[B * 8 + (row & 7)];
        if (fa < 0 || fb < 0) continue;
        const double v = acc[r];
        if (v == 0.0) continue;
        unsafeAtomicAdd(Jc + (int64_t)fa * a.nbf + fb, v);
    }
}

__global__ void __launch_bounds__(kThreads, 2) fock_mfma_f64_kernel(FockArgs a) {
    __shared__ double sV[4096];
    __shared__ double sB0[kOpElems];   // operand of the first K view
    __shared__ double sB1[kOpElems];   // operand of the second K view
    __shared__ double sBJ[kOpElems];   // operand of the J view

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;            // wave = row-tile of every view
    const WorkItem it = a.items[blockIdx.x];
    const int I = it.I, J = it.J, visit = it.visit;
    const int T = a.ntiles;

    // fragment coordinates of this lane: row within the row-tile and k-row
    const int fr = lane & 15;          // A row / B col / C col
    const int fk = lane >> 4;          // A k / B k-row / C row group

    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0}, accJ = {0, 0, 0, 0};
    int run_key = -1;

    // prefetch registers for the next block
    double pv[16];
    double pb0[4], pb1[4], pbj[4];

    auto fetch = [&](int e) {
        const int64_t b = a.entries[e];
        const int32_t* bt = a.blk_tiles + 4 * b;
        const int K = bt[2], L = bt[3];
        const double* src = a.vals + b * 4096;
#pragma unroll
        for (int x = 0; x < 16; ++x) pv[x] = __builtin_nontemporal_load(src + x * kThreads + tid);
        // operand tiles of this visit
        int a0, b0t, a1, b1t;
        const double* Sp;
        if (visit == 0) {  // X_JL, X_IL, S_KL
            a0 = J; b0t = L; a1 = I; b1t = L;
            Sp = a.S + ((int64_t)K * T + L) * kOpElems;
        } else {           // X_JK, X_IK, S_IJ
            a0 = J; b0t = K; a1 = I; b1t = K;
            Sp = a.S + ((int64_t)I * T + J) * kOpElems;
        }
        const double* X0 = a.X + ((int64_t)a0 * T + b0t) * kOpElems;
        const double* X1 = a.X + ((int64_t)a1 * T + b1t) * kOpElems;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            pb0[x] = X0[x * kThreads + tid];
            pb1[x] = X1[x * kThreads + tid];
            pbj[x] = Sp[x * kThreads + tid];
        }
        return (visit == 0) ? K : L;
    };

    int e = it.e0;
    int next_key = fetch(e);
    while (e < it.e1) {
        const int64_t b = a.entries[e];
        const int32_t* bt = a.blk_tiles + 4 * b;
        const int K = bt[2], L = bt[3];
        const int key = next_key;
        // run change: add the finished run's targets to K
        if (key != run_key && run_key >= 0) {
            if (visit == 0) {
                flush_k(a, I, run_key, w, acc0, lane);
                flush_k(a, J, run_key, w, acc1, lane);
            } else {
                flush_k(a, I, run_key, w, acc0, lane);
                flush_k(a, J, run_key, w, acc1, lane);
            }
            acc0 = d4{0, 0, 0, 0};
            acc1 = d4{0, 0, 0, 0};
        }
        run_key = key;
        // stage the prefetched block and operands
#pragma unroll
        for (int x = 0; x < 16; ++x) {
            const int n = x * kThreads + tid;
            sV[vpos(n >> 9, (n >> 6) & 7, (n >> 3) & 7, n & 7)] = pv[x];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            sB0[x * kThreads + tid] = pb0[x];
            sB1[x * kThreads + tid] = pb1[x];
            sBJ[x * kThreads + tid] = pbj[x];
        }
        __syncthreads();
        if (e + 1 < it.e1) next_key = fetch(e + 1);

        d4 accK = {0, 0, 0, 0};  // per-block J_KL (visit 1)
        // row-tile w of each view: rows 16w .. 16w+15 = (first index in {2w, 2w+1}) x 8
        const int r = 16 * w + fr;
        const int x1 = r >> 3, x2 = r & 7;   // first and second row index
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int q = 4 * s + fk;         // reduction index of this lane
            const int y1 = q >> 3, y2 = q & 7;
            const double bo0 = sB0[q * kCols + fr];
            const double bo1 = sB1[q * kCols + fr];
            const double boj = sBJ[q * kCols + fr];
            double v0, v1, vj;
            if (visit == 0) {
                // V2: rows (i,k) = (x1,x2), red (j,l) = (y1,y2)
                v0 = sV[vpos(x1, y1, x2, y2)];
                // V3^T: rows (j,k) = (x1,x2), red (i,l) = (y1,y2)
                v1 = sV[vpos(y1, x1, x2, y2)];
                // V1: rows (i,j) = (x1,x2), red (k,l) = (y1,y2)
                vj = sV[vpos(x1, x2, y1, y2)];
            } else {
                // V3: rows (i,l) = (x1,x2), red (j,k) = (y1,y2)
                v0 = sV[vpos(x1, y1, y2, x2)];
                // V2^T: rows (j,l) = (x1,x2), red (i,k) = (y1,y2)
                v1 = sV[vpos(y1, x1, y2, x2)];
                // V1^T: rows (k,l) = (x1,x2), red (i,j) = (y1,y2)
                vj = sV[vpos(y1, y2, x1, x2)];
            }
            acc0 = mfma(v0, bo0, acc0);
            acc1 = mfma(v1, bo1, acc1);
            if (visit == 0)
                accJ = mfma(vj, boj, accJ);
            else
                accK = mfma(vj, boj, accK);
        }
        if (visit == 1) flush_j(a, K, L, w, accK, lane);
        __syncthreads();
        ++e;
    }
    if (run_key >= 0) {
        flush_k(a, I, run_key, w, acc0, lane);
        flush_k(a, J, run_key, w, acc1, lane);
    }
    if (visit == 0) flush_j(a, I, J, w, accJ, lane);
}

// Operand tiles of a density group: for every tile pair (A, B),
//   X[A][B][(a,b)][c] = D_{c0+c}[A_a][B_b] (c < 8), D_{c0+c-8}[B_b][A_a] (c >= 8)
//   S[A][B][(a,b)][c] = D_{c0+c}[A_a][B_b] + D_{c0+c}[B_b][A_a]  (c < 8), 0 else
// with zeros for ghost slots and for densities beyond the group.
__global__ void prep_operands_kernel(const double* __restrict__ d, const int32_t* __restrict__ slot_fn,
                                     int nbf, int ntiles, int mg, int c0, double* X, double* S) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)ntiles * ntiles * kOpElems;
    if (idx >= total) return;
    const int c = (int)(idx % kCols);
    const int ab = (int)((idx / kCols) % 64);
    const int64_t tp = idx / kOpElems;
    const int A = (int)(tp / ntiles), B = (int)(tp % ntiles);
    const int fa = slot_fn[A * 8 + (ab >> 3)], fb = slot_fn[B * 8 + (ab & 7)];
    const int dens = c & 7;
    double x = 0.0, s = 0.0;
    if (fa >= 0 && fb >= 0 && dens < mg) {
        const double* Dc = d + (int64_t)(c0 + dens) * nbf * nbf;
        const double dab = Dc[(int64_t)fa * nbf + fb], dba = Dc[(int64_t)fb * nbf + fa];
        x = c < 8 ? dab : dba;
        s = c < 8 ? dab + dba : 0.0;
    }
    X[idx] = x;
    S[idx] = s;
}

}  // namespace

size_t fock_mfma_workspace_bytes(int ntiles) {
    return 2 * sizeof(double) * (size_t)ntiles * ntiles * kOpElems;
}

size_t fock_mfma_item_bytes() { return sizeof(WorkItem); }

hipError_t launch_fock_mfma_f64(const StoreView& sv, const int32_t* d_entries,
                                const void* d_items, int nitems, int m, const double* d,
                                double* j, double* k, double* workspace, hipStream_t s) {
    const int T = sv.ntiles;
    double* X = workspace;
    double* S = workspace + (size_t)T * T * kOpElems;
    for (int c0 = 0; c0 < m; c0 += 8) {
        const int mg = m - c0 < 8 ? m - c0 : 8;
        const int64_t total = (int64_t)T * T * kOpElems;
        prep_operands_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(
            d, sv.slot_fn, sv.nbf, T, mg, c0, X, S);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (nitems == 0) continue;
        FockArgs a;
        a.vals = (const double*)sv.vals;
        a.blk_tiles = sv.blk_tiles;
        a.slot_fn = sv.slot_fn;
        a.entries = d_entries;
        a.items = (const WorkItem*)d_items;
        a.X = X;
        a.S = S;
        a.J = j;
        a.K = k;
        a.nbf = sv.nbf;
        a.ntiles = T;
        a.mg = mg;
        a.c0 = c0;
        a.nitems = nitems;
        fock_mfma_f64_kernel<<<nitems, kThreads, 0, s>>>(a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace esmf
