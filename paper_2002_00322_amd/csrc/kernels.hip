// HIP kernels of libesmf for gfx950 (MI355X).
//
// Preparation: pair quantities and Schwarz factors, then the screened
// integral block store.  Build: the grouped J/K contraction over the store.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "eri_device.h"
#include "internal.h"

namespace esmf {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

__device__ inline double norm_s(double a) { return pow(2.0 * a / kPi, 0.75); }

// Gaussian product of two s primitives a, b (slot order): 1/zeta (zeta the
// exponent sum), centre P, E' = E (pi/zeta)^(3/2) with the prefactor
// E = n_a n_b exp(-a_a a_b |A_a - A_b|^2 / zeta), and the Schwarz factor
// sqrt((ab|ab)) = E sqrt(2 pi^(5/2) / (zeta^2 sqrt(2 zeta))).
__global__ void pair_build_kernel(int nslots, const int32_t* __restrict__ slot_fn,
                                  const double* __restrict__ centers,
                                  const double* __restrict__ alpha, double* pz, double* px,
                                  double* py, double* pzc, double* pe, double* pq) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nslots * nslots;
    if (idx >= total) return;
    int a = (int)(idx / nslots), b = (int)(idx % nslots);
    int fa = slot_fn[a], fb = slot_fn[b];
    if (fa < 0 || fb < 0) {
        pz[idx] = 1.0;
        px[idx] = 0.0;
        py[idx] = 0.0;
        pzc[idx] = 0.0;
        pe[idx] = 0.0;
        pq[idx] = 0.0;
        return;
    }
    double aa = alpha[fa], ab = alpha[fb];
    double z = aa + ab;
    double r2 = 0.0, P[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        double ca = centers[3 * fa + x], cb = centers[3 * fb + x];
        double d = ca - cb;
        r2 += d * d;
        P[x] = (aa * ca + ab * cb) / z;
    }
    double E = norm_s(aa) * norm_s(ab) * exp(-aa * ab * r2 / z);
    pz[idx] = 1.0 / z;
    px[idx] = P[0];
    py[idx] = P[1];
    pzc[idx] = P[2];
    pe[idx] = E * pow(kPi / z, 1.5);
    pq[idx] = E * sqrt(2.0 * pow(kPi, 2.5) / (z * z * sqrt(2.0 * z)));
}

// Granule presence: one workgroup per block, thread g tests granule g (its 16
// integrals share (i, j, k/2)); the waves' ballots are the block's 4 mask words.
__global__ void __launch_bounds__(256)
granule_mask_kernel(const int32_t* __restrict__ blk_tiles, int nslots,
                    const double* __restrict__ pq, double tau, uint64_t* mask, int32_t* count) {
    const int64_t b = blockIdx.x;
    const int I = blk_tiles[4 * b + 0], J = blk_tiles[4 * b + 1];
    const int K = blk_tiles[4 * b + 2], L = blk_tiles[4 * b + 3];
    const int g = threadIdx.x;
    const int i = g >> 5, j = (g >> 2) & 7, kp = g & 3;
    const double qab = pq[(int64_t)(I * kTile + i) * nslots + (J * kTile + j)];
    bool keep = false;
    for (int kk = 0; kk < 2; ++kk)
        for (int l = 0; l < kTile; ++l) {
            const double qcd = pq[(int64_t)(K * kTile + 2 * kp + kk) * nslots + (L * kTile + l)];
            keep |= qab * qcd > tau;
        }
    const uint64_t bal = __ballot(keep);
    __shared__ int cnt[4];
    if ((threadIdx.x & 63) == 0) {
        mask[4 * b + (threadIdx.x >> 6)] = bal;
        cnt[threadIdx.x >> 6] = __popcll(bal);
    }
    __syncthreads();
    if (threadIdx.x == 0) count[b] = cnt[0] + cnt[1] + cnt[2] + cnt[3];
}

// Fill of the kept granules: one workgroup per block, thread g computes the 16
// integrals of granule g if it is kept, at its rank among the kept granules.
template <typename StoreT>
__global__ void __launch_bounds__(256)
eri_fill_kernel(const int32_t* __restrict__ blk_tiles, const double* __restrict__ wts,
                const uint64_t* __restrict__ mask, const int64_t* __restrict__ off, int nslots,
                const double* __restrict__ pz, const double* __restrict__ px,
                const double* __restrict__ py, const double* __restrict__ pzc,
                const double* __restrict__ pe, const double* __restrict__ pq, double tau,
                StoreT* __restrict__ vals) {
    const int64_t b = blockIdx.x;
    const int I = blk_tiles[4 * b + 0], J = blk_tiles[4 * b + 1];
    const int K = blk_tiles[4 * b + 2], L = blk_tiles[4 * b + 3];
    const double w = wts[b];
    const int g = threadIdx.x, wv = g >> 6, ln = g & 63;
    const uint64_t* mk = mask + 4 * b;
    const uint64_t mw = mk[wv];
    if (!((mw >> ln) & 1)) return;
    int rank = __popcll(mw & ((ln == 0) ? 0ull : (~0ull >> (64 - ln))));
    for (int x = 0; x < wv; ++x) rank += __popcll(mk[x]);
    StoreT* out = vals + (off[b] + rank) * kGranule;
    const int i = g >> 5, j = (g >> 2) & 7, kp = g & 3;
    const int64_t ab = (int64_t)(I * kTile + i) * nslots + (J * kTile + j);
    const PairData pab{pz[ab], px[ab], py[ab], pzc[ab], pe[ab], pq[ab]};
    for (int u = 0; u < kGranule; ++u) {
        const int k = 2 * kp + (u >> 3), l = u & 7;
        const int64_t cd = (int64_t)(K * kTile + k) * nslots + (L * kTile + l);
        const PairData pcd{pz[cd], px[cd], py[cd], pzc[cd], pe[cd], pq[cd]};
        out[u] = (StoreT)screened_eri(w, pab, pcd, tau);
    }
}

}  // namespace

hipError_t launch_pair_build(int nslots, const int32_t* d_slot_fn, const double* d_centers,
                             const double* d_alpha, double* d_pz, double* d_px, double* d_py,
                             double* d_pzc, double* d_pe, double* d_pq, hipStream_t s) {
    int64_t total = (int64_t)nslots * nslots;
    int grid = (int)((total + 255) / 256);
    pair_build_kernel<<<grid, 256, 0, s>>>(nslots, d_slot_fn, d_centers, d_alpha, d_pz, d_px,
                                           d_py, d_pzc, d_pe, d_pq);
    return hipGetLastError();
}

hipError_t launch_granule_mask(int64_t nblocks, const int32_t* d_blk_tiles, int nslots,
                               const double* d_pq, double tau, uint64_t* d_mask,
                               int32_t* d_count, hipStream_t s) {
    const int64_t chunk = (int64_t)1 << 30;
    for (int64_t b0 = 0; b0 < nblocks; b0 += chunk) {
        int64_t nb = nblocks - b0 < chunk ? nblocks - b0 : chunk;
        granule_mask_kernel<<<(unsigned)nb, 256, 0, s>>>(d_blk_tiles + 4 * b0, nslots, d_pq, tau,
                                                         d_mask + 4 * b0, d_count + b0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_eri_fill(int64_t nblocks, const int32_t* d_blk_tiles, const double* d_w,
                           const uint64_t* d_mask, const int64_t* d_off, int nslots,
                           const double* d_pz, const double* d_px, const double* d_py,
                           const double* d_pzc, const double* d_pe, const double* d_pq,
                           double tau, void* d_vals, int fp32, hipStream_t s) {
    const int64_t chunk = (int64_t)1 << 30;
    for (int64_t b0 = 0; b0 < nblocks; b0 += chunk) {
        int64_t nb = nblocks - b0 < chunk ? nblocks - b0 : chunk;
        if (fp32)
            eri_fill_kernel<float><<<(unsigned)nb, 256, 0, s>>>(
                d_blk_tiles + 4 * b0, d_w + b0, d_mask + 4 * b0, d_off + b0, nslots, d_pz, d_px,
                d_py, d_pzc, d_pe, d_pq, tau, (float*)d_vals);
        else
            eri_fill_kernel<double><<<(unsigned)nb, 256, 0, s>>>(
                d_blk_tiles + 4 * b0, d_w + b0, d_mask + 4 * b0, d_off + b0, nslots, d_pz, d_px,
                d_py, d_pzc, d_pe, d_pq, tau, (double*)d_vals);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace esmf
