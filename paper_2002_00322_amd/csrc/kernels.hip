// HIP kernels of libesmf for gfx950 (MI355X).
//
// Preparation: pair quantities and Schwarz factors, then the screened
// integral block store.  Build: the grouped J/K contraction over the store.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace esmf {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Boys function F0(T) = int_0^1 exp(-T u^2) du: Taylor series below 1e-2
// (terms decay like T^k / (k! (2k+1)); 12 terms are far below FP64 rounding
// there), else (1/2) sqrt(pi/T) erf(sqrt(T)) with ROCm's device erf.
__device__ inline double boys_f0(double T) {
    if (T < 1e-2) {
        double term = 1.0, sum = 1.0;
#pragma unroll
        for (int k = 1; k <= 12; ++k) {
            term *= -T / (double)k;
            sum += term / (double)(2 * k + 1);
        }
        return sum;
    }
    return 0.5 * sqrt(kPi / T) * erf(sqrt(T));
}

__device__ inline double norm_s(double a) { return pow(2.0 * a / kPi, 0.75); }

// Gaussian product of two s primitives a, b (slot order): exponent zeta,
// centre P, prefactor E = n_a n_b exp(-a_a a_b |A_a - A_b|^2 / zeta), and the
// Schwarz factor sqrt((ab|ab)) = E sqrt(2 pi^(5/2) / (zeta^2 sqrt(2 zeta))).
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
    pz[idx] = z;
    px[idx] = P[0];
    py[idx] = P[1];
    pzc[idx] = P[2];
    pe[idx] = E;
    pq[idx] = E * sqrt(2.0 * pow(kPi, 2.5) / (z * z * sqrt(2.0 * z)));
}

// One workgroup per block (256 threads, 16 integrals each).  Block layout:
// value of (ij|kl) at ((i*T + j)*T + k)*T + l, T = kTile.
template <typename StoreT>
__global__ void __launch_bounds__(256)
eri_fill_kernel(const int32_t* __restrict__ blk_tiles, const double* __restrict__ wts,
                int nslots, const double* __restrict__ pz, const double* __restrict__ px,
                const double* __restrict__ py, const double* __restrict__ pzc,
                const double* __restrict__ pe, const double* __restrict__ pq, double tau,
                StoreT* __restrict__ vals) {
    const int64_t b = blockIdx.x;
    const int I = blk_tiles[4 * b + 0], J = blk_tiles[4 * b + 1];
    const int K = blk_tiles[4 * b + 2], L = blk_tiles[4 * b + 3];
    const double w = wts[b];
    StoreT* out = vals + b * (int64_t)kBlockElems;
    for (int e = threadIdx.x; e < kBlockElems; e += blockDim.x) {
        int l = e % kTile, k = (e / kTile) % kTile, j = (e / (kTile * kTile)) % kTile;
        int i = e / (kTile * kTile * kTile);
        int64_t ab = (int64_t)(I * kTile + i) * nslots + (J * kTile + j);
        int64_t cd = (int64_t)(K * kTile + k) * nslots + (L * kTile + l);
        double qab = pq[ab], qcd = pq[cd];
        double v = 0.0;
        if (qab * qcd > tau) {
            double z = pz[ab], e2 = pz[cd];
            double dx = px[ab] - px[cd], dy = py[ab] - py[cd], dz = pzc[ab] - pzc[cd];
            double R2 = dx * dx + dy * dy + dz * dz;
            double T = z * e2 / (z + e2) * R2;
            double pre = 2.0 * pow(kPi, 2.5) / (z * e2 * sqrt(z + e2));
            v = w * (pe[ab] * pe[cd] * pre * boys_f0(T));
        }
        out[e] = (StoreT)v;
    }
}

__global__ void zero_kernel(double* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0.0;
}

// J <- J + J^T per density (the block pass accumulates each symmetric pair
// contribution at one of its two positions).
__global__ void symmetrize_j_kernel(int n, int m, double* j) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nn = (int64_t)n * n;
    if (idx >= nn * m) return;
    int c = (int)(idx / nn);
    int64_t r = idx % nn;
    int p = (int)(r / n), q = (int)(r % n);
    double* Jc = j + (int64_t)c * nn;
    if (p < q) {
        double s = Jc[(int64_t)p * n + q] + Jc[(int64_t)q * n + p];
        Jc[(int64_t)p * n + q] = s;
        Jc[(int64_t)q * n + p] = s;
    } else if (p == q) {
        Jc[(int64_t)p * n + p] *= 2.0;
    }
}

// Straightforward FP64 build: one workgroup per stored block, densities one at
// a time.  For block (IJ|KL) and integral v = w (ij|kl) the ten contractions
// below realise every permutation of Eq. J_and_K (J through S = D + D^T at one
// of its two symmetric positions), each accumulated over the block's other two
// indices and added to J/K with device-scope FP64 atomics.
//   view 0: J[i][j] += sum_kl v S[k][l]     view 1: J[k][l] += sum_ij v S[i][j]
//   view 2: K[i][k] += sum_jl v D[j][l]     view 3: K[k][i] += sum_jl v D[l][j]
//   view 4: K[i][l] += sum_jk v D[j][k]     view 5: K[l][i] += sum_jk v D[k][j]
//   view 6: K[j][k] += sum_il v D[i][l]     view 7: K[k][j] += sum_il v D[l][i]
//   view 8: K[j][l] += sum_ik v D[i][k]     view 9: K[l][j] += sum_ik v D[k][i]
constexpr int kT = kTile;
constexpr int kT2 = kTile * kTile;
constexpr int kT3 = kTile * kTile * kTile;

__global__ void __launch_bounds__(256)
fock_fp64_simple_kernel(StoreView sv, int m, const double* __restrict__ d, double* j,
                        double* k) {
    __shared__ double V[kBlockElems];
    __shared__ double Dt[10][kT2];
    __shared__ int fn[4][kT];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    const int n = sv.nbf;
    const int64_t nn = (int64_t)n * n;
    const int32_t* bt = sv.blk_tiles + 4 * b;
    const double* src = (const double*)sv.vals + b * (int64_t)kBlockElems;
    for (int e = t; e < kBlockElems; e += blockDim.x) V[e] = src[e];
    if (t < 4 * kT) fn[t / kT][t % kT] = sv.slot_fn[bt[t / kT] * kT + (t % kT)];
    __syncthreads();
    // tile roles: 0 = I, 1 = J, 2 = K, 3 = L
    // Dt[x] = D[row role][col role] laid out [a][b]
    const int rowr[10] = {1, 3, 1, 2, 0, 3, 0, 2, 0, 2};
    const int colr[10] = {3, 1, 2, 1, 3, 0, 2, 0, 1, 3};
    for (int c = 0; c < m; ++c) {
        const double* Dc = d + (int64_t)c * nn;
        for (int e = t; e < 10 * kT2; e += blockDim.x) {
            int x = e / kT2, a = (e / kT) % kT, bb = e % kT;
            int pr = fn[rowr[x]][a], pc = fn[colr[x]][bb];
            double val = 0.0;
            if (pr >= 0 && pc >= 0) {
                val = Dc[(int64_t)pr * n + pc];
                if (x >= 8) val += Dc[(int64_t)pc * n + pr];  // S = D + D^T
            }
            Dt[x][a * kT + bb] = val;
        }
        __syncthreads();
        double* Jc = j + (int64_t)c * nn;
        double* Kc = k + (int64_t)c * nn;
        for (int o = t; o < 10 * kT2; o += blockDim.x) {
            const int view = o / kT2, r = o % kT2, r0 = r / kT, r1 = r % kT;
            double acc = 0.0;
            int orow, ocol;
            double* dst;
            switch (view) {
                case 0:  // (i,j) <- sum_kl v[i][j][k][l] S_KL[k][l]
                    for (int s = 0; s < kT2; ++s) acc += V[r0 * kT3 + r1 * kT2 + s] * Dt[9][s];
                    orow = fn[0][r0]; ocol = fn[1][r1]; dst = Jc;
                    break;
                case 1:  // (k,l) <- sum_ij v S_IJ[i][j]
                    for (int s = 0; s < kT2; ++s) acc += V[s * kT2 + r0 * kT + r1] * Dt[8][s];
                    orow = fn[2][r0]; ocol = fn[3][r1]; dst = Jc;
                    break;
                case 2:  // K[i][k] <- sum_jl v D_JL[j][l]
                case 3:  // K[k][i] <- sum_jl v D_LJ[l][j]
                    for (int jj = 0; jj < kT; ++jj)
                        for (int ll = 0; ll < kT; ++ll) {
                            double dv = view == 2 ? Dt[0][jj * kT + ll] : Dt[1][ll * kT + jj];
                            acc += V[r0 * kT3 + jj * kT2 + r1 * kT + ll] * dv;
                        }
                    if (view == 2) { orow = fn[0][r0]; ocol = fn[2][r1]; }
                    else { orow = fn[2][r1]; ocol = fn[0][r0]; }
                    dst = Kc;
                    break;
                case 4:  // K[i][l] <- sum_jk v D_JK[j][k]
                case 5:  // K[l][i] <- sum_jk v D_KJ[k][j]
                    for (int jj = 0; jj < kT; ++jj)
                        for (int kk = 0; kk < kT; ++kk) {
                            double dv = view == 4 ? Dt[2][jj * kT + kk] : Dt[3][kk * kT + jj];
                            acc += V[r0 * kT3 + jj * kT2 + kk * kT + r1] * dv;
                        }
                    if (view == 4) { orow = fn[0][r0]; ocol = fn[3][r1]; }
                    else { orow = fn[3][r1]; ocol = fn[0][r0]; }
                    dst = Kc;
                    break;
                case 6:  // K[j][k] <- sum_il v D_IL[i][l]
                case 7:  // K[k][j] <- sum_il v D_LI[l][i]
                    for (int ii = 0; ii < kT; ++ii)
                        for (int ll = 0; ll < kT; ++ll) {
                            double dv = view == 6 ? Dt[4][ii * kT + ll] : Dt[5][ll * kT + ii];
                            acc += V[ii * kT3 + r0 * kT2 + r1 * kT + ll] * dv;
                        }
                    if (view == 6) { orow = fn[1][r0]; ocol = fn[2][r1]; }
                    else { orow = fn[2][r1]; ocol = fn[1][r0]; }
                    dst = Kc;
                    break;
                default:  // 8: K[j][l] <- sum_ik v D_IK[i][k]; 9: K[l][j] <- sum_ik v D_KI[k][i]
                    for (int ii = 0; ii < kT; ++ii)
                        for (int kk = 0; kk < kT; ++kk) {
                            double dv = view == 8 ? Dt[6][ii * kT + kk] : Dt[7][kk * kT + ii];
                            acc += V[ii * kT3 + r0 * kT2 + kk * kT + r1] * dv;
                        }
                    if (view == 8) { orow = fn[1][r0]; ocol = fn[3][r1]; }
                    else { orow = fn[3][r1]; ocol = fn[1][r0]; }
                    dst = Kc;
                    break;
            }
            if (orow >= 0 && ocol >= 0 && acc != 0.0)
                unsafeAtomicAdd(dst + (int64_t)orow * n + ocol, acc);
        }
        __syncthreads();
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

hipError_t launch_eri_fill(int64_t nblocks, const int32_t* d_blk_tiles, const double* d_w,
                           int nslots, const double* d_pz, const double* d_px,
                           const double* d_py, const double* d_pzc, const double* d_pe,
                           const double* d_pq, double tau, void* d_vals, int fp32,
                           hipStream_t s) {
    // one launch per chunk of at most 2^30 blocks keeps the grid in range
    const int64_t chunk = (int64_t)1 << 30;
    for (int64_t b0 = 0; b0 < nblocks; b0 += chunk) {
        int64_t nb = nblocks - b0 < chunk ? nblocks - b0 : chunk;
        if (fp32)
            eri_fill_kernel<float><<<(unsigned)nb, 256, 0, s>>>(
                d_blk_tiles + 4 * b0, d_w + b0, nslots, d_pz, d_px, d_py, d_pzc, d_pe, d_pq,
                tau, (float*)d_vals + b0 * kBlockElems);
        else
            eri_fill_kernel<double><<<(unsigned)nb, 256, 0, s>>>(
                d_blk_tiles + 4 * b0, d_w + b0, nslots, d_pz, d_px, d_py, d_pzc, d_pe, d_pq,
                tau, (double*)d_vals + b0 * kBlockElems);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    int grid = (int)(g < 65536 ? g : 65536);
    zero_kernel<<<grid, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_fock_fp64_simple(const StoreView& sv, int m, const double* d, double* j,
                                   double* k, hipStream_t s) {
    const int64_t chunk = (int64_t)1 << 30;
    for (int64_t b0 = 0; b0 < sv.nblocks; b0 += chunk) {
        StoreView v = sv;
        v.vals = (const double*)sv.vals + b0 * kBlockElems;
        v.blk_tiles = sv.blk_tiles + 4 * b0;
        v.nblocks = sv.nblocks - b0 < chunk ? sv.nblocks - b0 : chunk;
        fock_fp64_simple_kernel<<<(unsigned)v.nblocks, 256, 0, s>>>(v, m, d, j, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_symmetrize_j(int nbf, int m, double* j, hipStream_t s) {
    int64_t total = (int64_t)nbf * nbf * m;
    int grid = (int)((total + 255) / 256);
    symmetrize_j_kernel<<<grid, 256, 0, s>>>(nbf, m, j);
    return hipGetLastError();
}

}  // namespace esmf
