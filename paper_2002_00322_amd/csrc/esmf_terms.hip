// The densities and the two-body energy of one ESMF objective evaluation,
// around the grouped build: the nine generalised densities whose Fock
// matrices the analytic derivatives need (Sec. "Shell-Pair Screening", the
// list of nine Fock builds, built from the matrices of Table tab:notations),
// and the two-body energy E_2 of Eq. esmf_energy_2b from the build's J and K.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace esmf {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// C = alpha op(A) op(B) + beta C, row-major, FP64, on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64):
//   op(A)[m][k] = TA ? A[k lda + m] : A[m lda + k]
//   op(B)[k][n] = TB ? B[n ldb + k] : B[k ldb + n]
// A workgroup of four waves computes a TM x TM tile of C; wave w owns the
// (TM/2) x (TM/2) quadrant (w / 2, w % 2) as (TM/32)^2 16 x 16 accumulators.
// K is staged through LDS in chunks of KC, both operands k-major ([k][row of
// the tile]), so a matrix-core operand is 16 consecutive doubles of one k row
// per 16 lanes.  The row stride TM + 16 puts the two k rows that one 32-lane
// half of a wave reads 128 bytes apart modulo the 256 bytes of the banks:
// 32 lanes of 8-byte reads meet 32 distinct bank pairs.  An operand stored
// with k contiguous in memory (A not transposed, B transposed) is loaded with
// consecutive threads on consecutive k, so its LDS stores walk down a column;
// row k's position x is therefore stored at x ^ sw(k), a permutation inside
// each aligned group of 16 (sw(k) < 16) that spreads such a column over
// distinct banks and leaves every 16-lane operand read inside its group:
// 16 consecutive threads hold k = 0..15 of one row and the next 16 the
// following row, and sw(k) = k & 14 takes the 8 even values per parity of k,
// so the two rows land on opposite halves of each group.
// The global loads of the next chunk are issued before the products of the
// current one.  Every element sums its products in the same order (chunks in
// order, four k per matrix-core step): results are deterministic.
//
// Matrix-core lane layout (lane l of 64):
//   A[16][4]: l holds A[l % 16][l / 16];  B[4][16]: l holds B[l / 16][l % 16];
//   C[16][16]: element r of l holds C[4 r + l / 16][l % 16].
template <int TM, bool TA, bool TB>
__global__ void __launch_bounds__(256)
gemm_mfma_kernel(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
                 const double* __restrict__ B, int ldb, double beta, double* __restrict__ C, int ldc) {
    constexpr int KC = 16;                  // k per LDS chunk
    constexpr int kS = TM + 16;             // LDS row stride (doubles)
    constexpr int kLd = TM * KC / 256;      // doubles per thread per operand and chunk
    constexpr int kF = TM / 32;             // 16 x 16 accumulators per quadrant edge
    static_assert(TM * KC % 256 == 0 && KC % 4 == 0 && TM % 32 == 0, "tile shape");
    static_assert((8 * kS) % 256 == 128, "bank stride");
    auto sw = [](int k) { return k & 14; };
    __shared__ double sA[KC * kS];
    __shared__ double sB[KC * kS];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
    double ra[kLd], rb[kLd];
    // thread element e of a chunk: (k, row) of the tile, in the order that
    // makes consecutive threads read consecutive addresses
    auto a_pos = [&](int e, int& kk, int& mm) {
        const int x = e * 256 + tid;
        if (TA) { kk = x / TM; mm = x % TM; } else { kk = x % KC; mm = x / KC; }
    };
    auto b_pos = [&](int e, int& kk, int& nn) {
        const int x = e * 256 + tid;
        if (TB) { kk = x % KC; nn = x / KC; } else { kk = x / TM; nn = x % TM; }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < kLd; ++e) {
            int kk, mm;
            a_pos(e, kk, mm);
            const int gk = k0 + kk, gm = m0 + mm;
            ra[e] = (gm < M && gk < K) ? (TA ? A[(int64_t)gk * lda + gm] : A[(int64_t)gm * lda + gk]) : 0.0;
            int kb, nb;
            b_pos(e, kb, nb);
            const int hk = k0 + kb, gn = n0 + nb;
            rb[e] = (hk < K && gn < N) ? (TB ? B[(int64_t)gn * ldb + hk] : B[(int64_t)hk * ldb + gn]) : 0.0;
        }
    };
    d4 acc[kF][kF];
#pragma unroll
    for (int i = 0; i < kF; ++i)
#pragma unroll
        for (int j = 0; j < kF; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    const int qr = (w >> 1) * (TM / 2), qc = (w & 1) * (TM / 2);
    if (K > 0) load(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kLd; ++e) {
            int kk, mm;
            a_pos(e, kk, mm);
            sA[kk * kS + (mm ^ sw(kk))] = ra[e];
            b_pos(e, kk, mm);
            sB[kk * kS + (mm ^ sw(kk))] = rb[e];
        }
        __syncthreads();
        if (k0 + KC < K) load(k0 + KC);
#pragma unroll
        for (int st = 0; st < KC / 4; ++st) {
            const int k = 4 * st + (lane >> 4);
            const int kr = k * kS + ((lane & 15) ^ sw(k));
            double a[kF], b[kF];
#pragma unroll
            for (int i = 0; i < kF; ++i) {
                a[i] = sA[kr + qr + 16 * i];
                b[i] = sB[kr + qc + 16 * i];
            }
#pragma unroll
            for (int i = 0; i < kF; ++i)
#pragma unroll
                for (int j = 0; j < kF; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < kF; ++i)
#pragma unroll
        for (int j = 0; j < kF; ++j) {
            const int n = n0 + qc + 16 * j + (lane & 15);
            if (n >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + qr + 16 * i + 4 * r + (lane >> 4);
                if (m >= M) continue;
                const int64_t c = (int64_t)m * ldc + n;
                C[c] = beta == 0.0 ? alpha * acc[i][j][r] : alpha * acc[i][j][r] + beta * C[c];
            }
        }
}

// 64 x 64 tiles (four products per pair of operand reads) for long
// reductions over a grid of at least four workgroups per compute unit; 32 x 32
// tiles (one product per pair, four times the workgroups) otherwise.  Measured
// on the shapes of the nine densities and the gradient, N = 1000..8000.
template <bool TA, bool TB>
hipError_t gemm(int M, int N, int K, double alpha, const double* A, int lda, const double* B, int ldb,
                double beta, double* C, int ldc, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    const int64_t big = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
    if (K >= 2048 && big >= 1024) {
        dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
        gemm_mfma_kernel<64, TA, TB><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    } else {
        dim3 grid((unsigned)((N + 31) / 32), (unsigned)((M + 31) / 32));
        gemm_mfma_kernel<32, TA, TB><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    }
    return hipGetLastError();
}

// M <- (M + M^T) / 2 in place (n x n, row-major): one thread per pair p < q,
// both positions written with the same value, so M is exactly symmetric.
__global__ void symmetrize_kernel(int n, double* M) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t npairs = (int64_t)n * (n - 1) / 2;
    if (t >= npairs) return;
    // pair t -> (p, q), p < q, row-major over the strict upper triangle
    int p = (int)((2.0 * n - 1.0 - sqrt((2.0 * n - 1.0) * (2.0 * n - 1.0) - 8.0 * (double)t)) / 2.0);
    auto row_start = [&](int r) { return (int64_t)r * (2 * (int64_t)n - r - 1) / 2; };
    while (p > 0 && row_start(p) > t) --p;
    while (p + 1 < n && row_start(p + 1) <= t) ++p;
    const int q = (int)(p + 1 + (t - row_start(p)));
    const double v = 0.5 * (M[(int64_t)p * n + q] + M[(int64_t)q * n + p]);
    M[(int64_t)p * n + q] = v;
    M[(int64_t)q * n + p] = v;
}

constexpr int kEnergyBlocks = 1024;
constexpr int kEnergyThreads = 256;

// Per-block partial sums of the element-wise terms of E_2:
//   N2 F1.D1 + 4 c0 F1.D2 + 2 F1.A + 2 F2.D2,  F_i = 2 J_i - K_i.
// The last term pairs F[D2] with D2 itself: it comes from the block of the
// energy quadratic in sigma (the Appendix's sigma-derivative of E carries the
// matching 4 Theta F[D2] Gamma^T).
__global__ void __launch_bounds__(kEnergyThreads)
energy_terms_kernel(int64_t nn, double n2, double c0, const double* __restrict__ d,
                    const double* __restrict__ j, const double* __restrict__ k, double* partial) {
    const double* D1 = d;
    const double* D2 = d + nn;
    const double* DA = d + 2 * nn;
    double t = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * kEnergyThreads + threadIdx.x; x < nn;
         x += (int64_t)kEnergyBlocks * kEnergyThreads) {
        const double f1 = 2.0 * j[x] - k[x];
        const double f2 = 2.0 * j[nn + x] - k[nn + x];
        t += n2 * f1 * D1[x] + 4.0 * c0 * f1 * D2[x] + 2.0 * f1 * DA[x] + 2.0 * f2 * D2[x];
    }
    __shared__ double red[kEnergyThreads];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int h = kEnergyThreads / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kEnergyThreads) energy_sum_kernel(const double* partial, double* e2) {
    __shared__ double red[kEnergyThreads];
    double t = 0.0;
    for (int b = threadIdx.x; b < kEnergyBlocks; b += kEnergyThreads) t += partial[b];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int h = kEnergyThreads / 2; h > 0; h /= 2) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *e2 = red[0];
}

}  // namespace

// Nine densities (row-major [9][N][N] into d; D1 and A exactly symmetric),
// with No = n_occ, Nv = n_virt:
//   1 Theta^T Theta          2 Theta^T sigma Gamma     3 A
//   4 R^T Theta              5 R^T sigma Gamma         6 Theta^T mu Gamma
//   7 Theta^T sigma Phi      8 Theta^T mu sigma^T Theta  9 B
// A = Gamma^T sigma^T sigma Gamma - Theta^T sigma sigma^T Theta and
// B = Phi^T sigma^T sigma Gamma - R^T sigma sigma^T Theta, through the
// intermediates SG = sigma Gamma, SP = sigma Phi, MG = mu Gamma [No][N],
// SS = sigma sigma^T, MS = mu sigma^T [No][No], SSt = SS Theta,
// MSt = MS Theta [No][N], held in `work` (5 No N + 2 No^2 doubles).
hipError_t launch_nine_densities(int n, int no, int nv, const double* theta, const double* gamma,
                                 const double* sigma, const double* mu, const double* r,
                                 const double* phi, double* d, double* work, hipStream_t s) {
    const int64_t nn = (int64_t)n * n;
    double* SG = work;
    double* SP = SG + (int64_t)no * n;
    double* MG = SP + (int64_t)no * n;
    double* SSt = MG + (int64_t)no * n;
    double* MSt = SSt + (int64_t)no * n;
    double* SS = MSt + (int64_t)no * n;
    double* MS = SS + (int64_t)no * no;
    hipError_t e;
#define ESMF_G(call)                     \
    do {                                 \
        e = (call);                      \
        if (e != hipSuccess) return e;   \
    } while (0)
    ESMF_G((gemm<false, false>(no, n, nv, 1.0, sigma, nv, gamma, n, 0.0, SG, n, s)));
    ESMF_G((gemm<false, false>(no, n, nv, 1.0, sigma, nv, phi, n, 0.0, SP, n, s)));
    ESMF_G((gemm<false, false>(no, n, nv, 1.0, mu, nv, gamma, n, 0.0, MG, n, s)));
    ESMF_G((gemm<false, true>(no, no, nv, 1.0, sigma, nv, sigma, nv, 0.0, SS, no, s)));
    ESMF_G((gemm<false, true>(no, no, nv, 1.0, mu, nv, sigma, nv, 0.0, MS, no, s)));
    ESMF_G((gemm<false, false>(no, n, no, 1.0, SS, no, theta, n, 0.0, SSt, n, s)));
    ESMF_G((gemm<false, false>(no, n, no, 1.0, MS, no, theta, n, 0.0, MSt, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, theta, n, theta, n, 0.0, d + 0 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, theta, n, SG, n, 0.0, d + 1 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, SG, n, SG, n, 0.0, d + 2 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, -1.0, theta, n, SSt, n, 1.0, d + 2 * nn, n, s)));
    // D1 = Theta^T Theta sums the same products in the same order for (p, q)
    // and (q, p); A's second product does not.  Both are symmetrised, so
    // that exact symmetry, which a build with them marked symmetric requires,
    // does not rest on how the matrix cores order a step's four products.
    if (n > 1) {
        const int64_t npairs = (int64_t)n * (n - 1) / 2;
        for (int x : {0, 2}) {
            symmetrize_kernel<<<(unsigned)((npairs + 255) / 256), 256, 0, s>>>(n, d + x * nn);
            ESMF_G(hipGetLastError());
        }
    }
    ESMF_G((gemm<true, false>(n, n, no, 1.0, r, n, theta, n, 0.0, d + 3 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, r, n, SG, n, 0.0, d + 4 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, theta, n, MG, n, 0.0, d + 5 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, theta, n, SP, n, 0.0, d + 6 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, theta, n, MSt, n, 0.0, d + 7 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, 1.0, SP, n, SG, n, 0.0, d + 8 * nn, n, s)));
    ESMF_G((gemm<true, false>(n, n, no, -1.0, r, n, SSt, n, 1.0, d + 8 * nn, n, s)));
#undef ESMF_G
    return hipSuccess;
}

size_t nine_densities_work_doubles(int n, int no) { return (size_t)5 * no * n + (size_t)2 * no * no; }

// E_2 (Eq. esmf_energy_2b) into the device scalar e2; `partial` holds
// kEnergyBlocks doubles.  Fixed block count and order: deterministic.
hipError_t launch_energy_two_body(int n, double n2, double c0, const double* d, const double* j,
                                  const double* k, double* e2, double* partial, hipStream_t s) {
    energy_terms_kernel<<<kEnergyBlocks, kEnergyThreads, 0, s>>>((int64_t)n * n, n2, c0, d, j, k, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    energy_sum_kernel<<<1, kEnergyThreads, 0, s>>>(partial, e2);
    return hipGetLastError();
}

size_t energy_partial_doubles() { return kEnergyBlocks; }

namespace {

// The matrices the gradient multiplies, from G and the builds of D1, D2, A
// (F_i = 2 J_i - K_i), element (p, q) of each:
//   F2, H = G + F1, P1 = 4 N2 H + 4 c0 (F2 + F2^T) + 2 (FA + FA^T),
//   P2 = 4 c0 H + 4 F2^T.
__global__ void __launch_bounds__(256)
gradient_prep_kernel(int n, double c0, double n2, const double* __restrict__ g, const double* __restrict__ j,
                     const double* __restrict__ k, double* F2, double* H, double* P1, double* P2) {
    const int64_t nn = (int64_t)n * n;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nn) return;
    const int64_t p = x / n, q = x % n;
    const int64_t xt = q * n + p;
    const double f1 = 2.0 * j[x] - k[x];
    const double f2 = 2.0 * j[nn + x] - k[nn + x];
    const double f2t = 2.0 * j[nn + xt] - k[nn + xt];
    const double fa = 2.0 * j[2 * nn + x] - k[2 * nn + x];
    const double fat = 2.0 * j[2 * nn + xt] - k[2 * nn + xt];
    const double h = g[x] + f1;
    F2[x] = f2;
    H[x] = h;
    P1[x] = 4.0 * n2 * h + 4.0 * c0 * (f2 + f2t) + 2.0 * (fa + fat);
    P2[x] = 4.0 * c0 * h + 4.0 * f2t;
}

constexpr int kDots = 7;  // G.D1, G.D2, G.A, F1.D1, F1.D2, F1.A, F2.D2

__global__ void __launch_bounds__(kEnergyThreads)
energy_dots_kernel(int64_t nn, const double* __restrict__ g, const double* __restrict__ d,
                   const double* __restrict__ j, const double* __restrict__ k, double* partial) {
    double t[kDots] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t x = (int64_t)blockIdx.x * kEnergyThreads + threadIdx.x; x < nn;
         x += (int64_t)kEnergyBlocks * kEnergyThreads) {
        const double d1 = d[x], d2 = d[nn + x], da = d[2 * nn + x];
        const double f1 = 2.0 * j[x] - k[x];
        const double f2 = 2.0 * j[nn + x] - k[nn + x];
        const double gg = g[x];
        t[0] += gg * d1;
        t[1] += gg * d2;
        t[2] += gg * da;
        t[3] += f1 * d1;
        t[4] += f1 * d2;
        t[5] += f1 * da;
        t[6] += f2 * d2;
    }
    __shared__ double red[kEnergyThreads];
    for (int c = 0; c < kDots; ++c) {
        red[threadIdx.x] = t[c];
        __syncthreads();
        for (int h = kEnergyThreads / 2; h > 0; h /= 2) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[c * kEnergyBlocks + blockIdx.x] = red[0];
        __syncthreads();
    }
}

// E_1, E_2, E and dE/dc0 into out[0..3]; E and s = 2 G.D1 + F1.D1 (the
// coefficient of sigma in d(E_1 + E_2)/dsigma / 4) into scal[0..1].
__global__ void __launch_bounds__(kEnergyThreads)
energy_final_kernel(double c0, double n2, const double* partial, double* out, double* scal) {
    __shared__ double red[kEnergyThreads];
    __shared__ double dot[kDots];
    for (int c = 0; c < kDots; ++c) {
        double t = 0.0;
        for (int b = threadIdx.x; b < kEnergyBlocks; b += kEnergyThreads) t += partial[c * kEnergyBlocks + b];
        red[threadIdx.x] = t;
        __syncthreads();
        for (int h = kEnergyThreads / 2; h > 0; h /= 2) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) dot[c] = red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gd1 = dot[0], gd2 = dot[1], ga = dot[2], f1d1 = dot[3], f1d2 = dot[4], f1a = dot[5],
                     f2d2 = dot[6];
        const double e1 = 2.0 * n2 * gd1 + 4.0 * c0 * gd2 + 2.0 * ga;
        const double e2 = n2 * f1d1 + 4.0 * c0 * f1d2 + 2.0 * f1a + 2.0 * f2d2;
        const double e = (e1 + e2) / n2;
        const double dnum_c0 = 4.0 * c0 * gd1 + 4.0 * gd2 + 2.0 * c0 * f1d1 + 4.0 * f1d2;
        out[0] = e1;
        out[1] = e2;
        out[2] = e;
        out[3] = (dnum_c0 - 2.0 * c0 * e) / n2;
        scal[0] = e;
        scal[1] = 2.0 * gd1 + f1d1;
    }
}

// Quotient by N2: dsigma = (dsigma + 4 (s - E) sigma) / N2 (the numerator's
// sigma-gradient lacked its 4 s sigma term, and dN2/dsigma = 4 sigma),
// dtheta /= N2, dgamma /= N2.
__global__ void __launch_bounds__(256)
gradient_final_kernel(int64_t ns, int64_t nt, int64_t ng, double n2, const double* __restrict__ scal,
                      const double* __restrict__ sigma, double* dsigma, double* dtheta, double* dgamma) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double inv = 1.0 / n2;
    if (x < ns) {
        dsigma[x] = (dsigma[x] + 4.0 * (scal[1] - scal[0]) * sigma[x]) * inv;
    } else if (x < ns + nt) {
        dtheta[x - ns] *= inv;
    } else if (x < ns + nt + ng) {
        dgamma[x - ns - nt] *= inv;
    }
}

__global__ void __launch_bounds__(256)
axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
             double c, const double* __restrict__ z, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * x[i] + b * y[i] + c * z[i];
}

}  // namespace

// The energy and its first derivatives (see esmf_energy_gradient), with the
// numerator N = E_1 + E_2 differentiated as
//   dN/dTheta = Theta P1 + (sigma Gamma) P2 - 4 (sigma sigma^T)(Theta H)
//   dN/dGamma = sigma^T Z,  Z = 4 (c0 Theta H + (sigma Gamma) H + Theta F2)
//   dN/dsigma = 4 s sigma + Z Gamma^T - 4 (Theta H Theta^T) sigma
// and divided by N2 (E's own dependence on N2 in the last step).  Scratch
// `work`: gradient_work_doubles(n, no).
hipError_t launch_energy_gradient(int n, int no, int nv, double c0, double n2, const double* theta,
                                  const double* gamma, const double* sigma, const double* g, const double* d,
                                  const double* j, const double* k, double* energy, double* dsigma,
                                  double* dtheta, double* dgamma, double* work, hipStream_t s) {
    const int64_t nn = (int64_t)n * n, on = (int64_t)no * n;
    double* F2 = work;
    double* H = F2 + nn;
    double* P1 = H + nn;
    double* P2 = P1 + nn;
    double* TH = P2 + nn;
    double* SG = TH + on;
    double* SGH = SG + on;
    double* TF2 = SGH + on;
    double* Z = TF2 + on;
    double* SS = Z + on;
    double* THT = SS + (int64_t)no * no;
    double* partial = THT + (int64_t)no * no;
    double* scal = partial + kDots * kEnergyBlocks;
    hipError_t e;
#define ESMF_G(call)                     \
    do {                                 \
        e = (call);                      \
        if (e != hipSuccess) return e;   \
    } while (0)
    gradient_prep_kernel<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(n, c0, n2, g, j, k, F2, H, P1, P2);
    ESMF_G(hipGetLastError());
    energy_dots_kernel<<<kEnergyBlocks, kEnergyThreads, 0, s>>>(nn, g, d, j, k, partial);
    ESMF_G(hipGetLastError());
    energy_final_kernel<<<1, kEnergyThreads, 0, s>>>(c0, n2, partial, energy, scal);
    ESMF_G(hipGetLastError());
    ESMF_G((gemm<false, false>(no, n, n, 1.0, theta, n, H, n, 0.0, TH, n, s)));
    ESMF_G((gemm<false, false>(no, n, nv, 1.0, sigma, nv, gamma, n, 0.0, SG, n, s)));
    ESMF_G((gemm<false, false>(no, n, n, 1.0, SG, n, H, n, 0.0, SGH, n, s)));
    ESMF_G((gemm<false, false>(no, n, n, 1.0, theta, n, F2, n, 0.0, TF2, n, s)));
    ESMF_G((gemm<false, true>(no, no, nv, 1.0, sigma, nv, sigma, nv, 0.0, SS, no, s)));
    ESMF_G((gemm<false, true>(no, no, n, 1.0, TH, n, theta, n, 0.0, THT, no, s)));
    axpby_kernel<<<(unsigned)((on + 255) / 256), 256, 0, s>>>(on, 4.0 * c0, TH, 4.0, SGH, 4.0, TF2, Z);
    ESMF_G(hipGetLastError());
    // dN/dTheta
    ESMF_G((gemm<false, false>(no, n, n, 1.0, theta, n, P1, n, 0.0, dtheta, n, s)));
    ESMF_G((gemm<false, false>(no, n, n, 1.0, SG, n, P2, n, 1.0, dtheta, n, s)));
    ESMF_G((gemm<false, false>(no, n, no, -4.0, SS, no, TH, n, 1.0, dtheta, n, s)));
    // dN/dGamma
    ESMF_G((gemm<true, false>(nv, n, no, 1.0, sigma, nv, Z, n, 0.0, dgamma, n, s)));
    // dN/dsigma without its 4 s sigma term
    ESMF_G((gemm<false, true>(no, nv, n, 1.0, Z, n, gamma, n, 0.0, dsigma, nv, s)));
    ESMF_G((gemm<false, false>(no, nv, no, -4.0, THT, no, sigma, nv, 1.0, dsigma, nv, s)));
    const int64_t ns = (int64_t)no * nv, nt = on, ng = (int64_t)nv * n;
    const int64_t tot = ns + nt + ng;
    gradient_final_kernel<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(ns, nt, ng, n2, scal, sigma, dsigma,
                                                                         dtheta, dgamma);
    ESMF_G(hipGetLastError());
#undef ESMF_G
    return hipSuccess;
}

size_t gradient_work_doubles(int n, int no) {
    return (size_t)4 * n * n + (size_t)5 * no * n + (size_t)2 * no * no + (size_t)kDots * kEnergyBlocks + 2;
}

}  // namespace esmf
