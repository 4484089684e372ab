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
// integrals of granule g if it is kept, into LDS at its rank among the kept
// granules; the workgroup then writes the block's packed granules, with the
// zero padding of its last row of 16 granules, as one contiguous run
// (consecutive threads, consecutive values).  A thread writing its own 16
// values straight to the store would put 8 useful bytes in every 32-byte
// write request of a wave.  The pair data of the block's 64 ket pairs are
// staged in LDS first (the lanes of a wave read 4 distinct ket pairs per
// integral: broadcasts), instead of 96 scattered global loads per thread.
template <typename StoreT>
__global__ void __launch_bounds__(256)
eri_fill_kernel(const int32_t* __restrict__ blk_tiles, const double* __restrict__ wts,
                const uint64_t* __restrict__ mask, const int64_t* __restrict__ off, int nslots,
                const double* __restrict__ pz, const double* __restrict__ px,
                const double* __restrict__ py, const double* __restrict__ pzc,
                const double* __restrict__ pe, const double* __restrict__ pq, double tau,
                StoreT* __restrict__ vals) {
    // granule r at sv[17 r .. 17 r + 15]: the odd stride spreads the 16
    // stores of the lanes of a wave over distinct banks
    constexpr int kStride = kGranule + 1;
    __shared__ StoreT sv[kGranules * kStride];
    __shared__ double sket[6 * 64];   // [array][k * 8 + l]: 1/z, Px, Py, Pz, E', Q
    const int64_t b = blockIdx.x;
    const int I = blk_tiles[4 * b + 0], J = blk_tiles[4 * b + 1];
    const int K = blk_tiles[4 * b + 2], L = blk_tiles[4 * b + 3];
    const double w = wts[b];
    const int g = threadIdx.x, wv = g >> 6, ln = g & 63;
    // 384 values, one or two per thread: value v is array v / 64, ket pair v % 64
    for (int v = g; v < 6 * 64; v += 256) {
        const int arr = v >> 6, kl = v & 63;
        const int64_t cd = (int64_t)(K * kTile + (kl >> 3)) * nslots + (L * kTile + (kl & 7));
        const double* src = arr == 0 ? pz : arr == 1 ? px : arr == 2 ? py : arr == 3 ? pzc : arr == 4 ? pe : pq;
        sket[v] = src[cd];
    }
    __syncthreads();
    const uint64_t* mk = mask + 4 * b;
    const uint64_t m0 = mk[0], m1 = mk[1], m2 = mk[2], m3 = mk[3];
    const uint64_t mw = wv == 0 ? m0 : wv == 1 ? m1 : wv == 2 ? m2 : m3;
    const int cnt = __popcll(m0) + __popcll(m1) + __popcll(m2) + __popcll(m3);
    if ((mw >> ln) & 1) {
        const int rank = (wv > 0 ? __popcll(m0) : 0) + (wv > 1 ? __popcll(m1) : 0) + (wv > 2 ? __popcll(m2) : 0) +
                         __popcll(mw & ((ln == 0) ? 0ull : (~0ull >> (64 - ln))));
        const int i = g >> 5, j = (g >> 2) & 7, kp = g & 3;
        const int64_t ab = (int64_t)(I * kTile + i) * nslots + (J * kTile + j);
        const PairData pab{pz[ab], px[ab], py[ab], pzc[ab], pe[ab], pq[ab]};
        for (int u = 0; u < kGranule; ++u) {
            const int kl = (2 * kp + (u >> 3)) * 8 + (u & 7);
            const PairData pcd{sket[kl], sket[64 + kl], sket[128 + kl], sket[192 + kl], sket[256 + kl],
                               sket[320 + kl]};
            sv[rank * kStride + u] = (StoreT)screened_eri(w, pab, pcd, tau);
        }
    }
    __syncthreads();
    const int nval = (cnt + kGranuleRow - 1) / kGranuleRow * kGranuleRow * kGranule;
    StoreT* out = vals + off[b] * kGranule;
    for (int x = g; x < nval; x += 256) {
        const int r = x / kGranule;
        out[x] = r < cnt ? sv[r * kStride + (x % kGranule)] : (StoreT)0;
    }
}

// ---- Cartesian functions of higher angular momentum -----------------------
// phi = N x_A^l y_A^m z_A^n exp(-a r_A^2), l, m, n <= 2, with
// N = (2a/pi)^(3/4) (4a)^((l+m+n)/2) / sqrt((2l-1)!! (2m-1)!! (2n-1)!!).
// Integrals by the McMurchie-Davidson scheme: Hermite expansion of each
// pair product about its centre P, Hermite Coulomb integrals R_tuv from the
// Boys functions F_n, n <= 8.

// F_0 .. F_8 at T.  For T <= 36 the tabulated Taylor expansion of McMurchie
// and Davidson (J. Comput. Phys. 26, 218 (1978)) about the nearest grid
// point T_g = g / 16, x = T_g - T (|x| <= 1/32):
//   F_8(T) = sum_{j=0}^{7} F_{8+j}(T_g) x^j / j!,
// with F_14 .. F_8 at T_g from the table's F_15(T_g) and exp(-T_g) by the
// downward recursion F_k = (2 T_g F_{k+1} + exp(-T_g)) / (2k + 1); then
// F_7 .. F_0 at T by the same recursion at T.  Above 36, where erf(sqrt T) is
// 1.0 in FP64, F_0 = (1/2) sqrt(pi / T) and the upward recursion
// F_{n+1} = ((2n + 1) F_n - exp(-T)) / (2T), stable there for n <= 8.
// Fixed loops, no division below 36.
__device__ void boys_fn8(double T, double* F) {
    const double et = exp(-T);
    if (T <= 36.0) {
        const double g = rint(T * kBoysPerUnit);
        const double Tg = g * (1.0 / kBoysPerUnit);
        const double x = Tg - T;
        const double* e = kBoysTableHigh[(int)g];
        const double t2 = 2.0 * Tg;
        static_assert(kBoysOrderHigh == 15, "F_8 is expanded over F_8 .. F_15");
        double f[8];
        f[7] = e[0];   // F_15(T_g)
#pragma unroll
        for (int k = 14; k >= 8; --k) f[k - 8] = (t2 * f[k - 7] + e[1]) * (1.0 / (2 * k + 1));
        double s = f[7];
#pragma unroll
        for (int j = 6; j >= 0; --j) s = f[j] + (x * (1.0 / (j + 1))) * s;
        F[8] = s;
        const double t2x = 2.0 * T;
#pragma unroll
        for (int n = 7; n >= 0; --n) F[n] = (t2x * F[n + 1] + et) * (1.0 / (2 * n + 1));
    } else {
        F[0] = 0.5 * sqrt(kPi / T);
#pragma unroll
        for (int n = 0; n < 8; ++n) F[n + 1] = ((double)(2 * n + 1) * F[n] - et) / (2.0 * T);
    }
}

// Hermite coefficients E_t (t <= la + lb <= 4) of one Cartesian direction:
// start from exp(-ab/p (A-B)^2) and raise the power of x_A la times, then of
// x_B lb times: E'_t = E_{t-1}/(2p) + X E_t + (t+1) E_{t+1}, X = P-A or P-B.
__device__ void hermite_coeffs(int la, int lb, double a, double b, double A, double B, double* e) {
    const double p = a + b, P = (a * A + b * B) / p, h = 0.5 / p;
    double c[5] = {exp(-a * b / p * (A - B) * (A - B)), 0.0, 0.0, 0.0, 0.0};
    int deg = 0;
    for (int step = 0; step < la + lb; ++step) {
        const double X = step < la ? P - A : P - B;
        double nc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int t = 0; t <= deg + 1; ++t) {
            double v = t <= deg ? X * c[t] : 0.0;
            if (t >= 1) v += h * c[t - 1];
            if (t + 1 <= deg) v += (double)(t + 1) * c[t + 1];
            nc[t] = v;
        }
        ++deg;
        for (int t = 0; t < 5; ++t) c[t] = nc[t];
    }
    for (int t = 0; t < 5; ++t) e[t] = c[t];
}

// Linear index of (t, u, v), t + u + v <= 8: triples of smaller sum first,
// then by u + v, then v.  165 triples in all.
__device__ __forceinline__ int tuv_index(int t, int u, int v) {
    const int s = t + u + v, r = u + v;
    return s * (s + 1) * (s + 2) / 6 + r * (r + 1) / 2 + v;
}
constexpr int kTuv = 165;

// R^0_tuv for t + u + v <= L: layers n = L .. 0, each from the one above,
//   R^n_000 = (-2 alpha)^n F_n,  R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{tuv}
// (the first non-zero index lowered: t, else u with Y, else v with Z).
__device__ void hermite_r0(int L, double alpha, double X, double Y, double Z, double* R0) {
    double F[9];
    boys_fn8(alpha * (X * X + Y * Y + Z * Z), F);
    double lay[2][kTuv];
    double fac[9];
    fac[0] = 1.0;
    for (int n = 1; n <= L; ++n) fac[n] = fac[n - 1] * (-2.0 * alpha);
    lay[L & 1][0] = fac[L] * F[L];
    for (int n = L - 1; n >= 0; --n) {
        double* cur = lay[n & 1];
        const double* up = lay[(n + 1) & 1];
        cur[0] = fac[n] * F[n];
        for (int sum = 1; sum <= L - n; ++sum)
            for (int r = 0; r <= sum; ++r)
                for (int v = 0; v <= r; ++v) {
                    const int u = r - v, t = sum - r;
                    double val;
                    if (t > 0)
                        val = (t > 1 ? (double)(t - 1) * up[tuv_index(t - 2, u, v)] : 0.0) +
                              X * up[tuv_index(t - 1, u, v)];
                    else if (u > 0)
                        val = (u > 1 ? (double)(u - 1) * up[tuv_index(t, u - 2, v)] : 0.0) +
                              Y * up[tuv_index(t, u - 1, v)];
                    else
                        val = (v > 1 ? (double)(v - 1) * up[tuv_index(t, u, v - 2)] : 0.0) +
                              Z * up[tuv_index(t, u, v - 1)];
                    cur[tuv_index(t, u, v)] = val;
                }
    }
    const int cnt = (L + 1) * (L + 2) * (L + 3) / 6;
    for (int i = 0; i < cnt; ++i) R0[i] = lay[0][i];
}

__device__ inline double cart_norm(double a, int l, int m, int n) {
    auto df = [](int k) { return k == 3 ? 3.0 : 1.0; };  // (2l-1)!! for l <= 2
    return pow(2.0 * a / kPi, 0.75) * pow(4.0 * a, 0.5 * (l + m + n)) / sqrt(df(2 * l - 1) * df(2 * m - 1) * df(2 * n - 1));
}

// Primitive integral (ab|cd) over normalised Cartesian primitives with
// centres A[k], exponents x[k] and powers l[k].
__device__ double cart_prim_eri(const double (&A)[4][3], const double (&x)[4], const int (&l)[4][3]) {
    int L = 0;
    for (int k = 0; k < 4; ++k) L += l[k][0] + l[k][1] + l[k][2];
    double eab[3][5], ecd[3][5];
    double P[3], Q[3];
    const double p = x[0] + x[1], q = x[2] + x[3];
    for (int d = 0; d < 3; ++d) {
        hermite_coeffs(l[0][d], l[1][d], x[0], x[1], A[0][d], A[1][d], eab[d]);
        hermite_coeffs(l[2][d], l[3][d], x[2], x[3], A[2][d], A[3][d], ecd[d]);
        P[d] = (x[0] * A[0][d] + x[1] * A[1][d]) / p;
        Q[d] = (x[2] * A[2][d] + x[3] * A[3][d]) / q;
    }
    double R[kTuv];
    hermite_r0(L, p * q / (p + q), P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], R);
    double sum = 0.0;
    for (int t = 0; t <= l[0][0] + l[1][0]; ++t)
        for (int u = 0; u <= l[0][1] + l[1][1]; ++u)
            for (int v = 0; v <= l[0][2] + l[1][2]; ++v) {
                const double e1 = eab[0][t] * eab[1][u] * eab[2][v];
                for (int tt = 0; tt <= l[2][0] + l[3][0]; ++tt)
                    for (int uu = 0; uu <= l[2][1] + l[3][1]; ++uu)
                        for (int vv = 0; vv <= l[2][2] + l[3][2]; ++vv) {
                            const double e2 = ecd[0][tt] * ecd[1][uu] * ecd[2][vv];
                            const double sg = ((tt + uu + vv) & 1) ? -e2 : e2;
                            sum += e1 * sg * R[tuv_index(t + tt, u + uu, v + vv)];
                        }
            }
    double nrm = 1.0;
    for (int k = 0; k < 4; ++k) nrm *= cart_norm(x[k], l[k][0], l[k][1], l[k][2]);
    return 2.0 * pow(kPi, 2.5) / (p * q * sqrt(p + q)) * sum * nrm;
}

// Description of the functions of a Cartesian basis: centre, powers, and the
// primitives [off[f], off[f+1]) of function f with exponents and
// coefficients (the function's normalisation included).  A primitive basis
// has one primitive of coefficient 1 per function.
struct CartBasis {
    const double* cen;
    const int8_t* lmn;
    const int32_t* off;
    const double* pexp;
    const double* pcoef;
};

// (ab|cd) over the functions fa, fb, fc, fd: the coefficient-weighted sum of
// the primitive integrals.
__device__ __attribute__((noinline)) double cart_eri(const CartBasis& B, int fa, int fb, int fc, int fd) {
    const int f[4] = {fa, fb, fc, fd};
    int l[4][3];
    double A[4][3];
    for (int k = 0; k < 4; ++k)
        for (int d = 0; d < 3; ++d) {
            l[k][d] = B.lmn[3 * f[k] + d];
            A[k][d] = B.cen[3 * f[k] + d];
        }
    double sum = 0.0;
    for (int ka = B.off[fa]; ka < B.off[fa + 1]; ++ka)
        for (int kb = B.off[fb]; kb < B.off[fb + 1]; ++kb)
            for (int kc = B.off[fc]; kc < B.off[fc + 1]; ++kc)
                for (int kd = B.off[fd]; kd < B.off[fd + 1]; ++kd) {
                    const double x[4] = {B.pexp[ka], B.pexp[kb], B.pexp[kc], B.pexp[kd]};
                    sum += B.pcoef[ka] * B.pcoef[kb] * B.pcoef[kc] * B.pcoef[kd] * cart_prim_eri(A, x, l);
                }
    return sum;
}

// A function the s-type pair data describe: an s function of one primitive
// of coefficient 1.
__device__ __forceinline__ bool is_simple(const CartBasis& B, int f) {
    return (B.lmn[3 * f] | B.lmn[3 * f + 1] | B.lmn[3 * f + 2]) == 0 && B.off[f + 1] - B.off[f] == 1 &&
           B.pcoef[B.off[f]] == 1.0;
}

// Schwarz factors of slot pairs with a function the s-type form does not
// describe: Q = sqrt((ab|ab)), over the value pair_build wrote.
__global__ void cart_pair_q_kernel(int nslots, const int32_t* __restrict__ slot_fn, CartBasis B, double* pq) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)nslots * nslots) return;
    const int fa = slot_fn[idx / nslots], fb = slot_fn[idx % nslots];
    if (fa < 0 || fb < 0 || (is_simple(B, fa) && is_simple(B, fb))) return;
    pq[idx] = sqrt(fmax(cart_eri(B, fa, fb, fa, fb), 0.0));
}

// Fill of the kept granules of a Cartesian basis: the s-type form where all
// four functions are simple s functions, the Cartesian one otherwise; the
// same screen Q_ab Q_cd > tau.
template <typename StoreT>
__global__ void __launch_bounds__(256)
eri_fill_cart_kernel(const int32_t* __restrict__ blk_tiles, const double* __restrict__ wts,
                     const uint64_t* __restrict__ mask, const int64_t* __restrict__ off, int nslots,
                     const double* __restrict__ pz, const double* __restrict__ px,
                     const double* __restrict__ py, const double* __restrict__ pzc,
                     const double* __restrict__ pe, const double* __restrict__ pq, double tau,
                     const int32_t* __restrict__ slot_fn, CartBasis B, StoreT* __restrict__ vals) {
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
    const int sa = I * kTile + i, sb = J * kTile + j;
    const int64_t ab = (int64_t)sa * nslots + sb;
    const PairData pab{pz[ab], px[ab], py[ab], pzc[ab], pe[ab], pq[ab]};
    const int fa = slot_fn[sa], fb = slot_fn[sb];
    const bool ab_simple = fa < 0 || fb < 0 || (is_simple(B, fa) && is_simple(B, fb));
    for (int u = 0; u < kGranule; ++u) {
        const int sc = K * kTile + 2 * kp + (u >> 3), sd = L * kTile + (u & 7);
        const int64_t cd = (int64_t)sc * nslots + sd;
        const PairData pcd{pz[cd], px[cd], py[cd], pzc[cd], pe[cd], pq[cd]};
        const int fc = slot_fn[sc], fd = slot_fn[sd];
        double v = 0.0;
        if (ab_simple && (fc < 0 || fd < 0 || (is_simple(B, fc) && is_simple(B, fd))))
            v = screened_eri(w, pab, pcd, tau);
        else if (fa >= 0 && fb >= 0 && fc >= 0 && fd >= 0 && pab.q * pcd.q > tau)
            v = w * cart_eri(B, fa, fb, fc, fd);
        out[u] = (StoreT)v;
    }
}

}  // namespace

hipError_t launch_cart_pair_q(int nslots, const int32_t* d_slot_fn, const double* d_centers, const int8_t* d_lmn,
                              const int32_t* d_off, const double* d_pexp, const double* d_pcoef, double* d_pq,
                              hipStream_t s) {
    const int64_t total = (int64_t)nslots * nslots;
    const CartBasis B{d_centers, d_lmn, d_off, d_pexp, d_pcoef};
    cart_pair_q_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(nslots, d_slot_fn, B, d_pq);
    return hipGetLastError();
}

hipError_t launch_eri_fill_cart(int64_t nblocks, const int32_t* d_blk_tiles, const double* d_w,
                                const uint64_t* d_mask, const int64_t* d_off, int nslots, const double* d_pz,
                                const double* d_px, const double* d_py, const double* d_pzc, const double* d_pe,
                                const double* d_pq, double tau, const int32_t* d_slot_fn, const double* d_centers,
                                const int8_t* d_lmn, const int32_t* d_poff, const double* d_pexp,
                                const double* d_pcoef, void* d_vals, int fp32, hipStream_t s) {
    const CartBasis B{d_centers, d_lmn, d_poff, d_pexp, d_pcoef};
    // one 256-thread workgroup per block; a launch holds fewer than 2^32
    // work items
    const int64_t chunk = (int64_t)1 << 22;
    for (int64_t b0 = 0; b0 < nblocks; b0 += chunk) {
        const int64_t nb = nblocks - b0 < chunk ? nblocks - b0 : chunk;
        if (fp32)
            eri_fill_cart_kernel<float><<<(unsigned)nb, 256, 0, s>>>(
                d_blk_tiles + 4 * b0, d_w + b0, d_mask + 4 * b0, d_off + b0, nslots, d_pz, d_px, d_py, d_pzc, d_pe,
                d_pq, tau, d_slot_fn, B, (float*)d_vals);
        else
            eri_fill_cart_kernel<double><<<(unsigned)nb, 256, 0, s>>>(
                d_blk_tiles + 4 * b0, d_w + b0, d_mask + 4 * b0, d_off + b0, nslots, d_pz, d_px, d_py, d_pzc, d_pe,
                d_pq, tau, d_slot_fn, B, (double*)d_vals);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

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
    // one 256-thread workgroup per block; a launch holds fewer than 2^32
    // work items
    const int64_t chunk = (int64_t)1 << 22;
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
    // one 256-thread workgroup per block; a launch holds fewer than 2^32
    // work items
    const int64_t chunk = (int64_t)1 << 22;
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
