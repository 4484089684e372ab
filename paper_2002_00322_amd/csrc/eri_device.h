// Device-side s-type electron repulsion integral of the library: shared by the
// store fill (prepare) and the integral-direct contraction, so that both hold
// the same value for every kept quartet.
#pragma once

#include <hip/hip_runtime.h>

namespace esmf {

constexpr double kPiD = 3.14159265358979323846264338327950288;

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
    return 0.5 * sqrt(kPiD / T) * erf(sqrt(T));
}

// Weighted, screened (ab|cd) of s primitives from the pair quantities of the
// two slot pairs (exponent sum z, centre P, prefactor E, Schwarz factor Q):
//   w E_ab E_cd 2 pi^(5/2) / (z_ab z_cd sqrt(z_ab + z_cd)) F0(T),
//   T = z_ab z_cd / (z_ab + z_cd) |P_ab - P_cd|^2,
// and 0 unless Q_ab Q_cd > tau (the quartet screen).
struct PairData {
    double z, px, py, pz, e, q;
};

__device__ inline double screened_eri(double w, const PairData& ab, const PairData& cd, double tau) {
    double v = 0.0;
    if (ab.q * cd.q > tau) {
        const double z = ab.z, e2 = cd.z;
        const double dx = ab.px - cd.px, dy = ab.py - cd.py, dz = ab.pz - cd.pz;
        const double R2 = dx * dx + dy * dy + dz * dz;
        const double T = z * e2 / (z + e2) * R2;
        const double pre = 2.0 * pow(kPiD, 2.5) / (z * e2 * sqrt(z + e2));
        v = w * (ab.e * cd.e * pre * boys_f0(T));
    }
    return v;
}

}  // namespace esmf
