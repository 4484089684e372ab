// Device-side s-type electron repulsion integral of the library: shared by the
// store fill (prepare) and the integral-direct contraction, so that both hold
// the same value for every kept quartet.
#pragma once

#include <hip/hip_runtime.h>

namespace esmf {

// The s-type integral in the form the library evaluates.  With
// rho = z_ab z_cd / (z_ab + z_cd), T = rho |P_ab - P_cd|^2 and
// G(T) = (2/sqrt(pi)) F0(T), the closed form
//   (ab|cd) = E_ab E_cd 2 pi^(5/2) / (z_ab z_cd sqrt(z_ab + z_cd)) F0(T)
// equals E'_ab E'_cd sqrt(rho) G(T) with E' = E (pi / z)^(3/2) per pair.
// Pair data therefore hold 1/z and E'; sqrt(rho) = (1/z_ab + 1/z_cd)^(-1/2).
// G(T) = erf(sqrt T) / sqrt T for T >= 1e-2 (ROCm's device erf, with
// sqrt T and its reciprocal from one reciprocal square root; 1 / sqrt T
// where that erf is exactly 1.0, T >= 36), else its
// Taylor series (2/sqrt(pi)) sum_k (-T)^k / (k! (2k+1)), 13 terms, far below
// FP64 rounding there; no division on either branch.  For
// T >= 36 the integral takes sqrt(rho) G(T) = sqrt(rho) / sqrt(T) =
// 1 / |P_ab - P_cd| (the point-charge limit, exact once erf is 1.0): one
// reciprocal square root instead of a square root and a division.
__device__ inline double boys_g(double T) {
    if (T < 1e-2) {
        // coefficients (2/sqrt(pi)) (-1)^k / (k! (2k+1)), k = 12 .. 0
        double g = 9.4227590646504113e-11;
        g = g * T - 1.2290555301717928e-09;
        g = g * T + 1.4807192815879218e-08;
        g = g * T - 1.6365844691234924e-07;
        g = g * T + 1.6462114365889248e-06;
        g = g * T - 1.492565035840625e-05;
        g = g * T + 0.00012055332981789664;
        g = g * T - 0.00085483270234508533;
        g = g * T + 0.0052239776254421879;
        g = g * T - 0.026866170645131252;
        g = g * T + 0.11283791670955126;
        g = g * T - 0.37612638903183754;
        g = g * T + 1.1283791670955126;
        return g;
    }
    // one reciprocal square root serves both sqrt(T) = T / sqrt(T) and the
    // quotient by it (no square root, no division)
    const double rs = rsqrt(T);
    // erf(r) rounds to 1.0 in FP64 from r ~ 5.92 (T ~ 35.1) on, so there
    // G = 1 / r exactly; most kept integrals of a large molecule lie there
    if (T >= 36.0) return rs;
    return erf(T * rs) * rs;
}

// Pair quantities of a slot pair: 1/z (z = exponent sum), centre P,
// E' = E (pi/z)^(3/2) (E = n_a n_b exp(-a_a a_b |A_a - A_b|^2 / z)), and the
// Schwarz factor Q = sqrt((ab|ab)).
struct PairData {
    double iz, px, py, pz, e, q;
};

// Weighted, screened (ab|cd): w E'_ab E'_cd sqrt(rho) G(T), and 0 unless
// Q_ab Q_cd > tau (the quartet screen).
__device__ inline double screened_eri(double w, const PairData& ab, const PairData& cd, double tau) {
    double v = 0.0;
    if (ab.q * cd.q > tau) {
        const double sr = rsqrt(ab.iz + cd.iz);   // sqrt(rho)
        const double dx = ab.px - cd.px, dy = ab.py - cd.py, dz = ab.pz - cd.pz;
        const double d2 = dx * dx + dy * dy + dz * dz;
        const double T = sr * sr * d2;
        const double g = T >= 36.0 ? rsqrt(d2) : sr * boys_g(T);   // sqrt(rho) G(T)
        v = w * (ab.e * cd.e * g);
    }
    return v;
}

}  // namespace esmf
