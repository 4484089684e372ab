// Device-side s-type electron repulsion integral of the library: shared by the
// store fill (prepare) and the integral-direct contraction, so that both hold
// the same value for every kept quartet.
#pragma once

#include <hip/hip_runtime.h>

#include "boys_table.h"

namespace esmf {

// The s-type integral in the form the library evaluates.  With
// rho = z_ab z_cd / (z_ab + z_cd), T = rho |P_ab - P_cd|^2 and
// G(T) = (2/sqrt(pi)) F0(T), the closed form
//   (ab|cd) = E_ab E_cd 2 pi^(5/2) / (z_ab z_cd sqrt(z_ab + z_cd)) F0(T)
// equals E'_ab E'_cd sqrt(rho) G(T) with E' = E (pi / z)^(3/2) per pair.
// Pair data therefore hold 1/z and E'; sqrt(rho) = (1/z_ab + 1/z_cd)^(-1/2).
//
// G(T) for 0 <= T <= 36: the tabulated Taylor expansion of McMurchie and
// Davidson (J. Comput. Phys. 26, 218 (1978)) about the grid point
// T_g = g / 16 nearest T, x = T_g - T (|x| <= 1/32):
//   G(T) = sum_{k=0}^{7} G_k(T_g) x^k / k!,   G_k = (2/sqrt(pi)) F_k.
// The table holds G_7(T_g) and (2/sqrt(pi)) exp(-T_g); G_6 .. G_0 at T_g follow
// by the (stable) downward recursion G_k = (2 T_g G_{k+1} + (2/sqrt(pi))
// exp(-T_g)) / (2k + 1), each step interleaved with a Horner step of the sum.
// The truncation error is below G_8 (1/32)^8 / 8! < 2e-18; against F0 from
// erf and its series the result is within 1e-15 relative.  No branch, no
// division, one 16-byte table load.
// For T > 36 the integral takes sqrt(rho) G(T) = 1 / |P_ab - P_cd| (the
// point-charge limit: erf(sqrt T) is 1.0 in FP64 there), one reciprocal
// square root.
__device__ inline double boys_g(double T) {
    const double g = rint(fmin(T, 36.0) * kBoysPerUnit);
    const double Tg = g * (1.0 / kBoysPerUnit);
    const double x = Tg - T;
    const double* e = kBoysTable[(int)g];
    const double ex = e[1];            // (2/sqrt(pi)) exp(-T_g)
    const double t2 = 2.0 * Tg;
    double gk = e[0];                  // G_7(T_g)
    double s = gk;
    static_assert(kBoysOrder == 7, "the recursion below runs from order 7");
#pragma unroll
    for (int k = kBoysOrder - 1; k >= 0; --k) {
        gk = (t2 * gk + ex) * (1.0 / (2 * k + 1));
        s = gk + (x * (1.0 / (k + 1))) * s;
    }
    return s;
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
        const double gt = sr * boys_g(T);   // table form, evaluated by every lane
        const double g = T > 36.0 ? rsqrt(d2) : gt;   // sqrt(rho) G(T)
        v = w * (ab.e * cd.e * g);
    }
    return v;
}

}  // namespace esmf
