/*
 * esmf_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference for the grouped multi-density Fock build
 * of excited-state mean-field theory (Zhao & Neuscamman, arXiv:2002.00322).
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library; the product path never does, and it
 * shares no code, header or table with the HIP library.
 *
 * What it computes (all FP64, Hartree atomic units, bohr):
 *   - normalised s-type Gaussian primitives phi_p(r) = n_p exp(-a_p |r-A_p|^2),
 *     n_p = (2 a_p / pi)^(3/4);
 *   - the two-electron integrals (pq|rs) in chemists' (1122) notation, as the
 *     paper's generalised J/K definition uses them (Sec. "Notation",
 *     Eq. J_and_K), from the textbook s-type closed form with the Boys
 *     function F0 (the paper takes its integrals from standard s/p/d engines,
 *     Sec. "Computational Details"; the s-type form is Szabo-Ostlund's);
 *   - the Schwarz factor Q_pq = sqrt((pq|pq));
 *   - screening: a quartet takes part iff Q_pq * Q_rs > tau, the product taken
 *     in FP64 (Sec. "Shell-Pair Screening" screens on the size of the
 *     integrals a pair can produce; the Schwarz product is that size's bound);
 *   - J[D]_pq = sum_rs D_rs (rs|pq) and K[D]_pq = sum_rs D_rs (pr|qs) for
 *     any, not necessarily symmetric, D (Eq. J_and_K), for m densities.
 *
 * Two contraction routes are provided:
 *   oracle_jk_literal   -- the definition written out: a plain quadruple sum
 *                          over all (p,q,r,s); O(m N^4); small N only.
 *   oracle_jk_canonical -- the paper's grouped build: one threaded loop over
 *                          the retained pairs (Sec. "Shell-Pair Screening"),
 *                          each unique integral visited once and scattered to
 *                          every density's J and K through its 8 index
 *                          permutations, with degeneracy weights.
 *   oracle_jk_entries   -- the definition evaluated one output entry at a
 *                          time (O(N^2) per entry), for sampled checks at
 *                          sizes where the full build is too slow.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORACLE_PI = 3.14159265358979323846264338327950288;

/* Boys function of order zero, F0(T) = int_0^1 exp(-T u^2) du.
 * Small T: its Taylor series sum_k (-T)^k / (k! (2k+1)), summed until a term
 * drops below 1e-17 of the sum. Otherwise the closed form
 * (1/2) sqrt(pi/T) erf(sqrt(T)). */
double oracle_boys_f0(double T)
{
    if (T < 1e-2) {
        double term = 1.0, sum = 1.0;
        for (int k = 1; k < 40; ++k) {
            term *= -T / (double)k;
            double c = term / (double)(2 * k + 1);
            sum += c;
            if (fabs(c) < 1e-17 * fabs(sum)) break;
        }
        return sum;
    }
    return 0.5 * sqrt(ORACLE_PI / T) * erf(sqrt(T));
}

/* Normalisation of an s primitive. */
static double norm_s(double a) { return pow(2.0 * a / ORACLE_PI, 0.75); }

/* Gaussian product of primitives p and q: exponent zeta, centre P, prefactor
 * E = n_p n_q exp(-a_p a_q |A_p - A_q|^2 / zeta). */
static void gaussian_product(const double* A, const double* alpha, int p, int q,
                             double* zeta, double P[3], double* E)
{
    double ap = alpha[p], aq = alpha[q];
    double z = ap + aq;
    double r2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        double d = A[3 * p + x] - A[3 * q + x];
        r2 += d * d;
        P[x] = (ap * A[3 * p + x] + aq * A[3 * q + x]) / z;
    }
    *zeta = z;
    *E = norm_s(ap) * norm_s(aq) * exp(-ap * aq * r2 / z);
}

/* (pq|rs) = E_pq E_rs 2 pi^(5/2) / (zeta eta sqrt(zeta+eta)) F0(T),
 * T = zeta eta / (zeta+eta) |P - Q|^2. */
double oracle_eri(const double* A, const double* alpha, int p, int q, int r, int s)
{
    double z, e, P[3], Q[3], Epq, Ers;
    gaussian_product(A, alpha, p, q, &z, P, &Epq);
    gaussian_product(A, alpha, r, s, &e, Q, &Ers);
    double R2 = 0.0;
    for (int x = 0; x < 3; ++x) {
        double d = P[x] - Q[x];
        R2 += d * d;
    }
    double T = z * e / (z + e) * R2;
    double pre = 2.0 * pow(ORACLE_PI, 2.5) / (z * e * sqrt(z + e));
    return Epq * Ers * pre * oracle_boys_f0(T);
}

/* ---- Cartesian Gaussian functions of higher angular momentum ----------
 * phi(r) = N x_A^l y_A^m z_A^n exp(-a |r - A|^2), x_A = x - A_x, with
 * N = (2a/pi)^(3/4) (4a)^((l+m+n)/2) / sqrt((2l-1)!! (2m-1)!! (2n-1)!!),
 * l, m, n <= 2 (s, p and d functions).  The paper's integrals over s, p and
 * d functions (Sec. "Computational Details") are evaluated here with the
 * McMurchie-Davidson scheme: each pair's product is expanded in Hermite
 * Gaussians about its centre P, and the Coulomb integral of two Hermite
 * Gaussians is a Hermite derivative of the Boys function. */

/* Boys functions F_n(T) = int_0^1 u^(2n) exp(-T u^2) du, n = 0..nmax.
 * T < 35: F_nmax from the convergent series
 *   exp(-T) sum_k (2T)^k / ((2 nmax + 1)(2 nmax + 3)...(2 nmax + 2k + 1)),
 * then downward F_n = (2T F_{n+1} + exp(-T)) / (2n + 1); otherwise F_0 in
 * closed form and upward F_{n+1} = ((2n + 1) F_n - exp(-T)) / (2T). */
void oracle_boys_fn(int nmax, double T, double* F)
{
    double et = exp(-T);
    if (T < 35.0) {
        double term = 1.0 / (double)(2 * nmax + 1), sum = term;
        for (int k = 1; k < 1000; ++k) {
            term *= 2.0 * T / (double)(2 * nmax + 2 * k + 1);
            sum += term;
            if (term < 1e-17 * sum) break;
        }
        F[nmax] = et * sum;
        for (int n = nmax - 1; n >= 0; --n) F[n] = (2.0 * T * F[n + 1] + et) / (double)(2 * n + 1);
    } else {
        F[0] = 0.5 * sqrt(ORACLE_PI / T) * erf(sqrt(T));
        for (int n = 0; n < nmax; ++n) F[n + 1] = ((double)(2 * n + 1) * F[n] - et) / (2.0 * T);
    }
}

static double dfact(int k) { double r = 1.0; for (; k > 1; k -= 2) r *= (double)k; return r; }

static double norm_cart(double a, const int* l)
{
    int L = l[0] + l[1] + l[2];
    return pow(2.0 * a / ORACLE_PI, 0.75) * pow(4.0 * a, 0.5 * L) /
           sqrt(dfact(2 * l[0] - 1) * dfact(2 * l[1] - 1) * dfact(2 * l[2] - 1));
}

/* Hermite expansion of a one-dimensional product x_A^i x_B^j
 * exp(-a x_A^2 - b x_B^2) = sum_t E[i][j][t] Lambda_t(x_P) about P:
 *   E[0][0][0] = exp(-ab/(a+b) (A - B)^2),
 *   E[i+1][j][t] = E[i][j][t-1] / (2p) + (P - A) E[i][j][t] + (t+1) E[i][j][t+1],
 *   E[i][j+1][t] = E[i][j][t-1] / (2p) + (P - B) E[i][j][t] + (t+1) E[i][j][t+1],
 * p = a + b, zero outside 0 <= t <= i + j. */
static void hermite_e(int la, int lb, double a, double b, double A, double B, double E[3][3][5])
{
    double p = a + b, P = (a * A + b * B) / p;
    memset(E, 0, sizeof(double) * 45);
    E[0][0][0] = exp(-a * b / p * (A - B) * (A - B));
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j <= lb; ++j) {
            if (i == 0 && j == 0) continue;
            int fromA = j == 0;          /* raise i from (i-1, 0), else j from (i, j-1) */
            int pi = fromA ? i - 1 : i, pj = fromA ? j : j - 1;
            double X = fromA ? P - A : P - B;
            for (int t = 0; t <= i + j; ++t) {
                double v = X * (t <= pi + pj ? E[pi][pj][t] : 0.0);
                if (t >= 1) v += E[pi][pj][t - 1] / (2.0 * p);
                if (t + 1 <= pi + pj) v += (double)(t + 1) * E[pi][pj][t + 1];
                E[i][j][t] = v;
            }
        }
}

/* Hermite Coulomb integrals R^0_{tuv}, t + u + v <= L (<= 8), of exponent
 * alpha and separation (X, Y, Z):
 *   R^n_{000} = (-2 alpha)^n F_n(alpha |PQ|^2),
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v}   (likewise u, v). */
static void hermite_r(int L, double alpha, double X, double Y, double Z, double R[9][9][9][9])
{
    double F[9];
    oracle_boys_fn(L, alpha * (X * X + Y * Y + Z * Z), F);
    double f = 1.0;
    for (int n = 0; n <= L; ++n) {
        R[n][0][0][0] = f * F[n];
        f *= -2.0 * alpha;
    }
    for (int sum = 1; sum <= L; ++sum)
        for (int t = 0; t <= sum; ++t)
            for (int u = 0; u <= sum - t; ++u) {
                int v = sum - t - u;
                for (int n = 0; n <= L - sum; ++n) {
                    double r;
                    if (t > 0)
                        r = (t > 1 ? (t - 1) * R[n + 1][t - 2][u][v] : 0.0) + X * R[n + 1][t - 1][u][v];
                    else if (u > 0)
                        r = (u > 1 ? (u - 1) * R[n + 1][t][u - 2][v] : 0.0) + Y * R[n + 1][t][u - 1][v];
                    else
                        r = (v > 1 ? (v - 1) * R[n + 1][t][u][v - 2] : 0.0) + Z * R[n + 1][t][u][v - 1];
                    R[n][t][u][v] = r;
                }
            }
}

/* (pq|rs) over Cartesian functions; lmn [n][3] holds each function's
 * (l, m, n).  For four s functions this is oracle_eri. */
double oracle_eri_cart(const double* A, const double* alpha, const int* lmn, int p, int q, int r, int s)
{
    const int* lp = lmn + 3 * p; const int* lq = lmn + 3 * q;
    const int* lr = lmn + 3 * r; const int* ls = lmn + 3 * s;
    double a = alpha[p], b = alpha[q], c = alpha[r], d = alpha[s];
    double zp = a + b, zq = c + d;
    double Eab[3][3][3][5], Ecd[3][3][3][5];
    double P[3], Q[3];
    for (int x = 0; x < 3; ++x) {
        hermite_e(lp[x], lq[x], a, b, A[3 * p + x], A[3 * q + x], Eab[x]);
        hermite_e(lr[x], ls[x], c, d, A[3 * r + x], A[3 * s + x], Ecd[x]);
        P[x] = (a * A[3 * p + x] + b * A[3 * q + x]) / zp;
        Q[x] = (c * A[3 * r + x] + d * A[3 * s + x]) / zq;
    }
    int L = lp[0] + lp[1] + lp[2] + lq[0] + lq[1] + lq[2] + lr[0] + lr[1] + lr[2] + ls[0] + ls[1] + ls[2];
    static __thread double R[9][9][9][9];
    hermite_r(L, zp * zq / (zp + zq), P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], R);
    double sum = 0.0;
    for (int t = 0; t <= lp[0] + lq[0]; ++t)
        for (int u = 0; u <= lp[1] + lq[1]; ++u)
            for (int v = 0; v <= lp[2] + lq[2]; ++v) {
                double eab = Eab[0][lp[0]][lq[0]][t] * Eab[1][lp[1]][lq[1]][u] * Eab[2][lp[2]][lq[2]][v];
                if (eab == 0.0) continue;
                for (int tt = 0; tt <= lr[0] + ls[0]; ++tt)
                    for (int uu = 0; uu <= lr[1] + ls[1]; ++uu)
                        for (int vv = 0; vv <= lr[2] + ls[2]; ++vv) {
                            double ecd = Ecd[0][lr[0]][ls[0]][tt] * Ecd[1][lr[1]][ls[1]][uu] *
                                         Ecd[2][lr[2]][ls[2]][vv];
                            double sg = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                            sum += eab * sg * ecd * R[0][t + tt][u + uu][v + vv];
                        }
            }
    double pre = 2.0 * pow(ORACLE_PI, 2.5) / (zp * zq * sqrt(zp + zq));
    return pre * sum * norm_cart(a, lp) * norm_cart(b, lq) * norm_cart(c, lr) * norm_cart(d, ls);
}

/* The integral of the build: the s-type closed form when all four functions
 * are s functions (or lmn is NULL), the Cartesian form otherwise. */
static double eri_any(const double* A, const double* alpha, const int* lmn, int p, int q, int r, int s)
{
    if (lmn) {
        const int* l[4] = {lmn + 3 * p, lmn + 3 * q, lmn + 3 * r, lmn + 3 * s};
        for (int k = 0; k < 4; ++k)
            if (l[k][0] | l[k][1] | l[k][2]) return oracle_eri_cart(A, alpha, lmn, p, q, r, s);
    }
    return oracle_eri(A, alpha, p, q, r, s);
}

/* Schwarz factors Q[p*n+q] = sqrt((pq|pq)) for all p, q (symmetric). */
static void schwarz_any(int n, const double* A, const double* alpha, const int* lmn, double* Q)
{
    for (int p = 0; p < n; ++p)
        for (int q = 0; q <= p; ++q) {
            double v = sqrt(eri_any(A, alpha, lmn, p, q, p, q));
            Q[p * n + q] = v;
            Q[q * n + p] = v;
        }
}

void oracle_schwarz(int n, const double* A, const double* alpha, double* Q)
{
    schwarz_any(n, A, alpha, NULL, Q);
}

void oracle_schwarz_cart(int n, const double* A, const double* alpha, const int* lmn, double* Q)
{
    schwarz_any(n, A, alpha, lmn, Q);
}

/* Screening predicate: the quartet takes part iff Q_pq * Q_rs > tau. */
static int keep_quartet(double qpq, double qrs, double tau) { return qpq * qrs > tau; }

/* Dense masked tensor T[((p*n+q)*n+r)*n+s] = (pq|rs) if kept else 0. Small n. */
static int eri_tensor_any(int n, const double* A, const double* alpha, const int* lmn, double tau, double* T)
{
    double* Q = (double*)malloc(sizeof(double) * (size_t)n * n);
    if (!Q) return -1;
    schwarz_any(n, A, alpha, lmn, Q);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    size_t idx = (((size_t)p * n + q) * n + r) * n + s;
                    T[idx] = keep_quartet(Q[p * n + q], Q[r * n + s], tau)
                                 ? eri_any(A, alpha, lmn, p, q, r, s) : 0.0;
                }
    free(Q);
    return 0;
}

int oracle_eri_tensor(int n, const double* A, const double* alpha, double tau, double* T)
{
    return eri_tensor_any(n, A, alpha, NULL, tau, T);
}

int oracle_eri_tensor_cart(int n, const double* A, const double* alpha, const int* lmn, double tau, double* T)
{
    return eri_tensor_any(n, A, alpha, lmn, tau, T);
}

/* Number of unique (8-fold) quartets that pass the screen, and number of pairs
 * p >= q with Q_pq * max Q > tau. */
static void count_any(int n, const double* A, const double* alpha, const int* lmn, double tau,
                  int64_t* n_pairs_kept, int64_t* n_quartets_kept)
{
    double* Q = (double*)malloc(sizeof(double) * (size_t)n * n);
    schwarz_any(n, A, alpha, lmn, Q);
    double qmax = 0.0;
    for (int i = 0; i < n * n; ++i) if (Q[i] > qmax) qmax = Q[i];
    int64_t np = 0, nq = 0;
    int64_t npair = (int64_t)n * (n + 1) / 2;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q <= p; ++q)
            if (keep_quartet(Q[p * n + q], qmax, tau)) ++np;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+ : nq)
    for (int64_t a = 0; a < npair; ++a) {
        int p = (int)floor((sqrt(8.0 * (double)a + 1.0) - 1.0) / 2.0);
        while ((int64_t)p * (p + 1) / 2 > a) --p;
        while ((int64_t)(p + 1) * (p + 2) / 2 <= a) ++p;
        int q = (int)(a - (int64_t)p * (p + 1) / 2);
        double qa = Q[p * n + q];
        for (int r = 0; r < n; ++r)
            for (int s = 0; s <= r; ++s) {
                int64_t b = (int64_t)r * (r + 1) / 2 + s;
                if (b > a) break;
                if (keep_quartet(qa, Q[r * n + s], tau)) ++nq;
            }
    }
    *n_pairs_kept = np;
    *n_quartets_kept = nq;
    free(Q);
}

void oracle_count(int n, const double* A, const double* alpha, double tau,
                  int64_t* n_pairs_kept, int64_t* n_quartets_kept)
{
    count_any(n, A, alpha, NULL, tau, n_pairs_kept, n_quartets_kept);
}

void oracle_count_cart(int n, const double* A, const double* alpha, const int* lmn, double tau,
                  int64_t* n_pairs_kept, int64_t* n_quartets_kept)
{
    count_any(n, A, alpha, lmn, tau, n_pairs_kept, n_quartets_kept);
}

/* The definition written out (Eq. J_and_K):
 *   J_i[p][q] = sum_{r,s} D_i[r][s] (rs|pq),  K_i[p][q] = sum_{r,s} D_i[r][s] (pr|qs),
 * over every index, no symmetry used. D, J, K are [m][n][n] row-major. */
static int jk_literal_any(int n, const double* A, const double* alpha, const int* lmn, double tau,
                      int m, const double* D, double* J, double* K)
{
    size_t nn = (size_t)n * n;
    double* Q = (double*)malloc(sizeof(double) * nn);
    if (!Q) return -1;
    schwarz_any(n, A, alpha, lmn, Q);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            for (int i = 0; i < m; ++i) {
                const double* Di = D + (size_t)i * nn;
                double jv = 0.0, kv = 0.0;
                for (int r = 0; r < n; ++r)
                    for (int s = 0; s < n; ++s) {
                        if (keep_quartet(Q[r * n + s], Q[p * n + q], tau))
                            jv += Di[r * n + s] * eri_any(A, alpha, lmn, r, s, p, q);
                        if (keep_quartet(Q[p * n + r], Q[q * n + s], tau))
                            kv += Di[r * n + s] * eri_any(A, alpha, lmn, p, r, q, s);
                    }
                J[(size_t)i * nn + (size_t)p * n + q] = jv;
                K[(size_t)i * nn + (size_t)p * n + q] = kv;
            }
        }
    free(Q);
    return 0;
}

int oracle_jk_literal(int n, const double* A, const double* alpha, double tau,
                      int m, const double* D, double* J, double* K)
{
    return jk_literal_any(n, A, alpha, NULL, tau, m, D, J, K);
}

int oracle_jk_literal_cart(int n, const double* A, const double* alpha, const int* lmn, double tau,
                      int m, const double* D, double* J, double* K)
{
    return jk_literal_any(n, A, alpha, lmn, tau, m, D, J, K);
}

/* The definition at selected entries only: for each t < count, with
 * i = dens[t], p = row[t], q = col[t]:
 *   Jout[t] = sum_{r,s} D_i[r][s] (rs|pq),  Kout[t] = sum_{r,s} D_i[r][s] (pr|qs). */
static int jk_entries_any(int n, const double* A, const double* alpha, const int* lmn, double tau,
                      int m, const double* D, int count, const int* dens,
                      const int* row, const int* col, double* Jout, double* Kout)
{
    size_t nn = (size_t)n * n;
    double* Q = (double*)malloc(sizeof(double) * nn);
    if (!Q) return -1;
    schwarz_any(n, A, alpha, lmn, Q);
    int bad = 0;
    #pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
    for (int t = 0; t < count; ++t) {
        int i = dens[t], p = row[t], q = col[t];
        if (i < 0 || i >= m || p < 0 || p >= n || q < 0 || q >= n) { bad = 1; continue; }
        const double* Di = D + (size_t)i * nn;
        double jv = 0.0, kv = 0.0;
        for (int r = 0; r < n; ++r)
            for (int s = 0; s < n; ++s) {
                if (keep_quartet(Q[r * n + s], Q[p * n + q], tau))
                    jv += Di[r * n + s] * eri_any(A, alpha, lmn, r, s, p, q);
                if (keep_quartet(Q[p * n + r], Q[q * n + s], tau))
                    kv += Di[r * n + s] * eri_any(A, alpha, lmn, p, r, q, s);
            }
        Jout[t] = jv;
        Kout[t] = kv;
    }
    free(Q);
    return bad ? -2 : 0;
}

int oracle_jk_entries(int n, const double* A, const double* alpha, double tau,
                      int m, const double* D, int count, const int* dens,
                      const int* row, const int* col, double* Jout, double* Kout)
{
    return jk_entries_any(n, A, alpha, NULL, tau, m, D, count, dens, row, col, Jout, Kout);
}

int oracle_jk_entries_cart(int n, const double* A, const double* alpha, const int* lmn, double tau,
                      int m, const double* D, int count, const int* dens,
                      const int* row, const int* col, double* Jout, double* Kout)
{
    return jk_entries_any(n, A, alpha, lmn, tau, m, D, count, dens, row, col, Jout, Kout);
}

/* The paper's grouped build (Sec. "Shell-Pair Screening"): one loop, threaded
 * over retained pairs pq (p >= q), inner loop over retained pairs rs with
 * pair index rs <= pq; each unique integral v is read once and applied to all
 * m densities through its 8 permutations
 *   (pq|rs) (qp|rs) (pq|sr) (qp|sr) (rs|pq) (sr|pq) (rs|qp) (sr|qp),
 * each permutation (ab|cd) adding D[c][d] v to J[a][b] and D[b][d] v to K[a][c].
 * A quartet whose permutations coincide is visited once but the 8 updates
 * count it 2, 4 or 8 times; the weight 1/2 per coincidence (p=q, r=s, pq=rs)
 * restores the count.
 * Only outer pairs with pair index in [pair_begin, pair_end) are visited (the
 * full build is [0, N(N+1)/2)); J and K receive the partial sums.
 * Per-thread accumulators are summed in thread order. Returns the number of
 * quartets visited through *n_visited. */
static int jk_canonical_range_any(int n, const double* A, const double* alpha, const int* lmn, double tau,
                              int m, const double* D, double* J, double* K,
                              int64_t pair_begin, int64_t pair_end, int64_t* n_visited)
{
    size_t nn = (size_t)n * n;
    int64_t npair = (int64_t)n * (n + 1) / 2;
    if (pair_begin < 0) pair_begin = 0;
    if (pair_end > npair) pair_end = npair;
    double* Q = (double*)malloc(sizeof(double) * nn);
    int* pp = (int*)malloc(sizeof(int) * (size_t)npair);
    int* pq = (int*)malloc(sizeof(int) * (size_t)npair);
    if (!Q || !pp || !pq) { free(Q); free(pp); free(pq); return -1; }
    schwarz_any(n, A, alpha, lmn, Q);
    double qmax = 0.0;
    for (size_t i = 0; i < nn; ++i) if (Q[i] > qmax) qmax = Q[i];
    /* retained pairs, in pair-index order */
    int64_t nk = 0;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q <= p; ++q)
            if (keep_quartet(Q[p * n + q], qmax, tau)) { pp[nk] = p; pq[nk] = q; ++nk; }
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    size_t per = (size_t)m * nn;
    double* acc = (double*)calloc((size_t)nthr * 2 * per, sizeof(double));
    if (!acc) { free(Q); free(pp); free(pq); return -1; }
    int64_t visited = 0;
    #pragma omp parallel reduction(+ : visited)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* Jt = acc + (size_t)tid * 2 * per;
        double* Kt = Jt + per;
        #pragma omp for schedule(static, 1)
        for (int64_t a = 0; a < nk; ++a) {
            int p = pp[a], q = pq[a];
            int64_t ia = (int64_t)p * (p + 1) / 2 + q;
            if (ia < pair_begin || ia >= pair_end) continue;
            double qa = Q[p * n + q];
            for (int64_t b = 0; b <= a; ++b) {
                int r = pp[b], s = pq[b];
                if (!keep_quartet(qa, Q[r * n + s], tau)) continue;
                double w = 1.0;
                if (p == q) w *= 0.5;
                if (r == s) w *= 0.5;
                if (a == b) w *= 0.5;
                double v = w * eri_any(A, alpha, lmn, p, q, r, s);
                ++visited;
                for (int i = 0; i < m; ++i) {
                    const double* Di = D + (size_t)i * nn;
                    double* Ji = Jt + (size_t)i * nn;
                    double* Ki = Kt + (size_t)i * nn;
                    /* J: permutation (ab|cd) adds D[c][d] v to J[a][b] */
                    Ji[p * n + q] += v * Di[r * n + s];
                    Ji[q * n + p] += v * Di[r * n + s];
                    Ji[p * n + q] += v * Di[s * n + r];
                    Ji[q * n + p] += v * Di[s * n + r];
                    Ji[r * n + s] += v * Di[p * n + q];
                    Ji[s * n + r] += v * Di[p * n + q];
                    Ji[r * n + s] += v * Di[q * n + p];
                    Ji[s * n + r] += v * Di[q * n + p];
                    /* K: permutation (ab|cd) adds D[b][d] v to K[a][c] */
                    Ki[p * n + r] += v * Di[q * n + s]; /* (pq|rs) */
                    Ki[q * n + r] += v * Di[p * n + s]; /* (qp|rs) */
                    Ki[p * n + s] += v * Di[q * n + r]; /* (pq|sr) */
                    Ki[q * n + s] += v * Di[p * n + r]; /* (qp|sr) */
                    Ki[r * n + p] += v * Di[s * n + q]; /* (rs|pq) */
                    Ki[s * n + p] += v * Di[r * n + q]; /* (sr|pq) */
                    Ki[r * n + q] += v * Di[s * n + p]; /* (rs|qp) */
                    Ki[s * n + q] += v * Di[r * n + p]; /* (sr|qp) */
                }
            }
        }
    }
    memset(J, 0, sizeof(double) * per);
    memset(K, 0, sizeof(double) * per);
    for (int t = 0; t < nthr; ++t) {
        const double* Jt = acc + (size_t)t * 2 * per;
        const double* Kt = Jt + per;
        for (size_t x = 0; x < per; ++x) { J[x] += Jt[x]; K[x] += Kt[x]; }
    }
    if (n_visited) *n_visited = visited;
    free(acc); free(Q); free(pp); free(pq);
    return 0;
}

int oracle_jk_canonical_range(int n, const double* A, const double* alpha, double tau,
                              int m, const double* D, double* J, double* K,
                              int64_t pair_begin, int64_t pair_end, int64_t* n_visited)
{
    return jk_canonical_range_any(n, A, alpha, NULL, tau, m, D, J, K, pair_begin, pair_end, n_visited);
}

int oracle_jk_canonical_range_cart(int n, const double* A, const double* alpha, const int* lmn, double tau,
                              int m, const double* D, double* J, double* K,
                              int64_t pair_begin, int64_t pair_end, int64_t* n_visited)
{
    return jk_canonical_range_any(n, A, alpha, lmn, tau, m, D, J, K, pair_begin, pair_end, n_visited);
}

static int jk_canonical_any(int n, const double* A, const double* alpha, const int* lmn, double tau,
                        int m, const double* D, double* J, double* K)
{
    int64_t v;
    return jk_canonical_range_any(n, A, alpha, lmn, tau, m, D, J, K, 0,
                                     (int64_t)n * (n + 1) / 2, &v);
}

int oracle_jk_canonical(int n, const double* A, const double* alpha, double tau,
                        int m, const double* D, double* J, double* K)
{
    return jk_canonical_any(n, A, alpha, NULL, tau, m, D, J, K);
}

int oracle_jk_canonical_cart(int n, const double* A, const double* alpha, const int* lmn, double tau,
                        int m, const double* D, double* J, double* K)
{
    return jk_canonical_any(n, A, alpha, lmn, tau, m, D, J, K);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
