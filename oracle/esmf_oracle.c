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

/* Schwarz factors Q[p*n+q] = sqrt((pq|pq)) for all p, q (symmetric). */
void oracle_schwarz(int n, const double* A, const double* alpha, double* Q)
{
    for (int p = 0; p < n; ++p)
        for (int q = 0; q <= p; ++q) {
            double v = sqrt(oracle_eri(A, alpha, p, q, p, q));
            Q[p * n + q] = v;
            Q[q * n + p] = v;
        }
}

/* Screening predicate: the quartet takes part iff Q_pq * Q_rs > tau. */
static int keep_quartet(double qpq, double qrs, double tau) { return qpq * qrs > tau; }

/* Dense masked tensor T[((p*n+q)*n+r)*n+s] = (pq|rs) if kept else 0. Small n. */
int oracle_eri_tensor(int n, const double* A, const double* alpha, double tau, double* T)
{
    double* Q = (double*)malloc(sizeof(double) * (size_t)n * n);
    if (!Q) return -1;
    oracle_schwarz(n, A, alpha, Q);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    size_t idx = (((size_t)p * n + q) * n + r) * n + s;
                    T[idx] = keep_quartet(Q[p * n + q], Q[r * n + s], tau)
                                 ? oracle_eri(A, alpha, p, q, r, s) : 0.0;
                }
    free(Q);
    return 0;
}

/* Number of unique (8-fold) quartets that pass the screen, and number of pairs
 * p >= q with Q_pq * max Q > tau. */
void oracle_count(int n, const double* A, const double* alpha, double tau,
                  int64_t* n_pairs_kept, int64_t* n_quartets_kept)
{
    double* Q = (double*)malloc(sizeof(double) * (size_t)n * n);
    oracle_schwarz(n, A, alpha, Q);
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

/* The definition written out (Eq. J_and_K):
 *   J_i[p][q] = sum_{r,s} D_i[r][s] (rs|pq),  K_i[p][q] = sum_{r,s} D_i[r][s] (pr|qs),
 * over every index, no symmetry used. D, J, K are [m][n][n] row-major. */
int oracle_jk_literal(int n, const double* A, const double* alpha, double tau,
                      int m, const double* D, double* J, double* K)
{
    size_t nn = (size_t)n * n;
    double* Q = (double*)malloc(sizeof(double) * nn);
    if (!Q) return -1;
    oracle_schwarz(n, A, alpha, Q);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            for (int i = 0; i < m; ++i) {
                const double* Di = D + (size_t)i * nn;
                double jv = 0.0, kv = 0.0;
                for (int r = 0; r < n; ++r)
                    for (int s = 0; s < n; ++s) {
                        if (keep_quartet(Q[r * n + s], Q[p * n + q], tau))
                            jv += Di[r * n + s] * oracle_eri(A, alpha, r, s, p, q);
                        if (keep_quartet(Q[p * n + r], Q[q * n + s], tau))
                            kv += Di[r * n + s] * oracle_eri(A, alpha, p, r, q, s);
                    }
                J[(size_t)i * nn + (size_t)p * n + q] = jv;
                K[(size_t)i * nn + (size_t)p * n + q] = kv;
            }
        }
    free(Q);
    return 0;
}

/* The definition at selected entries only: for each t < count, with
 * i = dens[t], p = row[t], q = col[t]:
 *   Jout[t] = sum_{r,s} D_i[r][s] (rs|pq),  Kout[t] = sum_{r,s} D_i[r][s] (pr|qs). */
int oracle_jk_entries(int n, const double* A, const double* alpha, double tau,
                      int m, const double* D, int count, const int* dens,
                      const int* row, const int* col, double* Jout, double* Kout)
{
    size_t nn = (size_t)n * n;
    double* Q = (double*)malloc(sizeof(double) * nn);
    if (!Q) return -1;
    oracle_schwarz(n, A, alpha, Q);
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
                    jv += Di[r * n + s] * oracle_eri(A, alpha, r, s, p, q);
                if (keep_quartet(Q[p * n + r], Q[q * n + s], tau))
                    kv += Di[r * n + s] * oracle_eri(A, alpha, p, r, q, s);
            }
        Jout[t] = jv;
        Kout[t] = kv;
    }
    free(Q);
    return bad ? -2 : 0;
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
int oracle_jk_canonical_range(int n, const double* A, const double* alpha, double tau,
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
    oracle_schwarz(n, A, alpha, Q);
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
                double v = w * oracle_eri(A, alpha, p, q, r, s);
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

int oracle_jk_canonical(int n, const double* A, const double* alpha, double tau,
                        int m, const double* D, double* J, double* K)
{
    int64_t v;
    return oracle_jk_canonical_range(n, A, alpha, tau, m, D, J, K, 0,
                                     (int64_t)n * (n + 1) / 2, &v);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
