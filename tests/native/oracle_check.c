/* Sanitizer run of the oracle (oracle/esmf_oracle.c, linked in): every
 * public routine on small seeded inputs, s and Cartesian functions, with the
 * literal and the grouped builds compared, so that AddressSanitizer and
 * UndefinedBehaviorSanitizer see each code path once.  Prints the largest
 * literal-versus-grouped difference and returns nonzero when it exceeds
 * 1e-12 or a routine fails. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_boys_f0(double T);
void oracle_boys_fn(int nmax, double T, double* F);
double oracle_eri(const double* A, const double* alpha, int p, int q, int r, int s);
double oracle_eri_cart(const double* A, const double* alpha, const int* lmn, int p, int q, int r, int s);
void oracle_schwarz(int n, const double* A, const double* alpha, double* Q);
void oracle_schwarz_cart(int n, const double* A, const double* alpha, const int* lmn, double* Q);
int oracle_eri_tensor(int n, const double* A, const double* alpha, double tau, double* T);
void oracle_count(int n, const double* A, const double* alpha, double tau, int64_t* np, int64_t* nq);
int oracle_jk_literal(int n, const double* A, const double* alpha, double tau, int m, const double* D,
                      double* J, double* K);
int oracle_jk_literal_cart(int n, const double* A, const double* alpha, const int* lmn, double tau, int m,
                           const double* D, double* J, double* K);
int oracle_jk_entries(int n, const double* A, const double* alpha, double tau, int m, const double* D, int cnt,
                      const int* dens, const int* rows, const int* cols, double* Jo, double* Ko);
int oracle_jk_canonical(int n, const double* A, const double* alpha, double tau, int m, const double* D,
                        double* J, double* K);
int oracle_jk_canonical_cart(int n, const double* A, const double* alpha, const int* lmn, double tau, int m,
                             const double* D, double* J, double* K);

static double urand(uint64_t* s) {
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    enum { N = 11, M = 3 };
    uint64_t seed = 12345;
    double A[3 * N], al[N], D[M * N * N], J1[M * N * N], K1[M * N * N], J2[M * N * N], K2[M * N * N];
    int lmn[3 * N];
    for (int i = 0; i < 3 * N; ++i) A[i] = 4.0 * urand(&seed);
    for (int i = 0; i < N; ++i) {
        al[i] = 0.2 + 2.0 * urand(&seed);
        lmn[3 * i] = lmn[3 * i + 1] = lmn[3 * i + 2] = 0;
        lmn[3 * i + (i % 3)] = i % 3 == 0 ? 0 : 1 + (i % 2);
    }
    for (int i = 0; i < M * N * N; ++i) D[i] = urand(&seed) - 0.5;
    double F[9];
    oracle_boys_fn(8, 0.3, F);
    volatile double sink = oracle_boys_f0(1e-3) + oracle_boys_f0(50.0) + F[8];
    sink += oracle_eri(A, al, 1, 2, 3, 4) + oracle_eri_cart(A, al, lmn, 1, 2, 3, 4);
    double Q[N * N];
    oracle_schwarz(N, A, al, Q);
    oracle_schwarz_cart(N, A, al, lmn, Q);
    double* T = (double*)malloc(sizeof(double) * N * N * N * N);
    if (!T || oracle_eri_tensor(N, A, al, 1e-4, T) != 0) return 3;
    free(T);
    int64_t np_ = 0, nq = 0;
    oracle_count(N, A, al, 1e-4, &np_, &nq);
    double worst = 0.0;
    for (int cart = 0; cart < 2; ++cart) {
        int r1 = cart ? oracle_jk_literal_cart(N, A, al, lmn, 1e-4, M, D, J1, K1)
                      : oracle_jk_literal(N, A, al, 1e-4, M, D, J1, K1);
        int r2 = cart ? oracle_jk_canonical_cart(N, A, al, lmn, 1e-4, M, D, J2, K2)
                      : oracle_jk_canonical(N, A, al, 1e-4, M, D, J2, K2);
        if (r1 || r2) return 4;
        for (int i = 0; i < M * N * N; ++i) {
            worst = fmax(worst, fabs(J1[i] - J2[i]));
            worst = fmax(worst, fabs(K1[i] - K2[i]));
        }
    }
    int dens[4] = {0, 1, 2, 2}, rows[4] = {0, 3, 10, 5}, cols[4] = {0, 7, 1, 5};
    double Jo[4], Ko[4];
    if (oracle_jk_entries(N, A, al, 1e-4, M, D, 4, dens, rows, cols, Jo, Ko) != 0) return 5;
    printf("max |literal - grouped| = %.3e (pairs %lld, quartets %lld)\n", worst, (long long)np_, (long long)nq);
    (void)sink;
    return worst < 1e-12 ? 0 : 6;
}
