/* Drives the C oracle (kfrts.c, hmm.c) through small and edge-case inputs so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer can report
 * any out-of-bounds access, leak or undefined operation.  Exit status 0 when
 * every call returns the expected code. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_kf_rts(int nx, int ny, long T, const double *F, const double *u, const double *Q, const double *H,
                  const double *d, const double *R, const double *m0, const double *P0, const double *y, double *m,
                  double *P, double *ms, double *Ps, double *mp_out, double *Pp_out, double *ll);
int oracle_kf_rts_tv(int nx, int ny, long T, const double *F, const double *u, const double *Q, const double *H,
                     const double *d, const double *R, const double *m0, const double *P0, const double *y,
                     double *m, double *P, double *ms, double *Ps, double *mp_out, double *Pp_out, double *ll);
int oracle_kf_rts_batched(int nx, int ny, int B, const long *offsets, int per_sequence, const double *F,
                          const double *u, const double *Q, const double *H, const double *d, const double *R,
                          const double *m0, const double *P0, const double *y, double *m, double *P, double *ms,
                          double *Ps, double *ll, int threads);
int oracle_hmm(int K, long T, const double *Pi, const double *p0, const double *L, double *alpha, double *gamma,
               double *ll);

static unsigned long long st = 88172645463325252ull;
static double rnd(void) {            /* xorshift64 in [-1, 1) */
    st ^= st << 13; st ^= st >> 7; st ^= st << 17;
    return (double)(st >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}
static double *arr(size_t n) { double *a = (double *)malloc(sizeof(double) * (n ? n : 1)); for (size_t i = 0; i < n; ++i) a[i] = rnd(); return a; }
static void spd(double *A, int n, double diag) {
    for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) A[i * n + j] = (i == j) ? diag : 0.01 * rnd();
    for (int i = 0; i < n; ++i) for (int j = 0; j < i; ++j) A[j * n + i] = A[i * n + j];
}

static int fails = 0;
#define EXPECT(c) do { if (!(c)) { fprintf(stderr, "FAILED %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

static void kf_case(int nx, int ny, long T) {
    double *F = arr(nx * nx), *Q = arr(nx * nx), *H = arr(ny * nx), *R = arr(ny * ny), *m0 = arr(nx), *P0 = arr(nx * nx);
    double *u = arr(nx), *d = arr(ny), *y = arr(T * ny);
    spd(Q, nx, 0.5); spd(R, ny, 1.0); spd(P0, nx, 1.0);
    for (int i = 0; i < nx * nx; ++i) F[i] *= 0.3;
    double *m = arr(T * nx), *P = arr(T * nx * nx), *ms = arr(T * nx), *Ps = arr(T * nx * nx);
    double *mp = arr(T * nx), *Pp = arr(T * nx * nx), *ll = arr(T);
    EXPECT(oracle_kf_rts(nx, ny, T, F, u, Q, H, d, R, m0, P0, y, m, P, ms, Ps, mp, Pp, ll) == 0);
    EXPECT(oracle_kf_rts(nx, ny, T, F, NULL, Q, H, NULL, R, m0, P0, y, m, P, NULL, NULL, NULL, NULL, NULL) == 0);
    /* time-varying: one row of every matrix per step */
    double *Ft = arr(T * nx * nx), *Qt = arr(T * nx * nx), *Ht = arr(T * ny * nx), *Rt = arr(T * ny * ny);
    for (long k = 0; k < T; ++k) {
        memcpy(Ft + k * nx * nx, F, sizeof(double) * nx * nx); memcpy(Qt + k * nx * nx, Q, sizeof(double) * nx * nx);
        memcpy(Ht + k * ny * nx, H, sizeof(double) * ny * nx); memcpy(Rt + k * ny * ny, R, sizeof(double) * ny * ny);
    }
    EXPECT(oracle_kf_rts_tv(nx, ny, T, Ft, NULL, Qt, Ht, NULL, Rt, m0, P0, y, m, P, ms, Ps, NULL, NULL, ll) == 0);
    /* a measurement covariance that is not positive definite */
    for (int i = 0; i < ny * ny; ++i) R[i] = -R[i];
    if (T > 0) EXPECT(oracle_kf_rts(nx, ny, T, F, u, Q, H, d, R, m0, P0, y, m, P, ms, Ps, NULL, NULL, NULL) != 0);
    free(F); free(Q); free(H); free(R); free(m0); free(P0); free(u); free(d); free(y);
    free(m); free(P); free(ms); free(Ps); free(mp); free(Pp); free(ll); free(Ft); free(Qt); free(Ht); free(Rt);
}

static void batched_case(void) {
    const int nx = 3, ny = 2, B = 6;
    long off[7] = {0, 0, 1, 5, 5, 12, 20};          /* empty, single-step and longer sequences */
    double *F = arr(B * nx * nx), *Q = arr(B * nx * nx), *H = arr(B * ny * nx), *R = arr(B * ny * ny);
    double *m0 = arr(B * nx), *P0 = arr(B * nx * nx), *y = arr(20 * ny);
    for (int b = 0; b < B; ++b) { spd(Q + b * nx * nx, nx, 0.5); spd(R + b * ny * ny, ny, 1.0); spd(P0 + b * nx * nx, nx, 1.0); }
    double *m = arr(20 * nx), *P = arr(20 * nx * nx), *ms = arr(20 * nx), *Ps = arr(20 * nx * nx), *ll = arr(20);
    EXPECT(oracle_kf_rts_batched(nx, ny, B, off, 1, F, NULL, Q, H, NULL, R, m0, P0, y, m, P, ms, Ps, ll, 3) == 0);
    EXPECT(oracle_kf_rts_batched(nx, ny, B, off, 0, F, NULL, Q, H, NULL, R, m0, P0, y, m, P, NULL, NULL, NULL, 0) == 0);
    free(F); free(Q); free(H); free(R); free(m0); free(P0); free(y); free(m); free(P); free(ms); free(Ps); free(ll);
}

static void hmm_case(int K, long T, int impossible) {
    double *Pi = arr(K * K), *p0 = arr(K), *L = arr(T * K);
    for (int i = 0; i < K; ++i) {
        double s = 0.0;
        for (int j = 0; j < K; ++j) { Pi[i * K + j] = fabs(Pi[i * K + j]) + ((i + j) % 3 == 0 ? 0.0 : 0.1); s += Pi[i * K + j]; }
        for (int j = 0; j < K; ++j) Pi[i * K + j] /= s;
        p0[i] = 1.0 / K;
    }
    if (impossible && T > 1) for (int j = 0; j < K; ++j) L[1 * K + j] = -INFINITY;
    double *a = arr(T * K), *g = arr(T * K), *ll = arr(T);
    const int r = oracle_hmm(K, T, Pi, p0, L, a, g, ll);
    EXPECT(impossible && T > 1 ? r == 2 : r == 0);
    EXPECT(oracle_hmm(K, T, Pi, p0, L, a, NULL, NULL) == r);
    free(Pi); free(p0); free(L); free(a); free(g); free(ll);
}

int main(void) {
    const int dims[][2] = {{1, 1}, {2, 1}, {4, 2}, {3, 5}, {6, 6}};
    const long Ts[] = {0, 1, 2, 7};
    for (size_t i = 0; i < sizeof dims / sizeof dims[0]; ++i)
        for (size_t t = 0; t < sizeof Ts / sizeof Ts[0]; ++t) kf_case(dims[i][0], dims[i][1], Ts[t]);
    batched_case();
    for (int K = 1; K <= 5; K += 2)
        for (size_t t = 0; t < sizeof Ts / sizeof Ts[0]; ++t) { hmm_case(K, Ts[t], 0); hmm_case(K, Ts[t], 1); }
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle driver: all checks passed\n");
    return 0;
}
