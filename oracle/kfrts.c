/*
 * Sequential FP64 Kalman filter + Rauch-Tung-Striebel smoother: the oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path calls, links or loads
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Sarkka & Garcia-Fernandez, "Temporal Parallelization of
 * Bayesian Smoothers"):
 *   model   x_k = F x_{k-1} + u + q_{k-1},  q ~ N(0,Q)
 *           y_k = H x_k + d + r_k,          r ~ N(0,R),   x_0 ~ N(m0,P0)
 *           (Section IV, linear/Gaussian state space model, time-invariant case)
 *   filter  the classic predict/update recursion (Section II-A, the Bayesian
 *           filter equations, in their Kalman form); the first data point is
 *           y_1, the prior sits on x_0 (Lemma 1, the k = 1 block, is exactly one
 *           such prediction followed by one update).
 *   smoother the classic RTS backward pass (Section II-A, the backward smoothing
 *           equation, in its Gaussian form) with gain G_k = P_k F^T (P^-_{k+1})^{-1}
 *           (the same gain as E_k in Lemma 3) and the last smoothed moment equal
 *           to the last filtered one (Lemma 3, k = n).
 *   loglik  the factors of the marginal likelihood, p(y_1:n) = prod_k
 *           p(y_k | y_1:k-1) (Section III-C), each the Gaussian density of y_k
 *           under the filter's one-step prediction: N(y_k; H m^-_k + d, S_k)
 *           with the innovation covariance S_k = H P^-_k H^T + R, evaluated
 *           as -(ny log(2 pi) + log det S_k + e_k^T S_k^{-1} e_k) / 2 from the
 *           Cholesky factor of S_k (log det = 2 sum log L_ii, and the
 *           quadratic form is |L^{-1} e_k|^2).
 *
 * The parallel method reaches this result exactly in exact arithmetic
 * (Theorems 1 and 2; Section V says the parallel and sequential solutions
 * coincide), so this plain recursion is the definition the GPU path is
 * compared against.
 *
 * Conventions: all matrices row-major, C index k-1 holds time step k.
 * Covariance outputs are symmetrised as (X + X^T)/2 after every step.
 * Inverses of symmetric positive definite matrices go through Cholesky;
 * a non-positive pivot returns the failing step (1-based) as a positive code.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ---- small dense helpers (row-major) ---------------------------------- */

/* C[m x n] = A[m x k] * B[k x n]  (optionally transposed operands) */
static void mm(int m, int k, int n, const double *A, int ta, const double *B, int tb,
               double *C)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) {
                double a = ta ? A[l * m + i] : A[i * k + l];
                double b = tb ? B[j * k + l] : B[l * n + j];
                s += a * b;
            }
            C[i * n + j] = s;
        }
}

static void symmetrise(int n, double *X)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) {
            double v = 0.5 * (X[i * n + j] + X[j * n + i]);
            X[i * n + j] = v;
            X[j * n + i] = v;
        }
}

/* In-place lower Cholesky factor of an SPD matrix; returns 0 on success. */
static int cholesky(int n, double *S)
{
    for (int j = 0; j < n; ++j) {
        double d = S[j * n + j];
        for (int l = 0; l < j; ++l) d -= S[j * n + l] * S[j * n + l];
        if (!(d > 0.0)) return 1;
        d = sqrt(d);
        S[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = S[i * n + j];
            for (int l = 0; l < j; ++l) v -= S[i * n + l] * S[j * n + l];
            S[i * n + j] = v / d;
        }
        for (int i = 0; i < j; ++i) S[i * n + j] = 0.0;
    }
    return 0;
}

/* log N(e; 0, L L^T) for a lower Cholesky factor L [n x n] and a residual e [n]. */
static double gauss_logpdf(int n, const double *L, const double *e, double *z)
{
    double logdet = 0.0, quad = 0.0;
    for (int i = 0; i < n; ++i) {
        double v = e[i];
        for (int l = 0; l < i; ++l) v -= L[i * n + l] * z[l];
        z[i] = v / L[i * n + i];
        quad += z[i] * z[i];
        logdet += 2.0 * log(L[i * n + i]);
    }
    return -0.5 * ((double)n * log(2.0 * acos(-1.0)) + logdet + quad);
}

/* Solve (L L^T) X = B in place, L lower [n x n], B [n x r]. */
static void chol_solve(int n, int r, const double *L, double *B)
{
    for (int c = 0; c < r; ++c) {
        for (int i = 0; i < n; ++i) {
            double v = B[i * r + c];
            for (int l = 0; l < i; ++l) v -= L[i * n + l] * B[l * r + c];
            B[i * r + c] = v / L[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double v = B[i * r + c];
            for (int l = i + 1; l < n; ++l) v -= L[l * n + i] * B[l * r + c];
            B[i * r + c] = v / L[i * n + i];
        }
    }
}

/* ---- the recursion ------------------------------------------------------ */

/*
 * One sequence.  u, d may be NULL (zero).  mp/Pp (predicted moments) may be
 * NULL, in which case an internal buffer is used.  ms/Ps may be NULL to run
 * the filter only.  ll (may be NULL) receives log p(y_k | y_1:k-1) per step.
 * Returns 0, or k (1-based step) whose Cholesky failed
 * (innovation covariance S_k in the filter, P^-_{k+1} in the smoother, the
 * latter reported as T + k).
 */
/*
 * The recursion with per-step model rows: step k (0-based) predicts with
 * F + k*sF, u + k*su, Q + k*sQ and updates with H + k*sH, d + k*sd, R + k*sR;
 * the RTS step at k uses the transition out of it, row k+1.  All strides 0:
 * one time-invariant model.
 */
static int kf_rts_rows(int nx, int ny, long T,
                       const double *F, long sF, const double *u, long su, const double *Q, long sQ,
                       const double *H, long sH, const double *d, long sd, const double *R, long sR,
                       const double *m0, const double *P0,
                       const double *y,
                       double *m, double *P, double *ms, double *Ps,
                       double *mp_out, double *Pp_out, double *ll)
{
    if (T <= 0) return 0;
    const int n2 = nx * nx;
    double *mp = mp_out, *Pp = Pp_out;
    double *own = NULL;
    if (!mp || !Pp) {
        own = (double *)malloc(sizeof(double) * (size_t)T * (size_t)(nx + n2));
        if (!own) return -1;
        mp = own;
        Pp = own + (size_t)T * nx;
    }
    double *work = (double *)malloc(sizeof(double) * (size_t)(6 * n2 + 6 * nx * ny + 4 * ny * ny + 4 * nx + 5 * ny + 16));
    if (!work) { free(own); return -1; }
    double *FP = work;              /* nx*nx */
    double *HP = FP + n2;           /* ny*nx */
    double *S = HP + nx * ny;       /* ny*ny */
    double *Lc = S + ny * ny;       /* ny*ny */
    double *Kt = Lc + ny * ny;      /* ny*nx : K^T */
    double *KS = Kt + nx * ny;      /* nx*ny */
    double *KSK = KS + nx * ny;     /* nx*nx */
    double *e = KSK + n2;           /* ny */
    double *G = e + ny;             /* nx*nx */
    double *D = G + n2;             /* nx*nx */
    double *GD = D + n2;            /* nx*nx */
    double *dm = GD + n2;           /* nx */
    double *z = dm + nx;            /* ny */
    int status = 0;

    const double *mprev = m0, *Pprev = P0;
    const double *F0 = F, *u0 = u, *Q0 = Q, *H0 = H, *d0 = d, *R0 = R;
    for (long k = 0; k < T; ++k) {
        F = F0 + k * sF; Q = Q0 + k * sQ; H = H0 + k * sH; R = R0 + k * sR;
        u = u0 ? u0 + k * su : NULL;
        d = d0 ? d0 + k * sd : NULL;
        double *mk = m + (size_t)k * nx, *Pk = P + (size_t)k * n2;
        double *mpk = mp + (size_t)k * nx, *Ppk = Pp + (size_t)k * n2;
        /* prediction: m^- = F m + u, P^- = F P F^T + Q */
        for (int i = 0; i < nx; ++i) {
            double s = u ? u[i] : 0.0;
            for (int l = 0; l < nx; ++l) s += F[i * nx + l] * mprev[l];
            mpk[i] = s;
        }
        mm(nx, nx, nx, F, 0, Pprev, 0, FP);
        mm(nx, nx, nx, FP, 0, F, 1, Ppk);
        for (int i = 0; i < n2; ++i) Ppk[i] += Q[i];
        symmetrise(nx, Ppk);
        /* update: S = H P^- H^T + R, K = P^- H^T S^{-1} */
        mm(ny, nx, nx, H, 0, Ppk, 0, HP);
        mm(ny, nx, ny, HP, 0, H, 1, S);
        for (int i = 0; i < ny * ny; ++i) S[i] += R[i];
        symmetrise(ny, S);
        memcpy(Lc, S, sizeof(double) * ny * ny);
        if (cholesky(ny, Lc)) { status = (int)(k + 1); goto done; }
        memcpy(Kt, HP, sizeof(double) * ny * nx); /* S K^T = H P^- */
        chol_solve(ny, nx, Lc, Kt);
        for (int i = 0; i < ny; ++i) {
            double s = y[(size_t)k * ny + i] - (d ? d[i] : 0.0);
            for (int l = 0; l < nx; ++l) s -= H[i * nx + l] * mpk[l];
            e[i] = s;
        }
        if (ll) ll[k] = gauss_logpdf(ny, Lc, e, z);
        for (int i = 0; i < nx; ++i) {
            double s = mpk[i];
            for (int l = 0; l < ny; ++l) s += Kt[l * nx + i] * e[l];
            mk[i] = s;
        }
        /* P = P^- - K S K^T */
        mm(nx, ny, ny, Kt, 1, S, 0, KS);
        mm(nx, ny, nx, KS, 0, Kt, 0, KSK);
        for (int i = 0; i < n2; ++i) Pk[i] = Ppk[i] - KSK[i];
        symmetrise(nx, Pk);
        mprev = mk;
        Pprev = Pk;
    }

    if (ms && Ps) {
        size_t last = (size_t)(T - 1);
        memcpy(ms + last * nx, m + last * nx, sizeof(double) * nx);
        memcpy(Ps + last * n2, P + last * n2, sizeof(double) * n2);
        for (long k = T - 2; k >= 0; --k) {
            const double *mk = m + (size_t)k * nx, *Pk = P + (size_t)k * n2;
            const double *mpn = mp + (size_t)(k + 1) * nx, *Ppn = Pp + (size_t)(k + 1) * n2;
            const double *msn = ms + (size_t)(k + 1) * nx, *Psn = Ps + (size_t)(k + 1) * n2;
            double *msk = ms + (size_t)k * nx, *Psk = Ps + (size_t)k * n2;
            F = F0 + (k + 1) * sF;            /* the transition out of step k */
            /* G = P_k F^T (P^-_{k+1})^{-1}:  P^-_{k+1} G^T = F P_k */
            memcpy(D, Ppn, sizeof(double) * n2);
            if (cholesky(nx, D)) { status = (int)(T + k + 1); goto done; }
            mm(nx, nx, nx, F, 0, Pk, 0, GD); /* F P_k */
            chol_solve(nx, nx, D, GD);       /* GD = G^T */
            for (int i = 0; i < nx; ++i)
                for (int j = 0; j < nx; ++j) G[i * nx + j] = GD[j * nx + i];
            for (int i = 0; i < nx; ++i) dm[i] = msn[i] - mpn[i];
            for (int i = 0; i < nx; ++i) {
                double s = mk[i];
                for (int l = 0; l < nx; ++l) s += G[i * nx + l] * dm[l];
                msk[i] = s;
            }
            for (int i = 0; i < n2; ++i) D[i] = Psn[i] - Ppn[i];
            mm(nx, nx, nx, G, 0, D, 0, GD);
            mm(nx, nx, nx, GD, 0, G, 1, KSK);
            for (int i = 0; i < n2; ++i) Psk[i] = Pk[i] + KSK[i];
            symmetrise(nx, Psk);
        }
    }
done:
    free(work);
    free(own);
    return status;
}

int oracle_kf_rts(int nx, int ny, long T,
                  const double *F, const double *u, const double *Q,
                  const double *H, const double *d, const double *R,
                  const double *m0, const double *P0,
                  const double *y,
                  double *m, double *P, double *ms, double *Ps,
                  double *mp_out, double *Pp_out, double *ll)
{
    return kf_rts_rows(nx, ny, T, F, 0, u, 0, Q, 0, H, 0, d, 0, R, 0, m0, P0, y, m, P, ms, Ps,
                       mp_out, Pp_out, ll);
}

/*
 * Time-varying model (Section IV in its general form): F, u, Q, H, d, R hold
 * one row per step; row k-1 holds F_{k-1}, u_{k-1}, Q_{k-1} (the transition
 * into step k) and H_k, d_k, R_k.  Same outputs and return codes.
 */
int oracle_kf_rts_tv(int nx, int ny, long T,
                     const double *F, const double *u, const double *Q,
                     const double *H, const double *d, const double *R,
                     const double *m0, const double *P0,
                     const double *y,
                     double *m, double *P, double *ms, double *Ps,
                     double *mp_out, double *Pp_out, double *ll)
{
    const long n2 = (long)nx * nx;
    return kf_rts_rows(nx, ny, T, F, n2, u, nx, Q, n2, H, (long)ny * nx, d, ny, R, (long)ny * ny, m0, P0,
                       y, m, P, ms, Ps, mp_out, Pp_out, ll);
}

/* ---- many independent sequences ----------------------------------------- */

typedef struct {
    int nx, ny, B;
    const long *offsets;
    const double *F, *u, *Q, *H, *d, *R, *m0, *P0;
    long sF, su, sQ, sH, sd, sR, sm0, sP0; /* per-sequence model strides (0 = shared) */
    const double *y;
    double *m, *P, *ms, *Ps, *ll;
    int next;
    pthread_mutex_t lock;
    int status;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *J = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int b = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (b >= J->B) break;
        long s = J->offsets[b], T = J->offsets[b + 1] - s;
        int nx = J->nx, ny = J->ny;
        int st = oracle_kf_rts(nx, ny, T,
                               J->F + b * J->sF, J->u ? J->u + b * J->su : NULL, J->Q + b * J->sQ,
                               J->H + b * J->sH, J->d ? J->d + b * J->sd : NULL, J->R + b * J->sR,
                               J->m0 + b * J->sm0, J->P0 + b * J->sP0,
                               J->y + s * ny, J->m + s * nx, J->P + s * nx * nx,
                               J->ms ? J->ms + s * nx : NULL, J->Ps ? J->Ps + s * nx * nx : NULL,
                               NULL, NULL, J->ll ? J->ll + s : NULL);
        if (st) {
            pthread_mutex_lock(&J->lock);
            if (!J->status) J->status = b + 1;
            pthread_mutex_unlock(&J->lock);
        }
    }
    return NULL;
}

/*
 * B sequences packed back to back (sequence b occupies steps offsets[b] ..
 * offsets[b+1]-1 of y/m/P/ms/Ps/ll).  per_sequence != 0 means model arrays hold
 * B stacked models; otherwise one model is shared.  Runs on `threads` host
 * threads (sequences are independent).  Returns 0 or 1 + first failing b.
 */
int oracle_kf_rts_batched(int nx, int ny, int B, const long *offsets, int per_sequence,
                          const double *F, const double *u, const double *Q,
                          const double *H, const double *d, const double *R,
                          const double *m0, const double *P0,
                          const double *y, double *m, double *P, double *ms, double *Ps,
                          double *ll, int threads)
{
    batch_job J;
    J.nx = nx; J.ny = ny; J.B = B; J.offsets = offsets;
    J.F = F; J.u = u; J.Q = Q; J.H = H; J.d = d; J.R = R; J.m0 = m0; J.P0 = P0;
    long ps = per_sequence ? 1 : 0;
    J.sF = ps * nx * nx; J.su = ps * nx; J.sQ = ps * nx * nx; J.sH = ps * ny * nx;
    J.sd = ps * ny; J.sR = ps * ny * ny; J.sm0 = ps * nx; J.sP0 = ps * nx * nx;
    J.y = y; J.m = m; J.P = P; J.ms = ms; J.Ps = Ps; J.ll = ll;
    J.next = 0; J.status = 0;
    pthread_mutex_init(&J.lock, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < threads; ++t)
        if (pthread_create(&th[started], NULL, batch_worker, &J) == 0) ++started;
    batch_worker(&J);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return J.status;
}
