/*
 * Sequential forward-backward for a discrete-state hidden Markov model: the
 * oracle of the discrete-state filter and smoother.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path calls, links or loads
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or constant with the HIP library.
 *
 * Model (the state-space model of Section II with a finite state space, whose
 * integrals become sums over the counting measure, as the paper's concluding
 * section notes):
 *     x_0 ~ p0,   p(x_k = j | x_{k-1} = i) = Pi[i][j],
 *     p(y_k | x_k = j) = exp(L[k-1][j])      (k = 1..T, row k-1 holds step k)
 * Only the log-likelihoods L enter, so the emission model is the caller's.
 *
 * Filter (the Bayesian filtering equations of Section II-A: prediction by the
 * Chapman-Kolmogorov sum, then Bayes' rule), normalised at every step:
 *     pred_k[j]  = sum_i alpha_{k-1}[i] Pi[i][j]              (alpha_0 = p0)
 *     u_k[j]     = pred_k[j] exp(L[k-1][j] - M_k),  M_k = max_j L[k-1][j]
 *     alpha_k    = u_k / sum_j u_k[j]                         p(x_k | y_1:k)
 *     ll_k       = log sum_j u_k[j] + M_k                     log p(y_k | y_1:k-1)
 * Smoother (the backward smoothing equation of Section II-A):
 *     gamma_T    = alpha_T
 *     gamma_k[i] = alpha_k[i] sum_j Pi[i][j] gamma_{k+1}[j] / pred_{k+1}[j]
 * where a term with pred_{k+1}[j] = 0 is left out (then gamma_{k+1}[j] = 0 too:
 * a state the filter cannot reach is never smoothed into).
 *
 * Returns 0, or the first step (1-based) whose normaliser sum_j u_k[j] is not
 * positive (the measurements are impossible under the model).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

int oracle_hmm(int K, long T, const double *Pi, const double *p0, const double *L,
               double *alpha, double *gamma, double *ll)
{
    double *pred = (double *)malloc(sizeof(double) * (size_t)K * (size_t)(T > 0 ? T : 1));
    if (!pred) return -1;
    int bad = 0;
    for (long k = 0; k < T; ++k) {
        const double *prev = k == 0 ? p0 : alpha + (k - 1) * K;
        double *pk = pred + k * K;
        for (int j = 0; j < K; ++j) {
            double s = 0.0;
            for (int i = 0; i < K; ++i) s += prev[i] * Pi[i * K + j];
            pk[j] = s;
        }
        const double *Lk = L + k * K;
        double M = Lk[0];
        for (int j = 1; j < K; ++j)
            if (Lk[j] > M) M = Lk[j];
        double *ak = alpha + k * K;
        double c = 0.0;
        for (int j = 0; j < K; ++j) {
            ak[j] = pk[j] * exp(Lk[j] - M);
            c += ak[j];
        }
        if (!(c > 0.0) && !bad) bad = (int)(k + 1);
        for (int j = 0; j < K; ++j) ak[j] /= c;
        if (ll) ll[k] = log(c) + M;
    }
    if (gamma && T > 0) {
        memcpy(gamma + (T - 1) * K, alpha + (T - 1) * K, sizeof(double) * K);
        for (long k = T - 2; k >= 0; --k) {
            const double *ak = alpha + k * K, *gn = gamma + (k + 1) * K, *pn = pred + (k + 1) * K;
            double *gk = gamma + k * K;
            for (int i = 0; i < K; ++i) {
                double s = 0.0;
                for (int j = 0; j < K; ++j)
                    if (pn[j] > 0.0) s += Pi[i * K + j] * gn[j] / pn[j];
                gk[i] = ak[i] * s;
            }
        }
    }
    free(pred);
    return bad;
}
