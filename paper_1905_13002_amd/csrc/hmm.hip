// hmm.hip -- discrete-state hidden Markov model: the parallel filter and
// smoother of Sections II-III with a finite state space (integrals become sums
// over the states; the concluding section of the paper notes the framework
// holds there).
//
// Model: x_0 ~ p0, p(x_k = j | x_{k-1} = i) = Pi[i][j], p(y_k | x_k = j) =
// exp(L[k-1][j]) (the caller's emission log-likelihoods).
//
// Filtering (Theorem 1, Definition 1).  The element of step k is the pair
// f_k[z][x] = p(x_k = x | y_k, x_{k-1} = z), g_k[z] = p(y_k | x_{k-1} = z).
// Written as one matrix Psi_k = diag(g_k) f_k, Psi_k[z][x] = Pi[z][x]
// exp(L[k-1][x]) (step 1: p0^T Pi diag(exp L[0]) in every row), Definition 1's
// operator is exactly the matrix product: (Psi_i Psi_j)[z][x] =
// g_i[z] (sum_y f_i[z][y] g_j[y]) f_ij[z][x] = g_ij[z] f_ij[z][x].  A matrix is
// stored row-normalised with a log-scale per row, (A, c): Psi = diag(e^c) A,
// rows of A summing to one (A = f, c = log g).  A row whose weight is zero
// (the data are impossible from that state) is kept as zeros with c = -inf.
// The prefix from step 1 has identical rows: the filtered marginal
// p(x_k | y_1:k) and c = log p(y_1:k).
//
// Smoothing (Theorem 2, Definition 2).  The element of step k < T is
// a_k(x | z) = p(x_k = x | y_1:k, x_{k+1} = z) = alpha_k[x] Pi[x][z] / pred_{k+1}[z]
// with pred_{k+1} = alpha_k^T Pi, and a_T(x | z) = alpha_T[x].  As matrices
// E[z][x] = a(x | z), the operator is E(a_i (x) a_j) = E(a_j) E(a_i); a
// suffix a_k (x) ... (x) a_e is V = E_e ... E_k, built from the right end of a
// block as V <- V diag(1/pred_{k+1}) Pi^T diag(alpha_k).  A state z that the
// filter cannot reach (pred_{k+1}[z] = 0) has no defined row; its column of
// diag(1/pred) is taken as zero (such a row never carries smoothing weight).
//
// Scan: the time axis is cut into blocks of l steps (Section III-C's block
// elements).  Rows of a block's running product evolve independently
// (row z of V Pi only reads row z of V), so wave w of a block's workgroup owns
// rows 16 w .. 16 w + 15 and runs its products on the matrix cores
// (v_mfma_f64_16x16x4f64) with no synchronisation between waves:
//   k_hmm_filter_reduce / k_hmm_smoother_reduce  one workgroup per block:
//       the block element (filter: left to right; smoother: right to left);
//   k_hmm_scan_level   one Hillis-Steele level over the block elements
//       (ceil(log2 nblk) launches, ping-pong buffers), full matrices;
//   k_hmm_filter_down / k_hmm_smoother_down  one wave per block: the
//       incoming prefix (suffix) of a block is a single row, so the block's
//       steps are re-run as the vector recursion alpha_k ∝ (alpha_{k-1}^T Pi)
//       ∘ exp(L[k-1]) (resp. gamma_k = alpha_k ∘ Pi (gamma_{k+1} / pred_{k+1})),
//       exactly Definitions 1 and 2 with a rank-one left (right) operand.
// States are padded to KP = 16 ceil(K / 16) with zero rows and columns.
// Everything is FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pks_internal.h"

namespace pks {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct HmmArgs {
    int K;                 // states
    int64_t T;             // steps
    int64_t l;             // steps per block
    int64_t nblk;          // blocks
    const double* Pi;      // [K][K]
    const double* p0;      // [K]
    const double* L;       // [T][K] log-likelihoods
    double* alpha;         // [T][K]
    double* logp;          // [T] log p(y_1:k) or nullptr
    double* gamma;         // [T][K]
    double* aggA;          // [nblk][KP][KP] block elements (filter: A; smoother: V)
    double* aggC;          // [nblk][KP] row log-scales (filter)
    double* aggA2;         // ping-pong partner
    double* aggC2;
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the 16 lanes that share lane / 16 (one row of a 16 x 16 tile)
__device__ __forceinline__ double sum16(double v) {
    v += __shfl_xor(v, 1, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 8, 16);
    return v;
}
__device__ __forceinline__ double max64(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ double sum64(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// exp(L[k][x] - M_k) for the lane's state x = lane (0 for padded states) and
// M_k = max_x L[k][x]
__device__ __forceinline__ double scaled_lik(const double* __restrict__ Lk, int K, int lane, double& M) {
    const double v = lane < K ? Lk[lane] : -HUGE_VAL;
    M = max64(v);
    return lane < K ? exp(v - M) : 0.0;
}

// ---------------------------------------------------------------------------
// Strip products on the matrix cores.  A 16 x KP strip X (rows of the wave)
// times a KP x KP matrix Y: lane l supplies X(l % 16, 4 s + l / 16) and
// Y(4 s + l / 16, 16 t + l % 16) and receives D(4 v + l / 16, 16 t + l % 16)
// in register v of tile t.  X comes from the wave's LDS stage (row stride KP
// + 1 doubles), Y from registers (Yf[s][t]).
// ---------------------------------------------------------------------------
template <int KP>
__device__ __forceinline__ void strip_times(const double* __restrict__ Xs, const double (&Yf)[KP / 4][KP / 16],
                                            f64x4 (&D)[KP / 16], int li, int lk) {
    constexpr int NT = KP / 16, NS = KP / 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) D[t] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double xa = Xs[li * (KP + 1) + 4 * s + lk];
#pragma unroll
        for (int t = 0; t < NT; ++t) D[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, Yf[s][t], D[t], 0, 0, 0);
    }
}

// write the strip held in D layout into the stage (rows 4 v + lk, columns 16 t + li)
template <int KP>
__device__ __forceinline__ void stage_strip(double* __restrict__ Xs, const f64x4 (&D)[KP / 16], int li, int lk) {
#pragma unroll
    for (int t = 0; t < KP / 16; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xs[(4 * v + lk) * (KP + 1) + 16 * t + li] = D[t][v];
}

// Y fragments of Pi (trans = false) or Pi^T (trans = true), zero outside K x K
template <int KP>
__device__ __forceinline__ void load_pi_frags(const double* __restrict__ Pi, int K, bool trans,
                                              double (&Yf)[KP / 4][KP / 16], int li, int lk) {
#pragma unroll
    for (int s = 0; s < KP / 4; ++s)
#pragma unroll
        for (int t = 0; t < KP / 16; ++t) {
            const int r = 4 * s + lk, c = 16 * t + li;
            const int i = trans ? c : r, j = trans ? r : c;
            Yf[s][t] = (r < K && c < K) ? Pi[i * K + j] : 0.0;
        }
}

// ---------------------------------------------------------------------------
// Filter reduce: the block element a_s (x) ... (x) a_e, left to right, starting
// from the identity (A = I, c = 0).  One step: A <- A Pi diag(exp(L_k - M_k)),
// rows renormalised, c += M_k + log(row sum); at the sequence's first step the
// rows of A are first replaced by p0 (a_1 does not depend on x_0).
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(KP / 16 * 64) void k_hmm_filter_reduce(HmmArgs a) {
    constexpr int NT = KP / 16;
    __shared__ double stage[NT][16 * (KP + 1)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int64_t s = (int64_t)blockIdx.x * a.l;
    const int64_t e = min(s + a.l, a.T);
    const int K = a.K;
    double* Xs = stage[w];
    double Yf[KP / 4][NT];
    load_pi_frags<KP>(a.Pi, K, false, Yf, li, lk);
    f64x4 D[NT];
    double c[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        c[v] = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) D[t][v] = (16 * w + 4 * v + lk == 16 * t + li) ? 1.0 : 0.0;
    }
    for (int64_t k = s; k < e; ++k) {
        if (k == 0) {
            const double* p0 = a.p0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double pv = (16 * t + li < K) ? p0[16 * t + li] : 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) D[t][v] = (16 * w + 4 * v + lk < K) ? pv : 0.0;
            }
        }
        stage_strip<KP>(Xs, D, li, lk);
        wave_sync_lds();
        strip_times<KP>(Xs, Yf, D, li, lk);
        double M;
        const double lh = scaled_lik(a.L + k * K, K, lane, M);
        double rs[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double lt = __shfl(lh, 16 * t + li, 64);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                D[t][v] *= lt;
                rs[v] += D[t][v];
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double r = sum16(rs[v]);
            const double inv = r > 0.0 ? 1.0 / r : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) D[t][v] *= inv;
            c[v] += M + log(r);
        }
        wave_sync_lds();                     // the stage is rewritten next step
    }
    double* A = a.aggA + (size_t)blockIdx.x * KP * KP;
    double* C = a.aggC + (size_t)blockIdx.x * KP;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(16 * w + 4 * v + lk) * KP + 16 * t + li] = D[t][v];
    if (li == 0)
#pragma unroll
        for (int v = 0; v < 4; ++v) C[16 * w + 4 * v + lk] = c[v];
}

// ---------------------------------------------------------------------------
// Smoother reduce: the block element a_s (x) ... (x) a_e from the right end,
// V = I, then for k = e .. s: V <- V diag(1/pred_{k+1}) Pi^T diag(alpha_k)
// (k < T - 1), or V <- rowsum(V) alpha_T^T at the sequence's last step.
// pred_{k+1} = alpha_k^T Pi is formed by every wave (lane y: state y).
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(KP / 16 * 64) void k_hmm_smoother_reduce(HmmArgs a) {
    constexpr int NT = KP / 16;
    __shared__ double stage[NT][16 * (KP + 1)];
    __shared__ double pi_col[NT][KP];                 // per wave: alpha_k, broadcast
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int64_t s = (int64_t)blockIdx.x * a.l;
    const int64_t e = min(s + a.l, a.T);
    const int K = a.K;
    double* Xs = stage[w];
    double* av = pi_col[w];
    double Yf[KP / 4][NT];
    load_pi_frags<KP>(a.Pi, K, true, Yf, li, lk);
    // column `lane` of Pi, for pred = alpha^T Pi
    double pc[KP];
#pragma unroll
    for (int x = 0; x < KP; ++x) pc[x] = (x < K && lane < K) ? a.Pi[x * K + lane] : 0.0;
    f64x4 D[NT];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < NT; ++t) D[t][v] = (16 * w + 4 * v + lk == 16 * t + li) ? 1.0 : 0.0;
    for (int64_t k = e - 1; k >= s; --k) {
        const double ak = lane < K ? a.alpha[k * K + lane] : 0.0;
        if (k == a.T - 1) {
            // V <- rowsum(V) alpha_T^T
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double r = 0.0;
#pragma unroll
                for (int t = 0; t < NT; ++t) r += D[t][v];
                r = sum16(r);
#pragma unroll
                for (int t = 0; t < NT; ++t) D[t][v] = r * __shfl(ak, 16 * t + li, 64);
            }
            continue;
        }
        if (lane < KP) av[lane] = ak;
        wave_sync_lds();
        double pred = 0.0;
#pragma unroll
        for (int x = 0; x < KP; ++x) pred = fma(av[x], pc[x], pred);
        const double ip = pred > 0.0 ? 1.0 / pred : 0.0;
        // W = V diag(1/pred): column 16 t + li of the lane's registers
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double it = __shfl(ip, 16 * t + li, 64);
#pragma unroll
            for (int v = 0; v < 4; ++v) D[t][v] *= it;
        }
        stage_strip<KP>(Xs, D, li, lk);
        wave_sync_lds();
        strip_times<KP>(Xs, Yf, D, li, lk);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const double at = __shfl(ak, 16 * t + li, 64);
#pragma unroll
            for (int v = 0; v < 4; ++v) D[t][v] *= at;
        }
        wave_sync_lds();
    }
    double* V = a.aggA + (size_t)blockIdx.x * KP * KP;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) V[(16 * w + 4 * v + lk) * KP + 16 * t + li] = D[t][v];
}

// ---------------------------------------------------------------------------
// One Hillis-Steele level at distance d over the block elements.
//   filter   (prefix): out[b] = in[b - d] (x) in[b] for b >= d, else in[b]:
//            X = A_left diag(exp(c_right - cmax)), B = X A_right, rows
//            renormalised, c = c_left + cmax + log(row sum);
//   smoother (suffix): out[b] = in[b] (x) in[b + d] for b + d < nblk:
//            V = V_right V_left (Definition 2 in matrix form).
// The right operand is read as Y fragments straight from memory.
// ---------------------------------------------------------------------------
template <int KP, bool FILTER>
__global__ __launch_bounds__(KP / 16 * 64) void k_hmm_scan_level(const double* __restrict__ inA,
                                                                 const double* __restrict__ inC, double* outA,
                                                                 double* outC, int64_t nblk, int64_t d) {
    constexpr int NT = KP / 16;
    __shared__ double stage[NT][16 * (KP + 1)];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
    const int64_t b = blockIdx.x;
    const size_t mat = (size_t)KP * KP;
    double* oA = outA + b * mat;
    const int64_t partner = FILTER ? b - d : b + d;
    const bool active = FILTER ? (b >= d) : (b + d < nblk);
    if (!active) {
        for (int i = threadIdx.x; i < KP * KP; i += blockDim.x) oA[i] = inA[b * mat + i];
        if (FILTER)
            for (int i = threadIdx.x; i < KP; i += blockDim.x) outC[b * KP + i] = inC[b * KP + i];
        return;
    }
    // operand roles: rows come from X (the strip), Y is the full right factor
    const double* X = FILTER ? inA + partner * mat : inA + partner * mat;   // filter: left = b - d; smoother: V_right = b + d
    const double* Y = inA + b * mat;                                         // filter: right = b; smoother: V_left = b
    double* Xs = stage[w];
    double cmax = 0.0, scale_y = 1.0;
    if (FILTER) {
        const double cy = lane < KP ? inC[b * KP + lane] : -HUGE_VAL;
        cmax = max64(cy);
        if (!(cmax > -HUGE_VAL)) cmax = 0.0;                 // every row of the right factor is zero
        scale_y = lane < KP ? exp(cy - cmax) : 0.0;          // weight of column `lane` of X
    }
    for (int i = lane; i < 16 * KP; i += 64) {
        const int r = i / KP, col = i - r * KP;
        double v = X[(size_t)(16 * w + r) * KP + col];
        if (FILTER) v *= __shfl(scale_y, col, 64);
        Xs[r * (KP + 1) + col] = v;
    }
    double Yf[KP / 4][NT];
#pragma unroll
    for (int s = 0; s < KP / 4; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t) Yf[s][t] = Y[(size_t)(4 * s + lk) * KP + 16 * t + li];
    wave_sync_lds();
    f64x4 D[NT];
    strip_times<KP>(Xs, Yf, D, li, lk);
    if (FILTER) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double r = 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) r += D[t][v];
            r = sum16(r);
            const double inv = r > 0.0 ? 1.0 / r : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) D[t][v] *= inv;
            if (li == 0) {
                const int row = 16 * w + 4 * v + lk;
                outC[b * KP + row] = inC[partner * KP + row] + cmax + log(r);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) oA[(size_t)(16 * w + 4 * v + lk) * KP + 16 * t + li] = D[t][v];
}

// ---------------------------------------------------------------------------
// Down-sweeps: one wave per block, lane x = state x.
// ---------------------------------------------------------------------------
template <int KP>
__global__ __launch_bounds__(64) void k_hmm_filter_down(HmmArgs a, const double* __restrict__ preA,
                                                        const double* __restrict__ preC) {
    __shared__ double av[KP];
    const int lane = threadIdx.x;
    const int K = a.K;
    const int64_t b = blockIdx.x;
    const int64_t s = b * a.l, e = min(s + a.l, a.T);
    double pc[KP];                                   // column `lane` of Pi
#pragma unroll
    for (int x = 0; x < KP; ++x) pc[x] = (x < K && lane < K) ? a.Pi[x * K + lane] : 0.0;
    // incoming prefix: the prior at the sequence start, else row 0 of the
    // inclusive prefix of the previous block (its rows are all the same)
    double al, lp;
    if (b == 0) {
        al = lane < K ? a.p0[lane] : 0.0;
        lp = 0.0;
    } else {
        al = lane < K ? preA[(size_t)(b - 1) * KP * KP + lane] : 0.0;
        lp = preC[(b - 1) * KP];
    }
    for (int64_t k = s; k < e; ++k) {
        if (lane < KP) av[lane] = al;
        wave_sync_lds();
        double pred = 0.0;
#pragma unroll
        for (int x = 0; x < KP; ++x) pred = fma(av[x], pc[x], pred);
        double M;
        const double lh = scaled_lik(a.L + k * K, K, lane, M);
        const double u = pred * lh;
        const double cs = sum64(u);
        al = u / cs;
        lp += M + log(cs);
        if (lane < K) a.alpha[k * K + lane] = al;
        if (a.logp && lane == 0) a.logp[k] = lp;
        wave_sync_lds();
    }
}

template <int KP>
__global__ __launch_bounds__(64) void k_hmm_smoother_down(HmmArgs a, const double* __restrict__ sufA) {
    __shared__ double pr[KP][KP + 1];                // Pi (row stride padded: lanes read their own rows)
    __shared__ double wv[KP];
    __shared__ double av[KP];
    const int lane = threadIdx.x;
    const int K = a.K;
    const int64_t b = blockIdx.x;
    const int64_t s = b * a.l, e = min(s + a.l, a.T);
    for (int i = lane; i < KP * KP; i += 64) {
        const int r = i / KP, c = i - r * KP;
        pr[r][c] = (r < K && c < K) ? a.Pi[r * K + c] : 0.0;
    }
    double pc[KP];                                   // column `lane` of Pi
#pragma unroll
    for (int x = 0; x < KP; ++x) pc[x] = (x < K && lane < K) ? a.Pi[x * K + lane] : 0.0;
    // incoming suffix: row 0 of the inclusive suffix of the next block (the
    // smoothed marginal of step e), or nothing for the last block
    double g = 0.0;
    if (b + 1 < a.nblk) g = lane < K ? sufA[(size_t)(b + 1) * KP * KP + lane] : 0.0;
    wave_sync_lds();
    for (int64_t k = e - 1; k >= s; --k) {
        const double ak = lane < K ? a.alpha[k * K + lane] : 0.0;
        if (k == a.T - 1) {
            g = ak;
        } else {
            if (lane < KP) av[lane] = ak;
            wave_sync_lds();
            double pred = 0.0;
#pragma unroll
            for (int x = 0; x < KP; ++x) pred = fma(av[x], pc[x], pred);
            if (lane < KP) wv[lane] = pred > 0.0 ? g / pred : 0.0;
            wave_sync_lds();
            double acc = 0.0;
            if (lane < KP)
#pragma unroll 8
                for (int y = 0; y < KP; ++y) acc = fma(pr[lane][y], wv[y], acc);
            g = ak * acc;
        }
        if (lane < K) a.gamma[k * K + lane] = g;
        wave_sync_lds();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <int KP>
hipError_t hmm_run(HmmArgs a, int passes, hipStream_t st) {
    constexpr int NTH = KP / 16 * 64;
    const unsigned nb = (unsigned)a.nblk;
    if (passes & 1) {
        prof_begin("k_hmm_filter_reduce", st);
        hipLaunchKernelGGL(k_hmm_filter_reduce<KP>, dim3(nb), dim3(NTH), 0, st, a);
        prof_end(st);
        double *iA = a.aggA, *iC = a.aggC, *oA = a.aggA2, *oC = a.aggC2;
        for (int64_t d = 1; d < a.nblk; d <<= 1) {
            prof_begin("k_hmm_scan_level", st);
            hipLaunchKernelGGL((k_hmm_scan_level<KP, true>), dim3(nb), dim3(NTH), 0, st, iA, iC, oA, oC, a.nblk, d);
            prof_end(st);
            std::swap(iA, oA);
            std::swap(iC, oC);
        }
        prof_begin("k_hmm_filter_down", st);
        hipLaunchKernelGGL(k_hmm_filter_down<KP>, dim3(nb), dim3(64), 0, st, a, iA, iC);
        prof_end(st);
    }
    if (passes & 2) {
        prof_begin("k_hmm_smoother_reduce", st);
        hipLaunchKernelGGL(k_hmm_smoother_reduce<KP>, dim3(nb), dim3(NTH), 0, st, a);
        prof_end(st);
        double *iA = a.aggA, *oA = a.aggA2;
        for (int64_t d = 1; d < a.nblk; d <<= 1) {
            prof_begin("k_hmm_scan_level", st);
            hipLaunchKernelGGL((k_hmm_scan_level<KP, false>), dim3(nb), dim3(NTH), 0, st, iA, nullptr, oA, nullptr,
                               a.nblk, d);
            prof_end(st);
            std::swap(iA, oA);
        }
        prof_begin("k_hmm_smoother_down", st);
        hipLaunchKernelGGL(k_hmm_smoother_down<KP>, dim3(nb), dim3(64), 0, st, a, iA);
        prof_end(st);
    }
    return hipGetLastError();
}

}  // namespace

int hmm_padded_states(int K) { return (K + 15) / 16 * 16; }

// Steps per block: enough blocks that every SIMD holds about two waves of the
// reduce kernels (KP / 16 waves per block), at least 4 steps per block.
int64_t hmm_block_len(int K, int64_t T) {
    const int strips = hmm_padded_states(K) / 16;
    const int64_t target_blocks = std::max<int64_t>(1, 2048 / strips);
    int64_t l = (T + target_blocks - 1) / target_blocks;
    return std::max<int64_t>(4, l);
}

size_t hmm_ws_bytes(int K, int64_t T) {
    const int KP = hmm_padded_states(K);
    const int64_t nblk = T > 0 ? (T + hmm_block_len(K, T) - 1) / hmm_block_len(K, T) : 0;
    const size_t per = sizeof(double) * ((size_t)KP * KP + KP);
    return 2 * per * (size_t)nblk + 256;
}

hipError_t launch_hmm(int K, int64_t T, const double* Pi, const double* p0, const double* L, double* alpha,
                      double* logp, double* gamma, void* ws, int passes, hipStream_t st) {
    HmmArgs a{};
    const int KP = hmm_padded_states(K);
    a.K = K;
    a.T = T;
    a.l = hmm_block_len(K, T);
    a.nblk = (T + a.l - 1) / a.l;
    a.Pi = Pi;
    a.p0 = p0;
    a.L = L;
    a.alpha = alpha;
    a.logp = logp;
    a.gamma = gamma;
    char* base = static_cast<char*>(ws);
    const size_t mats = sizeof(double) * (size_t)KP * KP * a.nblk, vecs = sizeof(double) * (size_t)KP * a.nblk;
    a.aggA = reinterpret_cast<double*>(base);
    a.aggA2 = reinterpret_cast<double*>(base + mats);
    a.aggC = reinterpret_cast<double*>(base + 2 * mats);
    a.aggC2 = reinterpret_cast<double*>(base + 2 * mats + vecs);
    switch (KP) {
        case 16: return hmm_run<16>(a, passes, st);
        case 32: return hmm_run<32>(a, passes, st);
        case 48: return hmm_run<48>(a, passes, st);
        case 64: return hmm_run<64>(a, passes, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace pks
