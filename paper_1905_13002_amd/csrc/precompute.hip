// precompute.hip -- per-model constants of the filtering elements (Lemma 1).
//
// For a time-invariant model every element with k > 1 shares
//   S = H Q H^T + R,  K = Q H^T S^-1,  A = (I - K H) F,  C = (I - K H) Q,
//   J = F^T H^T S^-1 H F,  W = F^T H^T S^-1,
// and b_k, eta_k are affine in y_k (b_k = c + K y_k, eta_k = w + W y_k with
// c = u - K (H u + d), w = -W (H u + d)).  The k = 1 element is one Kalman
// prediction and update from x_0 ~ N(m0, P0):
//   m1 = F m0 + u, P1 = F P0 F^T + Q, S1 = H P1 H^T + R, K1 = P1 H^T S1^-1,
//   b_1 = m1 + K1 (y_1 - H m1 - d), C_1 = P1 - K1 S1 K1^T, A_1 = 0,
//   eta_1 = 0, J_1 = 0.
// One workgroup per model, FP64 throughout, temporaries in workspace scratch.
// Symmetric results are symmetrised as (X + X^T)/2.  A Cholesky factor of S
// or S1 that does not exist marks the model in the numeric flag and fills
// its constants with NaN.
#include <math.h>

#include <algorithm>

#include "pks_internal.h"

namespace pks {

namespace {

constexpr int kThreads = 256;

struct PrecomputeArgs {
    int nx, ny, per_sequence;
    const double *F, *u, *Q, *H, *d, *R, *m0, *P0;
    double* consts64;
    float* consts32;
    int cw;
    double* scratch;
    int sw;
    int* status;
    int* model_fail;
    int mixed;
    int what;   // 1: filter constants, 2: smoother constants (F, Q, u), 3: both,
                // 4: only G, S, e (the one-step predictive density; small models)
    int reset;  // clear the numeric flag first
    int use_lds;  // temporaries and outputs in LDS (small models), copied out at the end
    int tv;       // time-varying model: one row of F, u, Q, H, d, R per step, model index = step
    const int64_t* offsets;   // time-varying, batched: [B+1] packed sequences (else nullptr)
    int B;
};

// Sequence holding step k of packed sequences (offsets[lo] <= k < offsets[lo + 1]).
__device__ __forceinline__ int seq_of_step(const int64_t* off, int B, int64_t k) {
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

// Sequence of step b of a time-varying model (0 for a single sequence).
__device__ __forceinline__ int tv_seq(const PrecomputeArgs& a, int b) {
    return a.offsets ? seq_of_step(a.offsets, a.B, b) : 0;
}

// Rows of the model arrays that model (or step) b reads: its filter constants
// (F, u, Q, H, d, R), its prior (m0, P0) and its smoother constants (F, Q, u).
// A time-varying model's step b predicts with the transition into step b and
// its smoothing element uses the transition out of it (row b + 1; the last
// step of a sequence never uses it); its prior is the shared one, or that of
// its sequence when packed sequences carry one prior each (per_sequence).
struct Rows {
    size_t f, p, s;
};
__device__ __forceinline__ Rows model_rows(const PrecomputeArgs& a, int b, int nmodels) {
    Rows r;
    const size_t ps = a.per_sequence ? 1 : 0;
    if (a.tv) {
        r.f = (size_t)b;
        r.p = a.per_sequence ? (size_t)tv_seq(a, b) : 0;
        r.s = (size_t)(b + 1 < nmodels ? b + 1 : b);
    } else {
        r.f = r.p = r.s = ps * (size_t)b;
    }
    return r;
}

// Before a time-varying precompute: clears the numeric flag (same rule as the
// precompute's own preparation; its workgroups then set the flag directly)
// and writes the offsets {0, T} of the model's one sequence.
__global__ void k_status_prepare(int* status, int reset, int64_t* offsets, int64_t T) {
    if (reset || status[1] != kStatusMagic) {
        status[0] = kStatusOk;
        status[1] = kStatusMagic;
    }
    offsets[0] = 0;
    offsets[1] = T;
}

// Debug fill of workspace memory: every 8-byte word becomes a pattern that is
// a NaN whether it is read as one double or as either of its two floats.
__global__ void k_poison(unsigned long long* p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0xFFF80000FFF80000ull;
}

// Offsets check (pks_check_offsets): result = the smallest index b at which
// offsets break a packing rule (offsets[0] = 0, non-decreasing, at most
// total, offsets[B] = total), else left at its initial 0x7fffffff.
__global__ void k_offsets_init(int* result) { *result = 0x7fffffff; }
__global__ void k_offsets_check(const int64_t* off, int B, int64_t total, int* result) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= B; b += gridDim.x * blockDim.x) {
        const int64_t v = off[b];
        const bool bad = (b == 0 && v != 0) || (b > 0 && v < off[b - 1]) || v > total || (b == B && v != total);
        if (bad) atomicMin(result, b);
    }
}

// out[m x n] = op(A) op(B); A is [m x k] (or [k x m] if ta), B is [k x n] (or [n x k] if tb)
__device__ void bmm(double* out, const double* A, bool ta, const double* B, bool tb, int m, int k, int n,
                    double alpha = 1.0, const double* add = nullptr) {
    for (int idx = threadIdx.x; idx < m * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        double s = 0.0;
        for (int l = 0; l < k; ++l) {
            const double a = ta ? A[l * m + i] : A[i * k + l];
            const double b = tb ? B[j * k + l] : B[l * n + j];
            s = fma(a, b, s);
        }
        out[idx] = (add ? add[idx] : 0.0) + alpha * s;
    }
    __syncthreads();
}

__device__ void bsym(double* X, int n) {
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        if (i > j) {
            const double v = 0.5 * (X[i * n + j] + X[j * n + i]);
            X[i * n + j] = v;
            X[j * n + i] = v;
        }
    }
    __syncthreads();
}

__device__ void bcopy(double* dst, const double* src, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// lower Cholesky factor in place; returns false (block-uniform) on failure
__device__ bool bchol(double* S, int n) {
    __shared__ int fail;
    if (threadIdx.x == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (threadIdx.x == 0) {
            const double dj = S[j * n + j];
            if (!(dj > 0.0)) fail = 1;
            S[j * n + j] = sqrt(dj);
        }
        __syncthreads();
        const double piv = S[j * n + j];
        for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) S[i * n + j] /= piv;
        __syncthreads();
        const int m = n - j - 1;   // trailing block size
        for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
            const int i = j + 1 + idx / m, l = j + 1 + idx % m;
            if (l <= i) S[i * n + l] = fma(-S[i * n + j], S[l * n + j], S[i * n + l]);
        }
        __syncthreads();
    }
    const bool ok = (fail == 0);
    __syncthreads();
    return ok;
}

// X <- (L L^T)^-1 X, X is [n x r]; one column per thread
__device__ void bsolve(const double* Lc, int n, double* X, int r) {
    for (int c = threadIdx.x; c < r; c += blockDim.x) {
        for (int i = 0; i < n; ++i) {
            double s = X[i * r + c];
            for (int l = 0; l < i; ++l) s = fma(-Lc[i * n + l], X[l * r + c], s);
            X[i * r + c] = s / Lc[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = X[i * r + c];
            for (int l = i + 1; l < n; ++l) s = fma(-Lc[l * n + i], X[l * r + c], s);
            X[i * r + c] = s / Lc[i * n + i];
        }
    }
    __syncthreads();
}

__device__ void btranspose(double* dst, const double* src, int rows, int cols) {   // dst[cols x rows]
    for (int idx = threadIdx.x; idx < rows * cols; idx += blockDim.x) {
        const int i = idx / cols, j = idx % cols;
        dst[j * rows + i] = src[idx];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_precompute(PrecomputeArgs a) {
    extern __shared__ double lds[];
    const int b = blockIdx.x;
    if (b == 0 && threadIdx.x == 0 && !a.tv) {
        // status[0] = first failing sequence (kStatusOk = none), status[1] = magic;
        // a workspace that was never prepared (wrong magic) starts clean.
        if (a.reset || a.status[1] != kStatusMagic) {
            a.status[0] = kStatusOk;
            a.status[1] = kStatusMagic;
        }
    }
    const int nx = a.nx, ny = a.ny, n2 = nx * nx, nm = nx * ny, m2 = ny * ny;
    const Rows rw = model_rows(a, b, gridDim.x);
    const double* F = a.F + rw.f * n2;
    const double* Q = a.Q + rw.f * n2;
    const double* H = a.H + rw.f * nm;
    const double* R = a.R + rw.f * m2;
    const double* m0 = a.m0 + rw.p * nx;
    const double* P0 = a.P0 + rw.p * n2;
    const double* u = a.u ? a.u + rw.f * nx : nullptr;
    const double* d = a.d ? a.d + rw.f * ny : nullptr;
    const ConstLayout CL = const_layout(nx, ny);
    double* gout = a.consts64 + (size_t)b * a.cw;
    double* out = a.use_lds ? lds : gout;
    double* sc = a.use_lds ? lds + a.cw : a.scratch + (size_t)b * a.sw;
    double* T1 = sc;          // ny x nx
    double* S = T1 + nm;      // ny x ny
    double* Lc = S + m2;      // ny x ny
    double* Kt = Lc + m2;     // ny x nx
    double* G = Kt + nm;      // ny x nx
    double* Z = G + nm;       // ny x nx
    double* e = Z + nm;       // ny
    double* m1 = e + ny;      // nx
    double* V = m1 + nx;      // nx x nx
    double* P1 = V + n2;      // nx x nx
    double* T2 = P1 + n2;     // ny x nx
    double* S1 = T2 + nm;     // ny x ny
    double* L1 = S1 + m2;     // ny x ny
    double* K1t = L1 + m2;    // ny x nx
    double* e1 = K1t + nm;    // ny
    double* U = e1 + ny;      // nx x ny
    double* uz = U + nm;      // nx   (u or 0)
    double* dz = uz + nx;     // ny   (d or 0)

    for (int i = threadIdx.x; i < nx; i += blockDim.x) uz[i] = u ? u[i] : 0.0;
    for (int i = threadIdx.x; i < ny; i += blockDim.x) dz[i] = d ? d[i] : 0.0;
    __syncthreads();
    bool ok = true;
    if (a.what & 1) {

    // ---- k > 1 elements ----
    bmm(T1, H, false, Q, false, ny, nx, nx);                 // H Q
    bmm(S, T1, false, H, true, ny, nx, ny, 1.0, R);          // H Q H^T + R
    bsym(S, ny);
    bcopy(Lc, S, m2);
    ok = bchol(Lc, ny);
    bcopy(Kt, T1, nm);
    bsolve(Lc, ny, Kt, nx);                                  // K^T = S^-1 H Q
    bmm(G, H, false, F, false, ny, nx, nx);                  // H F
    bcopy(Z, G, nm);
    bsolve(Lc, ny, Z, nx);                                   // S^-1 H F
    bcopy(out + CL.G, G, nm);                                // H F
    bcopy(out + CL.S, S, m2);                                // H Q H^T + R
    btranspose(out + CL.K, Kt, ny, nx);                      // K
    btranspose(out + CL.W, Z, ny, nx);                       // W = (S^-1 H F)^T
    bmm(out + CL.J, G, true, Z, false, nx, ny, nx);          // F^T H^T S^-1 H F
    bsym(out + CL.J, nx);
    bmm(out + CL.A, Kt, true, G, false, nx, ny, nx, -1.0, F);   // F - K H F
    bmm(out + CL.C, Kt, true, T1, false, nx, ny, nx, -1.0, Q);  // Q - K H Q
    bsym(out + CL.C, nx);
    bmm(e, H, false, uz, false, ny, nx, 1, 1.0, dz);          // H u + d
    bcopy(out + CL.e, e, ny);
    bmm(out + CL.c, Kt, true, e, false, nx, ny, 1, -1.0, uz);  // u - K e
    bmm(out + CL.w, Z, true, e, false, nx, ny, 1, -1.0);       // -W e

    // ---- k = 1 element (a time-varying model needs it at its first step only) ----
    if (!a.tv || b == 0 || (a.offsets && a.offsets[tv_seq(a, b)] == b)) {
    bmm(m1, F, false, m0, false, nx, nx, 1, 1.0, uz);        // F m0 + u
    bmm(V, F, false, P0, false, nx, nx, nx);                 // F P0
    bmm(P1, V, false, F, true, nx, nx, nx, 1.0, Q);          // F P0 F^T + Q
    bsym(P1, nx);
    bmm(T2, H, false, P1, false, ny, nx, nx);                // H P1
    bmm(S1, T2, false, H, true, ny, nx, ny, 1.0, R);         // H P1 H^T + R
    bsym(S1, ny);
    bcopy(L1, S1, m2);
    ok = bchol(L1, ny) && ok;
    bcopy(K1t, T2, nm);
    bsolve(L1, ny, K1t, nx);                                 // K1^T = S1^-1 H P1
    btranspose(out + CL.K1, K1t, ny, nx);
    bmm(e1, H, false, m1, false, ny, nx, 1, 1.0, dz);        // H m1 + d
    bmm(out + CL.c1, K1t, true, e1, false, nx, ny, 1, -1.0, m1);   // m1 - K1 e1
    bmm(U, K1t, true, S1, false, nx, ny, ny);                // K1 S1
    bmm(out + CL.C1, U, false, K1t, false, nx, ny, nx, -1.0, P1);  // P1 - K1 S1 K1^T
    bsym(out + CL.C1, nx);
    }
    }

    // ---- smoother constants ----
    if (a.what & 2) {
        bcopy(out + CL.F, a.F + rw.s * n2, n2);
        bcopy(out + CL.Q, a.Q + rw.s * n2, n2);
        for (int i = threadIdx.x; i < nx; i += blockDim.x) out[CL.u + i] = a.u ? a.u[rw.s * nx + i] : 0.0;
        __syncthreads();
    }

    if (!ok) {
        for (int i = threadIdx.x; i < CL.words; i += blockDim.x) out[i] = __builtin_nan("");
        __syncthreads();
    }
    if ((a.what & 1) && threadIdx.x == 0) {
        a.model_fail[b] = ok ? 0 : 1;
        if (a.tv && !ok) atomicMin(a.status, tv_seq(a, b));
    }
    if (a.use_lds) {
        const int lo = (a.what & 1) ? 0 : CL.F;
        const int hi = (a.what & 2) ? CL.words : CL.F;
        for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) gout[i] = out[i];
    }
    if (a.mixed) {
        float* o32 = a.consts32 + (size_t)b * a.cw;
        const int lo = (a.what & 1) ? 0 : CL.F;
        const int hi = (a.what & 2) ? CL.words : CL.F;
        for (int i = lo + threadIdx.x; i < hi; i += blockDim.x) o32[i] = (float)out[i];
    }
}


// ---------------------------------------------------------------------------
// Small models (nx, ny <= 4): one thread per model, every matrix in registers.
// Same formulas and output layout as the cooperative kernel above.
// ---------------------------------------------------------------------------
template <int NX, int NY>
struct SmallPre {
    // C[m x n] = op(A) op(B) with compile-time sizes
    template <int M, int K, int Nn, bool TA, bool TB>
    static __device__ __forceinline__ void mm(double* C, const double* A, const double* B) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < Nn; ++j) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < K; ++l) s = fma(TA ? A[l * M + i] : A[i * K + l], TB ? B[j * K + l] : B[l * Nn + j], s);
                C[i * Nn + j] = s;
            }
    }
    template <int Nn>
    static __device__ __forceinline__ void sym(double* X) {
#pragma unroll
        for (int i = 0; i < Nn; ++i)
#pragma unroll
            for (int j = 0; j < i; ++j) {
                const double v = 0.5 * (X[i * Nn + j] + X[j * Nn + i]);
                X[i * Nn + j] = v;
                X[j * Nn + i] = v;
            }
    }
    // lower Cholesky factor of S in L; returns false if a pivot is not positive
    template <int Nn>
    static __device__ __forceinline__ bool chol(const double* S, double* L) {
        bool ok = true;
#pragma unroll
        for (int j = 0; j < Nn; ++j) {
            double d = S[j * Nn + j];
#pragma unroll
            for (int l = 0; l < j; ++l) d = fma(-L[j * Nn + l], L[j * Nn + l], d);
            ok = ok && (d > 0.0);
            const double r = sqrt(d);
            const double rinv = 1.0 / r;   // one division per pivot; the column is scaled by it
            L[j * Nn + j] = r;
#pragma unroll
            for (int i = j + 1; i < Nn; ++i) {
                double v = S[i * Nn + j];
#pragma unroll
                for (int l = 0; l < j; ++l) v = fma(-L[i * Nn + l], L[j * Nn + l], v);
                L[i * Nn + j] = v * rinv;
            }
#pragma unroll
            for (int i = 0; i < j; ++i) L[i * Nn + j] = 0.0;
        }
        return ok;
    }
    // X[Nn x Rr] <- (L L^T)^-1 X
    template <int Nn, int Rr>
    static __device__ __forceinline__ void solve(const double* L, double* X) {
        double dinv[Nn];   // reciprocals of the diagonal, one division each
#pragma unroll
        for (int i = 0; i < Nn; ++i) dinv[i] = 1.0 / L[i * Nn + i];
#pragma unroll
        for (int c = 0; c < Rr; ++c) {
#pragma unroll
            for (int i = 0; i < Nn; ++i) {
                double s = X[i * Rr + c];
#pragma unroll
                for (int l = 0; l < i; ++l) s = fma(-L[i * Nn + l], X[l * Rr + c], s);
                X[i * Rr + c] = s * dinv[i];
            }
#pragma unroll
            for (int i = Nn - 1; i >= 0; --i) {
                double s = X[i * Rr + c];
#pragma unroll
                for (int l = i + 1; l < Nn; ++l) s = fma(-L[l * Nn + i], X[l * Rr + c], s);
                X[i * Rr + c] = s * dinv[i];
            }
        }
    }
};

// Makes one wave's LDS writes visible to its other lanes.  The fences cover
// LDS only, so the wave does not wait here for its global stores.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Writes the constants of the wave's 64 models field by field: every lane
// puts the n words of one field of its own model into an LDS stage, then the
// wave stores them with consecutive lanes on consecutive words (runs of n
// words per model) instead of one store per word that touches 64 models'
// lines.  In the mixed mode the scans read the float copy, and from the
// double copy only S (the rank-ny solves run in double), so only that field
// is written twice.  A model whose factorisation failed writes NaN.  Every
// lane of the wave must call emit.
template <int MAXN>
struct WaveWriter {
    double* stg;          // LDS [64][MAXN + 1]
    double* d;            // constants of the wave's first model
    float* f;             // their float copy (mixed mode) or nullptr
    int cw;               // words per model
    int nvalid;           // models of this wave that exist
    int s_off;            // offset of S (kept in double in the mixed mode too)
    template <int N>
    __device__ __forceinline__ void emit(int off, const double (&v)[N], bool ok) const {
        static_assert(N <= MAXN, "field larger than the stage");
        const int lane = threadIdx.x & 63;
        const bool dbl = !f || off == s_off;
        if (nvalid <= 8) {        // few models (a shared or small set): each lane stores its own
            if (lane < nvalid) {
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const double x = ok ? v[i] : __builtin_nan("");
                    if (dbl) d[(size_t)lane * cw + off + i] = x;
                    if (f) f[(size_t)lane * cw + off + i] = (float)x;
                }
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) stg[lane * (MAXN + 1) + i] = ok ? v[i] : __builtin_nan("");
        wave_sync_lds();
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const int e = r * 64 + lane, bl = e / N, i = e - bl * N;
            if (bl < nvalid) {
                const double x = stg[bl * (MAXN + 1) + i];
                if (dbl) d[(size_t)bl * cw + off + i] = x;
                if (f) f[(size_t)bl * cw + off + i] = (float)x;
            }
        }
        wave_sync_lds();          // the stage is refilled by the next field
    }
};

template <int NX, int NY>
__global__ __launch_bounds__(64) void k_precompute_small(PrecomputeArgs a, int nmodels) {
    using SP = SmallPre<NX, NY>;
    // Two independent chains per model, in different waves so that they run
    // concurrently: even blocks derive the shared constants of the steps k > 1,
    // odd blocks the first-step element (and copy F, Q, u).  The odd half also
    // factors S = H Q H^T + R, so it alone decides whether the model failed.
    constexpr int n2 = NX * NX, nm = NX * NY, m2 = NY * NY;
    constexpr int MAXN = n2 > nm ? (n2 > m2 ? n2 : m2) : (nm > m2 ? nm : m2);
    __shared__ double stg[64 * (MAXN + 1)];
    const int part = blockIdx.x & 1;
    const int b0 = (blockIdx.x >> 1) * blockDim.x;
    const int b = b0 + threadIdx.x;
    const bool active = b < nmodels;
    if (blockIdx.x == 0 && threadIdx.x == 0 && !a.tv) {
        if (a.reset || a.status[1] != kStatusMagic) {
            a.status[0] = kStatusOk;
            a.status[1] = kStatusMagic;
        }
    }
    // lanes past the last model repeat its arithmetic and write nothing
    const Rows rw = model_rows(a, active ? b : nmodels - 1, nmodels);
    double F[n2], Q[n2], H[nm], R[m2], m0[NX], P0[n2], u[NX], d[NY];
#pragma unroll
    for (int i = 0; i < n2; ++i) {
        F[i] = a.F[rw.f * n2 + i];
        Q[i] = a.Q[rw.f * n2 + i];
        P0[i] = a.P0[rw.p * n2 + i];
    }
#pragma unroll
    for (int i = 0; i < nm; ++i) H[i] = a.H[rw.f * nm + i];
#pragma unroll
    for (int i = 0; i < m2; ++i) R[i] = a.R[rw.f * m2 + i];
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        m0[i] = a.m0[rw.p * NX + i];
        u[i] = a.u ? a.u[rw.f * NX + i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NY; ++i) d[i] = a.d ? a.d[rw.f * NY + i] : 0.0;

    const ConstLayout CL = const_layout(NX, NY);
    const int nvalid = nmodels - b0 < 64 ? nmodels - b0 : 64;
    const WaveWriter<MAXN> out{stg, a.consts64 + (size_t)b0 * a.cw,
                               a.mixed ? a.consts32 + (size_t)b0 * a.cw : nullptr, a.cw, nvalid, CL.S};
    bool ok = true;
    if (a.what == 4 && part == 0) {
        double T1[nm], S[m2], Lc[m2], G[nm], e[NY];
        SP::template mm<NY, NX, NX, false, false>(T1, H, Q);          // H Q
        SP::template mm<NY, NX, NY, false, true>(S, T1, H);           // H Q H^T
#pragma unroll
        for (int i = 0; i < m2; ++i) S[i] += R[i];
        SP::template sym<NY>(S);
        ok = SP::template chol<NY>(S, Lc);
        SP::template mm<NY, NX, NX, false, false>(G, H, F);           // H F
        SP::template mm<NY, NX, 1, false, false>(e, H, u);           // H u + d
#pragma unroll
        for (int i = 0; i < NY; ++i) e[i] += d[i];
        out.emit(CL.G, G, ok);
        out.emit(CL.S, S, ok);
        out.emit(CL.e, e, ok);
    }
    if ((a.what & 1) && part == 0) {
        double T1[nm], S[m2], Lc[m2], Kt[nm], G[nm], Z[nm], X[n2], e[NY], v[NX], col[nm];
        SP::template mm<NY, NX, NX, false, false>(T1, H, Q);          // H Q
        SP::template mm<NY, NX, NY, false, true>(S, T1, H);           // H Q H^T
#pragma unroll
        for (int i = 0; i < m2; ++i) S[i] += R[i];
        SP::template sym<NY>(S);
        ok = SP::template chol<NY>(S, Lc);
#pragma unroll
        for (int i = 0; i < nm; ++i) Kt[i] = T1[i];
        SP::template solve<NY, NX>(Lc, Kt);                           // K^T = S^-1 H Q
        SP::template mm<NY, NX, NX, false, false>(G, H, F);           // H F
        out.emit(CL.G, G, ok);
        out.emit(CL.S, S, ok);
#pragma unroll
        for (int i = 0; i < nm; ++i) Z[i] = G[i];
        SP::template solve<NY, NX>(Lc, Z);                            // S^-1 H F
#pragma unroll
        for (int i = 0; i < NY; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j) col[j * NY + i] = Kt[i * NX + j];
        out.emit(CL.K, col, ok);
#pragma unroll
        for (int i = 0; i < NY; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j) col[j * NY + i] = Z[i * NX + j];
        out.emit(CL.W, col, ok);
        SP::template mm<NX, NY, NX, true, false>(X, G, Z);           // F^T H^T S^-1 H F
        SP::template sym<NX>(X);
        out.emit(CL.J, X, ok);
        SP::template mm<NX, NY, NX, true, false>(X, Kt, G);          // K H F
#pragma unroll
        for (int i = 0; i < n2; ++i) X[i] = F[i] - X[i];
        out.emit(CL.A, X, ok);
        SP::template mm<NX, NY, NX, true, false>(X, Kt, T1);         // K H Q
#pragma unroll
        for (int i = 0; i < n2; ++i) X[i] = Q[i] - X[i];
        SP::template sym<NX>(X);
        out.emit(CL.C, X, ok);
        SP::template mm<NY, NX, 1, false, false>(e, H, u);           // H u + d
#pragma unroll
        for (int i = 0; i < NY; ++i) e[i] += d[i];
        out.emit(CL.e, e, ok);
        SP::template mm<NX, NY, 1, true, false>(v, Kt, e);
#pragma unroll
        for (int i = 0; i < NX; ++i) v[i] = u[i] - v[i];
        out.emit(CL.c, v, ok);
        SP::template mm<NX, NY, 1, true, false>(v, Z, e);
#pragma unroll
        for (int i = 0; i < NX; ++i) v[i] = -v[i];
        out.emit(CL.w, v, ok);
    }
    // a time-varying model needs the first-step element at each sequence start
    // only: step 0 (wave 0) of a single sequence, every step of packed ones
    if ((a.what & 1) && part == 1 && (!a.tv || b0 == 0 || a.offsets)) {
        // k = 1: one prediction from the prior and one update
        double m1[NX], V[n2], P1[n2], T2[nm], S1[m2], L1[m2], K1t[nm], e1[NY], U[nm], X[n2], v[NX], col[nm];
        SP::template mm<NX, NX, 1, false, false>(m1, F, m0);
#pragma unroll
        for (int i = 0; i < NX; ++i) m1[i] += u[i];
        SP::template mm<NX, NX, NX, false, false>(V, F, P0);
        SP::template mm<NX, NX, NX, false, true>(P1, V, F);
#pragma unroll
        for (int i = 0; i < n2; ++i) P1[i] += Q[i];
        SP::template sym<NX>(P1);
        SP::template mm<NY, NX, NX, false, false>(T2, H, P1);
        SP::template mm<NY, NX, NY, false, true>(S1, T2, H);
#pragma unroll
        for (int i = 0; i < m2; ++i) S1[i] += R[i];
        SP::template sym<NY>(S1);
        {
            double T1[nm], S[m2], Lc[m2];
            SP::template mm<NY, NX, NX, false, false>(T1, H, Q);
            SP::template mm<NY, NX, NY, false, true>(S, T1, H);
#pragma unroll
            for (int i = 0; i < m2; ++i) S[i] += R[i];
            SP::template sym<NY>(S);
            ok = SP::template chol<NY>(S, Lc);
        }
        ok = SP::template chol<NY>(S1, L1) && ok;
#pragma unroll
        for (int i = 0; i < nm; ++i) K1t[i] = T2[i];
        SP::template solve<NY, NX>(L1, K1t);
#pragma unroll
        for (int i = 0; i < NY; ++i)
#pragma unroll
            for (int j = 0; j < NX; ++j) col[j * NY + i] = K1t[i * NX + j];
        out.emit(CL.K1, col, ok);
        SP::template mm<NY, NX, 1, false, false>(e1, H, m1);
#pragma unroll
        for (int i = 0; i < NY; ++i) e1[i] += d[i];
        SP::template mm<NX, NY, 1, true, false>(v, K1t, e1);
#pragma unroll
        for (int i = 0; i < NX; ++i) v[i] = m1[i] - v[i];
        out.emit(CL.c1, v, ok);
        SP::template mm<NX, NY, NY, true, false>(U, K1t, S1);        // K1 S1
        SP::template mm<NX, NY, NX, false, false>(X, U, K1t);        // K1 S1 K1^T
#pragma unroll
        for (int i = 0; i < n2; ++i) X[i] = P1[i] - X[i];
        SP::template sym<NX>(X);
        out.emit(CL.C1, X, ok);
    }
    if (active) {
        if ((a.what & 1) && part == 1) a.model_fail[b] = ok ? 0 : 1;
        if (a.tv && !ok) atomicMin(a.status, tv_seq(a, b));   // either half of a failing step
    }
    if ((a.what & 2) && part == 1) {
        double X[n2], v[NX];
#pragma unroll
        for (int i = 0; i < n2; ++i) X[i] = a.F[rw.s * n2 + i];
        out.emit(CL.F, X, true);
#pragma unroll
        for (int i = 0; i < n2; ++i) X[i] = a.Q[rw.s * n2 + i];
        out.emit(CL.Q, X, true);
#pragma unroll
        for (int i = 0; i < NX; ++i) v[i] = a.u ? a.u[rw.s * NX + i] : 0.0;
        out.emit(CL.u, v, true);
    }
}

template <int NX>
bool launch_small_pre_ny(int ny, PrecomputeArgs a, int nmodels, hipStream_t s) {
    const dim3 grid(2 * ((nmodels + 63) / 64)), block(64);    // even / odd blocks: the two halves
    switch (ny) {
        case 1: hipLaunchKernelGGL((k_precompute_small<NX, 1>), grid, block, 0, s, a, nmodels); return true;
        case 2: hipLaunchKernelGGL((k_precompute_small<NX, 2>), grid, block, 0, s, a, nmodels); return true;
        case 3: hipLaunchKernelGGL((k_precompute_small<NX, 3>), grid, block, 0, s, a, nmodels); return true;
        case 4: hipLaunchKernelGGL((k_precompute_small<NX, 4>), grid, block, 0, s, a, nmodels); return true;
        default: return false;
    }
}

bool launch_small_pre(int nx, int ny, PrecomputeArgs a, int nmodels, hipStream_t s) {
    switch (nx) {
        case 1: return launch_small_pre_ny<1>(ny, a, nmodels, s);
        case 2: return launch_small_pre_ny<2>(ny, a, nmodels, s);
        case 3: return launch_small_pre_ny<3>(ny, a, nmodels, s);
        case 4: return launch_small_pre_ny<4>(ny, a, nmodels, s);
        default: return false;
    }
}

}  // namespace

hipError_t launch_precompute(int nx, int ny, int32_t nmodels, const pks_model& model, void* ws,
                             const WsLayout& L, bool mixed, int what, bool reset, hipStream_t s, bool tv,
                             const int64_t* tv_offsets, int32_t B) {
    PrecomputeArgs a;
    a.nx = nx;
    a.ny = ny;
    a.per_sequence = model.per_sequence ? 1 : 0;
    a.F = model.F; a.u = model.u; a.Q = model.Q;
    a.H = model.H; a.d = model.d; a.R = model.R;
    a.m0 = model.m0; a.P0 = model.P0;
    char* base = static_cast<char*>(ws);
    a.consts64 = reinterpret_cast<double*>(base + L.consts64);
    a.consts32 = reinterpret_cast<float*>(base + L.consts32);
    a.cw = const_layout(nx, ny).words;
    a.scratch = reinterpret_cast<double*>(base + L.scratch);
    a.sw = precompute_scratch_words(nx, ny);
    a.status = reinterpret_cast<int*>(base + L.status);
    a.model_fail = reinterpret_cast<int*>(base + L.model_fail);
    a.mixed = mixed ? 1 : 0;
    a.what = what;
    a.reset = reset ? 1 : 0;
    a.tv = tv ? 1 : 0;
    a.offsets = tv ? tv_offsets : nullptr;
    a.B = B;
    if (tv)
        hipLaunchKernelGGL(k_status_prepare, dim3(1), dim3(1), 0, s, a.status, a.reset,
                           reinterpret_cast<int64_t*>(base + L.tv_offsets), (int64_t)nmodels);
    // Small models keep every temporary in LDS and run as one wave (barriers
    // are then nearly free); large ones use 256 threads and workspace scratch.
    const size_t lds_bytes = sizeof(double) * (size_t)(a.cw + a.sw);
    a.use_lds = lds_bytes <= 48 * 1024 ? 1 : 0;
    const int threads = (a.use_lds && nx <= 16 && ny <= 16) ? 64 : kThreads;
    // time-invariant models with 5 <= nx <= 16: the register-tile kernel (one wave per model)
    // (the likelihood's mode 4 takes the filter constants, which include G, S, e)
    if (!tv && a.what >= 1 && a.what <= 4 && w16_applies(nx, ny, true)) {
        prof_begin("k_w16_precompute", s);
        launch_w16_precompute(nx, ny, nmodels, model, a.consts64, a.mixed ? a.consts32 : nullptr, a.status,
                              a.model_fail, a.what == 4 ? 1 : a.what, reset, s);
        prof_end(s);
        return hipGetLastError();
    }
    prof_begin("k_precompute", s);
    if (!(nx <= 4 && ny <= 4 && launch_small_pre(nx, ny, a, nmodels, s))) {
        if (a.what == 4) a.what = 1;     // the cooperative kernel derives G, S, e with the rest
        hipLaunchKernelGGL(k_precompute, dim3(nmodels), dim3(threads), a.use_lds ? lds_bytes : 0, s, a);
    }
    prof_end(s);
    return hipGetLastError();
}

hipError_t launch_poison(void* p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 8;
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>(1024, (n + 255) / 256);
    hipLaunchKernelGGL(k_poison, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<unsigned long long*>(p), n);
    return hipGetLastError();
}

hipError_t launch_offsets_check(const int64_t* offsets, int B, int64_t total, int* result, hipStream_t s) {
    hipLaunchKernelGGL(k_offsets_init, dim3(1), dim3(1), 0, s, result);
    const int blocks = (int)std::min<int64_t>(1024, ((int64_t)B + 1 + 255) / 256);
    hipLaunchKernelGGL(k_offsets_check, dim3(blocks), dim3(256), 0, s, offsets, B, total, result);
    return hipGetLastError();
}

}  // namespace pks
