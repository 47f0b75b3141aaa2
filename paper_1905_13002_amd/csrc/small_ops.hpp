// small_ops.hpp -- register-resident scan elements and operators for small state
// dimensions (one element per lane, N = nx <= 4), gfx950.
//
// Filtering element (Lemma 1)  (A, b, C, eta, J): f(x|z) = N(x; A z + b, C),
//                                                  g(z) ∝ N_I(z; eta, J).
// Filtering operator (Lemma 2) with M = I + C_i J_j:
//   A_ij = A_j M^-1 A_i,  b_ij = A_j M^-1 (b_i + C_i eta_j) + b_j,
//   C_ij = A_j M^-1 C_i A_j^T + C_j,
//   eta_ij = A_i^T M^-T (eta_j - J_j b_i) + eta_i,  J_ij = A_i^T M^-T J_j A_i + J_i
//   (I + J_j C_i = M^T because C and J are symmetric, so one factorisation of
//   M serves both halves: A_i^T M^-T = (M^-1 A_i)^T).
// Smoothing element (Lemma 3) (E, g, L): a(x|z) = N(x; E z + g, L).
// Smoothing operator (Lemma 4): E_ij = E_i E_j, g_ij = E_i g_j + g_i,
//                               L_ij = E_i L_j E_i^T + L_i.
//
// Precision policy: R is the storage/product type (double, or float in the
// mixed mode).  The solve with M (LU with partial pivoting), the Cholesky
// factorisation in the smoothing element and the additions that complete a
// covariance run in double.  A product that is symmetric in exact arithmetic
// (X Y X^T, F P F^T, E F P, Y S^-1 Y^T) is formed once per entry of its lower
// triangle; in the FP32 smoothing operators both triangles are formed and
// averaged in double (sym_entry), which halves the rounding that an
// ill-conditioned F P F^T + Q amplifies.
//
// C, J, L and P are kept packed (lower triangle, row-major) in registers.
#pragma once
#include <hip/hip_runtime.h>

namespace pks {

__host__ __device__ constexpr int tri(int n) { return n * (n + 1) / 2; }
__host__ __device__ constexpr int sidx(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

template <int N, typename R> struct FElem { R A[N * N]; R b[N]; R C[tri(N)]; R eta[N]; R J[tri(N)]; };
template <int N, typename R> struct SElem { R E[N * N]; R g[N]; R L[tri(N)]; };
// Prefix whose A (or suffix whose E) is exactly zero: only the moments remain.
template <int N, typename R> struct Moments { R m[N]; R P[tri(N)]; };

// number of R words of each packed record (used for SoA global layouts)
template <int N> struct Words {
    static constexpr int F = N * N + N + tri(N) + N + tri(N);
    static constexpr int S = N * N + N + tri(N);
    static constexpr int M = N + tri(N);
};

// ---------------------------------------------------------------------------
// identities
// ---------------------------------------------------------------------------
template <int N, typename R> __device__ __forceinline__ void set_identity(FElem<N, R>& e) {
#pragma unroll
    for (int i = 0; i < N * N; ++i) e.A[i] = (i % (N + 1) == 0) ? R(1) : R(0);
#pragma unroll
    for (int i = 0; i < N; ++i) { e.b[i] = R(0); e.eta[i] = R(0); }
#pragma unroll
    for (int i = 0; i < tri(N); ++i) { e.C[i] = R(0); e.J[i] = R(0); }
}
template <int N, typename R> __device__ __forceinline__ void set_identity(SElem<N, R>& e) {
#pragma unroll
    for (int i = 0; i < N * N; ++i) e.E[i] = (i % (N + 1) == 0) ? R(1) : R(0);
#pragma unroll
    for (int i = 0; i < N; ++i) e.g[i] = R(0);
#pragma unroll
    for (int i = 0; i < tri(N); ++i) e.L[i] = R(0);
}
template <int N, typename R> __device__ __forceinline__ void set_zero(Moments<N, R>& x) {
#pragma unroll
    for (int i = 0; i < N; ++i) x.m[i] = R(0);
#pragma unroll
    for (int i = 0; i < tri(N); ++i) x.P[i] = R(0);
}

// Reciprocal in double: hardware estimate refined by two Newton steps
// (r <- r + r (1 - x r)), accurate to about one unit in the last place.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Reciprocal square root in double: hardware estimate refined by two Newton
// steps for 1/sqrt(x) (r <- r + r (1/2 - (x/2) r^2)).  A Cholesky pivot needs
// only 1/sqrt(d) (its square root is d times it), so one refined estimate
// replaces a square root followed by a reciprocal.
__device__ __forceinline__ double rsq64(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * r, r, 0.5);
    r = fma(r, e, r);
    e = fma(-h * r, r, 0.5);
    return fma(r, e, r);
}

// ---------------------------------------------------------------------------
// LU solve with partial pivoting, in double:  X <- M^-1 X  for W right-hand
// sides.  a[r][0..N) holds M, a[r][N..N+W) the right-hand sides.  Pivot rows
// are chosen by a running comparison (row k ends up holding the largest
// |a[.][k]|), rows are exchanged with selects so every index stays static;
// the exchange is skipped when no lane of the wave needs it.
// ---------------------------------------------------------------------------
template <int N, int W>
__device__ __forceinline__ void lu_solve_inplace(double (&a)[N][N + W]) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const bool sw = fabs(a[r][k]) > fabs(a[k][k]);
            if (__any(sw)) {
#pragma unroll
                for (int c = k; c < N + W; ++c) {
                    const double t = a[k][c];
                    a[k][c] = sw ? a[r][c] : t;
                    a[r][c] = sw ? t : a[r][c];
                }
            }
        }
        const double inv = rcp64(a[k][k]);
        a[k][k] = inv;
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            const double f = a[r][k] * inv;
#pragma unroll
            for (int c = k + 1; c < N + W; ++c) a[r][c] = fma(-f, a[k][c], a[r][c]);
        }
    }
    // back substitution (diagonal already inverted)
#pragma unroll
    for (int c = N; c < N + W; ++c) {
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            double s = a[i][c];
#pragma unroll
            for (int l = i + 1; l < N; ++l) s = fma(-a[i][l], a[l][c], s);
            a[i][c] = s * a[i][i];
        }
    }
}

// ---------------------------------------------------------------------------
// Lemma 2: full filtering combine  o = i (x) j   (o may alias j or i)
// ---------------------------------------------------------------------------
// With G (packed sequences), a right operand whose A is exactly zero (it starts
// a new sequence) passes its f-part through untouched, so a NaN in an earlier
// sequence cannot reach later ones through 0 * NaN.
template <int N, typename R>
__device__ __forceinline__ bool all_zero(const R (&X)[N * N]) {
    bool z = true;
#pragma unroll
    for (int i = 0; i < N * N; ++i) z = z && (X[i] == R(0));
    return z;
}

template <int N, typename R, bool G = false>
__device__ __forceinline__ void fcombine(const FElem<N, R>& ei, const FElem<N, R>& ej, FElem<N, R>& o) {
    constexpr int W = 2 * N + 1;               // [A_i | b_i + C_i eta_j | C_i]
    double a[N][N + W];
    // M = I + C_i J_j (products in R)
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R s = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) s = fma(ei.C[sidx(r, l)], ej.J[sidx(l, c)], s);
            a[r][c] = double(s) + (r == c ? 1.0 : 0.0);
        }
    R w[N];      // eta_j - J_j b_i
    R JA[N * N]; // J_j A_i
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R v = ei.b[r];
        R t = ej.eta[r];
#pragma unroll
        for (int l = 0; l < N; ++l) {
            v = fma(ei.C[sidx(r, l)], ej.eta[l], v);
            t = fma(-ej.J[sidx(r, l)], ei.b[l], t);
        }
        a[r][N + N] = double(v);
        w[r] = t;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R s = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) s = fma(ej.J[sidx(r, l)], ei.A[l * N + c], s);
            JA[r * N + c] = s;
            a[r][N + c] = double(ei.A[r * N + c]);
            a[r][N + N + 1 + c] = double(ei.C[sidx(r, c)]);
        }
    }
    lu_solve_inplace<N, W>(a);
    // X1 = M^-1 A_i, x2 = M^-1 v, X3 = M^-1 C_i (rounded to R)
    R X1[N * N], x2[N], X3[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        x2[r] = R(a[r][N + N]);
#pragma unroll
        for (int c = 0; c < N; ++c) {
            X1[r * N + c] = R(a[r][N + c]);
            X3[r * N + c] = R(a[r][N + N + 1 + c]);
        }
    }
    FElem<N, R> t;
    // eta_ij = X1^T w + eta_i ; J_ij = sym(X1^T JA) + J_i
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = ei.eta[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(X1[l * N + r], w[l], s);
        t.eta[r] = s;
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R s = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) s = fma(X1[l * N + r], JA[l * N + c], s);
            t.J[sidx(r, c)] = R(double(s) + double(ei.J[sidx(r, c)]));
        }
    // A_ij = A_j X1 ; b_ij = A_j x2 + b_j ; C_ij = sym(A_j X3 A_j^T) + C_j
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = ej.b[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(ej.A[r * N + l], x2[l], s);
        t.b[r] = s;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], X1[l * N + c], q);
            t.A[r * N + c] = q;
        }
    }
    {
        R Y[N * N];   // A_j X3
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) {
                R q = R(0);
#pragma unroll
                for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], X3[l * N + c], q);
                Y[r * N + c] = q;
            }
#pragma unroll
        for (int r = 0; r < N; ++r)   // (A_j X3) A_j^T, lower triangle
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                R q = R(0);
#pragma unroll
                for (int l = 0; l < N; ++l) q = fma(Y[r * N + l], ej.A[c * N + l], q);
                t.C[sidx(r, c)] = R(double(q) + double(ej.C[sidx(r, c)]));
            }
    }
    if (G && all_zero<N, R>(ej.A)) {
#pragma unroll
        for (int i = 0; i < N * N; ++i) t.A[i] = R(0);
#pragma unroll
        for (int i = 0; i < N; ++i) t.b[i] = ej.b[i];
#pragma unroll
        for (int i = 0; i < tri(N); ++i) t.C[i] = ej.C[i];
    }
    o = t;
}

// ---------------------------------------------------------------------------
// Lemma 2 with a left operand whose A is zero (a prefix that starts at a
// sequence's first step): only b and C of the result matter, and they are
// the filtered moments.  x <- x (x) j.
// ---------------------------------------------------------------------------
template <int N, typename R, bool G = false>
__device__ __forceinline__ void fcarry(Moments<N, R>& x, const FElem<N, R>& ej) {
    const bool pass = G && all_zero<N, R>(ej.A);
    constexpr int W = N + 1;                   // [m + P eta_j | P]
    double a[N][N + W];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R v = x.m[r];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R s = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) s = fma(x.P[sidx(r, l)], ej.J[sidx(l, c)], s);
            a[r][c] = double(s) + (r == c ? 1.0 : 0.0);
            v = fma(x.P[sidx(r, c)], ej.eta[c], v);
            a[r][N + 1 + c] = double(x.P[sidx(r, c)]);
        }
        a[r][N] = double(v);
    }
    lu_solve_inplace<N, W>(a);
    R x2[N], X3[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        x2[r] = R(a[r][N]);
#pragma unroll
        for (int c = 0; c < N; ++c) X3[r * N + c] = R(a[r][N + 1 + c]);
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = ej.b[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(ej.A[r * N + l], x2[l], s);
        x.m[r] = s;
    }
    R Y[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], X3[l * N + c], q);
            Y[r * N + c] = q;
        }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(Y[r * N + l], ej.A[c * N + l], q);
            x.P[sidx(r, c)] = R(double(q) + double(ej.C[sidx(r, c)]));
        }
    if (pass) {
#pragma unroll
        for (int i = 0; i < N; ++i) x.m[i] = ej.b[i];
#pragma unroll
        for (int i = 0; i < tri(N); ++i) x.P[i] = ej.C[i];
    }
}

// Entry (r, c) of the symmetric product Y X^T of the smoothing operators.
// FP64: one product per entry of the lower triangle.  FP32: both triangles
// are formed and averaged in double; a smoother with a rank-deficient Q is
// conditioned like F P F^T + Q, which amplifies the rounding of these
// products, and the average halves it.
template <int N, typename R>
__device__ __forceinline__ double sym_entry(const R (&Y)[N * N], const R* X, int r, int c) {
    R q = R(0);
#pragma unroll
    for (int l = 0; l < N; ++l) q = fma(Y[r * N + l], X[c * N + l], q);
    if constexpr (sizeof(R) == sizeof(double)) {
        return double(q);
    } else {
        R qt = R(0);
#pragma unroll
        for (int l = 0; l < N; ++l) qt = fma(Y[c * N + l], X[r * N + l], qt);
        return 0.5 * (double(q) + double(qt));
    }
}

// ---------------------------------------------------------------------------
// Lemma 4: smoothing combine  o = i (x) j
// ---------------------------------------------------------------------------
// With G, a left operand whose E is exactly zero (it ends a sequence) passes
// through untouched.
template <int N, typename R, bool G = false>
__device__ __forceinline__ void scombine(const SElem<N, R>& ei, const SElem<N, R>& ej, SElem<N, R>& o) {
    SElem<N, R> t;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = ei.g[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(ei.E[r * N + l], ej.g[l], s);
        t.g[r] = s;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ei.E[r * N + l], ej.E[l * N + c], q);
            t.E[r * N + c] = q;
        }
    }
    R Y[N * N];   // E_i L_j
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ei.E[r * N + l], ej.L[sidx(l, c)], q);
            Y[r * N + c] = q;
        }
#pragma unroll
    for (int r = 0; r < N; ++r)   // (E_i L_j) E_i^T, lower triangle
#pragma unroll
        for (int c = 0; c <= r; ++c)
            t.L[sidx(r, c)] = R(sym_entry<N, R>(Y, ei.E, r, c) + double(ei.L[sidx(r, c)]));
    if (G && all_zero<N, R>(ei.E)) {
#pragma unroll
        for (int i = 0; i < N * N; ++i) t.E[i] = R(0);
#pragma unroll
        for (int i = 0; i < N; ++i) t.g[i] = ei.g[i];
#pragma unroll
        for (int i = 0; i < tri(N); ++i) t.L[i] = ei.L[i];
    }
    o = t;
}

// Lemma 4 with a right operand whose E is zero (a suffix that ends at a
// sequence's last step): x <- i (x) x, moments only.
template <int N, typename R, bool G = false>
__device__ __forceinline__ void scarry(const SElem<N, R>& ei, Moments<N, R>& x) {
    const bool pass = G && all_zero<N, R>(ei.E);
    R g[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = ei.g[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(ei.E[r * N + l], x.m[l], s);
        g[r] = s;
    }
    R Y[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ei.E[r * N + l], x.P[sidx(l, c)], q);
            Y[r * N + c] = q;
        }
#pragma unroll
    for (int r = 0; r < N; ++r) x.m[r] = pass ? ei.g[r] : g[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c)
            x.P[sidx(r, c)] = pass ? ei.L[sidx(r, c)] : R(sym_entry<N, R>(Y, ei.E, r, c) + double(ei.L[sidx(r, c)]));
}

// ---------------------------------------------------------------------------
// Lemma 3: smoothing element from filtered moments (m, P) of step k < n:
//   E = P F^T (F P F^T + Q)^-1,  g = m - E (F m + u),  L = P - E F P.
// The Cholesky factorisation of F P F^T + Q and its solve run in double.
// Returns false if the factorisation does not exist (the element is NaN).
// ---------------------------------------------------------------------------
template <int N, typename R>
__device__ __forceinline__ bool build_selem(const R* __restrict__ F, const R* __restrict__ Q,
                                            const R* __restrict__ u, const Moments<N, R>& x,
                                            SElem<N, R>& e) {
    R V[N * N];   // F P
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(F[r * N + l], x.P[sidx(l, c)], q);
            V[r * N + c] = q;
        }
    // S = sym(V F^T) + Q in double, lower triangle; then Cholesky S = G G^T
    // (With FP32 products both triangles are formed and averaged in double:
    // with a rank-deficient Q the Cholesky factorisation below amplifies the
    // rounding of F P F^T by cond(F P F^T + Q), and the average halves it.)
    double S[tri(N)];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(V[r * N + l], F[c * N + l], q);
            if constexpr (sizeof(R) == sizeof(double)) {
                S[sidx(r, c)] = double(q) + double(Q[r * N + c]);
            } else {
                R qt = R(0);
#pragma unroll
                for (int l = 0; l < N; ++l) qt = fma(V[c * N + l], F[r * N + l], qt);
                S[sidx(r, c)] = 0.5 * (double(q) + double(qt)) + double(Q[r * N + c]);
            }
        }
    bool ok = true;
    double dinv[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double dj = S[sidx(j, j)];
#pragma unroll
        for (int l = 0; l < j; ++l) dj = fma(-S[sidx(j, l)], S[sidx(j, l)], dj);
        ok = ok && (dj > 0.0);
        dinv[j] = rsq64(dj);
        S[sidx(j, j)] = dj * dinv[j];
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            double v = S[sidx(i, j)];
#pragma unroll
            for (int l = 0; l < j; ++l) v = fma(-S[sidx(i, l)], S[sidx(j, l)], v);
            S[sidx(i, j)] = v * dinv[j];
        }
    }
    // E^T = S^-1 V  (column c of V solved by forward/back substitution)
    R Et[N * N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double z[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double s = double(V[i * N + c]);
#pragma unroll
            for (int l = 0; l < i; ++l) s = fma(-S[sidx(i, l)], z[l], s);
            z[i] = s * dinv[i];
        }
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            double s = z[i];
#pragma unroll
            for (int l = i + 1; l < N; ++l) s = fma(-S[sidx(l, i)], z[l], s);
            z[i] = s * dinv[i];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) Et[i * N + c] = R(z[i]);
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) e.E[r * N + c] = Et[c * N + r];
    // g = m - E (F m + u)
    R p[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = u[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(F[r * N + l], x.m[l], s);
        p[r] = s;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R s = x.m[r];
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(-e.E[r * N + l], p[l], s);
        e.g[r] = s;
    }
    // L = P - E V (lower triangle; both triangles averaged with FP32 products)
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(e.E[r * N + l], V[l * N + c], q);
            if constexpr (sizeof(R) == sizeof(double)) {
                e.L[sidx(r, c)] = R(double(x.P[sidx(r, c)]) - double(q));
            } else {
                R qt = R(0);
#pragma unroll
                for (int l = 0; l < N; ++l) qt = fma(e.E[c * N + l], V[l * N + r], qt);
                e.L[sidx(r, c)] = R(double(x.P[sidx(r, c)]) - 0.5 * (double(q) + double(qt)));
            }
        }
    return ok;
}

}  // namespace pks

namespace pks {

// ---------------------------------------------------------------------------
// Lemma 2 with a right operand that is a single step k > 1 of Lemma 1
// ("fresh"): J_j = F^T H^T S^-1 H F = W G with G = H F (M x N, M = ny < N).
// Then (I + C_i J_j)^-1 = I - Y Sigma^-1 G with Y = C_i G^T and
// Sigma = S + G C_i G^T (symmetric positive definite, M x M), so the solve is
// a Cholesky factorisation of Sigma (double) instead of an N x N LU.  The
// result is the same operator; J_j enters only through W and G.
// `ej` supplies A, b, C, eta of the step (its J is not read); `Gz` is G, or 0
// for a sequence's first step (whose J is 0).  S is read in double.
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void chol_small(double (&S)[M * M], double (&dinv)[M]) {
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = S[j * M + j];
#pragma unroll
        for (int l = 0; l < j; ++l) d = fma(-S[j * M + l], S[j * M + l], d);
        dinv[j] = rsq64(d);
        S[j * M + j] = d * dinv[j];
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double v = S[i * M + j];
#pragma unroll
            for (int l = 0; l < j; ++l) v = fma(-S[i * M + l], S[j * M + l], v);
            S[i * M + j] = v * dinv[j];
        }
    }
}
// x <- (L L^T)^-1 x, L lower (strictly lower part of S), dinv = 1 / diag(L)
template <int M>
__device__ __forceinline__ void chol_solve_vec(const double (&L)[M * M], const double (&dinv)[M], double (&x)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = x[i];
#pragma unroll
        for (int l = 0; l < i; ++l) s = fma(-L[i * M + l], x[l], s);
        x[i] = s * dinv[i];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        double s = x[i];
#pragma unroll
        for (int l = i + 1; l < M; ++l) s = fma(-L[l * M + i], x[l], s);
        x[i] = s * dinv[i];
    }
}

// Sigma = S + G Y (double), factorised in place
template <int N, int M, typename R>
__device__ __forceinline__ void make_sigma(const double* __restrict__ S, const R (&Gz)[M * N], const R (&Y)[N * M],
                                           double (&Sg)[M * M], double (&dinv)[M]) {
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(Gz[r * N + l], Y[l * M + c], q);
            Sg[r * M + c] = double(S[r * M + c]) + double(q);
            Sg[c * M + r] = Sg[r * M + c];
        }
    chol_small<M>(Sg, dinv);
}

template <int N, int M, typename R, bool G>
__device__ __forceinline__ void fcombine_fresh(FElem<N, R>& ei, const FElem<N, R>& ej, const R (&Gz)[M * N],
                                               const R* __restrict__ Wm, const double* __restrict__ S) {
    // Y = C_i G^T   [N x M]
    R Y[N * M];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ei.C[sidx(r, l)], Gz[c * N + l], q);
            Y[r * M + c] = q;
        }
    double Sg[M * M], dinv[M];
    make_sigma<N, M, R>(S, Gz, Y, Sg, dinv);
    // v = b_i + C_i eta_j ; Gv = G v ; Gb = G b_i ; GA = G A_i
    R v[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = ei.b[r];
#pragma unroll
        for (int l = 0; l < N; ++l) q = fma(ei.C[sidx(r, l)], ej.eta[l], q);
        v[r] = q;
    }
    R Gb[M], GA[M * N];
    double t2[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        R q = R(0), qb = R(0);
#pragma unroll
        for (int l = 0; l < N; ++l) {
            q = fma(Gz[r * N + l], v[l], q);
            qb = fma(Gz[r * N + l], ei.b[l], qb);
        }
        t2[r] = double(q);
        Gb[r] = qb;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R a = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) a = fma(Gz[r * N + l], ei.A[l * N + c], a);
            GA[r * N + c] = a;
        }
    }
    chol_solve_vec<M>(Sg, dinv, t2);
    // T1 = Sigma^-1 GA, Zt = Sigma^-1 Y^T (column by column, double)
    R T1[M * N], Zt[M * N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double x[M], z[M];
#pragma unroll
        for (int r = 0; r < M; ++r) {
            x[r] = double(GA[r * N + c]);
            z[r] = double(Y[c * M + r]);
        }
        chol_solve_vec<M>(Sg, dinv, x);
        chol_solve_vec<M>(Sg, dinv, z);
#pragma unroll
        for (int r = 0; r < M; ++r) {
            T1[r * N + c] = R(x[r]);
            Zt[r * N + c] = R(z[r]);
        }
    }
    // X1 = A_i - Y T1 ; x2 = v - Y t2 ; X3 = sym(C_i - Y Zt)
    R X1[N * N], x2[N], X3[tri(N)];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = v[r];
#pragma unroll
        for (int l = 0; l < M; ++l) q = fma(-Y[r * M + l], R(t2[l]), q);
        x2[r] = q;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R a = ei.A[r * N + c];
#pragma unroll
            for (int l = 0; l < M; ++l) a = fma(-Y[r * M + l], T1[l * N + c], a);
            X1[r * N + c] = a;
        }
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R p = R(0);
#pragma unroll
            for (int l = 0; l < M; ++l) p = fma(Y[r * M + l], Zt[l * N + c], p);
            X3[sidx(r, c)] = R(double(ei.C[sidx(r, c)]) - double(p));
        }
    // J_j b_i = W Gb ; J_j A_i = W GA
    R w[N], JA[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = ej.eta[r];
#pragma unroll
        for (int l = 0; l < M; ++l) q = fma(-Wm[r * M + l], Gb[l], q);
        w[r] = q;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R a = R(0);
#pragma unroll
            for (int l = 0; l < M; ++l) a = fma(Wm[r * M + l], GA[l * N + c], a);
            JA[r * N + c] = a;
        }
    }
    FElem<N, R> t;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = ei.eta[r];
#pragma unroll
        for (int l = 0; l < N; ++l) q = fma(X1[l * N + r], w[l], q);
        t.eta[r] = q;
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(X1[l * N + r], JA[l * N + c], q);
            t.J[sidx(r, c)] = R(double(q) + double(ei.J[sidx(r, c)]));
        }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = ej.b[r];
#pragma unroll
        for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], x2[l], q);
        t.b[r] = q;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R a = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) a = fma(ej.A[r * N + l], X1[l * N + c], a);
            t.A[r * N + c] = a;
        }
    }
    {
        R Yj[N * N];   // A_j X3
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int c = 0; c < N; ++c) {
                R q = R(0);
#pragma unroll
                for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], X3[sidx(l, c)], q);
                Yj[r * N + c] = q;
            }
#pragma unroll
        for (int r = 0; r < N; ++r)   // (A_j X3) A_j^T, lower triangle
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                R q = R(0);
#pragma unroll
                for (int l = 0; l < N; ++l) q = fma(Yj[r * N + l], ej.A[c * N + l], q);
                t.C[sidx(r, c)] = R(double(q) + double(ej.C[sidx(r, c)]));
            }
    }
    if (G && all_zero<N, R>(ej.A)) {
#pragma unroll
        for (int i = 0; i < N * N; ++i) t.A[i] = R(0);
#pragma unroll
        for (int i = 0; i < N; ++i) t.b[i] = ej.b[i];
#pragma unroll
        for (int i = 0; i < tri(N); ++i) t.C[i] = ej.C[i];
    }
    ei = t;
}

// x <- x (x) j for a prefix x with A = 0 and a single step j: the Kalman
// update with "measurement" G and noise S, then A_j, b_j, C_j.
template <int N, int M, typename R, bool G>
__device__ __forceinline__ void fcarry_fresh(Moments<N, R>& x, const FElem<N, R>& ej, const R (&Gz)[M * N],
                                             const double* __restrict__ S) {
    const bool pass = G && all_zero<N, R>(ej.A);
    R Y[N * M];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(x.P[sidx(r, l)], Gz[c * N + l], q);
            Y[r * M + c] = q;
        }
    double Sg[M * M], dinv[M];
    make_sigma<N, M, R>(S, Gz, Y, Sg, dinv);
    R v[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = x.m[r];
#pragma unroll
        for (int l = 0; l < N; ++l) q = fma(x.P[sidx(r, l)], ej.eta[l], q);
        v[r] = q;
    }
    double t2[M];
#pragma unroll
    for (int r = 0; r < M; ++r) {
        R q = R(0);
#pragma unroll
        for (int l = 0; l < N; ++l) q = fma(Gz[r * N + l], v[l], q);
        t2[r] = double(q);
    }
    chol_solve_vec<M>(Sg, dinv, t2);
    R Zt[M * N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double z[M];
#pragma unroll
        for (int r = 0; r < M; ++r) z[r] = double(Y[c * M + r]);
        chol_solve_vec<M>(Sg, dinv, z);
#pragma unroll
        for (int r = 0; r < M; ++r) Zt[r * N + c] = R(z[r]);
    }
    R x2[N], X3[tri(N)];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = v[r];
#pragma unroll
        for (int l = 0; l < M; ++l) q = fma(-Y[r * M + l], R(t2[l]), q);
        x2[r] = q;
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R p = R(0);
#pragma unroll
            for (int l = 0; l < M; ++l) p = fma(Y[r * M + l], Zt[l * N + c], p);
            X3[sidx(r, c)] = R(double(x.P[sidx(r, c)]) - double(p));
        }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        R q = ej.b[r];
#pragma unroll
        for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], x2[l], q);
        x.m[r] = pass ? ej.b[r] : q;
    }
    R Yj[N * N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(ej.A[r * N + l], X3[sidx(l, c)], q);
            Yj[r * N + c] = q;
        }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            R q = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) q = fma(Yj[r * N + l], ej.A[c * N + l], q);
            x.P[sidx(r, c)] = pass ? ej.C[sidx(r, c)] : R(double(q) + double(ej.C[sidx(r, c)]));
        }
}

}  // namespace pks
