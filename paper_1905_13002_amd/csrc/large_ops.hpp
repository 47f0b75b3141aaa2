// large_ops.hpp -- workgroup-cooperative matrix operations for the scan of
// large state dimensions (5 <= nx <= 64): one workgroup (256 threads) owns
// one scan element at a time; matrices live in an arena that is LDS when it
// fits and a per-workgroup workspace slot otherwise (generic addressing).
//
// Precision policy (as for small states): R is the storage/product type; the
// LU factorisation with partial pivoting of I + C_i J_j and its solves, the
// Cholesky factorisations and every covariance symmetrisation run in double.
#pragma once
#include <hip/hip_runtime.h>

namespace pks {
namespace large {

constexpr int kThreads = 256;

__device__ __forceinline__ double rcp64l(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// C[m x n] = alpha * op(A) op(B) (+ D), row-major with leading dimensions.
// op(A) = A [m x k] or A^T (A stored [k x m]); same for B.  Each thread
// computes a 4 x 4 block of C.  C may alias D but not A or B.
template <typename TA, typename TB, typename TC, typename TD>
__device__ void gemm(TC* C, int ldc, const TA* A, int lda, bool ta, const TB* B, int ldb, bool tb, int m, int n,
                     int k, double alpha = 1.0, const TD* D = nullptr, int ldd = 0) {
    const int bm = (m + 3) >> 2, bn = (n + 3) >> 2;
    for (int blk = threadIdx.x; blk < bm * bn; blk += blockDim.x) {
        const int i0 = (blk / bn) << 2, j0 = (blk % bn) << 2;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int l = 0; l < k; ++l) {
            double av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int i = i0 + a;
                av[a] = i < m ? double(ta ? A[l * lda + i] : A[i * lda + l]) : 0.0;
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = j0 + b;
                bv[b] = j < n ? double(tb ? B[j * ldb + l] : B[l * ldb + j]) : 0.0;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = i0 + a, j = j0 + b;
                if (i < m && j < n) {
                    double v = alpha * acc[a][b];
                    if (D) v += double(D[i * ldd + j]);
                    C[i * ldc + j] = TC(v);
                }
            }
    }
    __syncthreads();
}

// Products of the storage type: for R = float the sums run in float (the
// mixed mode keeps products in FP32), for R = double in double.
template <typename R>
__device__ void gemmR(R* C, int ldc, const R* A, int lda, bool ta, const R* B, int ldb, bool tb, int m, int n, int k,
                      R alpha = R(1), const R* D = nullptr, int ldd = 0) {
    const int bm = (m + 3) >> 2, bn = (n + 3) >> 2;
    for (int blk = threadIdx.x; blk < bm * bn; blk += blockDim.x) {
        const int i0 = (blk / bn) << 2, j0 = (blk % bn) << 2;
        R acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = R(0);
        for (int l = 0; l < k; ++l) {
            R av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int i = i0 + a;
                av[a] = i < m ? (ta ? A[l * lda + i] : A[i * lda + l]) : R(0);
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = j0 + b;
                bv[b] = j < n ? (tb ? B[j * ldb + l] : B[l * ldb + j]) : R(0);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = i0 + a, j = j0 + b;
                if (i < m && j < n) {
                    R v = alpha * acc[a][b];
                    if (D) v += D[i * ldd + j];
                    C[i * ldc + j] = v;
                }
            }
    }
    __syncthreads();
}

// out = (X + X^T)/2 + D (symmetrisation in double); out may alias D, not X
template <typename R>
__device__ void sym_add(R* out, const R* X, const R* D, int n) {
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        out[idx] = R(0.5 * (double(X[i * n + j]) + double(X[j * n + i])) + (D ? double(D[idx]) : 0.0));
    }
    __syncthreads();
}

template <typename T, typename U>
__device__ void copy(T* dst, const U* src, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = T(src[i]);
    __syncthreads();
}

template <typename T>
__device__ void fill(T* dst, T v, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = v;
    __syncthreads();
}

// y[m] = op(A) x (+ d), A [m x k] (or [k x m] if ta)
template <typename R>
__device__ void gemv(R* y, const R* A, int lda, bool ta, const R* x, int m, int k, const R* d = nullptr,
                     R alpha = R(1)) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        R s = R(0);
        for (int l = 0; l < k; ++l) s = fma(ta ? A[l * lda + i] : A[i * lda + l], x[l], s);
        y[i] = alpha * s + (d ? d[i] : R(0));
    }
    __syncthreads();
}

// In-place LU solve with partial pivoting (double): a is [n x (n + w)],
// row stride lda; on return columns n .. n+w-1 hold M^-1 times the right-hand
// sides.  `red` is a small double scratch (>= 2 * 64 entries).
__device__ void lu_solve(double* a, int lda, int n, int w, int* piv_sh) {
    const int tid = threadIdx.x;
    const int width = n + w;
    for (int k = 0; k < n; ++k) {
        // pivot: argmax |a[r][k]|, r >= k, by wave 0 (n <= 64)
        if (tid < 64) {
            const int r = k + tid;
            double v = r < n ? fabs(a[r * lda + k]) : -1.0;
            int idx = r;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(v, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            if (tid == 0) *piv_sh = idx;
        }
        __syncthreads();
        const int p = *piv_sh;
        if (p != k) {
            for (int c = tid; c < width; c += blockDim.x) {
                const double t = a[k * lda + c];
                a[k * lda + c] = a[p * lda + c];
                a[p * lda + c] = t;
            }
        }
        __syncthreads();
        const double inv = rcp64l(a[k * lda + k]);
        // multipliers then trailing update (rows k+1.., columns k+1..)
        const int rows = n - k - 1, cols = width - k - 1;
        for (int idx = tid; idx < rows * cols; idx += blockDim.x) {
            const int r = k + 1 + idx / cols, c = k + 1 + idx % cols;
            const double f = a[r * lda + k] * inv;
            a[r * lda + c] = fma(-f, a[k * lda + c], a[r * lda + c]);
        }
        __syncthreads();
    }
    // back substitution, one right-hand side column per thread
    for (int c = n + tid; c < width; c += blockDim.x) {
        for (int i = n - 1; i >= 0; --i) {
            double s = a[i * lda + c];
            for (int l = i + 1; l < n; ++l) s = fma(-a[i * lda + l], a[l * lda + c], s);
            a[i * lda + c] = s * rcp64l(a[i * lda + i]);
        }
    }
    __syncthreads();
}

// In-place lower Cholesky factor (double) of the n x n SPD matrix S (stride
// lds); returns false (workgroup-uniform) if a pivot is not positive.
__device__ bool cholesky(double* S, int lds, int n, int* flag_sh) {
    const int tid = threadIdx.x;
    if (tid == 0) *flag_sh = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = S[j * lds + j];
            if (!(d > 0.0)) *flag_sh = 1;
            S[j * lds + j] = sqrt(d);
        }
        __syncthreads();
        const double inv = rcp64l(S[j * lds + j]);
        for (int i = j + 1 + tid; i < n; i += blockDim.x) S[i * lds + j] *= inv;
        __syncthreads();
        const int m = n - j - 1;
        for (int idx = tid; idx < m * m; idx += blockDim.x) {
            const int i = j + 1 + idx / m, l = j + 1 + idx % m;
            if (l <= i) S[i * lds + l] = fma(-S[i * lds + j], S[l * lds + j], S[i * lds + l]);
        }
        __syncthreads();
    }
    const bool ok = *flag_sh == 0;
    __syncthreads();
    return ok;
}

// X [n x r] (stride ldx) <- (L L^T)^-1 X, one column per thread
__device__ void chol_solve(const double* L, int ldl, int n, double* X, int ldx, int r) {
    for (int c = threadIdx.x; c < r; c += blockDim.x) {
        for (int i = 0; i < n; ++i) {
            double s = X[i * ldx + c];
            for (int l = 0; l < i; ++l) s = fma(-L[i * ldl + l], X[l * ldx + c], s);
            X[i * ldx + c] = s * rcp64l(L[i * ldl + i]);
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = X[i * ldx + c];
            for (int l = i + 1; l < n; ++l) s = fma(-L[l * ldl + i], X[l * ldx + c], s);
            X[i * ldx + c] = s * rcp64l(L[i * ldl + i]);
        }
    }
    __syncthreads();
}

// workgroup-uniform test: every entry of X is zero
template <typename R>
__device__ bool all_zero(const R* X, int count, int* flag_sh) {
    if (threadIdx.x == 0) *flag_sh = 1;
    __syncthreads();
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        if (X[i] != R(0)) *flag_sh = 0;
    __syncthreads();
    const bool z = *flag_sh != 0;
    __syncthreads();
    return z;
}

}  // namespace large
}  // namespace pks
