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

// C[m x n] = alpha * op(A) op(B) (+ D), row-major with leading dimensions,
// products and sums in the storage type R (float in the mixed mode).  op(A) =
// A [m x k] or A^T (A stored [k x m]); same for B.  Each thread computes a
// BS x BS block of C.  C may alias D but not A or B.
template <int BS, typename R>
__device__ __forceinline__ void gemm_blocks(R* C, int ldc, const R* A, int lda, bool ta, const R* B, int ldb, bool tb,
                                            int m, int n, int k, R alpha, const R* D, int ldd) {
    const int bm = (m + BS - 1) / BS, bn = (n + BS - 1) / BS;
    for (int blk = threadIdx.x; blk < bm * bn; blk += blockDim.x) {
        const int i0 = (blk / bn) * BS, j0 = (blk % bn) * BS;
        R acc[BS][BS];
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int b = 0; b < BS; ++b) acc[a][b] = R(0);
        // unrolled so that the loads of several k steps are in flight together
#pragma unroll(BS == 4 ? 4 : 8)
        for (int l = 0; l < k; ++l) {
            R av[BS], bv[BS];
#pragma unroll
            for (int a = 0; a < BS; ++a) {
                const int i = i0 + a;
                av[a] = i < m ? (ta ? A[l * lda + i] : A[i * lda + l]) : R(0);
            }
#pragma unroll
            for (int b = 0; b < BS; ++b) {
                const int j = j0 + b;
                bv[b] = j < n ? (tb ? B[j * ldb + l] : B[l * ldb + j]) : R(0);
            }
#pragma unroll
            for (int a = 0; a < BS; ++a)
#pragma unroll
                for (int b = 0; b < BS; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int b = 0; b < BS; ++b) {
                const int i = i0 + a, j = j0 + b;
                if (i < m && j < n) {
                    R v = alpha * acc[a][b];
                    if (D) v += D[i * ldd + j];
                    C[i * ldc + j] = v;
                }
            }
    }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 product on the matrix cores: one wave per 16 x 16 tile of C, K in
// steps of 4 (v_mfma_f32_16x16x4f32).  Lane l supplies A(i0 + l % 16, k + l / 16)
// and B(k + l / 16, j0 + l % 16) and receives C(i0 + 4 (l / 16) + r, j0 + l % 16)
// in accumulator register r.  Out-of-range operands are read as zero, so any
// m, n, k work; every lane of a wave issues every MFMA.
__device__ __forceinline__ void gemm_mfma_f32(float* C, int ldc, const float* A, int lda, bool ta, const float* B,
                                              int ldb, bool tb, int m, int n, int k, float alpha, const float* D,
                                              int ldd) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
    for (int t = wave; t < tm * tn; t += nwaves) {
        const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
        const int ia = i0 + li, jb = j0 + li;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int l0 = 0; l0 < k; l0 += 4) {
            const int l = l0 + lk;
            const float av = (ia < m && l < k) ? (ta ? A[l * lda + ia] : A[ia * lda + l]) : 0.f;
            const float bv = (jb < n && l < k) ? (tb ? B[jb * ldb + l] : B[l * ldb + jb]) : 0.f;
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
        }
        const int j = j0 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 4 * lk + r;
            if (i < m && j < n) {
                float v = alpha * acc[r];
                if (D) v += D[i * ldd + j];
                C[i * ldc + j] = v;
            }
        }
    }
}

// Products of the storage type.  FP32 products with both output dimensions
// at least 32 (dense enough to fill 16 x 16 tiles) run on the matrix cores;
// everything else on the vector units, with the largest register block that
// still gives every thread of the workgroup a block of C.
template <typename R>
__device__ void gemmR(R* C, int ldc, const R* A, int lda, bool ta, const R* B, int ldb, bool tb, int m, int n, int k,
                      R alpha = R(1), const R* D = nullptr, int ldd = 0) {
    const int threads = blockDim.x;
    if constexpr (sizeof(R) == 4) {
        if (m >= 32 && n >= 32) {
            gemm_mfma_f32(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
            __syncthreads();
            return;
        }
    }
    if (((m + 3) >> 2) * ((n + 3) >> 2) >= threads)
        gemm_blocks<4, R>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
    else if (((m + 1) >> 1) * ((n + 1) >> 1) >= threads)
        gemm_blocks<2, R>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
    else
        gemm_blocks<1, R>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
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
#pragma unroll 8
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
    // back substitution U x = z, all right-hand sides at once: at step i the
    // entries of row i are final; rows above it are updated with row i scaled
    // by 1 / u_ii (scaled copies of the rows are written after the sweep)
    for (int i = n - 1; i > 0; --i) {
        const double inv = rcp64l(a[i * lda + i]);
        for (int idx = tid; idx < i * w; idx += blockDim.x) {
            const int r = idx / w, c = n + idx % w;
            a[r * lda + c] = fma(-a[r * lda + i] * inv, a[i * lda + c], a[r * lda + c]);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * w; idx += blockDim.x) {
        const int r = idx / w, c = n + idx % w;
        a[r * lda + c] *= rcp64l(a[r * lda + r]);
    }
    __syncthreads();
}

// In-place lower Cholesky factor (double) of the n x n SPD matrix S (stride
// lds); returns false (workgroup-uniform) if a pivot is not positive.  At step
// j column j is final; the trailing lower triangle is updated with that column
// scaled by 1 / sqrt(s_jj), and the scaled columns are written after the loop.
__device__ bool cholesky(double* S, int lds, int n, int* flag_sh) {
    const int tid = threadIdx.x;
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        const double d = S[j * lds + j];
        ok = ok && d > 0.0;
        const double inv = rcp64l(d);               // 1 / s_jj = (1 / sqrt(s_jj))^2
        const int m = n - j - 1;
        for (int idx = tid; idx < m * m; idx += blockDim.x) {
            const int i = j + 1 + idx / m, l = j + 1 + idx % m;
            if (l <= i) S[i * lds + l] = fma(-S[i * lds + j] * inv, S[l * lds + j], S[i * lds + l]);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
        const int i = idx / n, j = idx % n;
        if (j < i) S[i * lds + j] *= rcp64l(sqrt(S[j * lds + j]));
    }
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) S[j * lds + j] = sqrt(S[j * lds + j]);
    __syncthreads();
    (void)flag_sh;
    return ok;
}

// X [n x r] (stride ldx) <- (L L^T)^-1 X, all columns at once: one barrier per
// pivot row in each of the two triangular sweeps
__device__ void chol_solve(const double* L, int ldl, int n, double* X, int ldx, int r) {
    const int tid = threadIdx.x;
    // L z = x
    for (int i = 0; i + 1 < n; ++i) {
        const double inv = rcp64l(L[i * ldl + i]);
        const int rows = n - i - 1;
        for (int idx = tid; idx < rows * r; idx += blockDim.x) {
            const int j = i + 1 + idx / r, c = idx % r;
            X[j * ldx + c] = fma(-L[j * ldl + i] * inv, X[i * ldx + c], X[j * ldx + c]);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * r; idx += blockDim.x) {
        const int j = idx / r, c = idx % r;
        X[j * ldx + c] *= rcp64l(L[j * ldl + j]);
    }
    __syncthreads();
    // L^T x = z
    for (int i = n - 1; i > 0; --i) {
        const double inv = rcp64l(L[i * ldl + i]);
        for (int idx = tid; idx < i * r; idx += blockDim.x) {
            const int j = idx / r, c = idx % r;
            X[j * ldx + c] = fma(-L[i * ldl + j] * inv, X[i * ldx + c], X[j * ldx + c]);
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * r; idx += blockDim.x) {
        const int j = idx / r, c = idx % r;
        X[j * ldx + c] *= rcp64l(L[j * ldl + j]);
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
