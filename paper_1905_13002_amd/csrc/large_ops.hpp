// large_ops.hpp -- workgroup-cooperative matrix operations for the scan of
// large state dimensions (5 <= nx <= 64): one workgroup (one, two or four
// waves, by nx) owns one scan element at a time; matrices live in an arena
// that is LDS when it fits and a per-workgroup workspace slot otherwise (the
// kernels are instantiated for each placement, so LDS arenas are addressed
// with LDS instructions).
//
// Precision policy (as for small states): R is the storage/product type; the
// LU factorisation with partial pivoting of I + C_i J_j and its solves, the
// Cholesky factorisations and every covariance symmetrisation run in double.
#pragma once
#include <hip/hip_runtime.h>

namespace pks {
namespace large {

// Launch bound of the scan kernels: the largest workgroup (eight waves), and
// with it a cap of 256 registers per lane, so that two four-wave workgroups
// share a compute unit (at a bound of four waves the FP64 filter kernels took
// up to 266 and ran one workgroup per unit).
constexpr int kThreads = 512;

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
    constexpr int kUnrollK = BS == 4 ? 4 : 8;      // k steps whose loads are in flight together
    for (int blk = threadIdx.x; blk < bm * bn; blk += blockDim.x) {
        const int i0 = (blk / bn) * BS, j0 = (blk % bn) * BS;
        R acc[BS][BS];
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int b = 0; b < BS; ++b) acc[a][b] = R(0);
        // unrolled so that the loads of several k steps are in flight together
#pragma unroll kUnrollK
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

typedef double f64x4 __attribute__((ext_vector_type(4)));

// FP64 product on the matrix cores (v_mfma_f64_16x16x4f64), one wave per
// 16 x 16 tile of C, K in steps of 4.  Operands as for the FP32 instruction
// (lane l supplies A(i0 + l % 16, k + l / 16) and B(k + l / 16, j0 + l % 16)),
// but the FP64 result rows are interleaved: accumulator register r of lane l
// holds C(i0 + 4 r + l / 16, j0 + l % 16).  Four k steps are loaded before
// their products issue, so several operand loads are in flight.  Kept out of
// line: inlined, its registers count against every caller, including the
// kernels of small states that never take this path.
__device__ __noinline__ void gemm_mfma_f64(double* C, int ldc, const double* A, int lda, bool ta, const double* B,
                                              int ldb, bool tb, int m, int n, int k, double alpha, const double* D,
                                              int ldd) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
    for (int t = wave; t < tm * tn; t += nwaves) {
        const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
        const int ia = i0 + li, jb = j0 + li;
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        int l0 = 0;
        for (; l0 + 16 <= k; l0 += 16) {
            double av[4], bv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int l = l0 + 4 * q + lk;
                av[q] = ia < m ? (ta ? A[l * lda + ia] : A[ia * lda + l]) : 0.0;
                bv[q] = jb < n ? (tb ? B[jb * ldb + l] : B[l * ldb + jb]) : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
        }
        for (; l0 < k; l0 += 4) {
            const int l = l0 + lk;
            const double av = (ia < m && l < k) ? (ta ? A[l * lda + ia] : A[ia * lda + l]) : 0.0;
            const double bv = (jb < n && l < k) ? (tb ? B[jb * ldb + l] : B[l * ldb + jb]) : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        const int j = j0 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + 4 * r + lk;
            if (i < m && j < n) {
                double v = alpha * acc[r];
                if (D) v += D[i * ldd + j];
                C[i * ldc + j] = v;
            }
        }
    }
}

// Products of the storage type.  Products with both output dimensions at
// least 16 (dense enough to fill 16 x 16 tiles) run on the matrix cores;
// `sync` = false leaves out the closing workgroup barrier, for a product
// followed by others that neither read its output nor write its operands.
// everything else on the vector units, with the largest register block that
// still gives every thread of the workgroup a block of C.
template <typename R>
__device__ __forceinline__ void gemmR(R* C, int ldc, const R* A, int lda, bool ta, const R* B, int ldb, bool tb, int m, int n, int k,
                      R alpha = R(1), const R* D = nullptr, int ldd = 0, bool sync = true) {
    const int threads = blockDim.x;
    if (m >= 16 && n >= 16) {
        if constexpr (sizeof(R) == 4)
            gemm_mfma_f32(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
        else
            gemm_mfma_f64(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
        if (sync) __syncthreads();
        return;
    }
    if (((m + 3) >> 2) * ((n + 3) >> 2) >= threads)
        gemm_blocks<4, R>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
    else if (((m + 1) >> 1) * ((n + 1) >> 1) >= threads)
        gemm_blocks<2, R>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
    else
        gemm_blocks<1, R>(C, ldc, A, lda, ta, B, ldb, tb, m, n, k, alpha, D, ldd);
    if (sync) __syncthreads();
}

// Walks the row-major (row, col) pairs of a range with `cols` columns that
// thread t of a group of g threads owns (elements t, t + g, t + 2g, ...): one
// division up front, then additions only (the GPU has no integer divide, and
// a division per element costs more than the arithmetic it indexes).
struct Walk2 {
    int r, c, dr, dc, cols;
    __device__ __forceinline__ Walk2(int t, int g, int cols_) : cols(cols_) {
        if (cols_ <= 0) {
            r = 0x7fffffff;
            c = dr = dc = 0;
            return;
        }
        r = t / cols_;
        c = t - r * cols_;
        dr = g / cols_;
        dc = g - dr * cols_;
    }
    __device__ __forceinline__ void next() {
        r += dr;
        c += dc;
        if (c >= cols) {
            c -= cols;
            ++r;
        }
    }
};

// C[m x n] = TC(alpha * A B + D), A [m x k] (TA) and B [k x n] (TB), both
// row-major and untransposed, sums in double: products of storage values with
// FP64 solution blocks.  C may alias D but not A or B.
template <int BS, typename TA, typename TB, typename TC>
__device__ __forceinline__ void gemm_blocks_acc64(TC* C, int ldc, const TA* A, int lda, const TB* B, int ldb, int m,
                                                  int n, int k, double alpha, const TC* D, int ldd) {
    const int bm = (m + BS - 1) / BS, bn = (n + BS - 1) / BS;
    constexpr int kUnrollK = BS == 4 ? 4 : 8;      // k steps whose loads are in flight together
    for (int blk = threadIdx.x; blk < bm * bn; blk += blockDim.x) {
        const int i0 = (blk / bn) * BS, j0 = (blk % bn) * BS;
        double acc[BS][BS];
#pragma unroll
        for (int a = 0; a < BS; ++a)
#pragma unroll
            for (int b = 0; b < BS; ++b) acc[a][b] = 0.0;
#pragma unroll kUnrollK
        for (int l = 0; l < k; ++l) {
            double av[BS], bv[BS];
#pragma unroll
            for (int a = 0; a < BS; ++a) av[a] = i0 + a < m ? double(A[(i0 + a) * lda + l]) : 0.0;
#pragma unroll
            for (int b = 0; b < BS; ++b) bv[b] = j0 + b < n ? double(B[l * ldb + j0 + b]) : 0.0;
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
                if (i < m && j < n) C[i * ldc + j] = TC(alpha * acc[a][b] + (D ? double(D[i * ldd + j]) : 0.0));
            }
    }
}

template <typename TA, typename TB, typename TC>
__device__ __forceinline__ void gemm_acc64(TC* C, int ldc, const TA* A, int lda, const TB* B, int ldb, int m, int n, int k,
                           double alpha, const TC* D = nullptr, int ldd = 0, bool sync = true) {
    const int threads = blockDim.x;
    if (((m + 3) >> 2) * ((n + 3) >> 2) >= threads)
        gemm_blocks_acc64<4>(C, ldc, A, lda, B, ldb, m, n, k, alpha, D, ldd);
    else if (((m + 1) >> 1) * ((n + 1) >> 1) >= threads)
        gemm_blocks_acc64<2>(C, ldc, A, lda, B, ldb, m, n, k, alpha, D, ldd);
    else
        gemm_blocks_acc64<1>(C, ldc, A, lda, B, ldb, m, n, k, alpha, D, ldd);
    if (sync) __syncthreads();
}

// The next (up to) four pairs of a walk over `rows` rows; returns how many.
// Sweeps load the operands of all four before storing any result, so the four
// independent updates overlap their memory latency.
__device__ __forceinline__ int take4(Walk2& it, int rows, int (&r)[4], int (&c)[4]) {
    int k = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        r[u] = it.r < rows ? it.r : 0;
        c[u] = it.c;
        if (it.r < rows) {
            ++k;
            it.next();
        }
    }
    return k;
}

// X[j][c] -= Lc[j * sl] * inv * xi[c] for j = j0 .. j0 + rows - 1 and
// c = c0 .. c0 + w - 1, by one wave (Lc: the coefficient column or row, stride
// sl; xi: the pivot row, already final)
__device__ __forceinline__ void wave_axpy_rows(const double* Lc, int sl, double inv, const double* xi, double* X, int ldx,
                                               int j0, int rows, int c0, int w) {
    const int lane = threadIdx.x & 63;
    for (Walk2 it(lane, 64, w); it.r < rows;) {
        int rr[4], cc[4];
        const int k = take4(it, rows, rr, cc);
        double lj[4], xp[4], xc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < k) {
                lj[u] = Lc[(j0 + rr[u]) * sl];
                xp[u] = xi[c0 + cc[u]];
                xc[u] = X[(j0 + rr[u]) * ldx + c0 + cc[u]];
            }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < k) X[(j0 + rr[u]) * ldx + c0 + cc[u]] = fma(-lj[u] * inv, xp[u], xc[u]);
    }
}

// out = (X + X^T)/2 + D (symmetrisation in double); out may alias D, not X
template <typename R>
__device__ __forceinline__ void sym_add(R* out, const R* X, const R* D, int n, bool sync = true) {
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int i = it.r, j = it.c;
        const int idx = it.r * it.cols + it.c;
        out[idx] = R(0.5 * (double(X[i * n + j]) + double(X[j * n + i])) + (D ? double(D[idx]) : 0.0));
    }
    if (sync) __syncthreads();
}

template <typename T, typename U>
__device__ __forceinline__ void copy(T* dst, const U* src, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = T(src[i]);
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void fill(T* dst, T v, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) dst[i] = v;
    __syncthreads();
}

// y[m] = op(A) x (+ d), A [m x k] (or [k x m] if ta)
template <typename R>
__device__ __forceinline__ void gemv(R* y, const R* A, int lda, bool ta, const R* x, int m, int k, const R* d = nullptr,
                     R alpha = R(1), bool sync = true) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        R s = R(0);
#pragma unroll 8
        for (int l = 0; l < k; ++l) s = fma(ta ? A[l * lda + i] : A[i * lda + l], x[l], s);
        y[i] = alpha * s + (d ? d[i] : R(0));
    }
    if (sync) __syncthreads();
}

// Makes the LDS and global writes of one wave visible to its other lanes (a
// barrier for the lanes of one wave only; the other waves are not involved).
__device__ __forceinline__ void wave_sync_mem() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The right-hand-side columns [c0, c1) that wave `wave` of `nw` owns.
__device__ __forceinline__ void wave_columns(int r, int& c0, int& c1) {
    const int nw = blockDim.x >> 6, wave = threadIdx.x >> 6;
    const int per = (r + nw - 1) / nw;
    c0 = wave * per;
    c1 = c0 + per < r ? c0 + per : r;
}

// Upper-triangular back substitution U x = z on columns [c0, c1) of X by one
// wave: at step i row i is final; the rows above are updated with it scaled by
// 1 / u_ii on the fly, and the scaled rows are written after the sweep.
__device__ __forceinline__ void wave_upper_solve(const double* U, int ldu, int n, double* X, int ldx, int c0, int c1) {
    const int lane = threadIdx.x & 63, w = c1 - c0;
    for (int i = n - 1; i > 0; --i) {
        const double inv = rcp64l(U[i * ldu + i]);
        // rows 0 .. i-1: X[r][c] -= U[r][i] / u_ii * X[i][c]
        wave_axpy_rows(U + i, ldu, inv, X + i * ldx, X, ldx, 0, i, c0, w);
        wave_sync_mem();
    }
    for (Walk2 it(lane, 64, w); it.r < n; it.next()) {
        const int r = it.r, c = c0 + it.c;
        X[r * ldx + c] *= rcp64l(U[r * ldu + r]);
    }
    wave_sync_mem();
}

// In-place LU solve with partial pivoting (double): a is [n x (n + w)], row
// stride lda, n <= 64; on return columns n .. n+w-1 hold M^-1 times the
// right-hand sides.  Wave 0 factors M (pivot rows exchanged across M's
// columns, multipliers kept unscaled below the diagonal); then every wave
// applies the exchanges and both triangular sweeps to its own right-hand-side
// columns, synchronising only its own lanes.  piv_sh holds >= n + 1 ints.
__device__ __forceinline__ void lu_solve(double* a, int lda, int n, int w, int* piv_sh) {
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < 64) {
        for (int k = 0; k < n; ++k) {
            // pivot: argmax |a[r][k]|, r >= k (one row per lane)
            const int r0 = k + lane;
            double v = r0 < n ? fabs(a[r0 * lda + k]) : -1.0;
            int idx = r0;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(v, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (ov > v || (ov == v && oi < idx)) {
                    v = ov;
                    idx = oi;
                }
            }
            const int p = idx;
            if (lane == 0) piv_sh[k] = p;
            if (p != k) {
                for (int c = lane; c < n; c += 64) {
                    const double t = a[k * lda + c];
                    a[k * lda + c] = a[p * lda + c];
                    a[p * lda + c] = t;
                }
                wave_sync_mem();
            }
            // trailing update of M with the unscaled multipliers a[r][k] / a[k][k]
            const double inv = rcp64l(a[k * lda + k]);
            const int rows = n - k - 1;
            // rows k+1 .. n-1 of columns k+1 .. n-1 (column offset k+1)
            wave_axpy_rows(a + k, lda, inv, a + k * lda + k + 1, a + k + 1, lda, k + 1, rows, 0, rows);
            wave_sync_mem();
        }
    }
    __syncthreads();
    int c0, c1;
    wave_columns(w, c0, c1);
    c0 += n;
    c1 += n;
    const int wc = c1 - c0;
    if (wc > 0) {
        // row exchanges, in order
        for (int k = 0; k < n; ++k) {
            const int p = piv_sh[k];
            if (p != k) {
                for (int c = c0 + lane; c < c1; c += 64) {
                    const double t = a[k * lda + c];
                    a[k * lda + c] = a[p * lda + c];
                    a[p * lda + c] = t;
                }
                wave_sync_mem();
            }
        }
        // unit lower-triangular forward sweep
        for (int k = 0; k + 1 < n; ++k) {
            const double inv = rcp64l(a[k * lda + k]);
            // rows k+1 .. n-1: a[r][c] -= a[r][k] / a_kk * a[k][c]
            wave_axpy_rows(a + k, lda, inv, a + k * lda, a, lda, k + 1, n - k - 1, c0, wc);
            wave_sync_mem();
        }
        wave_upper_solve(a, lda, n, a, lda, c0, c1);
    }
    __syncthreads();
}

__device__ __forceinline__ double pick4(const double (&v)[4], int t) {
    return t == 0 ? v[0] : (t == 1 ? v[1] : (t == 2 ? v[2] : v[3]));
}

// Cholesky factor of an n x n SPD matrix, n <= 16, by one wave in registers
// (no workgroup barrier): lane 4 i + q holds row i, columns 4 q .. 4 q + 3
// (zero outside n).  Each column step takes the pivot, the lane's entry of
// column j and its four entries of row j by lane permutes, then updates the
// trailing square with l_i l_c (bitwise symmetric).  On return S holds L
// below the diagonal and L^T above it.  Returns false if a pivot is not
// positive (the same on every lane).
__device__ __forceinline__ bool cholesky_reg16_wave(double* S, int lds, int n) {
    const int lane = threadIdx.x & 63;
    const int i = lane >> 2, q = lane & 3, c0 = 4 * q;
    double s[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) s[t] = (i < n && c0 + t < n) ? S[i * lds + c0 + t] : 0.0;
    bool ok = true;
    for (int j = 0; j < n; ++j) {
        const int jq = j >> 2, jt = j & 3;
        const double mine = pick4(s, jt);                   // this lane's entry in column j (if its quad holds j)
        const double d = __shfl(mine, 4 * j + jq, 64);        // s_jj
        const double colv = __shfl(mine, 4 * i + jq, 64);     // s_ij
        double rowv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) rowv[t] = __shfl(s[t], 4 * j + q, 64);   // s_j,c0+t
        ok = ok && d > 0.0;
        const double isq = rcp64l(sqrt(d));
        const double li = colv * isq;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (i > j && c0 + t > j) s[t] = fma(-li, rowv[t] * isq, s[t]);
    }
    // the pivots: s_cc of this lane's columns sits in lane 4 c + q, entry t
    double dg[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) dg[t] = __shfl(s[t], 4 * (c0 + t) + q, 64);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int c = c0 + t;
        if (i < n && c < n) {
            if (c < i) {
                const double v = s[t] * rcp64l(sqrt(dg[t]));
                S[i * lds + c] = v;
                S[c * lds + i] = v;
            } else if (c == i) {
                S[i * lds + i] = sqrt(s[t]);
            }
        }
    }
    return ok;
}

// n <= 16: wave 0 factors, the workgroup waits
__device__ __forceinline__ bool cholesky_reg16(double* S, int lds, int n, int* flag_sh) {
    if (threadIdx.x < 64) {
        const bool ok = cholesky_reg16_wave(S, lds, n);
        if (threadIdx.x == 0) *flag_sh = ok ? 0 : 1;
    }
    __syncthreads();
    const bool ok = *flag_sh == 0;
    __syncthreads();
    return ok;
}

// Blocked Cholesky factor for 16 < n <= 64 (same storage: L below, L^T above
// the diagonal).  For each block column of 16: wave 0 factors the diagonal
// block in registers; one thread per row below solves that row of the panel
// (x L_JJ^T = s) and writes it to both triangles; the trailing square is
// updated with the panel product (FP64, register-blocked, bitwise symmetric).
__device__ __forceinline__ bool cholesky_blocked(double* S, int lds, int n, int* flag_sh) {
    const int tid = threadIdx.x;
    bool ok = true;
    for (int j0 = 0; j0 < n; j0 += 16) {
        const int bj = n - j0 < 16 ? n - j0 : 16;
        double* D = S + j0 * lds + j0;
        if (tid < 64) ok = cholesky_reg16_wave(D, lds, bj) && ok;
        __syncthreads();
        const int i0 = j0 + bj, rows = n - i0;
        for (int rr = tid; rr < rows; rr += blockDim.x) {
            const int i = i0 + rr;
            double x[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = c < bj ? S[i * lds + j0 + c] : 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                if (c < bj) {
                    double v = x[c];
#pragma unroll
                    for (int k = 0; k < c; ++k) v = fma(-x[k], D[c * lds + k], v);
                    x[c] = v * rcp64l(D[c * lds + c]);
                }
            }
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < bj) {
                    S[i * lds + j0 + c] = x[c];
                    S[(j0 + c) * lds + i] = x[c];
                }
        }
        __syncthreads();
        if (rows > 0) {
            double* P = S + i0 * lds + j0;            // the panel, rows i0 .. n-1
            double* T = S + i0 * lds + i0;            // the trailing square
            gemmR<double>(T, lds, P, lds, false, P, lds, true, rows, rows, bj, -1.0, T, lds);
        }
    }
    if (tid == 0) *flag_sh = ok ? 0 : 1;
    __syncthreads();
    const bool res = *flag_sh == 0;
    __syncthreads();
    return res;
}

// In-place Cholesky factor (double) of the n x n SPD matrix S (stride lds),
// n <= 64: on return the lower triangle holds L and the upper triangle L^T (so
// every triangular sweep reads rows).  Returns false (workgroup-uniform) if a
// pivot is not positive.  n <= 16: one wave in registers; larger: blocked by
// 16.  flag_sh holds one int.
__device__ __forceinline__ bool cholesky(double* S, int lds, int n, int* flag_sh) {
    if (n <= 16) return cholesky_reg16(S, lds, n, flag_sh);
    return cholesky_blocked(S, lds, n, flag_sh);
}

// Triangular sweeps with a factor block from cholesky() (n <= 16; L below,
// L^T above the diagonal): X [n x r] <- L^-1 X (fwd) and/or L^-T X (bwd).  The
// columns go in passes of 16, one pass per wave at a time: lane 4 i + q holds
// X[i][4 q .. 4 q + 3] of the pass and caches row i of the stored factor
// (L[i][j] for j < i, L[j][i] for j > i); each step finishes one row and sends
// it to the others by lane permutes (sweeps fully unrolled).  Ends with a
// workgroup barrier.
__device__ __forceinline__ void trsm_reg16(const double* L, int ldl, int n, double* X, int ldx, int r, bool fwd,
                                           bool bwd) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int i = lane >> 2, q = lane & 3, c0 = 4 * q;
    if (16 * wave < r) {
        double rw[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) rw[j] = (i < n && j < n) ? L[i * ldl + j] : 0.0;
        const double dinv = i < n ? rcp64l(L[i * ldl + i]) : 0.0;
        for (int cb = 16 * wave; cb < r; cb += 16 * nw) {
            double x[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = cb + c0 + t;
                x[t] = (i < n && c < r) ? X[i * ldx + c] : 0.0;
            }
            if (fwd) {
                // L z = x: row j is final once scaled by 1 / l_jj
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j < n) {
                        if (i == j) {
#pragma unroll
                            for (int t = 0; t < 4; ++t) x[t] *= dinv;
                        }
                        double zj[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) zj[t] = __shfl(x[t], 4 * j + q, 64);
                        if (i > j) {
#pragma unroll
                            for (int t = 0; t < 4; ++t) x[t] = fma(-rw[j], zj[t], x[t]);
                        }
                    }
                }
            }
            if (bwd) {
                // L^T x = z, from the last row up
#pragma unroll
                for (int j = 15; j >= 0; --j) {
                    if (j < n) {
                        if (i == j) {
#pragma unroll
                            for (int t = 0; t < 4; ++t) x[t] *= dinv;
                        }
                        double xj[4];
#pragma unroll
                        for (int t = 0; t < 4; ++t) xj[t] = __shfl(x[t], 4 * j + q, 64);
                        if (i < j) {
#pragma unroll
                            for (int t = 0; t < 4; ++t) x[t] = fma(-rw[j], xj[t], x[t]);
                        }
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int c = cb + c0 + t;
                if (i < n && c < r) X[i * ldx + c] = x[t];
            }
        }
    }
    __syncthreads();
}

// X [n x r] <- (L L^T)^-1 X for 16 < n <= 64: blocked sweeps, the diagonal
// blocks with trsm_reg16, the rest as FP64 products
__device__ __forceinline__ void chol_solve_blocked(const double* L, int ldl, int n, double* X, int ldx, int r) {
    for (int j0 = 0; j0 < n; j0 += 16) {
        const int bj = n - j0 < 16 ? n - j0 : 16, i0 = j0 + bj;
        trsm_reg16(L + j0 * ldl + j0, ldl, bj, X + j0 * ldx, ldx, r, true, false);
        if (i0 < n)
            gemmR<double>(X + i0 * ldx, ldx, L + i0 * ldl + j0, ldl, false, X + j0 * ldx, ldx, false, n - i0, r, bj,
                          -1.0, X + i0 * ldx, ldx);
    }
    const int last = ((n - 1) / 16) * 16;
    for (int j0 = last; j0 >= 0; j0 -= 16) {
        const int bj = n - j0 < 16 ? n - j0 : 16;
        trsm_reg16(L + j0 * ldl + j0, ldl, bj, X + j0 * ldx, ldx, r, false, true);
        if (j0 > 0)   // rows above: X[0 .. j0) -= (L^T)[0 .. j0, j0 .. j0+bj) X_J, L^T stored above the diagonal
            gemmR<double>(X, ldx, L + j0, ldl, false, X + j0 * ldx, ldx, false, j0, r, bj, -1.0, X, ldx);
    }
}

// X [n x r] (stride ldx) <- (L L^T)^-1 X for a factor from cholesky(), n <= 64
__device__ __forceinline__ void chol_solve(const double* L, int ldl, int n, double* X, int ldx, int r) {
    if (n <= 16) trsm_reg16(L, ldl, n, X, ldx, r, true, true);
    else chol_solve_blocked(L, ldl, n, X, ldx, r);
}

// workgroup-uniform test: every entry of X is zero
template <typename R>
__device__ __forceinline__ bool all_zero(const R* X, int count, int* flag_sh) {
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
