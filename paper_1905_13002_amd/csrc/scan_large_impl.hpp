// scan_large_impl.hpp -- the filtering and smoothing scans for large state
// dimensions (5 <= nx <= 64): arena layouts, workgroup operators, kernels and
// the launcher template run_large<R, SEG>.  Each (precision, batched)
// instantiation is compiled in a translation unit of its own
// (scan_large_{f64,f32}[_seg].hip); scan_large.hip holds the host-side sizing.
//
// The time axis is cut into P blocks of l consecutive steps (the block-level
// elements of the paper's Section III-C).  One workgroup owns one block:
//   reduce : fold the block's elements sequentially into its block element
//            (Lemma 2 / Lemma 4, workgroup-cooperative matrix operations),
//   scan   : Kogge-Stone over the P block elements in ceil(log2 P) launches
//            (out[i] = in[i - d] (x) in[i] for the filter, in[i] (x) in[i + d]
//            for the smoother), ping-pong between two workspace buffers,
//   down   : re-fold the block from the moments of everything before it
//            (after it, for the smoother), writing the outputs.
// Single steps k > 1 of a model with ny < nx use the rank-ny form of Lemma 2
// (J_k = W G with G = H F): a Cholesky factorisation of the ny x ny matrix
// S + G C G^T replaces the LU factorisation of I + C J.
// Sequences packed back to back are separated by the exact zeros A = 0 of a
// first step and E = 0 of a last step, as for small states.
#pragma once
#include "large_ops.hpp"
#include "pks_internal.h"

namespace pks {
namespace lg {

using namespace large;

// offsets (in R words) of the records in memory: full matrices, row-major
struct FLay {
    int A, b, C, eta, J, words;
};
__host__ __device__ inline FLay flay(int n) {
    FLay f;
    f.A = 0;
    f.b = n * n;
    f.C = f.b + n;
    f.eta = f.C + n * n;
    f.J = f.eta + n;
    f.words = f.J + n * n;
    return f;
}
struct SLay {
    int E, g, L, words;
};
__host__ __device__ inline SLay slay(int n) {
    SLay s;
    s.E = 0;
    s.g = n * n;
    s.L = s.g + n;
    s.words = s.L + n * n;
    return s;
}
// moments: m at 0, P at n

// ---------------------------------------------------------------------------
// arena layouts (R words unless noted).  Each kernel gets only the buffers its
// operators touch; the offsets of the others stay 0 and are never used by it.
// ---------------------------------------------------------------------------
enum ArenaKind : int { kArFRed = 0, kArFKs, kArFDown, kArSRed, kArSKs, kArSDown, kArKinds };

struct Arena {
    // R buffers
    int acc, out, sel, xv, X1, x2, X3, w, JA, Z, T, Y, mom;
    // double buffers (offsets in doubles from the double base)
    int aug, sig;
    int rwords, dwords;
};
__host__ __device__ inline Arena arena_layout(int n, int ny, int kind) {
    Arena a = {};
    const int n2 = n * n, fw = flay(n).words, sw = slay(n).words;
    const bool lowrank = ny < n;
    int o = 0, d = 0;
    switch (kind) {
        case kArFRed:                       // accumulator updated in place
            a.acc = o; o += fw;
            a.out = a.acc;
            a.xv = o; o += 2 * n + ny;      // b_k, eta_k of a single step
            break;
        case kArFDown:
            a.mom = o; o += n + n2;
            a.xv = o; o += 2 * n + ny;
            break;
        case kArSRed:                       // accumulator / result ping-pong
            a.acc = o; o += sw;
            a.out = o; o += sw;             // element of step k
            a.sel = o; o += sw;
            a.mom = o; o += n + n2;
            break;
        case kArSDown:
            a.acc = o; o += n + n2;         // smoothed moments
            a.out = o; o += sw;
            break;
        default:                            // scans over block elements: operands and result in the workspace
            break;
    }
    if (kind <= kArFDown) {
        const bool combine = kind != kArFDown;          // two elements (else moments (x) element)
        const bool full = kind == kArFKs || !lowrank;   // LU of I + C J (else rank-ny form)
        a.x2 = o; o += n;
        a.X3 = o; o += n2;
        a.w = o; o += n;
        if (full || !combine) {              // the rank-ny combine puts its n x n scratch in Y and sig
            a.Z = o; o += n2;
            a.T = o; o += n2;
        }
        if (combine) {
            a.X1 = o; o += n2;
            a.JA = o; o += n2;
        }
        if (full) {
            a.aug = d; d += n * (combine ? 3 * n + 1 : 2 * n + 1);
        } else {
            const int yw = n * ny + ny * n + ny;           // Y [n x ny], GA [ny x n], Gv / Gb
            const int sw2 = ny * ny + ny * (combine ? 2 * n + 1 : n + 1);
            a.Y = o; o += combine && yw < n2 ? n2 : yw;
            a.sig = d; d += combine && sw2 < n2 ? n2 : sw2;
        }
    } else {
        a.T = o; o += n2;
        a.Z = o; o += n2;
        if (kind != kArSKs) {
            a.x2 = o; o += n;
            a.aug = d; d += 2 * n2;         // F P F^T + Q and E^T
        }
    }
    a.rwords = (o + 3) & ~3;
    a.dwords = d;
    return a;
}

struct Ctx {
    int n, ny;
    FLay fl;
    SLay sl;
    Arena ar;
    char* base;     // arena base (LDS or workspace slot)
    template <typename R>
    __device__ R* r(int off) const { return reinterpret_cast<R*>(base) + off; }
    template <typename R>
    __device__ double* d(int off) const {
        const size_t rbytes = ((size_t)ar.rwords * sizeof(R) + 15) & ~size_t(15);
        return reinterpret_cast<double*>(base + rbytes) + off;
    }
};

template <typename R>
__host__ __device__ inline size_t arena_bytes(int n, int ny, int kind) {
    const Arena a = arena_layout(n, ny, kind);
    return (((size_t)a.rwords * sizeof(R) + 15) & ~size_t(15)) + sizeof(double) * a.dwords;
}

struct LargeArgs {
    ScanArgs s;
    int64_t blen;        // steps per block
    int64_t nblocks;
    void* agg[2];        // ping-pong block elements [nblocks][words]
    int final_buf;       // which agg buffer holds the scanned elements
    int slot_mask;       // bit k: kernels of arena kind k use workspace slots, not LDS
    char* slots;         // per-block arena slots in the workspace
    size_t slot_bytes;
};

// context of one kernel: dimensions, record layouts and its arena.  LDSA:
// the arena is the kernel's LDS (the base then comes straight from the shared
// array, so the operators, all inlined, address it with LDS instructions);
// else the block's workspace slot.
template <bool LDSA>
__device__ __forceinline__ void make_ctx(Ctx& c, const LargeArgs& la, char* lds, int kind) {
    c.n = la.s.nx;
    c.ny = la.s.ny;
    c.fl = flay(c.n);
    c.sl = slay(c.n);
    c.ar = arena_layout(c.n, c.ny, kind);
    if constexpr (LDSA) c.base = lds;
    else c.base = la.slots + (size_t)blockIdx.x * la.slot_bytes;
}

// sequence lookup (workgroup-uniform)
struct SeqL {
    int b;
    int64_t start, end;
};
template <bool SEG>
__device__ SeqL seq_at(const ScanArgs& a, int64_t k) {
    SeqL s;
    if (!SEG) {
        s.b = 0; s.start = 0; s.end = a.total;
        return s;
    }
    int lo = 0, hi = a.B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.offsets[mid] <= k) lo = mid; else hi = mid;
    }
    s.b = lo;
    s.start = a.offsets[lo];
    s.end = a.offsets[lo + 1];
    return s;
}
template <bool SEG>
__device__ __forceinline__ void seq_fwd(const ScanArgs& a, SeqL& s, int64_t k) {
    if (!SEG) return;
    while (k >= s.end && s.b < a.B - 1) { ++s.b; s.start = s.end; s.end = a.offsets[s.b + 1]; }
}
template <bool SEG>
__device__ __forceinline__ void seq_bwd(const ScanArgs& a, SeqL& s, int64_t k) {
    if (!SEG) return;
    while (k < s.start && s.b > 0) { --s.b; s.end = s.start; s.start = a.offsets[s.b]; }
}

// ---------------------------------------------------------------------------
// filtering operator pieces
// ---------------------------------------------------------------------------
// Output half of Lemma 2 given X1 = M^-1 A_i, x2 = M^-1 (b_i + C_i eta_j),
// X3 = M^-1 C_i, w = eta_j - J_j b_i and JA = J_j A_i (all in the arena):
//   A = A_j X1, b = A_j x2 + b_j, C = sym(A_j X3 A_j^T) + C_j,
//   eta = X1^T w + eta_i, J = sym(X1^T JA) + J_i.   Result in `out`, which may
// be ei itself.  Z and T are n x n scratch.
template <typename R>
__device__ __forceinline__ void fcombine_tail(const Ctx& c, const R* ei, const R* Aj, const R* bj, const R* Cj, R* out, R* Z, R* T) {
    const int n = c.n;
    R* X1 = c.r<R>(c.ar.X1);
    R* x2 = c.r<R>(c.ar.x2);
    R* X3 = c.r<R>(c.ar.X3);
    R* w = c.r<R>(c.ar.w);
    R* JA = c.r<R>(c.ar.JA);
    // five independent pieces, one barrier: each reads only scratch and the
    // constants and writes a buffer none of the others touches (eta, A, b of
    // `out` are written in place element by element where out is ei)
    gemv<R>(out + c.fl.eta, X1, n, true, w, n, n, ei + c.fl.eta, R(1), false);
    gemmR<R>(Z, n, X1, n, true, JA, n, false, n, n, n, R(1), nullptr, 0, false);
    gemmR<R>(out + c.fl.A, n, Aj, n, false, X1, n, false, n, n, n, R(1), nullptr, 0, false);
    gemv<R>(out + c.fl.b, Aj, n, false, x2, n, n, bj, R(1), false);
    gemmR<R>(T, n, Aj, n, false, X3, n, false, n, n, n);
    // J from Z while (A_j X3) A_j^T goes to X3, which the last product consumed
    sym_add<R>(out + c.fl.J, Z, ei + c.fl.J, n, false);
    gemmR<R>(X3, n, T, n, false, Aj, n, true, n, n, n);
    sym_add<R>(out + c.fl.C, X3, Cj, n);
}

// full Lemma 2: out = ei (x) ej; ej given by its parts (matrices may live in
// the model constants)
template <typename R>
__device__ __forceinline__ void fcombine_wg(const Ctx& c, const R* ei, const R* Aj, const R* bj, const R* Cj, const R* etaj,
                            const R* Jj, R* out, int* ish) {
    const int n = c.n, lda = 3 * n + 1;
    double* aug = c.d<R>(c.ar.aug);
    R* Z = c.r<R>(c.ar.Z);
    R* v = c.r<R>(c.ar.x2);
    // M = I + C_i J_j (products in R)
    gemmR<R>(Z, n, ei + c.fl.C, n, false, Jj, n, false, n, n, n, R(1), nullptr, 0, false);
    gemv<R>(v, ei + c.fl.C, n, false, etaj, n, n, ei + c.fl.b);          // b_i + C_i eta_j
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        aug[r * lda + q] = double(Z[idx]) + (r == q ? 1.0 : 0.0);
        aug[r * lda + n + q] = double(ei[c.fl.A + idx]);
        aug[r * lda + 2 * n + 1 + q] = double(ei[c.fl.C + idx]);
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x) aug[r * lda + 2 * n] = double(v[r]);
    __syncthreads();
    lu_solve(aug, lda, n, 2 * n + 1, ish);
    R* X1 = c.r<R>(c.ar.X1);
    R* x2 = c.r<R>(c.ar.x2);
    R* X3 = c.r<R>(c.ar.X3);
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        X1[idx] = R(aug[r * lda + n + q]);
        X3[idx] = R(aug[r * lda + 2 * n + 1 + q]);
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x) x2[r] = R(aug[r * lda + 2 * n]);
    __syncthreads();
    // w = eta_j - J_j b_i ; JA = J_j A_i
    gemv<R>(c.r<R>(c.ar.w), Jj, n, false, ei + c.fl.b, n, n, etaj, R(-1), false);
    gemmR<R>(c.r<R>(c.ar.JA), n, Jj, n, false, ei + c.fl.A, n, false, n, n, n);
    fcombine_tail<R>(c, ei, Aj, bj, Cj, out, Z, c.r<R>(c.ar.T));
}

// Lemma 2 with ej a single step k > 1 (J_j = W G, rank ny < nx)
template <typename R>
__device__ __forceinline__ void fcombine_fresh_wg(const Ctx& c, const R* ei, const R* Aj, const R* bj, const R* Cj, const R* etaj,
                                  const R* Gm, const R* Wm, const double* S, R* out, int* ish) {
    const int n = c.n, m = c.ny, rhs = 2 * n + 1;
    R* Y = c.r<R>(c.ar.Y);              // [n x m]
    R* GA = Y + n * m;                  // [m x n]
    R* Gv = GA + m * n;                 // [m]
    R* v = c.r<R>(c.ar.x2);
    double* sg = c.d<R>(c.ar.sig);      // Sigma [m x m]
    double* rh = sg + m * m;            // [m x (2n+1)] = [GA | Gv | Y^T]
    gemmR<R>(Y, m, ei + c.fl.C, n, false, Gm, n, true, n, m, n, R(1), nullptr, 0, false);   // C_i G^T
    gemv<R>(v, ei + c.fl.C, n, false, etaj, n, n, ei + c.fl.b, R(1), false);                   // b_i + C_i eta_j
    gemmR<R>(GA, n, Gm, n, false, ei + c.fl.A, n, false, m, n, n);                              // G A_i
    gemv<R>(Gv, Gm, n, false, v, m, n, nullptr, R(1), false);                                   // G v
    // G C_i G^T into the X1 buffer (free until X1 is formed)
    gemmR<R>(c.r<R>(c.ar.X1), m, Gm, n, false, Y, m, false, m, m, n);
    {
        const R* GY = c.r<R>(c.ar.X1);
        for (Walk2 it(threadIdx.x, blockDim.x, m); it.r < m; it.next()) {
            const int r = it.r, q = it.c;
            const int idx = it.r * it.cols + it.c;
            sg[idx] = S[idx] + 0.5 * (double(GY[r * m + q]) + double(GY[q * m + r]));
        }
        for (Walk2 it(threadIdx.x, blockDim.x, rhs); it.r < m; it.next()) {
            const int r = it.r, q = it.c;
            const int idx = it.r * it.cols + it.c;
            rh[idx] = q < n ? double(GA[r * n + q]) : (q == n ? double(Gv[r]) : double(Y[(q - n - 1) * m + r]));
        }
        __syncthreads();
    }
    cholesky(sg, m, m, ish);
    chol_solve(sg, m, m, rh, rhs, rhs);
    R* X1 = c.r<R>(c.ar.X1);
    R* x2 = c.r<R>(c.ar.x2);
    R* X3 = c.r<R>(c.ar.X3);
    // X1 = A_i - Y T1 ; x2 = v - Y t2 ; X3 = C_i - sym(Y Zt)   (T1, t2, Zt in rh),
    // products of Y with the FP64 solution summed in double.  Y Zt goes to the
    // JA buffer, free until JA is formed.
    // four independent pieces, one barrier (Gv was consumed by the right-hand side)
    gemm_acc64<R, double, R>(X1, n, Y, m, rh, rhs, n, n, m, -1.0, ei + c.fl.A, n, false);
    gemm_acc64<R, double, R>(x2, 1, Y, m, rh + n, rhs, n, 1, m, -1.0, v, 1, false);
    R* YZ = c.r<R>(c.ar.JA);
    gemm_acc64<R, double, R>(YZ, n, Y, m, rh + n + 1, rhs, n, n, m, -1.0, nullptr, 0, false);
    gemv<R>(Gv, Gm, n, false, ei + c.fl.b, m, n);                           // G b_i (reuses Gv)
    // X3 = C_i - sym(Y Zt) ; w = eta_j - W (G b_i) ; then JA = W (G A_i) over YZ
    sym_add<R>(X3, YZ, ei + c.fl.C, n, false);
    gemv<R>(c.r<R>(c.ar.w), Wm, m, false, Gv, n, m, etaj, R(-1));
    gemmR<R>(c.r<R>(c.ar.JA), n, Wm, m, false, GA, n, false, n, n, m);
    // the tail's scratch reuses the Sigma / right-hand-side region and the
    // Y | GA | Gv region, both consumed by now
    fcombine_tail<R>(c, ei, Aj, bj, Cj, out, reinterpret_cast<R*>(sg), Y);
}

// moments X (prefix with A = 0) <- X (x) a_j
template <typename R>
__device__ __forceinline__ void fcarry_wg(const Ctx& c, R* X, const R* Aj, const R* bj, const R* Cj, const R* etaj, const R* Jj,
                          int* ish) {
    const int n = c.n, lda = 2 * n + 1;
    R* m = X;
    R* P = X + n;
    double* aug = c.d<R>(c.ar.aug);
    R* Z = c.r<R>(c.ar.Z);
    R* v = c.r<R>(c.ar.w);
    gemmR<R>(Z, n, P, n, false, Jj, n, false, n, n, n);
    gemv<R>(v, P, n, false, etaj, n, n, m);
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        aug[r * lda + q] = double(Z[idx]) + (r == q ? 1.0 : 0.0);
        aug[r * lda + n + 1 + q] = double(P[idx]);
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x) aug[r * lda + n] = double(v[r]);
    __syncthreads();
    lu_solve(aug, lda, n, n + 1, ish);
    R* x2 = c.r<R>(c.ar.x2);
    R* X3 = c.r<R>(c.ar.X3);
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        X3[idx] = R(aug[r * lda + n + 1 + q]);
    }
    for (int r = threadIdx.x; r < n; r += blockDim.x) x2[r] = R(aug[r * lda + n]);
    __syncthreads();
    gemv<R>(m, Aj, n, false, x2, n, n, bj);
    R* T = c.r<R>(c.ar.T);
    gemmR<R>(T, n, Aj, n, false, X3, n, false, n, n, n);
    gemmR<R>(Z, n, T, n, false, Aj, n, true, n, n, n);
    sym_add<R>(P, Z, Cj, n);
}

template <typename R>
__device__ __forceinline__ void fcarry_fresh_wg(const Ctx& c, R* X, const R* Aj, const R* bj, const R* Cj, const R* etaj,
                                const R* Gm, const double* S, int* ish) {
    const int n = c.n, m = c.ny, rhs = n + 1;
    R* mm = X;
    R* P = X + n;
    R* Y = c.r<R>(c.ar.Y);
    R* Gv = Y + 2 * n * m;
    R* v = c.r<R>(c.ar.w);
    double* sg = c.d<R>(c.ar.sig);
    double* rh = sg + m * m;            // [m x (n+1)] = [Gv | Y^T]
    gemmR<R>(Y, m, P, n, false, Gm, n, true, n, m, n);                      // P G^T
    gemv<R>(v, P, n, false, etaj, n, n, mm);                                 // m + P eta_j
    gemv<R>(Gv, Gm, n, false, v, m, n);
    gemmR<R>(c.r<R>(c.ar.Z), m, Gm, n, false, Y, m, false, m, m, n);        // G P G^T
    {
        const R* GY = c.r<R>(c.ar.Z);
        for (Walk2 it(threadIdx.x, blockDim.x, m); it.r < m; it.next()) {
            const int r = it.r, q = it.c;
            const int idx = it.r * it.cols + it.c;
            sg[idx] = S[idx] + 0.5 * (double(GY[r * m + q]) + double(GY[q * m + r]));
        }
        for (Walk2 it(threadIdx.x, blockDim.x, rhs); it.r < m; it.next()) {
            const int r = it.r, q = it.c;
            const int idx = it.r * it.cols + it.c;
            rh[idx] = q == 0 ? double(Gv[r]) : double(Y[(q - 1) * m + r]);
        }
        __syncthreads();
    }
    cholesky(sg, m, m, ish);
    chol_solve(sg, m, m, rh, rhs, rhs);
    R* x2 = c.r<R>(c.ar.x2);
    R* X3 = c.r<R>(c.ar.X3);
    R* T = c.r<R>(c.ar.T);
    R* Z = c.r<R>(c.ar.Z);
    // X3 = P - sym(Y Zt), x2 = v - Y t (Zt, t in rh; sums in double); Y Zt
    // goes to T, free until the output products
    gemm_acc64<R, double, R>(T, n, Y, m, rh + 1, rhs, n, n, m, -1.0);
    gemm_acc64<R, double, R>(x2, 1, Y, m, rh, rhs, n, 1, m, -1.0, v, 1);
    sym_add<R>(X3, T, P, n);
    gemv<R>(mm, Aj, n, false, x2, n, n, bj);
    gemmR<R>(T, n, Aj, n, false, X3, n, false, n, n, n);
    gemmR<R>(Z, n, T, n, false, Aj, n, true, n, n, n);
    sym_add<R>(P, Z, Cj, n);
}

// b_k = c + K y_k, eta_k = w + W y_k (or b_1 = c1 + K1 y_1, eta_1 = 0) into xv
template <typename R>
__device__ __forceinline__ void build_fvec(const Ctx& c, const R* cst, const ConstLayout& CL, const R* yk, bool first) {
    const int n = c.n, ny = c.ny;
    R* bk = c.r<R>(c.ar.xv);
    R* ek = bk + n;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        R sb = first ? cst[CL.c1 + r] : cst[CL.c + r];
        R se = first ? R(0) : cst[CL.w + r];
#pragma unroll 4
        for (int q = 0; q < ny; ++q) {
            const R yq = yk[q];
            sb = fma(first ? cst[CL.K1 + r * ny + q] : cst[CL.K + r * ny + q], yq, sb);
            if (!first) se = fma(cst[CL.W + r * ny + q], yq, se);
        }
        bk[r] = sb;
        ek[r] = se;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// filter kernels
// ---------------------------------------------------------------------------
template <typename R, bool SEG, bool LDSA>
__global__ __launch_bounds__(kThreads) void k_large_filter_reduce(LargeArgs la) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int ish[72];   // flags; LU pivot rows
    const ScanArgs& a = la.s;
    Ctx c;
    make_ctx<LDSA>(c, la, lds, kArFRed);
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int n = c.n, n2 = n * n;
    const bool lowrank = a.ny < a.nx;
    const int64_t k0 = blockIdx.x * la.blen;
    const int64_t k1 = (k0 + la.blen < a.total) ? k0 + la.blen : a.total;
    R* acc = c.r<R>(c.ar.acc);
    const R* bk = c.r<R>(c.ar.xv);
    const R* ek = bk + n;
    const R* y = static_cast<const R*>(a.y);
    if (blockIdx.x == 0)   // models whose precompute failed (the precompute kernel has finished)
        for (int b = threadIdx.x; b < a.nmodels; b += blockDim.x)
            if (a.model_fail[b]) atomicMin(a.status, b);
    SeqL s = seq_at<SEG>(a, k0);
    for (int64_t k = k0; k < k1; ++k) {
        seq_fwd<SEG>(a, s, k);
        const int64_t moff = const_offset<SEG>(a, s.b, k);
        const R* cst = static_cast<const R*>(a.consts) + moff;
        const bool first = k == s.start;
        build_fvec<R>(c, cst, CL, y + k * a.ny, first);
        if (k == k0 || first) {
            // the element itself (a first step erases everything before it
            // in the f-part and leaves the g-part of the accumulator)
            const bool fresh_start = (k == k0);
            for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) {
                acc[c.fl.A + idx] = first ? R(0) : cst[CL.A + idx];
                acc[c.fl.C + idx] = first ? cst[CL.C1 + idx] : cst[CL.C + idx];
                if (fresh_start) acc[c.fl.J + idx] = first ? R(0) : cst[CL.J + idx];
            }
            for (int r = threadIdx.x; r < n; r += blockDim.x) {
                acc[c.fl.b + r] = bk[r];
                if (fresh_start) acc[c.fl.eta + r] = ek[r];
            }
            __syncthreads();
            continue;
        }
        // the combine updates the accumulator in place (every operand read
        // from it is consumed before the output block that overwrites it)
        if (lowrank)
            fcombine_fresh_wg<R>(c, acc, cst + CL.A, bk, cst + CL.C, ek, cst + CL.G, cst + CL.W,
                                 a.consts64 + moff + CL.S, acc, ish);
        else
            fcombine_wg<R>(c, acc, cst + CL.A, bk, cst + CL.C, ek, cst + CL.J, acc, ish);
    }
    R* dst = static_cast<R*>(la.agg[0]) + (size_t)blockIdx.x * c.fl.words;
    copy<R, R>(dst, acc, c.fl.words);
}

// out[i] = in[i - d] (x) in[i] (i >= d), else in[i]
template <typename R, bool SEG, bool LDSA>
__global__ __launch_bounds__(kThreads) void k_large_filter_ks(LargeArgs la, const void* in_, void* out_, int64_t d) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int ish[72];   // flags; LU pivot rows
    const ScanArgs& a = la.s;
    Ctx c;
    make_ctx<LDSA>(c, la, lds, kArFKs);
    const int64_t i = blockIdx.x;
    const int fw = c.fl.words;
    const R* in = static_cast<const R*>(in_);
    R* out = static_cast<R*>(out_) + (size_t)i * fw;
    const R* ej = in + (size_t)i * fw;
    if (i < d) {
        copy<R, R>(out, ej, fw);
        return;
    }
    const R* ei = in + (size_t)(i - d) * fw;
    fcombine_wg<R>(c, ei, ej + c.fl.A, ej + c.fl.b, ej + c.fl.C, ej + c.fl.eta, ej + c.fl.J, out, ish);
    if (SEG && all_zero<R>(ej + c.fl.A, c.n * c.n, ish)) {
        // the right operand starts a sequence: its f-part passes through
        // untouched (exactly what A_j = 0 gives, without 0 * NaN from the left)
        for (int idx = threadIdx.x; idx < c.n * c.n; idx += blockDim.x) {
            out[c.fl.A + idx] = R(0);
            out[c.fl.C + idx] = ej[c.fl.C + idx];
        }
        for (int r = threadIdx.x; r < c.n; r += blockDim.x) out[c.fl.b + r] = ej[c.fl.b + r];
        __syncthreads();
    }
}

template <typename R, bool SEG, bool LDSA>
__global__ __launch_bounds__(kThreads) void k_large_filter_down(LargeArgs la) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int ish[72];   // flags; LU pivot rows
    const ScanArgs& a = la.s;
    Ctx c;
    make_ctx<LDSA>(c, la, lds, kArFDown);
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int n = c.n, n2 = n * n;
    const bool lowrank = a.ny < a.nx;
    const int64_t blk = blockIdx.x;
    const int64_t k0 = blk * la.blen;
    const int64_t k1 = (k0 + la.blen < a.total) ? k0 + la.blen : a.total;
    R* X = c.r<R>(c.ar.mom);
    const R* bk = c.r<R>(c.ar.xv);
    const R* ek = bk + n;
    const R* y = static_cast<const R*>(a.y);
    R* mo = static_cast<R*>(a.m);
    R* Po = static_cast<R*>(a.P);
    if (blk > 0) {
        const R* prev = static_cast<const R*>(la.agg[la.final_buf]) + (size_t)(blk - 1) * c.fl.words;
        copy<R, R>(X, prev + c.fl.b, n);
        copy<R, R>(X + n, prev + c.fl.C, n2);
    } else {
        fill<R>(X, R(0), n + n2);
    }
    SeqL s = seq_at<SEG>(a, k0);
    for (int64_t k = k0; k < k1; ++k) {
        seq_fwd<SEG>(a, s, k);
        const int64_t moff = const_offset<SEG>(a, s.b, k);
        const R* cst = static_cast<const R*>(a.consts) + moff;
        const bool first = k == s.start;
        build_fvec<R>(c, cst, CL, y + k * a.ny, first);
        if (first) {
            copy<R, R>(X, bk, n);
            copy<R, R>(X + n, cst + CL.C1, n2);
        } else if (lowrank) {
            fcarry_fresh_wg<R>(c, X, cst + CL.A, bk, cst + CL.C, ek, cst + CL.G, a.consts64 + moff + CL.S, ish);
        } else {
            fcarry_wg<R>(c, X, cst + CL.A, bk, cst + CL.C, ek, cst + CL.J, ish);
        }
        for (int r = threadIdx.x; r < n; r += blockDim.x) mo[k * n + r] = X[r];
        for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) Po[k * n2 + idx] = X[n + idx];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// smoother
// ---------------------------------------------------------------------------
// Lemma 3 element of step k (not last) from moments (m, P) at `mom`, into e:
// E = P F^T (F P F^T + Q)^-1, g = m - E (F m + u), L = sym(P - E F P)
template <typename R>
__device__ __forceinline__ void build_selem_wg(const Ctx& c, const R* cst, const ConstLayout& CL, const R* m, const R* P, R* e,
                               int* status, int b, int* ish) {
    const int n = c.n;
    const R* F = cst + CL.F;
    R* V = c.r<R>(c.ar.T);
    R* Z = c.r<R>(c.ar.Z);
    double* S = c.d<R>(c.ar.aug);          // [n x n] then E^T as [n x n] after it
    double* Et = S + n * n;
    gemmR<R>(V, n, F, n, false, P, n, false, n, n, n);                 // F P
    gemmR<R>(Z, n, V, n, false, F, n, true, n, n, n);                  // F P F^T
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        S[idx] = 0.5 * (double(Z[r * n + q]) + double(Z[q * n + r])) + double(cst[CL.Q + idx]);
        Et[idx] = double(V[idx]);
    }
    __syncthreads();
    const bool ok = cholesky(S, n, n, ish);
    if (!ok && threadIdx.x == 0) atomicMin(status, b);
    chol_solve(S, n, n, Et, n, n);                                        // (F P F^T + Q)^-1 F P = E^T
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        e[c.sl.E + idx] = R(Et[q * n + r]);
    }
    __syncthreads();
    R* p = c.r<R>(c.ar.x2);
    gemv<R>(p, F, n, false, m, n, n, cst + CL.u);                        // F m + u
    gemv<R>(e + c.sl.g, e + c.sl.E, n, false, p, n, n, m, R(-1));        // m - E p
    gemmR<R>(Z, n, e + c.sl.E, n, false, V, n, false, n, n, n);         // E F P
    for (Walk2 it(threadIdx.x, blockDim.x, n); it.r < n; it.next()) {
        const int r = it.r, q = it.c;
        const int idx = it.r * it.cols + it.c;
        e[c.sl.L + idx] = R(double(P[idx]) - 0.5 * (double(Z[r * n + q]) + double(Z[q * n + r])));
    }
    __syncthreads();
}

// out = ei (x) ej (Lemma 4)
template <typename R>
__device__ __forceinline__ void scombine_wg(const Ctx& c, const R* ei, const R* ej, R* out) {
    const int n = c.n;
    R* T = c.r<R>(c.ar.T);
    R* Z = c.r<R>(c.ar.Z);
    gemmR<R>(out + c.sl.E, n, ei + c.sl.E, n, false, ej + c.sl.E, n, false, n, n, n);
    gemv<R>(out + c.sl.g, ei + c.sl.E, n, false, ej + c.sl.g, n, n, ei + c.sl.g);
    gemmR<R>(T, n, ei + c.sl.E, n, false, ej + c.sl.L, n, false, n, n, n);
    gemmR<R>(Z, n, T, n, false, ei + c.sl.E, n, true, n, n, n);
    sym_add<R>(out + c.sl.L, Z, ei + c.sl.L, n);
}

// moments Y (suffix with E = 0) <- ei (x) Y
template <typename R>
__device__ __forceinline__ void scarry_wg(const Ctx& c, const R* ei, R* Y) {
    const int n = c.n;
    R* T = c.r<R>(c.ar.T);
    R* Z = c.r<R>(c.ar.Z);
    R* g = c.r<R>(c.ar.x2);
    gemv<R>(g, ei + c.sl.E, n, false, Y, n, n, ei + c.sl.g);
    gemmR<R>(T, n, ei + c.sl.E, n, false, Y + n, n, false, n, n, n);
    gemmR<R>(Z, n, T, n, false, ei + c.sl.E, n, true, n, n, n);
    copy<R, R>(Y, g, n);
    sym_add<R>(Y + n, Z, ei + c.sl.L, n);
}

template <typename R>
__device__ __forceinline__ void load_moments(const Ctx& c, const ScanArgs& a, int64_t k, R* mom) {
    const int n = c.n;
    const R* m = static_cast<const R*>(a.m);
    const R* P = static_cast<const R*>(a.P);
    for (int r = threadIdx.x; r < n; r += blockDim.x) mom[r] = m[k * n + r];
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) mom[n + idx] = P[k * n * n + idx];
    __syncthreads();
}

template <typename R, bool SEG, bool LDSA>
__global__ __launch_bounds__(kThreads) void k_large_smoother_reduce(LargeArgs la) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int ish[72];   // flags; LU pivot rows
    const ScanArgs& a = la.s;
    Ctx c;
    make_ctx<LDSA>(c, la, lds, kArSRed);
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int n = c.n, n2 = n * n;
    const int64_t k0 = blockIdx.x * la.blen;
    const int64_t k1 = (k0 + la.blen < a.total) ? k0 + la.blen : a.total;
    R* acc = c.r<R>(c.ar.acc);
    R* e = c.r<R>(c.ar.out);                 // element of step k
    R* tmp = c.r<R>(c.ar.sel);
    R* mom = c.r<R>(c.ar.mom);
    SeqL s = seq_at<SEG>(a, k0);
    for (int64_t k = k0; k < k1; ++k) {
        seq_fwd<SEG>(a, s, k);
        const R* cst = static_cast<const R*>(a.consts) + const_offset<SEG>(a, s.b, k);
        load_moments<R>(c, a, k, mom);
        const bool last = k == s.end - 1;
        if (last) {
            fill<R>(e + c.sl.E, R(0), n2);
            copy<R, R>(e + c.sl.g, mom, n + n2);    // g = m, L = P (contiguous)
        } else {
            build_selem_wg<R>(c, cst, CL, mom, mom + n, e, a.status, s.b, ish);
        }
        if (k == k0) {
            copy<R, R>(acc, e, c.sl.words);
        } else {
            scombine_wg<R>(c, acc, e, tmp);
            // an accumulator ending a sequence (E = 0) passes through; else
            // the result becomes the accumulator
            if (!(SEG && all_zero<R>(acc + c.sl.E, n2, ish))) {
                R* t = acc;
                acc = tmp;
                tmp = t;
            }
        }
    }
    R* dst = static_cast<R*>(la.agg[0]) + (size_t)blockIdx.x * c.sl.words;
    copy<R, R>(dst, acc, c.sl.words);
}

// out[i] = in[i] (x) in[i + d] (i + d < n), else in[i]
template <typename R, bool SEG, bool LDSA>
__global__ __launch_bounds__(kThreads) void k_large_smoother_ks(LargeArgs la, const void* in_, void* out_, int64_t d,
                                                               int64_t nb) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int ish[72];   // flags; LU pivot rows
    const ScanArgs& a = la.s;
    Ctx c;
    make_ctx<LDSA>(c, la, lds, kArSKs);
    const int64_t i = blockIdx.x;
    const int sw = c.sl.words;
    const R* in = static_cast<const R*>(in_);
    R* out = static_cast<R*>(out_) + (size_t)i * sw;
    const R* ei = in + (size_t)i * sw;
    if (i + d >= nb || (SEG && all_zero<R>(ei + c.sl.E, c.n * c.n, ish))) {
        copy<R, R>(out, ei, sw);
        return;
    }
    scombine_wg<R>(c, ei, in + (size_t)(i + d) * sw, out);
}

template <typename R, bool SEG, bool LDSA>
__global__ __launch_bounds__(kThreads) void k_large_smoother_down(LargeArgs la) {
    extern __shared__ __align__(16) char lds[];
    __shared__ int ish[72];   // flags; LU pivot rows
    const ScanArgs& a = la.s;
    Ctx c;
    make_ctx<LDSA>(c, la, lds, kArSDown);
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int n = c.n, n2 = n * n;
    const int64_t blk = blockIdx.x;
    const int64_t k0 = blk * la.blen;
    const int64_t k1 = (k0 + la.blen < a.total) ? k0 + la.blen : a.total;
    if (k0 >= k1) return;
    R* Y = c.r<R>(c.ar.acc);
    R* e = c.r<R>(c.ar.out);
    R* mso = static_cast<R*>(a.ms);
    R* Pso = static_cast<R*>(a.Ps);
    if (blk + 1 < la.nblocks) {
        const R* nxt = static_cast<const R*>(la.agg[la.final_buf]) + (size_t)(blk + 1) * c.sl.words;
        copy<R, R>(Y, nxt + c.sl.g, n + n2);       // g, L contiguous
    } else {
        fill<R>(Y, R(0), n + n2);
    }
    SeqL s = seq_at<SEG>(a, k1 - 1);
    for (int64_t k = k1 - 1; k >= k0; --k) {
        seq_bwd<SEG>(a, s, k);
        const R* cst = static_cast<const R*>(a.consts) + const_offset<SEG>(a, s.b, k);
        // the filtered moments of step k are read where the filter wrote them
        const R* mk = static_cast<const R*>(a.m) + k * n;
        const R* Pk = static_cast<const R*>(a.P) + k * n2;
        if (k == s.end - 1) {
            copy<R, R>(Y, mk, n);
            copy<R, R>(Y + n, Pk, n2);
        } else {
            build_selem_wg<R>(c, cst, CL, mk, Pk, e, a.status, s.b, ish);
            scarry_wg<R>(c, e, Y);
        }
        for (int r = threadIdx.x; r < n; r += blockDim.x) mso[k * n + r] = Y[r];
        for (int idx = threadIdx.x; idx < n2; idx += blockDim.x) Pso[k * n2 + idx] = Y[n + idx];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// workgroup size: one wave for nx <= 16 (barriers are then nearly free and
// the products still give every lane work), two for nx <= 32, four above
// (eight where the arena's LDS keeps a second workgroup off the unit: see
// run_large)
__host__ __device__ inline int large_threads(int nx) { return nx <= 16 ? 64 : (nx <= 32 ? 128 : 256); }

// arenas up to this size live in LDS (gfx950 addresses 160 KB of LDS per
// workgroup; the kernels' static scratch is a few bytes)
constexpr size_t kMaxLdsArena = 160 * 1024 - 512;

template <typename K>
hipError_t allow_lds(K kernel, size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <typename R>
size_t kind_lds(const LargeArgs& la, int kind) {
    return ((la.slot_mask >> kind) & 1) ? 0 : arena_bytes<R>(la.s.nx, la.s.ny, kind);
}

template <typename R, bool SEG>
hipError_t run_large(LargeArgs la, bool smoother, hipStream_t s) {
    const dim3 grid((unsigned)la.nblocks);
    const auto in_lds = [&](int kind) { return ((la.slot_mask >> kind) & 1) == 0; };
    // above nx = 32, a kernel whose LDS arena leaves room for only one
    // workgroup per compute unit runs eight waves instead of four
    const auto block_of = [&](int kind) {
        if (la.s.nx > 32 && in_lds(kind) && kind_lds<R>(la, kind) > kMaxLdsArena / 2) return dim3(kThreads);
        return dim3(large_threads(la.s.nx));
    };
    hipError_t e;
    if (!smoother) {
        const size_t l_red = kind_lds<R>(la, kArFRed), l_ks = kind_lds<R>(la, kArFKs),
                     l_down = kind_lds<R>(la, kArFDown);
        auto kred = in_lds(kArFRed) ? k_large_filter_reduce<R, SEG, true> : k_large_filter_reduce<R, SEG, false>;
        auto kks = in_lds(kArFKs) ? k_large_filter_ks<R, SEG, true> : k_large_filter_ks<R, SEG, false>;
        auto kdown = in_lds(kArFDown) ? k_large_filter_down<R, SEG, true> : k_large_filter_down<R, SEG, false>;
        if ((e = allow_lds(kred, l_red)) != hipSuccess) return e;
        if ((e = allow_lds(kks, l_ks)) != hipSuccess) return e;
        if ((e = allow_lds(kdown, l_down)) != hipSuccess) return e;
        prof_begin("k_large_filter_reduce", s);
        hipLaunchKernelGGL(kred, grid, block_of(kArFRed), l_red, s, la);
        prof_end(s);
        int cur = 0;
        for (int64_t d = 1; d < la.nblocks; d <<= 1) {
            prof_begin("k_large_filter_ks", s);
            hipLaunchKernelGGL(kks, grid, block_of(kArFKs), l_ks, s, la, la.agg[cur], la.agg[cur ^ 1], d);
            prof_end(s);
            cur ^= 1;
        }
        la.final_buf = cur;
        prof_begin("k_large_filter_down", s);
        hipLaunchKernelGGL(kdown, grid, block_of(kArFDown), l_down, s, la);
        prof_end(s);
    } else {
        const size_t l_red = kind_lds<R>(la, kArSRed), l_ks = kind_lds<R>(la, kArSKs),
                     l_down = kind_lds<R>(la, kArSDown);
        auto kred = in_lds(kArSRed) ? k_large_smoother_reduce<R, SEG, true> : k_large_smoother_reduce<R, SEG, false>;
        auto kks = in_lds(kArSKs) ? k_large_smoother_ks<R, SEG, true> : k_large_smoother_ks<R, SEG, false>;
        auto kdown = in_lds(kArSDown) ? k_large_smoother_down<R, SEG, true> : k_large_smoother_down<R, SEG, false>;
        if ((e = allow_lds(kred, l_red)) != hipSuccess) return e;
        if ((e = allow_lds(kks, l_ks)) != hipSuccess) return e;
        if ((e = allow_lds(kdown, l_down)) != hipSuccess) return e;
        prof_begin("k_large_smoother_reduce", s);
        hipLaunchKernelGGL(kred, grid, block_of(kArSRed), l_red, s, la);
        prof_end(s);
        int cur = 0;
        for (int64_t d = 1; d < la.nblocks; d <<= 1) {
            prof_begin("k_large_smoother_ks", s);
            hipLaunchKernelGGL(kks, grid, block_of(kArSKs), l_ks, s, la, la.agg[cur], la.agg[cur ^ 1], d, la.nblocks);
            prof_end(s);
            cur ^= 1;
        }
        la.final_buf = cur;
        prof_begin("k_large_smoother_down", s);
        hipLaunchKernelGGL(kdown, grid, block_of(kArSDown), l_down, s, la);
        prof_end(s);
    }
    return hipGetLastError();
}

}  // namespace lg
}  // namespace pks
