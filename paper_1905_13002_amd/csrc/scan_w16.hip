// scan_w16.hip -- the filtering and smoothing scans of time-invariant models
// (one sequence or packed sequences) for 5 <= nx <= 16 and ny <= 16, every
// element held in the registers of one wavefront; also the model constants
// and the likelihood factors of one sequence at these sizes.
//
// Register layout of a 16 x 16 matrix X (smaller dimensions padded with
// zeros): lane l = 16 lk + li holds X(4 v + lk, li) in component v of an
// f64x4 -- the accumulator layout of v_mfma_f64_16x16x4f64.  In that layout
// component s of the tile of L^T and component s of the tile of R are
// exactly the A and B operands of the s-th K-slice of the product L R, so a
// product is four MFMAs with no data movement:
//     L R = mm(tile(L^T), tile(R)),   (L R)^T = mm(tile(R), tile(L^T)).
// Every matrix is therefore kept in the form its consumers read (C, J, L, P
// are symmetric, so their tiles serve both ways); a transpose, when one is
// needed, is a product with the identity.  A vector x is held replicated
// across the columns (lane: x(4 v + lk)), so a matrix-vector product is an
// MFMA product as well.
//
// The time axis is cut into blocks (the block-level elements of Section
// III-C), one wavefront per block:
//   reduce : fold the block's single-step elements (Lemma 1 / Lemma 3) into
//            its block element with the operators of Lemma 2 / Lemma 4,
//   scan   : Kogge-Stone over the block elements, ceil(log2 blocks) launches
//            (filter: out[i] = in[i - d] (x) in[i]; smoother: in[i] (x) in[i + d]),
//   down   : re-fold the block from the moments before it (after it, for the
//            smoother), writing the filtered (smoothed) moments.
// The solves are 16 x 16 inverses by Gauss-Jordan elimination in the same
// register layout: with partial pivoting for I + C_i J_j (Lemma 2) and its
// carry form I + P J (pivot rows chosen in place, the rows of the inverse
// gathered at the end), without pivoting for the positive definite
// F P F^T + Q of Lemma 3 (a non-positive pivot there is the numeric failure).
// All arithmetic is FP64 in both precisions (the constants come from the
// double copy the precompute writes); the precision sets the type of y and of
// the moments in memory.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>

#include "pks_internal.h"

namespace pks {
namespace w16 {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 256;                    // doubles of one tile in memory (lane-major)
// block element records (doubles): filter A, C, J tiles then b, eta;
// smoother E, L tiles then g
constexpr int kFA = 0, kFC = kTile, kFJ = 2 * kTile, kFb = 3 * kTile, kFeta = 3 * kTile + 16, kFRec = 3 * kTile + 32;
constexpr int kSE = 0, kSL = kTile, kSg = 2 * kTile, kSRec = 2 * kTile + 16;
constexpr int kStage = 16 * 17;               // LDS doubles per wave: the row gather of a pivoted inverse
constexpr int kThreads = 64;
constexpr int64_t kMaxBlocks = 2048;

struct W16Args {
    ScanArgs s;
    int64_t blen, nblocks;
    double* agg[2];          // ping-pong block elements [nblocks][kFRec]
    int final_buf;
    // smoothing elements of every step [total][kSRec], written by the filter
    // down-sweep of a combined filter + smoother call and read by the
    // smoother kernels instead of rebuilding them (nullptr: rebuilt)
    double* elem;
    int pivot_always;        // 1: the scan's combines skip the unpivoted attempt (PKS_PIVOTED_INVERSE=1)
};

__device__ __forceinline__ int lane_i() { return threadIdx.x & 15; }          // column
__device__ __forceinline__ int lane_k() { return (threadIdx.x >> 4) & 3; }    // row within a group of four

__device__ __forceinline__ f64x4 zero4() { return f64x4{0.0, 0.0, 0.0, 0.0}; }

__device__ __forceinline__ f64x4 eye() {
    const int li = lane_i(), lk = lane_k();
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = (4 * v + lk == li) ? 1.0 : 0.0;
    return t;
}

// L R + acc, given the tile of L^T and the tile of R.  KS: the K-slices of four
// that hold the contraction (entries beyond 4 KS of L's columns or R's rows
// are zero), so a contraction over ny <= 8 takes two MFMAs; a compile-time
// count, since a branch around each MFMA costs more than the MFMA
template <int KS = 4>
__device__ __forceinline__ f64x4 mm(const f64x4& lt, const f64x4& r, f64x4 acc) {
#pragma unroll
    for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(lt[s], r[s], acc, 0, 0, 0);
    return acc;
}
template <int KS = 4>
__device__ __forceinline__ f64x4 mm(const f64x4& lt, const f64x4& r) { return mm<KS>(lt, r, zero4()); }

// (X + X^T) / 2 + add, given the tiles of X and X^T
__device__ __forceinline__ f64x4 sym(const f64x4& x, const f64x4& xt, const f64x4& add) {
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = 0.5 * (x[v] + xt[v]) + add[v];
    return t;
}

// ---------------------------------------------------------------------------
// memory <-> registers
// ---------------------------------------------------------------------------
// tile of the rows x cols matrix X (row stride ld), zero outside it
template <typename T>
__device__ __forceinline__ f64x4 load_tile(const T* X, int rows, int cols, int ld) {
    const int li = lane_i(), lk = lane_k();
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lk;
        t[v] = (r < rows && li < cols) ? double(X[r * ld + li]) : 0.0;
    }
    return t;
}
// tile of X^T for the rows x cols matrix X
template <typename T>
__device__ __forceinline__ f64x4 load_tile_t(const T* X, int rows, int cols, int ld) {
    const int li = lane_i(), lk = lane_k();
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lk;
        t[v] = (li < rows && r < cols) ? double(X[li * ld + r]) : 0.0;
    }
    return t;
}
// replicated vector x[0..n), zero beyond
template <typename T>
__device__ __forceinline__ f64x4 load_vec(const T* x, int n) {
    const int lk = lane_k();
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lk;
        t[v] = r < n ? double(x[r]) : 0.0;
    }
    return t;
}
template <typename T>
__device__ __forceinline__ void store_tile(T* X, const f64x4& t, int n) {
    const int li = lane_i(), lk = lane_k();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lk;
        if (r < n && li < n) X[r * n + li] = T(t[v]);
    }
}
template <typename T>
__device__ __forceinline__ void store_vec(T* x, const f64x4& t, int n) {
    const int li = lane_i(), lk = lane_k();
    if (li != 0) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lk;
        if (r < n) x[r] = T(t[v]);
    }
}
// records: tiles lane-major (each lane's four doubles contiguous)
__device__ __forceinline__ void put_tile(double* p, const f64x4& t) {
    reinterpret_cast<f64x4*>(p)[threadIdx.x & 63] = t;
}
__device__ __forceinline__ f64x4 get_tile(const double* p) {
    return reinterpret_cast<const f64x4*>(p)[threadIdx.x & 63];
}

__device__ __forceinline__ double readlane_d(double x, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane k of the lane's own row of 16 (DPP row_newbcast; k a constant after unrolling)
__device__ __forceinline__ unsigned newbcast(unsigned x, int k) {
    switch (k) {
#define PKS_NB(K) case K: return (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x150 + K, 0xf, 0xf, false);
        PKS_NB(0) PKS_NB(1) PKS_NB(2) PKS_NB(3) PKS_NB(4) PKS_NB(5) PKS_NB(6) PKS_NB(7)
        PKS_NB(8) PKS_NB(9) PKS_NB(10) PKS_NB(11) PKS_NB(12) PKS_NB(13) PKS_NB(14) PKS_NB(15)
#undef PKS_NB
        default: return x;
    }
}
__device__ __forceinline__ double col_bcast(double x, int k) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = newbcast((unsigned)u, k), hi = newbcast((unsigned)(u >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// the value of lane 16 g + (lane % 16), g uniform: permlane16_swap of x with
// itself gives rows (0,0,2,2) and (1,1,3,3), permlane32_swap of one of those
// with itself its lower or upper half in both halves
__device__ __forceinline__ unsigned rowbcast(unsigned x, int g) {
    const auto q = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    const unsigned t = (g & 1) ? q[1] : q[0];
    const auto r = __builtin_amdgcn_permlane32_swap(t, t, false, false);
    return (g & 2) ? r[1] : r[0];
}
__device__ __forceinline__ double row_bcast(double x, int g) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = rowbcast((unsigned)u, g), hi = rowbcast((unsigned)(u >> 32), g);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// 1 / x: the hardware estimate refined by two Newton-Raphson steps
// (r <- r + r (1 - x r)), within an ulp or two of the quotient
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double pick(const f64x4& t, int q) {
    return q == 0 ? t[0] : (q == 1 ? t[1] : (q == 2 ? t[2] : t[3]));
}

// the tile of X^T through the wave's LDS stage (exact; keeps the matrix cores
// free for products)
__device__ __forceinline__ f64x4 tr(const f64x4& x, double* st) {
    const int li = lane_i(), lk = lane_k();
#pragma unroll
    for (int v = 0; v < 4; ++v) st[(4 * v + lk) * 17 + li] = x[v];
    wave_sync_lds();
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = st[li * 17 + 4 * v + lk];
    wave_sync_lds();
    return t;
}
// (X + X^T) / 2 + add
__device__ __forceinline__ f64x4 symt(const f64x4& x, const f64x4& add, double* st) { return sym(x, tr(x, st), add); }

// ---------------------------------------------------------------------------
// Inverses by Gauss-Jordan elimination in the register layout.  The pivot's
// column reaches the lanes of each row of 16 by a DPP broadcast, the pivot row
// reaches the other rows of 16 by the permlane swaps.  Only the first n pivots
// are taken: the matrices are padded with the identity, on which the
// remaining steps change nothing.
// ---------------------------------------------------------------------------
// Symmetric positive definite a: the pivots are the diagonal, in order, and
// the inverse is formed in place.  `ok` is cleared by a pivot that is not
// positive (the matrix is not positive definite) or not finite.
// det (optional): the product of the pivots as a mantissa product and an
// exponent sum (the pivots are the diagonal of the LDL^T factorisation)
struct Det {
    double mant = 1.0;
    int exp = 0;
};
template <bool SPD = true>
__device__ __forceinline__ f64x4 inv_diag(f64x4 a, int n, bool& ok, Det* det = nullptr) {
    const int li = lane_i(), lk = lane_k();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < n) {        // a guard, not an exit: the loop stays fully unrolled
            const int q = k >> 2, g = k & 3;
            const double pv = readlane_d(a[q], (g << 4) | k);          // a(k, k)
            double ck[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) ck[v] = col_bcast(a[v], k);    // a(4 v + lk, k)
            const double rk = row_bcast(a[q], g);                      // a(k, li)
            ok = ok && (SPD ? pv > 0.0 : pv != 0.0) && isfinite(pv);
            if (det) {
                int ex;
                det->mant *= frexp(pv, &ex);
                det->exp += ex;
            }
            const double r = recip(pv);
            const double rr = rk * r;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double f = ck[v] * r;
                if (4 * v + lk == k) a[v] = li == k ? r : rr;           // the pivot row
                else a[v] = li == k ? -f : fma(-f, rk, a[v]);
            }
        }
    }
    return a;
}

__device__ __forceinline__ f64x4 inv_spd(const f64x4& a, int n, bool& ok) { return inv_diag<true>(a, n, ok); }

// General a: partial pivoting without row exchanges (the pivot of column k is
// the entry of largest magnitude among the rows not used yet, lower rows
// winning ties), elimination on [a | I]; row k of the inverse is then row p_k
// of the right half, gathered through the LDS stage.  `ok` is cleared by a
// zero or non-finite pivot.
__device__ __forceinline__ f64x4 inv_piv(f64x4 a, int n, double* st, bool& ok) {
    const int li = lane_i(), lk = lane_k();
    f64x4 b = eye();
    unsigned used = 0;
    unsigned long long perm = 0xFEDCBA9876543210ull;      // p_k = k beyond n
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k >= n) continue;
        double ck[4];
        unsigned best = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ck[v] = col_bcast(a[v], k);                          // a(4 v + lk, k)
            const int row = 4 * v + lk;
            // |entry| as float with the low mantissa bits dropped, then the row
            const unsigned bits = __float_as_uint((float)fabs(ck[v]));
            const unsigned key = ((used >> row) & 1u) ? 0u : (((bits >> 4) << 5) | 16u | (unsigned)(15 - row));
            best = best > key ? best : key;
        }
        const unsigned g0 = (unsigned)__builtin_amdgcn_readlane((int)best, 0);
        const unsigned g1 = (unsigned)__builtin_amdgcn_readlane((int)best, 16);
        const unsigned g2 = (unsigned)__builtin_amdgcn_readlane((int)best, 32);
        const unsigned g3 = (unsigned)__builtin_amdgcn_readlane((int)best, 48);
        const unsigned m01 = g0 > g1 ? g0 : g1, m23 = g2 > g3 ? g2 : g3;
        const unsigned key = m01 > m23 ? m01 : m23;
        const int p = 15 - (int)(key & 15u);
        used |= 1u << p;
        perm = (perm & ~(15ull << (4 * k))) | ((unsigned long long)p << (4 * k));
        const int q = p >> 2, g = p & 3;
        const double pv = readlane_d(pick(f64x4{ck[0], ck[1], ck[2], ck[3]}, q), g << 4);   // a(p, k)
        const double ra = row_bcast(pick(a, q), g);              // row p of a and of b
        const double rb = row_bcast(pick(b, q), g);
        ok = ok && pv != 0.0 && isfinite(pv);
        const double r = recip(pv);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool prow = 4 * v + lk == p;
            const double f = ck[v] * r;
            a[v] = prow ? ra * r : fma(-f, ra, a[v]);
            b[v] = prow ? rb * r : fma(-f, rb, b[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) st[(4 * v + lk) * 17 + li] = b[v];
    wave_sync_lds();
    f64x4 out;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int p = (int)((perm >> (4 * (4 * v + lk))) & 15ull);
        out[v] = st[p * 17 + li];
    }
    wave_sync_lds();
    return out;
}

// ---------------------------------------------------------------------------
// operators (KY: K-slices of a contraction over ny; contractions over nx take all four)
// ---------------------------------------------------------------------------
struct FE {                 // filtering element (Lemma 1 / 2): tiles of A, C, J; b, eta
    f64x4 A, b, C, eta, J;
};

// constants of the filter kernels (double copy): tiles of A^T, C, J, K^T, W^T,
// G^T and S (the identity beyond ny), replicated c and w
struct FConst {
    f64x4 AT, C, J, KT, WT, GT, S, c, w;
    int n, ny;
};

// Output half of Lemma 2, given X1 = M^-1 A_i, x2 = M^-1 (b_i + C_i eta_j) and
// X3 = M^-1 C_i (M = I + C_i J_j) and the tile of A_j^T:
//   A = A_j X1, b = A_j x2 + b_j, C = A_j X3 A_j^T + C_j,
//   eta = X1^T (eta_j - J_j b_i) + eta_i, J = X1^T J_j A_i + J_i
__device__ __forceinline__ void fout(FE& e, const f64x4& X1, const f64x4& x2, const f64x4& X3, const f64x4& AjT,
                                     const f64x4& bj, const f64x4& Cj, const f64x4& etaj, const f64x4& Jj, double* st) {
    const f64x4 w = mm(-Jj, e.b, etaj);
    const f64x4 JA = mm(Jj, e.A);
    e.A = mm(AjT, X1);
    e.b = mm(AjT, x2, bj);
    const f64x4 U = mm(X3, AjT);                     // X3^T A_j^T
    e.C = symt(mm(AjT, U), Cj, st);                 // A_j sym(X3) A_j^T + C_j
    e.eta = mm(X1, w, e.eta);
    e.J = symt(mm(X1, JA), e.J, st);
}

// e <- e (x) (A_j, b_j, C_j, eta_j, J_j), Lemma 2, for two block elements: the
// inverse of M^T = I + J_j C_i (its tile is M^-1 as a left factor) with
// pivoting
// The inverse is first formed without pivoting and kept when its residual
// |M^T (M^T)^-1 - I| is below 1e-11 in every entry (the result is then as
// accurate as a pivoted one); otherwise it is formed again with pivoting.
__device__ __forceinline__ void fcombine(FE& e, const f64x4& AjT, const f64x4& bj, const f64x4& Cj, const f64x4& etaj,
                                         const f64x4& Jj, const f64x4& I, double* st, int n, bool pivot_always) {
    bool ok = !pivot_always;
    const f64x4 MT = mm(Jj, e.C, I);
    f64x4 NT = I;
    double dev = 1.0;
    if (ok) {
        NT = inv_diag<false>(MT, n, ok);
        const f64x4 R = mm(mm(e.C, Jj, I), NT);          // M^T (M^T)^-1 (the tile of M as left operand)
        dev = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) dev = fmax(dev, fabs(R[v] - I[v]));
#pragma unroll
        for (int mk = 1; mk < 64; mk <<= 1) dev = fmax(dev, __shfl_xor(dev, mk, 64));
    }
    if (!(ok && dev <= 1e-11)) NT = inv_piv(MT, n, st, ok);
    const f64x4 v = mm(e.C, etaj, e.b);               // b_i + C_i eta_j
    fout(e, mm(NT, e.A), mm(NT, v), mm(NT, e.C), AjT, bj, Cj, etaj, Jj, st);
}

// e <- e (x) a_j for a single step j > 1, where J_j = G^T S^-1 G (G = H F,
// S = H Q H^T + R): M^-1 = I - K G with K = C_i G^T Sigma^-1 and the ny x ny
// positive definite Sigma = S + G C_i G^T, so
//   X1 = A_i - K (G A_i), x2 = v - K (G v), X3 = C_i - K (G C_i).
// Y = X G^T, v = X eta + c, G Y and G v.  PK (ny < 16): the last column of
// G^T's tile is free, so eta rides there (and c in the same column of the
// accumulator) -- X (G^T | eta) + (0 | c) is one product, G (Y | v) another --
// and the column is then broadcast along the rows (DPP) and cleared.
template <bool PK>
__device__ __forceinline__ void yv(const f64x4& X, const FConst& f, const f64x4& eta, const f64x4& c, f64x4& Y,
                                   f64x4& v, f64x4& GY, f64x4& Gv) {
    if constexpr (PK) {
        const bool last = lane_i() == 15;
        f64x4 GTe, c15;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            GTe[q] = last ? eta[q] : f.GT[q];
            c15[q] = last ? c[q] : 0.0;
        }
        const f64x4 Yx = mm(X, GTe, c15);
        const f64x4 GYx = mm(f.GT, Yx);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = col_bcast(Yx[q], 15);
            Y[q] = last ? 0.0 : Yx[q];
            Gv[q] = col_bcast(GYx[q], 15);
            GY[q] = last ? 0.0 : GYx[q];
        }
    } else {
        Y = mm(X, f.GT);
        v = mm(X, eta, c);
        GY = mm(f.GT, Y);
        Gv = mm(f.GT, v);
    }
}

template <int KY, bool PK>
__device__ __forceinline__ void fcombine_fresh(FE& e, const FConst& f, const f64x4& bj, const f64x4& etaj, double* st) {
    f64x4 Y, v, GY, Gv;
    yv<PK>(e.C, f, etaj, e.b, Y, v, GY, Gv);          // C_i G^T, b_i + C_i eta_j, G C_i G^T, G v
    const f64x4 YT = tr(Y, st);                      // G C_i
    bool ok = true;
    const f64x4 Z = inv_spd(symt(GY, f.S, st), f.ny, ok);
    const f64x4 nKT = -mm<KY>(Z, YT);                // tile of -K^T
    const f64x4 X1 = mm<KY>(nKT, mm(f.GT, e.A), e.A);
    const f64x4 x2 = mm<KY>(nKT, Gv, v);
    const f64x4 X3 = mm<KY>(nKT, YT, e.C);
    fout(e, X1, x2, X3, f.AT, bj, f.C, etaj, f.J, st);
}

// filtered moments (m, P) <- (m, P) (x) a_j for a single step j > 1 (the
// prefix element has A = 0): with K = P G^T Sigma^-1, Sigma = S + G P G^T,
//   m = A_j (v - K G v) + b_j (v = m + P eta_j), P = A_j (P - K G P) A_j^T + C_j
template <int KY, bool PK>
__device__ __forceinline__ void fcarry_fresh(f64x4& m, f64x4& P, const FConst& f, const f64x4& bj, const f64x4& etaj,
                                             double* st) {
    f64x4 Y, v, GY, Gv;
    yv<PK>(P, f, etaj, m, Y, v, GY, Gv);              // P G^T, m + P eta_j, G P G^T, G v
    const f64x4 YT = tr(Y, st);                      // G P
    bool ok = true;
    const f64x4 Z = inv_spd(symt(GY, f.S, st), f.ny, ok);
    const f64x4 nKT = -mm<KY>(Z, YT);
    const f64x4 x2 = mm<KY>(nKT, Gv, v);
    const f64x4 X3 = mm<KY>(nKT, YT, P);
    m = mm(f.AT, x2, bj);
    const f64x4 U = mm(X3, f.AT);
    P = symt(mm(f.AT, U), f.C, st);
}

// constants of the smoother kernels: tiles of F^T and Q (the identity beyond
// nx), replicated u
struct SConst {
    f64x4 FT, Q, u;
    int n;
};

// smoothing element of step k (Lemma 3) from the filtered (m, P):
//   E = P F^T (F P F^T + Q)^-1, g = m - E (F m + u), L = P - E F P,
// returned as the tile of E^T, g and L
__device__ __forceinline__ void selem(const f64x4& m, const f64x4& P, const SConst& c, double* st, bool& ok, f64x4& ET,
                                      f64x4& g, f64x4& L) {

    const f64x4 FP = mm(c.FT, P);
    const f64x4 PFT = tr(FP, st);                     // P F^T
    const f64x4 Z = inv_spd(symt(mm(c.FT, PFT), c.Q, st), c.n, ok);
    ET = mm(Z, FP);                                  // (F P F^T + Q)^-1 F P
    g = mm(-ET, mm(c.FT, m, c.u), m);
    const f64x4 EFP = mm(ET, FP), EFPt = tr(EFP, st);
#pragma unroll
    for (int v = 0; v < 4; ++v) L[v] = P[v] - 0.5 * (EFP[v] + EFPt[v]);
}

// (E, g, L) <- e_k (x) (E, g, L), Lemma 4, e_k given by the tile of E_k^T:
//   E = E_k E, g = E_k g + g_k, L = E_k L E_k^T + L_k
__device__ __forceinline__ void sfold(f64x4& E, f64x4& g, f64x4& L, const f64x4& EkT, const f64x4& gk,
                                      const f64x4& Lk, double* st) {
    E = mm(EkT, E);
    g = mm(EkT, g, gk);
    const f64x4 T1T = mm(L, EkT);                    // (E_k L)^T
    L = symt(mm(T1T, EkT), Lk, st);
}
// smoothed moments (m, P) <- e_k (x) (m, P) (the suffix element has E = 0)
__device__ __forceinline__ void scarry(f64x4& m, f64x4& P, const f64x4& EkT, const f64x4& gk, const f64x4& Lk,
                                       double* st) {
    m = mm(EkT, m, gk);
    const f64x4 T1T = mm(P, EkT);
    P = symt(mm(T1T, EkT), Lk, st);
}

__host__ __device__ inline int slices(int n) { return (n + 3) >> 2; }

// the identity beyond n on the diagonal of t
__device__ __forceinline__ f64x4 pad_eye(f64x4 t, int n) {
    const int li = lane_i(), lk = lane_k();
#pragma unroll
    for (int v = 0; v < 4; ++v)
        if (4 * v + lk == li && li >= n) t[v] = 1.0;
    return t;
}

// constants of model b (one block per model; a shared model has stride 0)
__device__ __forceinline__ const double* cst_of(const ScanArgs& a, int b) {
    return a.consts64 + (int64_t)b * a.model_stride;
}

__device__ __forceinline__ FConst load_fconst(const ScanArgs& a, const ConstLayout& CL, int b) {
    const double* cst = cst_of(a, b);
    const int n = a.nx, m = a.ny;
    FConst f;
    f.AT = load_tile_t(cst + CL.A, n, n, n);
    f.C = load_tile(cst + CL.C, n, n, n);
    f.J = load_tile(cst + CL.J, n, n, n);
    f.KT = load_tile_t(cst + CL.K, n, m, m);
    f.WT = load_tile_t(cst + CL.W, n, m, m);
    f.GT = load_tile_t(cst + CL.G, m, n, n);
    f.S = pad_eye(load_tile(cst + CL.S, m, m, m), m);
    f.c = load_vec(cst + CL.c, n);
    f.w = load_vec(cst + CL.w, n);
    f.n = n;
    f.ny = m;
    return f;
}

__device__ __forceinline__ SConst load_sconst(const ScanArgs& a, const ConstLayout& CL, int b) {
    const double* cst = cst_of(a, b);
    const int n = a.nx;
    SConst c;
    c.FT = load_tile_t(cst + CL.F, n, n, n);
    c.Q = pad_eye(load_tile(cst + CL.Q, n, n, n), n);
    c.u = load_vec(cst + CL.u, n);
    c.n = n;
    return c;
}

// the first-step element of sequence b's model: b_1 = c1 + K1 y_1, C_1 = C1
template <int KY>
__device__ __forceinline__ void first_step(const ScanArgs& a, const ConstLayout& CL, int b, const f64x4& yk, f64x4& b1,
                                           f64x4& C1) {
    const double* cst = cst_of(a, b);
    b1 = mm<KY>(load_tile_t(cst + CL.K1, a.nx, a.ny, a.ny), yk, load_vec(cst + CL.c1, a.nx));
    C1 = load_tile(cst + CL.C1, a.nx, a.nx, a.nx);
}

__device__ __forceinline__ int64_t blk_end(const W16Args& w, int64_t k0) {
    return k0 + w.blen < w.s.total ? k0 + w.blen : w.s.total;
}

// The sequence holding step k: [start, end) and its index b (wave-uniform).
// One sequence (offsets == nullptr): [0, total).  Packed sequences are
// separated by the exact zeros of a first step (A = 0) and of a last step
// (E = 0): at a sequence's first step the filtering accumulator's A, b, C are
// replaced by the first-step element, at its last step the smoothing
// accumulator by (0, m, P); the scans over block elements pass a right
// (filter) or left (smoother) operand with A = 0 (E = 0) through, so a failed
// sequence cannot reach the next one.
struct SeqT {
    int b;
    int64_t start, end;
};
__device__ __forceinline__ SeqT seq_find(const ScanArgs& a, int64_t k) {
    SeqT q;
    if (!a.offsets) {
        q.b = 0;
        q.start = 0;
        q.end = a.total;
        return q;
    }
    int lo = 0, hi = a.B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.offsets[mid] <= k) lo = mid; else hi = mid;
    }
    q.b = lo;
    q.start = a.offsets[lo];
    q.end = a.offsets[lo + 1];
    return q;
}
__device__ __forceinline__ void seq_next(const ScanArgs& a, SeqT& q, int64_t k) {
    if (a.offsets)
        while (k >= q.end && q.b < a.B - 1) { ++q.b; q.start = q.end; q.end = a.offsets[q.b + 1]; }
}
__device__ __forceinline__ void seq_prev(const ScanArgs& a, SeqT& q, int64_t k) {
    if (a.offsets)
        while (k < q.start && q.b > 0) { --q.b; q.end = q.start; q.start = a.offsets[q.b]; }
}
// every entry of the tile exactly zero (wave-uniform)
__device__ __forceinline__ bool all_zero(const f64x4& t) {
    return __all(t[0] == 0.0 && t[1] == 0.0 && t[2] == 0.0 && t[3] == 0.0);
}

// ---------------------------------------------------------------------------
// filter kernels
// ---------------------------------------------------------------------------
template <typename R, int KY, bool PK>
__global__ __launch_bounds__(kThreads) void k_w16_filter_reduce(W16Args w) {
    __shared__ double st[kStage];
    const ScanArgs& a = w.s;
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int ny = a.ny;
    const int64_t k0 = blockIdx.x * w.blen, k1 = blk_end(w, k0);
    if (blockIdx.x == 0)     // models whose precompute failed
        for (int b = threadIdx.x; b < a.nmodels; b += kThreads)
            if (a.model_fail[b]) atomicMin(a.status, b);
    SeqT q = seq_find(a, k0);
    int mb = a.model_stride ? q.b : 0;        // the model whose constants are loaded
    FConst f = load_fconst(a, CL, mb);
    const R* y = static_cast<const R*>(a.y);
    FE e;
    f64x4 yk = load_vec(y + k0 * ny, ny);
    if (k0 == q.start) {     // a first step: A = 0, eta = 0, J = 0
        first_step<KY>(a, CL, q.b, yk, e.b, e.C);
        e.A = zero4();
        e.eta = zero4();
        e.J = zero4();
    } else {
        e.A = tr(f.AT, st);
        e.b = mm<KY>(f.KT, yk, f.c);
        e.C = f.C;
        e.eta = mm<KY>(f.WT, yk, f.w);
        e.J = f.J;
    }
    // y of the next step is loaded while the current one is folded
    f64x4 ynext = load_vec(y + (k0 + 1 < k1 ? k0 + 1 : k0) * ny, ny);
    for (int64_t k = k0 + 1; k < k1; ++k) {
        yk = ynext;
        ynext = load_vec(y + (k + 1 < k1 ? k + 1 : k) * ny, ny);
        seq_next(a, q, k);
        if (k == q.start) {  // a sequence starts: its first-step element replaces A, b, C
            first_step<KY>(a, CL, q.b, yk, e.b, e.C);
            e.A = zero4();
            if (a.model_stride && q.b != mb) {
                mb = q.b;
                f = load_fconst(a, CL, mb);
            }
            continue;
        }
        fcombine_fresh<KY, PK>(e, f, mm<KY>(f.KT, yk, f.c), mm<KY>(f.WT, yk, f.w), st);
    }
    double* rec = w.agg[0] + (size_t)blockIdx.x * kFRec;
    put_tile(rec + kFA, e.A);
    put_tile(rec + kFC, e.C);
    put_tile(rec + kFJ, e.J);
    store_vec(rec + kFb, e.b, 16);
    store_vec(rec + kFeta, e.eta, 16);
}

// out[i] = in[i - d] (x) in[i] (i >= d), else in[i]
__global__ __launch_bounds__(kThreads) void k_w16_filter_ks(W16Args w, const double* in, double* out, int64_t d) {
    __shared__ double st[kStage];
    const int64_t i = blockIdx.x;
    const double* rj = in + (size_t)i * kFRec;
    double* ro = out + (size_t)i * kFRec;
    const f64x4 Aj = get_tile(rj + kFA), Cj = get_tile(rj + kFC), Jj = get_tile(rj + kFJ);
    const f64x4 bj = load_vec(rj + kFb, 16), etaj = load_vec(rj + kFeta, 16);
    FE e;
    if (i < d) {
        e.A = Aj; e.C = Cj; e.J = Jj; e.b = bj; e.eta = etaj;
    } else {
        const int n = w.s.nx;
        const double* ri = in + (size_t)(i - d) * kFRec;
        e.A = get_tile(ri + kFA);
        e.C = get_tile(ri + kFC);
        e.J = get_tile(ri + kFJ);
        e.b = load_vec(ri + kFb, 16);
        e.eta = load_vec(ri + kFeta, 16);
        const f64x4 I = eye();
        fcombine(e, tr(Aj, st), bj, Cj, etaj, Jj, I, st, n, w.pivot_always != 0);
        if (w.s.offsets && all_zero(Aj)) {
            // the right operand starts a sequence: its A, b, C pass through
            // (exactly what A_j = 0 gives, without 0 * NaN from the left)
            e.A = Aj;
            e.b = bj;
            e.C = Cj;
        }
    }
    put_tile(ro + kFA, e.A);
    put_tile(ro + kFC, e.C);
    put_tile(ro + kFJ, e.J);
    store_vec(ro + kFb, e.b, 16);
    store_vec(ro + kFeta, e.eta, 16);
}

// x rounded to the storage type R (the value a later kernel reads back)
template <typename R>
__device__ __forceinline__ f64x4 stored(const f64x4& x) {
    f64x4 t;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = double(R(x[v]));
    return t;
}

template <typename R, int KY, bool PK>
__global__ __launch_bounds__(kThreads) void k_w16_filter_down(W16Args w) {
    __shared__ double st[kStage];
    const ScanArgs& a = w.s;
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int n = a.nx, ny = a.ny;
    const int64_t blk = blockIdx.x, k0 = blk * w.blen, k1 = blk_end(w, k0);
    SeqT q = seq_find(a, k0);
    int mb = a.model_stride ? q.b : 0;
    FConst f = load_fconst(a, CL, mb);
    SConst sc = {};
    if (w.elem) sc = load_sconst(a, CL, mb);
    const R* y = static_cast<const R*>(a.y);
    R* mo = static_cast<R*>(a.m);
    R* Po = static_cast<R*>(a.P);
    f64x4 m = zero4(), P = zero4();
    if (blk > 0) {           // the filtered moments at the end of the previous block
        const double* rec = w.agg[w.final_buf] + (size_t)(blk - 1) * kFRec;
        m = load_vec(rec + kFb, 16);
        P = get_tile(rec + kFC);
    }
    f64x4 ynext = load_vec(y + k0 * ny, ny);
    for (int64_t k = k0; k < k1; ++k) {
        const f64x4 yk = ynext;
        ynext = load_vec(y + (k + 1 < k1 ? k + 1 : k) * ny, ny);
        seq_next(a, q, k);
        if (a.model_stride && q.b != mb) {
            mb = q.b;
            f = load_fconst(a, CL, mb);
            if (w.elem) sc = load_sconst(a, CL, mb);
        }
        if (k == q.start) first_step<KY>(a, CL, q.b, yk, m, P);
        else fcarry_fresh<KY, PK>(m, P, f, mm<KY>(f.KT, yk, f.c), mm<KY>(f.WT, yk, f.w), st);
        store_vec(mo + k * n, m, n);
        store_tile(Po + k * n * n, P, n);
        if (w.elem && k + 1 < q.end) {
            // the smoothing element of step k (Lemma 3), from the moments as
            // stored (the same inputs the smoother kernels would read back)
            bool okk = true;
            f64x4 ET, g, L;
            selem(stored<R>(m), stored<R>(P), sc, st, okk, ET, g, L);
            double* e = w.elem + (size_t)k * kSRec;
            put_tile(e + kSE, ET);
            put_tile(e + kSL, L);
            store_vec(e + kSg, g, 16);
            if (!okk && threadIdx.x == 0) atomicMin(a.status, q.b);
        }
    }
}

// ---------------------------------------------------------------------------
// smoother kernels
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void load_moments(const ScanArgs& a, int64_t k, f64x4& m, f64x4& P) {
    const int n = a.nx;
    m = load_vec(static_cast<const R*>(a.m) + k * n, n);
    P = load_tile(static_cast<const R*>(a.P) + k * n * n, n, n, n);
}

// the smoothing element of step k (not the last of its sequence): stored by
// the filter down-sweep, or built from the filtered moments
template <typename R>
__device__ __forceinline__ void elem_at(const W16Args& w, int64_t k, const SConst& c, double* st, int b, f64x4& ET,
                                        f64x4& g, f64x4& L) {
    if (w.elem) {
        const double* e = w.elem + (size_t)k * kSRec;
        ET = get_tile(e + kSE);
        g = load_vec(e + kSg, 16);
        L = get_tile(e + kSL);
    } else {
        f64x4 m, P;
        load_moments<R>(w.s, k, m, P);
        bool ok = true;
        selem(m, P, c, st, ok, ET, g, L);
        if (!ok && threadIdx.x == 0) atomicMin(w.s.status, b);
    }
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_w16_smoother_reduce(W16Args w) {
    __shared__ double st[kStage];
    const ScanArgs& a = w.s;
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int64_t k0 = blockIdx.x * w.blen, k1 = blk_end(w, k0);
    SeqT q = seq_find(a, k1 - 1);
    int mb = a.model_stride ? q.b : 0;
    SConst c = {};
    if (!w.elem) c = load_sconst(a, CL, mb);
    f64x4 E, g, L;
    if (k1 == q.end) {      // the last step of a sequence: E = 0, g = m, L = P
        load_moments<R>(a, k1 - 1, g, L);
        E = zero4();
    } else {
        f64x4 ET;
        elem_at<R>(w, k1 - 1, c, st, q.b, ET, g, L);
        E = tr(ET, st);
    }
    if (w.elem) {           // stored elements: the next one down is loaded while the current one is folded
        const double* e = w.elem + (size_t)(k1 - 2 >= k0 ? k1 - 2 : k0) * kSRec;
        f64x4 ETn = get_tile(e + kSE), gn = load_vec(e + kSg, 16), Ln = get_tile(e + kSL);
        for (int64_t k = k1 - 2; k >= k0; --k) {
            seq_prev(a, q, k);
            const f64x4 ETk = ETn, gk = gn, Lk = Ln;
            e = w.elem + (size_t)(k - 1 >= k0 ? k - 1 : k0) * kSRec;
            ETn = get_tile(e + kSE);
            gn = load_vec(e + kSg, 16);
            Ln = get_tile(e + kSL);
            if (k == q.end - 1) {   // a sequence ends here (its slot holds no element): restart
                load_moments<R>(a, k, g, L);
                E = zero4();
            } else {
                sfold(E, g, L, ETk, gk, Lk, st);
            }
        }
    } else {
        for (int64_t k = k1 - 2; k >= k0; --k) {
            seq_prev(a, q, k);
            if (k == q.end - 1) {   // a sequence ends here: the accumulator restarts
                load_moments<R>(a, k, g, L);
                E = zero4();
                continue;
            }
            if (a.model_stride && q.b != mb) {
                mb = q.b;
                c = load_sconst(a, CL, mb);
            }
            f64x4 ETk, gk, Lk;
            elem_at<R>(w, k, c, st, q.b, ETk, gk, Lk);
            sfold(E, g, L, ETk, gk, Lk, st);
        }
    }
    double* rec = w.agg[0] + (size_t)blockIdx.x * kSRec;
    put_tile(rec + kSE, E);
    put_tile(rec + kSL, L);
    store_vec(rec + kSg, g, 16);
}

// out[i] = in[i] (x) in[i + d] (i + d < nb), else in[i]
__global__ __launch_bounds__(kThreads) void k_w16_smoother_ks(W16Args w, const double* in, double* out, int64_t d) {
    __shared__ double st[kStage];
    const int64_t i = blockIdx.x;
    const double* ri = in + (size_t)i * kSRec;
    double* ro = out + (size_t)i * kSRec;
    const f64x4 Ei = get_tile(ri + kSE), Li = get_tile(ri + kSL), gi = load_vec(ri + kSg, 16);
    f64x4 E, g, L;
    // the left operand ending a sequence (E = 0) passes through
    if (i + d >= w.nblocks || (w.s.offsets && all_zero(Ei))) {
        E = Ei; g = gi; L = Li;
    } else {
        const double* rj = in + (size_t)(i + d) * kSRec;
        E = get_tile(rj + kSE);
        L = get_tile(rj + kSL);
        g = load_vec(rj + kSg, 16);
        sfold(E, g, L, tr(Ei, st), gi, Li, st);
    }
    put_tile(ro + kSE, E);
    put_tile(ro + kSL, L);
    store_vec(ro + kSg, g, 16);
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_w16_smoother_down(W16Args w) {
    __shared__ double st[kStage];
    const ScanArgs& a = w.s;
    const ConstLayout CL = const_layout(a.nx, a.ny);
    const int n = a.nx;
    const int64_t blk = blockIdx.x, k0 = blk * w.blen, k1 = blk_end(w, k0);
    SeqT q = seq_find(a, k1 - 1);
    int mb = a.model_stride ? q.b : 0;
    SConst c = {};
    if (!w.elem) c = load_sconst(a, CL, mb);
    R* mso = static_cast<R*>(a.ms);
    R* Pso = static_cast<R*>(a.Ps);
    f64x4 ms = zero4(), Ps = zero4();
    if (blk + 1 < w.nblocks) {   // the smoothed moments at the start of the next block
        const double* rec = w.agg[w.final_buf] + (size_t)(blk + 1) * kSRec;
        ms = load_vec(rec + kSg, 16);
        Ps = get_tile(rec + kSL);
    }
    if (w.elem) {            // stored elements; step k - 1's is loaded while step k is folded
        const double* e = w.elem + (size_t)(k1 - 1) * kSRec;
        f64x4 ETn = get_tile(e + kSE), gn = load_vec(e + kSg, 16), Ln = get_tile(e + kSL);
        for (int64_t k = k1 - 1; k >= k0; --k) {
            seq_prev(a, q, k);
            const f64x4 ETk = ETn, gk = gn, Lk = Ln;
            e = w.elem + (size_t)(k - 1 >= k0 ? k - 1 : k0) * kSRec;
            ETn = get_tile(e + kSE);
            gn = load_vec(e + kSg, 16);
            Ln = get_tile(e + kSL);
            if (k == q.end - 1) load_moments<R>(a, k, ms, Ps);   // (its slot holds no element)
            else scarry(ms, Ps, ETk, gk, Lk, st);
            store_vec(mso + k * n, ms, n);
            store_tile(Pso + k * n * n, Ps, n);
        }
        return;
    }
    for (int64_t k = k1 - 1; k >= k0; --k) {
        seq_prev(a, q, k);
        if (k == q.end - 1) {
            load_moments<R>(a, k, ms, Ps);
        } else {
            if (a.model_stride && q.b != mb) {
                mb = q.b;
                c = load_sconst(a, CL, mb);
            }
            f64x4 ETk, gk, Lk;
            elem_at<R>(w, k, c, st, q.b, ETk, gk, Lk);
            scarry(ms, Ps, ETk, gk, Lk, st);
        }
        store_vec(mso + k * n, ms, n);
        store_tile(Pso + k * n * n, Ps, n);
    }
}

// ---------------------------------------------------------------------------
// Model constants of one model (5 <= nx <= 16, ny <= 16) in one wavefront,
// the same fields and formulas as the cooperative precompute kernel (Lemma 1
// for k > 1 and for the first step, the smoother's F, Q, u), with the
// positive definite solves as register inverses (a non-positive pivot marks
// the model as failed, its constants NaN).
// ---------------------------------------------------------------------------
struct PreArgs {
    int nx, ny;
    const double *F, *u, *Q, *H, *d, *R, *m0, *P0;
    double* consts64;
    float* consts32;     // nullptr: FP64 only
    int* status;
    int* model_fail;
    int what;            // 1: filter constants, 2: smoother constants, 3: both
    int reset;
    int per_sequence;    // model arrays hold one model per workgroup (else one shared)
};

template <typename T>
__device__ __forceinline__ void put_mat(T* X, const f64x4& t, int rows, int cols) {
    const int li = lane_i(), lk = lane_k();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + lk;
        if (r < rows && li < cols) X[r * cols + li] = T(t[v]);
    }
}

template <typename T>
__device__ __forceinline__ void put_fields(T* o, const ConstLayout& CL, int n, int m, int what, const f64x4& A,
                                           const f64x4& C, const f64x4& J, const f64x4& K, const f64x4& W,
                                           const f64x4& c, const f64x4& w, const f64x4& K1, const f64x4& c1,
                                           const f64x4& C1, const f64x4& G, const f64x4& S, const f64x4& e,
                                           const f64x4& F, const f64x4& Q, const f64x4& u) {
    if (what & 1) {
        put_mat(o + CL.A, A, n, n);
        put_mat(o + CL.C, C, n, n);
        put_mat(o + CL.J, J, n, n);
        put_mat(o + CL.K, K, n, m);
        put_mat(o + CL.W, W, n, m);
        store_vec(o + CL.c, c, n);
        store_vec(o + CL.w, w, n);
        put_mat(o + CL.K1, K1, n, m);
        store_vec(o + CL.c1, c1, n);
        put_mat(o + CL.C1, C1, n, n);
        put_mat(o + CL.G, G, m, n);
        put_mat(o + CL.S, S, m, m);
        store_vec(o + CL.e, e, m);
    }
    if (what & 2) {
        put_mat(o + CL.F, F, n, n);
        put_mat(o + CL.Q, Q, n, n);
        store_vec(o + CL.u, u, n);
    }
}

__global__ __launch_bounds__(kThreads) void k_w16_precompute(PreArgs a) {
    __shared__ double st[kStage];
    const int mdl = blockIdx.x;          // the model of this workgroup
    if (mdl == 0 && threadIdx.x == 0 && (a.reset || a.status[1] != kStatusMagic)) {
        a.status[0] = kStatusOk;
        a.status[1] = kStatusMagic;
    }
    const int n = a.nx, m = a.ny;
    const ConstLayout CL = const_layout(n, m);
    if (a.per_sequence) {                // this model's rows of the model arrays
        const int64_t b = mdl;
        a.F += b * n * n;
        a.Q += b * n * n;
        a.H += b * m * n;
        a.R += b * m * m;
        a.m0 += b * n;
        a.P0 += b * n * n;
        if (a.u) a.u += b * n;
        if (a.d) a.d += b * m;
    }
    a.consts64 += (int64_t)mdl * CL.words;
    if (a.consts32) a.consts32 += (int64_t)mdl * CL.words;
    a.model_fail += mdl;
    const f64x4 F = load_tile(a.F, n, n, n), FT = load_tile_t(a.F, n, n, n);
    const f64x4 Q = load_tile(a.Q, n, n, n);
    const f64x4 u = a.u ? load_vec(a.u, n) : zero4();
    const f64x4 Z0 = zero4();
    bool ok = true;
    f64x4 A = Z0, C = Z0, J = Z0, K = Z0, W = Z0, c = Z0, w = Z0, K1 = Z0, c1 = Z0, C1 = Z0, G = Z0, S = Z0, e = Z0;
    if (a.what & 1) {
        const f64x4 HT = load_tile_t(a.H, m, n, n), R = load_tile(a.R, m, m, m);
        const f64x4 d = a.d ? load_vec(a.d, m) : Z0;
        // k > 1: S = H Q H^T + R, K = Q H^T S^-1, G = H F, W = G^T S^-1,
        // J = W G, A = F - K G, C = Q - K H Q, e = H u + d, c = u - K e, w = -W e
        const f64x4 T1 = mm(HT, Q);                               // H Q
        S = symt(mm(tr(T1, st), HT, R), Z0, st);
        const f64x4 Si = inv_spd(S, m, ok);
        const f64x4 Kt = mm(Si, T1);                              // S^-1 H Q
        G = mm(HT, F);
        const f64x4 Zt = mm(Si, G);                               // S^-1 H F
        K = tr(Kt, st);
        W = tr(Zt, st);
        J = symt(mm(G, Zt), Z0, st);
        const f64x4 nKt = -Kt;
        A = mm(nKt, G, F);
        C = symt(mm(nKt, T1, Q), Z0, st);
        e = mm(HT, u, d);
        c = mm(nKt, e, u);
        w = mm(-Zt, e);
        // the first step: m1 = F m0 + u, P1 = F P0 F^T + Q, S1 = H P1 H^T + R,
        // K1 = P1 H^T S1^-1, c1 = m1 - K1 (H m1 + d), C1 = P1 - K1 S1 K1^T
        const f64x4 m1 = mm(FT, load_vec(a.m0, n), u);
        const f64x4 FP0 = mm(FT, load_tile(a.P0, n, n, n));
        const f64x4 P1 = symt(mm(tr(FP0, st), FT, Q), Z0, st);
        const f64x4 T2 = mm(HT, P1);                              // H P1
        const f64x4 S1 = symt(mm(tr(T2, st), HT, R), Z0, st);
        const f64x4 K1t = mm(inv_spd(S1, m, ok), T2);             // S1^-1 H P1
        K1 = tr(K1t, st);
        c1 = mm(-K1t, mm(HT, m1, d), m1);
        const f64x4 U = mm(K1t, S1);                              // K1 S1
        C1 = symt(mm(-tr(U, st), K1t, P1), Z0, st);
    }
    const f64x4 Fs = (a.what & 2) ? F : Z0, Qs = (a.what & 2) ? Q : Z0, us = (a.what & 2) ? u : Z0;
    if (ok) {
        put_fields(a.consts64, CL, n, m, a.what, A, C, J, K, W, c, w, K1, c1, C1, G, S, e, Fs, Qs, us);
        if (a.consts32)
            put_fields(a.consts32, CL, n, m, a.what, A, C, J, K, W, c, w, K1, c1, C1, G, S, e, Fs, Qs, us);
    } else {
        for (int i = threadIdx.x; i < CL.words; i += kThreads) {
            a.consts64[i] = __builtin_nan("");
            if (a.consts32) a.consts32[i] = __builtin_nanf("");
        }
    }
    if ((a.what & 1) && threadIdx.x == 0) a.model_fail[0] = ok ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Marginal likelihood factors (Section III-C) of one sequence with one model,
// 5 <= nx <= 16, ny <= 16: log N(y_k; G m_{k-1} + e, G P_{k-1} G^T + S0) from
// the filtered moments of the previous step (the prior at k = 0), one wave per
// run of consecutive steps.  The residual is a compensated dot product (the
// Dot2 scheme of Ogita, Rump and Oishi: every product's and every addition's
// rounding error kept and added at the end), one row per lane; the covariance
// is a register-tile product; its inverse and log-determinant come from the
// unpivoted Gauss-Jordan elimination (the pivots of a positive definite
// matrix are the diagonal of its LDL^T factorisation).
// ---------------------------------------------------------------------------
struct LLW {
    int nx, ny;
    int64_t total, per_wave;
    const double *m0, *P0, *cst;
    int cG, cS, ce;
    const void *y, *m, *P;
    double* step;
    int* status;
};

struct Dot2 {
    double s, c;
};
__device__ __forceinline__ void dot2_add(Dot2& a, double x) {
#pragma clang fp contract(off)
    const double t = a.s + x;
    const double z = t - a.s;
    a.c += (a.s - (t - z)) + (x - z);
    a.s = t;
}
__device__ __forceinline__ void dot2_sub_prod(Dot2& a, double g, double x) {
#pragma clang fp contract(off)
    const double p = g * x;
    const double e = fma(g, x, -p);       // g x = p + e exactly
    dot2_add(a, -p);
    a.c -= e;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_ll_w16(LLW a) {
    __shared__ double st[kStage];
    const int n = a.nx, m = a.ny, li = lane_i();
    const f64x4 GT = load_tile_t(a.cst + a.cG, m, n, n);
    const f64x4 S0 = pad_eye(load_tile(a.cst + a.cS, m, m, m), m);
    double Grow[16];                          // row li of G (the residual's row of this lane)
#pragma unroll
    for (int l = 0; l < 16; ++l) Grow[l] = (li < m && l < n) ? a.cst[a.cG + li * n + l] : 0.0;
    const double e_i = li < m ? a.cst[a.ce + li] : 0.0;
    const R* gy = static_cast<const R*>(a.y);
    const R* gm = static_cast<const R*>(a.m);
    const R* gP = static_cast<const R*>(a.P);
    const int64_t k0 = (int64_t)blockIdx.x * a.per_wave;
    const int64_t k1 = k0 + a.per_wave < a.total ? k0 + a.per_wave : a.total;
    // the previous step's moments (the prior at k = 0) and y_k; the next
    // step's are loaded while the current one is evaluated
    auto fetch = [&](int64_t k, f64x4& P, double (&mv)[16], double& yk) {
        if (k == 0) {
            P = load_tile(a.P0, n, n, n);
#pragma unroll
            for (int l = 0; l < 16; ++l) mv[l] = l < n ? a.m0[l] : 0.0;
        } else {
            P = load_tile(gP + (k - 1) * n * n, n, n, n);
#pragma unroll
            for (int l = 0; l < 16; ++l) mv[l] = l < n ? double(gm[(k - 1) * n + l]) : 0.0;
        }
        yk = li < m ? double(gy[k * m + li]) : 0.0;
    };
    f64x4 Pn;
    double mn[16], yn;
    fetch(k0, Pn, mn, yn);
    for (int64_t k = k0; k < k1; ++k) {
        const f64x4 P = Pn;
        double mv[16];
#pragma unroll
        for (int l = 0; l < 16; ++l) mv[l] = mn[l];
        const double yk = yn;
        fetch(k + 1 < k1 ? k + 1 : k, Pn, mn, yn);
        // r_i = y_i - e_i - (G m)_i for i = li
        Dot2 acc{yk, 0.0};
        dot2_add(acc, -e_i);
#pragma unroll
        for (int l = 0; l < 16; ++l) dot2_sub_prod(acc, Grow[l], mv[l]);
        const double ri = acc.s + acc.c;
        f64x4 r;                              // replicated: r(4 v + lk)
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = __shfl(ri, (threadIdx.x & 48) | (4 * v + lane_k()), 64);
        // S = G P G^T + S0, its inverse and log-determinant, r^T S^-1 r
        bool ok = true;
        Det det;
        const f64x4 Z = inv_diag<true>(symt(mm(GT, mm(P, GT)), S0, st), m, ok, &det);
        const double logdet = log(det.mant) + det.exp * 0.69314718055994530942;   // log 2
        const f64x4 Zr = mm(Z, r);
        double q = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) q += r[v] * Zr[v];
        q += __shfl_xor(q, 16, 64);
        q += __shfl_xor(q, 32, 64);
        if ((threadIdx.x & 63) == 0) {
            double ll = -0.5 * (m * 1.8378770664093454836 + q + logdet);   // log(2 pi) = 1.83787...
            if (!ok) {
                ll = __builtin_nan("");
                atomicMin(a.status, 0);
            }
            a.step[k] = ll;
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int64_t blocks_for(int64_t total) {
    int64_t nb = (total + 3) / 4;
    if (nb > kMaxBlocks) nb = kMaxBlocks;
    return nb < 1 ? 1 : nb;
}

size_t buffer_bytes(int64_t nb) { return ((size_t)nb * kFRec * sizeof(double) + 255) & ~size_t(255); }

// sequences up to this length keep every step's smoothing element between
// the filter down-sweep and the smoother kernels (4.2 KB a step)
constexpr int64_t kMaxStoredSteps = int64_t(1) << 18;
size_t elem_bytes(int64_t total) {
    return total <= kMaxStoredSteps ? (((size_t)total * kSRec * sizeof(double) + 255) & ~size_t(255)) : 0;
}

template <typename R>
hipError_t run(W16Args w, bool smoother, hipStream_t s) {
    const dim3 grid((unsigned)w.nblocks), block(kThreads);
    int cur = 0;
    if (!smoother) {
        prof_begin("k_w16_filter_reduce", s);
        switch (w.s.ny < 16 ? slices(w.s.ny) : 5) {
            case 1: hipLaunchKernelGGL((k_w16_filter_reduce<R, 1, true>), grid, block, 0, s, w); break;
            case 2: hipLaunchKernelGGL((k_w16_filter_reduce<R, 2, true>), grid, block, 0, s, w); break;
            case 3: hipLaunchKernelGGL((k_w16_filter_reduce<R, 3, true>), grid, block, 0, s, w); break;
            case 4: hipLaunchKernelGGL((k_w16_filter_reduce<R, 4, true>), grid, block, 0, s, w); break;
            default: hipLaunchKernelGGL((k_w16_filter_reduce<R, 4, false>), grid, block, 0, s, w); break;   // ny = 16
        }
        prof_end(s);
        for (int64_t d = 1; d < w.nblocks; d <<= 1) {
            prof_begin("k_w16_filter_ks", s);
            hipLaunchKernelGGL(k_w16_filter_ks, grid, block, 0, s, w, w.agg[cur], w.agg[cur ^ 1], d);
            prof_end(s);
            cur ^= 1;
        }
        w.final_buf = cur;
        prof_begin("k_w16_filter_down", s);
        switch (w.s.ny < 16 ? slices(w.s.ny) : 5) {
            case 1: hipLaunchKernelGGL((k_w16_filter_down<R, 1, true>), grid, block, 0, s, w); break;
            case 2: hipLaunchKernelGGL((k_w16_filter_down<R, 2, true>), grid, block, 0, s, w); break;
            case 3: hipLaunchKernelGGL((k_w16_filter_down<R, 3, true>), grid, block, 0, s, w); break;
            case 4: hipLaunchKernelGGL((k_w16_filter_down<R, 4, true>), grid, block, 0, s, w); break;
            default: hipLaunchKernelGGL((k_w16_filter_down<R, 4, false>), grid, block, 0, s, w); break;   // ny = 16
        }
        prof_end(s);
    } else {
        prof_begin("k_w16_smoother_reduce", s);
        hipLaunchKernelGGL(k_w16_smoother_reduce<R>, grid, block, 0, s, w);
        prof_end(s);
        for (int64_t d = 1; d < w.nblocks; d <<= 1) {
            prof_begin("k_w16_smoother_ks", s);
            hipLaunchKernelGGL(k_w16_smoother_ks, grid, block, 0, s, w, w.agg[cur], w.agg[cur ^ 1], d);
            prof_end(s);
            cur ^= 1;
        }
        w.final_buf = cur;
        prof_begin("k_w16_smoother_down", s);
        hipLaunchKernelGGL(k_w16_smoother_down<R>, grid, block, 0, s, w);
        prof_end(s);
    }
    return hipGetLastError();
}

}  // namespace w16

bool w16_applies(int nx, int ny, bool time_invariant) {
    return time_invariant && nx >= 5 && nx <= 16 && ny >= 1 && ny <= 16;
}

int64_t w16_default_blocks(int64_t total) { return w16::blocks_for(total); }

size_t w16_ws_bytes(int64_t total) { return 2 * w16::buffer_bytes(w16::blocks_for(total)) + w16::elem_bytes(total); }

bool launch_w16_precompute(int nx, int ny, int32_t nmodels, const pks_model& model, double* consts64, float* consts32,
                           int* status, int* model_fail, int what, bool reset, hipStream_t s) {
    if (!w16_applies(nx, ny, true) || what < 1 || what > 3 || nmodels < 1) return false;
    w16::PreArgs p;
    p.nx = nx;
    p.ny = ny;
    p.F = model.F; p.u = model.u; p.Q = model.Q;
    p.H = model.H; p.d = model.d; p.R = model.R;
    p.m0 = model.m0; p.P0 = model.P0;
    p.consts64 = consts64;
    p.consts32 = consts32;
    p.status = status;
    p.model_fail = model_fail;
    p.what = what;
    p.reset = reset ? 1 : 0;
    p.per_sequence = model.per_sequence ? 1 : 0;
    hipLaunchKernelGGL(w16::k_w16_precompute, dim3((unsigned)nmodels), dim3(w16::kThreads), 0, s, p);
    return true;
}

bool launch_ll_w16(int nx, int ny, int64_t total, const double* m0, const double* P0, const double* consts64, int cG,
                   int cS, int ce, const void* y, const void* m, const void* P, double* step, int* status, bool mixed,
                   hipStream_t s) {
    if (!w16_applies(nx, ny, true) || total < 1) return false;
    w16::LLW a;
    a.nx = nx;
    a.ny = ny;
    a.total = total;
    const int64_t waves = total < 2048 ? total : 2048;
    a.per_wave = (total + waves - 1) / waves;
    a.m0 = m0;
    a.P0 = P0;
    a.cst = consts64;
    a.cG = cG;
    a.cS = cS;
    a.ce = ce;
    a.y = y;
    a.m = m;
    a.P = P;
    a.step = step;
    a.status = status;
    const dim3 grid((unsigned)((total + a.per_wave - 1) / a.per_wave)), block(w16::kThreads);
    if (mixed) hipLaunchKernelGGL(w16::k_ll_w16<float>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(w16::k_ll_w16<double>, grid, block, 0, s, a);
    return true;
}

hipError_t launch_w16(ScanArgs a, void* region, bool mixed, bool smoother, bool both, hipStream_t s) {
    using namespace w16;
    W16Args w;
    w.s = a;
    const int64_t nb_max = blocks_for(a.total);
    // a tuned block count is honoured up to the count the workspace is sized for
    w.nblocks = (a.large_blocks > 0 && a.large_blocks < nb_max) ? a.large_blocks : nb_max;
    w.blen = (a.total + w.nblocks - 1) / w.nblocks;
    w.nblocks = (a.total + w.blen - 1) / w.blen;
    char* base = static_cast<char*>(region);
    w.agg[0] = reinterpret_cast<double*>(base);
    w.agg[1] = reinterpret_cast<double*>(base + buffer_bytes(nb_max));
    w.final_buf = 0;
    // a combined filter + smoother call passes the smoothing elements from
    // the filter down-sweep to the smoother kernels
    const char* pv = getenv("PKS_PIVOTED_INVERSE");
    w.pivot_always = (pv && pv[0] == '1') ? 1 : 0;
    w.elem = (both && elem_bytes(a.total) > 0) ? reinterpret_cast<double*>(base + 2 * buffer_bytes(nb_max)) : nullptr;
    return mixed ? run<float>(w, smoother, s) : run<double>(w, smoother, s);
}

}  // namespace pks
