// top_epl.hpp -- the top level of the small-state scans (nx <= 4): a
// device-wide scan of the per-wave aggregates that the reduce kernels leave,
// with one scan element spread over 16 lanes and its 4 x 4 products on the
// matrix cores.
//
// The top level is a chain of combines (the per-wave aggregates of the whole
// sequence are scanned), so what counts there is the latency of one combine,
// not the throughput of many.  One element per lane (the layout of the reduce
// and down-sweep kernels) costs about 1,600 dependent vector instructions per
// filtering combine; with 16 lanes per element a 4 x 4 product is one
// v_mfma_f64_4x4x4f64 and the (I + C_i J_j) solve a 4-step Gauss-Jordan
// elimination with lane exchanges.
//
// Grid: up to kTopMaxWg workgroups of 256 threads (one wave per SIMD: a
// combine is about 2,400 cycles of mostly issued instructions, so waves that
// share a SIMD slow each other down), 16 groups of 16 lanes each.  Group G of
// workgroup w folds E consecutive items, the 16 groups are scanned with a
// Kogge-Stone pattern through LDS, the workgroup publishes its aggregate (a
// flag per workgroup, release/acquire at device scope) and then combines the
// aggregates of all workgroups before it (after it, for the smoother): each
// group folds up to ceil(w / 16) of them and the groups are scanned again --
// a look-back over the whole window, so no workgroup waits for another's
// look-back, only for its aggregate.  Workgroups take their place in the
// order from an atomic ticket, so a workgroup only ever waits for workgroups
// that are already running.  Each group then re-folds its items from the
// incoming prefix in moments form (Lemma 2 with A = 0, Lemma 4 with E = 0)
// and writes one carry per item, as the down-sweeps expect.
//
// Element layout (per wave, four groups g = 0..3): lane 16 r + 4 g + c holds
// entry (r, c) of every 4 x 4 matrix of group g's element and entry r of every
// vector (the same value for every c).  States with nx < 4 are padded with
// zero rows and columns (identity elements with ones on the whole diagonal);
// the padding never mixes with the leading nx x nx block.  With A, B and C in
// this layout, v_mfma_f64_4x4x4f64 returns X^T Y for each group (its A operand
// takes entry (i, k) from lane 16 k + 4 g + i, B (k, j) from lane 16 k + 4 g + j,
// and D (i, j) lands in lane 16 i + 4 g + j), so X Y takes X^T as the first
// operand: elements keep A (E) and its transpose.
#pragma once
#include "pks_internal.h"
#include "small_ops.hpp"

namespace pks {
namespace {

constexpr int kTopThreads = 256;              // one wave per SIMD: the combines are issue-bound
constexpr int kTopGroups = kTopThreads / 16;   // groups (elements) per workgroup
constexpr int kTopMaxWg = kTopMaxWorkgroups;   // look-back window: one group per other workgroup
static_assert(kTopAggWords >= 6 * 16, "workgroup aggregate slots hold a filtering element");
constexpr int kTopSpin = 1 << 22;              // polls before a missing aggregate is reported

struct Lanes {
    int r, c, g4;   // row, column, 4 g (lane of entry (0, 0) within its row of 16 lanes)
};
__device__ __forceinline__ Lanes lanes_of(int lane) { return Lanes{lane >> 4, lane & 3, lane & 12}; }

// X^T Y for each group of the wave
__device__ __forceinline__ double mtm(double x, double y) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(x, y, 0.0, 0, 0, 0);
}
__device__ __forceinline__ double from_lane(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double transposed(double v, const Lanes& L) {
    return from_lane(v, 16 * L.c + L.g4 + L.r);
}
__device__ __forceinline__ double sym(double v, const Lanes& L) { return 0.5 * (v + transposed(v, L)); }
__device__ __forceinline__ double eye(const Lanes& L) { return L.r == L.c ? 1.0 : 0.0; }
// every entry of the group's matrix is exactly zero
__device__ __forceinline__ bool group_zero(double v, const Lanes& L) {
    const unsigned long long nz = __ballot(v != 0.0);
    return (nz & (0x000F000F000F000Full << L.g4)) == 0;
}
__device__ __forceinline__ double pick4(const double (&v)[4], int i) {
    return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
}

// Inverse of each group's 4 x 4 matrix: Gauss-Jordan elimination with
// partial pivoting (the row with the largest entry of the pivot column among
// the remaining rows), in double.  The lane exchanges go through LDS-routed
// permutes; gfx950's cross-row permlane swaps (three per 32-bit half to bring
// all four rows to every lane) measured slower here: 2,550 against 2,100
// cycles per inverse.
__device__ __forceinline__ double inverse4(double x, const Lanes& L) {
    double v = eye(L);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double col[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) col[q] = from_lane(x, 16 * q + L.g4 + p);
        int piv = p;
        double best = fabs(col[p]);
#pragma unroll
        for (int q = p + 1; q < 4; ++q) {
            const double a = fabs(col[q]);
            if (a > best) {
                best = a;
                piv = q;
            }
        }
        // rows p and piv trade places; every lane reads both (no divergent exchange)
        const double px = from_lane(x, 16 * piv + L.g4 + L.c), pv = from_lane(v, 16 * piv + L.g4 + L.c);
        const double ox = from_lane(x, 16 * p + L.g4 + L.c), ov = from_lane(v, 16 * p + L.g4 + L.c);
        const bool swapped = L.r == piv;
        const double rx = swapped ? ox : x, rv = swapped ? ov : v;
        const double f = swapped ? col[p] : pick4(col, L.r);   // column-p entry of this row after the exchange
        const double rp = rcp64(pick4(col, piv));
        const double nx = px * rp, nv = pv * rp;                 // the pivot row, normalised
        x = (L.r == p) ? nx : fma(-f, nx, rx);
        v = (L.r == p) ? nv : fma(-f, nv, rv);
    }
    return v;
}

// ---------------------------------------------------------------------------
// elements in the 16-lane layout
// ---------------------------------------------------------------------------
struct EF { double A, At, b, C, eta, J; };   // Lemma 1 / 2 (At = A^T)
struct ES { double E, Et, g, L; };           // Lemma 3 / 4 (Et = E^T)
struct EM { double m, P; };                  // moments (A = 0 prefix, E = 0 suffix)
constexpr int kEFWords = 6;
constexpr int kESWords = 4;

__device__ __forceinline__ void ident(EF& e, const Lanes& L) {
    e.A = e.At = eye(L);
    e.b = e.C = e.eta = e.J = 0.0;
}
__device__ __forceinline__ void ident(ES& e, const Lanes& L) {
    e.E = e.Et = eye(L);
    e.g = e.L = 0.0;
}

// o = i (x) j (Lemma 2).  M = I + C_i J_j; W = (M^T)^-1 = inverse of I + J_j C_i,
// so mtm(W, Y) = M^-1 Y.  With K = M^-1 A_i, A_i^T M^-T = K^T.
template <bool G>
__device__ __forceinline__ void epl_fcombine(const EF& ei, const EF& ej, EF& o, const Lanes& L) {
    const double W = inverse4(mtm(ej.J, ei.C) + eye(L), L);   // C, J symmetric: J_j^T C_i = J_j C_i
    const double K = mtm(W, ei.A);
    const double x2 = mtm(W, ei.b + mtm(ei.C, ej.eta));        // M^-1 (b_i + C_i eta_j)
    const double Z = mtm(W, ei.C);                             // M^-1 C_i (symmetric)
    const double w = ej.eta - mtm(ej.J, ei.b);                 // eta_j - J_j b_i
    const double JA = mtm(ej.J, ei.A);                         // J_j A_i
    EF t;
    t.A = mtm(ej.At, K);                                       // A_j M^-1 A_i
    t.At = mtm(K, ej.At);                                      // its transpose
    t.b = mtm(ej.At, x2) + ej.b;
    t.C = sym(mtm(ej.At, mtm(Z, ej.At)), L) + ej.C;            // A_j Z^T A_j^T
    t.eta = mtm(K, w) + ei.eta;                                // A_i^T M^-T w
    t.J = sym(mtm(K, JA), L) + ei.J;                           // A_i^T M^-T J_j A_i
    if (G && group_zero(ej.A, L)) {                            // j starts a sequence
        t.A = t.At = 0.0;
        t.b = ej.b;
        t.C = ej.C;
    }
    o = t;
}

// x <- x (x) j for a prefix x whose A is zero (moments only)
template <bool G>
__device__ __forceinline__ void epl_fcarry(EM& x, const EF& ej, const Lanes& L) {
    const double W = inverse4(mtm(ej.J, x.P) + eye(L), L);
    const double x2 = mtm(W, x.m + mtm(x.P, ej.eta));
    const double Z = mtm(W, x.P);
    double m = mtm(ej.At, x2) + ej.b;
    double P = sym(mtm(ej.At, mtm(Z, ej.At)), L) + ej.C;
    if (G && group_zero(ej.A, L)) {
        m = ej.b;
        P = ej.C;
    }
    x.m = m;
    x.P = P;
}

// o = i (x) j (Lemma 4)
template <bool G>
__device__ __forceinline__ void epl_scombine(const ES& ei, const ES& ej, ES& o, const Lanes& L) {
    ES t;
    t.E = mtm(ei.Et, ej.E);                                    // E_i E_j
    t.Et = mtm(ej.E, ei.Et);                                   // E_j^T E_i^T
    t.g = mtm(ei.Et, ej.g) + ei.g;
    t.L = sym(mtm(ei.Et, mtm(ej.L, ei.Et)), L) + ei.L;         // E_i L_j E_i^T
    if (G && group_zero(ei.E, L)) t = ei;                      // i ends a sequence
    o = t;
}

// x <- i (x) x for a suffix x whose E is zero (moments only)
template <bool G>
__device__ __forceinline__ void epl_scarry(const ES& ei, EM& x, const Lanes& L) {
    double m = mtm(ei.Et, x.m) + ei.g;
    double P = sym(mtm(ei.Et, mtm(x.P, ei.Et)), L) + ei.L;
    if (G && group_zero(ei.E, L)) {
        m = ei.g;
        P = ei.L;
    }
    x.m = m;
    x.P = P;
}

// ---------------------------------------------------------------------------
// transfers between the per-lane SoA records (word w of item i at
// base[w * n + i]) and the 16-lane layout
// ---------------------------------------------------------------------------
template <int N, typename R>
__device__ __forceinline__ void load_ef(const void* items, int64_t n, int64_t i, const Lanes& L, EF& e) {
    const R* p = static_cast<const R*>(items) + i;
    constexpr int ob = N * N, oC = ob + N, oe = oC + tri(N), oJ = oe + N;
    const bool in = L.r < N && L.c < N, rin = L.r < N;
    const int s = in ? sidx(L.r, L.c) : 0;
    e.A = in ? double(p[(int64_t)(L.r * N + L.c) * n]) : 0.0;
    e.At = in ? double(p[(int64_t)(L.c * N + L.r) * n]) : 0.0;
    e.C = in ? double(p[(int64_t)(oC + s) * n]) : 0.0;
    e.J = in ? double(p[(int64_t)(oJ + s) * n]) : 0.0;
    e.b = rin ? double(p[(int64_t)(ob + L.r) * n]) : 0.0;
    e.eta = rin ? double(p[(int64_t)(oe + L.r) * n]) : 0.0;
}
template <int N, typename R>
__device__ __forceinline__ void load_es(const void* items, int64_t n, int64_t i, const Lanes& L, ES& e) {
    const R* p = static_cast<const R*>(items) + i;
    constexpr int og = N * N, oL = og + N;
    const bool in = L.r < N && L.c < N, rin = L.r < N;
    e.E = in ? double(p[(int64_t)(L.r * N + L.c) * n]) : 0.0;
    e.Et = in ? double(p[(int64_t)(L.c * N + L.r) * n]) : 0.0;
    e.L = in ? double(p[(int64_t)(oL + sidx(L.r, L.c)) * n]) : 0.0;
    e.g = rin ? double(p[(int64_t)(og + L.r) * n]) : 0.0;
}
// moments record: m[N], then P packed (lower triangle)
template <int N, typename R>
__device__ __forceinline__ void store_em(void* carry, int64_t n, int64_t i, const Lanes& L, const EM& x) {
    R* p = static_cast<R*>(carry) + i;
    if (L.r < N && L.c == 0) p[(int64_t)L.r * n] = R(x.m);
    if (L.r < N && L.c <= L.r) p[(int64_t)(N + sidx(L.r, L.c)) * n] = R(x.P);
}

// whole elements through LDS (words-major, 16 entries each) and the workspace
template <int W>
__device__ __forceinline__ void put_words(double* dst, const double* w, int lane16) {
#pragma unroll
    for (int k = 0; k < W; ++k) dst[k * 16 + lane16] = w[k];
}
template <int W>
__device__ __forceinline__ void get_words(const double* src, double* w, int lane16) {
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = src[k * 16 + lane16];
}

// Wait until workgroup w's aggregate is published; false after kTopSpin polls.
__device__ __forceinline__ bool wait_published(int* flag) {
    for (int it = 0; it < kTopSpin; ++it) {
        if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

struct TopArgs {
    const void* items;   // SoA per-wave aggregates [words][n]
    int64_t n;
    void* carry;         // SoA moments [words][n]: prefix (suffix) of every item
    int E;               // items per group
    int nwg;             // workgroups (<= kTopMaxWg)
    double* wg_agg;      // [kTopMaxWg][6 words][16]: published workgroup aggregates
    int* flags;          // [0]: ticket counter; [1 + w]: aggregate of workgroup w published
    const int* model_fail;
    int nmodels;
    int* status;         // numeric flag; sequence 0 is reported if a published aggregate never arrives
};

// The published aggregate of workgroup src (waiting for its flag), or the
// identity when `use` is false.  A flag that never arrives is reported on the
// numeric flag (sequence 0) and the identity is used.
template <typename T>
__device__ __forceinline__ void fetch_published(const TopArgs& t, int src, bool use, int lane16, const Lanes& L,
                                                T& y) {
    constexpr int W = sizeof(T) / sizeof(double);
    if (use && wait_published(&t.flags[1 + src])) {
        get_words<W>(t.wg_agg + (int64_t)src * W * 16, reinterpret_cast<double*>(&y), lane16);
    } else {
        ident(y, L);
        if (use && lane16 == 0) atomicMin(t.status, 0);
    }
}

// Kogge-Stone over the groups of the workgroup through LDS `sh`
// ([kTopGroups][W words][16]); FWD: x_G <- x_{G-d} (x) x_G, else
// x_G <- x_G (x) x_{G+d}.  `levels` distances 1, 2, 4, ... (uniform).
template <typename T, int W, bool FWD, typename Comb>
__device__ __forceinline__ void group_scan(T& x, double* sh, int grp, int lane16, int levels, const Lanes& L,
                                           Comb comb) {
    for (int lv = 0, d = 1; lv < levels; ++lv, d <<= 1) {
        __syncthreads();
        put_words<W>(sh + grp * W * 16, reinterpret_cast<const double*>(&x), lane16);
        __syncthreads();
        const int src = FWD ? grp - d : grp + d;
        T y;
        if (src >= 0 && src < kTopGroups) get_words<W>(sh + src * W * 16, reinterpret_cast<double*>(&y), lane16);
        else ident(y, L);
        if (FWD) comb(y, x, x);
        else comb(x, y, x);
    }
}

// groups of workgroup w that hold items (the rest hold identities)
__device__ __forceinline__ int groups_used(const TopArgs& t, int w) {
    const int64_t left = t.n - (int64_t)w * kTopGroups * t.E;
    const int64_t g = (left + t.E - 1) / t.E;
    return g < kTopGroups ? (int)g : kTopGroups;
}

__device__ __forceinline__ int levels_for(int n) {
    int lv = 0;
    while ((1 << lv) < n) ++lv;
    return lv;
}

// ---------------------------------------------------------------------------
// FILTER: carry[i] = moments of items 0 .. i-1
// ---------------------------------------------------------------------------
template <int N, typename R, bool G>
__global__ __launch_bounds__(kTopThreads) void k_filter_top(TopArgs t) {
    __shared__ double sh[kTopGroups * kEFWords * 16];
    __shared__ double shm[2 * 16];
    __shared__ int ticket;
    const int tid = threadIdx.x, lane = tid & 63;
    const Lanes L = lanes_of(lane);
    const int grp = (tid >> 6) * 4 + (L.g4 >> 2);   // element (group) index within the workgroup
    const int lane16 = 4 * L.r + L.c;               // entry of this lane within its element
    if (tid == 0) ticket = atomicAdd(&t.flags[0], 1);
    __syncthreads();
    if (ticket >= t.nwg) {   // counter not cleared: report, touch nothing
        if (tid == 0) atomicMin(t.status, 0);
        return;
    }
    const int w = ticket;
    if (w == 0)
        for (int b = tid; b < t.nmodels; b += kTopThreads)
            if (t.model_fail[b]) atomicMin(t.status, b);
    auto comb = [&](const EF& a, const EF& b, EF& o) { epl_fcombine<G>(a, b, o, L); };
    // fold this group's items.  Loops run E times in every group (items past n
    // are identities), so the lane exchanges and matrix-core products inside
    // the combines always see the whole wave.
    const int64_t i0 = ((int64_t)w * kTopGroups + grp) * t.E;
    EF x;
    if (i0 < t.n) load_ef<N, R>(t.items, t.n, i0, L, x);
    else ident(x, L);
    for (int k = 1; k < t.E; ++k) {
        EF y;
        if (i0 + k < t.n) load_ef<N, R>(t.items, t.n, i0 + k, L, y);
        else ident(y, L);
        comb(x, y, x);
    }
    // groups past `used` hold identities and come last: fewer levels suffice,
    // and the workgroup aggregate is the inclusive scan of the last used group
    const int used = groups_used(t, w);
    group_scan<EF, kEFWords, true>(x, sh, grp, lane16, levels_for(used), L, comb);
    if (grp == used - 1) {
        put_words<kEFWords>(t.wg_agg + (int64_t)w * kEFWords * 16, reinterpret_cast<const double*>(&x), lane16);
        __threadfence();
        if (lane16 == 0) __hip_atomic_store(&t.flags[1 + w], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // this group's exclusive prefix within the workgroup
    __syncthreads();
    put_words<kEFWords>(sh + grp * kEFWords * 16, reinterpret_cast<const double*>(&x), lane16);
    __syncthreads();
    EF ex;
    if (grp > 0) get_words<kEFWords>(sh + (grp - 1) * kEFWords * 16, reinterpret_cast<double*>(&ex), lane16);
    else ident(ex, L);
    // look-back: the aggregates of workgroups 0 .. w-1, scanned across the groups
    EM X;
    X.m = X.P = 0.0;
    if (w > 0) {
        // group G folds the aggregates of workgroups G eb .. G eb + eb - 1 (< w)
        const int eb = (w + kTopGroups - 1) / kTopGroups, lb_used = (w + eb - 1) / eb;
        EF a;
        for (int k = 0; k < eb; ++k) {
            const int src = grp * eb + k;
            EF y;
            fetch_published(t, src, src < w, lane16, L, y);
            if (k == 0) a = y;
            else comb(a, y, a);
        }
        group_scan<EF, kEFWords, true>(a, sh, grp, lane16, levels_for(lb_used), L, comb);
        // the prefix contains step 1 (A = 0): its moments are b, C
        if (grp == lb_used - 1) {
            shm[lane16] = a.b;
            shm[16 + lane16] = a.C;
        }
        __syncthreads();
        X.m = shm[lane16];
        X.P = shm[16 + lane16];
    }
    epl_fcarry<G>(X, ex, L);
    for (int k = 0; k < t.E; ++k) {
        const int64_t i = i0 + k;
        if (i < t.n) store_em<N, R>(t.carry, t.n, i, L, X);
        if (k + 1 < t.E) {
            EF y;
            if (i < t.n) load_ef<N, R>(t.items, t.n, i, L, y);
            else ident(y, L);
            epl_fcarry<G>(X, y, L);
        }
    }
}

// ---------------------------------------------------------------------------
// SMOOTHER: carry[i] = moments of items i+1 .. n-1 (suffix; E of the product is 0)
// ---------------------------------------------------------------------------
template <int N, typename R, bool G>
__global__ __launch_bounds__(kTopThreads) void k_smoother_top(TopArgs t) {
    __shared__ double sh[kTopGroups * kESWords * 16];
    __shared__ double shm[2 * 16];
    __shared__ int ticket;
    const int tid = threadIdx.x, lane = tid & 63;
    const Lanes L = lanes_of(lane);
    const int grp = (tid >> 6) * 4 + (L.g4 >> 2);   // element (group) index within the workgroup
    const int lane16 = 4 * L.r + L.c;               // entry of this lane within its element
    if (tid == 0) ticket = atomicAdd(&t.flags[0], 1);
    __syncthreads();
    if (ticket >= t.nwg) {
        if (tid == 0) atomicMin(t.status, 0);
        return;
    }
    const int w = t.nwg - 1 - ticket;   // the last workgroup starts first
    auto comb = [&](const ES& a, const ES& b, ES& o) { epl_scombine<G>(a, b, o, L); };
    const int64_t i0 = ((int64_t)w * kTopGroups + grp) * t.E;
    ES x;
    if (i0 + t.E - 1 < t.n) load_es<N, R>(t.items, t.n, i0 + t.E - 1, L, x);
    else ident(x, L);
    for (int k = t.E - 2; k >= 0; --k) {
        ES y;
        if (i0 + k < t.n) load_es<N, R>(t.items, t.n, i0 + k, L, y);
        else ident(y, L);
        comb(y, x, x);
    }
    // identities past `used`: the suffix of group 0 needs levels_for(used) levels
    const int used = groups_used(t, w);
    group_scan<ES, kESWords, false>(x, sh, grp, lane16, levels_for(used), L, comb);
    if (grp == 0) {
        put_words<kESWords>(t.wg_agg + (int64_t)w * kESWords * 16, reinterpret_cast<const double*>(&x), lane16);
        __threadfence();
        if (lane16 == 0) __hip_atomic_store(&t.flags[1 + w], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    put_words<kESWords>(sh + grp * kESWords * 16, reinterpret_cast<const double*>(&x), lane16);
    __syncthreads();
    ES ex;
    if (grp < kTopGroups - 1) get_words<kESWords>(sh + (grp + 1) * kESWords * 16, reinterpret_cast<double*>(&ex), lane16);
    else ident(ex, L);
    // look-back: the aggregates of workgroups w+1 .. nwg-1 (group G holds w+1+G)
    EM X;
    X.m = X.P = 0.0;
    const int after = t.nwg - 1 - w;
    if (after > 0) {
        // group G folds the aggregates of workgroups w + 1 + G eb .. (+ eb - 1, < nwg)
        const int eb = (after + kTopGroups - 1) / kTopGroups, lb_used = (after + eb - 1) / eb;
        ES a;
        for (int k = eb - 1; k >= 0; --k) {
            const int off = grp * eb + k;
            ES y;
            fetch_published(t, w + 1 + off, off < after, lane16, L, y);
            if (k == eb - 1) a = y;
            else comb(y, a, a);
        }
        group_scan<ES, kESWords, false>(a, sh, grp, lane16, levels_for(lb_used), L, comb);
        // the suffix contains the last step (E = 0): its moments are g, L
        if (grp == 0) {
            shm[lane16] = a.g;
            shm[16 + lane16] = a.L;
        }
        __syncthreads();
        X.m = shm[lane16];
        X.P = shm[16 + lane16];
    }
    epl_scarry<G>(ex, X, L);
    for (int k = t.E - 1; k >= 0; --k) {
        const int64_t i = i0 + k;
        if (i < t.n) store_em<N, R>(t.carry, t.n, i, L, X);
        if (k > 0) {
            ES y;
            if (i < t.n) load_es<N, R>(t.items, t.n, i, L, y);
            else ident(y, L);
            epl_scarry<G>(y, X, L);
        }
    }
}

}  // namespace
}  // namespace pks
