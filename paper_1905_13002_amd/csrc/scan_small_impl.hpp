// scan_small_impl.hpp -- the filtering and smoothing scans for nx <= 4, one scan
// element per lane, elements in registers.
//
// The all-prefix-sums of the filtering elements (Theorem 1) and the suffix
// products of the smoothing elements (Theorem 2) are computed as a
// reduce-then-scan over block-level elements (the paper's blocks of length l,
// Section III-C):
//   reduce : thread t folds its EPT consecutive elements sequentially into one
//            block element; the 64 block elements of a wave are scanned with a
//            Kogge-Stone pattern over cross-lane shuffles (six combines); each
//            thread stores its in-wave exclusive prefix and lane 63 the wave
//            aggregate (struct-of-arrays in the workspace).
//   top    : a device-wide scan of the wave aggregates (top_epl.hpp: up to
//            64 workgroups with one element per 16 lanes, a look-back over
//            the published workgroup aggregates) stores, per wave, the
//            moments of everything before it.  Optionally one more level
//            (the same reduce over the wave aggregates) is inserted when the
//            number of waves is large.
//   down   : thread t applies the wave's incoming moments to its exclusive
//            prefix and then re-folds its EPT elements one by one; every
//            step of that fold is Lemma 2 (or 4) with a left prefix whose A
//            is zero (a right suffix whose E is zero), i.e. an exact Kalman
//            update+prediction (RTS step) in element form, whose moments are
//            the outputs.
// Every prefix that starts at a sequence's first step has A = 0 (Lemma 1,
// A_1 = 0) and every suffix that ends at a sequence's last step has E = 0
// (Lemma 3, E_n = 0); these exact zeros also separate sequences that are
// packed back to back, so batched scans need no segment flags.
#pragma once
#include "pks_internal.h"
#include "small_ops.hpp"
#include "top_epl.hpp"

namespace pks {

namespace {

constexpr int kBlock = 256;     // threads per workgroup (4 waves)

// ---------------------------------------------------------------------------
// struct-of-arrays helpers: record word w of item i lives at base[w*stride+i]
// ---------------------------------------------------------------------------
template <int W, typename R>
__device__ __forceinline__ void soa_store_words(R* __restrict__ base, int64_t stride, int64_t i, const R* w) {
#pragma unroll
    for (int k = 0; k < W; ++k) base[k * stride + i] = w[k];
}
template <int W, typename R>
__device__ __forceinline__ void soa_load_words(const R* __restrict__ base, int64_t stride, int64_t i, R* w) {
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = base[k * stride + i];
}

template <int N, typename R>
__device__ __forceinline__ void store_f(void* base, int64_t stride, int64_t i, const FElem<N, R>& e) {
    soa_store_words<Words<N>::F>(static_cast<R*>(base), stride, i, reinterpret_cast<const R*>(&e));
}
template <int N, typename R>
__device__ __forceinline__ void load_f(const void* base, int64_t stride, int64_t i, FElem<N, R>& e) {
    soa_load_words<Words<N>::F>(static_cast<const R*>(base), stride, i, reinterpret_cast<R*>(&e));
}
template <int N, typename R>
__device__ __forceinline__ void store_s(void* base, int64_t stride, int64_t i, const SElem<N, R>& e) {
    soa_store_words<Words<N>::S>(static_cast<R*>(base), stride, i, reinterpret_cast<const R*>(&e));
}
template <int N, typename R>
__device__ __forceinline__ void load_s(const void* base, int64_t stride, int64_t i, SElem<N, R>& e) {
    soa_load_words<Words<N>::S>(static_cast<const R*>(base), stride, i, reinterpret_cast<R*>(&e));
}
template <int N, typename R>
__device__ __forceinline__ void store_m(void* base, int64_t stride, int64_t i, const Moments<N, R>& x) {
    soa_store_words<Words<N>::M>(static_cast<R*>(base), stride, i, reinterpret_cast<const R*>(&x));
}
template <int N, typename R>
__device__ __forceinline__ void load_m(const void* base, int64_t stride, int64_t i, Moments<N, R>& x) {
    soa_load_words<Words<N>::M>(static_cast<const R*>(base), stride, i, reinterpret_cast<R*>(&x));
}

// cross-lane moves of whole records
template <int W, typename R>
__device__ __forceinline__ void shfl_up_words(R* w, unsigned d) {
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = __shfl_up(w[k], d, 64);
}
template <int W, typename R>
__device__ __forceinline__ void shfl_down_words(R* w, unsigned d) {
#pragma unroll
    for (int k = 0; k < W; ++k) w[k] = __shfl_down(w[k], d, 64);
}

// ---------------------------------------------------------------------------
// sequences: which packed sequence holds step k
// ---------------------------------------------------------------------------
struct Seq {
    int b;
    int64_t start, end;   // [start, end)
};

template <bool SEG>
__device__ __forceinline__ Seq seq_find(const ScanArgs& a, int64_t k) {
    Seq s;
    if (!SEG) {
        s.b = 0; s.start = 0; s.end = a.total;
        return s;
    }
    int lo = 0, hi = a.B;               // invariant: offsets[lo] <= k (offsets[0] = 0)
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
__device__ __forceinline__ void seq_forward(const ScanArgs& a, Seq& s, int64_t k) {
    if (!SEG) return;
    while (k >= s.end && s.b < a.B - 1) {
        ++s.b;
        s.start = s.end;
        s.end = a.offsets[s.b + 1];
    }
}
template <bool SEG>
__device__ __forceinline__ void seq_backward(const ScanArgs& a, Seq& s, int64_t k) {
    if (!SEG) return;
    while (k < s.start && s.b > 0) {
        --s.b;
        s.end = s.start;
        s.start = a.offsets[s.b];
    }
}

// ---------------------------------------------------------------------------
// element sources
// ---------------------------------------------------------------------------
// Lemma 1 element of step k (first = first step of its sequence).
template <int N, typename R>
__device__ __forceinline__ void build_felem(const R* __restrict__ cst, const ConstLayout& CL, int ny,
                                            const R* __restrict__ yk, bool first, FElem<N, R>& e) {
    if (!first) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
#pragma unroll
            for (int c = 0; c < N; ++c) e.A[r * N + c] = cst[CL.A + r * N + c];
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                e.C[sidx(r, c)] = cst[CL.C + r * N + c];
                e.J[sidx(r, c)] = cst[CL.J + r * N + c];
            }
            e.b[r] = cst[CL.c + r];
            e.eta[r] = cst[CL.w + r];
        }
        for (int q = 0; q < ny; ++q) {
            const R yq = yk[q];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                e.b[r] = fma(cst[CL.K + r * ny + q], yq, e.b[r]);
                e.eta[r] = fma(cst[CL.W + r * ny + q], yq, e.eta[r]);
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < N; ++r) {
#pragma unroll
            for (int c = 0; c < N; ++c) e.A[r * N + c] = R(0);
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                e.C[sidx(r, c)] = cst[CL.C1 + r * N + c];
                e.J[sidx(r, c)] = R(0);
            }
            e.b[r] = cst[CL.c1 + r];
            e.eta[r] = R(0);
        }
        for (int q = 0; q < ny; ++q) {
            const R yq = yk[q];
#pragma unroll
            for (int r = 0; r < N; ++r) e.b[r] = fma(cst[CL.K1 + r * ny + q], yq, e.b[r]);
        }
    }
}

// With ny = M < nx (M > 0) the measurement of a step is read into registers
// one step ahead (YV words), so that its load overlaps the previous step's
// arithmetic; otherwise (M = 0, any ny) the element reads y_k where it is
// stored.
template <int M> struct YV { static constexpr int n = M > 0 ? M : 1; };
template <int M, typename R>
__device__ __forceinline__ void load_y(const R* __restrict__ y, int64_t k, R (&v)[YV<M>::n]) {
    if constexpr (M > 0) {
#pragma unroll
        for (int q = 0; q < M; ++q) v[q] = y[k * M + q];
    }
}
template <int N, typename R, int M>
__device__ __forceinline__ void build_felem_step(const R* __restrict__ cst, const ConstLayout& CL, int ny,
                                                 const R* __restrict__ y, int64_t k, const R (&yv)[YV<M>::n],
                                                 bool first, FElem<N, R>& e) {
    if constexpr (M > 0) {
        // the same arithmetic as build_felem with y_k from registers
        build_felem<N, R>(cst, CL, 0, y, first, e);   // ny = 0: the y-free part
        if (!first) {
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    e.b[r] = fma(cst[CL.K + r * M + q], yv[q], e.b[r]);
                    e.eta[r] = fma(cst[CL.W + r * M + q], yv[q], e.eta[r]);
                }
        } else {
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int r = 0; r < N; ++r) e.b[r] = fma(cst[CL.K1 + r * M + q], yv[q], e.b[r]);
        }
    } else {
        build_felem<N, R>(cst, CL, ny, y + k * ny, first, e);
    }
}

template <int N, typename R>
__device__ __forceinline__ void load_moments_step(const R* __restrict__ m, const R* __restrict__ P, int64_t k,
                                                  Moments<N, R>& x) {
#pragma unroll
    for (int r = 0; r < N; ++r) x.m[r] = m[k * N + r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) x.P[sidx(r, c)] = P[k * N * N + r * N + c];
}

// the filtered covariance of step k (lower triangle)
template <int N, typename R>
__device__ __forceinline__ void load_cov_step(const R* __restrict__ P, int64_t k, Moments<N, R>& x) {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) x.P[sidx(r, c)] = P[k * N * N + r * N + c];
}

template <int N, typename R>
__device__ __forceinline__ void store_moments_step(R* __restrict__ m, R* __restrict__ P, int64_t k,
                                                   const Moments<N, R>& x) {
#pragma unroll
    for (int r = 0; r < N; ++r) m[k * N + r] = x.m[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) P[k * N * N + r * N + c] = x.P[sidx(r, c)];
}

// Lemma 3 element of step k from its filtered moments (last = last step of its sequence)
template <int N, typename R>
__device__ __forceinline__ void make_selem(const R* __restrict__ cst, const ConstLayout& CL, const Moments<N, R>& x,
                                           bool last, SElem<N, R>& e, int* status, int b) {
    if (last) {
#pragma unroll
        for (int i = 0; i < N * N; ++i) e.E[i] = R(0);
#pragma unroll
        for (int i = 0; i < N; ++i) e.g[i] = x.m[i];
#pragma unroll
        for (int i = 0; i < tri(N); ++i) e.L[i] = x.P[i];
    } else {
        const bool ok = build_selem<N, R>(cst + CL.F, cst + CL.Q, cst + CL.u, x, e);
        if (!ok) atomicMin(status, b);
    }
}


// Lemma 3 element from explicit F, Q, u pointers (constants staged in LDS)
template <int N, typename R>
__device__ __forceinline__ void make_selem_p(const R* F, const R* Q, const R* u, const Moments<N, R>& x, bool last,
                                             SElem<N, R>& e, int* status, int b) {
    if (last) {
#pragma unroll
        for (int i = 0; i < N * N; ++i) e.E[i] = R(0);
#pragma unroll
        for (int i = 0; i < N; ++i) e.g[i] = x.m[i];
#pragma unroll
        for (int i = 0; i < tri(N); ++i) e.L[i] = x.P[i];
    } else {
        const bool ok = build_selem<N, R>(F, Q, u, x, e);
        if (!ok) atomicMin(status, b);
    }
}

// ---------------------------------------------------------------------------
// One shared model (a single time-invariant sequence): every step has the
// same constants.  The step loops of the down-sweeps also store outputs, so
// the compiler cannot prove constants read from global memory invariant and
// re-reads them with vector memory instructions at every step; instead they
// are copied to LDS once per workgroup and read from there.  The filter
// stages its constants [0, F) when the rank-ny form applies (ny < nx <= 4,
// at most 156 words), the smoother the copies of F, Q, u (2 nx^2 + nx words).
// ---------------------------------------------------------------------------
constexpr int kStageF = 160;
template <int N>
struct StageS {
    static constexpr int words = 2 * N * N + N;
};
template <int N, typename R>
__device__ __forceinline__ void stage_filter_consts(const ScanArgs& a, const ConstLayout& CL, R* csh, double* ssh) {
    const R* g = static_cast<const R*>(a.consts);
    for (int i = threadIdx.x; i < CL.F; i += blockDim.x) csh[i] = g[i];
    for (int i = threadIdx.x; i < a.ny * a.ny; i += blockDim.x) ssh[i] = a.consts64[CL.S + i];
}
template <int N, typename R>
__device__ __forceinline__ void stage_smoother_consts(const ScanArgs& a, const ConstLayout& CL, R* fsh) {
    const R* g = static_cast<const R*>(a.consts);
    for (int i = threadIdx.x; i < StageS<N>::words; i += blockDim.x) fsh[i] = g[CL.F + i];
}

// ---------------------------------------------------------------------------
// Wave-cooperative moment transfers.  Lane l of a wave handles step
// kbase + l * stride; a direct per-lane access of its moments would touch a
// different cache line in every lane of every memory instruction.  Instead the
// 64 records pass through an LDS slice of the wave and are moved with
// consecutive lanes on consecutive units of the same record, so a memory
// instruction covers a few whole records.
// ---------------------------------------------------------------------------
template <int Bytes> struct UnitT;
template <> struct UnitT<16> { using T = unsigned int __attribute__((ext_vector_type(4))); };
template <> struct UnitT<8> { using T = unsigned int __attribute__((ext_vector_type(2))); };
template <> struct UnitT<4> { using T = unsigned int; };

template <int N, typename R>
struct MomStage {
    static constexpr int WM = N, WP = N * N;                         // words of m and of P
    static constexpr int BM = WM * (int)sizeof(R), BP = WP * (int)sizeof(R);
    // consecutive steps of one lane buffered before a write, so that a lane's
    // run of records fills whole 128-byte lines when the record divides 128
    static constexpr int GM = (128 % BM == 0 && BM < 128) ? 128 / BM : 1;
    static constexpr int GP = (128 % BP == 0 && BP < 128) ? 128 / BP : 1;
    static constexpr int UBP = (WP * sizeof(R)) % 16 == 0 ? 16 : ((WP * sizeof(R)) % 8 == 0 ? 8 : 4);
    static constexpr int UBM = (WM * sizeof(R)) % 16 == 0 ? 16 : ((WM * sizeof(R)) % 8 == 0 ? 8 : 4);
    static constexpr int UP = BP / UBP;                                 // units per P record
    static constexpr int UM = BM / UBM;                                 // units per m record
    // words per lane row, padded to an odd count so that lanes writing their
    // own rows fall into distinct LDS banks
    static constexpr int ROWM = GM * WM + ((GM * WM) % 2 == 0 ? 1 : 0);
    static constexpr int ROWP = GP * WP + ((GP * WP) % 2 == 0 ? 1 : 0);
    static constexpr int ROW = WP + WM + 1;                             // load stage row (padded)
    static constexpr int WORDS_LOAD = 64 * ROW;
    static constexpr int WORDS = 64 * (ROWM + ROWP) > WORDS_LOAD ? 64 * (ROWM + ROWP) : WORDS_LOAD;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// write the G buffered records of every lane: lane l's records are steps
// kfirst + l * stride .. + G - 1 (contiguous in memory), `rec_words` R words
// each, held in the stage at row l (ROW words per row)
template <int G, int U, int UB, int ROW, typename R>
__device__ __forceinline__ void wave_flush(R* __restrict__ dst, const R* st, int rec_words, int64_t kfirst,
                                           int64_t stride, int64_t total, int lane, int filled) {
    using UT = typename UnitT<UB>::T;
    constexpr int PER = G * U;                       // units per lane
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int f = lane + 64 * i, l = f / PER, v = f % PER, s = v / U;
        const int64_t k = kfirst + (int64_t)l * stride + s;
        if (s < filled && k < total) {
            UT val;
            __builtin_memcpy(&val, reinterpret_cast<const char*>(st + l * ROW) + v * UB, UB);
            // streaming store: the outputs are not read again by this kernel,
            // so they should not push out the input lines that still are
            __builtin_nontemporal_store(val, reinterpret_cast<UT*>(dst + (kfirst + (int64_t)l * stride) * rec_words) + v);
        }
    }
}

// Buffer this lane's moments of iteration e (step kw + lane * stride + e) and
// write the buffered runs when a run is complete or the loop ends.
template <int N, typename R>
__device__ __forceinline__ void wave_store_moments(R* __restrict__ m, R* __restrict__ P, int64_t kw, int e, int last_e,
                                                   int64_t stride, int64_t total, R* st, int lane,
                                                   const Moments<N, R>& x) {
    using S = MomStage<N, R>;
    R* sm = st;                       // [64][GM][N]
    R* sp = st + 64 * S::ROWM;        // [64][GP][N*N]
    R* rm = sm + lane * S::ROWM + (e % S::GM) * N;
    R* rp = sp + lane * S::ROWP + (e % S::GP) * (N * N);
#pragma unroll
    for (int r = 0; r < N; ++r) rm[r] = x.m[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) rp[r * N + c] = x.P[sidx(r, c)];
    const bool fm = (e % S::GM == S::GM - 1) || e == last_e;
    const bool fp = (e % S::GP == S::GP - 1) || e == last_e;
    if (fm || fp) wave_sync();
    if (fm) wave_flush<S::GM, S::UM, S::UBM, S::ROWM, R>(m, sm, N, kw + e - e % S::GM, stride, total, lane, e % S::GM + 1);
    if (fp) wave_flush<S::GP, S::UP, S::UBP, S::ROWP, R>(P, sp, N * N, kw + e - e % S::GP, stride, total, lane, e % S::GP + 1);
    if (fm || fp) wave_sync();
}

// the inverse of wave_flush: read the G records of every lane (steps
// kfirst + l * stride .. + G - 1, contiguous) into its stage row, whole lines
// per instruction; records at or beyond total read as zero
template <int G, int U, int UB, int ROW, typename R>
__device__ __forceinline__ void wave_fill(const R* __restrict__ src, R* st, int rec_words, int64_t kfirst,
                                          int64_t stride, int64_t total, int lane) {
    using UT = typename UnitT<UB>::T;
    constexpr int PER = G * U;                       // units per lane
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int f = lane + 64 * i, l = f / PER, v = f % PER, s = v / U;
        const int64_t k = kfirst + (int64_t)l * stride + s;
        UT val{};
        if (k < total) val = reinterpret_cast<const UT*>(src + (kfirst + (int64_t)l * stride) * rec_words)[v];
        __builtin_memcpy(reinterpret_cast<char*>(st + l * ROW) + v * UB, &val, UB);
    }
}

// reverse-order variant (the smoother produces steps from the last to the
// first): iteration e runs EPT-1 .. 0, so a run is complete at e % G == 0
template <int N, typename R>
__device__ __forceinline__ void wave_store_moments_rev(R* __restrict__ m, R* __restrict__ P, int64_t kw, int e,
                                                       int ept, int64_t stride, int64_t total, R* st, int lane,
                                                       const Moments<N, R>& x) {
    using S = MomStage<N, R>;
    R* sm = st;
    R* sp = st + 64 * S::ROWM;
    R* rm = sm + lane * S::ROWM + (e % S::GM) * N;
    R* rp = sp + lane * S::ROWP + (e % S::GP) * (N * N);
#pragma unroll
    for (int r = 0; r < N; ++r) rm[r] = x.m[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) rp[r * N + c] = x.P[sidx(r, c)];
    const bool fm = e % S::GM == 0;
    const bool fp = e % S::GP == 0;
    if (fm || fp) wave_sync();
    // the run written here is steps e .. min(e + G, ept) - 1 of every lane
    if (fm) wave_flush<S::GM, S::UM, S::UBM, S::ROWM, R>(m, sm, N, kw + e, stride, total, lane, min(S::GM, ept - e));
    if (fp) wave_flush<S::GP, S::UP, S::UBP, S::ROWP, R>(P, sp, N * N, kw + e, stride, total, lane, min(S::GP, ept - e));
    if (fm || fp) wave_sync();
}

// load this lane's moments (step kbase + lane * stride; zeros beyond total)
template <int N, typename R>
__device__ __forceinline__ void wave_load_moments(const R* __restrict__ m, const R* __restrict__ P, int64_t kbase,
                                                  int64_t stride, int64_t total, R* st, int lane, Moments<N, R>& x) {
    using S = MomStage<N, R>;
    using UP_T = typename UnitT<S::UBP>::T;
    using UM_T = typename UnitT<S::UBM>::T;
#pragma unroll
    for (int i = 0; i < S::UP; ++i) {
        const int f = lane + 64 * i, l = f / S::UP, u = f % S::UP;
        const int64_t k = kbase + (int64_t)l * stride;
        UP_T v{};
        if (k < total) v = reinterpret_cast<const UP_T*>(P + k * S::WP)[u];
        __builtin_memcpy(reinterpret_cast<char*>(st + l * S::ROW + N) + u * S::UBP, &v, S::UBP);
    }
#pragma unroll
    for (int i = 0; i < S::UM; ++i) {
        const int f = lane + 64 * i, l = f / S::UM, u = f % S::UM;
        const int64_t k = kbase + (int64_t)l * stride;
        UM_T v{};
        if (k < total) v = reinterpret_cast<const UM_T*>(m + k * S::WM)[u];
        __builtin_memcpy(reinterpret_cast<char*>(st + l * S::ROW) + u * S::UBM, &v, S::UBM);
    }
    wave_sync();
    const R* row = st + lane * S::ROW;
#pragma unroll
    for (int r = 0; r < N; ++r) x.m[r] = row[r];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) x.P[sidx(r, c)] = row[N + r * N + c];
    wave_sync();
}

// ---------------------------------------------------------------------------
// wave-level scans (Kogge-Stone over shuffles).  Lanes without a partner take
// the identity as the shuffled operand, so every lane runs the same combine.
// ---------------------------------------------------------------------------
// `lim`: a power of two >= the number of lanes that hold a real element (the
// others hold the identity), so fewer levels suffice when few lanes are used.
template <int N, typename R, bool G>
__device__ __forceinline__ void wave_inclusive_f(FElem<N, R>& incl, int lane, int lim = 64) {
#pragma unroll 1
    for (int d = 1; d < lim; d <<= 1) {
        FElem<N, R> o = incl;
        shfl_up_words<Words<N>::F>(reinterpret_cast<R*>(&o), d);
        if (lane >= d) fcombine<N, R, G>(o, incl, incl);
    }
}
template <int N, typename R>
__device__ __forceinline__ void wave_exclusive_from_inclusive_f(const FElem<N, R>& incl, FElem<N, R>& ex, int lane) {
    ex = incl;
    shfl_up_words<Words<N>::F>(reinterpret_cast<R*>(&ex), 1);
    if (lane == 0) set_identity(ex);
}
template <int N, typename R, bool G>
__device__ __forceinline__ void wave_inclusive_suffix_s(SElem<N, R>& incl, int lane, int lim = 64) {
#pragma unroll 1
    for (int d = 1; d < lim; d <<= 1) {
        SElem<N, R> o = incl;
        shfl_down_words<Words<N>::S>(reinterpret_cast<R*>(&o), d);
        if (lane + d < 64) scombine<N, R, G>(incl, o, incl);
    }
}
template <int N, typename R>
__device__ __forceinline__ void wave_exclusive_suffix_s(const SElem<N, R>& incl, SElem<N, R>& ex, int lane) {
    ex = incl;
    shfl_down_words<Words<N>::S>(reinterpret_cast<R*>(&ex), 1);
    if (lane == 63) set_identity(ex);
}

// The top level's workgroups draw tickets and publish flags that must start
// at zero: the kernel that runs just before each top level (a reduce kernel)
// clears them.
__device__ __forceinline__ void clear_top_flags(const ScanArgs& a) {
    if (blockIdx.x == 0 && threadIdx.x <= kTopMaxWg) a.top_flags[threadIdx.x] = 0;
}

// ===========================================================================
// FILTER
// ===========================================================================
// load G = H F (zero for a sequence's first step, whose J is 0)
template <int N, int M, typename R>
__device__ __forceinline__ void load_gz(const R* __restrict__ cst, const ConstLayout& CL, bool first, R (&Gz)[M * N]) {
#pragma unroll
    for (int i = 0; i < M * N; ++i) Gz[i] = first ? R(0) : cst[CL.G + i];
}

// reduce over steps (elements built from y).  M = ny when ny < nx: the
// single-step elements are folded with the rank-ny form of Lemma 2.
template <int N, typename R, int EPT, bool SEG, int M>
__global__ __launch_bounds__(kBlock) void k_filter_reduce(ScanArgs a) {
    clear_top_flags(a);
    // one shared model with the rank-ny form: constants from an LDS copy (the
    // first-step choice differs between lanes, and the constants read under it
    // would otherwise be vector loads from global memory at every step)
    constexpr bool STG = !SEG && M > 0;
    __shared__ R csh[STG ? kStageF : 1];
    __shared__ double ssh[STG ? 16 : 1];
    const ConstLayout CL = const_layout(N, a.ny);
    if constexpr (STG) {
        stage_filter_consts<N, R>(a, CL, csh, ssh);
        __syncthreads();
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t k0 = gt * EPT;
    const R* y = static_cast<const R*>(a.y);
    FElem<N, R> acc;
    set_identity(acc);
    if (k0 < a.total) {
        Seq s = seq_find<SEG>(a, k0);
        constexpr int MY = sizeof(R) == 8 ? M : 0;   // FP32 storage: read y in place (measured faster)
        R yv[YV<MY>::n];
        load_y<MY>(y, k0, yv);
#pragma unroll 1
        for (int e = 0; e < EPT; ++e) {
            const int64_t k = k0 + e;
            if (k < a.total) {
                R yn[YV<MY>::n];
                load_y<MY>(y, k + 1 < a.total ? k + 1 : k, yn);
                seq_forward<SEG>(a, s, k);
                const int64_t moff = const_offset<SEG>(a, s.b, k);
                const R* cst;
                const double* Sp;
                if constexpr (STG) {
                    cst = csh;
                    Sp = ssh;
                } else {
                    cst = static_cast<const R*>(a.consts) + moff;
                    Sp = a.consts64 + moff + CL.S;
                }
                const bool first = k == s.start;
                FElem<N, R> x;
                build_felem_step<N, R, MY>(cst, CL, a.ny, y, k, yv, first, x);
                if (e == 0) {
                    acc = x;
                } else if (M == 0) {
                    fcombine<N, R, SEG>(acc, x, acc);
                } else {
                    constexpr int MM = M > 0 ? M : 1;
                    R Gz[MM * N];
                    load_gz<N, MM, R>(cst, CL, first, Gz);
                    fcombine_fresh<N, MM, R, SEG>(acc, x, Gz, cst + CL.W, Sp);
                }
#pragma unroll
                for (int q = 0; q < YV<MY>::n; ++q) yv[q] = yn[q];
            }
        }
    }
    wave_inclusive_f<N, R, SEG>(acc, lane);
    FElem<N, R> ex;
    wave_exclusive_from_inclusive_f(acc, ex, lane);
    store_f(a.thr, a.nthr, gt, ex);
    if (lane == 63) store_f(a.agg, a.nwaves, gt >> 6, acc);
}

// reduce over explicit items (level 1: the level-0 wave aggregates)
template <int N, typename R, int EPT, bool G>
__global__ __launch_bounds__(kBlock) void k_filter_reduce_items(ScanArgs a) {
    clear_top_flags(a);
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t i0 = gt * EPT;
    FElem<N, R> acc;
    set_identity(acc);
#pragma unroll 1
    for (int e = 0; e < EPT; ++e) {
        const int64_t i = i0 + e;
        if (i < a.nwaves) {
            FElem<N, R> x;
            load_f(a.agg, a.nwaves, i, x);
            if (e == 0) acc = x;
            else fcombine<N, R, G>(acc, x, acc);
        }
    }
    wave_inclusive_f<N, R, G>(acc, lane);
    FElem<N, R> ex;
    wave_exclusive_from_inclusive_f(acc, ex, lane);
    store_f(a.thr1, a.nthr1, gt, ex);
    if (lane == 63) store_f(a.agg1, a.nwaves1, gt >> 6, acc);
}

// level-1 down: carries of the level-0 waves
template <int N, typename R, int EPT, bool G>
__global__ __launch_bounds__(kBlock) void k_filter_down_items(ScanArgs a) {
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i0 = gt * EPT;
    if (i0 >= a.nwaves) return;
    Moments<N, R> X;
    load_m(a.carry1, a.nwaves1, gt >> 6, X);
    FElem<N, R> pre;
    load_f(a.thr1, a.nthr1, gt, pre);
    fcarry<N, R, G>(X, pre);
#pragma unroll 1
    for (int e = 0; e < EPT; ++e) {
        const int64_t i = i0 + e;
        if (i < a.nwaves) {
            store_m(a.carry, a.nwaves, i, X);
            FElem<N, R> x;
            load_f(a.agg, a.nwaves, i, x);
            fcarry<N, R, G>(X, x);
        }
    }
}

// level-0 down: outputs m_k, P_k
template <int N, typename R, int EPT, bool SEG, int M>
__global__ __launch_bounds__(kBlock) void k_filter_down(ScanArgs a) {
    constexpr bool STG = !SEG && M > 0;
    __shared__ R stage[kBlock / 64][MomStage<N, R>::WORDS];
    __shared__ R csh[STG ? kStageF : 1];
    __shared__ double ssh[STG ? 16 : 1];
    const ConstLayout CL = const_layout(N, a.ny);
    if constexpr (STG) {
        stage_filter_consts<N, R>(a, CL, csh, ssh);
        __syncthreads();
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t k0 = gt * EPT;
    const int64_t kw = (gt - lane) * EPT;          // first step of the wave
    if (kw >= a.total) return;                     // whole wave beyond the end
    R* st = stage[threadIdx.x >> 6];
    const R* y = static_cast<const R*>(a.y);
    R* mo = static_cast<R*>(a.m);
    R* Po = static_cast<R*>(a.P);
    Moments<N, R> X;
    load_m(a.carry, a.nwaves, gt >> 6, X);
    {
        FElem<N, R> pre;
        load_f(a.thr, a.nthr, gt, pre);
        fcarry<N, R, SEG>(X, pre);
    }
    Seq s = seq_find<SEG>(a, k0 < a.total ? k0 : a.total - 1);
    constexpr int MY = sizeof(R) == 8 ? M : 0;   // FP32 storage: read y in place (measured faster)
    R yv[YV<MY>::n];
    load_y<MY>(y, k0 < a.total ? k0 : a.total - 1, yv);
#pragma unroll 1
    for (int e = 0; e < EPT; ++e) {
        const int64_t k = k0 + e;
        if (k < a.total) {
            R yn[YV<MY>::n];
            load_y<MY>(y, k + 1 < a.total ? k + 1 : k, yn);
            seq_forward<SEG>(a, s, k);
            const int64_t moff = const_offset<SEG>(a, s.b, k);
            const R* cst;
            const double* Sp;
            if constexpr (STG) {
                cst = csh;
                Sp = ssh;
            } else {
                cst = static_cast<const R*>(a.consts) + moff;
                Sp = a.consts64 + moff + CL.S;
            }
            const bool first = k == s.start;
            FElem<N, R> x;
            build_felem_step<N, R, MY>(cst, CL, a.ny, y, k, yv, first, x);
            if (M == 0) {
                fcarry<N, R, SEG>(X, x);
            } else {
                constexpr int MM = M > 0 ? M : 1;
                R Gz[MM * N];
                load_gz<N, MM, R>(cst, CL, first, Gz);
                fcarry_fresh<N, MM, R, SEG>(X, x, Gz, Sp);
            }
#pragma unroll
            for (int q = 0; q < YV<MY>::n; ++q) yv[q] = yn[q];
        }
        wave_store_moments<N, R>(mo, Po, kw, e, EPT - 1, EPT, a.total, st, lane, X);
    }
}

// Filter down-sweep fused with the smoother's reduce: the filtered moments of
// each step are still in registers, so the smoothing element (Lemma 3) is
// built and folded right away, and the smoother's per-thread prefixes and wave
// aggregates are written as by k_smoother_reduce (into the same workspace
// arrays: each thread reads its filter prefix before writing its smoother one).
template <int N, typename R, int EPT, bool SEG, int M>
__global__ __launch_bounds__(kBlock) void k_filter_down_smooth_reduce(ScanArgs a) {
    clear_top_flags(a);
    constexpr bool STG = !SEG && M > 0;
    __shared__ R stage[kBlock / 64][MomStage<N, R>::WORDS];
    __shared__ R csh[STG ? kStageF : 1];
    __shared__ double ssh[STG ? 16 : 1];
    __shared__ R fsh[STG ? StageS<N>::words : 1];
    const ConstLayout CL = const_layout(N, a.ny);
    if constexpr (STG) {
        stage_filter_consts<N, R>(a, CL, csh, ssh);
        stage_smoother_consts<N, R>(a, CL, fsh);
        __syncthreads();
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t k0 = gt * EPT;
    const int64_t kw = (gt - lane) * EPT;
    if (kw >= a.total) return;
    R* st = stage[threadIdx.x >> 6];
    const R* y = static_cast<const R*>(a.y);
    R* mo = static_cast<R*>(a.m);
    R* Po = static_cast<R*>(a.P);
    Moments<N, R> X;
    load_m(a.carry, a.nwaves, gt >> 6, X);
    {
        FElem<N, R> pre;
        load_f(a.thr, a.nthr, gt, pre);
        fcarry<N, R, SEG>(X, pre);
    }
    SElem<N, R> sacc;
    set_identity(sacc);
    Seq s = seq_find<SEG>(a, k0 < a.total ? k0 : a.total - 1);
    constexpr int MY = sizeof(R) == 8 ? M : 0;   // FP32 storage: read y in place (measured faster)
    R yv[YV<MY>::n];
    load_y<MY>(y, k0 < a.total ? k0 : a.total - 1, yv);
#pragma unroll 1
    for (int e = 0; e < EPT; ++e) {
        const int64_t k = k0 + e;
        if (k < a.total) {
            R yn[YV<MY>::n];
            load_y<MY>(y, k + 1 < a.total ? k + 1 : k, yn);
            seq_forward<SEG>(a, s, k);
            const int64_t moff = const_offset<SEG>(a, s.b, k);
            const R* cst;
            const double* Sp;
            const R* Fp;
            if constexpr (STG) {
                cst = csh;
                Sp = ssh;
                Fp = fsh;
            } else {
                cst = static_cast<const R*>(a.consts) + moff;
                Sp = a.consts64 + moff + CL.S;
                Fp = cst + CL.F;
            }
            const bool first = k == s.start;
            {
                FElem<N, R> x;
                build_felem_step<N, R, MY>(cst, CL, a.ny, y, k, yv, first, x);
                if (M == 0) {
                    fcarry<N, R, SEG>(X, x);
                } else {
                    constexpr int MM = M > 0 ? M : 1;
                    R Gz[MM * N];
                    load_gz<N, MM, R>(cst, CL, first, Gz);
                    fcarry_fresh<N, MM, R, SEG>(X, x, Gz, Sp);
                }
#pragma unroll
                for (int q = 0; q < YV<MY>::n; ++q) yv[q] = yn[q];
            }
            SElem<N, R> el;
            make_selem_p<N, R>(Fp, Fp + N * N, Fp + 2 * N * N, X, k == s.end - 1, el, a.status, s.b);
            if (e == 0) sacc = el;
            else scombine<N, R, SEG>(sacc, el, sacc);
        }
        wave_store_moments<N, R>(mo, Po, kw, e, EPT - 1, EPT, a.total, st, lane, X);
    }
    wave_inclusive_suffix_s<N, R, SEG>(sacc, lane);
    SElem<N, R> ex;
    wave_exclusive_suffix_s(sacc, ex, lane);
    store_s(a.thr, a.nthr, gt, ex);
    if (lane == 0) store_s(a.agg, a.nwaves, gt >> 6, sacc);
}

// ===========================================================================
// SMOOTHER (suffix direction)
// ===========================================================================
template <int N, typename R, int EPT, bool SEG>
__global__ __launch_bounds__(kBlock) void k_smoother_reduce(ScanArgs a) {
    clear_top_flags(a);
    __shared__ R fsh[SEG ? 1 : StageS<N>::words];
    const ConstLayout CL = const_layout(N, a.ny);
    if constexpr (!SEG) {
        stage_smoother_consts<N, R>(a, CL, fsh);
        __syncthreads();
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t k0 = gt * EPT;
    const R* m = static_cast<const R*>(a.m);
    const R* P = static_cast<const R*>(a.P);
    SElem<N, R> acc;
    set_identity(acc);
    if (k0 < a.total) {
        const int64_t klast = (k0 + EPT - 1 < a.total) ? k0 + EPT - 1 : a.total - 1;
        Seq s = seq_find<SEG>(a, klast);
        // the loads of the next (earlier) step are issued before this step's work
        Moments<N, R> xn;
        load_moments_step(m, P, klast, xn);
#pragma unroll 1
        for (int64_t k = klast; k >= k0; --k) {
            const Moments<N, R> x = xn;
            if (k > k0) load_moments_step(m, P, k - 1, xn);
            seq_backward<SEG>(a, s, k);
            const R* Fp;
            if constexpr (SEG) Fp = static_cast<const R*>(a.consts) + const_offset<SEG>(a, s.b, k) + CL.F;
            else Fp = fsh;
            SElem<N, R> el;
            make_selem_p<N, R>(Fp, Fp + N * N, Fp + 2 * N * N, x, k == s.end - 1, el, a.status, s.b);
            if (k == klast) acc = el;
            else scombine<N, R, SEG>(el, acc, acc);
        }
    }
    wave_inclusive_suffix_s<N, R, SEG>(acc, lane);
    SElem<N, R> ex;
    wave_exclusive_suffix_s(acc, ex, lane);
    store_s(a.thr, a.nthr, gt, ex);
    if (lane == 0) store_s(a.agg, a.nwaves, gt >> 6, acc);
}

template <int N, typename R, int EPT, bool G>
__global__ __launch_bounds__(kBlock) void k_smoother_reduce_items(ScanArgs a) {
    clear_top_flags(a);
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t i0 = gt * EPT;
    SElem<N, R> acc;
    set_identity(acc);
#pragma unroll 1
    for (int e = EPT - 1; e >= 0; --e) {
        const int64_t i = i0 + e;
        if (i < a.nwaves) {
            SElem<N, R> x;
            load_s(a.agg, a.nwaves, i, x);
            scombine<N, R, G>(x, acc, acc);
        }
    }
    wave_inclusive_suffix_s<N, R, G>(acc, lane);
    SElem<N, R> ex;
    wave_exclusive_suffix_s(acc, ex, lane);
    store_s(a.thr1, a.nthr1, gt, ex);
    if (lane == 0) store_s(a.agg1, a.nwaves1, gt >> 6, acc);
}

template <int N, typename R, int EPT, bool G>
__global__ __launch_bounds__(kBlock) void k_smoother_down_items(ScanArgs a) {
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i0 = gt * EPT;
    if (i0 >= a.nwaves) return;
    Moments<N, R> Y;
    load_m(a.carry1, a.nwaves1, gt >> 6, Y);
    SElem<N, R> pre;
    load_s(a.thr1, a.nthr1, gt, pre);
    scarry<N, R, G>(pre, Y);
#pragma unroll 1
    for (int e = EPT - 1; e >= 0; --e) {
        const int64_t i = i0 + e;
        if (i < a.nwaves) {
            store_m(a.carry, a.nwaves, i, Y);
            SElem<N, R> x;
            load_s(a.agg, a.nwaves, i, x);
            scarry<N, R, G>(x, Y);
        }
    }
}

template <int N, typename R, int EPT, bool SEG>
__global__ __launch_bounds__(kBlock) void k_smoother_down(ScanArgs a) {
    __shared__ R stage[kBlock / 64][MomStage<N, R>::WORDS];
    __shared__ R fsh[SEG ? 1 : StageS<N>::words];
    const ConstLayout CL = const_layout(N, a.ny);
    if constexpr (!SEG) {
        stage_smoother_consts<N, R>(a, CL, fsh);
        __syncthreads();
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t k0 = gt * EPT;
    const int64_t kw = (gt - lane) * EPT;
    if (kw >= a.total) return;
    R* st = stage[threadIdx.x >> 6];
    const R* m = static_cast<const R*>(a.m);
    const R* P = static_cast<const R*>(a.P);
    R* mso = static_cast<R*>(a.ms);
    R* Pso = static_cast<R*>(a.Ps);
    Moments<N, R> Y;
    load_m(a.carry, a.nwaves, gt >> 6, Y);
    {
        SElem<N, R> pre;
        load_s(a.thr, a.nthr, gt, pre);
        scarry<N, R, SEG>(pre, Y);
    }
    const int64_t klast = (k0 + EPT - 1 < a.total) ? k0 + EPT - 1 : a.total - 1;
    Seq s = seq_find<SEG>(a, klast);
    // When a lane's run of means is exactly one store group (FP32 means, 8 per
    // line), the filtered means of the whole run are read into the stage first,
    // whole lines per instruction, and each step replaces its own slot with the
    // smoothed mean: a line is never fetched twice.  Covariances are read
    // directly, one step ahead.
    using MS = MomStage<N, R>;
    constexpr bool kRunM = sizeof(R) == 4 && MS::GM == EPT;
    if constexpr (kRunM) {
        wave_fill<MS::GM, MS::UM, MS::UBM, MS::ROWM, R>(m, st, N, kw, EPT, a.total, lane);
        wave_sync();
    }
    Moments<N, R> xn;
    if constexpr (kRunM) load_cov_step(P, klast, xn);
    else load_moments_step(m, P, klast, xn);
#pragma unroll 1
    for (int e = EPT - 1; e >= 0; --e) {
        const int64_t k = k0 + e;
        Moments<N, R> x = xn;
        if (k <= klast && k > k0) {
            if constexpr (kRunM) load_cov_step(P, k - 1, xn);
            else load_moments_step(m, P, k - 1, xn);
        }
        if constexpr (kRunM) {
            const R* rm = st + lane * MS::ROWM + (e % MS::GM) * N;
#pragma unroll
            for (int r = 0; r < N; ++r) x.m[r] = rm[r];
        }
        if (k <= klast) {
            seq_backward<SEG>(a, s, k);
            const R* Fp;
            if constexpr (SEG) Fp = static_cast<const R*>(a.consts) + const_offset<SEG>(a, s.b, k) + CL.F;
            else Fp = fsh;
            SElem<N, R> el;
            make_selem_p<N, R>(Fp, Fp + N * N, Fp + 2 * N * N, x, k == s.end - 1, el, a.status, s.b);
            scarry<N, R, SEG>(el, Y);
        }
        wave_store_moments_rev<N, R>(mso, Pso, kw, e, EPT, EPT, a.total, st, lane, Y);
    }
}

// ===========================================================================
// launch helpers
// ===========================================================================
inline int64_t blocks_for_threads(int64_t nthr) { return (nthr + kBlock - 1) / kBlock; }

// the device-wide top level over n items (top_epl.hpp)
inline TopArgs top_args(const void* items, int64_t n, void* carry, const ScanArgs& a) {
    TopArgs t;
    t.items = items;
    t.n = n;
    t.carry = carry;
    const int64_t per_wg_max = (int64_t)kTopGroups * kTopMaxWg;
    t.E = (int)((n + per_wg_max - 1) / per_wg_max);
    if (t.E < 1) t.E = 1;
    const int64_t per_wg = (int64_t)kTopGroups * t.E;
    t.nwg = (int)((n + per_wg - 1) / per_wg);
    if (t.nwg < 1) t.nwg = 1;
    t.wg_agg = a.top_agg;
    t.flags = a.top_flags;
    t.model_fail = a.model_fail;
    t.nmodels = a.nmodels;
    t.status = a.status;
    return t;
}
template <int N, typename R, bool G>
void launch_filter_top(const void* items, int64_t n, void* carry, const ScanArgs& a, hipStream_t s) {
    const TopArgs t = top_args(items, n, carry, a);
    prof_begin("k_filter_top", s);
    hipLaunchKernelGGL((k_filter_top<N, R, G>), dim3(t.nwg), dim3(kTopThreads), 0, s, t);
    prof_end(s);
}
template <int N, typename R, bool G>
void launch_smoother_top(const void* items, int64_t n, void* carry, const ScanArgs& a, hipStream_t s) {
    const TopArgs t = top_args(items, n, carry, a);
    prof_begin("k_smoother_top", s);
    hipLaunchKernelGGL((k_smoother_top<N, R, G>), dim3(t.nwg), dim3(kTopThreads), 0, s, t);
    prof_end(s);
}

#define PKS_EPT1_SWITCH(KERNEL, ...)                                                                   \
    switch (a.ept1) {                                                                                  \
        case 1: hipLaunchKernelGGL((KERNEL<N, R, 1, SEG>), dim3(nb1), dim3(kBlock), 0, s, a); break;   \
        case 2: hipLaunchKernelGGL((KERNEL<N, R, 2, SEG>), dim3(nb1), dim3(kBlock), 0, s, a); break;   \
        case 4: hipLaunchKernelGGL((KERNEL<N, R, 4, SEG>), dim3(nb1), dim3(kBlock), 0, s, a); break;   \
        case 8: hipLaunchKernelGGL((KERNEL<N, R, 8, SEG>), dim3(nb1), dim3(kBlock), 0, s, a); break;   \
        default: return hipErrorInvalidValue;                                                          \
    }

template <int N, typename R, int EPT, bool SEG, int M>
hipError_t run_filter(ScanArgs a, hipStream_t s) {
    const int64_t nb0 = a.nthr / kBlock;
    prof_begin("k_filter_reduce", s);
    hipLaunchKernelGGL((k_filter_reduce<N, R, EPT, SEG, M>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    if (a.nwaves1 == 0) {
        launch_filter_top<N, R, SEG>(a.agg, a.nwaves, a.carry, a, s);
    } else {
        const int64_t nb1 = a.nthr1 / kBlock;
        prof_begin("k_filter_reduce_items", s);
        PKS_EPT1_SWITCH(k_filter_reduce_items)
        prof_end(s);
        launch_filter_top<N, R, SEG>(a.agg1, a.nwaves1, a.carry1, a, s);
        prof_begin("k_filter_down_items", s);
        PKS_EPT1_SWITCH(k_filter_down_items)
        prof_end(s);
    }
    prof_begin("k_filter_down", s);
    hipLaunchKernelGGL((k_filter_down<N, R, EPT, SEG, M>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    return hipGetLastError();
}

template <int N, typename R, int EPT, bool SEG>
hipError_t run_smoother(ScanArgs a, hipStream_t s) {
    const int64_t nb0 = a.nthr / kBlock;
    prof_begin("k_smoother_reduce", s);
    hipLaunchKernelGGL((k_smoother_reduce<N, R, EPT, SEG>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    if (a.nwaves1 == 0) {
        launch_smoother_top<N, R, SEG>(a.agg, a.nwaves, a.carry, a, s);
    } else {
        const int64_t nb1 = a.nthr1 / kBlock;
        prof_begin("k_smoother_reduce_items", s);
        PKS_EPT1_SWITCH(k_smoother_reduce_items)
        prof_end(s);
        launch_smoother_top<N, R, SEG>(a.agg1, a.nwaves1, a.carry1, a, s);
        prof_begin("k_smoother_down_items", s);
        PKS_EPT1_SWITCH(k_smoother_down_items)
        prof_end(s);
    }
    prof_begin("k_smoother_down", s);
    hipLaunchKernelGGL((k_smoother_down<N, R, EPT, SEG>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    return hipGetLastError();
}
// Both passes with the filter down-sweep and the smoother reduce fused.
template <int N, typename R, int EPT, bool SEG, int M>
hipError_t run_filter_smoother(ScanArgs a, hipStream_t s) {
    const int64_t nb0 = a.nthr / kBlock;
    prof_begin("k_filter_reduce", s);
    hipLaunchKernelGGL((k_filter_reduce<N, R, EPT, SEG, M>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    if (a.nwaves1 == 0) {
        launch_filter_top<N, R, SEG>(a.agg, a.nwaves, a.carry, a, s);
    } else {
        const int64_t nb1 = a.nthr1 / kBlock;
        prof_begin("k_filter_reduce_items", s);
        PKS_EPT1_SWITCH(k_filter_reduce_items)
        prof_end(s);
        launch_filter_top<N, R, SEG>(a.agg1, a.nwaves1, a.carry1, a, s);
        prof_begin("k_filter_down_items", s);
        PKS_EPT1_SWITCH(k_filter_down_items)
        prof_end(s);
    }
    prof_begin("k_filter_down_smooth_reduce", s);
    hipLaunchKernelGGL((k_filter_down_smooth_reduce<N, R, EPT, SEG, M>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    if (a.nwaves1 == 0) {
        launch_smoother_top<N, R, SEG>(a.agg, a.nwaves, a.carry, a, s);
    } else {
        const int64_t nb1 = a.nthr1 / kBlock;
        prof_begin("k_smoother_reduce_items", s);
        PKS_EPT1_SWITCH(k_smoother_reduce_items)
        prof_end(s);
        launch_smoother_top<N, R, SEG>(a.agg1, a.nwaves1, a.carry1, a, s);
        prof_begin("k_smoother_down_items", s);
        PKS_EPT1_SWITCH(k_smoother_down_items)
        prof_end(s);
    }
    prof_begin("k_smoother_down", s);
    hipLaunchKernelGGL((k_smoother_down<N, R, EPT, SEG>), dim3(nb0), dim3(kBlock), 0, s, a);
    prof_end(s);
    return hipGetLastError();
}
#undef PKS_EPT1_SWITCH

// passes: 1 filter, 2 smoother, 3 both.  With FP32 storage both passes use the
// fused filter down-sweep / smoother reduce; in FP64 the fused kernel needs
// more registers than one wave per SIMD leaves, and the two separate kernels
// measured faster, so FP64 runs the passes one after the other.
template <int N, typename R, int EPT, bool SEG, int M>
hipError_t run_passes(ScanArgs a, int passes, hipStream_t s) {
    if (passes == 3) {
        if constexpr (sizeof(R) == 4) {
            return run_filter_smoother<N, R, EPT, SEG, M>(a, s);
        } else {
            const hipError_t e = run_filter<N, R, EPT, SEG, M>(a, s);
            return e != hipSuccess ? e : run_smoother<N, R, EPT, SEG>(a, s);
        }
    }
    if (passes == 2) return run_smoother<N, R, EPT, SEG>(a, s);
    return run_filter<N, R, EPT, SEG, M>(a, s);
}

// rank-ny single-step combines when ny < nx (M = ny), the general form otherwise
template <int N, typename R, int EPT, bool SEG>
hipError_t run_m(ScanArgs a, int passes, hipStream_t s) {
    if (a.ny >= N || EPT < 8) return run_passes<N, R, EPT, SEG, 0>(a, passes, s);
    switch (a.ny) {
        case 1: return run_passes<N, R, EPT, SEG, 1>(a, passes, s);
        case 2: return run_passes<N, R, EPT, SEG, (N > 2 ? 2 : 0)>(a, passes, s);
        case 3: return run_passes<N, R, EPT, SEG, (N > 3 ? 3 : 0)>(a, passes, s);
        default: return run_passes<N, R, EPT, SEG, 0>(a, passes, s);
    }
}

template <int N, typename R, bool SEG>
hipError_t dispatch_ept(ScanArgs a, int passes, hipStream_t s) {
    switch (a.ept) {
        case 4: return run_m<N, R, 4, SEG>(a, passes, s);
        case 8: return run_m<N, R, 8, SEG>(a, passes, s);
        case 16: return run_m<N, R, 16, SEG>(a, passes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// All scan kernels of one state dimension and precision (one translation unit each).
template <int N, typename R>
hipError_t small_run(ScanArgs a, int passes, hipStream_t s) {
    return a.offsets != nullptr ? dispatch_ept<N, R, true>(a, passes, s) : dispatch_ept<N, R, false>(a, passes, s);
}

}  // namespace pks
