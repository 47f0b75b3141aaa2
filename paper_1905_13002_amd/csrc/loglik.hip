// loglik.hip -- the marginal likelihood of filtered sequences (Section III-C).
//
// p(y_1:n) is the product of the factors p(y_k | y_1:k-1), and each factor is
// the Gaussian density of y_k under the one-step prediction made from the
// filtered moments of step k-1 (from the prior x_0 ~ N(m0, P0) at the first
// step of a sequence):
//     m^-_k = F m_{k-1} + u,   P^-_k = F P_{k-1} F^T + Q,
//     y_k | y_1:k-1 ~ N(H m^-_k + d, H P^-_k H^T + R)
//                   = N(G m_{k-1} + e, G P_{k-1} G^T + S0)
// with the model constants G = H F, e = H u + d, S0 = H Q H^T + R of the
// precompute.  Given the filtered moments the factors are independent, so
// each step is evaluated on its own; the partial likelihoods p(y_1:k) are then
// a prefix sum of the log factors that restarts at every sequence start (the
// section's pairwise products of adjacent terms, taken in log space).
//
//   log N(r; 0, S) = -(ny log(2 pi) + 2 sum_i log L_ii + |L^-1 r|^2) / 2,
//   S = L L^T (Cholesky; a pivot that is not positive sets the numeric flag
//   and gives NaN, a NaN in y gives NaN without the flag).
// Every factor is evaluated in double; in the mixed mode the float y, m, P are
// widened first.
//
// Kernels
//   k_ll_small<NX,NY,R,SEG>  nx, ny <= 4: one step per lane, persistent over
//                            tiles of 256 steps; the moments of the previous
//                            steps are loaded coalesced and staged through LDS
//                            (odd row stride), the next tile's loads in flight
//                            while the current one is evaluated.
//   k_ll_wave<R,SEG>         nx, ny < 32 beyond the above: one wavefront per
//                            step; P_{k-1}, G P_{k-1} and S in LDS, the Cholesky
//                            factorisation and the forward substitution
//                            row-parallel across lanes.
//   k_ll_large<R,SEG>        nx or ny >= 32: one workgroup per step (persistent);
//                            G P_{k-1} and S0 + (G P_{k-1}) G^T on the matrix
//                            cores, S factorised and r^T S^-1 r solved with the
//                            register / blocked Cholesky of the large-state scans.
//   k_ll_tile_seq            batched: the sequence of every tile's first step
//                            (one search each), so that a lane only searches
//                            between two neighbouring entries.
//   k_ll_block_scan<SEG>     segmented inclusive prefix sums inside blocks of
//                            kLLBlock steps; per block its aggregate (whether
//                            a sequence starts in it, sum since the last start)
//                            and the position of its first sequence start.
//   k_ll_top<SEG>            one workgroup: exclusive scan of the block
//                            aggregates (the carry into each block) and the
//                            per-sequence totals.
//   k_ll_fixup               adds each block's carry to its steps before the
//                            block's first sequence start.
// The prefix sums use a fixed combination order, so results are reproducible
// run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "large_ops.hpp"
#include "pks_internal.h"

namespace pks {

namespace {

constexpr int kLLThreads = 256;                     // per-step kernels (a tile of 256 steps)
constexpr int kScanThreads = 1024;                  // block scan
constexpr int kLLPerThread = kLLBlock / kScanThreads; // steps per thread in the block scan
constexpr int kTopThreads = 1024;
constexpr double kLog2Pi = 1.8378770664093454836;   // log(2 pi)

struct LLArgs {
    int nx, ny;
    int64_t total;
    int32_t B;
    const int64_t* offsets;        // device [B+1]; nullptr = one sequence
    int per_sequence;
    const double* m0;              // model prior(s)
    const double* P0;
    const double* consts64;        // per-model constants (G, S0, e used here)
    int64_t cstride;               // doubles between models' constants (0 = shared)
    int64_t sstride;               // doubles between steps' constants (time-varying model; else 0)
    int cG, cS, ce;                // offsets of G, S0, e in a model's constants
    const void* y;
    const void* m;                 // filtered moments of every step
    const void* P;
    double* step;                  // [total] out: log p(y_k | y_1:k-1)
    int* status;
    const int* tile_seq;           // [tiles + 1] sequence of each tile's first step (batched)
};

// Residual y_k - G m - e with a compensated sum: every product and every
// addition keeps its rounding error (error-free transformations: the product's
// error from an FMA, the sum's by Knuth's TwoSum), and the errors are added at
// the end (the Dot2 scheme of Ogita, Rump and Oishi, "Accurate sum and dot
// product", SIAM J. Sci. Comput. 2005).  The result is as accurate as if it
// were computed in twice the working precision and then rounded.  Where the
// state is large (positions of 1e7 in the constant-velocity workload) the
// residual is a small difference of large numbers, and the plain sum would
// lose about seven digits of it.
struct Acc2 {
    double s, c;
};
__device__ __forceinline__ void acc2_add(Acc2& a, double x) {
#pragma clang fp contract(off)
    const double t = a.s + x;
    const double z = t - a.s;
    a.c += (a.s - (t - z)) + (x - z);
    a.s = t;
}
__device__ __forceinline__ void acc2_sub_prod(Acc2& a, double g, double x) {
#pragma clang fp contract(off)
    const double p = g * x;
    const double e = fma(g, x, -p);     // g x = p + e exactly
    acc2_add(a, -p);
    a.c -= e;
}
__device__ __forceinline__ double acc2_value(const Acc2& a) { return a.s + a.c; }

// sequence index and first step of step k (k < total)
template <bool SEG>
__device__ __forceinline__ int seq_of(const int64_t* off, int B, int64_t k, int64_t& start) {
    if (!SEG) {
        start = 0;
        return 0;
    }
    int lo = 0, hi = B;        // offsets[lo] <= k
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    start = off[lo];
    return lo;
}

// Sequence of step k when it is known to lie in [lo, hi] (from the tile table).
template <bool SEG>
__device__ __forceinline__ int seq_between(const int64_t* off, int lo, int hi, int64_t k, int64_t& start) {
    if (!SEG) {
        start = 0;
        return 0;
    }
    ++hi;                       // invariant: off[lo] <= k < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid;
    }
    start = off[lo];
    return lo;
}

// tile_seq[i] = sequence of step 256 i (i < tiles), tile_seq[tiles] = sequence
// of the last step: every step of tile i belongs to a sequence in
// [tile_seq[i], tile_seq[i + 1]].  One independent search per entry.
__global__ __launch_bounds__(kLLThreads) void k_ll_tile_seq(const int64_t* off, int B, int64_t total,
                                                             int64_t tiles, int* tile_seq) {
    const int64_t i = (int64_t)blockIdx.x * kLLThreads + threadIdx.x;
    if (i > tiles) return;
    const int64_t k = i < tiles ? i * kLLThreads : total - 1;
    int64_t start;
    tile_seq[i] = seq_of<true>(off, B, k, start);
}

// ---------------------------------------------------------------------------
// nx, ny <= 4: one step per lane
// ---------------------------------------------------------------------------
// The log factor of step k from the filtered moments of step k-1 (row: m then
// P, in LDS) or, at a sequence start, from the prior of its model.
template <int NX, int NY, typename R, bool SEG>
__device__ __forceinline__ void ll_step_small(const LLArgs& a, int64_t k, int b, bool first, const R* row) {
    constexpr int n2 = NX * NX;
    double m[NX], P[n2];
    if (first) {
        const int64_t ps = a.per_sequence ? b : 0;
#pragma unroll
        for (int i = 0; i < NX; ++i) m[i] = a.m0[ps * NX + i];
#pragma unroll
        for (int i = 0; i < n2; ++i) P[i] = a.P0[ps * n2 + i];
    } else {
#pragma unroll
        for (int i = 0; i < NX; ++i) m[i] = (double)row[i];
#pragma unroll
        for (int i = 0; i < n2; ++i) P[i] = (double)row[NX + i];
    }
    const double* cst = a.consts64 + a.cstride * b + k * a.sstride;
    double G[NY * NX], S[NY * NY], r[NY];
#pragma unroll
    for (int i = 0; i < NY * NX; ++i) G[i] = cst[a.cG + i];
#pragma unroll
    for (int i = 0; i < NY * NY; ++i) S[i] = cst[a.cS + i];
    const R* yk = static_cast<const R*>(a.y) + k * NY;
#pragma unroll
    for (int i = 0; i < NY; ++i) {
        Acc2 v{(double)yk[i], 0.0};
        acc2_add(v, -cst[a.ce + i]);
#pragma unroll
        for (int l = 0; l < NX; ++l) acc2_sub_prod(v, G[i * NX + l], m[l]);
        r[i] = acc2_value(v);
    }
    // S += G P G^T (lower triangle; the Cholesky factorisation reads only it)
    double T[NY * NX];
#pragma unroll
    for (int i = 0; i < NY; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double v = 0.0;
#pragma unroll
            for (int l = 0; l < NX; ++l) v += G[i * NX + l] * P[l * NX + j];
            T[i * NX + j] = v;
        }
#pragma unroll
    for (int i = 0; i < NY; ++i)
#pragma unroll
        for (int i2 = 0; i2 <= i; ++i2) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < NX; ++j) v += T[i * NX + j] * G[i2 * NX + j];
            S[i * NY + i2] += v;
        }
    // S = L L^T in place (lower), z = L^-1 r in place
    bool ok = true;
    double logdet = 0.0, quad = 0.0;
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        double dj = S[j * NY + j];
#pragma unroll
        for (int l = 0; l < j; ++l) dj -= S[j * NY + l] * S[j * NY + l];
        ok = ok && dj > 0.0;
        const double ljj = sqrt(dj);
        const double inv = 1.0 / ljj;
        S[j * NY + j] = ljj;
#pragma unroll
        for (int i = j + 1; i < NY; ++i) {
            double v = S[i * NY + j];
#pragma unroll
            for (int l = 0; l < j; ++l) v -= S[i * NY + l] * S[j * NY + l];
            S[i * NY + j] = v * inv;
        }
        double zj = r[j];
#pragma unroll
        for (int l = 0; l < j; ++l) zj -= S[j * NY + l] * r[l];
        r[j] = zj * inv;
        quad += r[j] * r[j];
        logdet += log(ljj);
    }
    double ll = -0.5 * (NY * kLog2Pi + quad) - logdet;
    if (!ok) {
        ll = __builtin_nan("");
        atomicMin(a.status, b);
    }
    a.step[k] = ll;
}

// Persistent over tiles of 256 steps: the moments of the steps before a tile
// (rows r = 0 .. 255 hold steps k0-1 .. k0+254) are loaded coalesced into
// registers, stored to an LDS stage with an odd row stride, and read back one
// row per lane.  The loads of the next tile are issued before the current
// tile is evaluated, so they are in flight during its arithmetic.
template <int NX, int NY, typename R, bool SEG>
__global__ __launch_bounds__(kLLThreads) void k_ll_small(LLArgs a, int64_t ntiles) {
    constexpr int n2 = NX * NX, RW = NX + n2;
    constexpr int ROW = (RW & 1) ? RW : RW + 1;     // odd row stride: lanes hit distinct banks
    __shared__ R stage[kLLThreads * ROW];
    const int t = threadIdx.x;
    const R* gm = static_cast<const R*>(a.m);
    const R* gP = static_cast<const R*>(a.P);
    // thread t carries words t + 256 j of the tile's m block (j < NX) and P block (j < n2)
    R buf[RW];
    auto load = [&](int64_t tile) {
        const int64_t k0 = tile * kLLThreads;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            const int i = t + kLLThreads * j, r = i / NX;
            const int64_t kk = k0 - 1 + r;
            buf[j] = (kk >= 0 && kk < a.total) ? gm[(k0 - 1) * NX + i] : R(0);
        }
#pragma unroll
        for (int j = 0; j < n2; ++j) {
            const int i = t + kLLThreads * j, r = i / n2;
            const int64_t kk = k0 - 1 + r;
            buf[NX + j] = (kk >= 0 && kk < a.total) ? gP[(k0 - 1) * n2 + i] : R(0);
        }
    };
    int64_t tile = blockIdx.x;
    if (tile < ntiles) load(tile);
    for (; tile < ntiles; tile += gridDim.x) {
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            const int i = t + kLLThreads * j, r = i / NX;
            stage[r * ROW + (i - r * NX)] = buf[j];
        }
#pragma unroll
        for (int j = 0; j < n2; ++j) {
            const int i = t + kLLThreads * j, r = i / n2;
            stage[r * ROW + NX + (i - r * n2)] = buf[NX + j];
        }
        __syncthreads();
        if (tile + gridDim.x < ntiles) load(tile + gridDim.x);
        const int64_t k0 = tile * kLLThreads, k = k0 + t;
        if (k < a.total) {
            int64_t start;
            const int b = SEG ? seq_between<true>(a.offsets, a.tile_seq[tile], a.tile_seq[tile + 1], k, start)
                              : seq_between<false>(a.offsets, 0, 0, k, start);
            ll_step_small<NX, NY, R, SEG>(a, k, b, k == start, stage + t * ROW);
        }
        __syncthreads();                            // the stage is rewritten next
    }
}

// ---------------------------------------------------------------------------
// any size: one wavefront per step
// ---------------------------------------------------------------------------
// Makes one wave's LDS writes visible to its other lanes (LDS only: the
// lanes exchange nothing through global memory here).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__host__ __device__ inline int ll_wave_words(int nx, int ny) {
    // P [nx][nx], T = G P [ny][nx], S [ny][ny], m [nx], r [ny], G [ny][nx]
    return nx * nx + ny * nx + ny * ny + nx + ny + ny * nx;
}

template <typename R, bool SEG>
__global__ __launch_bounds__(kLLThreads) void k_ll_wave(LLArgs a) {
    extern __shared__ __align__(16) double lds_ll[];
    const int nx = a.nx, ny = a.ny, n2 = nx * nx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double* P = lds_ll + (size_t)wave * ll_wave_words(nx, ny);
    double* T = P + n2;
    double* S = T + ny * nx;
    double* m = S + ny * ny;
    double* r = m + nx;
    double* G = r + ny;          // the step's G = H F, staged once per step
    const R* gm = static_cast<const R*>(a.m);
    const R* gP = static_cast<const R*>(a.P);
    const R* gy = static_cast<const R*>(a.y);
    for (int64_t k = (int64_t)blockIdx.x * nw + wave; k < a.total; k += (int64_t)gridDim.x * nw) {
        int64_t start;
        const int64_t tile = k / kLLThreads;
        const int b = SEG ? seq_between<true>(a.offsets, a.tile_seq[tile], a.tile_seq[tile + 1], k, start)
                          : seq_between<false>(a.offsets, 0, 0, k, start);
        const double* cst = a.consts64 + a.cstride * b + k * a.sstride;
        for (int i = lane; i < ny * nx; i += 64) G[i] = cst[a.cG + i];
        if (k == start) {
            const int64_t ps = a.per_sequence ? b : 0;
            for (int i = lane; i < n2; i += 64) P[i] = a.P0[ps * n2 + i];
            for (int i = lane; i < nx; i += 64) m[i] = a.m0[ps * nx + i];
        } else {
            for (int i = lane; i < n2; i += 64) P[i] = (double)gP[(k - 1) * n2 + i];
            for (int i = lane; i < nx; i += 64) m[i] = (double)gm[(k - 1) * nx + i];
        }
        wave_sync();
        for (int idx = lane; idx < ny * nx; idx += 64) {          // T = G P
            const int i = idx / nx, j = idx - i * nx;
            double v = 0.0;
#pragma unroll 4
            for (int l = 0; l < nx; ++l) v += G[i * nx + l] * P[l * nx + j];
            T[idx] = v;
        }
        for (int i = lane; i < ny; i += 64) {                      // r = y - G m - e
            Acc2 v{(double)gy[k * ny + i], 0.0};
            acc2_add(v, -cst[a.ce + i]);
#pragma unroll 4
            for (int l = 0; l < nx; ++l) acc2_sub_prod(v, G[i * nx + l], m[l]);
            r[i] = acc2_value(v);
        }
        wave_sync();
        for (int idx = lane; idx < ny * ny; idx += 64) {          // S = S0 + T G^T (lower)
            const int i = idx / ny, i2 = idx - i * ny;
            if (i2 > i) continue;
            double v = 0.0;
#pragma unroll 4
            for (int j = 0; j < nx; ++j) v += T[i * nx + j] * G[i2 * nx + j];
            S[idx] = cst[a.cS + idx] + v;
        }
        wave_sync();
        // right-looking Cholesky with the forward substitution of r alongside
        bool ok = true;
        double logdet = 0.0, quad = 0.0;
        for (int j = 0; j < ny; ++j) {
            const double dj = S[j * ny + j];
            ok = ok && dj > 0.0;
            const double ljj = sqrt(dj), inv = 1.0 / ljj;
            const double zj = r[j] * inv;
            quad += zj * zj;
            logdet += log(ljj);
            wave_sync();                                           // every lane has read row j
            for (int i = j + 1 + lane; i < ny; i += 64) {
                const double lij = S[i * ny + j] * inv;
                S[i * ny + j] = lij;
                r[i] -= lij * zj;
            }
            wave_sync();
            const int nt = ny - j - 1;
            for (int idx = lane; idx < nt * nt; idx += 64) {       // trailing lower triangle
                const int ii = idx / nt, jj = idx - ii * nt;
                if (jj > ii) continue;
                const int i = j + 1 + ii, i2 = j + 1 + jj;
                S[i * ny + i2] -= S[i * ny + j] * S[i2 * ny + j];
            }
            wave_sync();
        }
        if (lane == 0) {
            double ll = -0.5 * (ny * kLog2Pi + quad) - logdet;
            if (!ok) {
                ll = __builtin_nan("");
                atomicMin(a.status, b);
            }
            a.step[k] = ll;
        }
        wave_sync();                                               // LDS reuse by the next step
    }
}

// ---------------------------------------------------------------------------
// segmented prefix sums of the log factors
// ---------------------------------------------------------------------------
// (head, value): head = a sequence starts in the range, value = sum since the
// last start in it (or over all of it).  Associative; left operand first.
struct Seg {
    int h;
    double v;
};
__device__ __forceinline__ Seg seg_combine(Seg l, Seg r) {
    return Seg{l.h | r.h, r.h ? r.v : l.v + r.v};
}

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ Seg wave_scan(Seg x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Seg o;
        o.h = __shfl_up(x.h, d, 64);
        o.v = __shfl_up(x.v, d, 64);
        if (lane >= d) x = seg_combine(o, x);
    }
    return x;
}

// Exclusive scan over the block (NT threads): returns the combination of all
// earlier threads' values (identity for thread 0); *total gets the block's.
template <int NT>
__device__ __forceinline__ Seg block_exclusive(Seg x, Seg* total) {
    __shared__ int sh_h[NT / 64];
    __shared__ double sh_v[NT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const Seg inc = wave_scan(x);
    Seg ex;
    ex.h = __shfl_up(inc.h, 1, 64);
    ex.v = __shfl_up(inc.v, 1, 64);
    if (lane == 0) ex = Seg{0, 0.0};
    if (lane == 63) {
        sh_h[wave] = inc.h;
        sh_v[wave] = inc.v;
    }
    __syncthreads();
    Seg pre{0, 0.0};
    for (int w = 0; w < wave; ++w) pre = seg_combine(pre, Seg{sh_h[w], sh_v[w]});
    Seg all = pre;
    for (int w = wave; w < NT / 64; ++w) all = seg_combine(all, Seg{sh_h[w], sh_v[w]});
    *total = all;
    __syncthreads();                     // the shared words are reused by the next call
    return seg_combine(pre, ex);
}

struct LLScanArgs {
    int64_t total;
    int32_t B;
    const int64_t* offsets;
    const double* step;     // [total] log factors
    double* cum;            // [total] out: prefix sums inside each block
    int* blk_h;             // [nblk]
    double* blk_v;          // [nblk]
    int* blk_first;         // [nblk] position of the block's first sequence start (kLLBlock: none)
    double* carry;          // [nblk] sum carried into each block
    double* tot;            // [B] per-sequence totals (nullptr: not wanted)
    int64_t nblk;
    const int* tile_seq;    // as in LLArgs
};

template <bool SEG>
__global__ __launch_bounds__(kScanThreads) void k_ll_block_scan(LLScanArgs a) {
    __shared__ int first_sh;
    const int t = threadIdx.x;
    if (t == 0) first_sh = kLLBlock;
    const int64_t k0 = (int64_t)blockIdx.x * kLLBlock + (int64_t)t * kLLPerThread;
    double inc[kLLPerThread];
    int heads = 0;
    Seg x{0, 0.0};
    int64_t start = 0, end = a.total;
    int b = 0;
    if (SEG && k0 < a.total) {
        const int64_t tile = k0 / kLLThreads;
        b = seq_between<true>(a.offsets, a.tile_seq[tile], a.tile_seq[tile + 1], k0, start);
        end = a.offsets[b + 1];
    }
#pragma unroll
    for (int q = 0; q < kLLPerThread; ++q) {
        const int64_t k = k0 + q;
        double v = 0.0;
        int h = 0;
        if (k < a.total) {
            while (SEG && k >= end && b < a.B - 1) {   // next non-empty sequence (offsets
                ++b;                                     // past total stay in the last one)
                start = end;
                end = a.offsets[b + 1];
            }
            h = k == start;
            v = a.step[k];
        }
        x = seg_combine(x, Seg{h, v});
        inc[q] = x.v;
        heads |= h << q;
    }
    __syncthreads();                         // first_sh initialised
    if (heads) atomicMin(&first_sh, t * kLLPerThread + __builtin_ctz(heads));
    Seg blk;
    const Seg ex = block_exclusive<kScanThreads>(x, &blk);
#pragma unroll
    for (int q = 0; q < kLLPerThread; ++q) {
        const int64_t k = k0 + q;
        const bool own = heads & ((2 << q) - 1);   // a start among this thread's steps 0..q
        if (k < a.total) a.cum[k] = own ? inc[q] : ex.v + inc[q];
    }
    if (t == 0) {
        a.blk_h[blockIdx.x] = blk.h;
        a.blk_v[blockIdx.x] = blk.v;
        a.blk_first[blockIdx.x] = first_sh;
    }
}

template <bool SEG>
__global__ __launch_bounds__(kTopThreads) void k_ll_top(LLScanArgs a) {
    const int t = threadIdx.x;
    Seg run{0, 0.0};
    for (int64_t base = 0; base < a.nblk; base += kTopThreads) {
        const int64_t c = base + t;
        const Seg x = c < a.nblk ? Seg{a.blk_h[c], a.blk_v[c]} : Seg{0, 0.0};
        Seg chunk;
        const Seg ex = block_exclusive<kTopThreads>(x, &chunk);
        if (c < a.nblk) a.carry[c] = seg_combine(run, ex).v;
        run = seg_combine(run, chunk);
    }
    if (!a.tot) return;
    __syncthreads();                         // carries written by this workgroup
    for (int b = t; b < a.B; b += kTopThreads) {
        const int64_t s = SEG ? a.offsets[b] : 0;
        const int64_t e = SEG ? min(a.offsets[b + 1], a.total) : a.total;   // offsets past total: clamped
        double v = 0.0;
        if (e > s && e > 0) {
            const int64_t k = e - 1, c = k / kLLBlock;
            v = a.cum[k];
            if (s < c * kLLBlock) v += a.carry[c];
        }
        a.tot[b] = v;
    }
}

__global__ __launch_bounds__(kLLThreads) void k_ll_fixup(LLScanArgs a) {
    const int64_t k = (int64_t)blockIdx.x * kLLThreads + threadIdx.x;
    if (k >= a.total) return;
    const int64_t c = k / kLLBlock;
    if (k - c * kLLBlock < a.blk_first[c]) a.cum[k] += a.carry[c];
}

int device_cus() {
    static int cus = 0;
    if (cus <= 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Persistent grid: as many workgroups as fit on the device at once, but no
// more than there are tiles, with the tiles spread evenly over them.
template <int NX, int NY, typename R, bool SEG>
void launch_small_kernel(const LLArgs& a, hipStream_t s) {
    static int per_cu = 0;
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ll_small<NX, NY, R, SEG>, kLLThreads, 0) !=
                hipSuccess || per_cu <= 0)
            per_cu = 1;
    }
    const int64_t ntiles = (a.total + kLLThreads - 1) / kLLThreads;
    const int64_t slots = (int64_t)per_cu * device_cus();
    const int64_t rounds = (ntiles + slots - 1) / slots;
    const int64_t grid = (ntiles + rounds - 1) / rounds;
    hipLaunchKernelGGL((k_ll_small<NX, NY, R, SEG>), dim3((unsigned)grid), dim3(kLLThreads), 0, s, a, ntiles);
}

// ---------------------------------------------------------------------------
// nx or ny >= 32: one workgroup per step
// ---------------------------------------------------------------------------
// LDS: P_{k-1} [nx][nx] (widened to double), T = G P [ny][nx], S [ny][ny],
// G [ny][nx] (staged when the step's model differs from the previous step's),
// m [nx], r [ny], x [ny].  S0 and e are read from the constants.
__host__ __device__ inline int ll_large_words(int nx, int ny) {
    return nx * nx + 2 * ny * nx + ny * ny + nx + 2 * ny;
}

template <typename R, bool SEG>
__global__ __launch_bounds__(256) void k_ll_large(LLArgs a) {
    extern __shared__ __align__(16) double lds_ll[];
    __shared__ int flag_sh;
    const int nx = a.nx, ny = a.ny, n2 = nx * nx, tid = threadIdx.x, nt = blockDim.x;
    double* P = lds_ll;
    double* T = P + n2;
    double* S = T + ny * nx;
    double* G = S + ny * ny;
    double* m = G + ny * nx;
    double* r = m + nx;
    double* x = r + ny;
    const R* gm = static_cast<const R*>(a.m);
    const R* gP = static_cast<const R*>(a.P);
    const R* gy = static_cast<const R*>(a.y);
    const double* staged = nullptr;   // constants whose G is in LDS
    for (int64_t k = blockIdx.x; k < a.total; k += gridDim.x) {
        int64_t start;
        const int64_t tile = k / kLLThreads;
        const int b = SEG ? seq_between<true>(a.offsets, a.tile_seq[tile], a.tile_seq[tile + 1], k, start)
                          : seq_between<false>(a.offsets, 0, 0, k, start);
        const double* cst = a.consts64 + a.cstride * b + k * a.sstride;
        if (cst != staged) {
            for (int i = tid; i < ny * nx; i += nt) G[i] = cst[a.cG + i];
            staged = cst;
        }
        if (k == start) {
            const int64_t ps = a.per_sequence ? b : 0;
            for (int i = tid; i < n2; i += nt) P[i] = a.P0[ps * n2 + i];
            for (int i = tid; i < nx; i += nt) m[i] = a.m0[ps * nx + i];
        } else {
            for (int i = tid; i < n2; i += nt) P[i] = (double)gP[(k - 1) * n2 + i];
            for (int i = tid; i < nx; i += nt) m[i] = (double)gm[(k - 1) * nx + i];
        }
        __syncthreads();
        large::gemmR<double>(T, nx, G, nx, false, P, nx, false, ny, nx, nx);    // T = G P (ends with a barrier)
        for (int i = tid; i < ny; i += nt) {                                     // r = y - G m - e
            Acc2 v{(double)gy[k * ny + i], 0.0};
            acc2_add(v, -cst[a.ce + i]);
            for (int l = 0; l < nx; ++l) acc2_sub_prod(v, G[i * nx + l], m[l]);
            r[i] = x[i] = acc2_value(v);
        }
        large::gemmR<double>(S, ny, T, nx, false, G, nx, true, ny, ny, nx, 1.0, cst + a.cS, ny);   // S = S0 + T G^T
        const bool ok = large::cholesky(S, ny, ny, &flag_sh);                  // L below, L^T above the diagonal
        large::chol_solve(S, ny, ny, x, 1, 1);                                   // x = S^-1 r
        __syncthreads();
        if (tid == 0) {
            double quad = 0.0, logdet = 0.0;
            for (int i = 0; i < ny; ++i) {
                quad = fma(r[i], x[i], quad);
                logdet += log(S[i * ny + i]);
            }
            double ll = -0.5 * (ny * kLog2Pi + quad) - logdet;
            if (!ok) {
                ll = __builtin_nan("");
                atomicMin(a.status, b);
            }
            a.step[k] = ll;
        }
        __syncthreads();                                                          // LDS reuse by the next step
    }
}

template <int NX, typename R, bool SEG>
bool launch_small_ny(int ny, const LLArgs& a, hipStream_t s) {
    switch (ny) {
        case 1: launch_small_kernel<NX, 1, R, SEG>(a, s); return true;
        case 2: launch_small_kernel<NX, 2, R, SEG>(a, s); return true;
        case 3: launch_small_kernel<NX, 3, R, SEG>(a, s); return true;
        case 4: launch_small_kernel<NX, 4, R, SEG>(a, s); return true;
        default: return false;
    }
}

template <typename R, bool SEG>
bool launch_small_ll(const LLArgs& a, hipStream_t s) {
    switch (a.nx) {
        case 1: return launch_small_ny<1, R, SEG>(a.ny, a, s);
        case 2: return launch_small_ny<2, R, SEG>(a.ny, a, s);
        case 3: return launch_small_ny<3, R, SEG>(a.ny, a, s);
        case 4: return launch_small_ny<4, R, SEG>(a.ny, a, s);
        default: return false;
    }
}

template <typename R, bool SEG>
void launch_steps(const LLArgs& a, hipStream_t s) {
    prof_begin("k_ll_steps", s);
    if (!SEG && a.sstride == 0 && w16_applies(a.nx, a.ny, true)) {
        launch_ll_w16(a.nx, a.ny, a.total, a.m0, a.P0, a.consts64, a.cG, a.cS, a.ce, a.y, a.m, a.P, a.step, a.status,
                      sizeof(R) == 4, s);
    } else if (a.nx >= 32 || a.ny >= 32) {
        const size_t lds = sizeof(double) * (size_t)ll_large_words(a.nx, a.ny);
        const int threads = 256;
        const unsigned grid = (unsigned)std::min<int64_t>(a.total, 4096);
        hipLaunchKernelGGL((k_ll_large<R, SEG>), dim3(grid), dim3(threads), lds, s, a);
    } else if (!(a.nx <= 4 && a.ny <= 4 && launch_small_ll<R, SEG>(a, s))) {
        const size_t per_wave = sizeof(double) * (size_t)ll_wave_words(a.nx, a.ny);
        int waves = (int)std::min<size_t>(4, std::max<size_t>(1, (64 * 1024) / per_wave));
        const int64_t want = (a.total + waves - 1) / waves;
        const unsigned grid = (unsigned)std::min<int64_t>(want, 16384);
        hipLaunchKernelGGL((k_ll_wave<R, SEG>), dim3(grid), dim3(64 * waves), per_wave * waves, s, a);
    }
    prof_end(s);
}

}  // namespace

int64_t ll_blocks(int64_t total) { return (total + kLLBlock - 1) / kLLBlock; }

hipError_t launch_loglik(const pks_model& model, int32_t B, const int64_t* offsets, int64_t total,
                         const void* y, const void* m, const void* P, double* ll, double* tot,
                         bool cumulative, bool mixed, void* ws, const WsLayout& L, hipStream_t s, bool tv) {
    char* base = static_cast<char*>(ws);
    const ConstLayout CL = const_layout(model.nx, model.ny);
    LLArgs a{};
    a.nx = model.nx;
    a.ny = model.ny;
    a.total = total;
    a.B = B;
    a.offsets = offsets;
    a.per_sequence = model.per_sequence ? 1 : 0;
    a.m0 = model.m0;
    a.P0 = model.P0;
    a.consts64 = reinterpret_cast<const double*>(base + L.consts64);
    a.cstride = (model.per_sequence && !tv) ? CL.words : 0;
    a.sstride = tv ? CL.words : 0;
    a.cG = CL.G;
    a.cS = CL.S;
    a.ce = CL.e;
    a.y = y;
    a.m = m;
    a.P = P;
    a.status = reinterpret_cast<int*>(base + L.status);
    // the per-step factors go to the caller's array unless it receives the prefix sums
    double* ws_step = reinterpret_cast<double*>(base + L.ll_step);
    a.step = (ll && !cumulative) ? ll : ws_step;
    const bool seg = offsets != nullptr;
    const int64_t tiles = (total + kLLThreads - 1) / kLLThreads;
    int* tile_seq = reinterpret_cast<int*>(base + L.ll_tile_seq);
    a.tile_seq = tile_seq;
    if (seg) {
        prof_begin("k_ll_tile_seq", s);
        hipLaunchKernelGGL(k_ll_tile_seq, dim3((unsigned)((tiles + 1 + kLLThreads - 1) / kLLThreads)),
                           dim3(kLLThreads), 0, s, offsets, B, total, tiles, tile_seq);
        prof_end(s);
    }
    if (mixed) {
        if (seg) launch_steps<float, true>(a, s); else launch_steps<float, false>(a, s);
    } else {
        if (seg) launch_steps<double, true>(a, s); else launch_steps<double, false>(a, s);
    }
    if (!cumulative && !tot) return hipGetLastError();

    LLScanArgs c{};
    c.total = total;
    c.B = seg ? B : 1;
    c.offsets = offsets;
    c.step = a.step;
    c.cum = cumulative ? ll : reinterpret_cast<double*>(base + L.ll_cum);
    c.blk_h = reinterpret_cast<int*>(base + L.ll_blk_h);
    c.blk_v = reinterpret_cast<double*>(base + L.ll_blk_v);
    c.blk_first = reinterpret_cast<int*>(base + L.ll_blk_first);
    c.carry = reinterpret_cast<double*>(base + L.ll_carry);
    c.tot = tot;
    c.nblk = ll_blocks(total);
    c.tile_seq = tile_seq;
    prof_begin("k_ll_block_scan", s);
    if (seg) hipLaunchKernelGGL(k_ll_block_scan<true>, dim3((unsigned)c.nblk), dim3(kScanThreads), 0, s, c);
    else hipLaunchKernelGGL(k_ll_block_scan<false>, dim3((unsigned)c.nblk), dim3(kScanThreads), 0, s, c);
    prof_end(s);
    prof_begin("k_ll_top", s);
    if (seg) hipLaunchKernelGGL(k_ll_top<true>, dim3(1), dim3(kTopThreads), 0, s, c);
    else hipLaunchKernelGGL(k_ll_top<false>, dim3(1), dim3(kTopThreads), 0, s, c);
    prof_end(s);
    if (cumulative) {
        prof_begin("k_ll_fixup", s);
        hipLaunchKernelGGL(k_ll_fixup, dim3((unsigned)((total + kLLThreads - 1) / kLLThreads)), dim3(kLLThreads),
                           0, s, c);
        prof_end(s);
    }
    return hipGetLastError();
}

}  // namespace pks
