// pks_internal.h -- shared between the C-ABI layer and the kernel translation
// units: per-model constant layout, workspace layout and launch arguments.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pks.h"

namespace pks {

// ---------------------------------------------------------------------------
// Per-model constants written by the model-precompute kernel (Lemma 1 for a
// time-invariant model: A, C, J are the same for every k > 1 and b_k, eta_k
// are affine in y_k; the k = 1 element has its own K_1, C_1), followed by
// copies of F, Q, u for the smoothing elements (Lemma 3).
//   b_k   = c  + K  y_k,   c  = u - K (H u + d)
//   eta_k = w  + W  y_k,   w  = -W (H u + d),    W = F^T H^T S^-1
//   b_1   = c1 + K1 y_1,   c1 = m1 - K1 (H m1 + d), m1 = F m0 + u
// G = H F and S = H Q H^T + R are kept as well: J = F^T H^T S^-1 H F = W G has
// rank ny, which the single-step combines use.  With e = H u + d they also
// give the one-step predictive density of y_k from the filtered moments of
// step k-1: N(G m_{k-1} + e, G P_{k-1} G^T + S) (the marginal likelihood).
// All matrices row-major, full (not packed).
// ---------------------------------------------------------------------------
struct ConstLayout {
    int A, C, J, K, W, c, w, K1, c1, C1, F, Q, u, G, S, e, words;
};
__host__ __device__ inline ConstLayout const_layout(int nx, int ny) {
    ConstLayout L;
    int o = 0;
    const int n2 = nx * nx, nm = nx * ny;
    L.A = o; o += n2;
    L.C = o; o += n2;
    L.J = o; o += n2;
    L.K = o; o += nm;
    L.W = o; o += nm;
    L.c = o; o += nx;
    L.w = o; o += nx;
    L.K1 = o; o += nm;
    L.c1 = o; o += nx;
    L.C1 = o; o += n2;
    L.G = o; o += nm;        // H F         [ny][nx]  (J = W G: the rank-ny factors of J)
    L.S = o; o += ny * ny;   // H Q H^T + R [ny][ny]
    L.e = o; o += ny;        // H u + d     [ny]
    // smoother constants last: a filter-only precompute writes [0, F)
    L.F = o; o += n2;
    L.Q = o; o += n2;
    L.u = o; o += nx;
    L.words = (o + 15) & ~15;
    return L;
}

// scratch words per model used by the precompute kernel (double)
__host__ __device__ inline int precompute_scratch_words(int nx, int ny) {
    const int n2 = nx * nx, nm = nx * ny, m2 = ny * ny;
    return (6 * n2 + 8 * nm + 4 * m2 + 4 * nx + 4 * ny + 15) & ~15;
}

// Device-wide top level of the small-state scans: at most this many
// workgroups, each publishing one aggregate of kTopAggWords doubles.
constexpr int kTopMaxWorkgroups = 64;
constexpr int kTopAggWords = 6 * 16;

constexpr int kStatusOk = 0x7fffffff;     // "no failure" value of the numeric flag
constexpr int kStatusMagic = 0x504b5331;  // marks a prepared status word

// ---------------------------------------------------------------------------
// Workspace layout (byte offsets from ws), computed on the host.
// ---------------------------------------------------------------------------
struct WsLayout {
    size_t status;        // int32 first failing sequence (kStatusOk = none)
    size_t consts64;      // [nmodels][CW] double
    size_t consts32;      // [nmodels][CW] float
    size_t scratch;       // [nmodels][SW] double (precompute temporaries)
    size_t model_fail;    // [nmodels] int32
    size_t thr;           // per-thread exclusive prefixes, SoA (level 0)
    size_t agg;           // per-wave aggregates, SoA (level 0)
    size_t carry;         // per-wave incoming moments, SoA (level 0)
    size_t thr1, agg1, carry1;  // same for level 1 (scan over level-0 aggregates)
    size_t large;         // large-state path scratch
    size_t ll_step;       // [total] double: log p(y_k | y_1:k-1) when not returned
    size_t ll_cum;        // [total] double: prefix sums inside blocks of kLLBlock steps
    size_t ll_blk_h, ll_blk_v, ll_blk_first, ll_carry;   // [blocks] int32 / double
    size_t ll_tile_seq;   // [total / 256 + 2] int32: sequence of each 256-step tile's first step
    size_t tv_offsets;    // int64 {0, T}: a time-varying model's one sequence, for the SEG kernels
    size_t top_flags;     // int32 [1 + kTopMaxWorkgroups]: ticket counter and publish flags of the top level
    size_t top_agg;       // double [kTopMaxWorkgroups][kTopAggWords]: workgroup aggregates of the top level
    size_t total;
    // sizes used for capacity checks
    int64_t cap_thr, cap_waves, cap_thr1, cap_waves1;
};

WsLayout ws_layout(int nx, int ny, int64_t total, int32_t nmodels, pks_precision prec);

// ---------------------------------------------------------------------------
// Launch arguments of the small-state scan kernels.
// ---------------------------------------------------------------------------
struct ScanArgs {
    int nx, ny;
    int64_t total;               // steps (sum over sequences)
    int32_t B;                   // sequences
    const int64_t* offsets;      // device [B+1]; nullptr = one sequence [0, total)
    int64_t model_stride;        // R words between models in consts (0 = shared)
    int64_t step_stride;         // R words between steps' constants (time-varying model; else 0)
    const void* consts;          // R-typed constants of model 0
    const double* consts64;      // the same constants in double (S is always read in double)
    const void* y;               // filter input  [total][ny]
    void* m;                     // filter output [total][nx]  / smoother input
    void* P;                     // filter output [total][nx][nx] / smoother input
    void* ms;                    // smoother output
    void* Ps;
    // level-0 scan state
    void* thr;                   // SoA [words][nthr]
    void* agg;                   // SoA [words][nwaves]
    void* carry;                 // SoA [mwords][nwaves]
    int64_t nthr, nwaves;        // padded counts (SoA strides)
    // level-1 scan state (nwaves1 == 0: single level)
    void* thr1;
    void* agg1;
    void* carry1;
    int64_t nthr1, nwaves1;
    int ept, ept1;               // elements per thread at level 0 / 1
    int64_t large_blocks;        // large states: requested number of time blocks (0 = default)
    int* top_flags;              // top level: ticket counter + publish flags (cleared by the kernel before it)
    double* top_agg;             // top level: published workgroup aggregates
    int* status;
    const int* model_fail;       // [nmodels] 1 = the model's precompute failed
    int nmodels;
};

// Offset (in words) of the constants of step k of sequence b: one block per
// model (one per sequence), or one block per step for a time-varying model.
// The single-sequence kernels (SEG = false) serve one time-invariant model
// only, so their constants stay at offset 0 and loop-invariant; a
// time-varying model runs through the SEG kernels as one packed sequence.
template <bool SEG>
__host__ __device__ __forceinline__ int64_t const_offset(const ScanArgs& a, int b, int64_t k) {
    return SEG ? (int64_t)b * a.model_stride + k * a.step_stride : 0;
}

// Tile configuration chosen for a launch.
struct TileConfig {
    int ept = 16;    // elements per thread, level 0 (4, 8, 16)
    int ept1 = 0;    // elements per thread, level 1 (aggregates); 0 = no level 1
    int blocks = 0;  // large states (nx >= 5): blocks of the time axis (Section III-C's
                  // block elements); 0 = the default count
};

// Per-kernel timing (diagnostics).  While enabled on the calling thread,
// launchers bracket each kernel with prof_begin/prof_end, which record HIP
// events on the launch stream; both are no-ops otherwise.
void prof_begin(const char* kernel, hipStream_t s);
void prof_end(hipStream_t s);

// launchers (scan_small.hip)
bool small_supported(int nx);
// Model precompute (one workgroup per model); also prepares the numeric flag
// (cleared when `reset`, or when the workspace was never prepared).
// Time-varying models (`tv`): the arrays of `model` hold one row per step and
// every step gets its own constants (nmodels = steps): the filter constants of
// step k from row k, the smoother's F, Q, u from row k + 1; the prior is
// shared, or one per packed sequence (tv_offsets [B+1], model.per_sequence),
// and a failing factorisation flags its sequence directly.
hipError_t launch_precompute(int nx, int ny, int32_t nmodels, const pks_model& model,
                             void* ws, const WsLayout& L, bool mixed, int what, bool reset, hipStream_t s,
                             bool tv = false, const int64_t* tv_offsets = nullptr, int32_t B = 1);
// passes: 1 = filter, 2 = smoother, 3 = both (fused where possible)
hipError_t launch_small(ScanArgs a, bool mixed, int passes, hipStream_t s);
TileConfig small_default_config(int nx, int64_t total, bool mixed);

// Debug mode (pks_set_debug_poison, or the environment variable
// PKS_DEBUG_POISON set to anything but 0): every call first fills the
// floating-point regions of its workspace with NaN (launch_poison writes
// [p, p + bytes), 8-byte words), so a kernel that reads workspace memory this
// call has not written turns its outputs into NaN.
bool debug_poison();
hipError_t launch_poison(void* p, size_t bytes, hipStream_t s);
// the floating-point regions of a workspace with layout L (the numeric flag,
// the per-model failure flags and the integer tables are left alone)
hipError_t poison_workspace(void* ws, const WsLayout& L, hipStream_t s);

// Check of packed-sequence offsets (device [B+1]) against the packing rules;
// *result (device int) becomes the smallest offending index, or 0x7fffffff.
hipError_t launch_offsets_check(const int64_t* offsets, int B, int64_t total, int* result, hipStream_t s);

// marginal likelihood (loglik.hip)
constexpr int kLLBlock = 4096;      // steps per block of the prefix sums
int64_t ll_blocks(int64_t total);
// Per-step log predictive densities of the filtered sequences (ll: [total] or
// nullptr), or with `cumulative` their running sums within each sequence, and
// per-sequence totals (tot: [B] or nullptr).  offsets = nullptr: one sequence.
// Needs G, S, e of the model in ws (launch_precompute, what 4).
hipError_t launch_loglik(const pks_model& model, int32_t B, const int64_t* offsets, int64_t total,
                         const void* y, const void* m, const void* P, double* ll, double* tot,
                         bool cumulative, bool mixed, void* ws, const WsLayout& L, hipStream_t s,
                         bool tv = false);

// discrete-state hidden Markov model (hmm.hip), 1 <= K <= 64 states
int hmm_padded_states(int K);
int64_t hmm_block_len(int K, int64_t T);
size_t hmm_ws_bytes(int K, int64_t T);
// passes: 1 = filter (alpha, logp), 2 = smoother (gamma from alpha), 3 = both
hipError_t launch_hmm(int K, int64_t T, const double* Pi, const double* p0, const double* L, double* alpha,
                      double* logp, double* gamma, void* ws, int passes, hipStream_t st);

// large-state path (scan_large.hip), 5 <= nx <= 64
size_t large_ws_bytes(int nx, int ny, int64_t total, pks_precision prec);
// the default (and largest) number of time blocks of the large-state scans
int64_t large_default_blocks(int nx, int ny, int64_t total, bool mixed);
// both: the filter and the smoother of one call (the smoother follows the
// filter on the same stream and workspace)
hipError_t launch_large(ScanArgs a, void* region, bool mixed, bool smoother, bool both, hipStream_t s);

// register-resident large-state path (scan_w16.hip): time-invariant models
// (one sequence or packed sequences, shared or per-sequence models),
// 5 <= nx <= 16, ny <= 16
bool w16_applies(int nx, int ny, bool time_invariant);
int64_t w16_default_blocks(int64_t total);
size_t w16_ws_bytes(int64_t total);
hipError_t launch_w16(ScanArgs a, void* region, bool mixed, bool smoother, bool both, hipStream_t s);
// the marginal likelihood factors of one sequence with one time-invariant
// model, 5 <= nx <= 16, ny <= 16 (register tiles); false: not applicable
bool launch_ll_w16(int nx, int ny, int64_t total, const double* m0, const double* P0, const double* consts64, int cG,
                   int cS, int ce, const void* y, const void* m, const void* P, double* step, int* status, bool mixed,
                   hipStream_t s);
// the model constants of time-invariant models with 5 <= nx <= 16, ny <= 16,
// one wavefront per model (what: 1, 2 or 3 as for launch_precompute); false:
// not applicable, nothing launched
bool launch_w16_precompute(int nx, int ny, int32_t nmodels, const pks_model& model, double* consts64, float* consts32,
                           int* status, int* model_fail, int what, bool reset, hipStream_t s);

}  // namespace pks
