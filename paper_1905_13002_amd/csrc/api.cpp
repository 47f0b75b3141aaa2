// api.cpp -- the C ABI of libpks.so (declared in include/pks.h): argument
// validation, workspace layout, tile configuration and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "pks_internal.h"
#include "plan.h"

namespace pks {

namespace {

thread_local std::string g_last_error;

pks_status fail(pks_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

pks_status hip_fail(hipError_t e, const char* what) {
    return fail(PKS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

constexpr int kMinEpt = 4;          // smallest elements-per-thread any configuration uses
constexpr int kMaxDim = 64;

constexpr int64_t kMaxStepsTv = 0x7fffffff;   // time-varying: one constant block per step, indexed by int32

int felem_words(int nx) { return nx * nx + nx + nx * (nx + 1) / 2 + nx + nx * (nx + 1) / 2; }
int moment_words(int nx) { return nx + nx * (nx + 1) / 2; }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

pks_status check_model(const pks_model* model) {
    if (!model) return fail(PKS_E_ARG, "model is NULL");
    if (model->nx < 1 || model->nx > kMaxDim) return fail(PKS_E_ARG, "nx = %d outside [1, 64]", model->nx);
    if (model->ny < 1 || model->ny > kMaxDim) return fail(PKS_E_ARG, "ny = %d outside [1, 64]", model->ny);
    if (!model->F || !model->Q || !model->H || !model->R || !model->m0 || !model->P0)
        return fail(PKS_E_ARG, "model matrix pointer is NULL (F, Q, H, R, m0 and P0 are required)");
    return PKS_OK;
}

pks_status check_prec(pks_precision prec) {
    if (prec != PKS_FP64 && prec != PKS_MIXED_FP32) return fail(PKS_E_ARG, "unknown precision %d", (int)prec);
    return PKS_OK;
}

size_t rsize(pks_precision prec) { return prec == PKS_FP64 ? sizeof(double) : sizeof(float); }

}  // namespace

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
WsLayout ws_layout(int nx, int ny, int64_t total, int32_t nmodels, pks_precision prec) {
    WsLayout L{};
    const size_t rs = rsize(prec);
    const ConstLayout CL = const_layout(nx, ny);
    size_t o = 0;
    L.status = o; o += 256;
    L.consts64 = o; o = align256(o + sizeof(double) * (size_t)CL.words * nmodels);
    L.consts32 = o; o = align256(o + sizeof(float) * (size_t)CL.words * nmodels);
    L.scratch = o; o = align256(o + sizeof(double) * (size_t)precompute_scratch_words(nx, ny) * nmodels);
    L.model_fail = o; o = align256(o + sizeof(int32_t) * (size_t)nmodels);
    L.top_flags = o; o = align256(o + sizeof(int32_t) * (size_t)(1 + kTopMaxWorkgroups));
    // small-state scan: level 0 over steps, level 1 over level-0 wave aggregates
    const int64_t waves0 = round_up(std::max<int64_t>(1, ceil_div(total, 64 * kMinEpt)), 4);
    const int64_t thr0 = waves0 * 64;
    const int64_t waves1 = round_up(std::max<int64_t>(1, ceil_div(waves0, 64)), 4);   // >= 1 item per thread
    const int64_t thr1 = waves1 * 64;
    const bool small = small_supported(nx);
    const int fw = small ? felem_words(nx) : 0, mw = small ? moment_words(nx) : 0;
    L.cap_thr = thr0;
    L.cap_waves = waves0;
    L.cap_thr1 = thr1;
    L.cap_waves1 = waves1;
    L.thr = o; o = align256(o + rs * fw * (size_t)thr0);
    L.agg = o; o = align256(o + rs * fw * (size_t)waves0);
    L.carry = o; o = align256(o + rs * mw * (size_t)waves0);
    L.thr1 = o; o = align256(o + rs * fw * (size_t)thr1);
    L.agg1 = o; o = align256(o + rs * fw * (size_t)waves1);
    L.carry1 = o; o = align256(o + rs * mw * (size_t)waves1);
    L.top_agg = o; o = align256(o + sizeof(double) * (size_t)kTopMaxWorkgroups * kTopAggWords);
    L.large = o;
    if (!small) o = align256(o + large_ws_bytes(nx, ny, total, prec));
    const int64_t nblk = ll_blocks(total);
    L.ll_step = o; o = align256(o + sizeof(double) * (size_t)total);
    L.ll_cum = o; o = align256(o + sizeof(double) * (size_t)total);
    L.ll_blk_h = o; o = align256(o + sizeof(int32_t) * (size_t)nblk);
    L.ll_blk_v = o; o = align256(o + sizeof(double) * (size_t)nblk);
    L.ll_blk_first = o; o = align256(o + sizeof(int32_t) * (size_t)nblk);
    L.ll_carry = o; o = align256(o + sizeof(double) * (size_t)nblk);
    L.ll_tile_seq = o; o = align256(o + sizeof(int32_t) * (size_t)(total / 256 + 2));
    L.tv_offsets = o; o = align256(o + 2 * sizeof(int64_t));
    L.total = o;
    return L;
}

// ---------------------------------------------------------------------------
// debug: NaN-filled workspace
// ---------------------------------------------------------------------------
namespace {
std::atomic<int> g_poison{-1};   // -1: not yet read from the environment
}

bool debug_poison() {
    int v = g_poison.load(std::memory_order_relaxed);
    if (v < 0) {
        const char* e = std::getenv("PKS_DEBUG_POISON");
        v = (e && *e && std::strcmp(e, "0") != 0) ? 1 : 0;
        int expected = -1;
        if (!g_poison.compare_exchange_strong(expected, v)) v = expected;
    }
    return v > 0;
}

hipError_t poison_workspace(void* ws, const WsLayout& L, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    const size_t span[4][2] = {{L.consts64, L.model_fail},      // constants, precompute scratch
                               // (then the integer flags: model failures, top-level tickets)
                               {L.thr, L.ll_blk_h},             // scan state, large-state region, ll arrays
                               {L.ll_blk_v, L.ll_blk_first},
                               {L.ll_carry, L.ll_tile_seq}};
    for (const auto& r : span) {
        const hipError_t e = launch_poison(b + r[0], r[1] - r[0], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// scan argument assembly
// ---------------------------------------------------------------------------
ScanArgs make_scan_args(const pks_model& model, int32_t B, const int64_t* offsets, int64_t total,
                        pks_precision prec, void* ws, const WsLayout& L, TileConfig cfg, bool tv) {
    ScanArgs a{};
    char* base = static_cast<char*>(ws);
    const ConstLayout CL = const_layout(model.nx, model.ny);
    a.nx = model.nx;
    a.ny = model.ny;
    a.total = total;
    a.B = B;
    a.offsets = offsets;
    a.model_stride = (model.per_sequence && !tv) ? CL.words : 0;
    a.step_stride = tv ? CL.words : 0;
    a.consts = prec == PKS_FP64 ? (const void*)(base + L.consts64) : (const void*)(base + L.consts32);
    a.consts64 = reinterpret_cast<const double*>(base + L.consts64);
    a.thr = base + L.thr;
    a.agg = base + L.agg;
    a.carry = base + L.carry;
    a.ept = cfg.ept;
    a.large_blocks = cfg.blocks;
    a.nwaves = round_up(std::max<int64_t>(1, ceil_div(total, 64 * cfg.ept)), 4);
    a.nthr = a.nwaves * 64;
    a.ept1 = cfg.ept1;
    if (cfg.ept1 > 0) {
        a.thr1 = base + L.thr1;
        a.agg1 = base + L.agg1;
        a.carry1 = base + L.carry1;
        a.nwaves1 = round_up(std::max<int64_t>(1, ceil_div(a.nwaves, 64 * cfg.ept1)), 4);
        a.nthr1 = a.nwaves1 * 64;
    }
    a.status = reinterpret_cast<int*>(base + L.status);
    a.model_fail = reinterpret_cast<const int*>(base + L.model_fail);
    a.top_flags = reinterpret_cast<int*>(base + L.top_flags);
    a.top_agg = reinterpret_cast<double*>(base + L.top_agg);
    // a time-varying precompute flags failing steps itself: nothing to collect
    a.nmodels = tv ? 0 : (model.per_sequence ? B : 1);
    return a;
}

// Enqueue the requested passes.  passes: 1 = filter, 2 = smoother, 3 = both.
pks_status enqueue(const pks_model& model, int32_t B, const int64_t* offsets, int64_t total,
                   const void* y, void* m, void* P, void* ms, void* Ps, pks_precision prec,
                   void* ws, size_t ws_bytes, int passes, const TileConfig* forced, hipStream_t s, bool tv) {
    const int nmodels = tv ? (int)total : (model.per_sequence ? B : 1);
    const WsLayout L = ws_layout(model.nx, model.ny, total, tv ? nmodels : B, prec);
    if (ws_bytes < L.total)
        return fail(PKS_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    ws_bytes, L.total);
    if (total == 0) return PKS_OK;
    if (debug_poison()) {
        const hipError_t pe = poison_workspace(ws, L, s);
        if (pe != hipSuccess) return hip_fail(pe, "workspace fill");
    }
    const bool small = small_supported(model.nx);
    const bool mixed = prec == PKS_MIXED_FP32;
    TileConfig cfg = forced ? *forced : tuned_config(model.nx, model.ny, B, total, prec);
    if (cfg.ept < kMinEpt) cfg.ept = kMinEpt;
    if (!small_supported(model.nx)) cfg.ept1 = 0;   // the large-state path reads only cfg.blocks
    hipError_t e = launch_precompute(model.nx, model.ny, nmodels, model, ws, L, mixed, passes,
                                     (passes & 1) != 0, s, tv, tv ? offsets : nullptr, B);
    if (e != hipSuccess) return hip_fail(e, "precompute kernel");
    // a single time-varying sequence runs as one packed sequence (offsets {0, T},
    // written by the precompute's preparation kernel) through the per-step-constant
    // kernels; packed time-varying sequences keep the caller's offsets
    if (tv && !offsets) offsets = reinterpret_cast<const int64_t*>(static_cast<char*>(ws) + L.tv_offsets);
    ScanArgs a = make_scan_args(model, B, offsets, total, prec, ws, L, cfg, tv);
    a.y = y;
    a.m = m;
    a.P = P;
    a.ms = ms;
    a.Ps = Ps;
    if (!small) {
        void* region = static_cast<char*>(ws) + L.large;
        if (passes & 1) {
            e = launch_large(a, region, mixed, false, passes == 3, s);
            if (e != hipSuccess) return hip_fail(e, "filter kernels");
        }
        if (passes & 2) {
            e = launch_large(a, region, mixed, true, passes == 3, s);
            if (e != hipSuccess) return hip_fail(e, "smoother kernels");
        }
        return PKS_OK;
    }
    if (a.nthr > L.cap_thr || a.nwaves > L.cap_waves || a.nthr1 > L.cap_thr1 || a.nwaves1 > L.cap_waves1)
        return fail(PKS_E_ARG, "tile configuration (ept %d, ept1 %d) does not fit the workspace", cfg.ept, cfg.ept1);
    e = launch_small(a, mixed, passes, s);
    if (e != hipSuccess) return hip_fail(e, "scan kernels");
    return PKS_OK;
}

pks_status validate_io(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                       const void* y, const void* m, const void* P, const void* ms, const void* Ps,
                       pks_precision prec, void* ws, int passes, bool batched) {
    pks_status st = check_model(model);
    if (st) return st;
    st = check_prec(prec);
    if (st) return st;
    if (total < 0) return fail(PKS_E_ARG, "negative number of steps");
    if (batched) {
        if (B < 1) return fail(PKS_E_ARG, "B = %d must be >= 1", B);
        if (!offsets) return fail(PKS_E_ARG, "offsets is NULL");
    } else if (model->per_sequence) {
        return fail(PKS_E_ARG, "per_sequence models need a batched call");
    }
    if (!ws) return fail(PKS_E_ARG, "workspace is NULL");
    if (total == 0) return PKS_OK;
    const size_t rs = rsize(prec);
    const size_t ny = model->ny, nx = model->nx, T = (size_t)total;
    const size_t by = T * ny * rs, bm = T * nx * rs, bP = T * nx * nx * rs;
    if ((passes & 1) && (!y || !m || !P)) return fail(PKS_E_ARG, "y, m and P must not be NULL");
    if ((passes & 2) && (!m || !P || !ms || !Ps)) return fail(PKS_E_ARG, "m, P, ms and Ps must not be NULL");
    if (passes & 1) {
        if (overlaps(y, by, m, bm) || overlaps(y, by, P, bP) || overlaps(m, bm, P, bP))
            return fail(PKS_E_ARG, "filter outputs overlap the input or each other");
    }
    if (passes & 2) {
        if (overlaps(ms, bm, Ps, bP) || overlaps(ms, bm, m, bm) || overlaps(ms, bm, P, bP) ||
            overlaps(Ps, bP, m, bm) || overlaps(Ps, bP, P, bP))
            return fail(PKS_E_ARG, "smoother outputs overlap the inputs or each other");
        if (passes & 1) {
            if (overlaps(y, by, ms, bm) || overlaps(y, by, Ps, bP))
                return fail(PKS_E_ARG, "smoother outputs overlap y");
        }
    }
    return PKS_OK;
}

pks_status loglik_impl(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                       const void* y, const void* m, const void* P, double* ll, double* tot,
                       int32_t cumulative, pks_precision prec, void* ws, size_t ws_bytes, bool batched,
                       hipStream_t s, bool tv = false) {
    pks_status st = check_model(model);
    if (st) return st;
    st = check_prec(prec);
    if (st) return st;
    if (total < 0) return fail(PKS_E_ARG, "negative number of steps");
    if (batched) {
        if (B < 1) return fail(PKS_E_ARG, "B = %d must be >= 1", B);
        if (!offsets) return fail(PKS_E_ARG, "offsets is NULL");
    } else if (model->per_sequence) {
        return fail(PKS_E_ARG, "per_sequence models need a batched call");
    }
    if (!ws) return fail(PKS_E_ARG, "workspace is NULL");
    if (!ll && !tot) return fail(PKS_E_ARG, "ll and ll_total are both NULL");
    if (cumulative && !ll) return fail(PKS_E_ARG, "cumulative output needs ll");
    const WsLayout L = ws_layout(model->nx, model->ny, total, tv ? (int32_t)total : B, prec);
    if (ws_bytes < L.total)
        return fail(PKS_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required",
                    ws_bytes, L.total);
    const size_t rs = rsize(prec), nx = model->nx, ny = model->ny, T = (size_t)total;
    const size_t by = T * ny * rs, bm = T * nx * rs, bP = T * nx * nx * rs;
    const size_t bl = T * sizeof(double), bt = (size_t)B * sizeof(double);
    if (total > 0) {
        if (!y || !m || !P) return fail(PKS_E_ARG, "y, m and P must not be NULL");
        if (overlaps(ll, bl, y, by) || overlaps(ll, bl, m, bm) || overlaps(ll, bl, P, bP) ||
            overlaps(tot, bt, y, by) || overlaps(tot, bt, m, bm) || overlaps(tot, bt, P, bP) ||
            overlaps(tot, bt, ll, bl))
            return fail(PKS_E_ARG, "log-likelihood outputs overlap the inputs or each other");
    }
    if (total == 0) {
        if (tot) {
            const hipError_t e = hipMemsetAsync(tot, 0, bt, s);   // every sequence is empty: log 1
            if (e != hipSuccess) return hip_fail(e, "clearing ll_total");
        }
        return PKS_OK;
    }
    if (debug_poison()) {
        const hipError_t pe = poison_workspace(ws, L, s);
        if (pe != hipSuccess) return hip_fail(pe, "workspace fill");
    }
    const int nmodels = tv ? (int)total : (model->per_sequence ? B : 1);
    // only G, S, e of every model (or step) are read: precompute mode 4
    hipError_t e = launch_precompute(model->nx, model->ny, nmodels, *model, ws, L, false, 4, false, s, tv,
                                     (tv && batched) ? offsets : nullptr, B);
    if (e != hipSuccess) return hip_fail(e, "precompute kernel");
    e = launch_loglik(*model, B, batched ? offsets : nullptr, total, y, m, P, ll, tot, cumulative != 0,
                      prec == PKS_MIXED_FP32, ws, L, s, tv);
    if (e != hipSuccess) return hip_fail(e, "log-likelihood kernels");
    return PKS_OK;
}

void set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

// ---------------------------------------------------------------------------
// per-kernel timing
// ---------------------------------------------------------------------------
namespace {
struct ProfMark {
    std::string name;
    hipEvent_t start, stop;
};
struct Profiler {
    bool on = false;
    std::vector<ProfMark> marks;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
thread_local Profiler g_prof;
}  // namespace

void prof_begin(const char* kernel, hipStream_t s) {
    if (!g_prof.on) return;
    ProfMark m;
    m.name = kernel;
    m.start = g_prof.get();
    m.stop = g_prof.get();
    if (m.start) (void)hipEventRecord(m.start, s);
    g_prof.marks.push_back(m);
}

void prof_end(hipStream_t s) {
    if (!g_prof.on || g_prof.marks.empty()) return;
    if (g_prof.marks.back().stop) (void)hipEventRecord(g_prof.marks.back().stop, s);
}

pks_status tv_model(const pks_model_tv* t, int64_t T, pks_model* out) {
    if (!t) return fail(PKS_E_ARG, "model is NULL");
    if (T > kMaxStepsTv) return fail(PKS_E_UNSUPPORTED, "time-varying models support at most 2^31 - 1 steps");
    out->nx = t->nx;
    out->ny = t->ny;
    out->F = t->F; out->u = t->u; out->Q = t->Q;
    out->H = t->H; out->d = t->d; out->R = t->R;
    out->m0 = t->m0; out->P0 = t->P0;
    out->per_sequence = t->per_sequence;
    return PKS_OK;
}

}  // namespace pks

using namespace pks;

extern "C" {

pks_status pks_check_offsets(int32_t B, const int64_t* offsets, int64_t total, void* ws, int32_t* first_bad,
                             void* stream) {
    g_last_error.clear();
    if (first_bad) *first_bad = -1;
    if (B < 1) return fail(PKS_E_ARG, "B = %d must be >= 1", B);
    if (!offsets) return fail(PKS_E_ARG, "offsets is NULL");
    if (!ws) return fail(PKS_E_ARG, "workspace is NULL");
    if (total < 0) return fail(PKS_E_ARG, "negative number of steps");
    hipStream_t s = (hipStream_t)stream;
    // the third word of the workspace's status block (the numeric flag uses the first two)
    int* result = static_cast<int*>(ws) + 2;
    hipError_t e = launch_offsets_check(offsets, B, total, result, s);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, result, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "offsets check");
    if (h == 0x7fffffff) return PKS_OK;
    if (first_bad) *first_bad = h;
    return fail(PKS_E_ARG, "offsets break the packing rules at index %d", h);
}

pks_status pks_set_debug_poison(int32_t on) {
    pks::g_poison.store(on ? 1 : 0);
    return PKS_OK;
}

int32_t pks_debug_poison(void) { return pks::debug_poison() ? 1 : 0; }

size_t pks_workspace_bytes(int32_t nx, int32_t ny, int64_t total_steps, int32_t B, pks_precision prec) {
    if (nx < 1 || nx > 64 || ny < 1 || ny > 64 || total_steps < 0 || B < 1) return 0;
    if (prec != PKS_FP64 && prec != PKS_MIXED_FP32) return 0;
    return ws_layout(nx, ny, total_steps, B, prec).total;
}

pks_status pks_filter(const pks_model* model, int64_t T, const void* y, void* m, void* P,
                      pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_status st = validate_io(model, 1, nullptr, T, y, m, P, nullptr, nullptr, prec, ws, 1, false);
    if (st) return st;
    return enqueue(*model, 1, nullptr, T, y, m, P, nullptr, nullptr, prec, ws, ws_bytes, 1, nullptr,
                   (hipStream_t)stream);
}

pks_status pks_smooth(const pks_model* model, int64_t T, const void* m, const void* P, void* ms, void* Ps,
                      pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_status st = validate_io(model, 1, nullptr, T, nullptr, m, P, ms, Ps, prec, ws, 2, false);
    if (st) return st;
    return enqueue(*model, 1, nullptr, T, nullptr, const_cast<void*>(m), const_cast<void*>(P), ms, Ps, prec, ws,
                   ws_bytes, 2, nullptr, (hipStream_t)stream);
}

pks_status pks_filter_smooth(const pks_model* model, int64_t T, const void* y, void* m, void* P, void* ms,
                             void* Ps, pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_status st = validate_io(model, 1, nullptr, T, y, m, P, ms, Ps, prec, ws, 3, false);
    if (st) return st;
    return enqueue(*model, 1, nullptr, T, y, m, P, ms, Ps, prec, ws, ws_bytes, 3, nullptr, (hipStream_t)stream);
}

pks_status pks_filter_batched(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                              const void* y, void* m, void* P, pks_precision prec, void* ws, size_t ws_bytes,
                              void* stream) {
    g_last_error.clear();
    pks_status st = validate_io(model, B, offsets, total, y, m, P, nullptr, nullptr, prec, ws, 1, true);
    if (st) return st;
    return enqueue(*model, B, offsets, total, y, m, P, nullptr, nullptr, prec, ws, ws_bytes, 1, nullptr,
                   (hipStream_t)stream);
}

pks_status pks_smooth_batched(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                              const void* m, const void* P, void* ms, void* Ps, pks_precision prec, void* ws,
                              size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_status st = validate_io(model, B, offsets, total, nullptr, m, P, ms, Ps, prec, ws, 2, true);
    if (st) return st;
    return enqueue(*model, B, offsets, total, nullptr, const_cast<void*>(m), const_cast<void*>(P), ms, Ps, prec,
                   ws, ws_bytes, 2, nullptr, (hipStream_t)stream);
}

pks_status pks_loglik(const pks_model* model, int64_t T, const void* y, const void* m, const void* P,
                      double* ll, double* ll_total, int32_t cumulative, pks_precision prec, void* ws,
                      size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return loglik_impl(model, 1, nullptr, T, y, m, P, ll, ll_total, cumulative, prec, ws, ws_bytes, false,
                       (hipStream_t)stream);
}

pks_status pks_loglik_batched(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                              const void* y, const void* m, const void* P, double* ll, double* ll_total,
                              int32_t cumulative, pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return loglik_impl(model, B, offsets, total, y, m, P, ll, ll_total, cumulative, prec, ws, ws_bytes, true,
                       (hipStream_t)stream);
}

// ---- time-varying models --------------------------------------------------

size_t pks_workspace_bytes_tv(int32_t nx, int32_t ny, int64_t T, pks_precision prec) {
    if (nx < 1 || nx > 64 || ny < 1 || ny > 64 || T < 0 || T > kMaxStepsTv) return 0;
    if (prec != PKS_FP64 && prec != PKS_MIXED_FP32) return 0;
    return ws_layout(nx, ny, T, (int32_t)std::max<int64_t>(T, 1), prec).total;
}

pks_status pks_filter_tv(const pks_model_tv* model, int64_t T, const void* y, void* m, void* P,
                         pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, T, &mo);
    if (!st) st = validate_io(&mo, 1, nullptr, T, y, m, P, nullptr, nullptr, prec, ws, 1, false);
    if (st) return st;
    return enqueue(mo, 1, nullptr, T, y, m, P, nullptr, nullptr, prec, ws, ws_bytes, 1, nullptr,
                   (hipStream_t)stream, true);
}

pks_status pks_smooth_tv(const pks_model_tv* model, int64_t T, const void* m, const void* P, void* ms,
                         void* Ps, pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, T, &mo);
    if (!st) st = validate_io(&mo, 1, nullptr, T, nullptr, m, P, ms, Ps, prec, ws, 2, false);
    if (st) return st;
    return enqueue(mo, 1, nullptr, T, nullptr, const_cast<void*>(m), const_cast<void*>(P), ms, Ps, prec, ws,
                   ws_bytes, 2, nullptr, (hipStream_t)stream, true);
}

pks_status pks_filter_smooth_tv(const pks_model_tv* model, int64_t T, const void* y, void* m, void* P,
                                void* ms, void* Ps, pks_precision prec, void* ws, size_t ws_bytes,
                                void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, T, &mo);
    if (!st) st = validate_io(&mo, 1, nullptr, T, y, m, P, ms, Ps, prec, ws, 3, false);
    if (st) return st;
    return enqueue(mo, 1, nullptr, T, y, m, P, ms, Ps, prec, ws, ws_bytes, 3, nullptr, (hipStream_t)stream,
                   true);
}

pks_status pks_filter_tv_batched(const pks_model_tv* model, int32_t B, const int64_t* offsets, int64_t total,
                                 const void* y, void* m, void* P, pks_precision prec, void* ws, size_t ws_bytes,
                                 void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, total, &mo);
    if (!st) st = validate_io(&mo, B, offsets, total, y, m, P, nullptr, nullptr, prec, ws, 1, true);
    if (st) return st;
    return enqueue(mo, B, offsets, total, y, m, P, nullptr, nullptr, prec, ws, ws_bytes, 1, nullptr,
                   (hipStream_t)stream, true);
}

pks_status pks_smooth_tv_batched(const pks_model_tv* model, int32_t B, const int64_t* offsets, int64_t total,
                                 const void* m, const void* P, void* ms, void* Ps, pks_precision prec, void* ws,
                                 size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, total, &mo);
    if (!st) st = validate_io(&mo, B, offsets, total, nullptr, m, P, ms, Ps, prec, ws, 2, true);
    if (st) return st;
    return enqueue(mo, B, offsets, total, nullptr, const_cast<void*>(m), const_cast<void*>(P), ms, Ps, prec, ws,
                   ws_bytes, 2, nullptr, (hipStream_t)stream, true);
}

pks_status pks_loglik_tv_batched(const pks_model_tv* model, int32_t B, const int64_t* offsets, int64_t total,
                                 const void* y, const void* m, const void* P, double* ll, double* ll_total,
                                 int32_t cumulative, pks_precision prec, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, total, &mo);
    if (st) return st;
    return loglik_impl(&mo, B, offsets, total, y, m, P, ll, ll_total, cumulative, prec, ws, ws_bytes, true,
                       (hipStream_t)stream, true);
}

pks_status pks_loglik_tv(const pks_model_tv* model, int64_t T, const void* y, const void* m, const void* P,
                         double* ll, double* ll_total, int32_t cumulative, pks_precision prec, void* ws,
                         size_t ws_bytes, void* stream) {
    g_last_error.clear();
    pks_model mo;
    pks_status st = tv_model(model, T, &mo);
    if (st) return st;
    return loglik_impl(&mo, 1, nullptr, T, y, m, P, ll, ll_total, cumulative, prec, ws, ws_bytes, false,
                       (hipStream_t)stream, true);
}

// ---- discrete-state hidden Markov model --------------------------------------
namespace {
pks_status hmm_impl(const pks_hmm* model, int64_t T, const double* L, double* alpha, double* logp,
                    double* gamma, void* ws, size_t ws_bytes, int passes, hipStream_t s) {
    if (!model) return fail(PKS_E_ARG, "model is NULL");
    if (model->K < 1 || model->K > 64) return fail(PKS_E_ARG, "K = %d outside [1, 64]", model->K);
    if (!model->Pi || !model->p0) return fail(PKS_E_ARG, "Pi and p0 are required");
    if (T < 0) return fail(PKS_E_ARG, "negative number of steps");
    if (!ws) return fail(PKS_E_ARG, "workspace is NULL");
    const size_t need = hmm_ws_bytes(model->K, T);
    if (ws_bytes < need)
        return fail(PKS_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu bytes required", ws_bytes, need);
    if (T == 0) return PKS_OK;
    const size_t bK = (size_t)T * model->K * sizeof(double), bT = (size_t)T * sizeof(double);
    if ((passes & 1) && (!L || !alpha)) return fail(PKS_E_ARG, "L and alpha must not be NULL");
    if ((passes & 2) && (!alpha || !gamma)) return fail(PKS_E_ARG, "alpha and gamma must not be NULL");
    if ((passes & 1) && (overlaps(L, bK, alpha, bK) || overlaps(L, bK, logp, bT) || overlaps(alpha, bK, logp, bT)))
        return fail(PKS_E_ARG, "filter outputs overlap the input or each other");
    if ((passes & 2) && (overlaps(gamma, bK, alpha, bK) || overlaps(gamma, bK, logp, bT) ||
                         ((passes & 1) && overlaps(gamma, bK, L, bK))))
        return fail(PKS_E_ARG, "smoother output overlaps the inputs or the other outputs");
    if (debug_poison()) {
        const hipError_t pe = launch_poison(ws, need, s);
        if (pe != hipSuccess) return hip_fail(pe, "workspace fill");
    }
    const hipError_t e = launch_hmm(model->K, T, model->Pi, model->p0, L, alpha, logp, gamma, ws, passes, s);
    if (e != hipSuccess) return hip_fail(e, "HMM kernels");
    return PKS_OK;
}
}  // namespace

size_t pks_hmm_workspace_bytes(int32_t K, int64_t T) {
    if (K < 1 || K > 64 || T < 0) return 0;
    return hmm_ws_bytes(K, T);
}

pks_status pks_hmm_filter(const pks_hmm* model, int64_t T, const double* L, double* alpha, double* logp, void* ws,
                          size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return hmm_impl(model, T, L, alpha, logp, nullptr, ws, ws_bytes, 1, (hipStream_t)stream);
}

pks_status pks_hmm_smooth(const pks_hmm* model, int64_t T, const double* alpha, double* gamma, void* ws,
                          size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return hmm_impl(model, T, nullptr, const_cast<double*>(alpha), nullptr, gamma, ws, ws_bytes, 2,
                    (hipStream_t)stream);
}

pks_status pks_hmm_filter_smooth(const pks_hmm* model, int64_t T, const double* L, double* alpha, double* logp,
                                 double* gamma, void* ws, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    return hmm_impl(model, T, L, alpha, logp, gamma, ws, ws_bytes, 3, (hipStream_t)stream);
}

pks_status pks_read_numeric_status(void* ws, int32_t* first_bad_sequence, void* stream) {
    g_last_error.clear();
    if (!ws) return fail(PKS_E_ARG, "workspace is NULL");
    hipStream_t s = (hipStream_t)stream;
    int host[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(host, ws, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading the numeric flag");
    const bool prepared = host[1] == kStatusMagic;
    const int bad = prepared ? host[0] : kStatusOk;
    const int clean[2] = {kStatusOk, kStatusMagic};
    e = hipMemcpyAsync(ws, clean, sizeof clean, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "clearing the numeric flag");
    if (bad != kStatusOk) {
        if (first_bad_sequence) *first_bad_sequence = bad;
        return fail(PKS_E_NUMERIC, "a Cholesky factorisation failed in sequence %d", bad);
    }
    if (first_bad_sequence) *first_bad_sequence = -1;
    return PKS_OK;
}

pks_status pks_profile_start(void) {
    g_last_error.clear();
    g_prof.on = true;
    return PKS_OK;
}

pks_status pks_profile_stop(int32_t max_kernels, char* names, float* total_ms, int32_t* launches,
                            int32_t* n_kernels) {
    g_last_error.clear();
    g_prof.on = false;
    hipError_t e = hipDeviceSynchronize();
    std::vector<std::string> order;
    std::vector<double> tot;
    std::vector<int> cnt;
    for (auto& m : g_prof.marks) {
        float ms = 0.f;
        if (e == hipSuccess && m.start && m.stop) e = hipEventElapsedTime(&ms, m.start, m.stop);
        size_t i = 0;
        while (i < order.size() && order[i] != m.name) ++i;
        if (i == order.size()) {
            order.push_back(m.name);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[i] += ms;
        cnt[i] += 1;
        if (m.start) g_prof.pool.push_back(m.start);
        if (m.stop) g_prof.pool.push_back(m.stop);
    }
    g_prof.marks.clear();
    if (e != hipSuccess) return hip_fail(e, "kernel timing");
    const int n = (int)std::min<size_t>(order.size(), max_kernels > 0 ? (size_t)max_kernels : 0);
    for (int i = 0; i < n; ++i) {
        if (names) {
            strncpy(names + 64 * i, order[i].c_str(), 63);
            names[64 * i + 63] = 0;
        }
        if (total_ms) total_ms[i] = (float)tot[i];
        if (launches) launches[i] = cnt[i];
    }
    if (n_kernels) *n_kernels = n;
    return PKS_OK;
}

const char* pks_last_error(void) { return g_last_error.c_str(); }

const char* pks_version(void) { return "pks 0.1 (gfx950)"; }

}  // extern "C"
