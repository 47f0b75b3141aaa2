// plan.cpp -- HIP-graph plans, the tile-configuration cache and the autotuner.
//
// A plan captures the whole filter + smoother of one (batched) problem --
// status preparation, model precompute and every scan kernel -- into one HIP
// graph, so a replay is a single hipGraphLaunch.  The tile configuration
// (elements per thread at the step level, and whether a second scan level
// over the wave aggregates is used) comes from a small JSON cache written by
// pks_autotune, keyed by (nx, ny, precision, log2 steps, log2 sequences).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "plan.h"

namespace pks {

namespace {

std::mutex g_cache_mu;

int ilog2(int64_t v) {
    int r = 0;
    while (v > 1) { v >>= 1; ++r; }
    return r;
}

std::string cache_key(int nx, int ny, int32_t B, int64_t total, pks_precision prec) {
    char buf[128];
    snprintf(buf, sizeof buf, "nx%d_ny%d_%s_T%d_B%d", nx, ny, prec == PKS_FP64 ? "fp64" : "mixed",
             ilog2(std::max<int64_t>(1, total)), ilog2(std::max<int32_t>(1, B)));
    return buf;
}

const char* cache_path_or_env(const char* path) {
    if (path && *path) return path;
    const char* env = getenv("PKS_TUNE_CACHE");
    return (env && *env) ? env : nullptr;
}

// The cache is a flat JSON object {"key": [ept, ept1, blocks], ...}, one entry
// a line (entries of two numbers, from before the large-state tuning, read
// with blocks = 0).
std::map<std::string, TileConfig> read_cache(const char* path) {
    std::map<std::string, TileConfig> out;
    if (!path) return out;
    std::ifstream f(path);
    if (!f) return out;
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        const size_t b0 = line.find('[', q1);
        if (q1 == std::string::npos || b0 == std::string::npos) continue;
        int e0 = 0, e1 = 0, e2 = 0;
        const int n = sscanf(line.c_str() + b0, "[ %d , %d , %d ]", &e0, &e1, &e2);
        if (n >= 2) {
            TileConfig c;
            c.ept = e0;
            c.ept1 = e1;
            c.blocks = n == 3 ? e2 : 0;
            out[line.substr(q0 + 1, q1 - q0 - 1)] = c;
        }
    }
    return out;
}

bool write_cache(const char* path, const std::map<std::string, TileConfig>& m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t i = 0;
        for (const auto& kv : m) {
            f << "  \"" << kv.first << "\": [" << kv.second.ept << ", " << kv.second.ept1 << ", "
              << kv.second.blocks << "]"
              << (++i < m.size() ? "," : "") << "\n";
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path) == 0;
}

bool valid_config(const TileConfig& c, int nx) {
    if (!small_supported(nx)) return c.blocks >= 1;
    return (c.ept == 4 || c.ept == 8 || c.ept == 16) && (c.ept1 == 0 || c.ept1 == 1 || c.ept1 == 2 || c.ept1 == 4 || c.ept1 == 8);
}

struct Plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

TileConfig tuned_config(int nx, int ny, int32_t B, int64_t total, pks_precision prec, const char* path) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    const char* p = cache_path_or_env(path);
    if (p) {
        auto m = read_cache(p);
        auto it = m.find(cache_key(nx, ny, B, total, prec));
        if (it != m.end() && valid_config(it->second, nx)) return it->second;
    }
    return small_default_config(nx, total, prec == PKS_MIXED_FP32);
}

}  // namespace pks

using namespace pks;

namespace {

// Capture one filter + smoother pass of a validated request into a HIP graph
// (on a private stream) and instantiate it.  tv: time-varying model.
pks_status capture_plan(const pks_model& model, int32_t B, const int64_t* offsets, int64_t total, const void* y,
                        void* m, void* P, void* ms, void* Ps, pks_precision prec, void* ws, size_t ws_bytes,
                        const TileConfig& cfg, bool tv, void** plan) {
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        return PKS_E_HIP;
    }
    Plan* p = new Plan();
    pks_status st = PKS_OK;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = enqueue(model, B, offsets, total, y, m, P, ms, Ps, prec, ws, ws_bytes, 3, &cfg, cap, tv);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cap, &g);
        p->graph = g;
        if (st == PKS_OK && e2 != hipSuccess) e = e2;
    }
    if (st == PKS_OK && e == hipSuccess && p->graph) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    hipStreamDestroy(cap);
    if (st != PKS_OK || e != hipSuccess || !p->exec) {
        if (p->exec) hipGraphExecDestroy(p->exec);
        if (p->graph) hipGraphDestroy(p->graph);
        delete p;
        if (st != PKS_OK) return st;
        set_last_error(hipGetErrorString(e));
        return PKS_E_HIP;
    }
    *plan = p;
    return PKS_OK;
}

}  // namespace

extern "C" {

pks_status pks_plan_create(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                           const void* y, void* m, void* P, void* ms, void* Ps, pks_precision prec,
                           void* ws, size_t ws_bytes, const char* tune_cache, void* stream, void** plan) {
    set_last_error("");
    (void)stream;
    if (!plan) {
        set_last_error("plan is NULL");
        return PKS_E_ARG;
    }
    *plan = nullptr;
    const bool batched = offsets != nullptr;
    if (!batched && B != 1) {
        set_last_error("B must be 1 when offsets is NULL");
        return PKS_E_ARG;
    }
    pks_status st = validate_io(model, B, offsets, total, y, m, P, ms, Ps, prec, ws, 3, batched);
    if (st) return st;
    const TileConfig cfg = tuned_config(model->nx, model->ny, B, total, prec, tune_cache);
    return capture_plan(*model, B, offsets, total, y, m, P, ms, Ps, prec, ws, ws_bytes, cfg, false, plan);
}

pks_status pks_plan_create_tv(const pks_model_tv* model, int32_t B, const int64_t* offsets, int64_t total,
                              const void* y, void* m, void* P, void* ms, void* Ps, pks_precision prec,
                              void* ws, size_t ws_bytes, const char* tune_cache, void* stream, void** plan) {
    set_last_error("");
    (void)stream;
    if (!plan) {
        set_last_error("plan is NULL");
        return PKS_E_ARG;
    }
    *plan = nullptr;
    const bool batched = offsets != nullptr;
    if (!batched && B != 1) {
        set_last_error("B must be 1 when offsets is NULL");
        return PKS_E_ARG;
    }
    pks_model mo;
    pks_status st = tv_model(model, total, &mo);
    if (!st) st = validate_io(&mo, B, offsets, total, y, m, P, ms, Ps, prec, ws, 3, batched);
    if (st) return st;
    const TileConfig cfg = tuned_config(mo.nx, mo.ny, B, total, prec, tune_cache);
    return capture_plan(mo, B, offsets, total, y, m, P, ms, Ps, prec, ws, ws_bytes, cfg, true, plan);
}

pks_status pks_plan_launch(void* plan, void* stream) {
    set_last_error("");
    if (!plan) {
        set_last_error("plan is NULL");
        return PKS_E_ARG;
    }
    Plan* p = static_cast<Plan*>(plan);
    const hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        return PKS_E_HIP;
    }
    return PKS_OK;
}

pks_status pks_plan_destroy(void* plan) {
    set_last_error("");
    if (!plan) return PKS_OK;
    Plan* p = static_cast<Plan*>(plan);
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    delete p;
    return PKS_OK;
}

pks_status pks_autotune(int32_t nx, int32_t ny, int32_t B, int64_t total, pks_precision prec,
                        const char* cache_path, void* stream) {
    set_last_error("");
    const char* path = cache_path_or_env(cache_path);
    if (!path) {
        set_last_error("no cache path (argument or PKS_TUNE_CACHE)");
        return PKS_E_ARG;
    }
    if (nx < 1 || nx > 64 || ny < 1 || ny > 64 || B < 1 || total < 1) {
        set_last_error("invalid problem shape");
        return PKS_E_ARG;
    }
    if (prec != PKS_FP64 && prec != PKS_MIXED_FP32) {
        set_last_error("unknown precision");
        return PKS_E_ARG;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t rs = prec == PKS_FP64 ? 8 : 4;
    const int64_t T = total;
    // synthetic problem: a stable random-walk model (F = I with a weak
    // velocity-like coupling, Q = 0.1 I, H = [I 0], R = I), lengths equal.
    std::vector<double> hF(nx * nx, 0.0), hQ(nx * nx, 0.0), hH(ny * nx, 0.0), hR(ny * ny, 0.0), hm0(nx, 0.0),
        hP0(nx * nx, 0.0);
    for (int i = 0; i < nx; ++i) {
        hF[i * nx + i] = 1.0;
        if (i + 1 < nx) hF[i * nx + i + 1] = 0.1;
        hQ[i * nx + i] = 0.1;
        hP0[i * nx + i] = 1.0;
    }
    for (int i = 0; i < ny; ++i) {
        hH[i * nx + (i % nx)] = 1.0;
        hR[i * ny + i] = 1.0;
    }
    std::vector<int64_t> hoff(B + 1);
    for (int b = 0; b <= B; ++b) hoff[b] = (T * b) / B;
    const size_t bytes_model = sizeof(double) * (hF.size() + hQ.size() + hH.size() + hR.size() + hm0.size() + hP0.size());
    const size_t by = rs * T * ny, bm = rs * T * nx, bP = rs * T * nx * nx;
    const size_t wsb = ws_layout(nx, ny, T, B, prec).total;
    char* buf = nullptr;
    const size_t off_model = 0, off_off = (bytes_model + 255) & ~size_t(255);
    const size_t off_y = (off_off + sizeof(int64_t) * (B + 1) + 255) & ~size_t(255);
    const size_t off_m = (off_y + by + 255) & ~size_t(255);
    const size_t off_P = (off_m + bm + 255) & ~size_t(255);
    const size_t off_ms = (off_P + bP + 255) & ~size_t(255);
    const size_t off_Ps = (off_ms + bm + 255) & ~size_t(255);
    const size_t off_ws = (off_Ps + bP + 255) & ~size_t(255);
    const size_t all = off_ws + wsb;
    hipError_t e = hipMalloc(&buf, all);
    if (e != hipSuccess) {
        set_last_error(hipGetErrorString(e));
        return PKS_E_HIP;
    }
    pks_status result = PKS_OK;
    double* dm = reinterpret_cast<double*>(buf + off_model);
    size_t o = 0;
    auto put = [&](const std::vector<double>& v) {
        double* d = dm + o;
        hipMemcpy(d, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice);
        o += v.size();
        return d;
    };
    pks_model model{};
    model.nx = nx;
    model.ny = ny;
    model.F = put(hF);
    model.Q = put(hQ);
    model.H = put(hH);
    model.R = put(hR);
    model.m0 = put(hm0);
    model.P0 = put(hP0);
    model.per_sequence = 0;
    int64_t* doff = reinterpret_cast<int64_t*>(buf + off_off);
    hipMemcpy(doff, hoff.data(), sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice);
    hipMemset(buf + off_y, 0, by);
    const int64_t* offs = B > 1 ? doff : nullptr;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    TileConfig best = small_default_config(nx, total, prec == PKS_MIXED_FP32);
    float best_ms = 1e30f;
    // the candidates: register path (nx <= 4): elements per thread at both
    // levels; large states: the number of time blocks (Section III-C's block
    // length l = T / blocks), from the count the workspace is sized for down
    // to an eighth of it (fewer, longer blocks: less scan work across blocks,
    // fewer workgroups in flight)
    std::vector<TileConfig> cands;
    if (small_supported(nx)) {
        const int epts[3] = {4, 8, 16};
        const int ept1s[5] = {0, 1, 2, 4, 8};
        for (int ei = 0; ei < 3; ++ei)
            for (int li = 0; li < 5; ++li) {
                TileConfig c;
                c.ept = epts[ei];
                c.ept1 = ept1s[li];
                const int64_t waves = (T + 64 * c.ept - 1) / (64 * c.ept);
                if (c.ept1 == 0 && waves > (int64_t)64 * 256) continue;    // top level would be too long
                if (c.ept1 != 0 && waves < 128) continue;                  // second level not useful
                cands.push_back(c);
            }
    } else {
        const int64_t cap = large_default_blocks(nx, ny, T, prec == PKS_MIXED_FP32);
        for (int64_t nb = cap; nb >= 1 && cands.size() < 4; nb /= 2) {
            TileConfig c;
            c.blocks = (int)nb;
            cands.push_back(c);
        }
        best = cands.front();
    }
    for (const TileConfig& c : cands) {
        {
            float tot = 0.f;
            int reps = 0;
            pks_status st = PKS_OK;
            for (int r = 0; r < 4 && st == PKS_OK; ++r) {
                hipEventRecord(e0, s);
                st = enqueue(model, B, offs, T, buf + off_y, buf + off_m, buf + off_P, buf + off_ms, buf + off_Ps,
                             prec, buf + off_ws, wsb, 3, &c, s);
                hipEventRecord(e1, s);
                hipEventSynchronize(e1);
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                if (r > 0) {          // first run warms up
                    tot += ms;
                    ++reps;
                }
            }
            if (st != PKS_OK) {
                result = st;
                break;
            }
            const float avg = reps ? tot / reps : 1e30f;
            if (avg < best_ms) {
                best_ms = avg;
                best = c;
            }
        }
        if (result != PKS_OK) break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamSynchronize(s);
    hipFree(buf);
    if (result != PKS_OK) return result;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto m = read_cache(path);
    m[cache_key(nx, ny, B, total, prec)] = best;
    if (!write_cache(path, m)) {
        set_last_error("could not write the tuning cache");
        return PKS_E_ARG;
    }
    return PKS_OK;
}

}  // extern "C"
