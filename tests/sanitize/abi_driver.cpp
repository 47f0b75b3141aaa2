// Drives the host side of libpks (argument validation, workspace sizing, the
// tuning-cache parser, error reporting) through every rejection path, built
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host.  Device
// pointers are fake addresses that validation never dereferences; a request
// that passes validation reaches the HIP runtime, which fails cleanly when no
// GPU (or no device code) is present, so no kernel runs.  Exit status 0 when
// every call returns the expected code.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "pks.h"

static int fails = 0;
#define EXPECT(c)                                                                \
    do {                                                                         \
        if (!(c)) {                                                              \
            fprintf(stderr, "FAILED line %d: %s (%s)\n", __LINE__, #c, pks_last_error()); \
            ++fails;                                                             \
        }                                                                        \
    } while (0)

static void* fake(uintptr_t off) { return reinterpret_cast<void*>(uintptr_t(0x100000000ull) + off); }

static pks_model model(int nx, int ny) {
    pks_model m;
    memset(&m, 0, sizeof m);
    m.nx = nx;
    m.ny = ny;
    m.F = (const double*)fake(0x1000);
    m.Q = (const double*)fake(0x2000);
    m.H = (const double*)fake(0x3000);
    m.R = (const double*)fake(0x4000);
    m.m0 = (const double*)fake(0x5000);
    m.P0 = (const double*)fake(0x6000);
    return m;
}

int main() {
    // workspace sizing over a grid of shapes, both precisions, and bad shapes
    for (int nx = 1; nx <= 64; nx += (nx < 8 ? 1 : 7))
        for (int ny = 1; ny <= 64; ny += (ny < 4 ? 1 : 13))
            for (int64_t T : {int64_t(0), int64_t(1), int64_t(5), int64_t(1000), int64_t(1) << 20})
                for (int p = 0; p < 2; ++p) {
                    const size_t a = pks_workspace_bytes(nx, ny, T, 1, (pks_precision)p);
                    const size_t b = pks_workspace_bytes(nx, ny, T, 7, (pks_precision)p);
                    EXPECT(a > 0 && b >= a);
                    EXPECT(pks_workspace_bytes_tv(nx, ny, T, (pks_precision)p) > 0);
                }
    EXPECT(pks_workspace_bytes(0, 2, 10, 1, PKS_FP64) == 0 && pks_workspace_bytes(4, 65, 10, 1, PKS_FP64) == 0);
    EXPECT(pks_workspace_bytes(4, 2, -1, 1, PKS_FP64) == 0 && pks_workspace_bytes(4, 2, 10, 0, PKS_FP64) == 0);
    EXPECT(pks_workspace_bytes(4, 2, 10, 1, (pks_precision)9) == 0);
    EXPECT(pks_workspace_bytes_tv(4, 2, int64_t(1) << 40, PKS_FP64) == 0);
    for (int K = 1; K <= 64; ++K) EXPECT(pks_hmm_workspace_bytes(K, 12345) > 0);
    EXPECT(pks_hmm_workspace_bytes(0, 10) == 0 && pks_hmm_workspace_bytes(65, 10) == 0);

    // filter / smoother / batched / time-varying / likelihood argument errors
    pks_model m = model(4, 2);
    void *y = fake(0x100000), *mm = fake(0x200000), *P = fake(0x300000), *ms = fake(0x400000), *Ps = fake(0x500000);
    void* ws = fake(0x1000000);
    const size_t wsb = pks_workspace_bytes(4, 2, 16, 1, PKS_FP64);
    EXPECT(pks_filter(nullptr, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    pks_model bad = model(0, 2);
    EXPECT(pks_filter(&bad, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    bad = model(4, 2);
    bad.R = nullptr;
    EXPECT(pks_filter(&bad, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter(&m, -1, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter(&m, 16, nullptr, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter(&m, 16, y, mm, P, (pks_precision)3, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter(&m, 16, y, mm, P, PKS_FP64, nullptr, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter(&m, 16, y, (char*)y + 8, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter(&m, 16, y, mm, P, PKS_FP64, ws, wsb - 1, nullptr) == PKS_E_WORKSPACE);
    EXPECT(pks_filter(&m, 0, nullptr, nullptr, nullptr, PKS_FP64, ws, wsb, nullptr) == PKS_OK);
    EXPECT(pks_smooth(&m, 16, mm, P, mm, Ps, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter_smooth(&m, 16, y, mm, P, ms, y, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    pks_model per = model(4, 2);
    per.per_sequence = 1;
    EXPECT(pks_filter(&per, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    const int64_t* off = (const int64_t*)fake(0x900000);
    EXPECT(pks_filter_batched(&m, 0, off, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter_batched(&m, 2, nullptr, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_smooth_batched(&m, 2, off, 16, mm, P, nullptr, Ps, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    double *ll = (double*)fake(0xA00000), *tot = (double*)fake(0xB00000);
    EXPECT(pks_loglik(&m, 16, y, mm, P, nullptr, nullptr, 0, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_loglik(&m, 16, y, mm, P, nullptr, tot, 1, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_loglik(&m, 16, y, mm, P, (double*)y, tot, 0, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_loglik_batched(&m, 0, off, 16, y, mm, P, ll, tot, 0, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    pks_model_tv tv;
    memset(&tv, 0, sizeof tv);
    tv.nx = 4;
    tv.ny = 2;
    EXPECT(pks_filter_tv(nullptr, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter_tv(&tv, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr) == PKS_E_ARG);   // null matrices
    EXPECT(pks_loglik_tv(&tv, int64_t(1) << 40, y, mm, P, ll, tot, 0, PKS_FP64, ws, wsb, nullptr) ==
           PKS_E_UNSUPPORTED);

    // discrete-state model
    pks_hmm h;
    h.K = 4;
    h.Pi = (const double*)fake(0x1000);
    h.p0 = (const double*)fake(0x2000);
    const size_t hw = pks_hmm_workspace_bytes(4, 16);
    double *L = (double*)fake(0x100000), *al = (double*)fake(0x200000), *lp = (double*)fake(0x300000),
           *ga = (double*)fake(0x400000);
    EXPECT(pks_hmm_filter(nullptr, 16, L, al, lp, ws, hw, nullptr) == PKS_E_ARG);
    EXPECT(pks_hmm_filter(&h, 16, L, al, lp, ws, hw - 1, nullptr) == PKS_E_WORKSPACE);
    EXPECT(pks_hmm_filter(&h, 16, L, L + 1, lp, ws, hw, nullptr) == PKS_E_ARG);
    EXPECT(pks_hmm_smooth(&h, 16, al, al, ws, hw, nullptr) == PKS_E_ARG);
    EXPECT(pks_hmm_filter_smooth(&h, 0, nullptr, nullptr, nullptr, nullptr, ws, hw, nullptr) == PKS_OK);
    h.K = 65;
    EXPECT(pks_hmm_filter(&h, 16, L, al, lp, ws, hw, nullptr) == PKS_E_ARG);

    // plans, autotuner, status, diagnostics
    void* plan = nullptr;
    EXPECT(pks_plan_create(&m, 1, nullptr, 16, y, mm, P, ms, Ps, PKS_FP64, ws, wsb, nullptr, nullptr, nullptr) ==
           PKS_E_ARG);
    EXPECT(pks_plan_create(&m, 3, nullptr, 16, y, mm, P, ms, Ps, PKS_FP64, ws, wsb, nullptr, nullptr, &plan) ==
           PKS_E_ARG && plan == nullptr);
    EXPECT(pks_plan_launch(nullptr, nullptr) == PKS_E_ARG);
    EXPECT(pks_plan_destroy(nullptr) == PKS_OK);
    unsetenv("PKS_TUNE_CACHE");
    EXPECT(pks_autotune(4, 2, 1, 1000, PKS_FP64, nullptr, nullptr) == PKS_E_ARG);
    EXPECT(pks_autotune(0, 2, 1, 1000, PKS_FP64, "/tmp/unused.json", nullptr) == PKS_E_ARG);
    EXPECT(pks_read_numeric_status(nullptr, nullptr, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter_smooth_noalloc(nullptr, 16, y, mm, P, ms, Ps, PKS_FP64, nullptr) == PKS_E_ARG);
    EXPECT(pks_filter_smooth_noalloc(&m, int64_t(1) << 24, y, mm, P, ms, Ps, PKS_FP64, nullptr) ==
           PKS_E_UNSUPPORTED);
    EXPECT(pks_noalloc_scratch_bytes() > 0);
    EXPECT(std::string(pks_version()).find("pks") != std::string::npos);

    // a request that passes validation reads the tuning cache (malformed lines
    // are skipped) and then stops at the first HIP call, which fails without a
    // GPU: the parser and the argument assembly run under the sanitizers
    const char* cache = getenv("PKS_DRIVER_CACHE");
    if (cache) {
        FILE* f = fopen(cache, "w");
        if (f) {
            fputs("{\n  \"nx4_ny2_fp64_T4_B0\": [8, 1, 0],\n  \"broken\n  \"x\": [\n  \"nx4_ny2_fp64_T5_B0\": [99, 99]\n}\n",
                  f);
            fclose(f);
        }
        setenv("PKS_TUNE_CACHE", cache, 1);
        const pks_status st = pks_filter(&m, 16, y, mm, P, PKS_FP64, ws, wsb, nullptr);
        EXPECT(st == PKS_E_HIP || st == PKS_OK);
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("abi driver: all checks passed\n");
    return 0;
}
