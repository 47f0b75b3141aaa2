// scan_small.hip -- dispatch of the small-state (nx <= 4) scans to the
// per-dimension, per-precision kernel instantiations.
#include "pks_internal.h"

namespace pks {

template <int N, typename R>
hipError_t small_run(ScanArgs a, int passes, hipStream_t s);

namespace {

template <typename R>
hipError_t dispatch_n(ScanArgs a, int passes, hipStream_t s) {
    switch (a.nx) {
        case 1: return small_run<1, R>(a, passes, s);
        case 2: return small_run<2, R>(a, passes, s);
        case 3: return small_run<3, R>(a, passes, s);
        case 4: return small_run<4, R>(a, passes, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool small_supported(int nx) { return nx >= 1 && nx <= 4; }

// Defaults measured on MI355X (constant-velocity model, T = 2^20): FP64 is
// fastest with 16 steps per thread, the mixed mode with 8, both with a single
// scan level under the device-wide top level (which folds ceil(waves / 1024)
// aggregates per element).  Beyond 16384 waves (E > 16 sequential folds at the
// top) a second level of one aggregate per thread is inserted.
// pks_autotune overrides these per problem shape.
TileConfig small_default_config(int nx, int64_t total, bool mixed) {
    (void)nx;
    TileConfig c;
    // the longest per-thread fold that still gives every SIMD (1024 on the
    // chip) a wave; shorter sequences take the shortest fold (more threads,
    // a shorter dependent chain per thread)
    const int64_t simds = 1024;
    const int emax = mixed ? 8 : 16;
    c.ept = 4;
    for (int e = emax; e > 4; e >>= 1)
        if (total >= (int64_t)64 * e * simds) {
            c.ept = e;
            break;
        }
    const int64_t waves = (total + 64 * c.ept - 1) / (64 * c.ept);
    c.ept1 = waves > 16 * 1024 ? 1 : 0;
    return c;
}

hipError_t launch_small(ScanArgs a, bool mixed, int passes, hipStream_t s) {
    return mixed ? dispatch_n<float>(a, passes, s) : dispatch_n<double>(a, passes, s);
}

}  // namespace pks
