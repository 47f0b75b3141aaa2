// scan_large.hip -- host side of the large-state scans (5 <= nx <= 64):
// block counts, arena placement (LDS or workspace slot), workspace size and
// the dispatch to the per-precision instantiations of run_large.
#include "scan_large_impl.hpp"

namespace pks {
namespace lg {

extern template hipError_t run_large<double, false>(LargeArgs, bool, hipStream_t);
extern template hipError_t run_large<double, true>(LargeArgs, bool, hipStream_t);
extern template hipError_t run_large<float, false>(LargeArgs, bool, hipStream_t);
extern template hipError_t run_large<float, true>(LargeArgs, bool, hipStream_t);

namespace {

size_t arena_bytes_prec(int nx, int ny, bool mixed, int kind) {
    return mixed ? arena_bytes<float>(nx, ny, kind) : arena_bytes<double>(nx, ny, kind);
}

// arena kinds too large for LDS, and the largest of them (the workspace slot)
int slot_mask_of(int nx, int ny, bool mixed, size_t* slot_bytes) {
    int mask = 0;
    size_t big = 0;
    for (int k = 0; k < kArKinds; ++k) {
        const size_t b = arena_bytes_prec(nx, ny, mixed, k);
        if (b > kMaxLdsArena) {
            mask |= 1 << k;
            if (b > big) big = b;
        }
    }
    if (slot_bytes) *slot_bytes = (big + 255) & ~size_t(255);
    return mask;
}

// Blocks of the time axis: about 2048 one-wave workgroups for nx <= 16 and
// 1024 otherwise when every per-step kernel keeps its arena in LDS; 2048 when
// some arena lives in the workspace (more workgroups in flight hide its
// latency).  At least 4 steps per block.
int64_t large_blocks(int64_t total, int nx, int ny, bool mixed) {
    const bool in_lds = slot_mask_of(nx, ny, mixed, nullptr) == 0;
    const int64_t cap = (in_lds && nx > 16) ? 1024 : 2048;
    int64_t nb = (total + 3) / 4;
    if (nb > cap) nb = cap;
    return nb < 1 ? 1 : nb;
}

}  // namespace
}  // namespace lg

int64_t large_default_blocks(int nx, int ny, int64_t total, bool mixed) {
    if (w16_applies(nx, ny, true)) return w16_default_blocks(total);
    return lg::large_blocks(total, nx, ny, mixed);
}

size_t large_ws_bytes(int nx, int ny, int64_t total, pks_precision prec) {
    using namespace lg;
    const bool mixed = prec != PKS_FP64;
    const size_t rs = mixed ? 4 : 8;
    const int64_t nb = large_blocks(total, nx, ny, mixed);
    const size_t fw = (size_t)flay(nx).words;
    size_t slot = 0;
    slot_mask_of(nx, ny, mixed, &slot);
    const size_t lds_path = 2 * ((rs * fw * nb + 255) & ~size_t(255)) + slot * nb;
    // time-invariant models with nx <= 16 (one sequence or packed sequences)
    // take the register-resident path
    const size_t reg_path = w16_applies(nx, ny, true) ? w16_ws_bytes(total) : 0;
    return lds_path > reg_path ? lds_path : reg_path;
}

hipError_t launch_large(ScanArgs a, void* region, bool mixed, bool smoother, bool both, hipStream_t s) {
    using namespace lg;
    if (w16_applies(a.nx, a.ny, a.step_stride == 0))
        return launch_w16(a, region, mixed, smoother, both, s);
    LargeArgs la;
    la.s = a;
    const int64_t nb_max = large_blocks(a.total, a.nx, a.ny, mixed);
    // a tuned block count is honoured up to the count the workspace is sized for
    la.nblocks = (a.large_blocks > 0 && a.large_blocks < nb_max) ? a.large_blocks : nb_max;
    la.blen = (a.total + la.nblocks - 1) / la.nblocks;
    la.nblocks = (a.total + la.blen - 1) / la.blen;
    const size_t rs = mixed ? 4 : 8;
    const size_t fw = (size_t)flay(a.nx).words;
    const size_t one = (rs * fw * nb_max + 255) & ~size_t(255);
    char* base = static_cast<char*>(region);
    la.agg[0] = base;
    la.agg[1] = base + one;
    la.final_buf = 0;
    la.slot_mask = slot_mask_of(a.nx, a.ny, mixed, &la.slot_bytes);
    la.slots = la.slot_mask ? base + 2 * one : nullptr;
    const bool seg = a.offsets != nullptr;
    if (mixed) return seg ? run_large<float, true>(la, smoother, s) : run_large<float, false>(la, smoother, s);
    return seg ? run_large<double, true>(la, smoother, s) : run_large<double, false>(la, smoother, s);
}

}  // namespace pks
