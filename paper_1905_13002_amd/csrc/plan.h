// plan.h -- tile configuration cache, HIP-graph plans and the autotuner.
#pragma once
#include "pks_internal.h"

namespace pks {

// Tile configuration for a problem shape: the tuning cache entry if one
// exists (cache file: `path`, else $PKS_TUNE_CACHE), else the default.
TileConfig tuned_config(int nx, int ny, int32_t B, int64_t total, pks_precision prec,
                        const char* path = nullptr);

// Enqueue passes (1 = filter, 2 = smoother, 3 = both) of a validated request.
// tv: `model` holds one row per step (time-varying; single sequence).
pks_status enqueue(const pks_model& model, int32_t B, const int64_t* offsets, int64_t total,
                   const void* y, void* m, void* P, void* ms, void* Ps, pks_precision prec,
                   void* ws, size_t ws_bytes, int passes, const TileConfig* forced, hipStream_t s,
                   bool tv = false);

pks_status validate_io(const pks_model* model, int32_t B, const int64_t* offsets, int64_t total,
                       const void* y, const void* m, const void* P, const void* ms, const void* Ps,
                       pks_precision prec, void* ws, int passes, bool batched);

void set_last_error(const char* msg);

// A time-varying model viewed as a pks_model whose arrays hold one row per
// step (checks the step limit of time-varying models).
pks_status tv_model(const pks_model_tv* t, int64_t T, pks_model* out);

}  // namespace pks
