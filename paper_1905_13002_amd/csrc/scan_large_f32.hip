// Large-state scan kernels, FP32 (mixed) storage, single sequences.
#include "scan_large_impl.hpp"

template hipError_t pks::lg::run_large<float, false>(pks::lg::LargeArgs, bool, hipStream_t);
