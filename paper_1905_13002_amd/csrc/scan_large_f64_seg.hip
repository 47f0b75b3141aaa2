// Large-state scan kernels, FP64 storage, packed batched sequences.
#include "scan_large_impl.hpp"

template hipError_t pks::lg::run_large<double, true>(pks::lg::LargeArgs, bool, hipStream_t);
