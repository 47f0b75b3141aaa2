// Large-state scan kernels, FP64 storage, single sequences.
#include "scan_large_impl.hpp"

template hipError_t pks::lg::run_large<double, false>(pks::lg::LargeArgs, bool, hipStream_t);
