// Instantiates the small-state scan kernels for nx = 1, float storage.
#include "scan_small_impl.hpp"

namespace pks {
template hipError_t small_run<1, float>(ScanArgs, int, hipStream_t);
}
