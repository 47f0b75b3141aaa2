// Instantiates the small-state scan kernels for nx = 3, float storage.
#include "scan_small_impl.hpp"

namespace pks {
template hipError_t small_run<3, float>(ScanArgs, int, hipStream_t);
}
