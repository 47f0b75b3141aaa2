// Instantiates the small-state scan kernels for nx = 2, double storage.
#include "scan_small_impl.hpp"

namespace pks {
template hipError_t small_run<2, double>(ScanArgs, int, hipStream_t);
}
