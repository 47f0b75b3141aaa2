// Instantiates the small-state scan kernels for nx = 3, double storage.
#include "scan_small_impl.hpp"

namespace pks {
template hipError_t small_run<3, double>(ScanArgs, int, hipStream_t);
}
