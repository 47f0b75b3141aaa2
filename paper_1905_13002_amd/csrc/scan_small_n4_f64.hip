// Instantiates the small-state scan kernels for nx = 4, double storage.
#include "scan_small_impl.hpp"

namespace pks {
template hipError_t small_run<4, double>(ScanArgs, int, hipStream_t);
}
