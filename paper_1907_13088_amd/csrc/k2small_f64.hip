// The single-launch small-grid tolerance solve in double (k2small_impl.h).
#include "k2small_impl.h"

namespace mx {
template void small_tiles<double>(int, int, int *, int *);
template int small_capacity<double>(bool, int);
template hipError_t launch_small<double>(const SmallArgs<double> &, bool, hipStream_t);
}  // namespace mx
