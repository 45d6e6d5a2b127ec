// The single-launch small-grid tolerance solve in float (k2small_impl.h).
#include "k2small_impl.h"

namespace mx {
template void small_tiles<float>(int, int, int *, int *);
template int small_capacity<float>(bool, int);
template hipError_t launch_small<float>(const SmallArgs<float> &, bool, hipStream_t);
}  // namespace mx
