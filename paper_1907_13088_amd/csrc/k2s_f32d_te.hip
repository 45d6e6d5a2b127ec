// Instantiations of the streaming 2D sweep pass: float, delta form, TE block.
#include "k2s_impl.h"

namespace mx {
namespace stream2d {
template hipError_t launch<float, FM_DELTA, 1>(const Coef<float> &, int, int, const SweepArgs<float> &, hipStream_t,
                                           int *, int);
}  // namespace stream2d
}  // namespace mx
