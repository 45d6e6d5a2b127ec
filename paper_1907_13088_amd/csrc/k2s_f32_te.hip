// Instantiations of the streaming 2D sweep pass: float, standard form, TE block.
#include "k2s_impl.h"

namespace mx {
namespace stream2d {
template hipError_t launch<float, FM_STD, 1>(const Coef<float> &, int, int, const SweepArgs<float> &, hipStream_t,
                                           int *, int);
}  // namespace stream2d
}  // namespace mx
