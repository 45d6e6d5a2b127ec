// Instantiations of the fused 2D front and first sweep pass: 3 sweeps.
#include "k2fs_impl.h"

namespace mx {
namespace fused2d {
template hipError_t fs_dispatch_k<3>(const Coef<float> &, int, const FrontArgs<float> &, const float *const[3],
                                     const SweepArgs<float> &, hipStream_t, int *);
}  // namespace fused2d
}  // namespace mx
