// Instantiations of the streaming 2D sweep pass for float, delta form.
#include "k2s_impl.h"

namespace mx {
namespace stream2d {
template hipError_t launch<float, true>(const Coef<float> &, int, int, int,
                                                 const SweepArgs<float> &, hipStream_t, int *, int);
}  // namespace stream2d
}  // namespace mx
