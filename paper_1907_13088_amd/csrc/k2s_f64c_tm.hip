// Instantiations of the streaming 2D sweep pass: double, Chebyshev form, TM block.
#include "k2s_impl.h"

namespace mx {
namespace stream2d {
template hipError_t launch<double, FM_CHEB, 2>(const Coef<double> &, int, int, const SweepArgs<double> &, hipStream_t,
                                           int *, int);
}  // namespace stream2d
}  // namespace mx
