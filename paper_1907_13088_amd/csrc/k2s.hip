// Streaming 2D sweep pass: dispatch on element type and iterate form (the
// kernels are instantiated in k2s_f32*.hip and k2s_f64*.hip).
#include "mx_internal.h"

namespace mx {
namespace stream2d {
template <typename T, bool DELTA>
hipError_t launch(const Coef<T> &c, int blocks, int k, int flags, const SweepArgs<T> &a, hipStream_t s,
                  int *nwg, int slots);
extern template hipError_t launch<float, false>(const Coef<float> &, int, int, int, const SweepArgs<float> &,
                                                hipStream_t, int *, int);
extern template hipError_t launch<float, true>(const Coef<float> &, int, int, int, const SweepArgs<float> &,
                                               hipStream_t, int *, int);
extern template hipError_t launch<double, false>(const Coef<double> &, int, int, int,
                                                 const SweepArgs<double> &, hipStream_t, int *, int);
extern template hipError_t launch<double, true>(const Coef<double> &, int, int, int,
                                                const SweepArgs<double> &, hipStream_t, int *, int);
}  // namespace stream2d

template <typename T>
hipError_t launch_stream2d(const Coef<T> &c, int blocks, int k, bool delta, int flags, const SweepArgs<T> &a,
                           hipStream_t s, int *nwg, int slots)
{
    return delta ? stream2d::launch<T, true>(c, blocks, k, flags, a, s, nwg, slots)
                 : stream2d::launch<T, false>(c, blocks, k, flags, a, s, nwg, slots);
}

template hipError_t launch_stream2d<float>(const Coef<float> &, int, int, bool, int, const SweepArgs<float> &,
                                           hipStream_t, int *, int);
template hipError_t launch_stream2d<double>(const Coef<double> &, int, int, bool, int,
                                            const SweepArgs<double> &, hipStream_t, int *, int);

}  // namespace mx
