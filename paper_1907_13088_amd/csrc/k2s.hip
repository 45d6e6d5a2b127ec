// Streaming 2D sweep pass: dispatch on element type, iterate form and block
// set (the kernels are instantiated in k2s_{f32,f64}[d]_{te,tm,all}.hip).
#include "mx_internal.h"

namespace mx {
namespace stream2d {
template <typename T, bool DELTA, int BLK>
hipError_t launch(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots);
#define MX_STREAM_EXTERN(T, D, B)                                                                        \
    extern template hipError_t launch<T, D, B>(const Coef<T> &, int, int, const SweepArgs<T> &, hipStream_t, \
                                               int *, int);
MX_STREAM_EXTERN(float, false, 1)
MX_STREAM_EXTERN(float, false, 2)
MX_STREAM_EXTERN(float, false, 3)
MX_STREAM_EXTERN(float, true, 1)
MX_STREAM_EXTERN(float, true, 2)
MX_STREAM_EXTERN(float, true, 3)
MX_STREAM_EXTERN(double, false, 1)
MX_STREAM_EXTERN(double, false, 2)
MX_STREAM_EXTERN(double, false, 3)
MX_STREAM_EXTERN(double, true, 1)
MX_STREAM_EXTERN(double, true, 2)
MX_STREAM_EXTERN(double, true, 3)
#undef MX_STREAM_EXTERN
}  // namespace stream2d

int stream2d_kmax(bool f64, int block, bool delta)
{
    // must agree with stream2d::stream_kmax
    if (!f64) return block == 1 ? (delta ? 9 : 10) : block == 2 ? 16 : (delta ? 6 : 7);
    return block == 1 ? (delta ? 4 : 5) : block == 2 ? 8 : 3;
}

template <typename T>
hipError_t launch_stream2d(const Coef<T> &c, int block, int k, bool delta, int flags, const SweepArgs<T> &a,
                           hipStream_t s, int *nwg, int slots)
{
    if (block == 1)
        return delta ? stream2d::launch<T, true, 1>(c, k, flags, a, s, nwg, slots)
                     : stream2d::launch<T, false, 1>(c, k, flags, a, s, nwg, slots);
    if (block == 2)
        return delta ? stream2d::launch<T, true, 2>(c, k, flags, a, s, nwg, slots)
                     : stream2d::launch<T, false, 2>(c, k, flags, a, s, nwg, slots);
    if (block == 3)
        return delta ? stream2d::launch<T, true, 3>(c, k, flags, a, s, nwg, slots)
                     : stream2d::launch<T, false, 3>(c, k, flags, a, s, nwg, slots);
    return hipErrorInvalidValue;
}

template hipError_t launch_stream2d<float>(const Coef<float> &, int, int, bool, int, const SweepArgs<float> &,
                                           hipStream_t, int *, int);
template hipError_t launch_stream2d<double>(const Coef<double> &, int, int, bool, int,
                                            const SweepArgs<double> &, hipStream_t, int *, int);

}  // namespace mx
