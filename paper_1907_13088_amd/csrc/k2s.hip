// Streaming 2D sweep pass: dispatch on element type, iterate form and block
// set (the kernels are instantiated in k2s_{f32,f64}{,d,c}_{te,tm,all}.hip:
// standard, delta and Chebyshev forms).
#include "mx_internal.h"

namespace mx {
namespace stream2d {
template <typename T, int FORM, int BLK>
hipError_t launch(const Coef<T> &c, int k, int flags, const SweepArgs<T> &a, hipStream_t s, int *nwg, int slots);
#define MX_STREAM_EXTERN(T, F, B)                                                                        \
    extern template hipError_t launch<T, F, B>(const Coef<T> &, int, int, const SweepArgs<T> &, hipStream_t, \
                                               int *, int);
#define MX_STREAM_EXTERN_FORMS(T, F) MX_STREAM_EXTERN(T, F, 1) MX_STREAM_EXTERN(T, F, 2) MX_STREAM_EXTERN(T, F, 3)
MX_STREAM_EXTERN_FORMS(float, FM_STD)
MX_STREAM_EXTERN_FORMS(float, FM_DELTA)
MX_STREAM_EXTERN_FORMS(float, FM_CHEB)
MX_STREAM_EXTERN_FORMS(double, FM_STD)
MX_STREAM_EXTERN_FORMS(double, FM_DELTA)
MX_STREAM_EXTERN_FORMS(double, FM_CHEB)
#undef MX_STREAM_EXTERN_FORMS
#undef MX_STREAM_EXTERN

template <typename T, int FORM>
hipError_t launch_form(const Coef<T> &c, int block, int k, int flags, const SweepArgs<T> &a, hipStream_t s,
                       int *nwg, int slots)
{
    if (block == 1) return launch<T, FORM, 1>(c, k, flags, a, s, nwg, slots);
    if (block == 2) return launch<T, FORM, 2>(c, k, flags, a, s, nwg, slots);
    if (block == 3) return launch<T, FORM, 3>(c, k, flags, a, s, nwg, slots);
    return hipErrorInvalidValue;
}
}  // namespace stream2d

int stream2d_kmax(bool f64, int block, int form)
{
    // must agree with stream2d::stream_kmax
    if (form == FM_CHEB) return !f64 ? (block == 1 ? 10 : block == 2 ? 16 : 6) : (block == 1 ? 4 : block == 2 ? 8 : 2);
    if (form == FM_DELTA) return !f64 ? (block == 1 ? 12 : block == 2 ? 16 : 8) : (block == 1 ? 6 : block == 2 ? 10 : 3);
    return !f64 ? (block == 1 ? 14 : block == 2 ? 16 : 9) : (block == 1 ? 7 : block == 2 ? 12 : 4);
}

template <typename T>
hipError_t launch_stream2d(const Coef<T> &c, int block, int k, int form, int flags, const SweepArgs<T> &a,
                           hipStream_t s, int *nwg, int slots)
{
    if (form == FM_STD) return stream2d::launch_form<T, FM_STD>(c, block, k, flags, a, s, nwg, slots);
    if (form == FM_DELTA) return stream2d::launch_form<T, FM_DELTA>(c, block, k, flags, a, s, nwg, slots);
    if (form == FM_CHEB) return stream2d::launch_form<T, FM_CHEB>(c, block, k, flags, a, s, nwg, slots);
    return hipErrorInvalidValue;
}

template hipError_t launch_stream2d<float>(const Coef<float> &, int, int, int, int, const SweepArgs<float> &,
                                           hipStream_t, int *, int);
template hipError_t launch_stream2d<double>(const Coef<double> &, int, int, int, int,
                                            const SweepArgs<double> &, hipStream_t, int *, int);

}  // namespace mx
