// Fused 2D front and first sweep pass: launch dispatch (kernel in
// k2fs_impl.h, instantiated per sweep count in k2fs_k{3,4,5,6}.hip).
#include "mx_internal.h"

namespace mx {
namespace fused2d {
template <int K>
hipError_t fs_dispatch_k(const Coef<float> &c, int p, const FrontArgs<float> &fa, const float *const Bin[3],
                         const SweepArgs<float> &sa, hipStream_t s, int *nwg);
#define MX_FS_EXTERN(K)                                                                                         \
    extern template hipError_t fs_dispatch_k<K>(const Coef<float> &, int, const FrontArgs<float> &,             \
                                                const float *const[3], const SweepArgs<float> &, hipStream_t,   \
                                                int *);
MX_FS_EXTERN(3)
MX_FS_EXTERN(4)
MX_FS_EXTERN(5)
MX_FS_EXTERN(6)
#undef MX_FS_EXTERN
}  // namespace fused2d

bool front_sweep2d_ok(bool f64, int k, int p) { return !f64 && k >= 3 && k <= 6 && p >= 0 && p <= 4; }

template <>
hipError_t launch_front_sweep2d<float>(const Coef<float> &c, int p, int k, const FrontArgs<float> &fa,
                                       const float *const Bin[3], const SweepArgs<float> &sa, hipStream_t s,
                                       int *nwg)
{
    switch (k) {
    case 3: return fused2d::fs_dispatch_k<3>(c, p, fa, Bin, sa, s, nwg);
    case 4: return fused2d::fs_dispatch_k<4>(c, p, fa, Bin, sa, s, nwg);
    case 5: return fused2d::fs_dispatch_k<5>(c, p, fa, Bin, sa, s, nwg);
    case 6: return fused2d::fs_dispatch_k<6>(c, p, fa, Bin, sa, s, nwg);
    default: return hipErrorInvalidValue;
    }
}

// FP64: no fused kernel (front_sweep2d_ok is false)
template <>
hipError_t launch_front_sweep2d<double>(const Coef<double> &, int, int, const FrontArgs<double> &,
                                        const double *const[3], const SweepArgs<double> &, hipStream_t, int *)
{
    return hipErrorInvalidValue;
}

}  // namespace mx
