// Streaming 2D front pass: launch configuration (kernel in k2f_impl.h).
#include "k2f_impl.h"

namespace mx {
namespace {
using namespace front2d;

constexpr int FRX = 512;   // threads (columns) per workgroup strip

template <typename T, int BLK, int P, bool HASJ>
hipError_t front_j(const Coef<T> &c, const FrontArgs<T> &a, const T *const Bin[3], hipStream_t s, int *nwg)
{
    constexpr int W = front_aligned() ? FRX - 32 : FRX - (P > 1 ? P : 1) - (P > 2 ? P : 2);
    static std::atomic<int> resident[MX_MAX_DEVICES];
    const int slots = per_device(resident, [] {
        int o = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k2_front_stream<T, BLK, P, FRX, HASJ>, FRX, 0) != hipSuccess || o < 1) o = 1;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1) cu = 256;
        return std::min(o, 4) * cu;
    });
    const int nsx = (c.nx + W - 1) / W;
    int nsy = std::max(1, slots / nsx);
    nsy = std::min(nsy, c.ny);
    int L = (c.ny + nsy - 1) / nsy;
    L = std::max(L, std::min(c.ny, 16));
    nsy = (c.ny + L - 1) / L;
    const int n = nsx * nsy;
    *nwg = n;
    hipLaunchKernelGGL((k2_front_stream<T, BLK, P, FRX, HASJ>), dim3(n), dim3(FRX), 0, s, c, a, Bin[0], Bin[1], Bin[2],
                       L, nsx, n);
    return hipGetLastError();
}

template <typename T, int BLK, int P>
hipError_t front_p(const Coef<T> &c, const FrontArgs<T> &a, const T *const Bin[3], hipStream_t s, int *nwg)
{
    if (a.J0[0] != nullptr) return front_j<T, BLK, P, true>(c, a, Bin, s, nwg);
    return front_j<T, BLK, P, false>(c, a, Bin, s, nwg);
}

template <typename T, int BLK>
hipError_t front_b(const Coef<T> &c, int p, const FrontArgs<T> &a, const T *const Bin[3], hipStream_t s, int *nwg)
{
    switch (p) {
    case 0: return front_p<T, BLK, 0>(c, a, Bin, s, nwg);
    case 1: return front_p<T, BLK, 1>(c, a, Bin, s, nwg);
    case 2: return front_p<T, BLK, 2>(c, a, Bin, s, nwg);
    case 3: return front_p<T, BLK, 3>(c, a, Bin, s, nwg);
    case 4: return front_p<T, BLK, 4>(c, a, Bin, s, nwg);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename T>
hipError_t launch_front_stream2d(const Coef<T> &c, int blocks, int filter_passes, const FrontArgs<T> &a,
                                 const T *const Bin[3], hipStream_t s, int *nwg)
{
    switch (blocks) {
    case 1: return front_b<T, 1>(c, filter_passes, a, Bin, s, nwg);
    case 2: return front_b<T, 2>(c, filter_passes, a, Bin, s, nwg);
    case 3: return front_b<T, 3>(c, filter_passes, a, Bin, s, nwg);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_front_stream2d<float>(const Coef<float> &, int, int, const FrontArgs<float> &,
                                                 const float *const[3], hipStream_t, int *);
template hipError_t launch_front_stream2d<double>(const Coef<double> &, int, int, const FrontArgs<double> &,
                                                  const double *const[3], hipStream_t, int *);

}  // namespace mx
