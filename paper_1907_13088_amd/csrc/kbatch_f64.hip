// Batched 2D stepping: launchers and kernels for double (kernels in kbatch_impl.h).
#include "kbatch_impl.h"

namespace mx {
namespace batch2d {

template <>
hipError_t launch_front<double>(const GridDesc<double> *d, int ng, const int *items, int nitems, int L, int bin,
                              hipStream_t s)
{
    return launch_front_impl<double>(d, ng, items, nitems, L, bin, s);
}

template <>
hipError_t launch_front_sweep<double>(const GridDesc<double> *d, int ng, const int *items, int nitems, int L, int k,
                                    int bin, hipStream_t s)
{
    return launch_front_sweep_impl<double>(d, ng, items, nitems, L, k, bin, s);
}

template <>
hipError_t launch_sweep<double>(const GridDesc<double> *d, int ng, const int *items, int nitems, int L, int k,
                              bool first, bool last, int xin, int xout, hipStream_t s)
{
    return launch_sweep_impl<double>(d, ng, items, nitems, L, k, first, last, xin, xout, s);
}

template <>
int persistent_blocks<double>(int q)
{
    return persistent_blocks_disp<double, KMAX>(q);
}

template <>
hipError_t launch_persistent<double>(const GridDesc<double> *d, int ng, const int *items_f, const int *items_s, int Lf, int Ls,
                            int nsteps, int q, int npass, int nlow, int bin0, unsigned *cnt, int ndone, int *err,
                            int fuse, hipStream_t s)
{
    return persist_disp<double, KMAX>(d, ng, items_f, items_s, Lf, Ls, nsteps, q, npass, nlow, bin0, cnt, ndone, err, fuse,
                                 s);
}

}  // namespace batch2d
}  // namespace mx
