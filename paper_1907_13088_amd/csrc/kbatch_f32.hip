// Batched 2D stepping: launchers and instantiations for float.
#include "kbatch_impl.h"

namespace mx {
namespace batch2d {

template <>
hipError_t launch_front<float>(const GridDesc<float> *d, int ng, const int *items, int nitems, int L, int bin,
                             hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL((kb_front<float>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L, bin);
    return hipGetLastError();
}

template <int K>
static hipError_t sweep_k(const GridDesc<float> *d, int ng, const int *items, int nitems, int L, bool first, bool last,
                          int xin, int xout, hipStream_t s)
{
    if (last)
        hipLaunchKernelGGL((kb_sweep<float, K, stream2d::OM_LAST>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L,
                           (int)first, xin, xout);
    else
        hipLaunchKernelGGL((kb_sweep<float, K, stream2d::OM_STORE>), dim3(nitems), dim3(RX), 0, s, d, ng, items, L,
                           (int)first, xin, xout);
    return hipGetLastError();
}

template <>
hipError_t launch_sweep<float>(const GridDesc<float> *d, int ng, const int *items, int nitems, int L, int k, bool first,
                             bool last, int xin, int xout, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    switch (k) {
    case 1: return sweep_k<1>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 2: return sweep_k<2>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 3: return sweep_k<3>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 4: return sweep_k<4>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 5: return sweep_k<5>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 6: return sweep_k<6>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 7: return sweep_k<7>(d, ng, items, nitems, L, first, last, xin, xout, s);
    case 8: return sweep_k<8>(d, ng, items, nitems, L, first, last, xin, xout, s);
    default: return hipErrorInvalidValue;
    }
}

template <int Q>
static int occ_q()
{
    static int n = -1;
    if (n < 0) {
        int o = 0, dev = 0, cu = 0;
        (void)hipGetDevice(&dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kb_persistent<float, Q>, RX, 0) != hipSuccess) o = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cu = 0;
        n = o * cu;
    }
    return n;
}

template <>
int persistent_blocks<float>(int q)
{
    switch (q) {
    case 1: return occ_q<1>();
    case 2: return occ_q<2>();
    case 3: return occ_q<3>();
    case 4: return occ_q<4>();
    case 5: return occ_q<5>();
    case 6: return occ_q<6>();
    default: return 0;
    }
}

template <int Q>
static hipError_t persist_q(const GridDesc<float> *d, int ng, const int *items_f, const int *items_s, int Lf, int Ls,
                            int nsteps, int npass, int bin0, unsigned *bar, int *err, int nblocks, hipStream_t s)
{
    void *args[] = {(void *)&d, (void *)&ng, (void *)&items_f, (void *)&items_s, (void *)&Lf, (void *)&Ls,
                     (void *)&nsteps, (void *)&npass, (void *)&bin0, (void *)&bar, (void *)&err};
    return hipLaunchCooperativeKernel((const void *)kb_persistent<float, Q>, dim3(nblocks), dim3(RX), args, 0, s);
}

template <>
hipError_t launch_persistent<float>(const GridDesc<float> *d, int ng, const int *items_f, const int *items_s, int Lf,
                                  int Ls, int nsteps, int q, int npass, int bin0, unsigned *bar, int *err,
                                  int nblocks, hipStream_t s)
{
    switch (q) {
    case 1: return persist_q<1>(d, ng, items_f, items_s, Lf, Ls, nsteps, npass, bin0, bar, err, nblocks, s);
    case 2: return persist_q<2>(d, ng, items_f, items_s, Lf, Ls, nsteps, npass, bin0, bar, err, nblocks, s);
    case 3: return persist_q<3>(d, ng, items_f, items_s, Lf, Ls, nsteps, npass, bin0, bar, err, nblocks, s);
    case 4: return persist_q<4>(d, ng, items_f, items_s, Lf, Ls, nsteps, npass, bin0, bar, err, nblocks, s);
    case 5: return persist_q<5>(d, ng, items_f, items_s, Lf, Ls, nsteps, npass, bin0, bar, err, nblocks, s);
    case 6: return persist_q<6>(d, ng, items_f, items_s, Lf, Ls, nsteps, npass, bin0, bar, err, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace batch2d
}  // namespace mx
