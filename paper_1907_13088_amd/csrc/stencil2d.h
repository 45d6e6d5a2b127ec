// Point formulas of the 2D mass-matrix operator A (eqs matrixA_1st_2d ..
// matrixA_last_2d) with an explicit fused-multiply-add structure.  Every 2D
// sweep kernel evaluates A through these helpers and the library is built
// without automatic contraction, so the tile and the streaming schedules
// produce bitwise identical iterates.
#pragma once

#include <hip/hip_runtime.h>

namespace mx {

template <typename T>
__device__ __forceinline__ T fmad(T a, T b, T c) { return fma(a, b, c); }

// second difference f+ + f- - 2 f0
template <typename T>
__device__ __forceinline__ T d2(T fm, T f0, T fp) { return fmad(T(-2), f0, fp + fm); }

// (A x)_x = cxx Dyy Ex + cxy DxDy Ey:  lyy = Dyy Ex,  dg = DxDy Ey
template <typename T>
__device__ __forceinline__ T a_te_x(T cxx, T cxy, T lyy, T dg) { return fmad(cxx, lyy, cxy * dg); }

// (A x)_y = cyy Dxx Ey + cxy DxDy Ex:  lxx = Dxx Ey,  dh = DxDy Ex
template <typename T>
__device__ __forceinline__ T a_te_y(T cyy, T cxy, T lxx, T dh) { return fmad(cyy, lxx, cxy * dh); }

// (A x)_z = czx Dxx Ez + czy Dyy Ez + czz DxxDyy Ez
template <typename T>
__device__ __forceinline__ T a_tm(T czx, T czy, T czz, T lx, T ly, T lxy)
{
    return fmad(czz, lxy, fmad(czy, ly, czx * lx));
}

// b + (A x) with b as the innermost addend of the FMA chain (standard form)
template <typename T>
__device__ __forceinline__ T a_te_x_b(T cxx, T cxy, T lyy, T dg, T b) { return fmad(cxx, lyy, fmad(cxy, dg, b)); }

template <typename T>
__device__ __forceinline__ T a_te_y_b(T cyy, T cxy, T lxx, T dh, T b) { return fmad(cyy, lxx, fmad(cxy, dh, b)); }

template <typename T>
__device__ __forceinline__ T a_tm_b(T czx, T czy, T czz, T lx, T ly, T lxy, T b)
{
    return fmad(czz, lxy, fmad(czy, ly, fmad(czx, lx, b)));
}

}  // namespace mx
