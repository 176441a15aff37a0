// fwd_n6.hip -- instantiations of the forward kernels for N = 6 levels.
#include <type_traits>

#include "fwd_mfma.hpp"
#include "fwd_wave.hpp"

namespace mln {

template <typename Real>
hipError_t launch_fwd_n6(int route, bool comp, bool cf, const FwdArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  if (cf && !comp) return hipErrorInvalidValue;
  if (comp) {
    if constexpr (std::is_same<Real, float>::value) {
      if (route != ROUTE_ROT) return hipErrorInvalidValue;
      if (cf)
        hipLaunchKernelGGL((fwd_tile_kernel<6, float, ROUTE_ROT, true, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      else
        hipLaunchKernelGGL((fwd_tile_kernel<6, float, ROUTE_ROT, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  switch (route) {
    case ROUTE_ROT: hipLaunchKernelGGL((fwd_tile_kernel<6, Real, ROUTE_ROT, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    case ROUTE_DIAG: hipLaunchKernelGGL((fwd_tile_kernel<6, Real, ROUTE_DIAG, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    case ROUTE_RODR: hipLaunchKernelGGL((fwd_tile_kernel<6, Real, ROUTE_RODR, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_fwd_wave_n6(bool comp, int C, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st) {
  switch (C) {
    case 1:
      if (comp) {
        if constexpr (std::is_same<Real, float>::value)
          hipLaunchKernelGGL((fwd_wave_kernel<6, float, true, 1>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
        else
          return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((fwd_wave_kernel<6, Real, false, 1>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
      }
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fwd_mfma_n6(int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st) {
  constexpr int D = 6 * 6 - 1;
  if (nprod == 6) {
    const size_t lds = mfma_lds_bytes<D, 6>(W);
    hipError_t e = hipFuncSetAttribute((const void *)fwd_mfma_kernel<6, 6>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_mfma_kernel<6, 6>), dim3((unsigned)nblocks), dim3(W), lds, st, a);
  } else if (nprod == 3) {
    const size_t lds = mfma_lds_bytes<D, 3>(W);
    hipError_t e = hipFuncSetAttribute((const void *)fwd_mfma_kernel<6, 3>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_mfma_kernel<6, 3>), dim3((unsigned)nblocks), dim3(W), lds, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_bloch_n6(int route, bool comp, const BlochArgs<Real> &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.ncell + 255) / 256);
  if (comp) {
    if constexpr (std::is_same<Real, float>::value) {
      if (route != ROUTE_ROT) return hipErrorInvalidValue;
      hipLaunchKernelGGL((bloch_kernel<6, float, ROUTE_ROT, true>), dim3(nb), dim3(256), 0, st, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  switch (route) {
    case ROUTE_ROT: hipLaunchKernelGGL((bloch_kernel<6, Real, ROUTE_ROT, false>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_DIAG: hipLaunchKernelGGL((bloch_kernel<6, Real, ROUTE_DIAG, false>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_RODR: hipLaunchKernelGGL((bloch_kernel<6, Real, ROUTE_RODR, false>), dim3(nb), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_fwd_n6<double>(int, bool, bool, const FwdArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd_n6<float>(int, bool, bool, const FwdArgs<float> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd_wave_n6<double>(bool, int, const FwdArgs<double> &, int64_t, hipStream_t);
template hipError_t launch_fwd_wave_n6<float>(bool, int, const FwdArgs<float> &, int64_t, hipStream_t);
template hipError_t launch_bloch_n6<double>(int, bool, const BlochArgs<double> &, hipStream_t);
template hipError_t launch_bloch_n6<float>(int, bool, const BlochArgs<float> &, hipStream_t);

}  // namespace mln
