// fwd_n3.hip -- instantiations of the forward kernels for N = 3 levels.
#include <type_traits>

#include "fwd_quad.hpp"
#include "fwd_wave.hpp"

namespace mln {

template <typename Real>
hipError_t launch_fwd_n3(int route, bool comp, bool cf, const FwdArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  if (cf && !comp) {
    // plain single-precision state, float-float fields
    if constexpr (std::is_same<Real, float>::value) {
      if (route != ROUTE_ROT) return hipErrorInvalidValue;
      if (many_tiles(nblocks))
        hipLaunchKernelGGL((fwd_tile_kernel_many<3, float, false, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      else
        hipLaunchKernelGGL((fwd_tile_kernel<3, float, ROUTE_ROT, false, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (comp) {
    if constexpr (std::is_same<Real, float>::value) {
      if (route != ROUTE_ROT) return hipErrorInvalidValue;
      const bool many = many_tiles(nblocks);
      if (cf && many)
        hipLaunchKernelGGL((fwd_tile_kernel_many<3, float, true, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      else if (cf)
        hipLaunchKernelGGL((fwd_tile_kernel<3, float, ROUTE_ROT, true, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      else if (many)
        hipLaunchKernelGGL((fwd_tile_kernel_many<3, float, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      else
        hipLaunchKernelGGL((fwd_tile_kernel<3, float, ROUTE_ROT, true>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  switch (route) {
    case ROUTE_ROT:
      if (many_tiles(nblocks))
        hipLaunchKernelGGL((fwd_tile_kernel_many<3, Real, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      else
        hipLaunchKernelGGL((fwd_tile_kernel<3, Real, ROUTE_ROT, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
      break;
    case ROUTE_DIAG: hipLaunchKernelGGL((fwd_tile_kernel<3, Real, ROUTE_DIAG, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    case ROUTE_RODR: hipLaunchKernelGGL((fwd_tile_kernel<3, Real, ROUTE_RODR, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    case ROUTE_PADE: hipLaunchKernelGGL((fwd_tile_kernel<3, Real, ROUTE_PADE, false>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_fwd_wave_n3(bool comp, int C, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st) {
  switch (C) {
    case 1:
      if (comp) {
        if constexpr (std::is_same<Real, float>::value)
          hipLaunchKernelGGL((fwd_wave_kernel<3, float, true, 1>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
        else
          return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((fwd_wave_kernel<3, Real, false, 1>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
      }
      break;
    case 2:
      if (comp) {
        if constexpr (std::is_same<Real, float>::value)
          hipLaunchKernelGGL((fwd_wave_kernel<3, float, true, 2>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
        else
          return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((fwd_wave_kernel<3, Real, false, 2>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
      }
      break;
    case 4:
      if (comp) {
        if constexpr (std::is_same<Real, float>::value)
          hipLaunchKernelGGL((fwd_wave_kernel<3, float, true, 4>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
        else
          return hipErrorInvalidValue;
      } else {
        hipLaunchKernelGGL((fwd_wave_kernel<3, Real, false, 4>), dim3((unsigned)nblocks), dim3(64), 0, st, a);
      }
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_fwd_quad_n3(bool comp, bool cf, bool mf, int W, const FwdArgs<Real> &a, int64_t nblocks,
                              hipStream_t st) {
  if (cf && !comp) {
    if constexpr (std::is_same<Real, float>::value) return launch_quad<3, float, false, true>(W, a, nblocks, st, mf);
    return hipErrorInvalidValue;
  }
  if (comp) {
    if constexpr (std::is_same<Real, float>::value) {
      if (cf) return launch_quad<3, float, true, true>(W, a, nblocks, st, mf);
      return launch_quad<3, float, true, false>(W, a, nblocks, st, mf);
    }
    return hipErrorInvalidValue;
  }
  return launch_quad<3, Real, false, false>(W, a, nblocks, st, mf);
}

template <typename Real>
hipError_t launch_bloch_n3(int route, bool comp, const BlochArgs<Real> &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.ncell + 255) / 256);
  if (comp) {
    if constexpr (std::is_same<Real, float>::value) {
      if (route != ROUTE_ROT) return hipErrorInvalidValue;
      hipLaunchKernelGGL((bloch_kernel<3, float, ROUTE_ROT, true>), dim3(nb), dim3(256), 0, st, a);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  switch (route) {
    case ROUTE_ROT: hipLaunchKernelGGL((bloch_kernel<3, Real, ROUTE_ROT, false>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_DIAG: hipLaunchKernelGGL((bloch_kernel<3, Real, ROUTE_DIAG, false>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_RODR: hipLaunchKernelGGL((bloch_kernel<3, Real, ROUTE_RODR, false>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_PADE: hipLaunchKernelGGL((bloch_kernel<3, Real, ROUTE_PADE, false>), dim3(nb), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_adj_n3(const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  hipLaunchKernelGGL((adj_tile_kernel<3, Real>), dim3((unsigned)nblocks), dim3(W), 0, st, a);
  return hipGetLastError();
}

template hipError_t launch_adj_n3<double>(const AdjArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_adj_n3<float>(const AdjArgs<float> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd_n3<double>(int, bool, bool, const FwdArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd_n3<float>(int, bool, bool, const FwdArgs<float> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd_wave_n3<double>(bool, int, const FwdArgs<double> &, int64_t, hipStream_t);
template hipError_t launch_fwd_wave_n3<float>(bool, int, const FwdArgs<float> &, int64_t, hipStream_t);
template hipError_t launch_fwd_quad_n3<double>(bool, bool, bool, int, const FwdArgs<double> &, int64_t, hipStream_t);
template hipError_t launch_fwd_quad_n3<float>(bool, bool, bool, int, const FwdArgs<float> &, int64_t, hipStream_t);
template hipError_t launch_bloch_n3<double>(int, bool, const BlochArgs<double> &, hipStream_t);
template hipError_t launch_bloch_n3<float>(int, bool, const BlochArgs<float> &, hipStream_t);

}  // namespace mln
