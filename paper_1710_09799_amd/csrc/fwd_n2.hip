// fwd_n2.hip -- instantiations of the forward kernels for N = 2 levels.
#include "fwd_impl.hpp"

namespace mln {

template <typename Real>
hipError_t launch_fwd_n2(int route, const FwdArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  switch (route) {
    case ROUTE_ROT: hipLaunchKernelGGL((fwd_tile_kernel<2, Real, ROUTE_ROT>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    case ROUTE_DIAG: hipLaunchKernelGGL((fwd_tile_kernel<2, Real, ROUTE_DIAG>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    case ROUTE_RODR: hipLaunchKernelGGL((fwd_tile_kernel<2, Real, ROUTE_RODR>), dim3((unsigned)nblocks), dim3(W), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_bloch_n2(int route, const BlochArgs<Real> &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.ncell + 255) / 256);
  switch (route) {
    case ROUTE_ROT: hipLaunchKernelGGL((bloch_kernel<2, Real, ROUTE_ROT>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_DIAG: hipLaunchKernelGGL((bloch_kernel<2, Real, ROUTE_DIAG>), dim3(nb), dim3(256), 0, st, a); break;
    case ROUTE_RODR: hipLaunchKernelGGL((bloch_kernel<2, Real, ROUTE_RODR>), dim3(nb), dim3(256), 0, st, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_fwd_n2<double>(int, const FwdArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd_n2<float>(int, const FwdArgs<float> &, int64_t, int, hipStream_t);
template hipError_t launch_bloch_n2<double>(int, const BlochArgs<double> &, hipStream_t);
template hipError_t launch_bloch_n2<float>(int, const BlochArgs<float> &, hipStream_t);

}  // namespace mln
