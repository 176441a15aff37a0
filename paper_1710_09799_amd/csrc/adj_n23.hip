// adj_n23.hip -- instantiations of the four-lanes-per-cell adjoint kernel
// (N = 2 and 3).
#include "adj_quad.hpp"

namespace mln {

template <typename Real>
hipError_t launch_adj_quad(int N, const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  if (W < 16 || W > kMaxAdjQuadTile || W % 16) return hipErrorInvalidValue;
  constexpr bool f64 = sizeof(Real) == 8;
  switch (N) {
    case 2: hipLaunchKernelGGL((adj_quad_kernel<2, Real>), dim3((unsigned)nblocks), dim3(4 * W), 0, st, a); break;
    case 3:
      if (f64 && W <= 64)
        hipLaunchKernelGGL((adj_quad_kernel<3, Real, 256>), dim3((unsigned)nblocks), dim3(4 * W), 0, st, a);
      else
        hipLaunchKernelGGL((adj_quad_kernel<3, Real>), dim3((unsigned)nblocks), dim3(4 * W), 0, st, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_adj_quad<double>(int, const AdjArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_adj_quad<float>(int, const AdjArgs<float> &, int64_t, int, hipStream_t);

}  // namespace mln
