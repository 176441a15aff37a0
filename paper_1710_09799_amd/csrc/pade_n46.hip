// pade_n46.hip -- instantiations of the per-step Pade route for N = 4 and 6
// (one wavefront per cell, fwd_pade.hpp).
#include "fwd_pade.hpp"

namespace mln {

size_t pade_lds_bytes(int N, int real_bytes, int W) {
  if (N == 4) return real_bytes == 8 ? PadeLds<4, double>::bytes(W) : PadeLds<4, float>::bytes(W);
  if (N == 6) return real_bytes == 8 ? PadeLds<6, double>::bytes(W) : PadeLds<6, float>::bytes(W);
  return 0;
}

namespace {
template <int N, typename Real>
hipError_t fwd_pade_n(const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st) {
  const int W = a.owned + 2 * a.halo;
  if (W > kPadeThreads) return hipErrorInvalidValue;
  const size_t lds = PadeLds<N, Real>::bytes(W);
  if (lds > kPadeMaxLds) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void *)fwd_pade_kernel<N, Real>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fwd_pade_kernel<N, Real>), dim3((unsigned)nblocks), dim3(kPadeThreads), lds, st, a);
  return hipGetLastError();
}

template <int N, typename Real>
hipError_t bloch_pade_n(const BlochArgs<Real> &a, hipStream_t st) {
  const size_t lds = PadeLds<N, Real>::bloch_bytes();
  hipError_t e = hipFuncSetAttribute((const void *)bloch_pade_kernel<N, Real>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)((a.ncell + kPadeWaves - 1) / kPadeWaves);
  hipLaunchKernelGGL((bloch_pade_kernel<N, Real>), dim3(nb), dim3(kPadeThreads), lds, st, a);
  return hipGetLastError();
}
}  // namespace

template <typename Real>
hipError_t launch_fwd_pade(int N, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st) {
  switch (N) {
    case 4: return fwd_pade_n<4, Real>(a, nblocks, st);
    case 6: return fwd_pade_n<6, Real>(a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_bloch_pade(int N, const BlochArgs<Real> &a, hipStream_t st) {
  switch (N) {
    case 4: return bloch_pade_n<4, Real>(a, st);
    case 6: return bloch_pade_n<6, Real>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fwd_pade<double>(int, const FwdArgs<double> &, int64_t, hipStream_t);
template hipError_t launch_fwd_pade<float>(int, const FwdArgs<float> &, int64_t, hipStream_t);
template hipError_t launch_bloch_pade<double>(int, const BlochArgs<double> &, hipStream_t);
template hipError_t launch_bloch_pade<float>(int, const BlochArgs<float> &, hipStream_t);

}  // namespace mln
