// stream.hip -- instantiations and launcher of the streamed one-step kernel
// of the 1-D grid (fwd_stream.hpp), rotation route, N = 2, 3, 4, 6.
#include <algorithm>
#include <type_traits>

#include "fwd_stream.hpp"

namespace mln {

namespace {
// at most 16 workgroups per compute unit; each loops over its chunks of cells
// (measured on 2^24 two-level cells: 16 per CU moves 5.07 / 4.18 / 4.70 TB/s
// in FP64 / FP32 / compensated FP32, 8 per CU 4.80 / 3.72 / 4.15, 4 and 32
// per CU within 2 % of 16, one workgroup per chunk 4.17 / 2.60 / 3.35)
int max_stream_blocks() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 2048;
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = 16 * cus;
  }
  return cache[dev];
}

template <int N, typename Real, bool COMP>
hipError_t launch_n(const FwdArgs<Real> &a, hipStream_t st) {
  const int64_t nchunks = (a.nx + kStreamThreads * kStreamCells - 1) / (kStreamThreads * kStreamCells);
  const unsigned nb = (unsigned)std::min<int64_t>(nchunks, max_stream_blocks());
  if constexpr (std::is_same<Real, float>::value && N <= 3) {
    hipLaunchKernelGGL((fwd_stream_kernel_f32<N, COMP>), dim3(nb), dim3(kStreamThreads), 0, st, a);
  } else {
    hipLaunchKernelGGL((fwd_stream_kernel<N, Real, COMP>), dim3(nb), dim3(kStreamThreads), 0, st, a);
  }
  return hipGetLastError();
}

template <typename Real, bool COMP>
hipError_t launch_c(int N, const FwdArgs<Real> &a, hipStream_t st) {
  switch (N) {
    case 2: return launch_n<2, Real, COMP>(a, st);
    case 3: return launch_n<3, Real, COMP>(a, st);
    case 4: return launch_n<4, Real, COMP>(a, st);
    case 6: return launch_n<6, Real, COMP>(a, st);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

template <typename Real>
hipError_t launch_fwd_stream(int N, bool comp, const FwdArgs<Real> &a, hipStream_t st) {
  if (a.nsteps != 1) return hipErrorInvalidValue;
  if constexpr (std::is_same<Real, float>::value) {
    if (comp) return launch_c<float, true>(N, a, st);
    return launch_c<float, false>(N, a, st);
  } else {
    if (comp) return hipErrorInvalidValue;
    return launch_c<double, false>(N, a, st);
  }
}

template hipError_t launch_fwd_stream<double>(int, bool, const FwdArgs<double> &, hipStream_t);
template hipError_t launch_fwd_stream<float>(int, bool, const FwdArgs<float> &, hipStream_t);

}  // namespace mln
