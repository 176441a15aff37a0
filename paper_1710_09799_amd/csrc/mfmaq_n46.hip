// mfmaq_n46.hip -- instantiations of the four-lanes-per-cell split-BF16 MFMA
// kernel (N = 4 and 6; six or three products).
#include "fwd_mfmaq.hpp"

namespace mln {

namespace {
template <int N, int NPROD>
hipError_t launch_one(const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st) {
  const size_t lds = mfmaq_lds_bytes<N, NPROD>(W);
  hipError_t e = hipFuncSetAttribute((const void *)fwd_mfmaq_kernel<N, NPROD>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fwd_mfmaq_kernel<N, NPROD>), dim3((unsigned)nblocks), dim3(4 * W), lds, st, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_fwd_mfmaq(int N, int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st) {
  if (W < 16 || W > kMaxMfmaqTile || W % 16) return hipErrorInvalidValue;
  if (N == 4 && nprod == 6) return launch_one<4, 6>(a, nblocks, W, st);
  if (N == 4 && nprod == 3) return launch_one<4, 3>(a, nblocks, W, st);
  if (N == 6 && nprod == 6) return launch_one<6, 6>(a, nblocks, W, st);
  if (N == 6 && nprod == 3) return launch_one<6, 3>(a, nblocks, W, st);
  return hipErrorInvalidValue;
}

}  // namespace mln
