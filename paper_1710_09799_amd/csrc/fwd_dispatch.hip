// fwd_dispatch.hip -- selects the instantiation for the level count N.
#include "fwd_kernels.hpp"

namespace mln {

#define MLN_DECL(NN)                                                                              \
  template <typename Real>                                                                        \
  hipError_t launch_fwd_n##NN(int route, bool comp, bool cf, const FwdArgs<Real> &a, int64_t nblocks, int W, hipStream_t st); \
  template <typename Real>                                                                        \
  hipError_t launch_fwd_wave_n##NN(bool comp, int C, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st); \
  template <typename Real>                                                                        \
  hipError_t launch_bloch_n##NN(int route, bool comp, const BlochArgs<Real> &a, hipStream_t st);
template <typename Real>
hipError_t launch_fwd_quad_n2(bool comp, bool cf, bool mf, int W, const FwdArgs<Real> &a, int64_t nblocks,
                              hipStream_t st);
template <typename Real>
hipError_t launch_fwd_quad_n3(bool comp, bool cf, bool mf, int W, const FwdArgs<Real> &a, int64_t nblocks,
                              hipStream_t st);
hipError_t launch_fwd_mfma_n4(int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st);
hipError_t launch_fwd_mfma_n6(int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st);

hipError_t launch_fwd_mfma(int N, int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st) {
  switch (N) {
    case 4: return launch_fwd_mfma_n4(nprod, a, nblocks, W, st);
    case 6: return launch_fwd_mfma_n6(nprod, a, nblocks, W, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_adj_n2(const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st);
template <typename Real>
hipError_t launch_adj_n3(const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st);

MLN_DECL(2)
MLN_DECL(3)
MLN_DECL(4)
MLN_DECL(6)
#undef MLN_DECL

template <typename Real>
hipError_t launch_fwd(int N, int route, bool comp, bool cf, const FwdArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  if (route == ROUTE_PADE && N >= 4) return comp ? hipErrorInvalidValue : launch_fwd_pade<Real>(N, a, nblocks, st);
  switch (N) {
    case 2: return launch_fwd_n2<Real>(route, comp, cf, a, nblocks, W, st);
    case 3: return launch_fwd_n3<Real>(route, comp, cf, a, nblocks, W, st);
    case 4: return launch_fwd_n4<Real>(route, comp, cf, a, nblocks, W, st);
    case 6: return launch_fwd_n6<Real>(route, comp, cf, a, nblocks, W, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_bloch(int N, int route, bool comp, const BlochArgs<Real> &a, hipStream_t st) {
  if (route == ROUTE_PADE && N >= 4) return comp ? hipErrorInvalidValue : launch_bloch_pade<Real>(N, a, st);
  switch (N) {
    case 2: return launch_bloch_n2<Real>(route, comp, a, st);
    case 3: return launch_bloch_n3<Real>(route, comp, a, st);
    case 4: return launch_bloch_n4<Real>(route, comp, a, st);
    case 6: return launch_bloch_n6<Real>(route, comp, a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t launch_fwd_wave(int N, bool comp, int C, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st) {
  switch (N) {
    case 2: return launch_fwd_wave_n2<Real>(comp, C, a, nblocks, st);
    case 3: return launch_fwd_wave_n3<Real>(comp, C, a, nblocks, st);
    case 4: return launch_fwd_wave_n4<Real>(comp, C, a, nblocks, st);
    case 6: return launch_fwd_wave_n6<Real>(comp, C, a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fwd_wave<double>(int, bool, int, const FwdArgs<double> &, int64_t, hipStream_t);
template hipError_t launch_fwd_wave<float>(int, bool, int, const FwdArgs<float> &, int64_t, hipStream_t);

template <typename Real>
hipError_t launch_fwd_quad(int N, bool comp, bool cf, bool mf, int W, const FwdArgs<Real> &a, int64_t nblocks,
                           hipStream_t st) {
  switch (N) {
    case 2: return launch_fwd_quad_n2<Real>(comp, cf, mf, W, a, nblocks, st);
    case 3: return launch_fwd_quad_n3<Real>(comp, cf, mf, W, a, nblocks, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_fwd_quad<double>(int, bool, bool, bool, int, const FwdArgs<double> &, int64_t, hipStream_t);
template hipError_t launch_fwd_quad<float>(int, bool, bool, bool, int, const FwdArgs<float> &, int64_t, hipStream_t);

template <typename Real>
hipError_t launch_adj(int N, const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st) {
  switch (N) {
    case 2: return launch_adj_n2<Real>(a, nblocks, W, st);
    case 3: return launch_adj_n3<Real>(a, nblocks, W, st);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_adj<double>(int, const AdjArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_adj<float>(int, const AdjArgs<float> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd<double>(int, int, bool, bool, const FwdArgs<double> &, int64_t, int, hipStream_t);
template hipError_t launch_fwd<float>(int, int, bool, bool, const FwdArgs<float> &, int64_t, int, hipStream_t);
template hipError_t launch_bloch<double>(int, int, bool, const BlochArgs<double> &, hipStream_t);
template hipError_t launch_bloch<float>(int, int, bool, const BlochArgs<float> &, hipStream_t);

}  // namespace mln
