// floor.hip -- measurement diagnostics: the latency floor of one time step of
// the tile kernels, and the vector FMA rate of the chip.
//
// Step floor: workgroups of `threads` lanes that do, per step, what every
// tile kernel must do at least -- one value per lane written to LDS, one
// workgroup barrier, the two neighbours read back -- followed by a chain of
// CHAIN dependent FP32 FMAs (the length of a step's dependency chain).  Its
// time per step is what a step costs with no work beyond the exchange and
// the chain.
//
// FMA rate: every lane runs 16 independent FMA chains (plain, not packed,
// instructions) in FP32 or FP64 on a full chip of workgroups; the achieved
// FLOP/s is the vector peak the kernels can reach at the clock under load.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "handle.hpp"

namespace mln {
namespace {

__device__ __forceinline__ void floor_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <int CHAIN>
__global__ void __launch_bounds__(1024) step_floor_kernel(int nsteps, float *out) {
  __shared__ float s[2][1024 + 2];
  const int t = threadIdx.x;
  if (t < 2) {
    s[0][t ? blockDim.x + 1 : 0] = 0.0f;
    s[1][t ? blockDim.x + 1 : 0] = 0.0f;
  }
  float x = 1e-3f * (float)t;
  for (int k = 0; k < nsteps; ++k) {
    const int b = k & 1;
    s[b][t + 1] = x;
    floor_barrier();
    float y = s[b][t] + s[b][t + 2];
#pragma unroll
    for (int c = 0; c < CHAIN; ++c) y = fmaf(y, 0.999f, 1e-7f);
    x = y;
  }
  if (x == 12345.0f) out[blockIdx.x] = x;  // keeps the chain live; never true
}

template <typename T>
__global__ void __launch_bounds__(256) fma_rate_kernel(int iters, T *out) {
  constexpr int ILP = 16;
  T v[ILP];
#pragma unroll
  for (int i = 0; i < ILP; ++i) v[i] = (T)(threadIdx.x + i) * (T)1e-3;
  const T m = (T)0.999, c = (T)1e-7;
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int i = 0; i < ILP; ++i) v[i] = v[i] * m + c;
  }
  T acc = 0;
#pragma unroll
  for (int i = 0; i < ILP; ++i) acc += v[i];
  if (acc == (T)12345) out[blockIdx.x] = acc;  // keeps the chains live; never true
}

}  // namespace
}  // namespace mln

using namespace mln;

extern "C" int mln_measure_fma_rate(int32_t fp64, double *tflops) {
  if (!tflops) return set_err(MLN_EINVAL, "null output");
  const int blocks = 256 * 32, iters = 4096;  // 32 workgroups of 256 lanes per compute unit
  DevBuf out;
  HIP_TRY(out.alloc(sizeof(double) * blocks));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto launch = [&]() {
    if (fp64)
      hipLaunchKernelGGL(fma_rate_kernel<double>, dim3(blocks), dim3(256), 0, nullptr, iters, (double *)out.p);
    else
      hipLaunchKernelGGL(fma_rate_kernel<float>, dim3(blocks), dim3(256), 0, nullptr, iters, (float *)out.p);
    return hipGetLastError();
  };
  float ms = 0.f;
  hipError_t e = launch();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("fma rate: ") + hipGetErrorString(e));
  *tflops = 2.0 * 16 * (double)iters * blocks * 256 / (ms * 1e-3) / 1e12;
  return MLN_OK;
}

extern "C" int mln_measure_step_floor(int32_t workgroups, int32_t threads, int32_t steps, int32_t chain,
                                      double *us_per_step) {
  if (!us_per_step || workgroups < 1 || steps < 1 || threads < 64 || threads > 1024 || threads % 64)
    return set_err(MLN_EINVAL, "step floor: workgroups >= 1, steps >= 1, threads a multiple of 64 in [64, 1024]");
  if (chain != 0 && chain != 32 && chain != 64 && chain != 128)
    return set_err(MLN_EINVAL, "step floor: chain must be 0, 32, 64 or 128");
  DevBuf out;
  HIP_TRY(out.alloc(sizeof(float) * (size_t)workgroups));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto launch = [&](int n) {
    const dim3 g((unsigned)workgroups), b((unsigned)threads);
    float *o = (float *)out.p;
    switch (chain) {
      case 0: hipLaunchKernelGGL(step_floor_kernel<0>, g, b, 0, nullptr, n, o); break;
      case 32: hipLaunchKernelGGL(step_floor_kernel<32>, g, b, 0, nullptr, n, o); break;
      case 64: hipLaunchKernelGGL(step_floor_kernel<64>, g, b, 0, nullptr, n, o); break;
      default: hipLaunchKernelGGL(step_floor_kernel<128>, g, b, 0, nullptr, n, o); break;
    }
    return hipGetLastError();
  };
  // the difference of two launch lengths removes the launch overhead
  const int n1 = steps, n2 = 2 * steps;
  float ms1 = 0.f, ms2 = 0.f;
  hipError_t e = launch(n1);  // warm-up
  for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
    const int n = pass ? n2 : n1;
    if ((e = hipEventRecord(e0, nullptr)) != hipSuccess) break;
    if ((e = launch(n)) != hipSuccess) break;
    if ((e = hipEventRecord(e1, nullptr)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    (void)hipEventElapsedTime(pass ? &ms2 : &ms1, e0, e1);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("step floor: ") + hipGetErrorString(e));
  *us_per_step = 1e3 * (double)(ms2 - ms1) / (double)(n2 - n1);
  return MLN_OK;
}
