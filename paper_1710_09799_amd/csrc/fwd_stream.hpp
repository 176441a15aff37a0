#pragma once
// fwd_stream.hpp -- the coupled step of the 1-D grid streamed through HBM:
// one launch advances one time step, one thread per cell, and every cell's
// E, H and Bloch state are read from and written to device memory once per
// step.  This is the form whose bound is HBM bandwidth (the temporally
// blocked tile kernels keep the state on chip for many steps instead); it
// is the variant for grids far larger than the chip's registers.
//
// Per cell i (Sec. 4.1 update rules, Eq. maxwell on the Yee grid of Fig. 1):
//   H_i  = H_i + ch (E_{i+1} - E_i)                 (i <= nx-2)
//   medium cells: dP/dt and the Bloch state from E_i (cell_step)
//   E_i  = ca E_i + cb (-dP/dt + (H_i - H_{i-1}) / dx)     (1 <= i <= nx-2)
//   E_0  = source sample;  Mur at nx-1 (written by the thread of nx-2).
// The new H_{i-1} a thread needs is formed from the old values with the
// expression the owner of that face uses (bitwise equal), so threads do not
// exchange anything and a launch has no barrier after the factor staging.
// E, H and the state are ping-pong buffers (neighbours read the old E, H).
// The high part of the Bloch state and every output are accessed
// nontemporally: each is touched once per step, and keeping them out of the
// caches leaves those to the neighbour reads of E and H (measured on 2^24
// two-level cells: FP64 5.29 TB/s against 5.10, compensated FP32 4.96
// against 4.70, plain FP32 4.41 against 4.20).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fwd_impl.hpp"

namespace mln {

template <typename Real>
__device__ __forceinline__ Real stream_h(Real h, Real ch, Real e_right, Real e) {
  return h + ch * (e_right - e);
}

// C consecutive cells g0 .. g0+C-1 of the streamed step (cells >= nx-1 are
// skipped; the thread holding nx-2 also writes the Mur cell nx-1).  The C
// cells' E and H and their left and right neighbours are loaded once; H of
// the face left of each cell comes from the previous cell of the thread, or
// for the first cell is formed from the old values with the expression its
// owner uses.
template <int N, typename Real, bool COMP, int C>
__device__ __forceinline__ void stream_cells(const FwdArgs<Real> &a, const Real *sF, const double *sP,
                                             int64_t g0, int64_t zoff) {
  constexpr int D = N * N - 1;
  constexpr int DL = COMP ? D : 1;
  const int64_t nx = a.nx;
  const int64_t n = a.step0;
  const bool snap = n == a.snap_next;
  Real E[C + 2], Hold[C + 1];
  // E[k + 1] = E_{g0 + k}, E[0] = E_{g0 - 1}; Hold[k + 1] = H_{g0 + k}, Hold[0] = H_{g0 - 1}
#pragma unroll
  for (int k = 0; k <= C; ++k) {
    const int64_t g = g0 + k;
    E[k + 1] = g < nx ? a.Ein[g] : Real(0);
    Hold[k] = (g - 1 >= 0 && g - 1 < nx - 1) ? a.Hin[g - 1] : Real(0);
  }
  E[0] = g0 >= 1 ? a.Ein[g0 - 1] : Real(0);
  Real Hl = stream_h(Hold[0], a.ch, E[1], E[0]);  // new H_{g0-1}
#pragma unroll
  for (int k = 0; k < C; ++k) {
    const int64_t g = g0 + k;
    if (g >= nx - 1) break;
    const Real Ec = E[k + 1], Er = E[k + 2];
    const Real H = stream_h(Hold[k + 1], a.ch, Er, Ec);
    __builtin_nontemporal_store(H, &a.Hout[g]);
    Real P = 0;
    if (g >= a.mb && g < a.me) {
      const int64_t c = g - a.mb, nmed = a.me - a.mb;
      Real z[D], zl[DL];
#pragma unroll
      for (int j = 0; j < D; ++j) z[j] = __builtin_nontemporal_load(&a.zin[j * a.ld + c]);
#pragma unroll
      for (int j = 0; j < DL; ++j) zl[j] = COMP ? a.zin[(D + j) * a.ld + c] : Real(0);
      if (a.tape && n >= a.tape_step0) {
        Real *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
#pragma unroll
        for (int j = 0; j < D; ++j) tp[j * a.ld] = z[j];
        tp[D * a.ld] = Ec;
      }
      double *pp = (snap && a.pop_out) ? a.pop_out + a.snap_i0 * N * nmed + c : nullptr;
      P = cell_step<N, Real, ROUTE_ROT, COMP>(a.fac, sF, sP, Ec, z, zl, pp, nmed, zoff);
#pragma unroll
      for (int j = 0; j < D; ++j) __builtin_nontemporal_store(z[j], &a.zout[j * a.ld + c]);
      if constexpr (COMP) {
#pragma unroll
        for (int j = 0; j < D; ++j) a.zout[(D + j) * a.ld + c] = zl[j];
      }
    }
    const Real En = (g == 0) ? a.src[n + 1] : a.ca * Ec + a.cb * (-P + (H - Hl) * a.inv_dx);
    __builtin_nontemporal_store(En, &a.Eout[g]);
    if (snap && a.e_out) a.e_out[a.snap_i0 * nx + g] = (double)En;
    if (g == nx - 2) {  // first-order Mur boundary at cell nx-1
      const Real Eb = Ec + a.kmur * (En - Er);
      __builtin_nontemporal_store(Eb, &a.Eout[g + 1]);
      if (a.probe_out) a.probe_out[n + 1] = (double)Eb;
      if (snap && a.e_out) a.e_out[a.snap_i0 * nx + g + 1] = (double)Eb;
    }
    Hl = H;
  }
}

// A workgroup stages the factors once and then takes chunks of
// kStreamThreads * kStreamCells cells blockIdx.x, blockIdx.x + gridDim.x, ...
// (the launcher caps the grid at a few workgroups per compute unit), so the
// staging is not repeated for every chunk of a large grid.
template <int N, typename Real, bool COMP>
__device__ __forceinline__ void stream_grid(const FwdArgs<Real> &a, Real *sF, double *sP) {
  constexpr int CH = kStreamThreads * kStreamCells;
  if constexpr (!rot_smem<N>()) RotLds<N, Real, COMP>::stage(a.fac, sF);
  RotLds<N, Real, COMP>::stage_pop(a.fac, sP);
  __syncthreads();
  const int64_t nchunks = (a.nx + CH - 1) / CH;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    // keep the factor reads (LDS, and for large D the scalar loads indexed
    // with the loop-variant zero offset) inside the loop instead of holding
    // every factor in registers across it
    __asm__ volatile("" ::: "memory");
    const int64_t g0 = ch * CH + (int64_t)threadIdx.x * kStreamCells;
    if (g0 < a.nx - 1) stream_cells<N, Real, COMP, kStreamCells>(a, sF, sP, g0, a.opaque0 * ch);
  }
}

// FP64, and FP32 for N = 4, 6
template <int N, typename Real, bool COMP>
__global__ void __launch_bounds__(kStreamThreads) fwd_stream_kernel(FwdArgs<Real> a) {
  constexpr int D = N * N - 1;
  __shared__ Real sF[rot_smem<N>() ? 1 : RotLds<N, Real, COMP>::size];
  __shared__ double sP[N * D + N];
  stream_grid<N, Real, COMP>(a, sF, sP);
}

// FP32 and compensated FP32 for N = 2, 3, compiled for eight wavefronts per
// SIMD (measured on 2^24 two-level cells: 96.8 against 107-110 us per step
// in FP32, 133.5 against 137 in compensated FP32; the FP64 instances gain
// nothing, and they and the N = 4, 6 instances would spill, so they keep
// the default register budget)
template <int N, bool COMP>
__global__ void __launch_bounds__(kStreamThreads) __attribute__((amdgpu_waves_per_eu(8, 8)))
fwd_stream_kernel_f32(FwdArgs<float> a) {
  constexpr int D = N * N - 1;
  __shared__ float sF[rot_smem<N>() ? 1 : RotLds<N, float, COMP>::size];
  __shared__ double sP[N * D + N];
  stream_grid<N, float, COMP>(a, sF, sP);
}

}  // namespace mln
