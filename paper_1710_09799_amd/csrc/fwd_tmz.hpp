#pragma once
// fwd_tmz.hpp -- the coupled step on a two-dimensional TMz Yee grid: the
// medium step of every cell is the one of the 1-D kernels (rotation route,
// Sec. 4.1 update rules fused as in cell_step); the field step is the 2-D
// form of Eq. maxwell for E_z, H_x, H_y (the paper restricts its models to
// one dimension, Conclusion).
//
// Staggering (arrays row major, index j * nx + i): E_z at (i, j), H_x at
// (i, j + 1/2), H_y at (i + 1/2, j); periodic in y.  One launch per time step
// n -> n + 1, one thread per cell, 64 x 4 cells per workgroup (a wavefront
// is one row of 64 cells: every array access of a wavefront is one
// contiguous segment):
//   H_x(i, j)  -= chy (E(i, j+1) - E(i, j))          every column
//   H_y(i, j)  += chx (E(i+1, j) - E(i, j))          i <= nx-2
//   medium cells: dP/dt and the Bloch state from E^n(i, j) (cell_step)
//   E(i, j) = ca E + cb (-dP/dt + (H_y(i) - H_y(i-1)) / dx
//                              - (H_x(j) - H_x(j-1)) / dy)     1 <= i <= nx-2
//   E(0, j) = amplitude s[n+1] profile[j];  Mur at column nx-1.
// A thread needs the new H on the faces left of and below its cell; it forms
// them itself from the old values (the same expression as the neighbour that
// owns them, so the two agree to the bit) instead of exchanging them, so a
// launch has no barrier after the factor staging.  E and H are ping-pong
// buffers (neighbours read the old values); the Bloch state is updated in
// place (each cell's state belongs to one thread).  The Mur column is
// written by the thread of column nx-2, which holds the new E it needs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fwd_impl.hpp"

namespace mln {

constexpr int kTmzTX = 64;  // cells per workgroup along x (one wavefront)
constexpr int kTmzTY = 4;   // rows per workgroup

template <typename Real>
struct TmzArgs {
  FacDev<Real> fac;
  const Real *Ein;
  Real *Eout;
  const Real *Hxin;
  Real *Hxout;
  const Real *Hyin;
  Real *Hyout;
  Real *z;            // Bloch state, [rows][ld] (compensated: D high rows, then D low rows)
  const Real *src;    // amplitude * samples[n], n = 0..nt
  const Real *prof;   // transverse source profile, ny values
  int64_t nx, ny, mx0, mx1, my0, my1, ld;
  int64_t n;          // this launch takes step n -> n + 1
  Real chx, chy, ca, cb, idx, idy, kmur;
  int snap;           // step n + 1 completes snapshot snap_i
  int64_t snap_i;
  double *pop_out, *e_out, *probe_out;
  int64_t opaque0;    // always 0 (see FwdArgs)
};

template <typename Real>
__device__ __forceinline__ Real tmz_hy(Real hy, Real chx, Real e_right, Real e) {
  return hy + chx * (e_right - e);
}
template <typename Real>
__device__ __forceinline__ Real tmz_hx(Real hx, Real chy, Real e_up, Real e) {
  return hx - chy * (e_up - e);
}

template <int N, typename Real, bool COMP>
__device__ __forceinline__ void tmz_step(const TmzArgs<Real> &a, Real *sF, double *sP) {
  constexpr int D = N * N - 1;
  constexpr int DL = COMP ? D : 1;
  if constexpr (!rot_smem<N>()) RotLds<N, Real, COMP>::stage(a.fac, sF);
  RotLds<N, Real, COMP>::stage_pop(a.fac, sP);
  __syncthreads();

  const int tx = threadIdx.x % kTmzTX, ty = threadIdx.x / kTmzTX;
  const int64_t i = (int64_t)blockIdx.x * kTmzTX + tx;
  const int64_t j = (int64_t)blockIdx.y * kTmzTY + ty;
  if (i >= a.nx || j >= a.ny) return;
  const int64_t nx = a.nx;
  const int64_t jp = (j + 1 == a.ny) ? 0 : j + 1;
  const int64_t jm = (j == 0) ? a.ny - 1 : j - 1;
  const int64_t g = j * nx + i;

  const Real E = a.Ein[g];
  const Real Eup = a.Ein[jp * nx + i];
  const Real hx = tmz_hx(a.Hxin[g], a.chy, Eup, E);
  a.Hxout[g] = hx;
  if (i == nx - 1) return;  // the Mur column is written by the thread of column nx-2
  const Real Er = a.Ein[g + 1];
  const Real hy = tmz_hy(a.Hyin[g], a.chx, Er, E);
  a.Hyout[g] = hy;

  Real P = 0;
  if (i >= a.mx0 && i < a.mx1 && j >= a.my0 && j < a.my1) {
    const int64_t mw = a.mx1 - a.mx0, nmed = mw * (a.my1 - a.my0);
    const int64_t c = (j - a.my0) * mw + (i - a.mx0);
    Real z[D], zl[DL];
#pragma unroll
    for (int k = 0; k < D; ++k) z[k] = a.z[k * a.ld + c];
#pragma unroll
    for (int k = 0; k < DL; ++k) zl[k] = COMP ? a.z[(D + k) * a.ld + c] : Real(0);
    double *pp = (a.snap && a.pop_out) ? a.pop_out + a.snap_i * N * nmed + c : nullptr;
    P = cell_step<N, Real, ROUTE_ROT, COMP>(a.fac, sF, sP, E, z, zl, pp, nmed, a.opaque0 * a.n);
#pragma unroll
    for (int k = 0; k < D; ++k) a.z[k * a.ld + c] = z[k];
    if constexpr (COMP) {
#pragma unroll
      for (int k = 0; k < D; ++k) a.z[(D + k) * a.ld + c] = zl[k];
    }
  }

  Real En;
  if (i == 0) {
    En = a.src[a.n + 1] * a.prof[j];
  } else {
    const Real El = a.Ein[g - 1];
    const Real Edn = a.Ein[jm * nx + i];
    const Real hyl = tmz_hy(a.Hyin[g - 1], a.chx, E, El);
    const Real hxd = tmz_hx(a.Hxin[jm * nx + i], a.chy, E, Edn);
    const Real curl = (hy - hyl) * a.idx - (hx - hxd) * a.idy;
    En = a.ca * E + a.cb * (-P + curl);
  }
  a.Eout[g] = En;
  const size_t cells = (size_t)nx * a.ny;
  if (a.snap && a.e_out) a.e_out[a.snap_i * cells + g] = (double)En;
  if (i == nx - 2) {  // first-order Mur boundary on column nx-1
    const Real Eb = E + a.kmur * (En - Er);
    a.Eout[g + 1] = Eb;
    if (a.probe_out) a.probe_out[(a.n + 1) * a.ny + j] = (double)Eb;
    if (a.snap && a.e_out) a.e_out[a.snap_i * cells + g + 1] = (double)Eb;
  }
}

// N = 4, 6
template <int N, typename Real, bool COMP>
__global__ void __launch_bounds__(kTmzTX * kTmzTY) fwd_tmz_kernel(TmzArgs<Real> a) {
  constexpr int D = N * N - 1;
  __shared__ Real sF[rot_smem<N>() ? 1 : RotLds<N, Real, COMP>::size];
  __shared__ double sP[N * D + N];
  tmz_step<N, Real, COMP>(a, sF, sP);
}

// N = 2, 3 in FP64 and compensated FP32, compiled for at least five
// wavefronts per SIMD (measured on the 2048 x 512 three-level beam: FP64
// 26.9 against 27.9 us per step, compensated FP32 25.0 against 25.8, the
// same bits; seven or eight wavefronts spill and run 1.3-1.8x slower; N = 4,
// 6 would spill)
template <int N, typename Real, bool COMP>
__global__ void __launch_bounds__(kTmzTX * kTmzTY) __attribute__((amdgpu_waves_per_eu(5, 8)))
fwd_tmz_kernel_w5(TmzArgs<Real> a) {
  constexpr int D = N * N - 1;
  __shared__ Real sF[rot_smem<N>() ? 1 : RotLds<N, Real, COMP>::size];
  __shared__ double sP[N * D + N];
  tmz_step<N, Real, COMP>(a, sF, sP);
}

// N = 2, 3 in plain FP32, compiled for seven wavefronts per SIMD (71 VGPRs,
// no spills; 15.6 against 16.2 us per step on the same beam)
template <int N>
__global__ void __launch_bounds__(kTmzTX * kTmzTY) __attribute__((amdgpu_waves_per_eu(7, 8)))
fwd_tmz_kernel_w7(TmzArgs<float> a) {
  constexpr int D = N * N - 1;
  __shared__ float sF[rot_smem<N>() ? 1 : RotLds<N, float, false>::size];
  __shared__ double sP[N * D + N];
  tmz_step<N, float, false>(a, sF, sP);
}

}  // namespace mln
