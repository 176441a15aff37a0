// fwd_wave.hpp -- single-wavefront tile kernel of the rotation route.
//
// The tile kernel in fwd_impl.hpp spends most of a time step waiting: with
// one cell per thread and a few hundred tiles there is about one wavefront per
// SIMD, and each step crosses two workgroup barriers and two LDS round trips.
// This kernel removes both:
//   * one workgroup is one wavefront (64 lanes); lane l carries C consecutive
//     cells, so neighbours inside a lane are plain registers;
//   * the only cross-lane traffic per step is a wavefront shift by one lane
//     (DPP wave_shr / wave_shl) of the first and last E of each lane;
//   * the H face to the left of a lane's first cell, which the E update of
//     that cell needs, is kept as a private copy: the lane updates it with the
//     same operands and operations as its left neighbour updates its own last
//     face, so the two copies stay bit-identical and no second exchange (and
//     no barrier) is needed.
// The temporal blocking is unchanged: the tile covers 64*C cells, advances
// `nsteps <= halo` steps, and writes back its `owned` central cells.
#pragma once

#include "fwd_impl.hpp"

namespace mln {

// lane i receives lane i-1's value (SHR) or lane i+1's value (SHL); the lane
// with no source receives 0
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ float wave_shift(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double wave_shift(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <int N, typename Real, bool COMP, int C>
__global__ void __launch_bounds__(64) fwd_wave_kernel(FwdArgs<Real> a) {
  constexpr int D = N * N - 1;
  constexpr int DL = COMP ? D : 1;
  using L = RotLds<N, Real, COMP>;
  __shared__ Real sF[L::size];
  __shared__ Real sSrc[kMaxStepsPerLaunch];
  __shared__ double sP[N * D + N];
  L::stage(a.fac, sF);
  L::stage_pop(a.fac, sP);
  __syncthreads();
  const int lane = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const int64_t g0 = base + (int64_t)lane * C;
  const int64_t nmed = a.me - a.mb;

  Real E[C], H[C], z[C][D], zl[C][DL];
  Real Hl = 0;
  if (g0 - 1 >= 0 && g0 - 1 <= a.nx - 2) Hl = a.Hin[g0 - 1];
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const int64_t g = g0 + j;
    const bool in_dom = g >= 0 && g < a.nx;
    const bool med = g >= a.mb && g < a.me;
    E[j] = in_dom ? a.Ein[g] : Real(0);
    H[j] = (in_dom && g <= a.nx - 2) ? a.Hin[g] : Real(0);
#pragma unroll
    for (int i = 0; i < D; ++i) z[j][i] = med ? a.zin[i * a.ld + (g - a.mb)] : Real(0);
#pragma unroll
    for (int i = 0; i < DL; ++i) zl[j][i] = (COMP && med) ? a.zin[(D + i) * a.ld + (g - a.mb)] : Real(0);
  }
  // owned cells: tile-local index in [halo, halo + owned)
  auto owned_cell = [&](int j) {
    const int64_t t = (int64_t)lane * C + j;
    const int64_t g = g0 + j;
    return t >= a.halo && t < a.halo + a.owned && g >= 0 && g < a.nx;
  };

  // source samples of this launch (read by the tile holding cell 0)
  for (int i = threadIdx.x; i < a.nsteps; i += blockDim.x) sSrc[i] = a.src[a.step0 + 1 + i];
  __syncthreads();
  int64_t snap_next = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = n == snap_next;
    const Real El = wave_shift<kDppWaveShr1>(E[C - 1]);
    const Real Er = wave_shift<kDppWaveShl1>(E[0]);
    // H^{n+1/2}: the private copy of the face left of cell g0, then own faces
    if (g0 - 1 >= 0 && g0 - 1 <= a.nx - 2) Hl += a.ch * (E[0] - El);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t g = g0 + j;
      const Real Eright = (j + 1 < C) ? E[j + 1] : Er;
      if (g >= 0 && g <= a.nx - 2) H[j] += a.ch * (Eright - E[j]);
    }
    // Liouville step of every medium cell (and the adjoint tape)
    Real P[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t g = g0 + j;
      P[j] = 0;
      if (g >= a.mb && g < a.me) {
        const int64_t c = g - a.mb;
        const bool own = owned_cell(j);
        if (a.tape && own && n >= a.tape_step0) {
          Real *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
#pragma unroll
          for (int i = 0; i < D; ++i) tp[i * a.ld] = z[j][i];
          tp[D * a.ld] = E[j];
        }
        double *pp = (snap && own && a.pop_out) ? a.pop_out + si * N * nmed + c : nullptr;
        P[j] = cell_step<N, Real, ROUTE_ROT, COMP>(a.fac, sF, sP, E[j], z[j], zl[j], pp, nmed, a.opaque0 * s);
      }
    }
    // E^{n+1}
    Real Eold[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      Eold[j] = E[j];
      const int64_t g = g0 + j;
      const Real Hleft = (j == 0) ? Hl : H[j - 1];
      if (g >= 1 && g <= a.nx - 2)
        E[j] = a.ca * E[j] + a.cb * (-P[j] + (H[j] - Hleft) * a.inv_dx);
      else if (g == 0)
        E[j] = sSrc[s];
    }
    // first-order Mur boundary at cell nx-1 (needs E^n and E^{n+1} of nx-2)
    const Real Eln = wave_shift<kDppWaveShr1>(E[C - 1]);
#pragma unroll
    for (int j = 0; j < C; ++j) {
      if (g0 + j == a.nx - 1) {
        const Real prev_old = (j == 0) ? El : Eold[j - 1];
        const Real prev_new = (j == 0) ? Eln : E[j - 1];
        E[j] = prev_old + a.kmur * (prev_new - Eold[j]);
        if (a.probe_out && owned_cell(j)) a.probe_out[n + 1] = (double)E[j];
      }
    }
    if (snap) {
      if (a.e_out) {
#pragma unroll
        for (int j = 0; j < C; ++j)
          if (owned_cell(j)) a.e_out[si * a.nx + g0 + j] = (double)E[j];
      }
      snap_next += a.snap_every;
      ++si;
    }
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    if (!owned_cell(j)) continue;
    const int64_t g = g0 + j;
    a.Eout[g] = E[j];
    if (g <= a.nx - 2) a.Hout[g] = H[j];
    if (g >= a.mb && g < a.me) {
      const int64_t c = g - a.mb;
#pragma unroll
      for (int i = 0; i < D; ++i) a.zout[i * a.ld + c] = z[j][i];
      if constexpr (COMP) {
#pragma unroll
        for (int i = 0; i < D; ++i) a.zout[(D + i) * a.ld + c] = zl[j][i];
      }
    }
  }
}

}  // namespace mln
