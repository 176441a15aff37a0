#pragma once
// fwd_impl.hpp -- gfx950 kernels of the coupled Maxwell-Liouville-von
// Neumann time step (arXiv:1710.09799, Sec. 2-4).
//
// Structure of one launch ("tile kernel"):
//   * one workgroup owns a contiguous tile of `owned` cells and also loads
//     `halo` cells on each side; one thread carries one cell;
//   * the launch advances `nsteps <= halo` time steps entirely on chip: E and
//     H live in registers and are exchanged between neighbouring threads
//     through LDS, the Bloch state of the cell lives in registers;
//   * the error made at the tile edges (missing neighbours) travels inwards by
//     one cell per step, so after nsteps <= halo steps every owned cell is
//     exact; only owned cells are written back (ping-pong buffers).
// Per step and cell (Sec. 4.1 update rules, Fig. 1 staggering):
//   H^{n+1/2}_{i+1/2} = H^{n-1/2}_{i+1/2} + dt/(mu dx) (E^n_{i+1} - E^n_i)
//   d''  = exp(U E^n_i dt) d'                       (route dependent)
//   dP/dt = w . d'' + p0                            (Sec. 3 polarisation)
//   d'_next = A d'' + c   (A = exp(M dt), the two L1 half steps merged)
//   E^{n+1}_i = ca E^n_i + cb (-dP/dt + (H_{i+1/2} - H_{i-1/2})/dx)
// The state between steps is d' (after the first half step); populations of
// d^{n+1/2} = A0 d'' + b0 are formed in FP64 when recorded.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fwd_kernels.hpp"

namespace mln {

// sin(x) and cos(x) - 1.  Small arguments use the Taylor series of sine and
// of cos - 1 (exact to the last bit of the type for |x| < 0.05, and free of
// the cancellation that 1 - cos(x) suffers); larger ones call the device
// math library and form cos - 1 as -2 sin^2(x/2).
__device__ __forceinline__ void sincm1(double x, double &s, double &cm1) {
  const double x2 = x * x;
  if (fabs(x) < 0.05) {
    s = x * (1.0 + x2 * (-1.0 / 6.0 + x2 * (1.0 / 120.0 + x2 * (-1.0 / 5040.0 +
             x2 * (1.0 / 362880.0 + x2 * (-1.0 / 39916800.0))))));
    cm1 = x2 * (-0.5 + x2 * (1.0 / 24.0 + x2 * (-1.0 / 720.0 + x2 * (1.0 / 40320.0 +
            x2 * (-1.0 / 3628800.0)))));
  } else {
    const double h = sin(0.5 * x);
    s = sin(x);
    cm1 = -2.0 * h * h;
  }
}

__device__ __forceinline__ void sincm1(float x, float &s, float &cm1) {
  const float x2 = x * x;
  if (fabsf(x) < 0.05f) {
    s = x * (1.0f + x2 * (-1.0f / 6.0f + x2 * (1.0f / 120.0f + x2 * (-1.0f / 5040.0f))));
    cm1 = x2 * (-0.5f + x2 * (1.0f / 24.0f + x2 * (-1.0f / 720.0f)));
  } else {
    const float h = sinf(0.5f * x);
    s = sinf(x);
    cm1 = -2.0f * h * h;
  }
}

// d'' = exp(U E dt) d' for one cell, in place.  z holds T-coordinates for the
// rotation route and d-coordinates for routes D and R.
template <int N, typename Real, int ROUTE>
__device__ __forceinline__ void interaction(const FacDev<Real> &f, Real E, Real (&z)[N * N - 1]) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  if constexpr (ROUTE == ROUTE_ROT) {
    // T^T U T = blockdiag(theta_p J): each (u_ab, v_ab) pair turns by
    // theta_p E dt; the N-1 population directions are left alone.
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      Real s, cm1;
      sincm1(f.thdt[p] * E, s, cm1);
      const Real a = z[2 * p], b = z[2 * p + 1];
      z[2 * p] = a + (cm1 * a + s * b);
      z[2 * p + 1] = b + (cm1 * b - s * a);
    }
  } else if constexpr (ROUTE == ROUTE_DIAG) {
    // Eq. exp2: A_I = R exp(Lambda E dt) R^+ applied to d'; N^2-1 scalar
    // exponentials and two complex matrix-vector products.
    Real yr[D], yi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      Real ar = 0, ai = 0;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        ar += f.Rre[i * D + k] * z[i];
        ai -= f.Rim[i * D + k] * z[i];
      }
      Real s, cm1;
      sincm1(f.lamdt[k] * E, s, cm1);
      yr[k] = ar + (cm1 * ar - s * ai);
      yi[k] = ai + (cm1 * ai + s * ar);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Real acc = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) acc += f.Rre[i * D + k] * yr[k] - f.Rim[i * D + k] * yi[k];
      z[i] = acc;
    }
  } else {
    // generalised Rodrigues: A_I = I + sum_p sin(x_p) S_p + (1 - cos(x_p)) S_p^2
    Real out[D];
#pragma unroll
    for (int i = 0; i < D; ++i) out[i] = z[i];
#pragma unroll 1
    for (int p = 0; p < Q; ++p) {
      Real s, cm1;
      sincm1(f.thdt[p] * E, s, cm1);
      const Real *Sp = f.S + p * D * D, *S2p = f.S2 + p * D * D;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        Real a = 0, b = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          a += Sp[i * D + j] * z[j];
          b += S2p[i * D + j] * z[j];
        }
        out[i] += s * a - cm1 * b;
      }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) z[i] = out[i];
  }
}

// dP/dt from d'' and the merged L1 step d'_next = d'' + (A - I) d'' + c.
template <int N, typename Real>
__device__ __forceinline__ Real shared_factor(const FacDev<Real> &f, Real (&z)[N * N - 1]) {
  constexpr int D = N * N - 1;
  Real P = f.p0;
#pragma unroll
  for (int j = 0; j < D; ++j) P += f.wz[j] * z[j];
  Real nz[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Real acc = f.cz[i];
#pragma unroll
    for (int j = 0; j < D; ++j) acc += f.Km[i * D + j] * z[j];
    nz[i] = z[i] + acc;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) z[i] = nz[i];
  return P;
}

template <int N, typename Real>
__device__ __forceinline__ void record_pop(const FacDev<Real> &f, const Real (&z)[N * N - 1],
                                           double *pop, int64_t stride) {
  constexpr int D = N * N - 1;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double acc = f.popc[a];
#pragma unroll
    for (int j = 0; j < D; ++j) acc += f.pop[a * D + j] * (double)z[j];
    pop[a * stride] = acc;
  }
}

template <int N, typename Real, int ROUTE>
__global__ void __launch_bounds__(kMaxTile) fwd_tile_kernel(FwdArgs<Real> a) {
  constexpr int D = N * N - 1;
  __shared__ Real sE[kMaxTile];
  __shared__ Real sH[kMaxTile];
  __shared__ Real sMur;
  const int lid = threadIdx.x;
  const int W = blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const int64_t g = base + lid;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool tile_med = (base < a.me) && (base + W > a.mb);
  const bool has_right = (base <= a.nx - 1) && (base + W > a.nx - 1);
  const bool owned = in_dom && lid >= a.halo && lid < a.halo + a.owned;
  const int64_t c = g - a.mb;

  Real E = 0, H = 0;
  Real z[D];
  if (in_dom) {
    E = a.Ein[g];
    if (g < a.nx - 1) H = a.Hin[g];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) z[j] = is_med ? a.zin[j * a.ld + c] : Real(0);

  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = a.snap_every > 0 && ((n + 1) % a.snap_every) == 0;
    const int64_t si = snap ? (n + 1) / a.snap_every - 1 : 0;
    sE[lid] = E;
    __syncthreads();
    const Real Er = (lid + 1 < W) ? sE[lid + 1] : Real(0);
    const Real El = (lid > 0) ? sE[lid - 1] : Real(0);
    if (in_dom && g < a.nx - 1) H += a.ch * (Er - E);
    Real P = 0;
    if (tile_med && is_med) {
      interaction<N, Real, ROUTE>(a.fac, E, z);
      if (snap && owned && a.pop_out)
        record_pop<N, Real>(a.fac, z, a.pop_out + si * N * (a.me - a.mb) + c, a.me - a.mb);
      P = shared_factor<N, Real>(a.fac, z);
    }
    sH[lid] = H;
    __syncthreads();
    const Real Hl = (lid > 0) ? sH[lid - 1] : Real(0);
    const Real Eold = E;
    if (g >= 1 && g < a.nx - 1)
      E = a.ca * E + a.cb * (-P + (H - Hl) * a.inv_dx);
    else if (g == 0)
      E = a.src[n + 1];
    if (has_right) {  // first-order Mur boundary at cell nx-1
      if (g == a.nx - 2) sMur = E;
      __syncthreads();
      if (g == a.nx - 1) {
        E = El + a.kmur * (sMur - Eold);
        if (a.probe_out) a.probe_out[n + 1] = (double)E;
      }
    }
    if (snap && owned && a.e_out) a.e_out[si * a.nx + g] = (double)E;
  }
  if (owned) {
    a.Eout[g] = E;
    if (g < a.nx - 1) a.Hout[g] = H;
    if (is_med) {
#pragma unroll
      for (int j = 0; j < D; ++j) a.zout[j * a.ld + c] = z[j];
    }
  }
}

// Prescribed-field mode: one thread per medium cell, no FDTD.
template <int N, typename Real, int ROUTE>
__global__ void __launch_bounds__(256) bloch_kernel(BlochArgs<Real> a) {
  constexpr int D = N * N - 1;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  Real z[D];
#pragma unroll
  for (int j = 0; j < D; ++j) z[j] = a.z0[j];
  for (int64_t t = 0; t < a.nsteps; ++t) {
    const Real E = (Real)a.efield[t * a.ncell + c];
    interaction<N, Real, ROUTE>(a.fac, E, z);
    if (a.pop_out) record_pop<N, Real>(a.fac, z, a.pop_out + t * N * a.ncell + c, a.ncell);
    const Real P = shared_factor<N, Real>(a.fac, z);
    if (a.dp_out) a.dp_out[t * a.ncell + c] = (double)P;
  }
}

}  // namespace mln
