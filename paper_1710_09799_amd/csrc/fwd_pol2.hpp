#pragma once
// fwd_pol2.hpp -- both transverse field components of a wave along x, with
// the interaction Hamiltonian H_I = -mu_z E_z - mu_y E_y (the paper keeps
// E_z and -mu E_z only, Sec. 2, and names the fixed interaction form as a
// limitation, Conclusion).
//
// Fields: two independent Yee pairs on the grid of Fig. 1, (E_z, H_y) and
// (E_y, G) with G = -H_z, which obeys the update of (E_z, H_y) in the same
// form (Eq. maxwell for the other polarisation); the medium couples them.
//
// Medium step (Sec. 4.1 with the interaction factor split symmetrically so
// that every factor has a fixed generator and keeps the rotation form of
// the paper's exponential routes, Sec. 4.2):
//   d'  = A0 d + b0
//   d'' = exp(U_y E_y dt/2) exp(U_z E_z dt) exp(U_y E_y dt/2) d'
//   d^{n+1/2} = A0 d'' + b0,   dP_k/dt = w_k . d'' + p0_k   (k = z, y)
// carried in the rotation coordinates of U_y, u = T_y^T d' (T_k^T U_k T_k =
// blockdiag(theta_k J)): the two y factors are 2x2 rotations of u, the z
// factor is B Rot_z B^T with B = T_y^T T_z, and the two half steps of
// consecutive steps merge into K_u = T_y^T A0^2 T_y, c_u = T_y^T (A0 + I) b0.
// A step costs three D x D products (B^T, B, K_u) and three rotation sets.
//
// Two kernels share the cell arithmetic:
// * fwd_pol2_kernel: one launch per time step, one thread per cell, every
//   field and Bloch vector read from and written to device memory once per
//   step; the new H on the face left of a cell is formed from the old values
//   with the expression its owner uses (bitwise equal), so no thread waits
//   for another;
// * fwd_pol2_tile_kernel: several steps per launch (temporal blocking), one
//   thread per cell of a window of kPol2TileW cells; E_z, H_y, E_y and G of
//   the window in LDS (two buffers, one barrier per step), the Bloch vector
//   in registers; each workgroup owns kPol2TileW - 2 K - 1 cells and
//   recomputes K cells on its right and K + 1 on its left (the stencil
//   radius is one cell, two for the Mur cell), so neighbouring workgroups
//   never wait for each other;
// * fwd_pol2_quad_kernel: the same blocking with four lanes per cell (the
//   layout of the single-component quad kernel): lane r holds components
//   2r, 2r+1 of the Bloch vector in each coordinate system, so each rotation
//   is lane-local, and each of the three products is a gather of the other
//   lanes' components (DPP) and two rows per lane, with its factor rows in
//   registers for the whole launch; dP/dt is a quad sum.  A step then costs
//   a quarter of the single-lane products per lane, and 128-cell windows
//   spread a grid over more compute units.
// FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fwd_quad.hpp"

namespace mln {

constexpr int kPol2TileW = 256;      // threads (cells) per workgroup of the tile kernel
constexpr int kPol2MaxSteps = 64;    // steps per launch of the tile kernel: W - 2 K - 1 >= 127 owned cells
constexpr int kPol2QuadCells = 128;  // cells per window of the quad kernel (512 lanes)
constexpr int kPol2QuadMaxSteps = 48;  // C - 2 K - 1 >= 31 owned cells

// factor block (doubles): B, for N = 4, 6 also B^T (so that every product
// reads rows, which their scalar loads fetch in wide contiguous pieces; the
// N <= 3 kernels read B's columns from LDS, measured faster), K_u, c_u,
// w_z, w_y (in u-coordinates), the rotation angles per unit field
// theta_y dt/2 and theta_z dt, population rows in u-coordinates and their
// constants, p0_z, p0_y
template <int N>
struct Pol2Layout {
  static constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  static constexpr int nBt = N > 3 ? D * D : 0;
  static constexpr int oB = 0, oBt = D * D, oK = D * D + nBt, oc = oK + D * D, owz = oc + D, owy = owz + D;
  static constexpr int othy = owy + D, othz = othy + Q, opop = othz + Q, opopc = opop + N * D;
  static constexpr int op0 = opopc + N, size = op0 + 2;
};

struct Pol2Args {
  const double *fac;
  const double *Ezin, *Hyin, *Eyin, *Gin;
  double *Ezout, *Hyout, *Eyout, *Gout;
  const double *uin;    // state [D][ld] before the launch
  double *uout;         // state after the launch
  const double *src;    // source waveform, nt + 1 samples
  int64_t nx, mb, me, ld, n0;  // n0: the launch's first step (fields n0 -> n0 + 1)
  int nsteps, halo;            // tile kernel: steps in this launch (<= halo), steps per launch of the handle
  int64_t owned;               // tile kernel: cells owned by a workgroup, kPol2TileW - 2 halo - 1
  double amp_z, amp_y, ch, ca, cb, inv_dx, kmur;
  int64_t opaque0;             // always 0 (see Pol2FacSmem)
  int64_t snap_every, snap_next, snap_i0;  // first snapshot step >= n0 (-1: none) and its index
  double *ez_out, *ey_out, *pop_out, *probe_z, *probe_y;  // device records (NULL: not recorded)
};

// sin x and cos x - 1.  |x| <= 1/2 in the whole wavefront (every rotation
// angle of a time step in practice): the Taylor series through x^17 and
// x^16 in Estrin form (truncation below 1e-22 relative); otherwise the
// device library, kept out of line so that its argument reduction does not
// hold registers in the step.
__device__ __noinline__ double2 pol2_sincos_library(double x) {
  double s, c;
  sincos(x, &s, &c);
  return make_double2(s, c - 1.0);
}
__device__ __forceinline__ void pol2_sincm1(double x, double &s, double &cm1) {
  if (!__any(fabs(x) > 0.5)) {
    const double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
    const double sa = fma(x4, fma(x2, -1.0 / 5040.0, 1.0 / 120.0), fma(x2, -1.0 / 6.0, 1.0));
    const double sb = fma(x4, fma(x2, -1.0 / 1307674368000.0, 1.0 / 6227020800.0),
                          fma(x2, -1.0 / 39916800.0, 1.0 / 362880.0));
    s = x * fma(x8, fma(x8, 1.0 / 355687428096000.0, sb), sa);
    const double ca = fma(x4, fma(x2, 1.0 / 40320.0, -1.0 / 720.0), fma(x2, 1.0 / 24.0, -0.5));
    const double cb = fma(x4, fma(x2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0),
                          fma(x2, 1.0 / 479001600.0, -1.0 / 3628800.0));
    cm1 = x2 * fma(x8, fma(x8, -1.0 / 6402373705728000.0, cb), ca);
  } else {
    const double2 r = pol2_sincos_library(x);
    s = r.x;
    cm1 = r.y;
  }
}

// Factor access: from LDS for N <= 3, or through scalar loads of the factor
// block in device memory for N = 4, 6, whose D x D products (225 and 1225
// entries) would otherwise hold their LDS reads in vector registers.  The
// scalar loads' results live in scalar registers; p carries a zero offset
// that changes every step (Pol2Args::opaque0 times the step) so that the
// compiler keeps each load next to its use instead of hoisting all of them.
struct Pol2FacLds {
  const double *s;
  __device__ double operator[](int i) const { return s[i]; }
};
struct Pol2FacSmem {
  const double *p;
  __device__ double operator[](int i) const { return cld(p, i); }
};
template <int N>
constexpr bool pol2_smem() {
  return N > 3;
}

// sin and cos - 1 of the angles F[off + p] e, and the 2x2 rotations of the
// pairs (2p, 2p+1) by them
template <int Q, class FA>
__device__ __forceinline__ void pol2_angles(const FA &F, int off, double e, double (&s)[Q], double (&cm1)[Q]) {
#pragma unroll
  for (int p = 0; p < Q; ++p) pol2_sincm1(F[off + p] * e, s[p], cm1[p]);
}
template <int D, int Q>
__device__ __forceinline__ void pol2_rotate(double (&x)[D], const double (&s)[Q], const double (&cm1)[Q]) {
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    const double a = x[2 * p], b = x[2 * p + 1];
    x[2 * p] = a + (cm1[p] * a + s[p] * b);
    x[2 * p + 1] = b + (cm1[p] * b - s[p] * a);
  }
}

// the same rotations with each sin, cos - 1 formed where it is used
template <int D, int Q, class FA>
__device__ __forceinline__ void pol2_rotate_at(double (&x)[D], const FA &F, int off, double e) {
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    double s, cm1;
    pol2_sincm1(F[off + p] * e, s, cm1);
    const double a = x[2 * p], b = x[2 * p + 1];
    x[2 * p] = a + (cm1 * a + s * b);
    x[2 * p + 1] = b + (cm1 * b - s * a);
  }
}

// The medium step of one cell: u (= T_y^T d') -> T_y^T d'' through the split
// interaction factor, dP_z/dt and dP_y/dt from it, the populations of
// d^{n+1/2} into pp[lv * pstride] (pp NULL: not recorded), and the two half
// steps of this and the next step.  N <= 3 forms the y angles' sin and
// cos - 1 once for both half steps; N = 4, 6 form them twice (fewer live
// registers), with the same values.
template <int N, class FA>
__device__ __forceinline__ void pol2_medium(const FA &F, double (&u)[N * N - 1], double Ecz, double Ecy,
                                            double &Pz, double &Py, double *pp, int64_t pstride) {
  using L = Pol2Layout<N>;
  constexpr int D = L::D, Q = L::Q;
  constexpr bool reuse = N <= 3;
  double w[D], sy[reuse ? Q : 1], cy[reuse ? Q : 1];
  if constexpr (reuse) {
    pol2_angles<Q>(F, L::othy, Ecy, sy, cy);
    pol2_rotate<D, Q>(u, sy, cy);  // exp(U_y E_y dt/2)
  } else {
    pol2_rotate_at<D, Q>(u, F, L::othy, Ecy);
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {  // to z-rotation coordinates: w = B^T u
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) t += (L::nBt ? F[L::oBt + i * D + j] : F[L::oB + j * D + i]) * u[j];
    w[i] = t;
  }
  pol2_rotate_at<D, Q>(w, F, L::othz, Ecz);  // exp(U_z E_z dt)
#pragma unroll
  for (int i = 0; i < D; ++i) {  // back: u = B w
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) t += F[L::oB + i * D + j] * w[j];
    u[i] = t;
  }
  if constexpr (reuse) {
    pol2_rotate<D, Q>(u, sy, cy);  // exp(U_y E_y dt/2): u = T_y^T d''
  } else {
    pol2_rotate_at<D, Q>(u, F, L::othy, Ecy);
  }
  Pz = F[L::op0];
  Py = F[L::op0 + 1];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    Pz += F[L::owz + j] * u[j];
    Py += F[L::owy + j] * u[j];
  }
  if (pp) {
#pragma unroll
    for (int lv = 0; lv < N; ++lv) {
      double p = F[L::opopc + lv];
#pragma unroll
      for (int j = 0; j < D; ++j) p += F[L::opop + lv * D + j] * u[j];
      pp[lv * pstride] = p;
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {  // the two half steps of this and the next step
    double t = F[L::oc + i];
#pragma unroll
    for (int j = 0; j < D; ++j) t += F[L::oK + i * D + j] * u[j];
    w[i] = t;
  }
#pragma unroll
  for (int j = 0; j < D; ++j) u[j] = w[j];
}

// The field part of one cell g (0 <= g <= nx - 2) from the old E of the
// cell and its neighbours and the old H on its two faces: the new H on both
// faces (the left one as its owner forms it), then the new E (hard source
// at cell 0) with the medium's dP/dt, for one component pair.
struct Pol2Pair {
  double Hr, Hl;
};
__device__ __forceinline__ Pol2Pair pol2_faces(const Pol2Args &a, int64_t g, double El, double Ec, double Er,
                                               double Hl_old, double Hr_old) {
  Pol2Pair h;
  h.Hr = Hr_old + a.ch * (Er - Ec);
  h.Hl = g >= 1 ? Hl_old + a.ch * (Ec - El) : 0.0;
  return h;
}
__device__ __forceinline__ double pol2_e(const Pol2Args &a, int64_t g, double amp, int64_t n, double Ec,
                                         const Pol2Pair &h, double P) {
  return g == 0 ? amp * a.src[n + 1] : a.ca * Ec + a.cb * (-P + (h.Hr - h.Hl) * a.inv_dx);
}

template <int N, class FA>
__device__ __forceinline__ void pol2_cell(const Pol2Args &a, const FA &F, int64_t g) {
  constexpr int D = N * N - 1;
  const int64_t nx = a.nx, n = a.n0;
  const bool snap = n == a.snap_next;
  const double Ecz = a.Ezin[g], Erz = a.Ezin[g + 1], Elz = g >= 1 ? a.Ezin[g - 1] : 0.0;
  const double Ecy = a.Eyin[g], Ery = a.Eyin[g + 1], Ely = g >= 1 ? a.Eyin[g - 1] : 0.0;
  const Pol2Pair hz = pol2_faces(a, g, Elz, Ecz, Erz, g >= 1 ? a.Hyin[g - 1] : 0.0, a.Hyin[g]);
  const Pol2Pair hy = pol2_faces(a, g, Ely, Ecy, Ery, g >= 1 ? a.Gin[g - 1] : 0.0, a.Gin[g]);
  a.Hyout[g] = hz.Hr;
  a.Gout[g] = hy.Hr;
  double Pz = 0.0, Py = 0.0;
  if (g >= a.mb && g < a.me) {
    const int64_t c = g - a.mb, nmed = a.me - a.mb;
    double u[D];
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] = a.uin[j * a.ld + c];
    double *pp = (snap && a.pop_out) ? a.pop_out + a.snap_i0 * N * nmed + c : nullptr;
    pol2_medium<N>(F, u, Ecz, Ecy, Pz, Py, pp, nmed);
#pragma unroll
    for (int j = 0; j < D; ++j) a.uout[j * a.ld + c] = u[j];
  }
  const double Ezn = pol2_e(a, g, a.amp_z, n, Ecz, hz, Pz);
  const double Eyn = pol2_e(a, g, a.amp_y, n, Ecy, hy, Py);
  a.Ezout[g] = Ezn;
  a.Eyout[g] = Eyn;
  if (snap) {
    if (a.ez_out) a.ez_out[a.snap_i0 * nx + g] = Ezn;
    if (a.ey_out) a.ey_out[a.snap_i0 * nx + g] = Eyn;
  }
  if (g == nx - 2) {  // first-order Mur boundary at cell nx - 1, both components
    const double Ebz = Ecz + a.kmur * (Ezn - Erz), Eby = Ecy + a.kmur * (Eyn - Ery);
    a.Ezout[nx - 1] = Ebz;
    a.Eyout[nx - 1] = Eby;
    if (a.probe_z) a.probe_z[n + 1] = Ebz;
    if (a.probe_y) a.probe_y[n + 1] = Eby;
    if (snap) {
      if (a.ez_out) a.ez_out[a.snap_i0 * nx + nx - 1] = Ebz;
      if (a.ey_out) a.ey_out[a.snap_i0 * nx + nx - 1] = Eby;
    }
  }
}

template <int N>
__global__ void __launch_bounds__(256) fwd_pol2_kernel(Pol2Args a) {
  using L = Pol2Layout<N>;
  // the factor block in LDS (every lane reads the same element: broadcast);
  // read near its use instead of being held in registers across the step
  __shared__ double sF[pol2_smem<N>() ? 1 : L::size];
  if constexpr (!pol2_smem<N>()) {
    for (int i = threadIdx.x; i < L::size; i += blockDim.x) sF[i] = a.fac[i];
    __syncthreads();
  }
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nx - 1) return;  // cell nx - 1 (Mur) is written by the thread of nx - 2
  if constexpr (pol2_smem<N>()) {
    pol2_cell<N>(a, Pol2FacSmem{a.fac}, g);
  } else {
    pol2_cell<N>(a, Pol2FacLds{sF}, g);
  }
}

// a.nsteps steps (at most a.halo) on the window of workgroup b: cells
// o0 - halo - 1 .. o0 + owned + halo - 1 with o0 = b owned, thread i on cell
// o0 - halo - 1 + i.  Cells outside 0 .. nx-1 hold zero, as the one-step
// kernel's missing neighbours do.  After s steps the window's values are
// exact from its left end + s to its right end - s (the Mur cell from
// nx - 3 on), so after at most halo steps on the owned cells, which alone
// are written back and recorded.
template <int N>
__global__ void __launch_bounds__(kPol2TileW) fwd_pol2_tile_kernel(Pol2Args a) {
  using L = Pol2Layout<N>;
  constexpr int D = L::D, S = kPol2TileW + 2;
  __shared__ double sF[pol2_smem<N>() ? 1 : L::size];
  __shared__ double sE[2][2][S];  // [buffer][E_z, E_y][slot]; slot i + 1 holds thread i's cell
  __shared__ double sH[2][2][S];  // [buffer][H_y, G][slot]
  const int i = threadIdx.x, q = i + 1;
  const int64_t nx = a.nx;
  const int64_t o0 = (int64_t)blockIdx.x * a.owned, o1 = o0 + a.owned < nx ? o0 + a.owned : nx;
  const int64_t g = o0 - a.halo - 1 + i;
  if constexpr (!pol2_smem<N>())
    for (int k = i; k < L::size; k += kPol2TileW) sF[k] = a.fac[k];
  for (int k = i; k < 2 * 2 * S; k += kPol2TileW) {
    (&sE[0][0][0])[k] = 0.0;
    (&sH[0][0][0])[k] = 0.0;
  }
  __syncthreads();
  const bool act = g >= 0 && g < nx - 1;  // cells with a step of their own (nx - 1: Mur, from nx - 2)
  const bool med = g >= a.mb && g < a.me;
  const bool own = g >= o0 && g < o1;
  const bool last = o1 == nx;  // this workgroup records the Mur cell
  const int64_t c = g - a.mb, nmed = a.me - a.mb;
  if (g >= 0 && g < nx) {
    sE[0][0][q] = a.Ezin[g];
    sE[0][1][q] = a.Eyin[g];
  }
  if (act) {
    sH[0][0][q] = a.Hyin[g];
    sH[0][1][q] = a.Gin[g];
  }
  double u[D];
  if (med) {
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] = a.uin[j * a.ld + c];
  }
  __syncthreads();
  int b = 0;
  int64_t sn = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.n0 + s;
    const bool snap = n == sn;
    if (act) {
      const double Ecz = sE[b][0][q], Erz = sE[b][0][q + 1], Elz = sE[b][0][q - 1];
      const double Ecy = sE[b][1][q], Ery = sE[b][1][q + 1], Ely = sE[b][1][q - 1];
      const Pol2Pair hz = pol2_faces(a, g, Elz, Ecz, Erz, sH[b][0][q - 1], sH[b][0][q]);
      const Pol2Pair hy = pol2_faces(a, g, Ely, Ecy, Ery, sH[b][1][q - 1], sH[b][1][q]);
      double Pz = 0.0, Py = 0.0;
      if (med) {
        double *pp = (snap && own && a.pop_out) ? a.pop_out + si * N * nmed + c : nullptr;
        if constexpr (pol2_smem<N>()) {
          pol2_medium<N>(Pol2FacSmem{a.fac + a.opaque0 * s}, u, Ecz, Ecy, Pz, Py, pp, nmed);
        } else {
          pol2_medium<N>(Pol2FacLds{sF}, u, Ecz, Ecy, Pz, Py, pp, nmed);
        }
      }
      const double Ezn = pol2_e(a, g, a.amp_z, n, Ecz, hz, Pz);
      const double Eyn = pol2_e(a, g, a.amp_y, n, Ecy, hy, Py);
      sH[b ^ 1][0][q] = hz.Hr;
      sH[b ^ 1][1][q] = hy.Hr;
      sE[b ^ 1][0][q] = Ezn;
      sE[b ^ 1][1][q] = Eyn;
      if (snap && own) {
        if (a.ez_out) a.ez_out[si * nx + g] = Ezn;
        if (a.ey_out) a.ey_out[si * nx + g] = Eyn;
      }
      if (g == nx - 2) {  // first-order Mur boundary at cell nx - 1, both components
        const double Ebz = Ecz + a.kmur * (Ezn - Erz), Eby = Ecy + a.kmur * (Eyn - Ery);
        sE[b ^ 1][0][q + 1] = Ebz;
        sE[b ^ 1][1][q + 1] = Eby;
        if (last) {
          if (a.probe_z) a.probe_z[n + 1] = Ebz;
          if (a.probe_y) a.probe_y[n + 1] = Eby;
          if (snap) {
            if (a.ez_out) a.ez_out[si * nx + nx - 1] = Ebz;
            if (a.ey_out) a.ey_out[si * nx + nx - 1] = Eby;
          }
        }
      }
    }
    __syncthreads();
    b ^= 1;
    if (snap) {
      sn += a.snap_every;
      ++si;
    }
  }
  if (own) {
    a.Ezout[g] = sE[b][0][q];
    a.Eyout[g] = sE[b][1][q];
    if (g < nx - 1) {
      a.Hyout[g] = sH[b][0][q];
      a.Gout[g] = sH[b][1][q];
    }
    if (med) {
#pragma unroll
      for (int j = 0; j < D; ++j) a.uout[j * a.ld + c] = u[j];
    }
  }
}

// every lane of a quad receives the two components of lanes 0 .. NJ-1:
// u[2J], u[2J+1] from lane J
template <int NJ>
__device__ __forceinline__ void pol2_gather(double x0, double x1, double (&u)[2 * NJ]) {
  u[0] = quad_bcast<0>(x0);
  u[1] = quad_bcast<0>(x1);
  if constexpr (NJ > 1) {
    u[2] = quad_bcast<1>(x0);
    u[3] = quad_bcast<1>(x1);
  }
  if constexpr (NJ > 2) {
    u[4] = quad_bcast<2>(x0);
    u[5] = quad_bcast<2>(x1);
  }
  if constexpr (NJ > 3) {
    u[6] = quad_bcast<3>(x0);
    u[7] = quad_bcast<3>(x1);
  }
}

// Window as in fwd_pol2_tile_kernel, kPol2QuadCells cells of four lanes.
template <int N>
__global__ void __launch_bounds__(4 * kPol2QuadCells) fwd_pol2_quad_kernel(Pol2Args a) {
  using L = Pol2Layout<N>;
  constexpr int D = L::D, Q = L::Q, C = kPol2QuadCells, S = C + 2, NJ = (D + 1) / 2;
  static_assert(D <= 8 && Q <= 3, "four lanes of two components each");
  __shared__ double sE[2][2][S];  // [buffer][E_z, E_y][slot]; slot k + 1 holds the window's cell k
  __shared__ double sH[2][2][S];  // [buffer][H_y, G][slot]
  __shared__ double sP[N * D + N];  // population rows in u-coordinates and their constants
  const int lane = threadIdx.x & 3, k = threadIdx.x >> 2, q = k + 1;
  const int r0 = 2 * lane, r1 = 2 * lane + 1;
  const int64_t nx = a.nx;
  const int64_t o0 = (int64_t)blockIdx.x * a.owned, o1 = o0 + a.owned < nx ? o0 + a.owned : nx;
  const int64_t g = o0 - a.halo - 1 + k;
  for (int t = threadIdx.x; t < N * D + N; t += 4 * C) sP[t] = a.fac[L::opop + t];
  for (int t = threadIdx.x; t < 2 * 2 * S; t += 4 * C) {
    (&sE[0][0][0])[t] = 0.0;
    (&sH[0][0][0])[t] = 0.0;
  }
  // the lane's factor rows, held for the launch: columns r0, r1 of B (for
  // B^T u), rows r0, r1 of B and of K_u, and its entries of c, w_z, w_y;
  // zero for components beyond D
  double bt0[D], bt1[D], b0[D], b1[D], k0[D], k1[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    bt0[j] = r0 < D ? a.fac[L::oB + j * D + r0] : 0.0;
    bt1[j] = r1 < D ? a.fac[L::oB + j * D + r1] : 0.0;
    b0[j] = r0 < D ? a.fac[L::oB + r0 * D + j] : 0.0;
    b1[j] = r1 < D ? a.fac[L::oB + r1 * D + j] : 0.0;
    k0[j] = r0 < D ? a.fac[L::oK + r0 * D + j] : 0.0;
    k1[j] = r1 < D ? a.fac[L::oK + r1 * D + j] : 0.0;
  }
  const double c0 = r0 < D ? a.fac[L::oc + r0] : 0.0, c1 = r1 < D ? a.fac[L::oc + r1] : 0.0;
  const double wz0 = r0 < D ? a.fac[L::owz + r0] : 0.0, wz1 = r1 < D ? a.fac[L::owz + r1] : 0.0;
  const double wy0 = r0 < D ? a.fac[L::owy + r0] : 0.0, wy1 = r1 < D ? a.fac[L::owy + r1] : 0.0;
  const double thy = lane < Q ? a.fac[L::othy + lane] : 0.0, thz = lane < Q ? a.fac[L::othz + lane] : 0.0;
  const double p0z = a.fac[L::op0], p0y = a.fac[L::op0 + 1];
  __syncthreads();
  const bool act = g >= 0 && g < nx - 1;
  const bool med = g >= a.mb && g < a.me;
  const bool own = g >= o0 && g < o1;
  const bool last = o1 == nx;
  const int64_t c = g - a.mb, nmed = a.me - a.mb;
  if (lane == 0 && g >= 0 && g < nx) {
    sE[0][0][q] = a.Ezin[g];
    sE[0][1][q] = a.Eyin[g];
  }
  if (lane == 0 && act) {
    sH[0][0][q] = a.Hyin[g];
    sH[0][1][q] = a.Gin[g];
  }
  double x0 = 0.0, x1 = 0.0;  // the lane's two components of u
  if (med) {
    if (r0 < D) x0 = a.uin[r0 * a.ld + c];
    if (r1 < D) x1 = a.uin[r1 * a.ld + c];
  }
  __syncthreads();
  int b = 0;
  int64_t sn = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.n0 + s;
    const bool snap = n == sn;
    if (act) {
      const double Ecz = sE[b][0][q], Erz = sE[b][0][q + 1], Elz = sE[b][0][q - 1];
      const double Ecy = sE[b][1][q], Ery = sE[b][1][q + 1], Ely = sE[b][1][q - 1];
      const Pol2Pair hz = pol2_faces(a, g, Elz, Ecz, Erz, sH[b][0][q - 1], sH[b][0][q]);
      const Pol2Pair hy = pol2_faces(a, g, Ely, Ecy, Ery, sH[b][1][q - 1], sH[b][1][q]);
      double Pz = 0.0, Py = 0.0;
      if (med) {
        double sy, cy, sz, cz;
        pol2_sincm1(thy * Ecy, sy, cy);  // the same angles for both y half steps
        double t0 = x0, t1 = x1;
        x0 = t0 + (cy * t0 + sy * t1);  // exp(U_y E_y dt/2), lane-local
        x1 = t1 + (cy * t1 - sy * t0);
        double u[2 * NJ];  // gather: every lane receives the whole vector
pol2_gather<NJ>(x0, x1, u);
        double w0 = 0.0, w1 = 0.0;  // w = B^T u, components r0, r1
#pragma unroll
        for (int j = 0; j < D; ++j) {
          w0 += bt0[j] * u[j];
          w1 += bt1[j] * u[j];
        }
        pol2_sincm1(thz * Ecz, sz, cz);
        t0 = w0 + (cz * w0 + sz * w1);  // exp(U_z E_z dt)
        t1 = w1 + (cz * w1 - sz * w0);
pol2_gather<NJ>(t0, t1, u);
        w0 = 0.0;  // u = B w
        w1 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          w0 += b0[j] * u[j];
          w1 += b1[j] * u[j];
        }
        x0 = w0 + (cy * w0 + sy * w1);  // exp(U_y E_y dt/2): u = T_y^T d''
        x1 = w1 + (cy * w1 - sy * w0);
        Pz = p0z + quad_sum(wz0 * x0 + wz1 * x1);
        Py = p0y + quad_sum(wy0 * x0 + wy1 * x1);
        if (snap && own && a.pop_out) {
#pragma unroll
          for (int lv = 0; lv < N; ++lv) {
            const double pr = (r0 < D ? sP[lv * D + r0] * x0 : 0.0) + (r1 < D ? sP[lv * D + r1] * x1 : 0.0);
            const double p = sP[N * D + lv] + quad_sum(pr);
            if (lane == 0) a.pop_out[(si * N + lv) * nmed + c] = p;
          }
        }
pol2_gather<NJ>(x0, x1, u);
        w0 = c0;  // the two half steps of this and the next step
        w1 = c1;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          w0 += k0[j] * u[j];
          w1 += k1[j] * u[j];
        }
        x0 = w0;
        x1 = w1;
      }
      const double Ezn = pol2_e(a, g, a.amp_z, n, Ecz, hz, Pz);
      const double Eyn = pol2_e(a, g, a.amp_y, n, Ecy, hy, Py);
      if (lane == 0) {
        sH[b ^ 1][0][q] = hz.Hr;
        sH[b ^ 1][1][q] = hy.Hr;
        sE[b ^ 1][0][q] = Ezn;
        sE[b ^ 1][1][q] = Eyn;
        if (snap && own) {
          if (a.ez_out) a.ez_out[si * nx + g] = Ezn;
          if (a.ey_out) a.ey_out[si * nx + g] = Eyn;
        }
        if (g == nx - 2) {  // first-order Mur boundary at cell nx - 1, both components
          const double Ebz = Ecz + a.kmur * (Ezn - Erz), Eby = Ecy + a.kmur * (Eyn - Ery);
          sE[b ^ 1][0][q + 1] = Ebz;
          sE[b ^ 1][1][q + 1] = Eby;
          if (last) {
            if (a.probe_z) a.probe_z[n + 1] = Ebz;
            if (a.probe_y) a.probe_y[n + 1] = Eby;
            if (snap) {
              if (a.ez_out) a.ez_out[si * nx + nx - 1] = Ebz;
              if (a.ey_out) a.ey_out[si * nx + nx - 1] = Eby;
            }
          }
        }
      }
    }
    __syncthreads();
    b ^= 1;
    if (snap) {
      sn += a.snap_every;
      ++si;
    }
  }
  if (own) {
    if (lane == 0) {
      a.Ezout[g] = sE[b][0][q];
      a.Eyout[g] = sE[b][1][q];
      if (g < nx - 1) {
        a.Hyout[g] = sH[b][0][q];
        a.Gout[g] = sH[b][1][q];
      }
    }
    if (med) {
      if (r0 < D) a.uout[r0 * a.ld + c] = x0;
      if (r1 < D) a.uout[r1 * a.ld + c] = x1;
    }
  }
}

}  // namespace mln
