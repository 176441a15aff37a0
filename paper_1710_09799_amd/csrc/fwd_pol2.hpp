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
// One launch advances one time step, one thread per cell (the form streamed
// through HBM): E, H, E_y, G and the state are read once and written once.
// The new H on the face left of a cell is formed from the old values with
// the expression its owner uses (bitwise equal), so no thread waits for
// another.  FP64.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mln {

// factor block (doubles): B, K_u, c_u, w_z, w_y (in u-coordinates), the
// rotation angles per unit field theta_y dt/2 and theta_z dt, population
// rows in u-coordinates and their constants, p0_z, p0_y
template <int N>
struct Pol2Layout {
  static constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  static constexpr int oB = 0, oK = D * D, oc = 2 * D * D, owz = oc + D, owy = owz + D;
  static constexpr int othy = owy + D, othz = othy + Q, opop = othz + Q, opopc = opop + N * D;
  static constexpr int op0 = opopc + N, size = op0 + 2;
};

struct Pol2Args {
  const double *fac;
  const double *Ezin, *Hyin, *Eyin, *Gin;
  double *Ezout, *Hyout, *Eyout, *Gout;
  double *u;            // state [D][ld], updated in place (each thread owns its cell)
  const double *src;    // source waveform, nt + 1 samples
  int64_t nx, mb, me, ld, n;  // n: the step taken (fields n -> n + 1)
  double amp_z, amp_y, ch, ca, cb, inv_dx, kmur;
  int snap;
  int64_t snap_i;
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

// the 2x2 rotations of the pairs (2p, 2p+1) by angle th[p] e
template <int D, int Q>
__device__ __forceinline__ void pol2_rotate(double (&x)[D], const double *th, double e) {
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    double s, cm1;
    pol2_sincm1(th[p] * e, s, cm1);
    const double a = x[2 * p], b = x[2 * p + 1];
    x[2 * p] = a + (cm1 * a + s * b);
    x[2 * p + 1] = b + (cm1 * b - s * a);
  }
}

template <int N>
__device__ __forceinline__ void pol2_cell(const Pol2Args &a, const double *F, int64_t g) {
  using L = Pol2Layout<N>;
  constexpr int D = L::D, Q = L::Q;
  const int64_t nx = a.nx;
  // (E_z, H_y): old E of the cell and its neighbours, new H on both faces
  const double Ecz = a.Ezin[g], Erz = a.Ezin[g + 1], Elz = g >= 1 ? a.Ezin[g - 1] : 0.0;
  const double Hrz = a.Hyin[g] + a.ch * (Erz - Ecz);
  const double Hlz = g >= 1 ? a.Hyin[g - 1] + a.ch * (Ecz - Elz) : 0.0;
  // (E_y, G)
  const double Ecy = a.Eyin[g], Ery = a.Eyin[g + 1], Ely = g >= 1 ? a.Eyin[g - 1] : 0.0;
  const double Hry = a.Gin[g] + a.ch * (Ery - Ecy);
  const double Hly = g >= 1 ? a.Gin[g - 1] + a.ch * (Ecy - Ely) : 0.0;
  a.Hyout[g] = Hrz;
  a.Gout[g] = Hry;
  double Pz = 0.0, Py = 0.0;
  if (g >= a.mb && g < a.me) {
    const int64_t c = g - a.mb, nmed = a.me - a.mb;
    double u[D], w[D];
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] = a.u[j * a.ld + c];
    pol2_rotate<D, Q>(u, F + L::othy, Ecy);  // exp(U_y E_y dt/2)
#pragma unroll
    for (int i = 0; i < D; ++i) {  // to z-rotation coordinates: w = B^T u
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) s += F[L::oB + j * D + i] * u[j];
      w[i] = s;
    }
    pol2_rotate<D, Q>(w, F + L::othz, Ecz);  // exp(U_z E_z dt)
#pragma unroll
    for (int i = 0; i < D; ++i) {  // back: u = B w
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) s += F[L::oB + i * D + j] * w[j];
      u[i] = s;
    }
    pol2_rotate<D, Q>(u, F + L::othy, Ecy);  // exp(U_y E_y dt/2): u = T_y^T d''
    Pz = F[L::op0];
    Py = F[L::op0 + 1];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      Pz += F[L::owz + j] * u[j];
      Py += F[L::owy + j] * u[j];
    }
    if (a.snap && a.pop_out) {
#pragma unroll
      for (int lv = 0; lv < N; ++lv) {
        double p = F[L::opopc + lv];
#pragma unroll
        for (int j = 0; j < D; ++j) p += F[L::opop + lv * D + j] * u[j];
        a.pop_out[(a.snap_i * N + lv) * nmed + c] = p;
      }
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {  // the two half steps of this and the next step
      double s = F[L::oc + i];
#pragma unroll
      for (int j = 0; j < D; ++j) s += F[L::oK + i * D + j] * u[j];
      w[i] = s;
    }
#pragma unroll
    for (int j = 0; j < D; ++j) a.u[j * a.ld + c] = w[j];
  }
  double Ezn, Eyn;
  if (g == 0) {  // hard sources
    Ezn = a.amp_z * a.src[a.n + 1];
    Eyn = a.amp_y * a.src[a.n + 1];
  } else {
    Ezn = a.ca * Ecz + a.cb * (-Pz + (Hrz - Hlz) * a.inv_dx);
    Eyn = a.ca * Ecy + a.cb * (-Py + (Hry - Hly) * a.inv_dx);
  }
  a.Ezout[g] = Ezn;
  a.Eyout[g] = Eyn;
  if (a.snap) {
    if (a.ez_out) a.ez_out[a.snap_i * nx + g] = Ezn;
    if (a.ey_out) a.ey_out[a.snap_i * nx + g] = Eyn;
  }
  if (g == nx - 2) {  // first-order Mur boundary at cell nx - 1, both components
    const double Ebz = Ecz + a.kmur * (Ezn - Erz), Eby = Ecy + a.kmur * (Eyn - Ery);
    a.Ezout[nx - 1] = Ebz;
    a.Eyout[nx - 1] = Eby;
    if (a.probe_z) a.probe_z[a.n + 1] = Ebz;
    if (a.probe_y) a.probe_y[a.n + 1] = Eby;
    if (a.snap) {
      if (a.ez_out) a.ez_out[a.snap_i * nx + nx - 1] = Ebz;
      if (a.ey_out) a.ey_out[a.snap_i * nx + nx - 1] = Eby;
    }
  }
}

template <int N>
__global__ void __launch_bounds__(256) fwd_pol2_kernel(Pol2Args a) {
  using L = Pol2Layout<N>;
  // the factor block in LDS (every lane reads the same element: broadcast);
  // read near its use instead of being held in registers across the step
  __shared__ double sF[L::size];
  for (int i = threadIdx.x; i < L::size; i += blockDim.x) sF[i] = a.fac[i];
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < a.nx - 1) pol2_cell<N>(a, sF, g);  // cell nx - 1 (Mur) is written by the thread of nx - 2
}

}  // namespace mln
