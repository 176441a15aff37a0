// fwd_kernels.hpp -- argument blocks and launchers of the forward kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mln {

enum { ROUTE_ROT = 0, ROUTE_DIAG = 1, ROUTE_RODR = 2 };

constexpr int kMaxTile = 256;  // threads (= cells) per tile workgroup

// Device copies of the per-medium factors, in the precision of the state.
// Indices are uniform across a wavefront, so the compiler reads them with
// scalar loads.  Layouts are row-major.
template <typename Real>
struct FacDev {
  const Real *Km;     // D x D: K - I (rotation route) or A - I (routes D, R)
  const Real *cz;     // D      inhomogeneous part of the merged L1 step
  const Real *wz;     // D      polarisation weights
  const Real *thdt;   // q      theta_p * dt (rotation and Rodrigues routes)
  const Real *Rre;    // D x D  route D eigenvectors, real part
  const Real *Rim;    // D x D  route D eigenvectors, imaginary part
  const Real *lamdt;  // D      route D: Im(lambda_k) * dt
  const Real *S;      // q x D x D  route R S_p
  const Real *S2;     // q x D x D  route R S_p^2
  Real p0;
  const double *pop;  // N x D  FP64 population map applied to the state after exp(U E dt)
  const double *popc; // N
};

template <typename Real>
struct FwdArgs {
  FacDev<Real> fac;
  const Real *Ein;
  Real *Eout;
  const Real *Hin;
  Real *Hout;
  const Real *zin;
  Real *zout;
  const Real *src;    // amplitude * samples[n], n = 0..nt
  int64_t nx, mb, me, ld;
  int64_t step0;
  int nsteps, halo, owned;
  Real ch, ca, cb, inv_dx, kmur;
  int64_t snap_every;
  double *pop_out, *e_out, *probe_out;
};

template <typename Real>
struct BlochArgs {
  FacDev<Real> fac;
  const Real *z0;
  const double *efield;  // nsteps x ncell
  int64_t ncell, nsteps;
  double *pop_out, *dp_out;
};

template <typename Real>
hipError_t launch_fwd(int N, int route, const FwdArgs<Real> &a, int64_t nblocks, int W, hipStream_t st);
template <typename Real>
hipError_t launch_bloch(int N, int route, const BlochArgs<Real> &a, hipStream_t st);

}  // namespace mln
