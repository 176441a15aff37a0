// mln_internal.hpp -- types shared by the host set-up code and the HIP runtime
// of the MLN library.  Not part of the public ABI (see include/mln.h).
#pragma once

#include <complex>
#include <string>
#include <vector>

#include "../../include/mln.h"

namespace mln {

using cplx = std::complex<double>;

// Physical constants, CODATA 2018.
constexpr double kHbar = 1.054571817e-34;
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.25663706212e-6;

// All one-time FP64 quantities of one medium at one time step.
struct Factors {
  int N = 0, D = 0, q = 0;
  std::vector<cplx> gen;                 // D x (N x N) generators
  std::vector<double> M, U, deq, v, d0;  // Eq. elems2, d_eq, Eq. comp_mu, d(rho0)
  std::vector<double> A0, b0;            // exact L1 half step d -> A0 d + b0
  std::vector<double> T, theta;          // T^T U T = blockdiag(theta_i J), J = [[0,1],[-1,0]]
  std::vector<cplx> R, lam;              // route D: U = R diag(lam) R^+
  std::vector<double> S, S2;             // route R: S_i and S_i^2 (q x D x D)
  // full-step quantities (two half steps merged)
  std::vector<double> A, c;              // A = A0^2, c = (A0 + I) b0   (d-coordinates)
  std::vector<double> w;                 // dP/dt = w . d'' + p0        (d-coordinates)
  std::vector<double> K, cz, wz;         // the same in T-coordinates z = T^T d
  double p0 = 0.0;
  std::vector<double> popd, popz, popc;  // rho_aa of d^{n+1/2} = popc_a + pop{d,z}[a,:] . (d''|z'')
  std::vector<double> dprime0, z0;       // state after the first half step of step 0
  // Reference state of the rotation route: the kernels carry y = z' - zr.
  // zr is a fixed point of the field-free step (K zr + cz = zr): the initial
  // state if it is one (then y starts at exactly zero), else the solution of
  // (I - K) zr = cz when that system is regular.  For a fixed point the step's
  // constant term rz and the polarisation offset pr are exactly zero (dP/dt
  // vanishes in a stationary state), so a medium at rest stays exactly at
  // rest.  Without a fixed point zr = 0, rz = cz, pr = p0.
  std::vector<double> zr, rz, y0, popcy;
  double pr = 0.0;
};

// Validates the medium and builds every factor.  Returns an MLN_* code; on
// failure *err holds a message.
int build_factors(const mln_medium *med, double dt, Factors *f, std::string *err);

// Chain rule from d-coordinate gradients (dJ/dA with A = exp(M dt), dJ/dc,
// dJ/dw, dJ/dp0, dJ/dU, dJ/dd'_0) to the physical inputs; fills d_h0,
// d_dipole, d_jump_rate, d_dephasing and d_density of *out (d_amplitude is not
// touched).
int chain_rule(const mln_medium *med, double dt, const double *gA, const double *gc, const double *gw,
               double gp0, const double *gU, const double *gd0, mln_grads *out, std::string *err);

}  // namespace mln
