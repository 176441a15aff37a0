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

// Factor reads go through the constant address space: the factor block is
// never written by a kernel, and wave-uniform constant loads become scalar
// (SMEM) loads whose results live in SGPRs, instead of per-lane vector loads
// re-issued every step.
template <typename T>
__device__ __forceinline__ T cld(const T *p, int i) {
  return ((const __attribute__((address_space(4))) T *)p)[i];
}

// Workgroup barrier for kernels whose threads communicate only through LDS
// within a launch: it waits for this wavefront's LDS operations (so its LDS
// writes are visible after the barrier) but not for its global-memory loads
// and stores, which stay in flight across the barrier (__syncthreads waits for
// those as well).  The memory clobber keeps the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void lds_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// sin(x) and cos(x) - 1.  For |x| <= 1/2 (every cell-step of any practical
// field: the per-step rotation angles are ~1e-3 .. 1e-2) the Taylor series of
// sine and of cos - 1 are summed to the last bit of the type, which also avoids
// the cancellation 1 - cos(x) suffers: a short series when every angle of the
// wavefront is below 1/16, a longer one (Estrin form) up to 1/2.  Beyond that
// the whole wavefront takes the device math library path instead (each test is
// wave-uniform, so the common path has no divergence).
__device__ __forceinline__ bool wave_any(bool p) { return __any(p); }

__device__ __forceinline__ void sincm1(double x, double &s, double &cm1) {
  if (__builtin_expect(!wave_any(fabs(x) > 0.0625), 1)) {
    // |x| <= 1/16: terms through x^9 (sine) and x^10 (cos - 1) leave a
    // truncation below 1e-19 relative
    const double x2 = x * x, x4 = x2 * x2;
    const double s0 = fma(x2, -1.0 / 6.0, 1.0);
    const double s1 = fma(x4, 1.0 / 362880.0, fma(x2, -1.0 / 5040.0, 1.0 / 120.0));
    s = x * fma(x4, s1, s0);
    const double c0 = fma(x2, 1.0 / 24.0, -0.5);
    const double c1 = fma(x4, -1.0 / 3628800.0, fma(x2, 1.0 / 40320.0, -1.0 / 720.0));
    cm1 = x2 * fma(x4, c1, c0);
  } else if (!wave_any(fabs(x) > 0.5)) {
    const double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
    // sin x = x (1 - x^2/3! + x^4/5! - ... - x^14/15! + x^16/17!)
    const double s0 = fma(x2, -1.0 / 6.0, 1.0);
    const double s1 = fma(x2, -1.0 / 5040.0, 1.0 / 120.0);
    const double s2 = fma(x2, -1.0 / 39916800.0, 1.0 / 362880.0);
    const double s3 = fma(x2, -1.0 / 1307674368000.0, 1.0 / 6227020800.0);
    const double s4 = 1.0 / 355687428096000.0;
    const double sa = fma(x4, s1, s0), sb = fma(x4, s3, s2);
    s = x * fma(x8, fma(x8, s4, sb), sa);
    // cos x - 1 = x^2 (-1/2! + x^2/4! - ... + x^16/18!)
    const double c0 = fma(x2, 1.0 / 24.0, -0.5);
    const double c1 = fma(x2, 1.0 / 40320.0, -1.0 / 720.0);
    const double c2 = fma(x2, 1.0 / 479001600.0, -1.0 / 3628800.0);
    const double c3 = fma(x2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);
    const double c4 = -1.0 / 6402373705728000.0;
    const double ca = fma(x4, c1, c0), cb = fma(x4, c3, c2);
    cm1 = x2 * fma(x8, fma(x8, c4, cb), ca);
  } else {
    const double h = sin(0.5 * x);
    s = sin(x);
    cm1 = -2.0 * h * h;
  }
}

__device__ __forceinline__ void sincm1(float x, float &s, float &cm1) {
  if (__builtin_expect(!wave_any(fabsf(x) > 0.0625f), 1)) {
    // |x| <= 1/16: sin x = x + x^3 (-1/3! + x^2/5!), cos x - 1 =
    // x^2 (-1/2 + x^2 (1/4! - x^2/6!)); truncation below 1e-11 relative
    const float x2 = x * x;
    s = fmaf(x * x2, fmaf(x2, 1.0f / 120.0f, -1.0f / 6.0f), x);
    cm1 = x2 * fmaf(x2, fmaf(x2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f);
  } else if (!wave_any(fabsf(x) > 0.5f)) {
    const float x2 = x * x, x4 = x2 * x2;
    // sin x = x (1 - x^2/3! + x^4/5! - x^6/7! + x^8/9!)
    const float sa = fmaf(x2, -1.0f / 6.0f, 1.0f), sb = fmaf(x2, -1.0f / 5040.0f, 1.0f / 120.0f);
    s = x * fmaf(x4, fmaf(x4, 1.0f / 362880.0f, sb), sa);
    // cos x - 1 = x^2 (-1/2 + x^2/4! - x^4/6! + x^6/8! - x^8/10!)
    const float ca = fmaf(x2, 1.0f / 24.0f, -0.5f), cb = fmaf(x2, 1.0f / 40320.0f, -1.0f / 720.0f);
    cm1 = x2 * fmaf(x4, fmaf(x4, -1.0f / 3628800.0f, cb), ca);
  } else {
    const float h = sinf(0.5f * x);
    s = sinf(x);
    cm1 = -2.0f * h * h;
  }
}

// The same with the device-library path (|x| > 1/2 somewhere in the
// wavefront) kept out of line: kernels whose register budget is tight do not
// carry that path's registers through their step loop.
// (returns (sin x, cos x - 1) by value: results in registers, no stack frame)
__device__ __noinline__ float2 sincm1_library(float x) {
  const float h = sinf(0.5f * x);
  return make_float2(sinf(x), -2.0f * h * h);
}

__device__ __forceinline__ void sincm1_lean(float x, float &s, float &cm1) {
  if (!wave_any(fabsf(x) > 0.0625f)) {
    const float x2 = x * x;
    s = fmaf(x * x2, fmaf(x2, 1.0f / 120.0f, -1.0f / 6.0f), x);
    cm1 = x2 * fmaf(x2, fmaf(x2, -1.0f / 720.0f, 1.0f / 24.0f), -0.5f);
  } else if (!wave_any(fabsf(x) > 0.5f)) {
    const float x2 = x * x, x4 = x2 * x2;
    const float sa = fmaf(x2, -1.0f / 6.0f, 1.0f), sb = fmaf(x2, -1.0f / 5040.0f, 1.0f / 120.0f);
    s = x * fmaf(x4, fmaf(x4, 1.0f / 362880.0f, sb), sa);
    const float ca = fmaf(x2, 1.0f / 24.0f, -0.5f), cb = fmaf(x2, 1.0f / 40320.0f, -1.0f / 720.0f);
    cm1 = x2 * fmaf(x4, fmaf(x4, -1.0f / 3628800.0f, cb), ca);
  } else {
    const float2 r = sincm1_library(x);
    s = r.x;
    cm1 = r.y;
  }
}

// Two-float arithmetic for the compensated state (Knuth's two-sum, Dekker's
// fast two-sum): hi + lo carries about 48 significant bits.
__device__ __forceinline__ void add_comp(float &hi, float &lo, float d) {
  const float s = hi + d;
  const float bb = s - hi;
  const float e = (hi - (s - bb)) + (d - bb);
  const float l2 = lo + e;
  const float h2 = s + l2;
  lo = l2 - (h2 - s);
  hi = h2;
}

// Rotation-route factors staged in LDS once per launch.  Layout (offsets in
// elements of Real): K - I (D*D), constant term (D), polarisation weights (D),
// theta*dt (Q), reference state (D), and for the compensated state the low
// parts of K - I (D*D), of the constant term (D) and of theta*dt (Q).
template <int N, typename Real, bool COMP>
struct RotLds {
  static constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  static constexpr int oK = 0, oc = D * D, ow = oc + D, oth = ow + D, ozr = oth + Q;
  static constexpr int oKl = ozr + D, ocl = oKl + (COMP ? D * D : 0), otl = ocl + (COMP ? D : 0);
  static constexpr int size = otl + (COMP ? Q : 0);
  // FP64 population map (N x D) and offsets (N), used on recording steps only
  static __device__ void stage_pop(const FacDev<Real> &f, double *sP) {
    for (int i = threadIdx.x; i < N * D; i += blockDim.x) sP[i] = cld(f.pop, i);
    for (int i = threadIdx.x; i < N; i += blockDim.x) sP[N * D + i] = cld(f.popc, i);
  }
  static __device__ void stage(const FacDev<Real> &f, Real *sF) {
    for (int i = threadIdx.x; i < D * D; i += blockDim.x) {
      sF[oK + i] = cld(f.Km, i);
      if constexpr (COMP) sF[oKl + i] = cld(f.Km_lo, i);
    }
    for (int i = threadIdx.x; i < D; i += blockDim.x) {
      sF[oc + i] = cld(f.cz, i);
      sF[ow + i] = cld(f.wz, i);
      sF[ozr + i] = cld(f.zr, i);
      if constexpr (COMP) sF[ocl + i] = cld(f.cz_lo, i);
    }
    for (int i = threadIdx.x; i < Q; i += blockDim.x) {
      sF[oth + i] = cld(f.thdt, i);
      if constexpr (COMP) sF[otl + i] = cld(f.th_lo, i);
    }
  }
};

// Factor access of the rotation route: from LDS (small D, where the
// compiler keeps them in registers) or through scalar loads (large D, where a
// per-FMA LDS read would make the step LDS-bound).
template <int N, typename Real, bool COMP>
struct LdsAcc {
  using L = RotLds<N, Real, COMP>;
  const Real *sF;
  __device__ Real K(int i) const { return sF[L::oK + i]; }
  __device__ Real Kl(int i) const { return sF[L::oKl + i]; }
  __device__ Real c(int i) const { return sF[L::oc + i]; }
  __device__ Real cl(int i) const { return sF[L::ocl + i]; }
  __device__ Real w(int i) const { return sF[L::ow + i]; }
  __device__ Real th(int i) const { return sF[L::oth + i]; }
  __device__ Real thl(int i) const { return sF[L::otl + i]; }
  __device__ Real zr(int i) const { return sF[L::ozr + i]; }
};
template <typename Real>
struct SmemAcc {
  const FacDev<Real> *f;
  int64_t o;  // loop-variant zero offset
  __device__ Real K(int i) const { return cld(f->Km + o, i); }
  __device__ Real Kl(int i) const { return cld(f->Km_lo + o, i); }
  __device__ Real c(int i) const { return cld(f->cz + o, i); }
  __device__ Real cl(int i) const { return cld(f->cz_lo + o, i); }
  __device__ Real w(int i) const { return cld(f->wz + o, i); }
  __device__ Real th(int i) const { return cld(f->thdt + o, i); }
  __device__ Real thl(int i) const { return cld(f->th_lo + o, i); }
  __device__ Real zr(int i) const { return cld(f->zr + o, i); }
};

// Rotation route, one cell: y'' = Rot(y) + (Rot - I) zr (the state is
// y = z' - zr), dP/dt = w.y'' + p, y_next = y'' + (K - I) y'' + r.
template <int N, typename Real, class Acc>
__device__ __forceinline__ Real rot_cell(const Acc &F, Real p0, Real E, Real (&z)[N * N - 1],
                                         const double *sP, double *pout, int64_t stride) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    Real s, cm1;
    sincm1(F.th(p) * E, s, cm1);
    const Real a = z[2 * p], b = z[2 * p + 1];
    const Real ar = F.zr(2 * p), br = F.zr(2 * p + 1);
    z[2 * p] = a + ((cm1 * a + s * b) + (cm1 * ar + s * br));
    z[2 * p + 1] = b + ((cm1 * b - s * a) + (cm1 * br - s * ar));
  }
  if (pout) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double acc = sP[N * D + a];
#pragma unroll
      for (int j = 0; j < D; ++j) acc += sP[a * D + j] * (double)z[j];
      pout[a * stride] = acc;
    }
  }
  Real P = p0;
#pragma unroll
  for (int j = 0; j < D; ++j) P += F.w(j) * z[j];
  Real nz[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Real acc = F.c(i);
#pragma unroll
    for (int j = 0; j < D; ++j) acc += F.K(i * D + j) * z[j];
    nz[i] = z[i] + acc;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) z[i] = nz[i];
  return P;
}

// Compensated rotation-route cell step.  The increments (cos - 1) y + sin y'
// and (K - I) y'' are formed from the high parts (the low parts would change
// them by ~1e-9 of themselves, with a sign that varies from step to step) and
// added to hi + lo exactly; K - I, the constant term and theta*dt are float
// pairs, and two accumulators keep the low-part products from being absorbed
// by the high-part sum.
template <int N, class Acc>
__device__ __forceinline__ float rot_cell_comp(const Acc &F, float p0, float E, float (&z)[N * N - 1],
                                               float (&zl)[N * N - 1], const double *sP, double *pout,
                                               int64_t stride) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    float s, cm1;
    sincm1(fmaf(F.th(p), E, F.thl(p) * E), s, cm1);
    const float a = z[2 * p], b = z[2 * p + 1];
    const float ar = F.zr(2 * p), br = F.zr(2 * p + 1);
    add_comp(z[2 * p], zl[2 * p], (cm1 * a + s * b) + (cm1 * ar + s * br));
    add_comp(z[2 * p + 1], zl[2 * p + 1], (cm1 * b - s * a) + (cm1 * br - s * ar));
  }
  if (pout) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
      double acc = sP[N * D + a];
#pragma unroll
      for (int j = 0; j < D; ++j) acc += sP[a * D + j] * ((double)z[j] + (double)zl[j]);
      pout[a * stride] = acc;
    }
  }
  float P = p0;
#pragma unroll
  for (int j = 0; j < D; ++j) P += F.w(j) * z[j];
  float dl[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    float ah = F.c(i), al = F.cl(i);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      ah = fmaf(F.K(i * D + j), z[j], ah);
      al = fmaf(F.Kl(i * D + j), z[j], al);
    }
    dl[i] = ah + al;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) add_comp(z[i], zl[i], dl[i]);
  return P;
}

// d'' = exp(U E dt) d' for one cell, in place.  z holds T-coordinates for the
// rotation route and d-coordinates for routes D and R.
template <int N, typename Real, int ROUTE>
__device__ __forceinline__ void interaction(const FacDev<Real> &f, Real E, Real (&z)[N * N - 1]) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  if constexpr (ROUTE == ROUTE_ROT) {
    // T^T U T = blockdiag(theta_p J): each (u_ab, v_ab) pair turns by
    // theta_p E dt; the N-1 population directions are left alone.
    // The state is y = z' - zr; Rot(y + zr) - zr = Rot(y) + (Rot - I) zr.
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      Real s, cm1;
      sincm1(cld(f.thdt, p) * E, s, cm1);
      const Real a = z[2 * p], b = z[2 * p + 1];
      const Real ar = cld(f.zr, 2 * p), br = cld(f.zr, 2 * p + 1);
      z[2 * p] = a + ((cm1 * a + s * b) + (cm1 * ar + s * br));
      z[2 * p + 1] = b + ((cm1 * b - s * a) + (cm1 * br - s * ar));
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
        ar += cld(f.Rre, i * D + k) * z[i];
        ai -= cld(f.Rim, i * D + k) * z[i];
      }
      Real s, cm1;
      sincm1(cld(f.lamdt, k) * E, s, cm1);
      yr[k] = ar + (cm1 * ar - s * ai);
      yi[k] = ai + (cm1 * ai + s * ar);
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      Real acc = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) acc += cld(f.Rre, i * D + k) * yr[k] - cld(f.Rim, i * D + k) * yi[k];
      z[i] = acc;
    }
  } else if constexpr (ROUTE == ROUTE_PADE) {
    // The generic per-step route the paper measures the other two against:
    // exp(X), X = E dt U = x V (x = E ||dt U||_1, ||V||_1 = 1), by the
    // diagonal Pade approximant r_m(X) = q_m(X)^-1 p_m(X) with scaling
    // (Higham 2005: the degree m in {3, 5, 7} and the scaling 2^s from
    // ||X||_1 = |x|), applied to the state: p_m(X) d from m products with V,
    // q_m(X) = sum (-1)^k b_k x^k V^k formed from the precomputed powers V^k,
    // and q_m(X) f = p_m(X) d solved by Gaussian elimination (q_m(X) = b_0 I +
    // O(||X||), no pivoting needed).
    const Real xs = E * f.unorm;
    const Real xn = xs < 0 ? -xs : xs;
    int m = 7;
    if (!wave_any(xn > Real(1.495585217958292e-2)))
      m = 3;
    else if (!wave_any(xn > Real(2.539398330063230e-1)))
      m = 5;
    int sc = 0;  // scaling exponent of this lane
    if (m == 7)
      while (sc < 60 && xn > Real(9.504178996162932e-1) * (Real)(1ull << sc)) ++sc;
    const Real x = xs / (Real)(1ull << sc);
    double b[kPadeMax + 1];
    if (m == 3) {
      b[0] = 120; b[1] = 60; b[2] = 12; b[3] = 1;
    } else if (m == 5) {
      b[0] = 30240; b[1] = 15120; b[2] = 3360; b[3] = 420; b[4] = 30; b[5] = 1;
    } else {
      b[0] = 17297280; b[1] = 8648640; b[2] = 1995840; b[3] = 277200;
      b[4] = 25200; b[5] = 1512; b[6] = 56; b[7] = 1;
    }
#pragma unroll 1
    for (int rep = 0; rep < (1 << sc); ++rep) {
      Real Qm[D][D], pd[D], v[D];
#pragma unroll
      for (int i = 0; i < D; ++i) {
        v[i] = z[i];
        pd[i] = (Real)b[0] * z[i];
#pragma unroll
        for (int j = 0; j < D; ++j) Qm[i][j] = (i == j) ? (Real)b[0] : Real(0);
      }
      Real xk = 1;
#pragma unroll 1
      for (int k = 1; k <= m; ++k) {
        xk *= x;
        const Real cp = (Real)b[k] * xk, cq = (k & 1) ? -cp : cp;
        const Real *Uk = f.Up + (k - 1) * D * D;
        Real nv[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          Real acc = 0;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            acc += cld(f.Up, i * D + j) * v[j];
            Qm[i][j] += cq * cld(Uk, i * D + j);
          }
          nv[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
          v[i] = nv[i];
          pd[i] += cp * nv[i];
        }
      }
      // forward elimination and back substitution
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const Real inv = Real(1) / Qm[c][c];
#pragma unroll
        for (int i = c + 1; i < D; ++i) {
          const Real l = Qm[i][c] * inv;
#pragma unroll
          for (int j = c + 1; j < D; ++j) Qm[i][j] -= l * Qm[c][j];
          pd[i] -= l * pd[c];
        }
      }
#pragma unroll
      for (int i = D - 1; i >= 0; --i) {
        Real acc = pd[i];
#pragma unroll
        for (int j = i + 1; j < D; ++j) acc -= Qm[i][j] * z[j];
        z[i] = acc / Qm[i][i];
      }
    }
  } else {
    // generalised Rodrigues: A_I = I + sum_p sin(x_p) S_p + (1 - cos(x_p)) S_p^2
    Real out[D];
#pragma unroll
    for (int i = 0; i < D; ++i) out[i] = z[i];
#pragma unroll 1
    for (int p = 0; p < Q; ++p) {
      Real s, cm1;
      sincm1(cld(f.thdt, p) * E, s, cm1);
      const Real *Sp = f.S + p * D * D, *S2p = f.S2 + p * D * D;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        Real a = 0, b = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          a += cld(Sp, i * D + j) * z[j];
          b += cld(S2p, i * D + j) * z[j];
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
  for (int j = 0; j < D; ++j) P += cld(f.wz, j) * z[j];
  Real nz[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    Real acc = cld(f.cz, i);
#pragma unroll
    for (int j = 0; j < D; ++j) acc += cld(f.Km, i * D + j) * z[j];
    nz[i] = z[i] + acc;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) z[i] = nz[i];
  return P;
}

template <int N, typename Real, bool COMP>
__device__ __forceinline__ void record_pop(const FacDev<Real> &f, const Real (&z)[N * N - 1],
                                           const Real (&zl)[COMP ? N * N - 1 : 1], double *pop,
                                           int64_t stride) {
  constexpr int D = N * N - 1;
#pragma unroll
  for (int a = 0; a < N; ++a) {
    double acc = cld(f.popc, a);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double zj = (double)z[j];
      if constexpr (COMP) zj += (double)zl[j];
      acc += cld(f.pop, a * D + j) * zj;
    }
    pop[a * stride] = acc;
  }
}

// one Liouville cell step: exp(U E dt), optional population record, merged L1
// factors of the rotation route through scalar loads when D > 8
template <int N>
constexpr bool rot_smem() { return N * N - 1 > 8; }

template <int N, typename Real, int ROUTE, bool COMP>
__device__ __forceinline__ Real cell_step(const FacDev<Real> &f, const Real *sF, const double *sP, Real E,
                                          Real (&z)[N * N - 1],
                                          Real (&zl)[COMP ? N * N - 1 : 1], double *pop,
                                          int64_t stride, int64_t zoff) {
  if constexpr (COMP || ROUTE == ROUTE_ROT) {
    if constexpr (rot_smem<N>()) {
      SmemAcc<Real> F{&f, zoff};
      if constexpr (COMP)
        return rot_cell_comp<N>(F, f.p0, E, z, zl, sP, pop, stride);
      else
        return rot_cell<N, Real>(F, f.p0, E, z, sP, pop, stride);
    } else {
      LdsAcc<N, Real, COMP> F{sF};
      if constexpr (COMP)
        return rot_cell_comp<N>(F, f.p0, E, z, zl, sP, pop, stride);
      else
        return rot_cell<N, Real>(F, f.p0, E, z, sP, pop, stride);
    }
  } else {
    interaction<N, Real, ROUTE>(f, E, z);
    if (pop) record_pop<N, Real, COMP>(f, z, zl, pop, stride);
    return shared_factor<N, Real>(f, z);
  }
}

// One tile (one cell per thread, W = blockDim.x cells) of the forward step.
// COMP: compensated (float-float) state; CF: E and H as float-float pairs too.
template <int N, typename Real, int ROUTE, bool COMP, bool CF>
__device__ __forceinline__ void block_tile(const FwdArgs<Real> &a, int64_t tile) {
  constexpr int D = N * N - 1;
  constexpr int DL = COMP ? D : 1;
  constexpr int FL = CF ? kMaxTile : 1;  // low parts of the exchanged fields
  __shared__ Real sE[kMaxTile], sEl[FL];
  __shared__ Real sH[kMaxTile], sHl[FL];
  __shared__ Real sSrc[kMaxStepsPerLaunch], sSrcl[CF ? kMaxStepsPerLaunch : 1];
  __shared__ Real sMur, sMurl;
  __shared__ Real sF[ROUTE == ROUTE_ROT ? RotLds<N, Real, COMP>::size : 1];
  __shared__ double sP[ROUTE == ROUTE_ROT ? N * (N * N - 1) + N : 1];
  if constexpr (ROUTE == ROUTE_ROT) {
    RotLds<N, Real, COMP>::stage(a.fac, sF);
    RotLds<N, Real, COMP>::stage_pop(a.fac, sP);
  }
  const int lid = threadIdx.x;
  const int W = blockDim.x;
  const int64_t base = tile * a.owned - a.halo;
  const int64_t g = base + lid;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool tile_med = (base < a.me) && (base + W > a.mb);
  const bool has_right = (base <= a.nx - 1) && (base + W > a.nx - 1);
  const bool owned = in_dom && lid >= a.halo && lid < a.halo + a.owned;
  const int64_t c = g - a.mb;

  Real E = 0, H = 0, Elo = 0, Hlo = 0;
  Real z[D], zl[DL];
  if (in_dom) {
    E = a.Ein[g];
    if (g < a.nx - 1) H = a.Hin[g];
    if constexpr (CF) {
      Elo = a.Ein[a.nx + g];
      if (g < a.nx - 1) Hlo = a.Hin[a.nx + g];
    }
  }
#pragma unroll
  for (int j = 0; j < D; ++j) z[j] = is_med ? a.zin[j * a.ld + c] : Real(0);
#pragma unroll
  for (int j = 0; j < DL; ++j) zl[j] = (COMP && is_med) ? a.zin[(D + j) * a.ld + c] : Real(0);

  // source samples of this launch (read by the tile holding cell 0)
  for (int i = threadIdx.x; i < a.nsteps; i += blockDim.x) {
    sSrc[i] = a.src[a.step0 + 1 + i];
    if constexpr (CF) sSrcl[i] = a.src[a.nt + 1 + a.step0 + 1 + i];
  }
  __syncthreads();
  int64_t snap_next = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = n == snap_next;
    sE[lid] = E;
    if constexpr (CF) sEl[lid] = Elo;
    __syncthreads();
    const Real Er = (lid + 1 < W) ? sE[lid + 1] : Real(0);
    const Real El = (lid > 0) ? sE[lid - 1] : Real(0);
    Real Erl = 0, Ell = 0;
    if constexpr (CF) {
      Erl = (lid + 1 < W) ? sEl[lid + 1] : Real(0);
      Ell = (lid > 0) ? sEl[lid - 1] : Real(0);
    }
    if (in_dom && g < a.nx - 1) {
      if constexpr (CF)
        add_comp(H, Hlo, a.ch * ((Er - E) + (Erl - Elo)));
      else
        H += a.ch * (Er - E);
    }
    Real P = 0;
    if (a.tape && owned && is_med && n >= a.tape_step0) {
      Real *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
#pragma unroll
      for (int j = 0; j < D; ++j) tp[j * a.ld] = z[j];
      tp[D * a.ld] = E;
    }
    if (tile_med && is_med) {
      double *pp = (snap && owned && a.pop_out) ? a.pop_out + si * N * (a.me - a.mb) + c : nullptr;
      P = cell_step<N, Real, ROUTE, COMP>(a.fac, sF, sP, E, z, zl, pp, a.me - a.mb, a.opaque0 * s);
    }
    sH[lid] = H;
    if constexpr (CF) sHl[lid] = Hlo;
    __syncthreads();
    const Real Hl = (lid > 0) ? sH[lid - 1] : Real(0);
    const Real Eold = E, Eoldl = Elo;
    if (g >= 1 && g < a.nx - 1) {
      if constexpr (CF) {
        const Real Hll = (lid > 0) ? sHl[lid - 1] : Real(0);
        add_comp(E, Elo, a.cam1 * E + a.cb * (-P + ((H - Hl) + (Hlo - Hll)) * a.inv_dx));
      } else {
        E = a.ca * E + a.cb * (-P + (H - Hl) * a.inv_dx);
      }
    } else if (g == 0) {
      E = sSrc[s];
      if constexpr (CF) Elo = sSrcl[s];
    }
    if (has_right) {  // first-order Mur boundary at cell nx-1
      if (g == a.nx - 2) {
        sMur = E;
        sMurl = Elo;
      }
      __syncthreads();
      if (g == a.nx - 1) {
        if constexpr (CF) {
          E = El;
          Elo = Ell;
          add_comp(E, Elo, a.kmur * ((sMur - Eold) + (sMurl - Eoldl)));
        } else {
          E = El + a.kmur * (sMur - Eold);
        }
        if (a.probe_out) a.probe_out[n + 1] = (double)E + (double)Elo;
      }
    }
    if (snap) {
      if (owned && a.e_out) a.e_out[si * a.nx + g] = (double)E + (double)Elo;
      snap_next += a.snap_every;
      ++si;
    }
  }
  if (owned) {
    a.Eout[g] = E;
    if (g < a.nx - 1) a.Hout[g] = H;
    if constexpr (CF) {
      a.Eout[a.nx + g] = Elo;
      if (g < a.nx - 1) a.Hout[a.nx + g] = Hlo;
    }
    if (is_med) {
#pragma unroll
      for (int j = 0; j < D; ++j) a.zout[j * a.ld + c] = z[j];
      if constexpr (COMP) {
#pragma unroll
        for (int j = 0; j < D; ++j) a.zout[(D + j) * a.ld + c] = zl[j];
      }
    }
  }
}

template <int N, typename Real, int ROUTE, bool COMP, bool CF = false>
__global__ void __launch_bounds__(kMaxTile) fwd_tile_kernel(FwdArgs<Real> a) {
  block_tile<N, Real, ROUTE, COMP, CF>(a, blockIdx.x);
}

// The rotation route compiled for seven wavefronts per SIMD, for launches of
// many tiles (many_tiles).  Measured with tile 256 and 16 steps per launch,
// cell-updates/s against the default build: two-level 2^24 cells FP64
// 1.95e11 / 1.71e11, compensated FP32 2.04e11 / 1.90e11; three-level 2^20
// cells FP64 9.69e10 / 9.24e10; but three-level 20000 cells (90 tiles) FP64
// 1.14e10 / 1.28e10, compensated FP32 7.2e9 / 1.10e10.  The budget spills
// 0-132 B per lane.
template <int N, typename Real, bool COMP, bool CF = false>
__global__ void __launch_bounds__(kMaxTile) __attribute__((amdgpu_waves_per_eu(7, 8)))
fwd_tile_kernel_many(FwdArgs<Real> a) {
  block_tile<N, Real, ROUTE_ROT, COMP, CF>(a, blockIdx.x);
}

// Prescribed-field mode: one thread per medium cell, no FDTD.
template <int N, typename Real, int ROUTE, bool COMP>
__global__ void __launch_bounds__(256) bloch_kernel(BlochArgs<Real> a) {
  constexpr int D = N * N - 1;
  constexpr int DL = COMP ? D : 1;
  __shared__ Real sF[ROUTE == ROUTE_ROT ? RotLds<N, Real, COMP>::size : 1];
  __shared__ double sP[ROUTE == ROUTE_ROT ? N * (N * N - 1) + N : 1];
  if constexpr (ROUTE == ROUTE_ROT) {
    RotLds<N, Real, COMP>::stage(a.fac, sF);
    RotLds<N, Real, COMP>::stage_pop(a.fac, sP);
  }
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncell) return;
  Real z[D], zl[DL];
#pragma unroll
  for (int j = 0; j < D; ++j) z[j] = a.z0[j];
#pragma unroll
  for (int j = 0; j < DL; ++j) zl[j] = COMP ? a.z0[D + j] : Real(0);
  for (int64_t t = 0; t < a.nsteps; ++t) {
    const Real E = (Real)a.efield[t * a.ncell + c];
    double *pp = a.pop_out ? a.pop_out + t * N * a.ncell + c : nullptr;
    const Real P = cell_step<N, Real, ROUTE, COMP>(a.fac, sF, sP, E, z, zl, pp, a.ncell, a.opaque0 * t);
    if (a.dp_out) a.dp_out[t * a.ncell + c] = (double)P;
  }
}

// ---------------------------------------------------------------------------
// Reverse-time (adjoint) tile kernel: the exact transpose of one forward
// time step of the rotation route, applied for steps n_hi-1 .. n_hi-nsteps.
// Forward step n (Sec. 4.1 update rules, Fig. 1):
//   H_i += ch (E_{i+1} - E_i);  z'' = Rot(theta dt E_i) z';  P = w.z'' + p0;
//   z'_next = K z'' + c;  E_i <- ca E_i + cb (-P + (H_i - H_{i-1})/dx);
//   E_0 <- amplitude s[n+1];  E_{nx-1} <- E_{nx-2} + kmur (E'_{nx-2} - E_{nx-1}).
// The reverse sweep carries lE = dJ/dE, lH = dJ/dH, lz = dJ/dz' per cell and
// accumulates, for owned cells only, dJ/dK = sum lz' z''^T, dJ/dc, dJ/dw,
// dJ/dp0, dJ/damplitude, and the moments sum E^m lhat zhat^T with
// lhat = Rot(-x/2) lz'', zhat = Rot(x/2) z', from which the host forms dJ/dU.
template <int N, typename Real>
__global__ void __launch_bounds__(kMaxTile) adj_tile_kernel(AdjArgs<Real> a) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  constexpr bool F64 = sizeof(Real) == 8;
  constexpr int NM = adj_moments(F64);
  constexpr int NACC = adj_nacc(N, F64);
  __shared__ Real sE[kMaxTile];
  __shared__ Real sH[kMaxTile];
  __shared__ double sRed[kMaxTile / 64][NACC];
  using LF = RotLds<N, Real, false>;
  __shared__ Real sF[LF::size];
  LF::stage(a.fac, sF);
  const int lid = threadIdx.x;
  const int W = blockDim.x;
  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const int64_t g = base + lid;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool owned = in_dom && lid >= a.halo && lid < a.halo + a.owned;
  const int64_t c = g - a.mb;
  const Real cbdx = a.cb * a.inv_dx;

  Real lE = 0, lH = 0, lz[D];
  if (in_dom) {
    lE = a.lEin[g];
    if (g < a.nx - 1) lH = a.lHin[g];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) lz[j] = is_med ? a.lzin[j * a.ld + c] : Real(0);
  Real aK[D * D], aM[NM][D * D], ac[D], aw[D], ap0 = 0, aamp = 0;
#pragma unroll
  for (int i = 0; i < D * D; ++i) {
    aK[i] = 0;
#pragma unroll
    for (int m = 0; m < NM; ++m) aM[m][i] = 0;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) { ac[i] = 0; aw[i] = 0; }
  // objective weights and source samples of this launch, staged in LDS
  __shared__ double sG[kMaxStepsPerLaunch], sS[kMaxStepsPerLaunch];
  for (int i = threadIdx.x; i < a.nsteps; i += blockDim.x) {
    sG[i] = a.gprobe[a.n_hi - i];
    sS[i] = a.samples[a.n_hi - i];
  }
  __syncthreads();
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.n_hi - 1 - s;
    if (g == a.nx - 1) lE += (Real)sG[s];
    sE[lid] = lE;
    __syncthreads();
    const Real lEr = (lid + 1 < W) ? sE[lid + 1] : Real(0);
    const Real lErr = (lid + 2 < W) ? sE[lid + 2] : Real(0);
    // the Mur update also reads E^{n+1}_{nx-2}
    Real lEe = lE, lEre = lEr;
    if (g == a.nx - 2) lEe += a.kmur * lEr;
    if (g == a.nx - 3) lEre += a.kmur * lErr;
    const bool interior = g >= 1 && g <= a.nx - 2;
    const bool rinterior = g + 1 >= 1 && g + 1 <= a.nx - 2;
    Real newE = 0, lP = 0;
    if (interior) {
      newE = a.ca * lEe;
      lP = -a.cb * lEe;
    }
    if (in_dom && g <= a.nx - 2) {
      if (interior) lH += cbdx * lEe;
      if (rinterior) lH -= cbdx * lEre;
    }
    if (g == 0 && owned) aamp += (Real)sS[s] * lE;
    if (g == a.nx - 1) newE = -a.kmur * lE;
    if (g == a.nx - 2) newE += lEr;
    if (is_med) {
      const Real *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
      Real z[D];
#pragma unroll
      for (int j = 0; j < D; ++j) z[j] = tp[j * a.ld] + sF[LF::ozr + j];
      const Real E = tp[D * a.ld];
      Real sn[Q], cm[Q];
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        sincm1(sF[LF::oth + p] * E, sn[p], cm[p]);
        const Real x0 = z[2 * p], x1 = z[2 * p + 1];
        z[2 * p] = x0 + (cm[p] * x0 + sn[p] * x1);
        z[2 * p + 1] = x1 + (cm[p] * x1 - sn[p] * x0);
      }
      // lz'' = K^T lz' + w lP
      Real l2[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        Real acc = lz[j] + sF[LF::ow + j] * lP;
#pragma unroll
        for (int i = 0; i < D; ++i) acc += sF[LF::oK + i * D + j] * lz[i];
        l2[j] = acc;
      }
      if (owned) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
          ac[i] += lz[i];
          aw[i] += lP * z[i];
#pragma unroll
          for (int j = 0; j < D; ++j) aK[i * D + j] += lz[i] * z[j];
        }
        ap0 += lP;
      }
      Real dE = 0;
#pragma unroll
      for (int p = 0; p < Q; ++p)
        dE += sF[LF::oth + p] * (l2[2 * p] * z[2 * p + 1] - l2[2 * p + 1] * z[2 * p]);
      newE += dE;
      if (owned) {
        // half-angle rotations: zhat = Rot(x/2) z', lhat = Rot(-x/2) lz''
        Real zh[D], lh[D];
#pragma unroll
        for (int j = 2 * Q; j < D; ++j) {
          zh[j] = tp[j * a.ld] + sF[LF::ozr + j];
          lh[j] = l2[j];
        }
#pragma unroll
        for (int p = 0; p < Q; ++p) {
          Real sh, ch2;
          sincm1(Real(0.5) * sF[LF::oth + p] * E, sh, ch2);
          const Real x0 = tp[(2 * p) * a.ld] + sF[LF::ozr + 2 * p];
          const Real x1 = tp[(2 * p + 1) * a.ld] + sF[LF::ozr + 2 * p + 1];
          zh[2 * p] = x0 + (ch2 * x0 + sh * x1);
          zh[2 * p + 1] = x1 + (ch2 * x1 - sh * x0);
          const Real y0 = l2[2 * p], y1 = l2[2 * p + 1];
          lh[2 * p] = y0 + (ch2 * y0 - sh * y1);
          lh[2 * p + 1] = y1 + (ch2 * y1 + sh * y0);
        }
        Real Em = E;
        const Real E2 = E * E;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
#pragma unroll
          for (int i = 0; i < D; ++i) {
            const Real li = Em * lh[i];
#pragma unroll
            for (int j = 0; j < D; ++j) aM[m][i * D + j] += li * zh[j];
          }
          Em *= E2;
        }
      }
      // lz' = Rot(x)^T lz''
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        const Real y0 = l2[2 * p], y1 = l2[2 * p + 1];
        l2[2 * p] = y0 + (cm[p] * y0 - sn[p] * y1);
        l2[2 * p + 1] = y1 + (cm[p] * y1 + sn[p] * y0);
      }
#pragma unroll
      for (int j = 0; j < D; ++j) lz[j] = l2[j];
    }
    sH[lid] = lH;
    __syncthreads();
    const Real lHl = (lid > 0) ? sH[lid - 1] : Real(0);
    if (in_dom) {
      if (g <= a.nx - 2) newE -= a.ch * lH;
      if (g >= 1) newE += a.ch * lHl;
    }
    lE = newE;
  }
  if (owned) {
    a.lEout[g] = lE;
    if (g < a.nx - 1) a.lHout[g] = lH;
    if (is_med) {
#pragma unroll
      for (int j = 0; j < D; ++j) a.lzout[j * a.ld + c] = lz[j];
    }
  }
  // per-tile reduction of the accumulators: wavefront butterfly, then LDS
  const int wid = lid / 64;
  int k = 0;
  auto put = [&](Real x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((lid & 63) == 0) sRed[wid][k] = (double)x;
    ++k;
  };
#pragma unroll
  for (int i = 0; i < D * D; ++i) put(aK[i]);
#pragma unroll
  for (int i = 0; i < D; ++i) put(ac[i]);
#pragma unroll
  for (int i = 0; i < D; ++i) put(aw[i]);
  put(ap0);
  put(aamp);
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int i = 0; i < D * D; ++i) put(aM[m][i]);
  __syncthreads();
  for (int i = lid; i < NACC; i += W) {
    double t = 0.0;
    for (int w = 0; w < W / 64; ++w) t += sRed[w][i];
    a.partial[(int64_t)blockIdx.x * NACC + i] += t;
  }
}

}  // namespace mln
