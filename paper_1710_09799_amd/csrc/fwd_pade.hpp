#pragma once
// fwd_pade.hpp -- the per-step Pade route for N >= 4: one wavefront per cell.
//
// The generic route the paper measures its two structured routes against
// (Sec. 5.3): every cell-step evaluates exp(X), X = E dt U, by a scaled
// diagonal Pade approximant and applies it to the state.  For N <= 3 the
// D x D linear system of one cell fits in one thread's registers (the tile
// kernel's Pade branch); for N = 4 (D = 15) and N = 6 (D = 35) it does not, so
// here one wavefront carries one cell: lane i owns row i of the system.
//
// Per cell-step (wave-uniform degree m and scaling s from |E| ||dt U||_1,
// Higham 2005 thresholds, as in the tile kernel):
//   X = E dt U = x V with x = E ||dt U||_1 / 2^s and the powers V^k of
//   V = dt U / ||dt U||_1 precomputed;
//   q_i.  = b_0 e_i + sum_k (-1)^k b_k x^k V^k_i.      (row i of q_m(X))
//   p_i   = b_0 d_i + sum_k b_k x^k V^k_i. d           (row i of p_m(X) d)
//   Gauss-Jordan on the rows (no pivoting: q_m(X) = b_0 (I + O(||X||)) with
//   ||X|| below the degree's threshold), the pivot row read from its lane's
//   registers;
//   d_i <- p_i / q_ii, repeated 2^s times.
// Then the merged L1 step d'_next = d'' + (A - I) d'' + c and
// dP/dt = w . d'' + p0 (lane i forms row i, every lane the dot product).
//
// Tile structure: as the tile kernel (temporal blocking, halo, ping-pong),
// with the states of the tile's cells in LDS (W x D), E and H in the
// registers of one thread per cell, and the powers V^k, A - I, c, w
// staged in LDS once per launch.
#include "fwd_impl.hpp"

namespace mln {

constexpr int kPadeWaves = 8;  // wavefronts (cells processed at once) per workgroup
constexpr int kPadeThreads = 64 * kPadeWaves;

// LDS layout of the per-step Pade kernels, in elements of Real.
template <int N, typename Real>
struct PadeLds {
  static constexpr int D = N * N - 1;
  static constexpr int up = 0;                      // kPadeMax x D x D powers V^k
  static constexpr int km = up + kPadeMax * D * D;  // D x D  A - I
  static constexpr int cz = km + D * D;             // D
  static constexpr int wz = cz + D;                 // D
  static constexpr int scr = wz + D;                // per wavefront: one state (D, prescribed-field mode)
  static constexpr int scr_stride = D + 1;
  static constexpr int tile = scr + kPadeWaves * scr_stride;  // then sz (W x D), sE, sH, sP (W), sSrc, sMur
  static constexpr size_t bytes(int W) {
    return sizeof(Real) * ((size_t)tile + (size_t)(D + 3) * W + kMaxStepsPerLaunch + 2);
  }
  static constexpr size_t bloch_bytes() { return sizeof(Real) * (size_t)tile; }
};

// Make a value that is equal on every lane visibly uniform (scalar registers).
__device__ __forceinline__ double wave_uniform(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float wave_uniform(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// Value of v on lane `src` (a compile-time lane after unrolling), returned in
// scalar registers.
__device__ __forceinline__ double lane_value(double v, int src) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ float lane_value(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// Orders this wavefront's LDS writes before its later LDS reads of other
// lanes' data (LDS executes one wavefront's operations in issue order).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Stage the factors the route reads every step into LDS.
template <int N, typename Real>
__device__ __forceinline__ void pade_stage(const FacDev<Real> &f, Real *L) {
  using Lay = PadeLds<N, Real>;
  constexpr int D = Lay::D;
  for (int i = threadIdx.x; i < kPadeMax * D * D; i += blockDim.x) L[Lay::up + i] = f.Up[i];
  for (int i = threadIdx.x; i < D * D; i += blockDim.x) L[Lay::km + i] = f.Km[i];
  for (int i = threadIdx.x; i < D; i += blockDim.x) {
    L[Lay::cz + i] = f.cz[i];
    L[Lay::wz + i] = f.wz[i];
  }
}

// d <- exp(E dt U) d for the cell of this wavefront; d is the cell's state in
// LDS (read by every lane, row i rewritten by lane i).
template <int N, typename Real>
__device__ __forceinline__ void pade_wave(const Real *L, Real unorm, Real E, Real *d, int lane) {
  using Lay = PadeLds<N, Real>;
  constexpr int D = Lay::D;
  const int row = lane < D ? lane : D - 1;  // lanes beyond D repeat the last row
  const Real xs = wave_uniform(E) * unorm;  // X = E dt U = xs V, ||V||_1 = 1
  const Real xn = xs < 0 ? -xs : xs;
  int m = 7;
  if (!(xn > Real(1.495585217958292e-2)))
    m = 3;
  else if (!(xn > Real(2.539398330063230e-1)))
    m = 5;
  int sc = 0;
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
    // the lane masks row == j are cheap to form where they are used; kept
    // from the compiler's loop-invariant hoisting, which would hold 2 D of
    // them in scalar registers across the step loop
    int r = row;
    __asm__ volatile("" : "+v"(r));
    // row r of q_m(X) and of p_m(X) d
    Real q[D];
#pragma unroll
    for (int j = 0; j < D; ++j) q[j] = (j == r) ? (Real)b[0] : Real(0);
    Real p = (Real)b[0] * d[r];
    Real xk = 1;
#pragma unroll 1
    for (int k = 1; k <= m; ++k) {
      xk *= x;
      const Real cp = (Real)b[k] * xk, cq = (k & 1) ? -cp : cp;
      const Real *u = L + Lay::up + ((k - 1) * D + r) * D;
      Real acc = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const Real uij = u[j];
        q[j] += cq * uij;
        acc += uij * d[j];
        // bound the loads the scheduler hoists (register pressure)
        if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
      }
      p += cp * acc;
    }
    // Gauss-Jordan elimination, one row per lane; the pivot row is read from
    // lane c's registers (no LDS round trip on the elimination's critical path)
    Real diag = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const Real inv = Real(1) / lane_value(q[c], c);
      const Real l = (r == c) ? Real(0) : q[c] * inv;
#pragma unroll
      for (int j = c + 1; j < D; ++j) q[j] -= l * lane_value(q[j], c);
      p -= l * lane_value(p, c);
      diag = (r == c) ? q[c] : diag;
    }
    wave_lds_sync();
    if (lane < D) d[lane] = p / diag;
    wave_lds_sync();
  }
}

// Populations of the state after exp(U E dt) (lanes a < N), FP64.
template <int N, typename Real>
__device__ __forceinline__ void pade_record_pop(const FacDev<Real> &f, const Real *d, int lane, double *pop,
                                                int64_t stride) {
  constexpr int D = N * N - 1;
  if (lane < N) {
    double acc = f.popc[lane];
#pragma unroll
    for (int j = 0; j < D; ++j) acc += f.pop[lane * D + j] * (double)d[j];
    pop[lane * stride] = acc;
  }
}

// dP/dt = w . d'' + p0 (returned on every lane) and the merged L1 step
// d <- d + (A - I) d + c in place, row i by lane i.
template <int N, typename Real>
__device__ __forceinline__ Real pade_shared_factor(const Real *L, Real p0, Real *d, int lane) {
  using Lay = PadeLds<N, Real>;
  constexpr int D = Lay::D;
  const int row = lane < D ? lane : D - 1;
  Real P = p0;
  const Real *km = L + Lay::km + row * D;
  Real acc = L[Lay::cz + row];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const Real dj = d[j];
    P += L[Lay::wz + j] * dj;
    acc += km[j] * dj;
  }
  const Real nd = d[row] + acc;
  wave_lds_sync();
  if (lane < D) d[lane] = nd;
  wave_lds_sync();
  return P;
}

template <int N, typename Real>
__global__ void __launch_bounds__(kPadeThreads) fwd_pade_kernel(FwdArgs<Real> a) {
  using Lay = PadeLds<N, Real>;
  constexpr int D = Lay::D;
  extern __shared__ __align__(16) unsigned char smem[];
  Real *L = (Real *)smem;
  const int W = a.owned + 2 * a.halo;
  Real *sz = L + Lay::tile;  // state of tile cell l at sz[l * D]
  Real *sE = sz + D * W, *sH = sE + W, *sP = sH + W, *sSrc = sP + W, *sMur = sSrc + kMaxStepsPerLaunch;
  pade_stage<N, Real>(a.fac, L);

  const int lid = threadIdx.x, lane = lid & 63, wave = lid >> 6;
  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const bool cell_thread = lid < W;
  const int64_t g = base + lid;
  const bool in_dom = cell_thread && g >= 0 && g < a.nx;
  const bool is_med = cell_thread && g >= a.mb && g < a.me;
  const bool has_right = (base <= a.nx - 1) && (base + W > a.nx - 1);
  const bool owned = in_dom && lid >= a.halo && lid < a.halo + a.owned;

  Real E = 0, H = 0;
  if (in_dom) {
    E = a.Ein[g];
    if (g < a.nx - 1) H = a.Hin[g];
  }
  if (cell_thread) {
    for (int j = 0; j < D; ++j) sz[lid * D + j] = is_med ? a.zin[j * a.ld + (g - a.mb)] : Real(0);
  }
  for (int i = lid; i < a.nsteps; i += blockDim.x) sSrc[i] = a.src[a.step0 + 1 + i];
  __syncthreads();

  int64_t snap_next = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = n == snap_next;
    if (cell_thread) sE[lid] = E;
    __syncthreads();
    if (in_dom && g < a.nx - 1) {
      const Real Er = (lid + 1 < W) ? sE[lid + 1] : Real(0);
      H += a.ch * (Er - E);
    }
    // Liouville step of every medium cell of the tile, one cell per wavefront
    for (int cl = wave; cl < W; cl += kPadeWaves) {
      const int64_t gc = base + cl;
      if (gc < a.mb || gc >= a.me) {
        if (lane == 0) sP[cl] = 0;
        continue;
      }
      Real *d = sz + cl * D;
      pade_wave<N, Real>(L, a.fac.unorm, sE[cl], d, lane);
      const bool own_c = gc < a.nx && cl >= a.halo && cl < a.halo + a.owned;
      if (snap && own_c && a.pop_out)
        pade_record_pop<N, Real>(a.fac, d, lane, a.pop_out + si * N * (a.me - a.mb) + (gc - a.mb), a.me - a.mb);
      const Real P = pade_shared_factor<N, Real>(L, a.fac.p0, d, lane);
      if (lane == 0) sP[cl] = P;
    }
    if (cell_thread) sH[lid] = H;
    __syncthreads();
    const Real Eold = E;
    if (cell_thread) {
      const Real Hl = (lid > 0) ? sH[lid - 1] : Real(0);
      if (g >= 1 && g < a.nx - 1)
        E = a.ca * E + a.cb * (-sP[lid] + (H - Hl) * a.inv_dx);
      else if (g == 0)
        E = sSrc[s];
    }
    if (has_right) {  // first-order Mur boundary at cell nx-1
      if (cell_thread && g == a.nx - 2) sMur[0] = E;
      __syncthreads();
      if (cell_thread && g == a.nx - 1) {
        E = (lid > 0 ? sE[lid - 1] : Real(0)) + a.kmur * (sMur[0] - Eold);
        if (a.probe_out) a.probe_out[n + 1] = (double)E;
      }
    }
    if (snap) {
      if (owned && a.e_out) a.e_out[si * a.nx + g] = (double)E;
      snap_next += a.snap_every;
      ++si;
    }
  }
  __syncthreads();
  if (owned) {
    a.Eout[g] = E;
    if (g < a.nx - 1) a.Hout[g] = H;
    if (is_med)
      for (int j = 0; j < D; ++j) a.zout[j * a.ld + (g - a.mb)] = sz[lid * D + j];
  }
}

// Prescribed-field mode of the per-step Pade route: one wavefront per cell.
template <int N, typename Real>
__global__ void __launch_bounds__(kPadeThreads) bloch_pade_kernel(BlochArgs<Real> a) {
  using Lay = PadeLds<N, Real>;
  constexpr int D = Lay::D;
  extern __shared__ __align__(16) unsigned char smem[];
  Real *L = (Real *)smem;
  pade_stage<N, Real>(a.fac, L);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * kPadeWaves + (threadIdx.x >> 6);
  if (c >= a.ncell) return;  // no workgroup barrier follows
  Real *d = L + Lay::scr + (threadIdx.x / 64) * Lay::scr_stride;
  if (lane < D) d[lane] = a.z0[lane];
  wave_lds_sync();
  for (int64_t t = 0; t < a.nsteps; ++t) {
    const Real E = (Real)a.efield[t * a.ncell + c];
    pade_wave<N, Real>(L, a.fac.unorm, E, d, lane);
    if (a.pop_out) pade_record_pop<N, Real>(a.fac, d, lane, a.pop_out + t * N * a.ncell + c, a.ncell);
    const Real P = pade_shared_factor<N, Real>(L, a.fac.p0, d, lane);
    if (a.dp_out && lane == 0) a.dp_out[t * a.ncell + c] = (double)P;
  }
}

}  // namespace mln
