// fwd_quad.hpp -- rotation-route tile kernel with four lanes per cell.
//
// For small level counts the per-step work of one cell (q rotations, the
// D x D shared-factor product, dP/dt, the Yee updates) is a long dependency
// chain, and a few hundred tiles give about one wavefront per SIMD, so a step
// costs the latency of that chain.  Here one cell is spread over a quad of
// lanes (N <= 3, D <= 8):
//   * in T-coordinates every lane owns one 2-component slice of the state:
//     lanes 0..q-1 a rotation pair (u_ab, v_ab), the next lane the population
//     components; the exp(U E dt) rotation is lane-local;
//   * the quad gathers the rotated state with DPP quad_perm broadcasts, each
//     lane forms two rows of (K - I) y'' from its rows of K held in registers
//     for the whole launch, and dP/dt is a two-step quad reduction whose
//     addition order gives bit-identical sums on all four lanes;
//   * E, H and the Yee updates are replicated in the four lanes (identical
//     operands, identical results), the H face left of each cell is kept as a
//     private copy (it is updated exactly as the neighbour updates it), so a
//     step needs one LDS exchange of E and one workgroup barrier
//     (double-buffered exchange array);
//   * a workgroup holds up to 256 cells (1024 lanes, 4 wavefronts per SIMD).
// Temporal blocking as in the other tile kernels: a launch advances
// nsteps <= halo steps and writes back the owned central cells.
//
// Matrix-core form (MF): the shared-factor product of the 16 cells of a
// wavefront is one 16 x 8 by 8 x 16 product, done by two 16x16x4 MFMA
// instructions.  Lanes are then laid out 16 r + (cell mod 16), so that the
// B operand (component 2r resp. 2r+1 of cell j at lane 16r + j) is the
// rotated state each lane already holds, and four result rows of cell j
// land on lane 16r + j (rows 4r .. 4r+3 in FP32, rows r, r+4, r+8, r+12 in
// FP64); the A operand stacks the factor rows so that these are rows 2r,
// 2r+1 of (K - I) and, with the compensated state, of its low part.  The constant c enters as the accumulator.  The four lanes
// of a cell sit in the four 16-lane rows of the wavefront, so dP/dt is
// summed with the gfx950 row swaps (v_permlane32_swap, v_permlane16_swap)
// instead of DPP, in an order that again gives bitwise-equal sums.
#pragma once

#include <type_traits>

#include "fwd_impl.hpp"

namespace mln {

// DPP quad_perm: every lane of a quad receives lane J's value
template <int J>
__device__ __forceinline__ float quad_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), J | (J << 2) | (J << 4) | (J << 6), 0xf,
                                                 0xf, false));
}
template <int J>
__device__ __forceinline__ double quad_bcast(double x) {
  constexpr int c = J | (J << 2) | (J << 4) | (J << 6);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), c, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), c, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// lane i of a quad receives lane perm(i) for quad_perm [1,0,3,2] and [2,3,0,1]
template <int CTRL>
__device__ __forceinline__ float quad_perm(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_perm(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
constexpr int kQuadSwap1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);  // [1,0,3,2]
constexpr int kQuadSwap2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);  // [2,3,0,1]

// (x0 + x1) + (x2 + x3) on every lane, in an order that makes the four
// results bitwise equal
template <typename Real>
__device__ __forceinline__ Real quad_sum(Real x) {
  const Real a = x + quad_perm<kQuadSwap1>(x);
  return a + quad_perm<kQuadSwap2>(a);
}

// (x_r0 + x_r2) + (x_r1 + x_r3) over the four 16-lane rows of a wavefront,
// bitwise equal on all four rows.  permlane32_swap(x, x) returns x with rows
// 2, 3 replaced by rows 0, 1 (first) and x with rows 0, 1 replaced by rows
// 2, 3 (second), so first + second adds the lower row's value first on both
// sides; permlane16_swap does the same for rows 0 <-> 1 and 2 <-> 3.
__device__ __forceinline__ float row_sum(float x) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  const float s = __uint_as_float(p[0]) + __uint_as_float(p[1]);
  const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(s), __float_as_uint(s), false, false);
  return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}
__device__ __forceinline__ double row_sum(double x) {
  const unsigned lo = (unsigned)__double2loint(x), hi = (unsigned)__double2hiint(x);
  const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double s = __hiloint2double((int)ph[0], (int)pl[0]) + __hiloint2double((int)ph[1], (int)pl[1]);
  const unsigned slo = (unsigned)__double2loint(s), shi = (unsigned)__double2hiint(s);
  const auto ql = __builtin_amdgcn_permlane16_swap(slo, slo, false, false);
  const auto qh = __builtin_amdgcn_permlane16_swap(shi, shi, false, false);
  return __hiloint2double((int)qh[0], (int)ql[0]) + __hiloint2double((int)qh[1], (int)ql[1]);
}

// DPP row rotation: lane i of each 16-lane row receives lane (i - N) mod 16
// of that row
template <int N>
__device__ __forceinline__ float row_ror(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x120 + N, 0xf, 0xf, false));
}
template <int N>
__device__ __forceinline__ double row_ror(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x120 + N, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x120 + N, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

typedef float mf_f32x4 __attribute__((ext_vector_type(4)));
typedef double mf_f64x4 __attribute__((ext_vector_type(4)));
template <typename Real>
struct MfAcc;
template <>
struct MfAcc<float> {
  typedef mf_f32x4 type;
  static __device__ __forceinline__ type mac(float a, float b, type c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfAcc<double> {
  typedef mf_f64x4 type;
  static __device__ __forceinline__ type mac(double a, double b, type c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// One tile (index `tile` of the problem described by `a`) on one workgroup of
// 4 W lanes.
template <int N, typename Real, bool COMP, bool CF, bool MF = false>
__device__ __forceinline__ void quad_tile(const FwdArgs<Real> &a, int64_t tile) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  static_assert(D <= 8, "four lanes of two components each");
  // exchanged E of cell c at index c + 1; indices 0 and W + 1 stay zero
  __shared__ Real sE[2][kMaxQuadTile + 2], sEl[2][CF ? kMaxQuadTile + 2 : 1];
  __shared__ Real sSrc[kMaxStepsPerLaunch], sSrcl[CF ? kMaxStepsPerLaunch : 1];
  __shared__ Real sMur, sMurl;
  // Single-precision three-level kernels keep the probe values of a launch
  // in LDS and store them after the step loop: a global store in the loop
  // makes the next step wait for its completion there (measured: 4-9 %
  // faster).  The other instantiations run as fast or faster with the store
  // in the loop and keep it.
  constexpr bool kProbeLds = N == 3 && std::is_same<Real, float>::value && !CF;
  __shared__ Real sPr[kProbeLds ? kMaxStepsPerLaunch : 1];
  const int t = threadIdx.x;
  // state components 2r, 2r+1 of cell cl; DPP form: lane 4 cl + r; matrix-
  // core form: wavefront cl / 16, lane 16 r + (cl mod 16)
  const int r = MF ? ((t >> 4) & 3) : (t & 3);
  const int cl = MF ? (((t >> 6) << 4) | (t & 15)) : (t >> 2);
  const int W = blockDim.x >> 2;
  const int64_t base = tile * a.owned - a.halo;
  const int64_t g = base + cl;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool tile_med = (base < a.me) && (base + W > a.mb);
  const bool has_right = (base <= a.nx - 1) && (base + W > a.nx - 1);
  const bool owned = in_dom && cl >= a.halo && cl < a.halo + a.owned;
  const int64_t c = g - a.mb;
  const int64_t nmed = a.me - a.mb;
  const int i0 = 2 * r, i1 = 2 * r + 1;
  const bool v0 = i0 < D, v1 = i1 < D;

  // this lane's rows of the factors, in registers for the whole launch
  Real K0[8], K1[8], K0l[8], K1l[8];
  // MF: the A operands, columns 2r and 2r+1 of row (t mod 16) of the stacked
  // factor.  Result item v of lane 16 q + j is row 4q + v of the product in
  // the FP32 instruction and row 4v + q in the FP64 one; the stacked row that
  // lands there is row 2q + (v & 1) of (K - I) for v < 2 and of its low part
  // for v >= 2 (zero without the compensated state).
  Real Am0 = 0, Am1 = 0;
  if constexpr (MF) {
    constexpr bool f64 = std::is_same<Real, double>::value;
    const int row = t & 15;
    const int q = f64 ? (row & 3) : (row >> 2), v = f64 ? (row >> 2) : (row & 3);
    const bool lo = v >= 2;
    const int ki = 2 * q + (v & 1);
    const bool okr = ki < D && (COMP || !lo);
    if (okr && i0 < D) Am0 = cld(lo ? a.fac.Km_lo : a.fac.Km, ki * D + i0);
    if (okr && i1 < D) Am1 = cld(lo ? a.fac.Km_lo : a.fac.Km, ki * D + i1);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      K0[j] = (v0 && j < D) ? cld(a.fac.Km, i0 * D + j) : Real(0);
      K1[j] = (v1 && j < D) ? cld(a.fac.Km, i1 * D + j) : Real(0);
      K0l[j] = (COMP && v0 && j < D) ? cld(a.fac.Km_lo, i0 * D + j) : Real(0);
      K1l[j] = (COMP && v1 && j < D) ? cld(a.fac.Km_lo, i1 * D + j) : Real(0);
    }
  }
  // Cells outside the medium in a tile that holds medium cells run the
  // matrix-core kernel's medium step with zero angle, constants, weights and
  // p0: their state and their dP/dt stay exactly zero, so that step has no
  // per-cell branch.
  const bool m0 = v0 && is_med, m1 = v1 && is_med;
  const Real c0 = m0 ? cld(a.fac.cz, i0) : Real(0), c1 = m1 ? cld(a.fac.cz, i1) : Real(0);
  const Real c0l = (COMP && m0) ? cld(a.fac.cz_lo, i0) : Real(0);
  const Real c1l = (COMP && m1) ? cld(a.fac.cz_lo, i1) : Real(0);
  const Real w0 = m0 ? cld(a.fac.wz, i0) : Real(0), w1 = m1 ? cld(a.fac.wz, i1) : Real(0);
  const Real zr0 = v0 ? cld(a.fac.zr, i0) : Real(0), zr1 = v1 ? cld(a.fac.zr, i1) : Real(0);
  const bool rot = r < Q && is_med;
  const Real th = rot ? cld(a.fac.thdt, r) : Real(0);
  const Real thl = (COMP && rot) ? cld(a.fac.th_lo, r) : Real(0);
  const Real p0 = is_med ? a.fac.p0 : Real(0);

  // E, H and the private copy Hl of the face left of the cell; with CF each
  // has a low part (Elo, Hlo, Hll)
  Real E = 0, H = 0, Hl = 0, Elo = 0, Hlo = 0, Hll = 0;
  Real y0 = 0, y1 = 0, l0 = 0, l1 = 0;
  if (in_dom) {
    E = a.Ein[g];
    if (g <= a.nx - 2) H = a.Hin[g];
    if (g >= 1) Hl = a.Hin[g - 1];
    if constexpr (CF) {
      Elo = a.Ein[a.nx + g];
      if (g <= a.nx - 2) Hlo = a.Hin[a.nx + g];
      if (g >= 1) Hll = a.Hin[a.nx + g - 1];
    }
  }
  if (is_med) {
    if (v0) y0 = a.zin[i0 * a.ld + c];
    if (v1) y1 = a.zin[i1 * a.ld + c];
    if constexpr (COMP) {
      if (v0) l0 = a.zin[(D + i0) * a.ld + c];
      if (v1) l1 = a.zin[(D + i1) * a.ld + c];
    }
  }

  // source samples of this launch (read by the tile holding cell 0)
  for (int i = threadIdx.x; i < a.nsteps; i += blockDim.x) {
    sSrc[i] = a.src[a.step0 + 1 + i];
    if constexpr (CF) sSrcl[i] = a.src[a.nt + 1 + a.step0 + 1 + i];
  }
  if (threadIdx.x < 4) {  // the zero pads of both exchange buffers
    const int b = threadIdx.x & 1, i = (threadIdx.x >> 1) ? W + 1 : 0;
    sE[b][i] = Real(0);
    if constexpr (CF) sEl[b][i] = Real(0);
  }
  __syncthreads();
  // the step loop keeps its bookkeeping in 32-bit scalars and its field
  // updates free of divergent branches (the step's time is the length of
  // one wavefront's instruction stream): the next snapshot as a step index
  // within this launch (-1: none), the cell's role as loop-invariant masks
  int s_snap = (a.snap_next >= a.step0 && a.snap_next < a.step0 + a.nsteps) ? (int)(a.snap_next - a.step0) : -1;
  const int snap_gap = (int)(a.snap_every < kMaxStepsPerLaunch ? a.snap_every : kMaxStepsPerLaunch);
  const bool interior = g >= 1 && g <= a.nx - 2;
  const bool is_src = g == 0;
  int64_t si = a.snap_i0;
  // MF: the product of step n is consumed at the start of step n + 1, after
  // the exchange and its barrier, so the matrix-core latency overlaps them
  // (pd: the rotation increments with the compensated state, else y'')
  typename MfAcc<Real>::type pacc = {0, 0, 0, 0};
  Real pd0 = COMP ? Real(0) : y0, pd1 = COMP ? Real(0) : y1;  // applying these leaves y as loaded
  auto mf_apply = [&]() {
    if constexpr (COMP) {
      add_comp(y0, l0, pd0 + (pacc[0] + pacc[2]));
      add_comp(y1, l1, pd1 + (pacc[1] + pacc[3]));
    } else {
      y0 = pd0 + pacc[0];
      y1 = pd1 + pacc[1];
    }
  };
  for (int s = 0; s < a.nsteps; ++s) {
    const bool snap = s == s_snap;
    const int b = s & 1;
    // every lane of the quad writes the cell's E (the four values are
    // bitwise equal), so the exchange write needs no branch
    sE[b][cl + 1] = E;
    if constexpr (CF) sEl[b][cl + 1] = Elo;
    lds_barrier();
    const Real El = sE[b][cl], Er = sE[b][cl + 2];
    const Real src = sSrc[s];
    Real Ell = 0, Erl = 0, srcl = 0;
    if constexpr (CF) {
      Ell = sEl[b][cl];
      Erl = sEl[b][cl + 2];
      srcl = sSrcl[s];
    }
    // H at both faces of the cell; the private copy Hl is updated with the
    // operands and operations the left neighbour uses for its own face, so
    // the two stay bitwise equal.  Faces outside the grid (left of cell 0,
    // right of cell nx-1, and those of cells beyond the grid in edge tiles)
    // are updated too, without a branch: nothing reads them.
    if constexpr (CF) {
      add_comp(Hl, Hll, a.ch * ((E - El) + (Elo - Ell)));
      add_comp(H, Hlo, a.ch * ((Er - E) + (Erl - Elo)));
    } else {
      Hl += a.ch * (E - El);
      H += a.ch * (Er - E);
    }
    Real P = 0;
    if constexpr (MF) {
      // the matrix-core product and the row sums take every lane of the
      // wavefront: the branch is uniform (tile_med, snap, pop_out), the
      // cell's own role (is_med, owned) only selects what is kept
      if (tile_med) {
        mf_apply();
        if (a.tape) {
          const int64_t n = a.step0 + s;
          if (owned && is_med && n >= a.tape_step0) {
            Real *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
            if (v0) tp[i0 * a.ld] = y0;
            if (v1) tp[i1 * a.ld] = y1;
            if (r == 0) tp[D * a.ld] = E;
          }
        }
        Real sn, cm;
        if constexpr (COMP)
          sincm1(fmaf(th, E, thl * E), sn, cm);
        else
          sincm1(th * E, sn, cm);
        const Real d0 = (cm * y0 + sn * y1) + (cm * zr0 + sn * zr1);
        const Real d1 = (cm * y1 - sn * y0) + (cm * zr1 - sn * zr0);
        const Real u0 = y0 + d0, u1 = y1 + d1;
        if (snap && a.pop_out) {
          // population of level lv = popc + pop row lv . y'' (FP64): each
          // lane's two terms, summed over the cell's four lanes
          Real e0 = 0, e1 = 0;
          if constexpr (COMP) {
            const Real bb0 = u0 - y0, bb1 = u1 - y1;
            e0 = l0 + ((y0 - (u0 - bb0)) + (d0 - bb0));
            e1 = l1 + ((y1 - (u1 - bb1)) + (d1 - bb1));
          }
          const double z0 = (double)u0 + (double)e0, z1 = (double)u1 + (double)e1;
          double mine = 0.0;
#pragma unroll
          for (int lv = 0; lv < N; ++lv) {
            const double pr0 = v0 ? cld(a.fac.pop, lv * D + i0) : 0.0;
            const double pr1 = v1 ? cld(a.fac.pop, lv * D + i1) : 0.0;
            const double sum = row_sum(pr0 * z0 + pr1 * z1);
            if (lv == r) mine = cld(a.fac.popc, lv) + sum;
          }
          if (owned && is_med && r < N) a.pop_out[si * N * nmed + (int64_t)r * nmed + c] = mine;
        }
        const Real ps = row_sum(w0 * u0 + w1 * u1);
        pacc = {c0, c1, c0l, c1l};
        pacc = MfAcc<Real>::mac(Am0, u0, pacc);
        pacc = MfAcc<Real>::mac(Am1, u1, pacc);
        pd0 = COMP ? d0 : u0;
        pd1 = COMP ? d1 : u1;
        P = p0 + ps;
      }
    } else if (tile_med && is_med) {
      // (the DPP kernel keeps the per-cell branch: measured faster here
      // than the branch-free form the matrix-core kernel uses)
      if (a.tape) {
        const int64_t n = a.step0 + s;
        if (owned && n >= a.tape_step0) {
          Real *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
          if (v0) tp[i0 * a.ld] = y0;
          if (v1) tp[i1 * a.ld] = y1;
          if (r == 0) tp[D * a.ld] = E;
        }
      }
      // y'' = Rot(y) + (Rot - I) zr on this lane's pair; a lane without a
      // pair has th = 0, so its increment is exactly zero (no divergence)
      Real sn, cm;
      if constexpr (COMP)
        sincm1(fmaf(th, E, thl * E), sn, cm);
      else
        sincm1(th * E, sn, cm);
      const Real d0 = (cm * y0 + sn * y1) + (cm * zr0 + sn * zr1);
      const Real d1 = (cm * y1 - sn * y0) + (cm * zr1 - sn * zr0);
      // high parts of y''; the rotation increment joins the shared-factor
      // increment below in one compensated addition
      const Real u0 = y0 + d0, u1 = y1 + d1;
      // gather y'' of the quad
      Real zz[8];
      zz[0] = quad_bcast<0>(u0);
      zz[1] = quad_bcast<0>(u1);
      zz[2] = quad_bcast<1>(u0);
      zz[3] = quad_bcast<1>(u1);
      zz[4] = quad_bcast<2>(u0);
      zz[5] = quad_bcast<2>(u1);
      zz[6] = quad_bcast<3>(u0);
      zz[7] = quad_bcast<3>(u1);
      if (snap && owned && is_med && a.pop_out) {
        // all four lanes take part in the broadcasts; lanes 0..N-1 each
        // form the population of one level.  With COMP the low parts of
        // y'' are l + the rounding error of y + d (two-sum).
        double ll[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) ll[j] = 0.0;
        if constexpr (COMP) {
          const Real bb0 = u0 - y0, bb1 = u1 - y1;
          const Real e0 = l0 + ((y0 - (u0 - bb0)) + (d0 - bb0));
          const Real e1 = l1 + ((y1 - (u1 - bb1)) + (d1 - bb1));
          ll[0] = (double)quad_bcast<0>(e0);
          ll[1] = (double)quad_bcast<0>(e1);
          ll[2] = (double)quad_bcast<1>(e0);
          ll[3] = (double)quad_bcast<1>(e1);
          ll[4] = (double)quad_bcast<2>(e0);
          ll[5] = (double)quad_bcast<2>(e1);
          ll[6] = (double)quad_bcast<3>(e0);
          ll[7] = (double)quad_bcast<3>(e1);
        }
        if (r < N) {
          double acc = cld(a.fac.popc, r);
#pragma unroll
          for (int j = 0; j < D; ++j) acc += cld(a.fac.pop, r * D + j) * ((double)zz[j] + ll[j]);
          a.pop_out[si * N * nmed + (int64_t)r * nmed + c] = acc;
        }
      }
      P = p0 + quad_sum(w0 * u0 + w1 * u1);
      // y_next = y'' + (K - I) y'' + constant, rows 2r and 2r+1
      Real a0 = c0, a1 = c1, b0 = c0l, b1 = c1l;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        a0 += K0[j] * zz[j];
        a1 += K1[j] * zz[j];
        if constexpr (COMP) {
          b0 += K0l[j] * zz[j];
          b1 += K1l[j] * zz[j];
        }
      }
      if constexpr (COMP) {
        add_comp(y0, l0, d0 + (a0 + b0));
        add_comp(y1, l1, d1 + (a1 + b1));
      } else {
        y0 = u0 + a0;
        y1 = u1 + a1;
      }
    }
    const Real Eold = E, Eoldl = Elo;
    {
      // interior cells: the Yee update; cell 0: the source sample; other
      // cells (nx-1, set below, and cells beyond the grid) keep E
      Real En = E, Enl = Elo;
      if constexpr (CF)
        add_comp(En, Enl, a.cam1 * E + a.cb * (-P + ((H - Hl) + (Hlo - Hll)) * a.inv_dx));
      else
        En = a.ca * E + a.cb * (-P + (H - Hl) * a.inv_dx);
      E = interior ? En : (is_src ? src : E);
      if constexpr (CF) Elo = interior ? Enl : (is_src ? srcl : Elo);
    }
    if (has_right) {  // first-order Mur boundary at cell nx-1
      if (g == a.nx - 2 && r == 0) {
        sMur = E;
        sMurl = Elo;
      }
      lds_barrier();
      if (g == a.nx - 1) {
        if constexpr (CF) {
          E = El;
          Elo = Ell;
          add_comp(E, Elo, a.kmur * ((sMur - Eold) + (sMurl - Eoldl)));
        } else {
          E = El + a.kmur * (sMur - Eold);
        }
        if constexpr (kProbeLds) {
          if (owned && r == 0) sPr[s] = E;
        } else {
          if (a.probe_out && owned && r == 0) a.probe_out[a.step0 + s + 1] = (double)E + (double)Elo;
        }
      }
    }
    if (snap) {
      if (owned && r == 0 && a.e_out) a.e_out[si * a.nx + g] = (double)E + (double)Elo;
      s_snap += snap_gap;
      ++si;
    }
  }
  if constexpr (MF) {
    if (tile_med) mf_apply();
  }
  if constexpr (kProbeLds) {
    if (a.probe_out && has_right && owned && r == 0 && g == a.nx - 1)
      for (int s = 0; s < a.nsteps; ++s) a.probe_out[a.step0 + 1 + s] = (double)sPr[s];
  }
  if (owned) {
    if (r == 0) {
      a.Eout[g] = E;
      if (g <= a.nx - 2) a.Hout[g] = H;
      if constexpr (CF) {
        a.Eout[a.nx + g] = Elo;
        if (g <= a.nx - 2) a.Hout[a.nx + g] = Hlo;
      }
    }
    if (is_med) {
      if (v0) a.zout[i0 * a.ld + c] = y0;
      if (v1) a.zout[i1 * a.ld + c] = y1;
      if constexpr (COMP) {
        if (v0) a.zout[(D + i0) * a.ld + c] = l0;
        if (v1) a.zout[(D + i1) * a.ld + c] = l1;
      }
    }
  }
}

// COMP: compensated (float-float) state; CF: E and H as float-float pairs too.
// LB: the launch bound the instance is compiled for (lanes per workgroup).
// The LB = 512 instance may use up to 256 VGPRs per lane, which keeps the
// FP64 and two-float-field step loops free of spills but leaves room for
// one such workgroup per compute unit; LB = 1024 (at most 128 VGPRs) lets
// two 512-lane workgroups share a compute unit.
template <int N, typename Real, bool COMP, bool CF = false, int LB = 1024, bool MF = false>
__global__ void __launch_bounds__(LB) fwd_quad_kernel(FwdArgs<Real> a) {
  quad_tile<N, Real, COMP, CF, MF>(a, blockIdx.x);
}

// Compute units of the current device (cached per device).
inline int quad_device_cus() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

// The LB = 512 instance for tiles of at most 128 cells when every tile has a
// compute unit of its own, for the instances whose LB = 1024 build spills
// (FP64 and two-float fields at N = 3: 36 and 20 bytes per lane; the
// compensated-FP32 state fits 128 VGPRs and runs faster there); else LB = 1024.
// MF (the matrix-core product): one build, LB = 1024 (the factor rows are
// two registers instead of 32).
template <int N, typename Real, bool COMP, bool CF>
hipError_t launch_quad(int W, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st, bool mf = false) {
  constexpr bool wide = std::is_same<Real, double>::value || CF;
  if (mf)
    hipLaunchKernelGGL((fwd_quad_kernel<N, Real, COMP, CF, 1024, true>), dim3((unsigned)nblocks), dim3(4 * W), 0, st, a);
  else if (wide && 4 * W <= 512 && nblocks <= quad_device_cus())
    hipLaunchKernelGGL((fwd_quad_kernel<N, Real, COMP, CF, 512>), dim3((unsigned)nblocks), dim3(4 * W), 0, st, a);
  else
    hipLaunchKernelGGL((fwd_quad_kernel<N, Real, COMP, CF, 1024>), dim3((unsigned)nblocks), dim3(4 * W), 0, st, a);
  return hipGetLastError();
}

}  // namespace mln
