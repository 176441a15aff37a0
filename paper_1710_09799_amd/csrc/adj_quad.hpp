// adj_quad.hpp -- reverse-time (adjoint) tile kernel with four lanes per cell.
//
// The reverse of one fused step (Yee updates, exp(U E dt) rotations, merged
// L1 factor, dP/dt) in the layout of the forward four-lanes-per-cell kernel:
// lane r of a cell's quad owns state rows 2r and 2r+1 in T-coordinates (the
// rotation pair r for r < q, the population rows after that).  Per step and
// cell it forms
//   lz'' = K^T lz' + w lP                    (rows 2r, 2r+1 from K's columns)
//   dJ/dE += sum_p theta_p (lz''_u z''_v - lz''_v z''_u)   (quad sum)
//   lz'  = Rot(x)^T lz''
// and accumulates, for owned cells, rows 2r and 2r+1 of
//   dJ/dK += lz' z''^T,  dJ/dc += lz',  dJ/dw += lP z'',  dJ/dp0 += lP,
//   Gamma_m += E^m lhat zhat^T  (lhat = Rot(-x/2) lz'', zhat = Rot(x/2) z'),
// from which the host forms dJ/dU (the half-angle moment expansion of the
// derivative of exp(U E dt) with respect to U).  The forward state z' and E of
// every step come from the tape written by the forward kernel's recomputation
// of the segment.  The quad gathers the full vectors it needs (lz', z'',
// zhat) with DPP broadcasts.  The adjoint Yee updates are replicated in the
// four lanes; the adjoint E is exchanged through LDS (one barrier per step,
// double-buffered) and the adjoint H of the face left of each cell is a
// private copy kept bitwise equal to the neighbour's.
// The accumulator order is that of the one-cell-per-thread adjoint kernel
// (dJ/dK, dJ/dc, dJ/dw, dJ/dp0, dJ/damplitude, Gamma_1, Gamma_3[, Gamma_5]);
// each tile adds its sums to partial[tile][*].
#pragma once

#include "fwd_quad.hpp"

namespace mln {


// LB: the launch bound the instance is built for; the 256-lane instance
// (tiles of at most 64 cells) has the whole register file of a SIMD for one
// wavefront, which the FP64 three-level reverse step needs to run without
// spilling (its 512-lane build spills 216 bytes per lane).
template <int N, typename Real, int LB = 4 * kMaxAdjQuadTile>
__global__ void __launch_bounds__(LB) adj_quad_kernel(AdjArgs<Real> a) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  static_assert(D <= 8, "four lanes of two components each");
  constexpr bool F64 = sizeof(Real) == 8;
  constexpr int NM = adj_moments(F64);
  constexpr int NACC = adj_nacc(N, F64);
  constexpr int kMaxWaves = 4 * kMaxAdjQuadTile / 64;
  // exchanged adjoint E of cell c at sE[b][c + 1] (double-buffered); indices
  // 0, W + 1 and W + 2 stay zero
  __shared__ Real sE[2][kMaxAdjQuadTile + 3];
  __shared__ double sG[kMaxStepsPerLaunch], sS[kMaxStepsPerLaunch];
  __shared__ double sRed[kMaxWaves][NACC];

  const int t = threadIdx.x;
  const int r = t & 3;
  const int cl = t >> 2;
  const int W = blockDim.x >> 2;
  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const int64_t g = base + cl;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool owned = in_dom && cl >= a.halo && cl < a.halo + a.owned;
  const int64_t c = g - a.mb;
  const int i0 = 2 * r, i1 = 2 * r + 1;
  const bool v0 = i0 < D, v1 = i1 < D;
  const bool rot = r < Q;
  const Real cbdx = a.cb * a.inv_dx;

  // columns i0, i1 of K = I + Km (rows of K^T), w, zr, theta dt of this lane
  Real KT0[8], KT1[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    KT0[i] = (v0 && i < D) ? cld(a.fac.Km, i * D + i0) : Real(0);
    KT1[i] = (v1 && i < D) ? cld(a.fac.Km, i * D + i1) : Real(0);
  }
  const Real w0 = v0 ? cld(a.fac.wz, i0) : Real(0), w1 = v1 ? cld(a.fac.wz, i1) : Real(0);
  const Real zr0 = v0 ? cld(a.fac.zr, i0) : Real(0), zr1 = v1 ? cld(a.fac.zr, i1) : Real(0);
  const Real th = rot ? cld(a.fac.thdt, r) : Real(0);

  // lHl: private copy of the adjoint H of the face left of the cell, updated
  // with the operands and operations the left neighbour uses for its own
  Real lE = 0, lH = 0, lHl = 0, lz0 = 0, lz1 = 0;
  if (in_dom) {
    lE = a.lEin[g];
    if (g < a.nx - 1) lH = a.lHin[g];
    if (g >= 1) lHl = a.lHin[g - 1];
  }
  if (is_med) {
    if (v0) lz0 = a.lzin[i0 * a.ld + c];
    if (v1) lz1 = a.lzin[i1 * a.ld + c];
  }
  Real aK0[8], aK1[8], aM0[NM][8], aM1[NM][8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    aK0[j] = 0;
    aK1[j] = 0;
#pragma unroll
    for (int m = 0; m < NM; ++m) {
      aM0[m][j] = 0;
      aM1[m][j] = 0;
    }
  }
  Real ac0 = 0, ac1 = 0, aw0 = 0, aw1 = 0, ap0 = 0, aamp = 0;

  for (int i = t; i < a.nsteps; i += blockDim.x) {
    sG[i] = a.gprobe[a.n_hi - i];
    sS[i] = a.samples[a.n_hi - i];
  }
  if (t < 6) sE[t & 1][t < 2 ? 0 : (t < 4 ? W + 1 : W + 2)] = Real(0);
  // tape values (y' of this lane's rows and E) of the step being reversed
  // (t*) and of the step after it (u*): loaded two steps ahead, since one
  // step takes about as long as a load from HBM
  Real ty0 = 0, ty1 = 0, tE = 0, uy0 = 0, uy1 = 0, uE = 0;
  auto tape_load = [&](int64_t nn, Real &y0, Real &y1, Real &e) {
    if (is_med && nn >= a.tape_step0) {
      const Real *tp = a.tape + (nn - a.tape_step0) * (D + 1) * a.ld + c;
      y0 = v0 ? tp[i0 * a.ld] : Real(0);
      y1 = v1 ? tp[i1 * a.ld] : Real(0);
      e = tp[D * a.ld];
    }
  };
  if (a.nsteps > 0) tape_load(a.n_hi - 1, ty0, ty1, tE);
  if (a.nsteps > 1) tape_load(a.n_hi - 2, uy0, uy1, uE);
  __syncthreads();
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.n_hi - 1 - s;
    if (g == a.nx - 1) lE += (Real)sG[s];
    const int b = s & 1;
    if (r == 0) sE[b][cl + 1] = lE;
    lds_barrier();
    const Real lEl = sE[b][cl], lEr = sE[b][cl + 2], lErr = sE[b][cl + 3];
    // the left neighbour's own H update (its lEe and lEre from lEl, lE, lEr)
    {
      Real lEeL = lEl, lEreL = lE;
      if (g - 1 == a.nx - 2) lEeL += a.kmur * lE;
      if (g - 1 == a.nx - 3) lEreL += a.kmur * lEr;
      if (g >= 1 && g <= a.nx - 1) {
        if (g >= 2) lHl += cbdx * lEeL;
        if (g <= a.nx - 2) lHl -= cbdx * lEreL;
      }
    }
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
    if (g == 0 && owned && r == 0) aamp += (Real)sS[s] * lE;
    if (g == a.nx - 1) newE = -a.kmur * lE;
    if (g == a.nx - 2) newE += lEr;
    if (is_med) {
      const Real x0 = v0 ? ty0 + zr0 : Real(0);  // z' of this lane's rows
      const Real x1 = v1 ? ty1 + zr1 : Real(0);
      const Real E = tE;
      ty0 = uy0;
      ty1 = uy1;
      tE = uE;
      if (s + 2 < a.nsteps) tape_load(n - 2, uy0, uy1, uE);
      Real sn = 0, cm = 0, z0 = x0, z1 = x1;  // z'' = Rot(x) z'
      if (rot) {
        sincm1(th * E, sn, cm);
        z0 = x0 + (cm * x0 + sn * x1);
        z1 = x1 + (cm * x1 - sn * x0);
      }
      // lz'' = K^T lz' + w lP, rows i0 and i1
      Real lzz[8];
      lzz[0] = quad_bcast<0>(lz0);
      lzz[1] = quad_bcast<0>(lz1);
      lzz[2] = quad_bcast<1>(lz0);
      lzz[3] = quad_bcast<1>(lz1);
      lzz[4] = quad_bcast<2>(lz0);
      lzz[5] = quad_bcast<2>(lz1);
      lzz[6] = quad_bcast<3>(lz0);
      lzz[7] = quad_bcast<3>(lz1);
      Real l20 = lz0 + w0 * lP, l21 = lz1 + w1 * lP;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        l20 += KT0[i] * lzz[i];
        l21 += KT1[i] * lzz[i];
      }
      Real zz[8];
      zz[0] = quad_bcast<0>(z0);
      zz[1] = quad_bcast<0>(z1);
      zz[2] = quad_bcast<1>(z0);
      zz[3] = quad_bcast<1>(z1);
      zz[4] = quad_bcast<2>(z0);
      zz[5] = quad_bcast<2>(z1);
      zz[6] = quad_bcast<3>(z0);
      zz[7] = quad_bcast<3>(z1);
      // dJ/dE of this step's rotation: one pair per lane, summed over the quad
      const Real dEl = rot ? th * (l20 * z1 - l21 * z0) : Real(0);
      newE += quad_sum(dEl);
      // half-angle vectors: zhat = Rot(x/2) z' and lhat = Rot(-x/2) lz''
      Real zh0 = x0, zh1 = x1, lh0 = l20, lh1 = l21;
      if (rot) {
        Real sh, ch2;
        sincm1(Real(0.5) * th * E, sh, ch2);
        zh0 = x0 + (ch2 * x0 + sh * x1);
        zh1 = x1 + (ch2 * x1 - sh * x0);
        lh0 = l20 + (ch2 * l20 - sh * l21);
        lh1 = l21 + (ch2 * l21 + sh * l20);
      }
      Real zhh[8];
      zhh[0] = quad_bcast<0>(zh0);
      zhh[1] = quad_bcast<0>(zh1);
      zhh[2] = quad_bcast<1>(zh0);
      zhh[3] = quad_bcast<1>(zh1);
      zhh[4] = quad_bcast<2>(zh0);
      zhh[5] = quad_bcast<2>(zh1);
      zhh[6] = quad_bcast<3>(zh0);
      zhh[7] = quad_bcast<3>(zh1);
      if (owned) {
        ac0 += lz0;
        ac1 += lz1;
        aw0 += lP * z0;
        aw1 += lP * z1;
        if (r == 0) ap0 += lP;
        Real Em = E;
        const Real E2 = E * E;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          const Real p0 = Em * lh0, p1 = Em * lh1;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            aM0[m][j] += p0 * zhh[j];
            aM1[m][j] += p1 * zhh[j];
          }
          Em *= E2;
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
          aK0[j] += lz0 * zz[j];
          aK1[j] += lz1 * zz[j];
        }
      }
      // lz' = Rot(x)^T lz''
      if (rot) {
        lz0 = l20 + (cm * l20 - sn * l21);
        lz1 = l21 + (cm * l21 + sn * l20);
      } else {
        lz0 = l20;
        lz1 = l21;
      }
    }
    if (in_dom) {
      if (g <= a.nx - 2) newE -= a.ch * lH;
      if (g >= 1) newE += a.ch * lHl;
    }
    lE = newE;
  }
  if (owned) {
    if (r == 0) {
      a.lEout[g] = lE;
      if (g < a.nx - 1) a.lHout[g] = lH;
    }
    if (is_med) {
      if (v0) a.lzout[i0 * a.ld + c] = lz0;
      if (v1) a.lzout[i1 * a.ld + c] = lz1;
    }
  }
  // per-tile sums: over the 16 cells of a wavefront (lanes of equal r: the
  // lanes 4 and 8 apart within each 16-lane row by DPP row rotations, then
  // the four rows by the permlane swaps), then over the wavefronts through LDS
  const int wid = t >> 6;
  auto wsum = [&](Real x) {
    x += row_ror<4>(x);
    x += row_ror<8>(x);
    return row_sum(x);
  };
  const bool lead = (t & 63) < 4;  // lanes 0..3 of the wavefront hold the sums
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const Real s0 = wsum(aK0[j]), s1 = wsum(aK1[j]);
    if (lead && j < D) {
      if (v0) sRed[wid][i0 * D + j] = (double)s0;
      if (v1) sRed[wid][i1 * D + j] = (double)s1;
    }
  }
  {
    const Real s0 = wsum(ac0), s1 = wsum(ac1), s2 = wsum(aw0), s3 = wsum(aw1);
    if (lead) {
      if (v0) sRed[wid][D * D + i0] = (double)s0;
      if (v1) sRed[wid][D * D + i1] = (double)s1;
      if (v0) sRed[wid][D * D + D + i0] = (double)s2;
      if (v1) sRed[wid][D * D + D + i1] = (double)s3;
    }
    const Real s4 = wsum(ap0), s5 = wsum(aamp);
    if ((t & 63) == 0) {
      sRed[wid][D * D + 2 * D] = (double)s4;
      sRed[wid][D * D + 2 * D + 1] = (double)s5;
    }
  }
  constexpr int oM = D * D + 2 * D + 2;
#pragma unroll
  for (int m = 0; m < NM; ++m) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const Real s0 = wsum(aM0[m][j]), s1 = wsum(aM1[m][j]);
      if (lead && j < D) {
        if (v0) sRed[wid][oM + m * D * D + i0 * D + j] = (double)s0;
        if (v1) sRed[wid][oM + m * D * D + i1 * D + j] = (double)s1;
      }
    }
  }
  __syncthreads();
  const int nw = blockDim.x >> 6;
  for (int i = t; i < NACC; i += blockDim.x) {
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) acc += sRed[w][i];
    // the tile's own slot (no other tile adds to it; launches are ordered on
    // the stream, so the sums are deterministic): a no-return atomic add
    // lets the wavefront finish without waiting for the old value
    atomicAdd(&a.partial[(int64_t)blockIdx.x * NACC + i], acc);
  }
}

}  // namespace mln
