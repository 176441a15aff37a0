// fwd_mfmaq.hpp -- split-BF16 shared-factor transform on the matrix cores with
// four lanes per cell (N = 4, 6).
//
// The one-cell-per-thread MFMA kernel leaves about one wavefront per SIMD on
// the six-level grid (224 tiles x 4 wavefronts for 1024 SIMDs), and each
// thread carries the whole per-cell vector work (q rotations, D compensated
// additions, the BF16 splits), so a step costs the latency of that chain.
// Here a cell is a quad of lanes, as in the four-lanes-per-cell kernel for
// small N:
//   * lane r of a quad owns "slots" of the state: the rotation pairs
//     p = r, r+4, r+8, .. (both components of a pair in the same lane, so the
//     exp(U E dt) rotation stays lane-local) and the population rows
//     2q + r, 2q + r + 4, ..; S slots per lane (padded to a multiple of 4);
//   * the shared factor K - I is used in this slot order (rows and columns
//     permuted: slot k = S r + i), split once per launch into three (or two)
//     BF16 parts in the A-operand layouts of v_mfma_f32_16x16x32_bf16 (the
//     first K - K mod 32 columns) and v_mfma_f32_16x16x16_bf16 (a remaining
//     16), with K = 4 S a multiple of 16; the high part lives in registers,
//     the others in LDS in lane order (conflict-free reads);
//   * the products of each 16-row block go to two accumulators, the main
//     terms and (six-product form) the small cross terms, which halves the
//     dependency chain of accumulating MFMAs; E is updated while the matrix
//     cores work, before the results are read back;
//   * every lane splits the high parts of its slots of y'' into BF16 parts and
//     writes them, contiguous, into its cell's LDS record; a wavefront holds
//     16 cells, multiplies exactly its own 16 records (one 16-column block),
//     and writes the FP32 result rows back over the same records, so the
//     matrix-core phase needs no workgroup barrier, only wavefront ordering
//     of its LDS accesses;
//   * each lane adds the results of its slots (plus the rotation increment
//     and the constant term) to its compensated hi + lo state with one
//     two-sum per slot.
// No adjoint tape is written (the adjoint is built for N <= 3).
// E, H and the source are float-float pairs, replicated in the four lanes of
// the quad; the H face left of each cell is a private copy (updated with the
// operands and operations the neighbour uses, so both stay bitwise equal); one
// workgroup barrier per step exchanges E (double-buffered).
#pragma once

#include "fwd_mfma.hpp"
#include "fwd_quad.hpp"

namespace mln {

typedef short shortx4_t __attribute__((ext_vector_type(4)));
typedef short shortx8_t __attribute__((ext_vector_type(8)));

// slot layout of the four-lanes-per-cell split-BF16 kernel
template <int N>
struct QuadSlots {
  static constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  static constexpr int NP = (Q + 3) / 4;           // rotation pairs per lane
  static constexpr int NPOP = (N - 1 + 3) / 4;     // population rows per lane
  static constexpr int USED = 2 * NP + NPOP;       // slots that can hold a row
  static constexpr int S = (USED + 3) / 4 * 4;     // slots per lane
  static constexpr int K = 4 * S;                  // GEMM size (rows = columns)
  static constexpr int NB = K / 16;                // 16-row blocks of the output
  static constexpr int KB32 = K / 32;              // 32-wide blocks of the contraction
  static constexpr int R16 = (K % 32) / 16;        // and a remaining 16-wide block (0 or 1)
  // state row held in slot i of lane r, or -1 (padding)
  __host__ __device__ static constexpr int row(int r, int i) {
    if (i < 2 * NP) {
      const int p = r + 4 * (i / 2);
      return p < Q ? 2 * p + (i & 1) : -1;
    }
    if (i < USED) {
      const int j = r + 4 * (i - 2 * NP);
      return j < N - 1 ? 2 * Q + j : -1;
    }
    return -1;
  }
  __host__ __device__ static constexpr int row_of_slot(int k) { return row(k / S, k % S); }
  // LDS record per cell (in bf16 units): NPART parts of K values, each part
  // padded by 8 (16-byte aligned parts for the 8-value B-operand reads); the
  // FP32 result row (K floats = 2 K bf16) overlays the start.  Records start
  // 16-byte aligned, and their stride in dwords is 4 mod 8 so that the 16
  // cells of a B-operand read spread over the banks.
  static constexpr int KP = K + 8;
  template <int NPART>
  static constexpr int rec() {
    constexpr int need = NPART * KP > 2 * K ? NPART * KP : 2 * K;
    constexpr int r8 = (need + 7) / 8 * 8;
    return (r8 / 2) % 8 == 0 ? r8 + 8 : r8;
  }
};

// dynamic LDS: the records, then a parking area for the rotation increments
// (USED rounded up to even floats per lane, slot-pair-major), then the middle
// and low BF16 parts of the factor in A-operand lane order
template <int N, int NPROD>
constexpr size_t mfmaq_lds_bytes(int W) {
  using SL = QuadSlots<N>;
  return (size_t)W * SL::template rec<NPROD == 6 ? 3 : 2>() * 2 + (size_t)4 * W * ((SL::USED + 1) / 2 * 2) * 4 +
         (size_t)(NPROD == 6 ? 2 : 1) * SL::NB * (SL::KB32 * 64 * 16 + SL::R16 * 64 * 8);
}

constexpr int kMaxMfmaqTile = 256;  // cells per tile (1024 lanes)

template <int N, int NPROD>
__global__ void __launch_bounds__(4 * kMaxMfmaqTile) fwd_mfmaq_kernel(FwdArgs<float> a) {
  using SL = QuadSlots<N>;
  constexpr int D = SL::D, S = SL::S, K = SL::K, NB = SL::NB, NP = SL::NP, USED = SL::USED, KP = SL::KP;
  constexpr int KB32 = SL::KB32, R16 = SL::R16;
  constexpr int NPART = NPROD == 6 ? 3 : 2;
  constexpr int REC = SL::template rec<NPART>();
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned short *sY = (unsigned short *)smem;  // record of cell c at sY + c * REC
  // parking area: float2 (slots 2 h, 2 h + 1) of lane t at sPark[h * 4 W + t]
  constexpr int NH = (USED + 1) / 2;
  // (E, low part of E) of cell c at index c + 1; indices 0 and W + 1 stay zero
  __shared__ float2 sE[2][kMaxMfmaqTile + 2];
  __shared__ float sSrc[kMaxStepsPerLaunch], sSrcl[kMaxStepsPerLaunch];
  __shared__ float sMur, sMurl;
  // per-slot constants (slot order): (reference state, polarisation weight,
  // constant term, its low part); per lane and pair: (theta dt, low part)
  __shared__ float4 sCst[K];
  __shared__ float2 sTh[4][NP];
  __shared__ double sPop[N][K], sPopc[N];

  const int t = threadIdx.x;
  const int r = t & 3;
  const int cl = t >> 2;  // cell within the tile
  const int lane = t & 63, wave = t >> 6;
  const int W = blockDim.x >> 2;
  float2 *sPark = (float2 *)(smem + (size_t)W * REC * 2);
  // middle (and low) factor parts, per part: the 32-wide fragments
  // (mb, kb) of lane at byte ((KB32 mb + kb) 64 + lane) 16, then the 16-wide
  // fragment of block mb at byte NB KB32 1024 + (64 mb + lane) 8
  constexpr int APART = NB * (KB32 * 64 * 16 + R16 * 64 * 8);
  unsigned char *sA = smem + (size_t)W * REC * 2 + (size_t)4 * W * NH * 8;
  for (int k = t; k < K; k += blockDim.x) {
    const int j = SL::row_of_slot(k);
    sCst[k] = j >= 0 ? make_float4(cld(a.fac.zr, j), cld(a.fac.wz, j), cld(a.fac.cz, j), cld(a.fac.cz_lo, j))
                     : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int lv = 0; lv < N; ++lv) sPop[lv][k] = j >= 0 ? cld(a.fac.pop, lv * D + j) : 0.0;
  }
  for (int k = t; k < 4 * NP; k += blockDim.x) {
    const int p = (k / NP) + 4 * (k % NP);  // pair i = k % NP of lane k / NP
    sTh[k / NP][k % NP] = p < SL::Q ? make_float2(cld(a.fac.thdt, p), cld(a.fac.th_lo, p)) : make_float2(0.0f, 0.0f);
  }
  for (int k = t; k < N; k += blockDim.x) sPopc[k] = cld(a.fac.popc, k);
  for (int i = t; i < a.nsteps; i += blockDim.x) {
    sSrc[i] = a.src[a.step0 + 1 + i];
    sSrcl[i] = a.src[a.nt + 1 + a.step0 + 1 + i];
  }
  for (int k = t; k < W * REC; k += blockDim.x) sY[k] = 0;
  if (t < 4) sE[t & 1][(t >> 1) ? W + 1 : 0] = make_float2(0.0f, 0.0f);

  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const int64_t g = base + cl;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool tile_med = (base < a.me) && (base + W > a.mb);
  const bool has_right = (base <= a.nx - 1) && (base + W > a.nx - 1);
  const bool owned = in_dom && cl >= a.halo && cl < a.halo + a.owned;
  const int64_t c = g - a.mb;
  const int64_t nmed = a.me - a.mb;

  // K - I in slot order, split into BF16 parts, A-operand layouts: lane
  // holds A[16 mb + lane%16][32 kb + 8 (lane/16) + i] (i < 8) of a 32-wide
  // block and A[16 mb + lane%16][32 KB32 + 4 (lane/16) + i] (i < 4) of the
  // 16-wide one.  The high part stays in registers; the middle and low parts
  // go to LDS (written once, by the first wavefront).
  shortx8_t Ah[NB][KB32 > 0 ? KB32 : 1];
  shortx4_t Ah16[NB];
  auto split3 = [&](int jm, int jk, short &h, short &md, short &lo) {
    const bool v = jm >= 0 && jk >= 0;
    const float x = v ? cld(a.fac.Km, jm * D + jk) : 0.0f;
    const float xl = v ? cld(a.fac.Km_lo, jm * D + jk) : 0.0f;
    const unsigned short hh = f2bf(x);
    const float r1 = (x - bf2f(hh)) + xl;
    const unsigned short mm = f2bf(r1);
    h = (short)hh;
    md = (short)mm;
    lo = (short)f2bf(r1 - bf2f(mm));
  };
#pragma unroll
  for (int mb = 0; mb < NB; ++mb) {
    const int jm = SL::row_of_slot(16 * mb + (lane & 15));
#pragma unroll
    for (int kb = 0; kb < KB32; ++kb) {
      shortx8_t am, al;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        short h, md, lo;
        split3(jm, SL::row_of_slot(32 * kb + 8 * (lane >> 4) + i), h, md, lo);
        Ah[mb][kb][i] = h;
        am[i] = md;
        al[i] = lo;
      }
      if (wave == 0) {
        *(shortx8_t *)(sA + ((KB32 * mb + kb) * 64 + lane) * 16) = am;
        if constexpr (NPROD == 6) *(shortx8_t *)(sA + APART + ((KB32 * mb + kb) * 64 + lane) * 16) = al;
      }
    }
    if constexpr (R16 > 0) {
      shortx4_t am, al;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        short h, md, lo;
        split3(jm, SL::row_of_slot(32 * KB32 + 4 * (lane >> 4) + i), h, md, lo);
        Ah16[mb][i] = h;
        am[i] = md;
        al[i] = lo;
      }
      if (wave == 0) {
        *(shortx4_t *)(sA + NB * KB32 * 1024 + (64 * mb + lane) * 8) = am;
        if constexpr (NPROD == 6) *(shortx4_t *)(sA + APART + NB * KB32 * 1024 + (64 * mb + lane) * 8) = al;
      }
    }
  }

  // fields (float-float), private copy of the left H face, state slots
  float E = 0, H = 0, Hl = 0, Elo = 0, Hlo = 0, Hll = 0;
  if (in_dom) {
    E = a.Ein[g];
    Elo = a.Ein[a.nx + g];
    if (g <= a.nx - 2) {
      H = a.Hin[g];
      Hlo = a.Hin[a.nx + g];
    }
    if (g >= 1) {
      Hl = a.Hin[g - 1];
      Hll = a.Hin[a.nx + g - 1];
    }
  }
  float y[USED], l[USED];
#pragma unroll
  for (int i = 0; i < USED; ++i) {
    const int j = SL::row(r, i);
    y[i] = (is_med && j >= 0) ? a.zin[j * a.ld + c] : 0.0f;
    l[i] = (is_med && j >= 0) ? a.zin[(D + j) * a.ld + c] : 0.0f;
  }
  __syncthreads();

  int64_t snap_next = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = n == snap_next;
    const int b = s & 1;
    if (r == 0) sE[b][cl + 1] = make_float2(E, Elo);
    lds_barrier();
    const float2 eL = sE[b][cl], eR = sE[b][cl + 2];
    const float El = eL.x, Ell = eL.y, Er = eR.x, Erl = eR.y;
    if (in_dom) {
      if (g >= 1) add_comp(Hl, Hll, a.ch * ((E - El) + (Elo - Ell)));
      if (g <= a.nx - 2) add_comp(H, Hlo, a.ch * ((Er - E) + (Erl - Elo)));
    }
    float P = 0.0f;
    floatx4_t acc[NB], acs[NB];
    const unsigned short *brec = sY + (size_t)(16 * wave + (lane & 15)) * REC;
    if (tile_med) {
      // per-slot constants are read from LDS inside the step loop: the offset
      // zo is always 0, but opaque to the compiler, so the loads are not
      // hoisted into registers (the state, the factor parts and the
      // accumulators already fill the register budget of 1024-lane tiles)
      const int zo = (int)(a.opaque0 * s);
      const float4 *cst = sCst + S * r + zo;
      const float2 *th = &sTh[r][zo];
      float d[USED];
      // rotations of this lane's pairs (a padding pair has theta = 0)
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        float sn, cm;
        const float2 tt = th[i];
        sincm1_lean(fmaf(tt.x, E, tt.y * E), sn, cm);
        const float y0 = y[2 * i], y1 = y[2 * i + 1];
        const float r0 = cst[2 * i].x, r1 = cst[2 * i + 1].x;
        d[2 * i] = (cm * y0 + sn * y1) + (cm * r0 + sn * r1);
        d[2 * i + 1] = (cm * y1 - sn * y0) + (cm * r1 - sn * r0);
      }
#pragma unroll
      for (int i = 2 * NP; i < USED; ++i) d[i] = 0.0f;
      // high parts of y'' are y + d, recomputed where used (same rounding)
      float pw = 0.0f;
#pragma unroll
      for (int i = 0; i < USED; ++i) pw += cst[i].y * (y[i] + d[i]);
      const float qs = quad_sum(pw);  // every lane of the tile takes part
      if (is_med) P = a.fac.p0 + qs;
      if (snap && owned && is_med && a.pop_out) {
        // populations of d^{n+1/2} in FP64: low parts of y'' are l + the
        // rounding error of y + d (two-sum); partial sums over this lane's
        // slots, completed over the quad
#pragma unroll 1
        for (int lv = 0; lv < N; ++lv) {
          double pp = 0.0;
#pragma unroll
          for (int i = 0; i < USED; ++i) {
            const float ui = y[i] + d[i];
            const float bb = ui - y[i];
            const float e = l[i] + ((y[i] - (ui - bb)) + (d[i] - bb));
            pp += sPop[lv][S * r + i] * ((double)ui + (double)e);
          }
          const double tot = quad_sum(pp) + sPopc[lv];
          if ((lv & 3) == r) a.pop_out[si * N * nmed + (int64_t)lv * nmed + c] = tot;
        }
      }
      // the rotation increments wait in LDS while the factor parts and the
      // accumulators occupy the registers
#pragma unroll
      for (int h = 0; h < NH; ++h)
        sPark[h * 4 * W + t] = make_float2(d[2 * h], 2 * h + 1 < USED ? d[2 * h + 1] : 0.0f);
      // BF16 parts of this lane's slots of y'' into the cell's record
      // (padding slots rewritten as zeros: the result row overlays them)
      unsigned short *rec = sY + (size_t)cl * REC + S * r;
#pragma unroll
      for (int i4 = 0; i4 < S / 4; ++i4) {
        unsigned short ph[4], pm[4], pl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float x = (4 * i4 + i < USED && is_med) ? y[4 * i4 + i] + d[4 * i4 + i] : 0.0f;
          ph[i] = f2bf(x);
          const float r1 = x - bf2f(ph[i]);
          pm[i] = f2bf(r1);
          pl[i] = f2bf(r1 - bf2f(pm[i]));
        }
        *(uint2 *)&rec[4 * i4] = make_uint2(ph[0] | ((unsigned)ph[1] << 16), ph[2] | ((unsigned)ph[3] << 16));
        *(uint2 *)&rec[KP + 4 * i4] = make_uint2(pm[0] | ((unsigned)pm[1] << 16), pm[2] | ((unsigned)pm[3] << 16));
        if constexpr (NPART == 3)
          *(uint2 *)&rec[2 * KP + 4 * i4] = make_uint2(pl[0] | ((unsigned)pl[1] << 16), pl[2] | ((unsigned)pl[3] << 16));
      }
      // the wavefront's 16 records are complete (all writes of this
      // wavefront precede its reads below)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // (K - I) y'' for the 16 cells of this wavefront: column n = lane%16 is
      // cell 16 wave + n; main terms in acc, the small cross terms in acs
#pragma unroll
      for (int mb = 0; mb < NB; ++mb) {
        acc[mb] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
        acs[mb] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
      }
      const unsigned char *ab = sA + zo;
#pragma unroll
      for (int kb = 0; kb < KB32; ++kb) {
        const int k0 = 32 * kb + 8 * (lane >> 4);
        const bf16x8_t Bh = __builtin_bit_cast(bf16x8_t, *(const shortx8_t *)&brec[k0]);
        const bf16x8_t Bm = __builtin_bit_cast(bf16x8_t, *(const shortx8_t *)&brec[KP + k0]);
        bf16x8_t Bl;
        if constexpr (NPART == 3) Bl = __builtin_bit_cast(bf16x8_t, *(const shortx8_t *)&brec[2 * KP + k0]);
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) {
          const int off = ((KB32 * mb + kb) * 64 + lane) * 16;
          const bf16x8_t Am = __builtin_bit_cast(bf16x8_t, *(const shortx8_t *)(ab + off));
          const bf16x8_t Ahi = __builtin_bit_cast(bf16x8_t, Ah[mb][kb]);
          if constexpr (NPROD == 6) {
            const bf16x8_t Al = __builtin_bit_cast(bf16x8_t, *(const shortx8_t *)(ab + APART + off));
            acs[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, Bh, acs[mb], 0, 0, 0);
            acs[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am, Bm, acs[mb], 0, 0, 0);
            acs[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi, Bl, acs[mb], 0, 0, 0);
          }
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am, Bh, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi, Bm, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi, Bh, acc[mb], 0, 0, 0);
        }
      }
      if constexpr (R16 > 0) {
        const int k0 = 32 * KB32 + 4 * (lane >> 4);
        const shortx4_t Bh = *(const shortx4_t *)&brec[k0];
        const shortx4_t Bm = *(const shortx4_t *)&brec[KP + k0];
        shortx4_t Bl;
        if constexpr (NPART == 3) Bl = *(const shortx4_t *)&brec[2 * KP + k0];
#pragma unroll
        for (int mb = 0; mb < NB; ++mb) {
          const int off = NB * KB32 * 1024 + (64 * mb + lane) * 8;
          const shortx4_t Am = *(const shortx4_t *)(ab + off);
          if constexpr (NPROD == 6) {
            const shortx4_t Al = *(const shortx4_t *)(ab + APART + off);
            acs[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Al, Bh, acs[mb], 0, 0, 0);
            acs[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Am, Bm, acs[mb], 0, 0, 0);
            acs[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ah16[mb], Bl, acs[mb], 0, 0, 0);
          }
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Am, Bh, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ah16[mb], Bm, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(Ah16[mb], Bh, acc[mb], 0, 0, 0);
        }
      }
    }
    // E is updated while the matrix cores work (it needs P, not the product)
    const float Eold = E, Eoldl = Elo;
    if (g >= 1 && g <= a.nx - 2) {
      add_comp(E, Elo, a.cam1 * E + a.cb * (-P + ((H - Hl) + (Hlo - Hll)) * a.inv_dx));
    } else if (g == 0) {
      E = sSrc[s];
      Elo = sSrcl[s];
    }
    if (tile_med) {
      // C layout: lane holds rows 16 mb + 4 (lane/16) + j of its column;
      // every read of these records has fed the accumulators already
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      float *res = (float *)brec;
#pragma unroll
      for (int mb = 0; mb < NB; ++mb)
        *(floatx4_t *)&res[16 * mb + 4 * (lane >> 4)] = NPROD == 6 ? acc[mb] + acs[mb] : acc[mb];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (is_med) {
        const int zo = (int)(a.opaque0 * s);
        const float4 *cst = sCst + S * r + zo;
        const float *rs = (const float *)(sY + (size_t)cl * REC) + S * r;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const float2 dd = sPark[h * 4 * W + t];
          const float4 c0 = cst[2 * h];
          add_comp(y[2 * h], l[2 * h], dd.x + (rs[2 * h] + (c0.z + c0.w)));
          if (2 * h + 1 < USED) {
            const float4 c1 = cst[2 * h + 1];
            add_comp(y[2 * h + 1], l[2 * h + 1], dd.y + (rs[2 * h + 1] + (c1.z + c1.w)));
          }
        }
      }
    }
    if (has_right) {  // first-order Mur boundary at cell nx-1
      if (g == a.nx - 2 && r == 0) {
        sMur = E;
        sMurl = Elo;
      }
      lds_barrier();
      if (g == a.nx - 1) {
        E = El;
        Elo = Ell;
        add_comp(E, Elo, a.kmur * ((sMur - Eold) + (sMurl - Eoldl)));
        if (a.probe_out && owned && r == 0) a.probe_out[n + 1] = (double)E + (double)Elo;
      }
    }
    if (snap) {
      if (owned && r == 0 && a.e_out) a.e_out[si * a.nx + g] = (double)E + (double)Elo;
      snap_next += a.snap_every;
      ++si;
    }
  }
  if (owned) {
    if (r == 0) {
      a.Eout[g] = E;
      a.Eout[a.nx + g] = Elo;
      if (g <= a.nx - 2) {
        a.Hout[g] = H;
        a.Hout[a.nx + g] = Hlo;
      }
    }
    if (is_med) {
#pragma unroll
      for (int i = 0; i < USED; ++i) {
        const int j = SL::row(r, i);
        if (j >= 0) {
          a.zout[j * a.ld + c] = y[i];
          a.zout[(D + j) * a.ld + c] = l[i];
        }
      }
    }
  }
}

}  // namespace mln
