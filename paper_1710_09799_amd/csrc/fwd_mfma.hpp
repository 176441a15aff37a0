// fwd_mfma.hpp -- rotation-route tile kernel whose shared-factor transform
// runs on the matrix cores (gfx950 v_mfma_f32_16x16x32_bf16).
//
// Per time step the tile's cells need y_next = y'' + (K - I) y'' + r with one
// (D x D) factor shared by all cells: a real GEMM (D x D) . (D x cells).  The
// kernel keeps the Liouville state in a compensated single-precision pair
// (hi + lo) per cell and runs everything except that GEMM on the vector ALUs,
// one cell per thread, exactly as the workgroup-tile kernel does.  The GEMM:
//   * K - I is split once per launch into three bfloat16 parts
//     (A = A_h + A_m + A_l, 24 significant bits) held in registers in the
//     MFMA A-operand layout;
//   * every cell splits the high part of its rotated state y'' into three
//     bfloat16 parts and stores them in its LDS record (cell-major, padded so
//     the B-operand reads of 16 consecutive cells hit distinct banks); the
//     FP32 result row of the cell overlays the start of the same record: only
//     the wavefront that multiplies a 16-cell block touches those records, and
//     its reads precede its writes through the accumulator dependency;
//   * each wavefront multiplies its share of 16-cell column blocks with
//     NPROD split products accumulated in FP32 (6: hh hm mh hl mm lh, error
//     ~2^-24 |K - I| |y''|; 3: hh hm mh with two-part splits, ~2^-16);
//   * the FP32 results go back through LDS and are added to hi + lo exactly.
// Padding: D components -> 16 * MB rows (M) and 32 * KB columns (K), zeros.
#pragma once

#include "fwd_impl.hpp"

namespace mln {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// round-to-nearest-even float -> bfloat16 bits, and back
__device__ __forceinline__ unsigned short f2bf(float x) {
  __bf16 b = (__bf16)x;
  return __builtin_bit_cast(unsigned short, b);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

template <int D>
struct MfmaShape {
  static constexpr int MB = (D + 15) / 16;   // 16-row blocks of the output
  static constexpr int KB = (D + 31) / 32;   // 32-wide blocks of the contraction
  static constexpr int KP = 32 * KB + 8;     // bf16 per cell row in LDS (padded)
  static constexpr int MP = 16 * MB + 4;     // floats per cell row of the result (padded)
};

// LDS record of one cell: NPART rows of KP bfloat16 (the result row of MP
// floats overlays its start)
template <int D, int NPROD>
constexpr int mfma_rec_bf16() {
  return (NPROD == 6 ? 3 : 2) * MfmaShape<D>::KP;
}
template <int D, int NPROD>
constexpr size_t mfma_lds_bytes(int W) {
  return (size_t)W * mfma_rec_bf16<D, NPROD>() * 2;
}

template <int N, int NPROD>
__global__ void __launch_bounds__(256) fwd_mfma_kernel(FwdArgs<float> a) {
  constexpr int D = N * N - 1, Q = N * (N - 1) / 2;
  using S = MfmaShape<D>;
  constexpr int MB = S::MB, KB = S::KB, KP = S::KP, MP = S::MP;
  constexpr int NPART = NPROD == 6 ? 3 : 2;
  constexpr int REC = mfma_rec_bf16<D, NPROD>();
  static_assert(2 * MP <= REC, "result row fits in the record");
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned short *sY = (unsigned short *)smem;  // record of cell c at sY + c * REC
  __shared__ float sE[2][kMaxTile], sEl[2][kMaxTile];  // exchanged fields, high and low parts
  __shared__ float sMur, sMurl;
  __shared__ float sSrc[kMaxStepsPerLaunch], sSrcl[kMaxStepsPerLaunch];
  __shared__ double sP[N * D + N];
  using L = RotLds<N, float, true>;
  __shared__ float sF[L::size];
  L::stage(a.fac, sF);
  L::stage_pop(a.fac, sP);
  for (int i = threadIdx.x; i < a.nsteps; i += blockDim.x) {
    sSrc[i] = a.src[a.step0 + 1 + i];
    sSrcl[i] = a.src[a.nt + 1 + a.step0 + 1 + i];
  }

  const int lid = threadIdx.x;
  const int W = blockDim.x;
  const int lane = lid & 63, wave = lid >> 6, nwave = W >> 6;
  const int64_t base = (int64_t)blockIdx.x * a.owned - a.halo;
  const int64_t g = base + lid;
  const bool in_dom = g >= 0 && g < a.nx;
  const bool is_med = g >= a.mb && g < a.me;
  const bool tile_med = (base < a.me) && (base + W > a.mb);
  const bool has_right = (base <= a.nx - 1) && (base + W > a.nx - 1);
  const bool owned = in_dom && lid >= a.halo && lid < a.halo + a.owned;
  const int64_t c = g - a.mb;
  const int64_t nmed = a.me - a.mb;

  for (int k = 0; k < REC; ++k) sY[(size_t)lid * REC + k] = 0;

  // split K - I into bf16 parts in the A-operand layout:
  // lane holds A[16 mb + lane%16][32 kb + 8 (lane/16) + i], i = 0..7
  bf16x8_t Ah[MB][KB], Am[MB][KB], Al[MB][KB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int m = 16 * mb + (lane & 15), k = 32 * kb + 8 * (lane >> 4) + i;
        float x = 0.0f;
        if (m < D && k < D) x = cld(a.fac.Km, m * D + k);
        const float xl = (m < D && k < D) ? cld(a.fac.Km_lo, m * D + k) : 0.0f;
        const unsigned short h = f2bf(x);
        const float r1 = (x - bf2f(h)) + xl;
        const unsigned short md = f2bf(r1);
        const unsigned short lo = f2bf(r1 - bf2f(md));
        Ah[mb][kb][i] = __builtin_bit_cast(__bf16, h);
        Am[mb][kb][i] = __builtin_bit_cast(__bf16, md);
        Al[mb][kb][i] = __builtin_bit_cast(__bf16, lo);
      }
  __syncthreads();

  // fields as float-float pairs (E, Elo), (H, Hlo)
  float E = 0, H = 0, Elo = 0, Hlo = 0;
  float z[D], zl[D];
  if (in_dom) {
    E = a.Ein[g];
    Elo = a.Ein[a.nx + g];
    if (g < a.nx - 1) {
      H = a.Hin[g];
      Hlo = a.Hin[a.nx + g];
    }
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    z[j] = is_med ? a.zin[j * a.ld + c] : 0.0f;
    zl[j] = is_med ? a.zin[(D + j) * a.ld + c] : 0.0f;
  }

  int64_t snap_next = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = n == snap_next;
    const int b = s & 1;
    sE[b][lid] = E;
    sEl[b][lid] = Elo;
    __syncthreads();
    const float Er = (lid + 1 < W) ? sE[b][lid + 1] : 0.0f;
    const float El = (lid > 0) ? sE[b][lid - 1] : 0.0f;
    const float Erl = (lid + 1 < W) ? sEl[b][lid + 1] : 0.0f;
    const float Ell = (lid > 0) ? sEl[b][lid - 1] : 0.0f;
    if (in_dom && g < a.nx - 1) add_comp(H, Hlo, a.ch * ((Er - E) + (Erl - Elo)));
    float P = 0.0f;
    if (tile_med && is_med) {
      if (a.tape && owned && n >= a.tape_step0) {
        float *tp = a.tape + (n - a.tape_step0) * (D + 1) * a.ld + c;
#pragma unroll
        for (int j = 0; j < D; ++j) tp[j * a.ld] = z[j];
        tp[D * a.ld] = E;
      }
      // compensated rotation y'' = Rot(y) + (Rot - I) zr
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        float sn, cm;
        sincm1(fmaf(sF[L::oth + p], E, sF[L::otl + p] * E), sn, cm);
        const float y0 = z[2 * p], y1 = z[2 * p + 1];
        const float r0 = sF[L::ozr + 2 * p], r1 = sF[L::ozr + 2 * p + 1];
        add_comp(z[2 * p], zl[2 * p], (cm * y0 + sn * y1) + (cm * r0 + sn * r1));
        add_comp(z[2 * p + 1], zl[2 * p + 1], (cm * y1 - sn * y0) + (cm * r1 - sn * r0));
      }
      if (snap && owned && a.pop_out) {
#pragma unroll
        for (int lv = 0; lv < N; ++lv) {
          double acc = sP[N * D + lv];
#pragma unroll
          for (int j = 0; j < D; ++j) acc += sP[lv * D + j] * ((double)z[j] + (double)zl[j]);
          a.pop_out[si * N * nmed + lv * nmed + c] = acc;
        }
      }
      P = a.fac.p0;
#pragma unroll
      for (int j = 0; j < D; ++j) P += sF[L::ow + j] * z[j];
      // split the high part of y'' into bf16 parts for the B operand; the
      // padding columns are rewritten as zeros (the result row overlays them)
      unsigned short *rec = sY + (size_t)lid * REC;
#pragma unroll
      for (int k8 = 0; k8 < 4 * KB; ++k8) {
        unsigned short ph[8], pm[8], pl[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int j = 8 * k8 + i;
          const float x = (j < D) ? z[j] : 0.0f;
          ph[i] = f2bf(x);
          const float r1 = x - bf2f(ph[i]);
          pm[i] = f2bf(r1);
          pl[i] = f2bf(r1 - bf2f(pm[i]));
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          rec[8 * k8 + i] = ph[i];
          rec[KP + 8 * k8 + i] = pm[i];
          if constexpr (NPART == 3) rec[2 * KP + 8 * k8 + i] = pl[i];
        }
      }
    }
    __syncthreads();
    // (K - I) y'' on the matrix cores: wave w takes 16-cell blocks w, w+nwave, ..
    if (tile_med) {
      for (int nb = wave; nb < W / 16; nb += nwave) {
        const int cell = 16 * nb + (lane & 15);
        floatx4_t acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = floatx4_t{0.0f, 0.0f, 0.0f, 0.0f};
        const unsigned short *rec = sY + (size_t)cell * REC;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          const int k0 = 32 * kb + 8 * (lane >> 4);
          const bf16x8_t Bh = *(const bf16x8_t *)&rec[k0];
          const bf16x8_t Bm = *(const bf16x8_t *)&rec[KP + k0];
          bf16x8_t Bl;
          if constexpr (NPART == 3) Bl = *(const bf16x8_t *)&rec[2 * KP + k0];
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            if constexpr (NPROD == 6) {
              acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al[mb][kb], Bh, acc[mb], 0, 0, 0);
              acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am[mb][kb], Bm, acc[mb], 0, 0, 0);
              acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah[mb][kb], Bl, acc[mb], 0, 0, 0);
            }
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am[mb][kb], Bh, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah[mb][kb], Bm, acc[mb], 0, 0, 0);
            acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah[mb][kb], Bh, acc[mb], 0, 0, 0);
          }
        }
        // C layout: lane holds rows 16 mb + 4 (lane/16) + j of column (cell);
        // all reads of this block's records are done (they fed acc)
        float *res = (float *)(sY + (size_t)cell * REC);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) *(floatx4_t *)&res[16 * mb + 4 * (lane >> 4)] = acc[mb];
      }
    }
    __syncthreads();
    if (tile_med && is_med) {
      const float *res = (const float *)(sY + (size_t)lid * REC);
#pragma unroll
      for (int i = 0; i < D; ++i) add_comp(z[i], zl[i], res[i] + (sF[L::oc + i] + sF[L::ocl + i]));
    }
    const float Eold = E, Eoldl = Elo;
    // H of the face left of this cell comes from the neighbour (LDS)
    sE[b][lid] = H;
    sEl[b][lid] = Hlo;
    __syncthreads();
    const float Hleft = (lid > 0) ? sE[b][lid - 1] : 0.0f;
    const float Hleftl = (lid > 0) ? sEl[b][lid - 1] : 0.0f;
    if (g >= 1 && g < a.nx - 1) {
      add_comp(E, Elo, a.cam1 * E + a.cb * (-P + ((H - Hleft) + (Hlo - Hleftl)) * a.inv_dx));
    } else if (g == 0) {
      E = sSrc[s];
      Elo = sSrcl[s];
    }
    if (has_right) {
      if (g == a.nx - 2) {
        sMur = E;
        sMurl = Elo;
      }
      __syncthreads();
      if (g == a.nx - 1) {
        E = El;
        Elo = Ell;
        add_comp(E, Elo, a.kmur * ((sMur - Eold) + (sMurl - Eoldl)));
        if (a.probe_out && owned) a.probe_out[n + 1] = (double)E + (double)Elo;
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
    a.Eout[a.nx + g] = Elo;
    if (g < a.nx - 1) {
      a.Hout[g] = H;
      a.Hout[a.nx + g] = Hlo;
    }
    if (is_med) {
#pragma unroll
      for (int j = 0; j < D; ++j) {
        a.zout[j * a.ld + c] = z[j];
        a.zout[(D + j) * a.ld + c] = zl[j];
      }
    }
  }
}

}  // namespace mln
