// fwd_pstd.hpp -- the coupled time step with a pseudo-spectral (PSTD) field
// solver on a periodic grid (the paper names PSTD as a field solver its
// Liouville treatment combines with: Introduction, Sec. 4).
//
// One workgroup advances one problem of nx cells (nx a power of two); a
// launch of n_inst workgroups advances n_inst independent problems that share
// the grid.  Per step, in the staggered leapfrog of the Yee kernels:
//   H^{n+1/2} = H^{n-1/2} + (dt / mu) D+ E^n      D+ = d/dx at x_i + dx/2
//   P         = Liouville cell step with E^n        (rotation route, Sec. 4.1)
//   E^{n+1}   = ca E^n + cb (-P + D- H^{n+1/2})     D- = d/dx at x_i
// D+ and D- multiply the Fourier mode of wavenumber kappa by
// i kappa exp(+-i kappa dx / 2) (H sits half a cell to the right of E); the
// Nyquist mode is dropped.
//
// Layout (all of it in one workgroup's registers and LDS):
//   * thread t owns cells t + c T, c < C (T = nx / C threads): E^n and the
//     Bloch state of those cells live in registers for the whole launch;
//   * H lives in Fourier space for the whole launch, each mode pair
//     (k, M - k), M = nx / 2, in the registers of one thread, so a step takes
//     one forward and one inverse FFT; H returns to real space at the end of
//     the launch;
//   * a real signal f of length nx is packed into M complex values
//     z_j = f_{2j} + i f_{2j+1} (the half-length transform of real data):
//     the packed buffer is simply the nx reals in cell order;
//   * forward FFT: radix-2 decimation in frequency, natural order in,
//     bit-reversed order out; the mode-wise step works in bit-reversed order;
//     inverse FFT: decimation in time, bit-reversed order in, natural order
//     out, so no permutation pass is needed;
//   * LDS holds the packed buffer, swizzled (element i at i ^ 5 ((i >> 4) & 3):
//     the groups of the short-span passes and contiguous runs alike then fall
//     on distinct 16-byte bank slots), and tables laid out in the order the
//     lanes read them: per radix-4 pass its twiddles W_4h^j, j < h, and per
//     mode pair its unpacking factor exp(-2 pi i k / nx) and half-cell shift
//     exp(-i pi k / nx).
#pragma once

#include "fwd_impl.hpp"

namespace mln {

constexpr int kPstdMinCells = 64;

struct PstdInst {
  FacDev<double> fac;
  double *E;        // nx: E_i at x_i = i dx (updated in place)
  double *H;        // nx: H_i at x_i + dx / 2 (updated in place)
  double *z;        // D x ld: rotation-route state of the medium cells (in place)
  double *probe;    // nt + 1 samples of E_{nx-1}, or null
  double *e_out;    // snapshots x nx, or null
  double *pop_out;  // snapshots x N x nmed, or null
};

struct PstdArgs {
  const PstdInst *inst;
  const double2 *tab;  // pass twiddles (pt_size), then per mode pair u < M/2 its
                       // exp(-2 pi i k / nx), then its exp(-i pi k / nx)
  int pt_size;
  int64_t nx, mb, me, ld;
  int log2m;           // M = nx / 2 = 2^log2m
  int nsteps;
  int64_t step0;
  int64_t snap_every, snap_next, snap_i0;
  double ca, cb;
  double ah;           // (dt / mu) 2 pi / (nx dx): H-update factor per unit of k
  double be;           // (cb / M) 2 pi / (nx dx): E-update factor per unit of k
  int64_t opaque0;     // 0 at run time (keeps per-step factor loads inside the loop)
};

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 c_mulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i * a
__device__ __forceinline__ double2 c_i(double2 a) { return make_double2(-a.y, a.x); }

// Slot of packed element i in LDS: an XOR of bits 0-3 by 5 ((i >> 4) & 3), a
// bijection inside every block of 16 elements.
__device__ __forceinline__ int psw(int i) { return i ^ (((i >> 4) & 3) * 5); }

// Slot (in reals) of cell i's value in the packed buffer: element i / 2,
// real part for even i, imaginary part for odd i.
__device__ __forceinline__ int pstd_real_slot(int64_t i) { return 2 * psw((int)(i >> 1)) + (int)(i & 1); }

// Twiddles W_4h^j (j < h) of the radix-4 pass of span h start at
// (h - h0) / 3 in the pass table (h0 = 1 or 2: the smallest span; the spans
// of the passes grow by factors of 4).
__device__ __forceinline__ int pstd_pt_off(int h, int lm) { return (h - ((lm & 1) ? 2 : 1)) / 3; }

// Number of pass-table entries for a transform of length 2^lm.
__host__ __device__ inline int pstd_pt_size(int lm) { return ((1 << lm) - ((lm & 1) ? 2 : 1)) / 3; }

// Position of mode k in the bit-reversed output of the forward transform.
__device__ __forceinline__ int pstd_pos(int k, int lm) { return (int)(__brev((unsigned)k) >> (32 - lm)); }

// The mode pairs (k, M - k), k = 1 .. M/2, are numbered u = 0 .. M/2 - 1 by
// the position of k: u = 0 is k = M/2 (position 1, its own partner), u > 0
// the even position 2u (k = rev(2u) < M/2).  Consecutive threads then touch
// consecutive positions (and the partners, whose positions are those of k
// with the low bits inverted, nearly so) instead of positions M/2 apart,
// which would put a whole wavefront on the same LDS banks.
__device__ __forceinline__ int pstd_pair_pos(int u) { return u ? 2 * u : 1; }
__device__ __forceinline__ int pstd_pair_k(int u, int lm) { return pstd_pos(pstd_pair_pos(u), lm); }

// -i * a
__device__ __forceinline__ double2 c_mi(double2 a) { return make_double2(a.y, -a.x); }

// Unnormalised forward DFT of length M = 2^lm in place (exp(-2 pi i j k / M)):
// natural order in, bit-reversed order out.  The radix-2 stages of
// decimation in frequency (span half = M/2 down to 1) run two at a time:
// one pass over groups i0 + {0, h, 2h, 3h}, i0 mod 4h = j < h, applies the
// stage of span 2h (twiddles W_4h^j and W_4h^(j+h) = -i W_4h^j) and then
// the stage of span h (twiddle W_2h^j = (W_4h^j)^2), W_L = exp(-2 pi i / L).
// An odd stage count leaves the span-1 stage (twiddle 1) for last.  Ends
// with a barrier.
__device__ __forceinline__ void pstd_fft_dif(double2 *buf, const double2 *pt, int lm, int lh_first = -1) {
  const int M = 1 << lm;
  int lh = lh_first < 0 ? lm - 1 : lh_first;
  for (; lh >= 1; lh -= 2) {
    const int lq = lh - 1, h = 1 << lq;
    const double2 *tw = pt + pstd_pt_off(h, lm);
    for (int q = threadIdx.x; q < M / 4; q += blockDim.x) {
      const int j = q & (h - 1);
      const int i0 = ((q >> lq) << (lq + 2)) | j;
      const int s0 = psw(i0), s1 = psw(i0 + h), s2 = psw(i0 + 2 * h), s3 = psw(i0 + 3 * h);
      const double2 a0 = buf[s0], a1 = buf[s1], a2 = buf[s2], a3 = buf[s3];
      const double2 w1 = tw[j];
      const double2 w2 = c_mul(w1, w1);
      const double2 b0 = c_add(a0, a2), b1 = c_add(a1, a3);
      const double2 b2 = c_mul(c_sub(a0, a2), w1);
      const double2 b3 = c_mi(c_mul(c_sub(a1, a3), w1));
      buf[s0] = c_add(b0, b1);
      buf[s1] = c_mul(c_sub(b0, b1), w2);
      buf[s2] = c_add(b2, b3);
      buf[s3] = c_mul(c_sub(b2, b3), w2);
    }
    __syncthreads();
  }
  if (lh == 0) {
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int s0 = psw(2 * b), s1 = psw(2 * b + 1);
      const double2 u = buf[s0], v = buf[s1];
      buf[s0] = c_add(u, v);
      buf[s1] = c_sub(u, v);
    }
    __syncthreads();
  }
}

// Unnormalised inverse DFT of length M in place (exp(+2 pi i j k / M)):
// bit-reversed order in, natural order out.  Decimation in time, spans
// 1, 2, ..., M/2: the span-1 stage alone first when the stage count is odd,
// then two stages per pass (span h with twiddle conj W_2h^j, then span 2h
// with conj W_4h^j and conj W_4h^(j+h) = i conj W_4h^j).  Ends with a
// barrier.
__device__ __forceinline__ void pstd_fft_dit_inv(double2 *buf, const double2 *pt, int lm, bool skip_last = false) {
  const int M = 1 << lm;
  const int lh_end = skip_last ? lm - 2 : lm;  // passes with lh + 1 < lh_end
  int lh = 0;
  if (lm & 1) {
    for (int b = threadIdx.x; b < M / 2; b += blockDim.x) {
      const int s0 = psw(2 * b), s1 = psw(2 * b + 1);
      const double2 u = buf[s0], v = buf[s1];
      buf[s0] = c_add(u, v);
      buf[s1] = c_sub(u, v);
    }
    __syncthreads();
    lh = 1;
  }
  for (; lh + 1 < lh_end; lh += 2) {
    const int h = 1 << lh;
    const double2 *tw = pt + pstd_pt_off(h, lm);
    for (int q = threadIdx.x; q < M / 4; q += blockDim.x) {
      const int j = q & (h - 1);
      const int i0 = ((q >> lh) << (lh + 2)) | j;
      const int s0 = psw(i0), s1 = psw(i0 + h), s2 = psw(i0 + 2 * h), s3 = psw(i0 + 3 * h);
      const double2 a0 = buf[s0], a1 = buf[s1], a2 = buf[s2], a3 = buf[s3];
      const double2 u1 = c_conj(tw[j]);
      const double2 v = c_mul(u1, u1);
      const double2 t1 = c_mul(a1, v), t3 = c_mul(a3, v);
      const double2 b0 = c_add(a0, t1), b1 = c_sub(a0, t1);
      const double2 b2 = c_add(a2, t3), b3 = c_sub(a2, t3);
      const double2 q2 = c_mul(b2, u1);
      const double2 q3 = c_i(c_mul(b3, u1));
      buf[s0] = c_add(b0, q2);
      buf[s2] = c_sub(b0, q2);
      buf[s1] = c_add(b1, q3);
      buf[s3] = c_sub(b1, q3);
    }
    __syncthreads();
  }
}

// Exchange a double with the other lane of the pair (2e, 2e + 1) (DPP
// quad_perm [1, 0, 3, 2] on both halves).
__device__ __forceinline__ double pstd_pair_swap(double x) {
  constexpr int ctrl = 1 | (0 << 2) | (3 << 4) | (2 << 6);
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), ctrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), ctrl, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// With C >= 4 cells per thread (thread t owns cells t + c T, M = C T / 2),
// the lanes 2e and 2e + 1 hold the real and the imaginary parts of the
// packed elements e + c T / 2, which are C / 4 whole groups of the first
// forward pass and of the last inverse pass (span-M/4 radix 4: elements
// q + r M / 4, q = e + g T / 2, r < 4, from cells c = g + r C / 4).  Those
// passes then run on the cells' own values: a complex product needs the
// other lane's component, one pair exchange, and with sg = -1 on the real
// and +1 on the imaginary lane it reads own * w.x + sg * other * w.y.

// First forward pass from the values x of the thread's cells; writes the
// pass's outputs (this lane's components).  No barrier.
template <int C>
__device__ __forceinline__ void pstd_dif_first_regs(double *bufd, const double2 *pt, int lm, int T, int t,
                                                    const double (&x)[C]) {
  static_assert(C % 4 == 0, "whole groups per thread");
  const int h = 1 << (lm - 2);
  const double2 *tw = pt + pstd_pt_off(h, lm);
  const int p = t & 1, e0 = t >> 1;
  const double sg = p ? 1.0 : -1.0;
#pragma unroll
  for (int g = 0; g < C / 4; ++g) {
    const int q = e0 + g * (T / 2);
    const double a0 = x[g], a1 = x[g + C / 4], a2 = x[g + C / 2], a3 = x[g + 3 * C / 4];
    const double2 w1 = tw[q];
    const double2 w2 = c_mul(w1, w1);
    const double b0 = a0 + a2, b1 = a1 + a3;
    const double d02 = a0 - a2, d13 = a1 - a3;
    const double o02 = pstd_pair_swap(d02), o13 = pstd_pair_swap(d13);
    const double b2 = d02 * w1.x + sg * o02 * w1.y;         // (a0 - a2) w1
    const double b3 = d13 * w1.y - sg * o13 * w1.x;         // (a1 - a3) (-i w1)
    const double d01 = b0 - b1, d23 = b2 - b3;
    const double o01 = pstd_pair_swap(d01), o23 = pstd_pair_swap(d23);
    bufd[2 * psw(q) + p] = b0 + b1;
    bufd[2 * psw(q + h) + p] = d01 * w2.x + sg * o01 * w2.y;
    bufd[2 * psw(q + 2 * h) + p] = b2 + b3;
    bufd[2 * psw(q + 3 * h) + p] = d23 * w2.x + sg * o23 * w2.y;
  }
}

// Last inverse pass: reads the pass's inputs and returns this lane's
// component of the outputs for the thread's cells in y.
template <int C>
__device__ __forceinline__ void pstd_dit_last_regs(const double2 *buf, const double2 *pt, int lm, int T, int t,
                                                   double (&y)[C]) {
  static_assert(C % 4 == 0, "whole groups per thread");
  const int h = 1 << (lm - 2);
  const double2 *tw = pt + pstd_pt_off(h, lm);
  const int p = t & 1, e0 = t >> 1;
#pragma unroll
  for (int g = 0; g < C / 4; ++g) {
    const int q = e0 + g * (T / 2);
    const double2 a0 = buf[psw(q)], a1 = buf[psw(q + h)], a2 = buf[psw(q + 2 * h)], a3 = buf[psw(q + 3 * h)];
    const double2 u1 = c_conj(tw[q]);
    const double2 v = c_mul(u1, u1);
    const double2 t1 = c_mul(a1, v), t3 = c_mul(a3, v);
    const double2 b0 = c_add(a0, t1), b1 = c_sub(a0, t1);
    const double2 b2 = c_add(a2, t3), b3 = c_sub(a2, t3);
    const double2 q2 = c_mul(b2, u1);
    const double2 q3 = c_i(c_mul(b3, u1));
    const double2 c0 = c_add(b0, q2), c1 = c_add(b1, q3), c2 = c_sub(b0, q2), c3 = c_sub(b1, q3);
    y[g] = p ? c0.y : c0.x;
    y[g + C / 4] = p ? c1.y : c1.x;
    y[g + C / 2] = p ? c2.y : c2.x;
    y[g + 3 * C / 4] = p ? c3.y : c3.x;
  }
}

// Modes k and M - k of the length-nx DFT F of a real signal from its packed
// transform Z: with w = exp(-2 pi i k / nx), S = (Z_k + conj Z_{M-k}) / 2 and
// Dd = (Z_k - conj Z_{M-k}) / 2, F_k = S - i w Dd and conj F_{M-k} = S + i w Dd.
__device__ __forceinline__ void pstd_unpack(double2 Zk, double2 Zm, double2 w, double2 &Fk, double2 &Fm) {
  const double2 S = c_scale(c_add(Zk, c_conj(Zm)), 0.5);
  const double2 Dd = c_scale(c_sub(Zk, c_conj(Zm)), 0.5);
  const double2 iwD = c_i(c_mul(w, Dd));
  Fk = c_sub(S, iwD);
  Fm = c_conj(c_add(S, iwD));
}

// Inverse of pstd_unpack: the packed spectrum of a real signal from its DFT
// modes k and M - k (even part Xe, odd part Xo: Z_k = Xe + i Xo,
// Z_{M-k} = conj Xe + i conj Xo).
__device__ __forceinline__ void pstd_pack(double2 Gk, double2 Gm, double2 w, double2 &Zk, double2 &Zm) {
  const double2 Xe = c_scale(c_add(Gk, c_conj(Gm)), 0.5);
  const double2 Xo = c_scale(c_mulc(c_sub(Gk, c_conj(Gm)), w), 0.5);
  Zk = c_add(Xe, c_i(Xo));
  Zm = c_add(c_conj(Xe), c_i(c_conj(Xo)));
}

// N levels, C cells per thread (blockDim.x = nx / C <= TMAX threads).  With
// TMAX = 256 a workgroup is one wavefront per SIMD, which may hold up to 512
// registers per lane (VGPRs and AGPRs); with 512, two per SIMD share them.
template <int N, int C, int TMAX>
__global__ void __launch_bounds__(TMAX) fwd_pstd_kernel(PstdArgs a) {
  constexpr int D = N * N - 1;
  constexpr int R = (C + 3) / 4;  // mode pairs per thread: (M / 2) / T rounded up
  using L = RotLds<N, double, false>;
  extern __shared__ double2 pstd_lds[];
  __shared__ double sF[L::size];
  __shared__ double sP[N * D + N];
  const int lm = a.log2m, M = 1 << lm;
  double2 *buf = pstd_lds;            // M packed elements, swizzled
  double *bufd = reinterpret_cast<double *>(buf);
  double2 *pt = pstd_lds + M;         // pass twiddles
  double2 *mw = pt + a.pt_size;       // per mode pair: exp(-2 pi i k / nx)
  double2 *me = mw + M / 2;           //                exp(-i pi k / nx)
  const PstdInst in = a.inst[blockIdx.x];
  const int T = blockDim.x, t = threadIdx.x;
  const int64_t nx = a.nx, nmed = a.me - a.mb;

  L::stage(in.fac, sF);
  L::stage_pop(in.fac, sP);
  for (int i = t; i < a.pt_size + M; i += T) pt[i] = a.tab[i];

  double E[C];
  double z[C][D];
  double zl[1] = {0.0};
  // first and last passes on the cells' own values, where the registers
  // leave room for them (whole groups per thread, at most 32 state
  // components per thread: N = 2 with 4 or 8 cells, N = 3 with 4)
  constexpr bool REG = C % 4 == 0 && D * C <= 32;
  constexpr int CR = REG ? C : 1;
  double Hc[CR];  // with REG: H of the thread's cells (at entry and at exit)
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t i = t + (int64_t)c * T;
    E[c] = in.E[i];
    const bool med = i >= a.mb && i < a.me;
#pragma unroll
    for (int j = 0; j < D; ++j) z[c][j] = med ? in.z[j * a.ld + (i - a.mb)] : 0.0;
    if constexpr (REG)
      Hc[c] = in.H[i];
    else
      bufd[pstd_real_slot(i)] = in.H[i];
  }
  __syncthreads();  // also orders the tables
  if constexpr (REG) {
    pstd_dif_first_regs<C>(bufd, pt, lm, T, t, Hc);
    __syncthreads();
  }

  // H into Fourier space: modes k and M - k of the pairs this thread owns;
  // the k = 0 slot (DC and Nyquist modes, which no update touches) is kept
  // as packed for the way back.
  pstd_fft_dif(buf, pt, lm, REG ? lm - 3 : -1);
  double2 hk[R], hm[R];
  double2 h0 = make_double2(0.0, 0.0);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int u = t + r * T;
    hk[r] = hm[r] = make_double2(0.0, 0.0);
    if (u < M / 2) {
      const int k = pstd_pair_k(u, lm);
      pstd_unpack(buf[psw(pstd_pair_pos(u))], buf[psw(pstd_pos(M - k, lm))], mw[u], hk[r], hm[r]);
    }
  }
  if (t == 0) h0 = buf[0];
  __syncthreads();

  int64_t snap_next = a.snap_next, si = a.snap_i0;
  for (int s = 0; s < a.nsteps; ++s) {
    const int64_t n = a.step0 + s;
    const bool snap = n == snap_next;
    int ts = t;  // per-step copy: addresses are recomputed, not held across steps
    asm volatile("" : "+v"(ts));
    if constexpr (REG) {
      pstd_dif_first_regs<C>(bufd, pt, lm, T, ts, E);
    } else {
#pragma unroll
      for (int c = 0; c < C; ++c) bufd[pstd_real_slot(ts + c * T)] = E[c];
    }
    __syncthreads();
    pstd_fft_dif(buf, pt, lm, REG ? lm - 3 : -1);
    // Mode-wise: H += (dt / mu) i kappa e^{+i kappa dx / 2} F(E^n); then the
    // packed spectrum of (cb / M) D- H for the inverse transform.  With
    // e = exp(-i pi k / nx): e^{+i kappa_k dx / 2} = conj e and
    // e^{+i kappa_{M-k} dx / 2} = i e.
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = t + r * T;
      if (u < M / 2) {
        const int k = pstd_pair_k(u, lm);
        const int pk = psw(pstd_pair_pos(u)), pm = psw(pstd_pos(M - k, lm));
        const double2 w = mw[u];
        const double2 e = me[u];
        double2 Fk, Fm;
        pstd_unpack(buf[pk], buf[pm], w, Fk, Fm);
        const double kk = (double)k, km = (double)(M - k);
        hk[r] = c_add(hk[r], c_scale(c_i(c_mul(c_conj(e), Fk)), a.ah * kk));
        hm[r] = c_sub(hm[r], c_scale(c_mul(e, Fm), a.ah * km));
        const double2 Gk = c_scale(c_i(c_mul(e, hk[r])), a.be * kk);
        const double2 Gm = c_scale(c_mul(c_conj(e), hm[r]), a.be * km);
        double2 Zk, Zm;
        pstd_pack(Gk, Gm, w, Zk, Zm);
        buf[pk] = Zk;
        buf[pm] = Zm;
      }
    }
    if (t == 0) buf[0] = make_double2(0.0, 0.0);
    __syncthreads();
    pstd_fft_dit_inv(buf, pt, lm, REG);
    double Dh[CR];  // with REG: (cb / M) D- H of the thread's cells
    if constexpr (REG) pstd_dit_last_regs<C>(buf, pt, lm, T, ts, Dh);
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t i = ts + (int64_t)c * T;
      double P = 0.0;
      if (i >= a.mb && i < a.me) {
        const int64_t cm = i - a.mb;
        double *pp = (snap && in.pop_out) ? in.pop_out + si * N * nmed + cm : nullptr;
        P = cell_step<N, double, ROUTE_ROT, false>(in.fac, sF, sP, E[c], z[c], zl, pp, nmed, a.opaque0 * s);
      }
      double dh;
      if constexpr (REG)
        dh = Dh[c];
      else
        dh = bufd[pstd_real_slot(i)];
      E[c] = a.ca * E[c] - a.cb * P + dh;
      if (i == nx - 1 && in.probe) in.probe[n + 1] = E[c];
      if (snap && in.e_out) in.e_out[si * nx + i] = E[c];
    }
    if (snap) {
      snap_next += a.snap_every;
      ++si;
    }
    // No barrier here: the next step writes E^{n+1} into exactly the slots
    // of the buffer that this thread (or, with REG, the other lane of its
    // pair, in the same wavefront and so in order) has just read, which no
    // other thread touches before the barrier that follows those writes.
  }

  // H back to real space (after every thread has read its last D- H)
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int u = t + r * T;
    if (u < M / 2) {
      const int k = pstd_pair_k(u, lm);
      double2 Zk, Zm;
      pstd_pack(hk[r], hm[r], mw[u], Zk, Zm);
      buf[psw(pstd_pair_pos(u))] = Zk;
      buf[psw(pstd_pos(M - k, lm))] = Zm;
    }
  }
  if (t == 0) buf[0] = h0;
  __syncthreads();
  pstd_fft_dit_inv(buf, pt, lm, REG);
  if constexpr (REG) pstd_dit_last_regs<C>(buf, pt, lm, T, t, Hc);
  const double inv_m = 1.0 / (double)M;
  // a fresh copy of the thread index, so that the write-back addresses are
  // computed here rather than kept live from the loads at entry
  int tb = t;
  asm volatile("" : "+v"(tb));
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int64_t i = tb + (int64_t)c * T;
    if constexpr (REG)
      in.H[i] = Hc[c] * inv_m;
    else
      in.H[i] = bufd[pstd_real_slot(i)] * inv_m;
    in.E[i] = E[c];
    if (i >= a.mb && i < a.me) {
#pragma unroll
      for (int j = 0; j < D; ++j) in.z[j * a.ld + (i - a.mb)] = z[c][j];
    }
  }
}

}  // namespace mln
