// fwd_kernels.hpp -- argument blocks and launchers of the forward kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mln {

enum { ROUTE_ROT = 0, ROUTE_DIAG = 1, ROUTE_RODR = 2, ROUTE_PADE = 3 };

constexpr int kMaxTile = 256;      // threads (= cells) per tile workgroup
constexpr int kMaxQuadTile = 256;  // cells per tile of the four-lanes-per-cell kernel
constexpr int64_t kQuadMaxAutoCells = 100000;  // automatic variant: quad kernel below this grid size
constexpr int kMaxStepsPerLaunch = 128;  // time steps fused into one launch (halo <= tile/2 < 128)
constexpr int kMaxAdjQuadTile = 128;    // cells per four-lanes-per-cell reverse tile (512 lanes)
constexpr int kStreamThreads = 256;       // threads per workgroup of the streamed kernel
constexpr int kStreamCells = 1;           // consecutive cells per thread of the streamed kernel
constexpr int kPadeMax = 7;              // highest Pade degree of the per-step Pade route
constexpr size_t kPadeMaxLds = 160 * 1024;  // LDS of one compute unit

// Launches of the one-cell-per-thread tile kernels with at least four tiles
// per compute unit fill the default register budget's occupancy (three to
// five 256-thread workgroups per unit), so they take the builds compiled for
// seven wavefronts per SIMD; launches with fewer tiles keep the default
// build, whose step does not pay for the spills of the smaller budget.
inline bool many_tiles(int64_t nblocks) {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = cus;
  }
  return nblocks >= 4 * (int64_t)cache[dev];
}

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
  const Real *Km_lo;  // D x D  low parts of Km, cz, thdt (compensated FP32 only)
  const Real *cz_lo;
  const Real *th_lo;
  const Real *zr;     // D      reference state of the rotation route (state is z' - zr)
  const Real *Up;     // kPadeMax x D x D  per-step Pade route: V^k, k = 1..kPadeMax, V = dt U / unorm
  Real unorm;         // ||dt U||_1 (X = E dt U = (E unorm) V)
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
  // Fields: E and H are nx values each; with compensated fields (CF) they
  // are float-float pairs, nx high parts followed by nx low parts, and so is
  // src.
  const Real *src;    // amplitude * samples[n], n = 0..nt (then the low parts with CF)
  int64_t nx, mb, me, ld;
  int64_t step0;
  int nsteps, halo, owned;
  Real ch, ca, cb, inv_dx, kmur;
  Real cam1;          // ca - 1 (rounded from the FP64 value)
  int64_t nt;         // source samples src[0..nt]
  int64_t snap_every;
  int64_t snap_next;  // first step index n >= step0 that completes a snapshot ((n+1) % snap_every == 0)
  int64_t snap_i0;    // snapshot index of that step
  double *pop_out, *e_out, *probe_out;
  // optional tape for the adjoint: z' (D rows, high parts) and E (1 row) of
  // every medium cell at every step n >= tape_step0, row stride ld
  Real *tape;
  int64_t tape_step0;
  // always 0; the kernels index the shared factor with (opaque0 * step) so that
  // its scalar loads stay inside the step loop for large D instead of being
  // hoisted into more SGPRs than exist
  int64_t opaque0;
};

// Reverse-time (adjoint) tile kernel arguments.  Adjoint fields lE (of E),
// lH (of H), lz (of z') use the same tiling as the forward kernel.
template <typename Real>
struct AdjArgs {
  FacDev<Real> fac;
  const Real *lEin;
  Real *lEout;
  const Real *lHin;
  Real *lHout;
  const Real *lzin;
  Real *lzout;
  const Real *tape;        // written by the forward kernel for steps >= tape_step0
  int64_t tape_step0;
  const double *gprobe;    // dJ/dprobe[n], n = 0..nt
  const double *samples;   // source samples s[n] (E at cell 0 = amplitude * s[n])
  int64_t nx, mb, me, ld;
  int64_t n_hi;            // this launch reverses steps n_hi-1 down to n_hi-nsteps
  int nsteps, halo, owned;
  Real ch, ca, cb, inv_dx, kmur;
  double *partial;         // [gridDim.x][nacc] per-tile gradient sums (accumulated)
};

template <typename Real>
struct BlochArgs {
  FacDev<Real> fac;
  int64_t opaque0;  // always 0 (see FwdArgs)
  const Real *z0;
  const double *efield;  // nsteps x ncell
  int64_t ncell, nsteps;
  double *pop_out, *dp_out;
};

// comp = true selects the compensated single-precision state (float only,
// rotation route only): z holds D rows of high parts followed by D rows of
// low parts.  cf = true (with comp) also carries E, H and the source samples
// as float-float pairs.
template <typename Real>
hipError_t launch_fwd(int N, int route, bool comp, bool cf, const FwdArgs<Real> &a, int64_t nblocks, int W,
                      hipStream_t st);
template <typename Real>
hipError_t launch_bloch(int N, int route, bool comp, const BlochArgs<Real> &a, hipStream_t st);

// Single-wavefront tile kernel of the rotation route (fwd_wave.hpp): 64 lanes,
// C cells per lane (C = 1, 2, 4 for N <= 4; C = 1 for N = 6).
template <typename Real>
hipError_t launch_fwd_wave(int N, bool comp, int C, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st);

// Workgroup tile kernel of the rotation route with the shared-factor GEMM on
// the matrix cores, split-BF16 with NPROD = 6 or 3 products (fwd_mfma.hpp);
// compensated FP32 state; N = 4 or 6; W = 64, 128 or 256 cells.
hipError_t launch_fwd_mfma(int N, int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st);
// The same transform with four lanes per cell (fwd_mfmaq.hpp): N = 4 or 6,
// W cells per tile (multiple of 16, at most 256), 4 W lanes; compensated
// state and fields.
hipError_t launch_fwd_mfmaq(int N, int nprod, const FwdArgs<float> &a, int64_t nblocks, int W, hipStream_t st);

// Per-step Pade route for N = 4 and 6 (fwd_pade.hpp): one wavefront per cell,
// 512 threads per workgroup, tile of a.owned + 2 a.halo <= 512 cells whose
// states sit in LDS (pade_lds_bytes(N, sizeof(Real), W) bytes, at most
// kPadeMaxLds); FP64 or plain FP32.
template <typename Real>
hipError_t launch_fwd_pade(int N, const FwdArgs<Real> &a, int64_t nblocks, hipStream_t st);
template <typename Real>
hipError_t launch_bloch_pade(int N, const BlochArgs<Real> &a, hipStream_t st);
size_t pade_lds_bytes(int N, int real_bytes, int W);

// Streamed one-step kernel of the rotation route (fwd_stream.hpp): one launch
// per time step (a.nsteps must be 1), one thread per cell; N = 2, 3, 4, 6;
// FP64, FP32 or the compensated FP32 state (plain fields).
template <typename Real>
hipError_t launch_fwd_stream(int N, bool comp, const FwdArgs<Real> &a, hipStream_t st);

// Four-lanes-per-cell tile kernel of the rotation route (fwd_quad.hpp), N <= 3;
// W cells per tile (W in 32..256, multiple of 16), 4 W threads; mf: the
// shared-factor product on the matrix cores.
template <typename Real>
hipError_t launch_fwd_quad(int N, bool comp, bool cf, bool mf, int W, const FwdArgs<Real> &a, int64_t nblocks,
                           hipStream_t st);

// Batched launch (fwd_batch.hpp): per-problem arguments for reading from
// ping-pong slot 0 and from slot 1 (step0, nsteps and the snapshot schedule
// are filled in per launch), and the workgroup -> (problem, tile) table.
template <typename Real>
struct BatchInst {
  FwdArgs<Real> a[2];
  int32_t n_levels;  // 2 or 3
  int32_t pad_;
};
struct BatchTile {
  int32_t inst;
  int32_t tile;
};

// Four-lanes-per-cell tiles of many problems (N = 2 and 3) in one launch of
// nblocks workgroups of 4 W lanes.  Real = double (plain) or float (plain or
// compensated).
template <typename Real>
hipError_t launch_fwd_quad_batch(bool comp, bool cf, int W, const BatchInst<Real> *inst, const BatchTile *tiles,
                                 int64_t nblocks, int64_t step0, int nsteps, int slot, hipStream_t st);

// Number of gradient accumulators per tile for N levels in precision Real:
// dJ/dK (D*D), dJ/dc (D), dJ/dw (D), dJ/dp0, dJ/damplitude, and the moments
// sum E^m lhat zhat^T for m = 1, 3 (and 5 in FP64), D*D each.
constexpr int adj_moments(bool fp64) { return fp64 ? 3 : 2; }
constexpr int adj_nacc(int N, bool fp64) {
  return (N * N - 1) * (N * N - 1) * (1 + adj_moments(fp64)) + 2 * (N * N - 1) + 2;
}

template <typename Real>
hipError_t launch_adj(int N, const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st);
// Four-lanes-per-cell adjoint kernel (adj_quad.hpp), N = 2 or 3, W <= 128
// cells per tile (4 W lanes, W a multiple of 16).
template <typename Real>
hipError_t launch_adj_quad(int N, const AdjArgs<Real> &a, int64_t nblocks, int W, hipStream_t st);

}  // namespace mln
