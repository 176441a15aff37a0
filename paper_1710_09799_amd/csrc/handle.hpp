// handle.hpp -- the state behind an mln_handle, shared by the single-problem
// ABI (mln_abi.hip) and the batched ABI (batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mln.h"
#include "fwd_kernels.hpp"
#include "mln_internal.hpp"

namespace mln {

// Record a message for mln_last_error() and return `code`.
int set_err(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_err(e_ == hipErrorOutOfMemory ? MLN_ENOMEM : MLN_EHIP,                 \
                     std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)

// A device allocation owned by the handle.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) {
    release();
    bytes = n;
    return hipMalloc(&p, n ? n : 1);
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Deep copy of an mln_medium (the handle keeps it for the adjoint's chain rule).
struct MediumCopy {
  std::vector<double> h0, mu, jump, rate, relax, rho0;
  mln_medium m{};
  void set(const mln_medium *src) {
    const int N = src->n_levels, NN = N * N;
    h0.assign(src->h0, src->h0 + 2 * NN);
    mu.assign(src->dipole, src->dipole + 2 * NN);
    rho0.assign(src->rho0, src->rho0 + 2 * NN);
    if (src->n_jump > 0) {
      jump.assign(src->jump, src->jump + 2 * NN * src->n_jump);
      rate.assign(src->jump_rate, src->jump_rate + src->n_jump);
    }
    if (src->relax_superop) relax.assign(src->relax_superop, src->relax_superop + 2 * NN * NN);
    m = *src;
    m.h0 = h0.data();
    m.dipole = mu.data();
    m.rho0 = rho0.data();
    m.jump = jump.empty() ? nullptr : jump.data();
    m.jump_rate = rate.empty() ? nullptr : rate.data();
    m.relax_superop = relax.empty() ? nullptr : relax.data();
  }
};

}  // namespace mln

struct mln_handle {
  using DevBuf = mln::DevBuf;
  mln::Factors f;
  mln::MediumCopy medium;
  mln_grid grid{};
  double amp = 0.0;
  std::vector<double> samples;
  int prec = MLN_FP64, route = MLN_ROUTE_ROTATION;
  bool comp = false;  // compensated FP32 state (two floats per component)
  bool cf = false;    // compensated FP32 fields and source samples (two floats each)
  int mfma = 0;       // split-BF16 products of the MFMA shared-factor kernel (6, 3) or 0
  hipStream_t stream = nullptr;
  int device = 0;  // the device current at mln_init
  int64_t nmed = 0, ld = 0, step = 0;
  int W = 256, halo = 0, owned = 0;  // cells per tile, halo = max steps per launch
  bool wave = false;                  // single-wavefront tile kernel (W = 64 * C cells)
  bool quad = false;                  // four-lanes-per-cell tile kernel (W cells, 4 W threads)
  bool qmf = false;                   // ... with the shared-factor product on the matrix cores
  bool streamed = false;              // one step per launch, state streamed through HBM
  int64_t ntiles = 0;
  int rs = 8;  // bytes per real of the state
  // device state (ping-pong)
  DevBuf E[2], H[2], z[2];
  int cur = 0;
  DevBuf src, fac, pop, popc;
  mln::FacDev<double> fd{};
  mln::FacDev<float> ff{};
  // recording
  mln_record rec{};
  int64_t nsnap = 0;
  DevBuf st_pop, st_e, st_probe;  // device staging for host outputs
  double *d_pop = nullptr, *d_e = nullptr, *d_probe = nullptr;
  // initial state on the host
  std::vector<unsigned char> z_init, e_init;
  // checkpoints of the forward run (for the adjoint)
  int64_t ckpt_every = 0, nckpt = 0, ckpt_count = 0;
  bool ckpt_ok = false;
  // the whole forward tape kept in device memory (ckpt_every = MLN_TAPE_ALL):
  // mln_run writes z' and E of every step, mln_grad reverses without
  // recomputation; tape_ok while the run so far started at step 0 untouched
  bool tape_all = false, tape_ok = false;
  DevBuf ckpt;
  // adjoint buffers (allocated by the first mln_grad)
  DevBuf lE[2], lH[2], lz[2], tape, partial, gprobe, samples_dev;
  // with checkpoints, mln_grad rebuilds the next segment on aux_stream into
  // the other tape buffer (tape2) while the current one is reversed;
  // ev_rec[b] / ev_rev[b]: tape buffer b written / read
  DevBuf tape2;
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  double fd_coef[6] = {0, 0, 0, 0, 0, 0};  // ch, ca, cb, inv_dx, kmur, ca - 1
  // the same coefficients for the single-precision kernels: ch and inv_dx
  // chosen so that ch * cb * inv_dx (the squared Courant number that sets the
  // phase velocity of the Yee scheme) matches the FP64 product far below FP32
  // rounding; H is then carried in units scaled by ch32 / ch, undone by
  // h_scale32 = ch / ch32 where H leaves the library
  float fc32[6] = {0, 0, 0, 0, 0, 0};
  double h_scale32 = 1.0;
  // mln_run from step 0 (no checkpoints, no tape) replays one HIP graph of
  // the run's launches, captured on a private stream on first use and
  // dropped when the kernel configuration changes
  bool use_graph = true;
  // reverse-kernel tiling (mln_configure_adjoint): variant 0 = automatic
  int adj_variant = 0, adj_W = 0, adj_K = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t run_graph = nullptr;
  hipGraphExec_t run_exec = nullptr;
  void drop_graph() {
    if (run_exec) (void)hipGraphExecDestroy(run_exec);
    if (run_graph) (void)hipGraphDestroy(run_graph);
    run_exec = nullptr;
    run_graph = nullptr;
  }
  ~mln_handle() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (aux_stream) {
      (void)hipStreamSynchronize(aux_stream);
      (void)hipStreamDestroy(aux_stream);
    }
    for (hipEvent_t e : {ev_start, ev_rec[0], ev_rec[1], ev_rev[0], ev_rev[1]})
      if (e) (void)hipEventDestroy(e);
  }
};

namespace mln {

// Restore the initial state (step 0) of the handle.  Synchronises the stream.
int reset_state(mln_handle *h);
// After the last step: synchronise, copy host-side outputs back and check the
// probe for non-finite values.
int finish_run(mln_handle *h);

// FDTD coefficients in the precision of the kernels.
inline void fdtd_coefs(const mln_handle *h, double &ch, double &ca, double &cb, double &inv_dx, double &kmur,
                       double &cam1) {
  ch = h->fd_coef[0]; ca = h->fd_coef[1]; cb = h->fd_coef[2];
  inv_dx = h->fd_coef[3]; kmur = h->fd_coef[4]; cam1 = h->fd_coef[5];
}
inline void fdtd_coefs(const mln_handle *h, float &ch, float &ca, float &cb, float &inv_dx, float &kmur,
                       float &cam1) {
  ch = h->fc32[0]; ca = h->fc32[1]; cb = h->fc32[2];
  inv_dx = h->fc32[3]; kmur = h->fc32[4]; cam1 = h->fc32[5];
}

// Upload the factors of `route` (FP64 Factors f at time step dt) in precision
// Real into fac (factor block), pop and popc (FP64 population maps); fd then
// points into them.
template <typename Real>
int upload_factors(const Factors &f, int route, double dt, DevBuf &fac, DevBuf &pop, DevBuf &popc,
                   FacDev<Real> &fd);

// Fill h->fc32 and h->h_scale32 from h->fd_coef.
void tune_fp32_coefs(mln_handle *h);
// Single-precision H coefficient ch32 and 1/dx (inv_dx32) within 256 ulps of
// their rounded values whose product with the rounded cb is closest to the
// FP64 product ch * cb * inv_dx (the Yee scheme's phase velocity); H is then
// carried scaled by ch32 / ch.
void courant_pair32(double ch, double cb, double inv_dx, float &ch32, float &inv_dx32);

template <typename Real>
inline FwdArgs<Real> make_args(mln_handle *h, const FacDev<Real> &fd, int64_t step0, int nsteps,
                        bool record = true, Real *tape = nullptr, int64_t tape_step0 = 0) {
  FwdArgs<Real> a{};
  a.fac = fd;
  const int in = h->cur, out = 1 - h->cur;
  a.Ein = (const Real *)h->E[in].p;
  a.Eout = (Real *)h->E[out].p;
  a.Hin = (const Real *)h->H[in].p;
  a.Hout = (Real *)h->H[out].p;
  a.zin = (const Real *)h->z[in].p;
  a.zout = (Real *)h->z[out].p;
  a.src = (const Real *)h->src.p;
  a.nx = h->grid.nx;
  a.mb = h->grid.med_begin;
  a.me = h->grid.med_end;
  a.ld = h->ld;
  a.step0 = step0;
  a.nsteps = nsteps;
  a.halo = h->halo;
  a.owned = h->owned;
  fdtd_coefs(h, a.ch, a.ca, a.cb, a.inv_dx, a.kmur, a.cam1);
  a.nt = h->grid.nt;
  a.snap_every = record ? h->rec.snap_every : 0;
  // first step n >= step0 with (n+1) % snap_every == 0, and its snapshot index
  a.snap_next = -1;
  a.snap_i0 = 0;
  if (a.snap_every > 0) {
    const int64_t k = step0 / a.snap_every;  // snapshots completed before step0
    a.snap_next = (k + 1) * a.snap_every - 1;
    a.snap_i0 = k;
  }
  a.pop_out = record ? h->d_pop : nullptr;
  a.e_out = record ? h->d_e : nullptr;
  a.probe_out = record ? h->d_probe : nullptr;
  a.tape = tape;
  a.tape_step0 = tape_step0;
  a.opaque0 = 0;
  return a;
}

}  // namespace mln
