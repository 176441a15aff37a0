// mln_abi.hip -- the C ABI declared in include/mln.h: validation, one-time
// factor upload, device state, the launch loop over fused time steps,
// recording and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "handle.hpp"

using namespace mln;

namespace {
thread_local std::string g_last_error;
}  // namespace

// ---- device scratch of the no-allocation entry point --------------------
// mln_bloch_only stages the initial Bloch state of the prescribed-field run in
// a small device buffer it allocates per call; mln_bloch_only_noalloc stages
// it here instead.  Each device holds its own copy of this array (its address
// differs per device) until the process ends.  In host code the array's name
// is not a device address: the address is looked up with hipGetSymbolAddress
// once per device (in mln_init, with that device current) and only that
// address is used (copies, kernel arguments).
static __device__ __align__(256) unsigned char scratch[MLN_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Address of `scratch` on the current device, resolved on first use.
int scratch_setup(int *device) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_err(MLN_ENOTSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(MLN_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *device = dev;
  return MLN_OK;
}

void *scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_dev[device] : nullptr;
}
}  // namespace

int mln::set_err(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}


// The Yee update advances E by cb * inv_dx * (H_{i+1/2} - H_{i-1/2}) and H by
// ch * (E_{i+1} - E_i), so the discrete wave speed depends on the product
// ch * cb * inv_dx (the squared Courant number over eps_r mu_r).  Rounding the
// three factors to FP32 independently leaves that product off by up to
// ~1.8e-7 relative, a systematic phase-velocity error whose effect on E grows
// with the distance travelled (about 1e-5 after 50 wavelengths).  cb also
// scales the polarisation term and keeps its rounded value; ch and inv_dx are
// searched within +-256 ulps of their rounded values for the pair whose
// product with cb is closest to the FP64 value (typically within 1e-10).
// inv_dx appears nowhere else; a different ch rescales the carried H, which
// mln_get_fields undoes.
void mln::courant_pair32(double ch, double cb, double inv_dx, float &ch32, float &inv_dx32) {
  const long double target = (long double)ch * cb * inv_dx;
  const float cbf = (float)cb;
  float best_ch = (float)ch, best_idx = (float)inv_dx;
  long double best = std::fabs((long double)best_ch * best_idx * cbf - target);
  constexpr int K = 256;
  float c = (float)ch;
  for (int i = 0; i < K; ++i) c = std::nextafter(c, 0.0f);
  for (int i = -K; i <= K; ++i, c = std::nextafter(c, 2.0f * c)) {
    float idx = (float)inv_dx;
    for (int j = 0; j < K; ++j) idx = std::nextafter(idx, 0.0f);
    for (int j = -K; j <= K; ++j, idx = std::nextafter(idx, 2.0f * idx)) {
      const long double e = std::fabs((long double)c * idx * cbf - target);
      if (e < best) {
        best = e;
        best_ch = c;
        best_idx = idx;
      }
    }
  }
  ch32 = best_ch;
  inv_dx32 = best_idx;
}

void mln::tune_fp32_coefs(mln_handle *h) {
  const double *c = h->fd_coef;
  for (int i = 0; i < 6; ++i) h->fc32[i] = (float)c[i];
  courant_pair32(c[0], c[2], c[3], h->fc32[0], h->fc32[3]);
  h->h_scale32 = c[0] / (double)h->fc32[0];
}

// Upload the factors of the chosen route in precision Real.  The layout of
// the device block is a concatenation of arrays; FacDev points into it.
template <typename Real>
int mln::upload_factors(const Factors &f, int route, double dt, DevBuf &fac, DevBuf &pop, DevBuf &popc,
                        FacDev<Real> &fd) {
  const int D = f.D, q = f.q;
  std::vector<Real> blk;
  auto push = [&](const std::vector<double> &v) {
    size_t off = blk.size();
    for (double x : v) blk.push_back((Real)x);
    while (blk.size() % 16) blk.push_back(0);
    return off;
  };
  const bool rot = route == MLN_ROUTE_ROTATION;
  std::vector<double> Km = rot ? f.K : f.A;
  for (int i = 0; i < D; ++i) Km[i * D + i] -= 1.0;
  std::vector<double> thdt(q), rre(D * D), rim(D * D), lamdt(D);
  for (int p = 0; p < q; ++p) thdt[p] = f.theta[p] * dt;
  for (int i = 0; i < D * D; ++i) {
    rre[i] = f.R[i].real();
    rim[i] = f.R[i].imag();
  }
  for (int k = 0; k < D; ++k) lamdt[k] = f.lam[k].imag() * dt;
  size_t oK = push(Km), oc = push(rot ? f.rz : f.c), ow = push(rot ? f.wz : f.w);
  size_t oth = push(thdt), orr = push(rre), ori = push(rim), ol = push(lamdt);
  size_t oS = push(f.S), oS2 = push(f.S2);
  size_t ozr = push(rot ? f.zr : std::vector<double>(D, 0.0));
  // per-step Pade route: ||dt U||_1 and the powers V^k, k = 1..kPadeMax, of
  // V = dt U / ||dt U||_1, so that X = E dt U = (E ||dt U||_1) V with both
  // factors of order one (powers of E itself overflow single precision)
  std::vector<double> Up;
  double unorm = 0.0;
  if (route == MLN_ROUTE_PADE) {
    for (int j = 0; j < D; ++j) {
      double cs = 0.0;
      for (int i = 0; i < D; ++i) cs += std::fabs(f.U[i * D + j] * dt);
      unorm = std::max(unorm, cs);
    }
    const double vs = unorm > 0.0 ? dt / unorm : 0.0;
    std::vector<double> V(D * D), P(D * D);
    for (int i = 0; i < D * D; ++i) V[i] = P[i] = f.U[i] * vs;
    Up.assign((size_t)kPadeMax * D * D, 0.0);
    for (int k = 0; k < kPadeMax; ++k) {
      std::copy(P.begin(), P.end(), Up.begin() + (size_t)k * D * D);
      std::vector<double> nP(D * D, 0.0);
      for (int i = 0; i < D; ++i)
        for (int l = 0; l < D; ++l)
          for (int j = 0; j < D; ++j) nP[i * D + j] += P[i * D + l] * V[l * D + j];
      P.swap(nP);
    }
  }
  size_t oUp = push(Up);
  // low parts x - (float)x of the factors the compensated state uses
  auto lo_of = [](const std::vector<double> &v) {
    std::vector<double> r(v.size());
    for (size_t i = 0; i < v.size(); ++i) r[i] = v[i] - (double)(Real)v[i];
    return r;
  };
  const std::vector<double> &cvec = rot ? f.rz : f.c;
  size_t oKl = push(lo_of(Km)), ocl = push(lo_of(cvec)), otl = push(lo_of(thdt));
  HIP_TRY(fac.alloc(blk.size() * sizeof(Real)));
  HIP_TRY(hipMemcpy(fac.p, blk.data(), blk.size() * sizeof(Real), hipMemcpyHostToDevice));
  const Real *b = (const Real *)fac.p;
  fd.Km = b + oK;
  fd.cz = b + oc;
  fd.wz = b + ow;
  fd.thdt = b + oth;
  fd.Rre = b + orr;
  fd.Rim = b + ori;
  fd.lamdt = b + ol;
  fd.S = b + oS;
  fd.S2 = b + oS2;
  fd.Km_lo = b + oKl;
  fd.cz_lo = b + ocl;
  fd.th_lo = b + otl;
  fd.zr = b + ozr;
  fd.Up = b + oUp;
  fd.unorm = (Real)unorm;
  fd.p0 = (Real)(rot ? f.pr : f.p0);
  const std::vector<double> &pm = rot ? f.popz : f.popd;
  HIP_TRY(pop.alloc(pm.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(pop.p, pm.data(), pm.size() * sizeof(double), hipMemcpyHostToDevice));
  const std::vector<double> &pc = rot ? f.popcy : f.popc;
  HIP_TRY(popc.alloc(pc.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(popc.p, pc.data(), pc.size() * sizeof(double), hipMemcpyHostToDevice));
  fd.pop = (const double *)pop.p;
  fd.popc = (const double *)popc.p;
  return MLN_OK;
}

template int mln::upload_factors<double>(const Factors &, int, double, DevBuf &, DevBuf &, DevBuf &,
                                         FacDev<double> &);
template int mln::upload_factors<float>(const Factors &, int, double, DevBuf &, DevBuf &, DevBuf &,
                                        FacDev<float> &);

namespace {

template <typename Real>
int upload_factors(mln_handle *h, FacDev<Real> &fd) {
  return mln::upload_factors<Real>(h->f, h->route, h->grid.dt, h->fac, h->pop, h->popc, fd);
}

template <typename Real>
void build_init_state(mln_handle *h) {
  const Factors &f = h->f;
  const int D = f.D;
  const std::vector<double> &s0 = (h->route == MLN_ROUTE_ROTATION) ? f.y0 : f.dprime0;
  const int rows = h->comp ? 2 * D : D;
  h->z_init.assign(sizeof(Real) * rows * h->ld, 0);
  Real *zi = (Real *)h->z_init.data();
  for (int j = 0; j < D; ++j)
    for (int64_t c = 0; c < h->nmed; ++c) {
      zi[j * h->ld + c] = (Real)s0[j];
      if (h->comp) zi[(D + j) * h->ld + c] = (Real)(s0[j] - (double)(Real)s0[j]);
    }
  // E (and with the compensated state its low parts after nx high parts)
  const int64_t nx = h->grid.nx;
  h->e_init.assign(sizeof(Real) * (h->cf ? 2 : 1) * nx, 0);
  const double e0 = h->amp * h->samples[0];
  ((Real *)h->e_init.data())[0] = (Real)e0;
  if (h->cf) ((Real *)h->e_init.data())[nx] = (Real)(e0 - (double)(Real)e0);
}

size_t state_slot_bytes(const mln_handle *h) { return h->E[0].bytes + h->H[0].bytes + h->z[0].bytes; }

// copy the current forward state into checkpoint slot k, or back
int ckpt_copy(mln_handle *h, int64_t k, bool save) {
  unsigned char *slot = (unsigned char *)h->ckpt.p + k * state_slot_bytes(h);
  DevBuf *bufs[3] = {&h->E[h->cur], &h->H[h->cur], &h->z[h->cur]};
  size_t off = 0;
  for (DevBuf *b : bufs) {
    if (save)
      HIP_TRY(hipMemcpyAsync(slot + off, b->p, b->bytes, hipMemcpyDeviceToDevice, h->stream));
    else
      HIP_TRY(hipMemcpyAsync(b->p, slot + off, b->bytes, hipMemcpyDeviceToDevice, h->stream));
    off += b->bytes;
  }
  return MLN_OK;
}

// Advance the forward state from h->step by n steps in launches of at most
// `halo` steps that never cross a checkpoint boundary; saves checkpoints when
// the run started from step 0.
int forward_steps(mln_handle *h, int64_t n, bool record, void *tape, int64_t tape_step0, bool save_ckpt) {
  while (n > 0) {
    int64_t k = std::min<int64_t>(n, h->halo);
    if (h->ckpt_every > 0) {
      const int64_t r = h->step % h->ckpt_every;
      if (save_ckpt && r == 0 && h->ckpt_ok && h->step / h->ckpt_every == h->ckpt_count) {
        int rc = ckpt_copy(h, h->ckpt_count, true);
        if (rc) return rc;
        ++h->ckpt_count;
      }
      k = std::min<int64_t>(k, h->ckpt_every - r);
    }
    hipError_t e;
    if (h->streamed) {
      if (h->prec == MLN_FP64) {
        auto args = make_args<double>(h, h->fd, h->step, 1, record, (double *)tape, tape_step0);
        e = launch_fwd_stream<double>(h->f.N, false, args, h->stream);
      } else {
        auto args = make_args<float>(h, h->ff, h->step, 1, record, (float *)tape, tape_step0);
        e = launch_fwd_stream<float>(h->f.N, h->comp, args, h->stream);
      }
    } else if (h->prec == MLN_FP64) {
      auto args = make_args<double>(h, h->fd, h->step, (int)k, record, (double *)tape, tape_step0);
      e = h->quad   ? launch_fwd_quad<double>(h->f.N, false, false, h->qmf, h->W, args, h->ntiles, h->stream)
          : h->wave ? launch_fwd_wave<double>(h->f.N, false, h->W / 64, args, h->ntiles, h->stream)
                    : launch_fwd<double>(h->f.N, h->route, false, false, args, h->ntiles, h->W, h->stream);
    } else {
      auto args = make_args<float>(h, h->ff, h->step, (int)k, record, (float *)tape, tape_step0);
      e = (h->mfma && h->quad) ? launch_fwd_mfmaq(h->f.N, h->mfma, args, h->ntiles, h->W, h->stream)
          : h->mfma ? launch_fwd_mfma(h->f.N, h->mfma, args, h->ntiles, h->W, h->stream)
          : h->quad ? launch_fwd_quad<float>(h->f.N, h->comp, h->cf, h->qmf, h->W, args, h->ntiles, h->stream)
          : h->wave ? launch_fwd_wave<float>(h->f.N, h->comp, h->W / 64, args, h->ntiles, h->stream)
                    : launch_fwd<float>(h->f.N, h->route, h->comp, h->cf, args, h->ntiles, h->W, h->stream);
    }
    if (e != hipSuccess) return set_err(MLN_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    h->cur = 1 - h->cur;
    h->step += k;
    n -= k;
  }
  return MLN_OK;
}

// Choose and validate the forward kernel (variant 0: automatic) and its
// tiling (0: defaults); sets the tile bookkeeping of the handle.
int set_kernel(mln_handle *h, int variant_req, int tile, int steps_per_launch) {
  if (variant_req < 0 || variant_req > 5) return set_err(MLN_EINVAL, "unknown kernel variant");
  h->drop_graph();
  const bool rot = h->route == MLN_ROUTE_ROTATION;
  int variant = variant_req;
  if (variant == 4) {
    // streamed: one step per launch, one thread per cell
    if (!rot || h->cf || h->mfma)
      return set_err(MLN_ENOTSUPPORTED,
                     "the streamed kernel runs the rotation route in FP64, FP32 or compensated FP32");
    if ((tile != 0 && tile != kStreamThreads) || steps_per_launch > 1)
      return set_err(MLN_EINVAL, "the streamed kernel takes tile 0 or 256 and one step per launch");
    h->streamed = true;
    h->quad = h->wave = h->qmf = false;
    h->W = kStreamThreads;
    h->halo = 1;
    h->owned = kStreamThreads;
    h->ntiles = (h->grid.nx + kStreamThreads - 1) / kStreamThreads;
    return MLN_OK;
  }
  h->streamed = false;
  // automatic choice: four lanes per cell while the grid is too small to
  // fill the chip with one cell per thread (the step is latency-bound there,
  // and four lanes give four times the wavefronts); one cell per thread on
  // large grids, where the quad's replicated field work costs issue slots
  // (measured crossover near 1e5 cells at N = 2, 3)
  if (variant == 0) {
    variant = !rot ? 1 : (h->f.N <= 3 ? (h->grid.nx < kQuadMaxAutoCells ? 3 : 1) : (h->f.N == 4 && !h->cf ? 2 : 1));
    // the matrix-core product pays off with the compensated state at N = 3
    // and with compensated fields (measured; FP64 and plain FP32 run faster
    // on the DPP product, whose FMA chain is shorter than the MFMA latency)
    if (variant == 3 && !h->mfma && h->comp && (h->f.N == 3 || h->cf)) variant = 5;
  }
  if (h->mfma) {
    // one cell per thread (1) or four lanes per cell (3, the default)
    if (variant_req == 0) variant = 3;
    if (variant != 1 && variant != 3)
      return set_err(MLN_ENOTSUPPORTED, "the split-BF16 MFMA kernels are workgroup-tile or four-lanes-per-cell kernels");
  }
  // variant 5: the four-lanes-per-cell kernel with its shared-factor
  // product on the matrix cores (N <= 3, FP64 / FP32 / compensated modes)
  h->qmf = variant == 5;
  if (h->qmf && (h->mfma || h->f.N > 3))
    return set_err(MLN_ENOTSUPPORTED, "the matrix-core quad kernel is built for N <= 3 in FP64 and FP32 modes");
  if (h->qmf) variant = 3;
  h->wave = variant == 2;
  if (h->wave && h->cf)
    return set_err(MLN_ENOTSUPPORTED, "the wavefront kernel keeps E and H in plain precision");
  h->quad = variant == 3;
  if ((h->wave || h->quad) && !rot)
    return set_err(MLN_ENOTSUPPORTED, "the wavefront and quad kernels implement the rotation route");
  if (h->quad && h->f.N > 3 && !h->mfma)
    return set_err(MLN_ENOTSUPPORTED, "the quad kernel is built for N <= 3 (N = 4, 6: split-BF16 precisions)");
  // the per-step Pade route for N >= 4 keeps the tile's states in LDS and is
  // bound by arithmetic: smaller tiles, short halos
  const bool pade_wave = h->route == MLN_ROUTE_PADE && h->f.N >= 4;
  h->W = tile > 0 ? tile : ((h->quad && !h->mfma) || pade_wave ? 128 : kMaxTile);
  if (h->quad) {
    if (h->W > kMaxQuadTile || h->W < 32 || h->W % 16)
      return set_err(MLN_EINVAL, "quad kernel tile must be a multiple of 16 in [32, 256]");
  } else if (h->W > kMaxTile || h->W < 64 || h->W % 64) {
    return set_err(MLN_EINVAL, "tile must be a multiple of 64 in [64, 256]");
  }
  if (h->wave && (h->W == 192 || (h->f.N == 6 && h->W != 64)))
    return set_err(MLN_ENOTSUPPORTED, "wavefront kernel tiles: 64, 128 or 256 cells (64 for N = 6)");
  int K = steps_per_launch > 0
              ? steps_per_launch
              : (pade_wave ? 8 : (h->wave ? h->W / 8 : (h->mfma ? 16 : (h->quad ? h->W / 4 : 32))));
  if (steps_per_launch <= 0 && h->quad) {
    // the quad kernels: a step costs about the same with any number of
    // tiles up to about one per compute unit, and every launch has a fixed
    // cost (prologue, epilogue, kernel boundary), so take the largest step
    // count that keeps the tiles within the compute units.  Matrix-core
    // forms: even counts up to 24 at N = 3, 30 at N = 4, 6, tiles up to the
    // unit count; DPP form: up to 56, tiles up to 9/10 of the units (on
    // 20000 cells 20 steps and 228 tiles beat 24 steps and 250 tiles by 7 %;
    // on 2000 cells 56 steps run 1.3x faster than 16).  Larger grids keep
    // the fixed default above.
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
      cus = 256;
    const bool mf = h->qmf || h->mfma;
    const int kmax = std::min(mf ? (h->qmf ? 24 : 30) : 56, (h->W - 1) / 2);
    const int64_t maxtiles = mf ? cus : cus * 9 / 10;
    for (int k = mf ? kmax & ~1 : kmax; k >= 8; k -= mf ? 2 : 1)
      if ((h->grid.nx + (h->W - 2 * k) - 1) / (h->W - 2 * k) <= maxtiles) {
        K = k;
        break;
      }
  }
  if (2 * K >= h->W || K > kMaxStepsPerLaunch)
    return set_err(MLN_EINVAL, "steps_per_launch must be below tile/2 (and at most 128)");
  if (pade_wave && pade_lds_bytes(h->f.N, h->rs, h->W) > kPadeMaxLds)
    return set_err(MLN_EINVAL, "tile too large for the LDS of the per-step Pade kernel");
  h->halo = K;
  h->owned = h->W - 2 * K;
  h->ntiles = (h->grid.nx + h->owned - 1) / h->owned;
  return MLN_OK;
}

// Capture the launches of a whole run from step 0 (forward_steps enqueues
// kernels only when there are no checkpoints or tape) on the private capture
// stream; nothing runs during the capture, so step and ping-pong slot are
// restored afterwards.
int capture_run(mln_handle *h) {
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  hipStream_t user = h->stream;
  h->stream = h->cap_stream;
  hipError_t e = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    h->stream = user;
    return set_err(MLN_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  int rc = forward_steps(h, h->grid.nt, true, nullptr, 0, false);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(h->cap_stream, &g);
  h->stream = user;
  h->step = 0;
  h->cur = 0;
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : set_err(MLN_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  h->run_graph = g;
  e = hipGraphInstantiate(&h->run_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    h->drop_graph();
    return set_err(MLN_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  return MLN_OK;
}

int validate_grid(const mln_grid *g, const mln_source *s) {
  if (!g || !s) return set_err(MLN_EINVAL, "null grid or source");
  if (g->nx < 3) return set_err(MLN_EINVAL, "nx must be >= 3");
  if (g->nt < 0) return set_err(MLN_EINVAL, "nt must be >= 0");
  if (!(g->dx > 0) || !(g->dt > 0) || !std::isfinite(g->dx) || !std::isfinite(g->dt))
    return set_err(MLN_EINVAL, "dx and dt must be positive");
  if (g->med_begin < 1 || g->med_end < g->med_begin || g->med_end > g->nx - 1)
    return set_err(MLN_EINVAL, "medium must satisfy 1 <= med_begin <= med_end <= nx-1");
  if (!(g->eps_r > 0) || !(g->mu_r > 0) || !(g->sigma >= 0))
    return set_err(MLN_EINVAL, "eps_r, mu_r must be > 0 and sigma >= 0");
  double cl = 1.0 / std::sqrt(kEps0 * g->eps_r * kMu0 * g->mu_r);
  if (cl * g->dt / g->dx > 1.0 + 1e-12) return set_err(MLN_ECOURANT, "Courant number c dt/dx exceeds 1");
  if (!s->samples || s->n_samples < g->nt + 1)
    return set_err(MLN_EINVAL, "source needs nt+1 samples");
  if (!std::isfinite(s->amplitude)) return set_err(MLN_EINVAL, "non-finite source amplitude");
  for (int64_t i = 0; i <= g->nt; ++i)
    if (!std::isfinite(s->samples[i])) return set_err(MLN_EINVAL, "non-finite source sample");
  return MLN_OK;
}

template <typename Real>
int init_typed(mln_handle *h, FacDev<Real> &fd) {
  int rc = upload_factors<Real>(h, fd);
  if (rc) return rc;
  const int64_t nx = h->grid.nx;
  const int D = h->f.D;
  // source samples (then their low parts with the compensated state)
  const int64_t ns = h->grid.nt + 1;
  std::vector<Real> src((h->cf ? 2 : 1) * ns);
  for (int64_t i = 0; i < ns; ++i) {
    const double v = h->amp * h->samples[i];
    src[i] = (Real)v;
    if (h->cf) src[ns + i] = (Real)(v - (double)(Real)v);
  }
  HIP_TRY(h->src.alloc(src.size() * sizeof(Real)));
  HIP_TRY(hipMemcpy(h->src.p, src.data(), src.size() * sizeof(Real), hipMemcpyHostToDevice));
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(h->E[b].alloc((h->cf ? 2 : 1) * nx * sizeof(Real)));
    HIP_TRY(h->H[b].alloc((h->cf ? 2 : 1) * nx * sizeof(Real)));
    HIP_TRY(h->z[b].alloc((size_t)(h->comp ? 2 * D : D) * h->ld * sizeof(Real)));
  }
  build_init_state<Real>(h);
  return MLN_OK;
}

}  // namespace

int mln::reset_state(mln_handle *h) {
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(hipMemsetAsync(h->H[b].p, 0, h->H[b].bytes, h->stream));
    HIP_TRY(hipMemcpyAsync(h->E[b].p, h->e_init.data(), h->e_init.size(), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->z[b].p, h->z_init.data(), h->z_init.size(), hipMemcpyHostToDevice, h->stream));
  }
  h->cur = 0;
  h->step = 0;
  h->ckpt_count = 0;
  h->ckpt_ok = h->ckpt_every > 0;
  h->tape_ok = h->tape_all;
  if (h->d_probe) {
    double p0 = (h->grid.nx - 1 == 0) ? h->amp * h->samples[0] : 0.0;
    HIP_TRY(hipMemcpyAsync(h->d_probe, &p0, sizeof(double), hipMemcpyHostToDevice, h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return MLN_OK;
}

int mln::finish_run(mln_handle *h) {
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (!h->rec.out_on_device) {
    const int N = h->f.N;
    if (h->st_pop.p)
      HIP_TRY(hipMemcpy(h->rec.pop_out, h->st_pop.p, sizeof(double) * h->nsnap * N * h->nmed, hipMemcpyDeviceToHost));
    if (h->st_e.p)
      HIP_TRY(hipMemcpy(h->rec.e_out, h->st_e.p, sizeof(double) * h->nsnap * h->grid.nx, hipMemcpyDeviceToHost));
    if (h->st_probe.p)
      HIP_TRY(hipMemcpy(h->rec.probe_out, h->st_probe.p, sizeof(double) * (h->grid.nt + 1), hipMemcpyDeviceToHost));
    if (h->rec.probe_out)
      for (int64_t i = 0; i <= h->grid.nt; ++i)
        if (!std::isfinite(h->rec.probe_out[i])) return set_err(MLN_ENONFINITE, "non-finite probe value");
  }
  return MLN_OK;
}

extern "C" {

int mln_version(void) { return 100; }

const char *mln_last_error(void) { return g_last_error.c_str(); }

const char *mln_strerror(int code) {
  switch (code) {
    case MLN_OK: return "ok";
    case MLN_EINVAL: return "invalid argument";
    case MLN_ENOTHERMITIAN: return "operator is not Hermitian";
    case MLN_ENOTTRACEPRESERVING: return "relaxation superoperator is not trace preserving";
    case MLN_ECOURANT: return "Courant condition violated";
    case MLN_EBADRHO: return "initial density matrix is not a valid state";
    case MLN_ENOMEM: return "out of memory";
    case MLN_EHIP: return "HIP runtime error";
    case MLN_ENOTSUPPORTED: return "not supported";
    case MLN_ENONFINITE: return "non-finite value in the output";
    case MLN_ESTATE: return "call not valid in this state";
    case MLN_ENUMERIC: return "factorisation failed";
    default: return "unknown error";
  }
}

int mln_setup_factors(const mln_medium *medium, double dt, mln_factors *out) {
  if (!out) return set_err(MLN_EINVAL, "null output");
  Factors f;
  std::string err;
  int rc = build_factors(medium, dt, &f, &err);
  if (rc) return set_err(rc, err);
  auto put = [](double *dst, const std::vector<double> &v) {
    if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(double));
  };
  auto putc = [](double *dst, const std::vector<cplx> &v) {
    if (dst)
      for (size_t i = 0; i < v.size(); ++i) {
        dst[2 * i] = v[i].real();
        dst[2 * i + 1] = v[i].imag();
      }
  };
  putc(out->gen, f.gen);
  put(out->M, f.M);
  put(out->U, f.U);
  put(out->deq, f.deq);
  put(out->v, f.v);
  put(out->d0, f.d0);
  put(out->A0, f.A0);
  put(out->b0, f.b0);
  put(out->T, f.T);
  put(out->theta, f.theta);
  putc(out->R, f.R);
  putc(out->lam, f.lam);
  put(out->S, f.S);
  put(out->K, f.K);
  put(out->c, f.cz);
  put(out->w, f.wz);
  if (out->p0) *out->p0 = f.p0;
  return MLN_OK;
}

int mln_chain_rule(const mln_medium *medium, double dt, const double *gA, const double *gc,
                   const double *gw, double gp0, const double *gU, const double *gd0,
                   mln_grads *out) {
  if (!gA || !gc || !gw || !gU || !gd0) return set_err(MLN_EINVAL, "null gradient input");
  std::string err;
  int rc = chain_rule(medium, dt, gA, gc, gw, gp0, gU, gd0, out, &err);
  if (rc) return set_err(rc, err);
  return MLN_OK;
}

int mln_init(const mln_medium *medium, const mln_grid *grid, const mln_source *source,
             const mln_record *record, const mln_options *options, mln_handle **out) {
  if (!out) return set_err(MLN_EINVAL, "null output handle");
  *out = nullptr;
  int rc = validate_grid(grid, source);
  if (rc) return rc;
  std::unique_ptr<mln_handle> h(new mln_handle());
  rc = scratch_setup(&h->device);
  if (rc) return rc;
  std::string err;
  rc = build_factors(medium, grid->dt, &h->f, &err);
  if (rc) return set_err(rc, err);
  h->medium.set(medium);
  h->grid = *grid;
  h->amp = source->amplitude;
  h->samples.assign(source->samples, source->samples + grid->nt + 1);
  mln_options opt{};
  if (options) opt = *options;
  h->prec = opt.precision;
  h->route = opt.route;
  h->stream = (hipStream_t)opt.stream;
  if (h->route < 0 || h->route > 3) return set_err(MLN_EINVAL, "unknown route");
  if (h->f.N == 5) return set_err(MLN_ENOTSUPPORTED, "kernels are built for N = 2, 3, 4 and 6");
  if (h->prec < MLN_FP64 || h->prec > MLN_FP32_FIELDS)
    return set_err(MLN_ENOTSUPPORTED, "unknown precision");
  h->comp = h->prec >= MLN_FP32_COMP && h->prec <= MLN_FP32_COMP_FIELDS;
  h->mfma = h->prec == MLN_FP32_BF16SPLIT ? 6 : (h->prec == MLN_FP32_BF16X3 ? 3 : 0);
  h->cf = h->prec == MLN_FP32_COMP_FIELDS || h->prec == MLN_FP32_FIELDS || h->mfma;
  if ((h->comp || h->cf) && h->route != MLN_ROUTE_ROTATION)
    return set_err(MLN_ENOTSUPPORTED, "the compensated FP32 state and fields are built for the rotation route only");
  if (h->prec == MLN_FP32_FIELDS && h->f.N > 3)
    return set_err(MLN_ENOTSUPPORTED, "MLN_FP32_FIELDS is built for N <= 3");
  if (h->mfma && h->f.N != 4 && h->f.N != 6)
    return set_err(MLN_ENOTSUPPORTED, "the split-BF16 MFMA kernel is built for N = 4 and 6");
  h->rs = (h->prec == MLN_FP64) ? 8 : 4;
  // FDTD coefficients (Eq. maxwell on the Yee grid, semi-implicit sigma)
  const double eps = kEps0 * grid->eps_r, mu = kMu0 * grid->mu_r;
  const double cl = 1.0 / std::sqrt(eps * mu);
  const double sg = grid->sigma * grid->dt / (2.0 * eps);
  h->fd_coef[0] = grid->dt / (mu * grid->dx);
  h->fd_coef[1] = (1.0 - sg) / (1.0 + sg);
  h->fd_coef[2] = (grid->dt / eps) / (1.0 + sg);
  h->fd_coef[3] = 1.0 / grid->dx;
  h->fd_coef[4] = (cl * grid->dt - grid->dx) / (cl * grid->dt + grid->dx);
  h->fd_coef[5] = -2.0 * sg / (1.0 + sg);
  tune_fp32_coefs(h.get());
  rc = set_kernel(h.get(), opt.variant, opt.tile, opt.steps_per_launch);
  if (rc) return rc;
  h->nmed = grid->med_end - grid->med_begin;
  h->ld = std::max<int64_t>(1, (h->nmed + 63) / 64 * 64);
  // recording
  h->rec = record ? *record : mln_record{};
  if (h->rec.snap_every < 0) return set_err(MLN_EINVAL, "snap_every must be >= 0");
  h->nsnap = h->rec.snap_every > 0 ? grid->nt / h->rec.snap_every : 0;
  const int N = h->f.N;
  if (h->rec.out_on_device) {
    h->d_pop = h->rec.pop_out;
    h->d_e = h->rec.e_out;
    h->d_probe = h->rec.probe_out;
  } else {
    if (h->rec.pop_out && h->nsnap) {
      HIP_TRY(h->st_pop.alloc(sizeof(double) * h->nsnap * N * std::max<int64_t>(h->nmed, 1)));
      h->d_pop = (double *)h->st_pop.p;
    }
    if (h->rec.e_out && h->nsnap) {
      HIP_TRY(h->st_e.alloc(sizeof(double) * h->nsnap * grid->nx));
      h->d_e = (double *)h->st_e.p;
    }
    if (h->rec.probe_out) {
      HIP_TRY(h->st_probe.alloc(sizeof(double) * (grid->nt + 1)));
      h->d_probe = (double *)h->st_probe.p;
    }
  }
  if (h->nsnap == 0) {
    h->d_pop = nullptr;
    h->d_e = nullptr;
  }
  rc = (h->prec == MLN_FP64) ? init_typed<double>(h.get(), h->fd) : init_typed<float>(h.get(), h->ff);
  if (rc) return rc;
  if (opt.ckpt_every < 0 && opt.ckpt_every != MLN_TAPE_ALL)
    return set_err(MLN_EINVAL, "ckpt_every must be >= 0 or MLN_TAPE_ALL");
  if (opt.ckpt_every == MLN_TAPE_ALL) {
    if (h->route != MLN_ROUTE_ROTATION || h->f.N > 3)
      return set_err(MLN_ENOTSUPPORTED, "the adjoint is built for the rotation route and N <= 3");
    h->tape_all = true;
    const size_t bytes = (size_t)h->rs * (h->f.D + 1) * (size_t)h->ld * (size_t)std::max<int64_t>(grid->nt, 1);
    HIP_TRY(h->tape.alloc(bytes));
  }
  h->ckpt_every = std::max<int32_t>(opt.ckpt_every, 0);
  if (h->ckpt_every > 0) {
    h->nckpt = (grid->nt + h->ckpt_every - 1) / h->ckpt_every;
    HIP_TRY(h->ckpt.alloc(std::max<int64_t>(h->nckpt, 1) * state_slot_bytes(h.get())));
  }
  rc = reset_state(h.get());
  if (rc) return rc;
  *out = h.release();
  return MLN_OK;
}

int mln_step(mln_handle *h, int64_t n_steps) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  if (n_steps < 0) return set_err(MLN_EINVAL, "n_steps must be >= 0");
  int64_t left = std::min<int64_t>(n_steps, h->grid.nt - h->step);
  if (h->tape_all && h->tape_ok) return forward_steps(h, left, true, h->tape.p, 0, true);
  return forward_steps(h, left, true, nullptr, 0, true);
}

int mln_run(mln_handle *h) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  int rc;
  if (h->use_graph && h->step == 0 && h->cur == 0 && h->grid.nt > 0 && h->ckpt_every == 0 && !h->tape_all) {
    if (!h->run_exec && (rc = capture_run(h))) return rc;
    HIP_TRY(hipGraphLaunch(h->run_exec, h->stream));
    const int64_t launches = h->streamed ? h->grid.nt : (h->grid.nt + h->halo - 1) / h->halo;
    h->step = h->grid.nt;
    h->cur = (int)(launches & 1);
  } else {
    rc = mln_step(h, h->grid.nt - h->step);
    if (rc) return rc;
  }
  return finish_run(h);
}

int mln_use_graph(mln_handle *h, int32_t on) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  h->use_graph = on != 0;
  return MLN_OK;
}

int mln_reset(mln_handle *h) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  return reset_state(h);
}

int mln_current_step(const mln_handle *h, int64_t *step) {
  if (!h || !step) return set_err(MLN_EINVAL, "null argument");
  *step = h->step;
  return MLN_OK;
}

namespace {
struct KernelChoice {
  bool quad, qmf, wave, streamed;
  int W, halo, owned;
  int64_t ntiles;
};
KernelChoice save_kernel(const mln_handle *h) {
  return {h->quad, h->qmf, h->wave, h->streamed, h->W, h->halo, h->owned, h->ntiles};
}
void restore_kernel(mln_handle *h, const KernelChoice &k) {
  h->quad = k.quad;
  h->qmf = k.qmf;
  h->wave = k.wave;
  h->streamed = k.streamed;
  h->W = k.W;
  h->halo = k.halo;
  h->owned = k.owned;
  h->ntiles = k.ntiles;
}
}  // namespace

int mln_configure(mln_handle *h, int32_t variant, int32_t tile, int32_t steps_per_launch) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  if (h->step != 0) return set_err(MLN_ESTATE, "configure a handle at step 0 (mln_reset)");
  const KernelChoice old = save_kernel(h);
  int rc = set_kernel(h, variant, tile, steps_per_launch);
  if (rc) restore_kernel(h, old);
  return rc;
}

int mln_tune(mln_handle *h, int32_t trial_steps, int32_t *variant, int32_t *tile, int32_t *steps_per_launch) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  if (h->step != 0) return set_err(MLN_ESTATE, "tune a handle at step 0 (mln_reset)");
  if (trial_steps < 1) return set_err(MLN_EINVAL, "trial_steps must be >= 1");
  // (variant, cells per tile, steps per launch; 0: the automatic step
  // count, the largest that keeps one tile per compute unit); candidates the
  // handle's precision, route or level count does not allow are skipped
  static const int cand[][3] = {{3, 64, 8},   {3, 128, 16}, {3, 128, 20}, {3, 128, 32}, {3, 256, 16},
                                {3, 256, 32}, {1, 64, 8},   {1, 128, 8},  {1, 128, 16}, {1, 128, 32},
                                {1, 256, 8},  {1, 256, 16}, {1, 256, 32}, {2, 64, 8},   {2, 128, 16},
                                {2, 256, 32}, {4, 256, 1},  {5, 64, 8},   {5, 128, 16}, {5, 128, 20},
                                {5, 128, 0},  {5, 128, 32}, {5, 256, 16}, {5, 256, 32}};
  const KernelChoice start = save_kernel(h);
  KernelChoice best_k = start;
  double best = INFINITY;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = MLN_OK;
  for (const auto &c : cand) {
    if (set_kernel(h, c[0], c[1], c[2]) != MLN_OK) continue;
    const int kk = h->halo;  // the resolved steps per launch
    // one warm-up launch, then whole launches, all within the run length
    const int64_t steps = std::max<int64_t>(2 * kk, (trial_steps + kk - 1) / kk * kk);
    if (steps + kk > h->grid.nt) continue;
    if ((rc = reset_state(h)) || (rc = forward_steps(h, kk, false, nullptr, 0, false))) break;
    if (hipEventRecord(e0, h->stream) != hipSuccess) { rc = set_err(MLN_EHIP, "event record"); break; }
    if ((rc = forward_steps(h, steps, false, nullptr, 0, false))) break;
    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = set_err(MLN_EHIP, "event synchronize");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms / (double)steps < best) {
      best = ms / (double)steps;
      best_k = save_kernel(h);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  restore_kernel(h, rc ? start : best_k);
  const int rc2 = reset_state(h);
  if (rc) return rc;
  if (rc2) return rc2;
  if (variant) *variant = h->streamed ? 4 : (h->qmf ? 5 : (h->quad ? 3 : (h->wave ? 2 : 1)));
  if (tile) *tile = h->W;
  if (steps_per_launch) *steps_per_launch = h->halo;
  return MLN_OK;
}

int mln_configure_adjoint(mln_handle *h, int32_t variant, int32_t tile, int32_t steps_per_launch) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  if (variant == 0) {
    if (tile || steps_per_launch) return set_err(MLN_EINVAL, "the automatic reverse tiling takes tile 0 and steps 0");
    h->adj_variant = h->adj_W = h->adj_K = 0;
    return MLN_OK;
  }
  if (variant != 1 && variant != 3)
    return set_err(MLN_EINVAL, "reverse-kernel variant must be 0 (automatic), 1 or 3");
  if (h->route != MLN_ROUTE_ROTATION || h->f.N > 3)
    return set_err(MLN_ENOTSUPPORTED, "the adjoint is built for the rotation route and N <= 3");
  const int W = tile > 0 ? tile : (variant == 1 ? kMaxTile : kMaxAdjQuadTile);
  if (variant == 1 ? (W < 64 || W > kMaxTile || W % 64) : (W < 16 || W > kMaxAdjQuadTile || W % 16))
    return set_err(MLN_EINVAL, variant == 1 ? "reverse tile must be a multiple of 64 in [64, 256]"
                                            : "reverse quad tile must be a multiple of 16 in [16, 128]");
  const int K = steps_per_launch > 0 ? steps_per_launch : W / 4;
  if (steps_per_launch < 0 || 2 * K >= W || K > kMaxStepsPerLaunch)
    return set_err(MLN_EINVAL, "reverse steps per launch must be in [1, tile/2)");
  h->adj_variant = variant;
  h->adj_W = W;
  h->adj_K = K;
  return MLN_OK;
}

int mln_get_config(const mln_handle *h, int32_t *variant, int32_t *tile, int32_t *steps_per_launch) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  if (variant) *variant = h->streamed ? 4 : (h->qmf ? 5 : (h->quad ? 3 : (h->wave ? 2 : 1)));
  if (tile) *tile = h->W;
  if (steps_per_launch) *steps_per_launch = h->halo;
  return MLN_OK;
}

int mln_get_fields(mln_handle *h, double *E, double *H) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int64_t nx = h->grid.nx;
  const int parts = h->cf ? 2 : 1;  // high parts, then low parts
  std::vector<unsigned char> buf(h->rs * nx * parts);
  auto conv = [&](double *dst, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
      if (h->rs == 8) {
        dst[i] = ((double *)buf.data())[i];
      } else {
        const float *f = (const float *)buf.data();
        dst[i] = (double)f[i] + (parts == 2 ? (double)f[nx + i] : 0.0);
      }
    }
  };
  if (E) {
    HIP_TRY(hipMemcpy(buf.data(), h->E[h->cur].p, buf.size(), hipMemcpyDeviceToHost));
    conv(E, nx);
  }
  if (H) {
    HIP_TRY(hipMemcpy(buf.data(), h->H[h->cur].p, buf.size(), hipMemcpyDeviceToHost));
    conv(H, nx - 1);
    if (h->rs == 4)
      for (int64_t i = 0; i < nx - 1; ++i) H[i] *= h->h_scale32;
  }
  return MLN_OK;
}

}  // extern "C"

namespace {

// Inverse of a D x D row-major matrix by Gauss-Jordan elimination with
// partial pivoting (FP64; false if singular).
bool invert(int D, const std::vector<double> &A, std::vector<double> &inv) {
  std::vector<double> a(A);
  inv.assign((size_t)D * D, 0.0);
  for (int i = 0; i < D; ++i) inv[(size_t)i * D + i] = 1.0;
  for (int c = 0; c < D; ++c) {
    int pr = c;
    for (int r = c + 1; r < D; ++r)
      if (std::fabs(a[(size_t)r * D + c]) > std::fabs(a[(size_t)pr * D + c])) pr = r;
    if (a[(size_t)pr * D + c] == 0.0) return false;
    for (int k = 0; k < D; ++k) {
      std::swap(a[(size_t)c * D + k], a[(size_t)pr * D + k]);
      std::swap(inv[(size_t)c * D + k], inv[(size_t)pr * D + k]);
    }
    const double piv = 1.0 / a[(size_t)c * D + c];
    for (int k = 0; k < D; ++k) {
      a[(size_t)c * D + k] *= piv;
      inv[(size_t)c * D + k] *= piv;
    }
    for (int r = 0; r < D; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * D + c];
      if (f == 0.0) continue;
      for (int k = 0; k < D; ++k) {
        a[(size_t)r * D + k] -= f * a[(size_t)c * D + k];
        inv[(size_t)r * D + k] -= f * inv[(size_t)c * D + k];
      }
    }
  }
  return true;
}

// Bloch vectors d (D x nmed, component-major) of the state after the
// completed steps.  The device carries, per cell, the state after the first
// L1 half step of the next step, d' = A0 d + b0 (Sec. 4.1): in T-coordinates
// as the deviation y = T^T d' - zr (rotation route, compensated FP32 as
// high + low rows) or as d' itself (other routes).  d = A0^-1 (d' - b0).
int read_bloch(mln_handle *h, std::vector<double> &d) {
  const Factors &f = h->f;
  const int D = f.D;
  const int64_t nm = h->nmed, ld = h->ld;
  const int rows = h->comp ? 2 * D : D;
  std::vector<unsigned char> raw((size_t)rows * ld * h->rs);
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (nm > 0) HIP_TRY(hipMemcpy(raw.data(), h->z[h->cur].p, raw.size(), hipMemcpyDeviceToHost));
  auto at = [&](int row, int64_t c) {
    return h->rs == 8 ? ((const double *)raw.data())[row * ld + c] : (double)((const float *)raw.data())[row * ld + c];
  };
  std::vector<double> inv;
  if (!invert(D, f.A0, inv)) return set_err(MLN_ENUMERIC, "half-step propagator is singular");
  const bool rot = h->route == MLN_ROUTE_ROTATION;
  d.assign((size_t)D * nm, 0.0);
  std::vector<double> zp(D), dp(D);
  for (int64_t c = 0; c < nm; ++c) {
    for (int j = 0; j < D; ++j) zp[j] = at(j, c) + (h->comp ? at(D + j, c) : 0.0) + (rot ? f.zr[j] : 0.0);
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      if (rot)
        for (int j = 0; j < D; ++j) acc += f.T[(size_t)i * D + j] * zp[j];
      else
        acc = zp[i];
      dp[i] = acc - f.b0[i];
    }
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int j = 0; j < D; ++j) acc += inv[(size_t)i * D + j] * dp[j];
      d[(size_t)i * nm + c] = acc;
    }
  }
  return MLN_OK;
}

// Write n real values into a device buffer of the kernels' precision (with
// the compensated fields, the high parts then the low parts).
template <typename T>
void to_real(const double *src, int64_t n, int64_t stride, bool split, double scale, std::vector<unsigned char> &out,
             int64_t at) {
  T *o = (T *)out.data();
  for (int64_t i = 0; i < n; ++i) {
    const double v = src[i] * scale;
    o[at + i] = (T)v;
    if (split) o[at + stride + i] = (T)(v - (double)(T)v);
  }
}

}  // namespace

extern "C" {

int mln_get_state(const mln_handle *hc, double *E, double *H, double *rho_diag) {
  mln_handle *h = const_cast<mln_handle *>(hc);
  if (!h) return set_err(MLN_EINVAL, "null handle");
  int rc = mln_get_fields(h, E, H);
  if (rc || !rho_diag) return rc;
  std::vector<double> d;
  rc = read_bloch(h, d);
  if (rc) return rc;
  // rho_aa = 1/N + (1/2) sum_l d_l (s_l)_aa (Eq. comp_rho)
  const Factors &f = h->f;
  const int N = f.N, D = f.D;
  const int64_t nm = h->nmed;
  for (int a = 0; a < N; ++a)
    for (int64_t c = 0; c < nm; ++c) {
      double acc = 1.0 / N;
      for (int l = 0; l < D; ++l) acc += 0.5 * d[(size_t)l * nm + c] * f.gen[((size_t)l * N + a) * N + a].real();
      rho_diag[(size_t)a * nm + c] = acc;
    }
  return MLN_OK;
}

int mln_get_bloch(const mln_handle *hc, double *d) {
  mln_handle *h = const_cast<mln_handle *>(hc);
  if (!h || !d) return set_err(MLN_EINVAL, "null argument");
  std::vector<double> v;
  int rc = read_bloch(h, v);
  if (rc) return rc;
  std::copy(v.begin(), v.end(), d);
  return MLN_OK;
}

int mln_set_state(mln_handle *h, const double *E, const double *H, const double *d) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  const int64_t nx = h->grid.nx, nm = h->nmed, ld = h->ld;
  const Factors &f = h->f;
  const int D = f.D;
  for (int64_t i = 0; E && i < nx; ++i)
    if (!std::isfinite(E[i])) return set_err(MLN_EINVAL, "non-finite E");
  for (int64_t i = 0; H && i < nx - 1; ++i)
    if (!std::isfinite(H[i])) return set_err(MLN_EINVAL, "non-finite H");
  for (int64_t i = 0; d && i < (int64_t)D * nm; ++i)
    if (!std::isfinite(d[i])) return set_err(MLN_EINVAL, "non-finite Bloch vector");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const bool f32 = h->rs == 4;
  if (E || H) {
    const int parts = h->cf ? 2 : 1;
    std::vector<unsigned char> buf((size_t)h->rs * nx * parts, 0);
    if (E) {
      if (f32) to_real<float>(E, nx, nx, h->cf, 1.0, buf, 0);
      else to_real<double>(E, nx, nx, false, 1.0, buf, 0);
      HIP_TRY(hipMemcpy(h->E[h->cur].p, buf.data(), buf.size(), hipMemcpyHostToDevice));
    }
    if (H) {
      std::fill(buf.begin(), buf.end(), 0);
      if (f32) to_real<float>(H, nx - 1, nx, h->cf, 1.0 / h->h_scale32, buf, 0);
      else to_real<double>(H, nx - 1, nx, false, 1.0, buf, 0);
      HIP_TRY(hipMemcpy(h->H[h->cur].p, buf.data(), buf.size(), hipMemcpyHostToDevice));
    }
  }
  if (d && nm > 0) {
    // d' = A0 d + b0; rotation route: y = T^T d' - zr
    const bool rot = h->route == MLN_ROUTE_ROTATION;
    const int rows = h->comp ? 2 * D : D;
    std::vector<double> st((size_t)rows * ld, 0.0), dp(D);
    for (int64_t c = 0; c < nm; ++c) {
      for (int i = 0; i < D; ++i) {
        double acc = f.b0[i];
        for (int j = 0; j < D; ++j) acc += f.A0[(size_t)i * D + j] * d[(size_t)j * nm + c];
        dp[i] = acc;
      }
      for (int j = 0; j < D; ++j) {
        double v = dp[j];
        if (rot) {
          v = -f.zr[j];
          for (int i = 0; i < D; ++i) v += f.T[(size_t)i * D + j] * dp[i];
        }
        st[(size_t)j * ld + c] = v;
      }
    }
    std::vector<unsigned char> buf((size_t)rows * ld * h->rs, 0);
    if (f32) {
      float *o = (float *)buf.data();
      for (int j = 0; j < D; ++j)
        for (int64_t c = 0; c < nm; ++c) {
          const double v = st[(size_t)j * ld + c];
          o[(size_t)j * ld + c] = (float)v;
          if (h->comp) o[(size_t)(D + j) * ld + c] = (float)(v - (double)(float)v);
        }
    } else {
      std::memcpy(buf.data(), st.data(), (size_t)D * ld * sizeof(double));
    }
    HIP_TRY(hipMemcpy(h->z[h->cur].p, buf.data(), buf.size(), hipMemcpyHostToDevice));
  }
  h->ckpt_ok = false;  // checkpoints of the run so far no longer lead here
  h->tape_ok = false;
  return MLN_OK;
}

int mln_state_bytes(const mln_handle *h, int64_t *bytes) {
  if (!h || !bytes) return set_err(MLN_EINVAL, "null argument");
  *bytes = (int64_t)(sizeof(int64_t) + h->E[0].bytes + h->H[0].bytes + h->z[0].bytes);
  return MLN_OK;
}

int mln_save_state(mln_handle *h, void *host_buf) {
  if (!h || !host_buf) return set_err(MLN_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(h->stream));
  unsigned char *p = (unsigned char *)host_buf;
  std::memcpy(p, &h->step, sizeof(int64_t));
  p += sizeof(int64_t);
  HIP_TRY(hipMemcpy(p, h->E[h->cur].p, h->E[0].bytes, hipMemcpyDeviceToHost));
  p += h->E[0].bytes;
  HIP_TRY(hipMemcpy(p, h->H[h->cur].p, h->H[0].bytes, hipMemcpyDeviceToHost));
  p += h->H[0].bytes;
  HIP_TRY(hipMemcpy(p, h->z[h->cur].p, h->z[0].bytes, hipMemcpyDeviceToHost));
  return MLN_OK;
}

int mln_load_state(mln_handle *h, const void *host_buf) {
  if (!h || !host_buf) return set_err(MLN_EINVAL, "null argument");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const unsigned char *p = (const unsigned char *)host_buf;
  int64_t step;
  std::memcpy(&step, p, sizeof(int64_t));
  if (step < 0 || step > h->grid.nt) return set_err(MLN_EINVAL, "checkpoint step out of range");
  p += sizeof(int64_t);
  for (int b = 0; b < 2; ++b) {
    const unsigned char *q = p;
    HIP_TRY(hipMemcpy(h->E[b].p, q, h->E[0].bytes, hipMemcpyHostToDevice));
    q += h->E[0].bytes;
    HIP_TRY(hipMemcpy(h->H[b].p, q, h->H[0].bytes, hipMemcpyHostToDevice));
    q += h->H[0].bytes;
    HIP_TRY(hipMemcpy(h->z[b].p, q, h->z[0].bytes, hipMemcpyHostToDevice));
  }
  h->step = step;
  h->cur = 0;
  h->ckpt_ok = false;
  h->tape_ok = false;
  return MLN_OK;
}

int mln_bloch_only(mln_handle *h, const double *efield, int64_t n_steps, double *pop_out, double *dp_out) {
  if (!h || !efield || n_steps < 0) return set_err(MLN_EINVAL, "bad argument");
  const int64_t nc = h->nmed;
  const int N = h->f.N, D = h->f.D;
  if (nc == 0 || n_steps == 0) return MLN_OK;
  DevBuf de, dpop, ddp, dz0;
  const double *e_dev = efield;
  double *pop_dev = pop_out, *dp_dev = dp_out;
  if (!h->rec.out_on_device) {
    HIP_TRY(de.alloc(sizeof(double) * nc * n_steps));
    HIP_TRY(hipMemcpy(de.p, efield, sizeof(double) * nc * n_steps, hipMemcpyHostToDevice));
    e_dev = (const double *)de.p;
    if (pop_out) {
      HIP_TRY(dpop.alloc(sizeof(double) * nc * n_steps * N));
      pop_dev = (double *)dpop.p;
    }
    if (dp_out) {
      HIP_TRY(ddp.alloc(sizeof(double) * nc * n_steps));
      dp_dev = (double *)ddp.p;
    }
  }
  const std::vector<double> &s0 = (h->route == MLN_ROUTE_ROTATION) ? h->f.y0 : h->f.dprime0;
  hipError_t e;
  if (h->prec == MLN_FP64) {
    HIP_TRY(dz0.alloc(sizeof(double) * D));
    HIP_TRY(hipMemcpy(dz0.p, s0.data(), sizeof(double) * D, hipMemcpyHostToDevice));
    BlochArgs<double> a{h->fd, 0, (const double *)dz0.p, e_dev, nc, n_steps, pop_dev, dp_dev};
    e = launch_bloch<double>(N, h->route, false, a, h->stream);
  } else {
    std::vector<float> z0f(2 * D);
    for (int j = 0; j < D; ++j) {
      z0f[j] = (float)s0[j];
      z0f[D + j] = (float)(s0[j] - (double)z0f[j]);
    }
    HIP_TRY(dz0.alloc(sizeof(float) * 2 * D));
    HIP_TRY(hipMemcpy(dz0.p, z0f.data(), sizeof(float) * 2 * D, hipMemcpyHostToDevice));
    BlochArgs<float> a{h->ff, 0, (const float *)dz0.p, e_dev, nc, n_steps, pop_dev, dp_dev};
    e = launch_bloch<float>(N, h->route, h->comp, a, h->stream);
  }
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("bloch launch: ") + hipGetErrorString(e));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (!h->rec.out_on_device) {
    if (pop_out) HIP_TRY(hipMemcpy(pop_out, pop_dev, sizeof(double) * nc * n_steps * N, hipMemcpyDeviceToHost));
    if (dp_out) HIP_TRY(hipMemcpy(dp_out, dp_dev, sizeof(double) * nc * n_steps, hipMemcpyDeviceToHost));
  }
  return MLN_OK;
}

int mln_bloch_only_noalloc(mln_handle *h, const double *efield, int64_t n_steps, double *pop_out,
                           double *dp_out) {
  if (!h || !efield || n_steps < 0) return set_err(MLN_EINVAL, "bad argument");
  const int64_t nc = h->nmed;
  const int N = h->f.N, D = h->f.D;
  if (nc == 0 || n_steps == 0) return MLN_OK;
  const bool f64 = h->prec == MLN_FP64;
  const size_t need = f64 ? sizeof(double) * D : sizeof(float) * 2 * D;
  constexpr int kMaxD = 35;  // N <= 6
  if (D > kMaxD || need > MLN_NOALLOC_SCRATCH_BYTES)
    return set_err(MLN_EINVAL, "initial state of " + std::to_string(need) + " bytes exceeds the " +
                                   std::to_string(MLN_NOALLOC_SCRATCH_BYTES) + "-byte scratch");
  void *sp = scratch_of(h->device);
  if (!sp) return set_err(MLN_ESTATE, "scratch address of the handle's device was not set up");
  const std::vector<double> &s0 = (h->route == MLN_ROUTE_ROTATION) ? h->f.y0 : h->f.dprime0;
  hipError_t e;
  if (f64) {
    HIP_TRY(hipMemcpyAsync(sp, s0.data(), need, hipMemcpyHostToDevice, h->stream));
    BlochArgs<double> a{h->fd, 0, (const double *)sp, efield, nc, n_steps, pop_out, dp_out};
    e = launch_bloch<double>(N, h->route, false, a, h->stream);
  } else {
    float z0f[2 * kMaxD];
    for (int j = 0; j < D; ++j) {
      z0f[j] = (float)s0[j];
      z0f[D + j] = (float)(s0[j] - (double)z0f[j]);
    }
    HIP_TRY(hipMemcpyAsync(sp, z0f, need, hipMemcpyHostToDevice, h->stream));
    BlochArgs<float> a{h->ff, 0, (const float *)sp, efield, nc, n_steps, pop_out, dp_out};
    e = launch_bloch<float>(N, h->route, h->comp, a, h->stream);
  }
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("bloch launch: ") + hipGetErrorString(e));
  // z0f lives on this stack frame: the copy and the kernel end before return
  HIP_TRY(hipStreamSynchronize(h->stream));
  return MLN_OK;
}

int mln_grad(mln_handle *h, const double *dJ_dprobe, mln_grads *out) {
  if (!h || !dJ_dprobe || !out) return set_err(MLN_EINVAL, "null argument");
  if (h->ckpt_every <= 0 && !h->tape_all)
    return set_err(MLN_ESTATE, "handle was created without checkpoints or tape (ckpt_every = 0)");
  if (h->route != MLN_ROUTE_ROTATION || h->f.N > 3)
    return set_err(MLN_ENOTSUPPORTED, "the adjoint is built for the rotation route and N <= 3");
  const int64_t nt = h->grid.nt;
  if (h->tape_all ? (!h->tape_ok || h->step != nt)
                  : (!h->ckpt_ok || h->step != nt || h->ckpt_count != h->nckpt))
    return set_err(MLN_ESTATE, "mln_grad needs a completed run from step 0 (mln_reset + mln_run)");
  const int N = h->f.N, D = h->f.D, q = h->f.q;
  const bool f64 = h->prec == MLN_FP64;
  const int nacc = N == 2 ? adj_nacc(2, f64) : adj_nacc(3, f64);
  const int nm = adj_moments(f64);
  const size_t rs = h->rs;
  // reverse-kernel tiling (the tape is read by cell, so it need not be the
  // forward one): mln_configure_adjoint's if set; else after the streamed
  // forward kernel (one step per launch) the one-cell-per-thread tile kernel,
  // 256 cells and 16 steps per launch; after a four-lanes-per-cell forward
  // kernel the four-lanes-per-cell reverse kernel on 128-cell tiles with the
  // largest even step count up to 48 that keeps the tiles within the compute
  // units (a reverse launch has a fixed cost of about eight steps: prologue,
  // per-tile sums, kernel boundary), 16 where none does; otherwise the
  // forward kernel's tiling
  bool rquad = h->quad;
  int rW = h->W, rhalo = h->halo, rowned = h->owned;
  int64_t rtiles = h->ntiles;
  if (h->adj_variant) {
    // set by mln_configure_adjoint
    rquad = h->adj_variant == 3;
    rW = h->adj_W;
    rhalo = h->adj_K;
    rowned = rW - 2 * rhalo;
    rtiles = (h->grid.nx + rowned - 1) / rowned;
  } else if (h->streamed) {
    rquad = false;
    rW = kMaxTile;
    rhalo = 16;
    rowned = rW - 2 * rhalo;
    rtiles = (h->grid.nx + rowned - 1) / rowned;
  } else if (rquad && !(f64 && N == 3)) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
      cus = 256;
    rW = kMaxAdjQuadTile;
    rhalo = 16;
    for (int k = 48; k > 16; k -= 2)
      if ((h->grid.nx + (rW - 2 * k) - 1) / (rW - 2 * k) <= cus) {
        rhalo = k;
        break;
      }
    rowned = rW - 2 * rhalo;
    rtiles = (h->grid.nx + rowned - 1) / rowned;
  } else if (rquad && f64 && N == 3 && rW > 64) {
    // the FP64 three-level reverse step runs spill-free only on the
    // 256-lane build: 64-cell tiles, 16 steps per launch (the tape is read
    // by cell, so the reverse tiling need not be the forward one)
    rW = 64;
    rhalo = 16;
    rowned = rW - 2 * rhalo;
    rtiles = (h->grid.nx + rowned - 1) / rowned;
  }
  if (!h->gprobe.p) {
    for (int b = 0; b < 2; ++b) {
      HIP_TRY(h->lE[b].alloc(rs * h->grid.nx));
      HIP_TRY(h->lH[b].alloc(rs * h->grid.nx));
      HIP_TRY(h->lz[b].alloc(rs * D * h->ld));
    }
    if (!h->tape_all) HIP_TRY(h->tape.alloc(rs * (size_t)h->ckpt_every * (D + 1) * h->ld));
    if (!h->tape_all && h->nckpt > 1) HIP_TRY(h->tape2.alloc(rs * (size_t)h->ckpt_every * (D + 1) * h->ld));
    HIP_TRY(h->gprobe.alloc(sizeof(double) * (nt + 1)));
    HIP_TRY(h->samples_dev.alloc(sizeof(double) * (nt + 1)));
    HIP_TRY(hipMemcpy(h->samples_dev.p, h->samples.data(), sizeof(double) * (nt + 1), hipMemcpyHostToDevice));
  }
  // per-tile partial sums: the tiling may have changed since an earlier call
  // (mln_configure at step 0)
  if (h->partial.bytes < sizeof(double) * rtiles * nacc) HIP_TRY(h->partial.alloc(sizeof(double) * rtiles * nacc));
  HIP_TRY(hipMemcpyAsync(h->gprobe.p, dJ_dprobe, sizeof(double) * (nt + 1), hipMemcpyHostToDevice, h->stream));
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(hipMemsetAsync(h->lE[b].p, 0, h->lE[b].bytes, h->stream));
    HIP_TRY(hipMemsetAsync(h->lH[b].p, 0, h->lH[b].bytes, h->stream));
    HIP_TRY(hipMemsetAsync(h->lz[b].p, 0, h->lz[b].bytes, h->stream));
  }
  HIP_TRY(hipMemsetAsync(h->partial.p, 0, h->partial.bytes, h->stream));
  int lc = 0;
  // segments: the checkpoint intervals (each rebuilt from its checkpoint,
  // writing the tape), or with the whole tape in memory one segment and no
  // recomputation.  With two or more checkpoint intervals the rebuild of
  // segment k-1 runs on a second stream into the other of two tape buffers
  // while segment k is reversed on the handle's stream (the two kernels are
  // latency-bound and fit on one compute unit together); events order each
  // reverse sweep after its rebuild and each rebuild after the sweep that
  // last read its buffer.
  const int64_t nseg = h->tape_all ? 1 : h->nckpt;
  const bool overlap = !h->tape_all && nseg > 1;
  if (overlap && !h->aux_stream) {
    HIP_TRY(hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&h->ev_start, hipEventDisableTiming));
    for (int b = 0; b < 2; ++b) {
      HIP_TRY(hipEventCreateWithFlags(&h->ev_rec[b], hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&h->ev_rev[b], hipEventDisableTiming));
    }
  }
  if (overlap) {
    HIP_TRY(hipEventRecord(h->ev_start, h->stream));
    HIP_TRY(hipStreamWaitEvent(h->aux_stream, h->ev_start, 0));
  }
  // the rebuilds enqueue on h->stream: point it at the second stream for
  // them, and restore it (and let the second stream drain) on every exit
  struct Restore {
    mln_handle *h;
    hipStream_t main;
    bool overlap;
    ~Restore() {
      h->stream = main;
      if (overlap) (void)hipStreamSynchronize(h->aux_stream);
    }
  } restore{h, h->stream, overlap};
  DevBuf *tapes[2] = {&h->tape, &h->tape2};
  for (int64_t seg = nseg - 1, it = 0; seg >= 0; --seg, ++it) {
    const int64_t s0 = h->tape_all ? 0 : seg * h->ckpt_every;
    const int64_t s1 = h->tape_all ? nt : std::min<int64_t>(s0 + h->ckpt_every, nt);
    const int tb = overlap ? (int)(it & 1) : 0;
    void *tape_p = tapes[tb]->p;
    if (!h->tape_all) {
      if (overlap) {
        h->stream = h->aux_stream;
        if (it >= 2) HIP_TRY(hipStreamWaitEvent(h->aux_stream, h->ev_rev[tb], 0));
      }
      h->cur = 0;
      int rc = ckpt_copy(h, seg, false);
      if (rc) return rc;
      h->step = s0;
      rc = forward_steps(h, s1 - s0, false, tape_p, s0, false);
      if (rc) return rc;
      if (overlap) {
        HIP_TRY(hipEventRecord(h->ev_rec[tb], h->aux_stream));
        h->stream = restore.main;
        HIP_TRY(hipStreamWaitEvent(h->stream, h->ev_rec[tb], 0));
      }
    }
    for (int64_t n_hi = s1; n_hi > s0;) {
      const int k = (int)std::min<int64_t>(rhalo, n_hi - s0);
      hipError_t e;
      if (f64) {
        AdjArgs<double> a{};
        a.fac = h->fd;
        a.lEin = (const double *)h->lE[lc].p;
        a.lEout = (double *)h->lE[1 - lc].p;
        a.lHin = (const double *)h->lH[lc].p;
        a.lHout = (double *)h->lH[1 - lc].p;
        a.lzin = (const double *)h->lz[lc].p;
        a.lzout = (double *)h->lz[1 - lc].p;
        a.tape = (const double *)tape_p;
        a.tape_step0 = s0;
        a.gprobe = (const double *)h->gprobe.p;
        a.samples = (const double *)h->samples_dev.p;
        a.nx = h->grid.nx; a.mb = h->grid.med_begin; a.me = h->grid.med_end; a.ld = h->ld;
        a.n_hi = n_hi; a.nsteps = k; a.halo = rhalo; a.owned = rowned;
        double cam1;
        fdtd_coefs(h, a.ch, a.ca, a.cb, a.inv_dx, a.kmur, cam1);
        a.partial = (double *)h->partial.p;
        e = (rquad && rW <= 128) ? launch_adj_quad<double>(N, a, rtiles, rW, h->stream)
                    : launch_adj<double>(N, a, rtiles, rW, h->stream);
      } else {
        AdjArgs<float> a{};
        a.fac = h->ff;
        a.lEin = (const float *)h->lE[lc].p;
        a.lEout = (float *)h->lE[1 - lc].p;
        a.lHin = (const float *)h->lH[lc].p;
        a.lHout = (float *)h->lH[1 - lc].p;
        a.lzin = (const float *)h->lz[lc].p;
        a.lzout = (float *)h->lz[1 - lc].p;
        a.tape = (const float *)tape_p;
        a.tape_step0 = s0;
        a.gprobe = (const double *)h->gprobe.p;
        a.samples = (const double *)h->samples_dev.p;
        a.nx = h->grid.nx; a.mb = h->grid.med_begin; a.me = h->grid.med_end; a.ld = h->ld;
        a.n_hi = n_hi; a.nsteps = k; a.halo = rhalo; a.owned = rowned;
        float cam1;
        fdtd_coefs(h, a.ch, a.ca, a.cb, a.inv_dx, a.kmur, cam1);
        a.partial = (double *)h->partial.p;
        e = (rquad && rW <= 128) ? launch_adj_quad<float>(N, a, rtiles, rW, h->stream)
                    : launch_adj<float>(N, a, rtiles, rW, h->stream);
      }
      if (e != hipSuccess) return set_err(MLN_EHIP, std::string("adjoint launch: ") + hipGetErrorString(e));
      lc = 1 - lc;
      n_hi -= k;
    }
    if (overlap) HIP_TRY(hipEventRecord(h->ev_rev[tb], h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (!h->tape_all) {
    h->step = nt;  // the forward buffers now hold an intermediate state; mln_reset before stepping again
    h->ckpt_ok = false;
  }
  // gather: per-tile partial sums, lz'_0 summed over the medium, lE^0 at cell 0
  std::vector<double> part(rtiles * nacc), acc(nacc, 0.0);
  HIP_TRY(hipMemcpy(part.data(), h->partial.p, sizeof(double) * part.size(), hipMemcpyDeviceToHost));
  for (int64_t t = 0; t < rtiles; ++t)
    for (int i = 0; i < nacc; ++i) acc[i] += part[t * nacc + i];
  std::vector<unsigned char> zb(rs * D * h->ld), eb(rs);
  HIP_TRY(hipMemcpy(zb.data(), h->lz[lc].p, zb.size(), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(eb.data(), h->lE[lc].p, rs, hipMemcpyDeviceToHost));
  auto rd = [&](const unsigned char *p, int64_t i) {
    return rs == 8 ? ((const double *)p)[i] : (double)((const float *)p)[i];
  };
  std::vector<double> gz0(D, 0.0);
  for (int j = 0; j < D; ++j)
    for (int64_t c = 0; c < h->nmed; ++c) gz0[j] += rd(zb.data(), j * h->ld + c);
  // unpack (same order as the kernel)
  int k = 0;
  std::vector<double> GK(D * D), Gc(D), Gw(D);
  for (int i = 0; i < D * D; ++i) GK[i] = acc[k++];
  for (int i = 0; i < D; ++i) Gc[i] = acc[k++];
  for (int i = 0; i < D; ++i) Gw[i] = acc[k++];
  const double Gp0 = acc[k++];
  double Gamp = acc[k++] + h->samples[0] * rd(eb.data(), 0);
  std::vector<std::vector<double>> Mom(nm, std::vector<double>(D * D));
  for (int m = 0; m < nm; ++m)
    for (int i = 0; i < D * D; ++i) Mom[m][i] = acc[k++];
  // dJ/dB = dt [M1 + ad_Bt^2(M3)/24 + ad_Bt^4(M5)/1920], Bt = T^T U T dt (block diagonal)
  const double dt = h->grid.dt;
  std::vector<double> Bt(D * D, 0.0);
  for (int p = 0; p < q; ++p) {
    Bt[(2 * p) * D + 2 * p + 1] = h->f.theta[p] * dt;
    Bt[(2 * p + 1) * D + 2 * p] = -h->f.theta[p] * dt;
  }
  auto ad = [&](const std::vector<double> &X) {
    std::vector<double> r(D * D, 0.0);
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double s2 = 0.0;
        for (int l = 0; l < D; ++l) s2 += Bt[i * D + l] * X[l * D + j] - X[i * D + l] * Bt[l * D + j];
        r[i * D + j] = s2;
      }
    return r;
  };
  std::vector<double> GB = Mom[0];
  {
    std::vector<double> a2 = ad(ad(Mom[1]));
    for (int i = 0; i < D * D; ++i) GB[i] += a2[i] / 24.0;
    if (nm > 2) {
      std::vector<double> a4 = ad(ad(ad(ad(Mom[2]))));
      for (int i = 0; i < D * D; ++i) GB[i] += a4[i] / 1920.0;
    }
    for (double &x : GB) x *= dt;
  }
  // z -> d coordinates: d = T z
  const std::vector<double> &T = h->f.T;
  auto sandwich = [&](const std::vector<double> &X) {  // T X T^T
    std::vector<double> t1(D * D, 0.0), r(D * D, 0.0);
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j)
        for (int l = 0; l < D; ++l) t1[i * D + j] += T[i * D + l] * X[l * D + j];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j)
        for (int l = 0; l < D; ++l) r[i * D + j] += t1[i * D + l] * T[j * D + l];
    return r;
  };
  auto tvec = [&](const std::vector<double> &x) {
    std::vector<double> r(D, 0.0);
    for (int i = 0; i < D; ++i)
      for (int l = 0; l < D; ++l) r[i] += T[i * D + l] * x[l];
    return r;
  };
  std::vector<double> gA = sandwich(GK), gU = sandwich(GB), gc = tvec(Gc), gw = tvec(Gw), gd0 = tvec(gz0);
  std::string err;
  int rc = chain_rule(&h->medium.m, dt, gA.data(), gc.data(), gw.data(), Gp0, gU.data(), gd0.data(), out, &err);
  if (rc) return set_err(rc, err);
  if (out->d_amplitude) *out->d_amplitude = Gamp;
  return MLN_OK;
}

void mln_free(mln_handle *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
