// mln_abi.hip -- the C ABI declared in include/mln.h: validation, one-time
// factor upload, device state, the launch loop over fused time steps,
// recording and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mln.h"
#include "fwd_kernels.hpp"
#include "mln_internal.hpp"

using namespace mln;

namespace {

thread_local std::string g_last_error;

int set_err(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

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
    bytes = n;
    return hipMalloc(&p, n ? n : 1);
  }
};

}  // namespace

struct mln_handle {
  Factors f;
  mln_grid grid{};
  double amp = 0.0;
  std::vector<double> samples;
  int prec = MLN_FP64, route = MLN_ROUTE_ROTATION;
  hipStream_t stream = nullptr;
  int64_t nmed = 0, ld = 0, step = 0;
  int W = 256, halo = 0, owned = 0;
  int64_t ntiles = 0;
  int rs = 8;  // bytes per real of the state
  // device state (ping-pong)
  DevBuf E[2], H[2], z[2];
  int cur = 0;
  DevBuf src, fac, pop, popc;
  FacDev<double> fd{};
  FacDev<float> ff{};
  // recording
  mln_record rec{};
  int64_t nsnap = 0;
  DevBuf st_pop, st_e, st_probe;  // device staging for host outputs
  double *d_pop = nullptr, *d_e = nullptr, *d_probe = nullptr;
  // initial state on the host
  std::vector<unsigned char> z_init, e_init;
  double fd_coef[5] = {0, 0, 0, 0, 0};  // ch, ca, cb, inv_dx, kmur
};

namespace {

// Upload the factors of the chosen route in precision Real.  The layout of
// the device block is a concatenation of arrays; FacDev points into it.
template <typename Real>
int upload_factors(mln_handle *h, FacDev<Real> &fd) {
  const Factors &f = h->f;
  const int D = f.D, q = f.q;
  std::vector<Real> blk;
  auto push = [&](const std::vector<double> &v) {
    size_t off = blk.size();
    for (double x : v) blk.push_back((Real)x);
    while (blk.size() % 16) blk.push_back(0);
    return off;
  };
  const bool rot = h->route == MLN_ROUTE_ROTATION;
  std::vector<double> Km = rot ? f.K : f.A;
  for (int i = 0; i < D; ++i) Km[i * D + i] -= 1.0;
  std::vector<double> thdt(q), rre(D * D), rim(D * D), lamdt(D);
  for (int p = 0; p < q; ++p) thdt[p] = f.theta[p] * h->grid.dt;
  for (int i = 0; i < D * D; ++i) {
    rre[i] = f.R[i].real();
    rim[i] = f.R[i].imag();
  }
  for (int k = 0; k < D; ++k) lamdt[k] = f.lam[k].imag() * h->grid.dt;
  size_t oK = push(Km), oc = push(rot ? f.cz : f.c), ow = push(rot ? f.wz : f.w);
  size_t oth = push(thdt), orr = push(rre), ori = push(rim), ol = push(lamdt);
  size_t oS = push(f.S), oS2 = push(f.S2);
  HIP_TRY(h->fac.alloc(blk.size() * sizeof(Real)));
  HIP_TRY(hipMemcpy(h->fac.p, blk.data(), blk.size() * sizeof(Real), hipMemcpyHostToDevice));
  const Real *b = (const Real *)h->fac.p;
  fd.Km = b + oK;
  fd.cz = b + oc;
  fd.wz = b + ow;
  fd.thdt = b + oth;
  fd.Rre = b + orr;
  fd.Rim = b + ori;
  fd.lamdt = b + ol;
  fd.S = b + oS;
  fd.S2 = b + oS2;
  fd.p0 = (Real)f.p0;
  const std::vector<double> &pm = rot ? f.popz : f.popd;
  HIP_TRY(h->pop.alloc(pm.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(h->pop.p, pm.data(), pm.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(h->popc.alloc(f.popc.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(h->popc.p, f.popc.data(), f.popc.size() * sizeof(double), hipMemcpyHostToDevice));
  fd.pop = (const double *)h->pop.p;
  fd.popc = (const double *)h->popc.p;
  return MLN_OK;
}

template <typename Real>
void build_init_state(mln_handle *h) {
  const Factors &f = h->f;
  const int D = f.D;
  const std::vector<double> &s0 = (h->route == MLN_ROUTE_ROTATION) ? f.z0 : f.dprime0;
  h->z_init.assign(sizeof(Real) * D * h->ld, 0);
  Real *zi = (Real *)h->z_init.data();
  for (int j = 0; j < D; ++j)
    for (int64_t c = 0; c < h->nmed; ++c) zi[j * h->ld + c] = (Real)s0[j];
  h->e_init.assign(sizeof(Real) * h->grid.nx, 0);
  ((Real *)h->e_init.data())[0] = (Real)(h->amp * h->samples[0]);
}

int reset_state(mln_handle *h) {
  const size_t rs = h->rs;
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(hipMemsetAsync(h->H[b].p, 0, h->H[b].bytes, h->stream));
    HIP_TRY(hipMemcpyAsync(h->E[b].p, h->e_init.data(), rs * h->grid.nx, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipMemcpyAsync(h->z[b].p, h->z_init.data(), h->z_init.size(), hipMemcpyHostToDevice, h->stream));
  }
  h->cur = 0;
  h->step = 0;
  if (h->d_probe) {
    double p0 = (h->grid.nx - 1 == 0) ? h->amp * h->samples[0] : 0.0;
    HIP_TRY(hipMemcpyAsync(h->d_probe, &p0, sizeof(double), hipMemcpyHostToDevice, h->stream));
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return MLN_OK;
}

template <typename Real>
FwdArgs<Real> make_args(mln_handle *h, const FacDev<Real> &fd, int64_t step0, int nsteps) {
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
  a.ch = (Real)h->fd_coef[0];
  a.ca = (Real)h->fd_coef[1];
  a.cb = (Real)h->fd_coef[2];
  a.inv_dx = (Real)h->fd_coef[3];
  a.kmur = (Real)h->fd_coef[4];
  a.snap_every = h->rec.snap_every;
  a.pop_out = h->d_pop;
  a.e_out = h->d_e;
  a.probe_out = h->d_probe;
  return a;
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
  std::vector<Real> src(h->grid.nt + 1);
  for (int64_t i = 0; i <= h->grid.nt; ++i) src[i] = (Real)(h->amp * h->samples[i]);
  HIP_TRY(h->src.alloc(src.size() * sizeof(Real)));
  HIP_TRY(hipMemcpy(h->src.p, src.data(), src.size() * sizeof(Real), hipMemcpyHostToDevice));
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(h->E[b].alloc(nx * sizeof(Real)));
    HIP_TRY(h->H[b].alloc(nx * sizeof(Real)));
    HIP_TRY(h->z[b].alloc((size_t)D * h->ld * sizeof(Real)));
  }
  build_init_state<Real>(h);
  return MLN_OK;
}

}  // namespace

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

int mln_init(const mln_medium *medium, const mln_grid *grid, const mln_source *source,
             const mln_record *record, const mln_options *options, mln_handle **out) {
  if (!out) return set_err(MLN_EINVAL, "null output handle");
  *out = nullptr;
  int rc = validate_grid(grid, source);
  if (rc) return rc;
  std::unique_ptr<mln_handle> h(new mln_handle());
  std::string err;
  rc = build_factors(medium, grid->dt, &h->f, &err);
  if (rc) return set_err(rc, err);
  h->grid = *grid;
  h->amp = source->amplitude;
  h->samples.assign(source->samples, source->samples + grid->nt + 1);
  mln_options opt{};
  if (options) opt = *options;
  h->prec = opt.precision;
  h->route = opt.route;
  h->stream = (hipStream_t)opt.stream;
  if (h->route < 0 || h->route > 2) return set_err(MLN_EINVAL, "unknown route");
  if (h->f.N == 5) return set_err(MLN_ENOTSUPPORTED, "kernels are built for N = 2, 3, 4 and 6");
  if (h->prec != MLN_FP64 && h->prec != MLN_FP32)
    return set_err(MLN_ENOTSUPPORTED, "precision not built in this library version");
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
  // tiling
  h->W = opt.tile > 0 ? opt.tile : kMaxTile;
  if (h->W > kMaxTile || h->W < 64 || h->W % 64) return set_err(MLN_EINVAL, "tile must be a multiple of 64 in [64, 256]");
  int K = opt.steps_per_launch > 0 ? opt.steps_per_launch : 32;
  if (2 * K >= h->W) return set_err(MLN_EINVAL, "steps_per_launch must be below tile/2");
  h->halo = K;
  h->owned = h->W - 2 * K;
  h->ntiles = (grid->nx + h->owned - 1) / h->owned;
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
  rc = reset_state(h.get());
  if (rc) return rc;
  *out = h.release();
  return MLN_OK;
}

int mln_step(mln_handle *h, int64_t n_steps) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  if (n_steps < 0) return set_err(MLN_EINVAL, "n_steps must be >= 0");
  int64_t left = std::min<int64_t>(n_steps, h->grid.nt - h->step);
  while (left > 0) {
    int k = (int)std::min<int64_t>(left, h->halo);
    hipError_t e;
    if (h->prec == MLN_FP64)
      e = launch_fwd<double>(h->f.N, h->route, make_args<double>(h, h->fd, h->step, k), h->ntiles, h->W, h->stream);
    else
      e = launch_fwd<float>(h->f.N, h->route, make_args<float>(h, h->ff, h->step, k), h->ntiles, h->W, h->stream);
    if (e != hipSuccess) return set_err(MLN_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    h->cur = 1 - h->cur;
    h->step += k;
    left -= k;
  }
  return MLN_OK;
}

int mln_run(mln_handle *h) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  int rc = mln_step(h, h->grid.nt - h->step);
  if (rc) return rc;
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

int mln_reset(mln_handle *h) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  return reset_state(h);
}

int mln_current_step(const mln_handle *h, int64_t *step) {
  if (!h || !step) return set_err(MLN_EINVAL, "null argument");
  *step = h->step;
  return MLN_OK;
}

int mln_get_fields(mln_handle *h, double *E, double *H) {
  if (!h) return set_err(MLN_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int64_t nx = h->grid.nx;
  std::vector<unsigned char> buf(h->rs * nx);
  auto conv = [&](double *dst, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      dst[i] = (h->rs == 8) ? ((double *)buf.data())[i] : (double)((float *)buf.data())[i];
  };
  if (E) {
    HIP_TRY(hipMemcpy(buf.data(), h->E[h->cur].p, h->rs * nx, hipMemcpyDeviceToHost));
    conv(E, nx);
  }
  if (H) {
    HIP_TRY(hipMemcpy(buf.data(), h->H[h->cur].p, h->rs * nx, hipMemcpyDeviceToHost));
    conv(H, nx - 1);
  }
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
  const std::vector<double> &s0 = (h->route == MLN_ROUTE_ROTATION) ? h->f.z0 : h->f.dprime0;
  hipError_t e;
  if (h->prec == MLN_FP64) {
    HIP_TRY(dz0.alloc(sizeof(double) * D));
    HIP_TRY(hipMemcpy(dz0.p, s0.data(), sizeof(double) * D, hipMemcpyHostToDevice));
    BlochArgs<double> a{h->fd, (const double *)dz0.p, e_dev, nc, n_steps, pop_dev, dp_dev};
    e = launch_bloch<double>(N, h->route, a, h->stream);
  } else {
    std::vector<float> z0f(s0.begin(), s0.end());
    HIP_TRY(dz0.alloc(sizeof(float) * D));
    HIP_TRY(hipMemcpy(dz0.p, z0f.data(), sizeof(float) * D, hipMemcpyHostToDevice));
    BlochArgs<float> a{h->ff, (const float *)dz0.p, e_dev, nc, n_steps, pop_dev, dp_dev};
    e = launch_bloch<float>(N, h->route, a, h->stream);
  }
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("bloch launch: ") + hipGetErrorString(e));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (!h->rec.out_on_device) {
    if (pop_out) HIP_TRY(hipMemcpy(pop_out, pop_dev, sizeof(double) * nc * n_steps * N, hipMemcpyDeviceToHost));
    if (dp_out) HIP_TRY(hipMemcpy(dp_out, dp_dev, sizeof(double) * nc * n_steps, hipMemcpyDeviceToHost));
  }
  return MLN_OK;
}

void mln_free(mln_handle *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
