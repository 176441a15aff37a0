// tmz.hip -- the two-dimensional TMz solver of include/mln.h (mln_tmz_*):
// validation, factor upload, device state, the per-step launch loop and the
// kernel instantiations of fwd_tmz.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <type_traits>
#include <vector>

#include "fwd_tmz.hpp"
#include "handle.hpp"

using namespace mln;

struct mln_tmz {
  Factors f;
  int N = 0, prec = MLN_FP64;
  bool comp = false;
  mln_tmz_grid grid{};
  mln_tmz_record rec{};
  hipStream_t stream = nullptr;
  int64_t nmed = 0, ld = 0, step = 0, nsnap = 0;
  int rs = 8;  // bytes per real
  DevBuf fac, pop, popc;
  FacDev<double> fd{};
  FacDev<float> ff{};
  DevBuf E[2], Hx[2], Hy[2], z, src, prof;
  int cur = 0;
  std::vector<double> src_host, prof_host;
  // FDTD coefficients: chx, chy, ca, cb, 1/dx, 1/dy, kmur (FP64), and the
  // single-precision set with (chx, 1/dx) and (chy, 1/dy) chosen so that
  // their products with cb match the FP64 ones (H_y, H_x carried scaled by
  // chx32/chx and chy32/chy; hs_x, hs_y undo that where H leaves the library)
  double c64[7] = {0, 0, 0, 0, 0, 0, 0};
  float c32[7] = {0, 0, 0, 0, 0, 0, 0};
  double hs_x = 1.0, hs_y = 1.0;
};

namespace {

template <int N, typename Real, bool COMP>
hipError_t launch_n(const TmzArgs<Real> &a, hipStream_t st) {
  const dim3 grid((unsigned)((a.nx + kTmzTX - 1) / kTmzTX), (unsigned)((a.ny + kTmzTY - 1) / kTmzTY));
  if constexpr (N <= 3 && std::is_same<Real, float>::value && !COMP) {
    hipLaunchKernelGGL((fwd_tmz_kernel_w7<N>), grid, dim3(kTmzTX * kTmzTY), 0, st, a);
  } else if constexpr (N <= 3) {
    hipLaunchKernelGGL((fwd_tmz_kernel_w5<N, Real, COMP>), grid, dim3(kTmzTX * kTmzTY), 0, st, a);
  } else {
    hipLaunchKernelGGL((fwd_tmz_kernel<N, Real, COMP>), grid, dim3(kTmzTX * kTmzTY), 0, st, a);
  }
  return hipGetLastError();
}

template <typename Real, bool COMP>
hipError_t launch_tmz(int N, const TmzArgs<Real> &a, hipStream_t st) {
  switch (N) {
    case 2: return launch_n<2, Real, COMP>(a, st);
    case 3: return launch_n<3, Real, COMP>(a, st);
    case 4: return launch_n<4, Real, COMP>(a, st);
    case 6: return launch_n<6, Real, COMP>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// host values -> device reals (FP32: scaled by 1/hscale), into buf at offset 0
template <typename Real>
void to_dev(const double *v, size_t n, double scale, std::vector<unsigned char> &buf) {
  buf.assign(n * sizeof(Real), 0);
  Real *o = (Real *)buf.data();
  for (size_t i = 0; i < n; ++i) o[i] = (Real)(v[i] * scale);
}

template <typename Real>
void from_dev(const std::vector<unsigned char> &buf, size_t n, double scale, double *out) {
  const Real *v = (const Real *)buf.data();
  for (size_t i = 0; i < n; ++i) out[i] = (double)v[i] * scale;
}

int tmz_write_probe0(mln_tmz *t) {
  if (!t->rec.probe_out) return MLN_OK;
  const int64_t nx = t->grid.nx, ny = t->grid.ny;
  std::vector<unsigned char> buf((size_t)nx * ny * t->rs);
  HIP_TRY(hipMemcpy(buf.data(), t->E[t->cur].p, buf.size(), hipMemcpyDeviceToHost));
  std::vector<double> e((size_t)nx * ny), p0(ny);
  if (t->rs == 8)
    from_dev<double>(buf, e.size(), 1.0, e.data());
  else
    from_dev<float>(buf, e.size(), 1.0, e.data());
  for (int64_t j = 0; j < ny; ++j) p0[j] = e[(size_t)j * nx + nx - 1];
  HIP_TRY(hipMemcpy(t->rec.probe_out, p0.data(), ny * sizeof(double), hipMemcpyHostToDevice));
  return MLN_OK;
}

int tmz_reset(mln_tmz *t) {
  const int64_t nx = t->grid.nx, ny = t->grid.ny;
  const size_t cells = (size_t)nx * ny;
  std::vector<double> e(cells, 0.0);
  for (int64_t j = 0; j < ny; ++j) e[(size_t)j * nx] = t->src_host[0] * t->prof_host[j];
  std::vector<unsigned char> buf;
  if (t->rs == 8)
    to_dev<double>(e.data(), cells, 1.0, buf);
  else
    to_dev<float>(e.data(), cells, 1.0, buf);
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(hipMemcpy(t->E[b].p, buf.data(), buf.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(t->Hx[b].p, 0, t->Hx[b].bytes));
    HIP_TRY(hipMemset(t->Hy[b].p, 0, t->Hy[b].bytes));
  }
  // Bloch state: the rotation route's initial deviation y0 in every cell
  const int D = t->f.D;
  const int rows = t->comp ? 2 * D : D;
  std::vector<unsigned char> zb((size_t)rows * t->ld * t->rs, 0);
  for (int k = 0; k < D; ++k)
    for (int64_t c = 0; c < t->nmed; ++c) {
      const double v = t->f.y0[k];
      if (t->rs == 8) {
        ((double *)zb.data())[(size_t)k * t->ld + c] = v;
      } else {
        float *o = (float *)zb.data();
        o[(size_t)k * t->ld + c] = (float)v;
        if (t->comp) o[(size_t)(D + k) * t->ld + c] = (float)(v - (double)(float)v);
      }
    }
  HIP_TRY(hipMemcpy(t->z.p, zb.data(), zb.size(), hipMemcpyHostToDevice));
  t->cur = 0;
  t->step = 0;
  return tmz_write_probe0(t);
}

template <typename Real>
TmzArgs<Real> tmz_args(mln_tmz *t, const FacDev<Real> &fd, const Real (&c)[7]) {
  TmzArgs<Real> a{};
  a.fac = fd;
  const int in = t->cur, out = 1 - t->cur;
  a.Ein = (const Real *)t->E[in].p;
  a.Eout = (Real *)t->E[out].p;
  a.Hxin = (const Real *)t->Hx[in].p;
  a.Hxout = (Real *)t->Hx[out].p;
  a.Hyin = (const Real *)t->Hy[in].p;
  a.Hyout = (Real *)t->Hy[out].p;
  a.z = (Real *)t->z.p;
  a.src = (const Real *)t->src.p;
  a.prof = (const Real *)t->prof.p;
  a.nx = t->grid.nx;
  a.ny = t->grid.ny;
  a.mx0 = t->grid.mx0;
  a.mx1 = t->grid.mx1;
  a.my0 = t->grid.my0;
  a.my1 = t->grid.my1;
  a.ld = t->ld;
  a.chx = c[0];
  a.chy = c[1];
  a.ca = c[2];
  a.cb = c[3];
  a.idx = c[4];
  a.idy = c[5];
  a.kmur = c[6];
  a.pop_out = t->rec.pop_out;
  a.e_out = t->rec.e_out;
  a.probe_out = t->rec.probe_out;
  a.opaque0 = 0;
  return a;
}

template <typename Real>
int tmz_steps_typed(mln_tmz *t, const FacDev<Real> &fd, const Real (&c)[7], int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    TmzArgs<Real> a = tmz_args<Real>(t, fd, c);
    a.n = t->step;
    const int64_t se = t->rec.snap_every;
    a.snap = (se > 0 && (t->step + 1) % se == 0) ? 1 : 0;
    a.snap_i = se > 0 ? (t->step + 1) / se - 1 : 0;
    hipError_t e;
    if constexpr (sizeof(Real) == 8)
      e = launch_tmz<double, false>(t->N, a, t->stream);
    else
      e = t->comp ? launch_tmz<float, true>(t->N, a, t->stream) : launch_tmz<float, false>(t->N, a, t->stream);
    if (e != hipSuccess) return set_err(MLN_EHIP, std::string("TMz launch: ") + hipGetErrorString(e));
    t->cur = 1 - t->cur;
    ++t->step;
  }
  return MLN_OK;
}

int tmz_steps(mln_tmz *t, int64_t n) {
  if (t->rs == 8) {
    const double(&c)[7] = t->c64;
    return tmz_steps_typed<double>(t, t->fd, c, n);
  }
  const float(&c)[7] = t->c32;
  return tmz_steps_typed<float>(t, t->ff, c, n);
}

}  // namespace

extern "C" {

int mln_tmz_init(const mln_medium *medium, const mln_tmz_grid *grid, const mln_tmz_source *source,
                 const mln_tmz_record *record, int32_t precision, void *stream, mln_tmz **out) {
  if (!out) return set_err(MLN_EINVAL, "null output handle");
  *out = nullptr;
  if (!medium || !grid || !source) return set_err(MLN_EINVAL, "need a medium, a grid and a source");
  const mln_tmz_grid &g = *grid;
  if (g.nx < 3 || g.ny < 1 || g.nt < 0) return set_err(MLN_EINVAL, "need nx >= 3, ny >= 1, nt >= 0");
  if (g.ny > (int64_t)kTmzTY * 65535) return set_err(MLN_EINVAL, "ny beyond the launch grid");
  if (!(g.dx > 0) || !(g.dy > 0) || !(g.dt > 0) || !std::isfinite(g.dx) || !std::isfinite(g.dy) ||
      !std::isfinite(g.dt))
    return set_err(MLN_EINVAL, "dx, dy and dt must be positive");
  if (g.mx0 < 1 || g.mx1 < g.mx0 || g.mx1 > g.nx - 1 || g.my0 < 0 || g.my1 < g.my0 || g.my1 > g.ny)
    return set_err(MLN_EINVAL, "medium must satisfy 1 <= mx0 <= mx1 <= nx-1 and 0 <= my0 <= my1 <= ny");
  if (!(g.eps_r > 0) || !(g.mu_r > 0) || !(g.sigma >= 0))
    return set_err(MLN_EINVAL, "eps_r, mu_r must be > 0 and sigma >= 0");
  if (!source->samples || source->n < g.nt + 1 || !source->profile || !std::isfinite(source->amplitude))
    return set_err(MLN_EINVAL, "source needs nt + 1 samples, a finite amplitude and a profile");
  for (int64_t n = 0; n <= g.nt; ++n)
    if (!std::isfinite(source->samples[n])) return set_err(MLN_EINVAL, "non-finite source sample");
  for (int64_t j = 0; j < g.ny; ++j)
    if (!std::isfinite(source->profile[j])) return set_err(MLN_EINVAL, "non-finite source profile");
  if (precision != MLN_FP64 && precision != MLN_FP32 && precision != MLN_FP32_COMP)
    return set_err(MLN_ENOTSUPPORTED, "the TMz solver is built for MLN_FP64, MLN_FP32 and MLN_FP32_COMP");
  const double eps = kEps0 * g.eps_r, mu = kMu0 * g.mu_r;
  const double cl = 1.0 / std::sqrt(eps * mu);
  if (cl * g.dt * std::sqrt(1.0 / (g.dx * g.dx) + 1.0 / (g.dy * g.dy)) > 1.0)
    return set_err(MLN_ECOURANT, "2-D Yee update unstable: c dt sqrt(1/dx^2 + 1/dy^2) > 1");

  std::unique_ptr<mln_tmz> t(new mln_tmz());
  std::string err;
  int rc = build_factors(medium, g.dt, &t->f, &err);
  if (rc) return set_err(rc, err);
  t->N = t->f.N;
  if (t->N != 2 && t->N != 3 && t->N != 4 && t->N != 6)
    return set_err(MLN_ENOTSUPPORTED, "the TMz kernels are built for N = 2, 3, 4 and 6");
  t->grid = g;
  t->rec = record ? *record : mln_tmz_record{};
  if (t->rec.snap_every < 0) return set_err(MLN_EINVAL, "snap_every must be >= 0");
  t->nsnap = t->rec.snap_every > 0 ? g.nt / t->rec.snap_every : 0;
  if (t->nsnap == 0) {
    t->rec.e_out = nullptr;
    t->rec.pop_out = nullptr;
  }
  t->prec = precision;
  t->comp = precision == MLN_FP32_COMP;
  t->rs = precision == MLN_FP64 ? 8 : 4;
  t->stream = (hipStream_t)stream;
  t->nmed = (g.mx1 - g.mx0) * (g.my1 - g.my0);
  t->ld = std::max<int64_t>(1, (t->nmed + 63) / 64 * 64);
  // FDTD coefficients (2-D form of Eq. maxwell, semi-implicit sigma)
  const double sg = g.sigma * g.dt / (2.0 * eps);
  t->c64[0] = g.dt / (mu * g.dx);
  t->c64[1] = g.dt / (mu * g.dy);
  t->c64[2] = (1.0 - sg) / (1.0 + sg);
  t->c64[3] = (g.dt / eps) / (1.0 + sg);
  t->c64[4] = 1.0 / g.dx;
  t->c64[5] = 1.0 / g.dy;
  t->c64[6] = (cl * g.dt - g.dx) / (cl * g.dt + g.dx);
  for (int k = 0; k < 7; ++k) t->c32[k] = (float)t->c64[k];
  courant_pair32(t->c64[0], t->c64[3], t->c64[4], t->c32[0], t->c32[4]);
  courant_pair32(t->c64[1], t->c64[3], t->c64[5], t->c32[1], t->c32[5]);
  t->hs_x = t->c64[1] / (double)t->c32[1];  // H_x is carried scaled by chy32 / chy
  t->hs_y = t->c64[0] / (double)t->c32[0];  // H_y by chx32 / chx
  if (t->rs == 8) {
    rc = upload_factors<double>(t->f, MLN_ROUTE_ROTATION, g.dt, t->fac, t->pop, t->popc, t->fd);
  } else {
    rc = upload_factors<float>(t->f, MLN_ROUTE_ROTATION, g.dt, t->fac, t->pop, t->popc, t->ff);
  }
  if (rc) return rc;
  // source samples (amplitude applied) and profile in the field precision
  t->src_host.resize(g.nt + 1);
  for (int64_t n = 0; n <= g.nt; ++n) t->src_host[n] = source->amplitude * source->samples[n];
  t->prof_host.assign(source->profile, source->profile + g.ny);
  std::vector<unsigned char> buf;
  const size_t cells = (size_t)g.nx * g.ny;
  if (t->rs == 8) to_dev<double>(t->src_host.data(), t->src_host.size(), 1.0, buf);
  else to_dev<float>(t->src_host.data(), t->src_host.size(), 1.0, buf);
  HIP_TRY(t->src.alloc(buf.size()));
  HIP_TRY(hipMemcpy(t->src.p, buf.data(), buf.size(), hipMemcpyHostToDevice));
  if (t->rs == 8) to_dev<double>(t->prof_host.data(), g.ny, 1.0, buf);
  else to_dev<float>(t->prof_host.data(), g.ny, 1.0, buf);
  HIP_TRY(t->prof.alloc(buf.size()));
  HIP_TRY(hipMemcpy(t->prof.p, buf.data(), buf.size(), hipMemcpyHostToDevice));
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(t->E[b].alloc(cells * t->rs));
    HIP_TRY(t->Hx[b].alloc(cells * t->rs));
    HIP_TRY(t->Hy[b].alloc(cells * t->rs));
  }
  const int D = t->f.D;
  HIP_TRY(t->z.alloc((size_t)(t->comp ? 2 * D : D) * t->ld * t->rs));
  rc = tmz_reset(t.get());
  if (rc) return rc;
  *out = t.release();
  return MLN_OK;
}

int mln_tmz_step(mln_tmz *t, int64_t n_steps) {
  if (!t) return set_err(MLN_EINVAL, "null handle");
  if (n_steps < 0) return set_err(MLN_EINVAL, "n_steps must be >= 0");
  return tmz_steps(t, std::min<int64_t>(n_steps, t->grid.nt - t->step));
}

int mln_tmz_run(mln_tmz *t) {
  if (!t) return set_err(MLN_EINVAL, "null handle");
  const int rc = mln_tmz_step(t, t->grid.nt - t->step);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(t->stream));
  return MLN_OK;
}

int mln_tmz_reset(mln_tmz *t) {
  if (!t) return set_err(MLN_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(t->stream));
  return tmz_reset(t);
}

int mln_tmz_current_step(const mln_tmz *t, int64_t *step) {
  if (!t || !step) return set_err(MLN_EINVAL, "null argument");
  *step = t->step;
  return MLN_OK;
}

int mln_tmz_set_fields(mln_tmz *t, const double *Ez, const double *Hx, const double *Hy) {
  if (!t) return set_err(MLN_EINVAL, "null handle");
  const size_t cells = (size_t)t->grid.nx * t->grid.ny;
  for (const double *a : {Ez, Hx, Hy})
    for (size_t i = 0; a && i < cells; ++i)
      if (!std::isfinite(a[i])) return set_err(MLN_EINVAL, "non-finite field value");
  HIP_TRY(hipStreamSynchronize(t->stream));
  std::vector<unsigned char> buf;
  const double sx = t->rs == 8 ? 1.0 : 1.0 / t->hs_x, sy = t->rs == 8 ? 1.0 : 1.0 / t->hs_y;
  const double *src[3] = {Ez, Hx, Hy};
  const double scale[3] = {1.0, sx, sy};
  DevBuf *dst[3] = {&t->E[t->cur], &t->Hx[t->cur], &t->Hy[t->cur]};
  for (int k = 0; k < 3; ++k) {
    if (!src[k]) continue;
    if (t->rs == 8) to_dev<double>(src[k], cells, scale[k], buf);
    else to_dev<float>(src[k], cells, scale[k], buf);
    HIP_TRY(hipMemcpy(dst[k]->p, buf.data(), buf.size(), hipMemcpyHostToDevice));
  }
  if (Ez && t->step == 0) return tmz_write_probe0(t);
  return MLN_OK;
}

int mln_tmz_get_fields(mln_tmz *t, double *Ez, double *Hx, double *Hy) {
  if (!t) return set_err(MLN_EINVAL, "null handle");
  const size_t cells = (size_t)t->grid.nx * t->grid.ny;
  HIP_TRY(hipStreamSynchronize(t->stream));
  std::vector<unsigned char> buf(cells * t->rs);
  double *dst[3] = {Ez, Hx, Hy};
  const double scale[3] = {1.0, t->rs == 8 ? 1.0 : t->hs_x, t->rs == 8 ? 1.0 : t->hs_y};
  DevBuf *src[3] = {&t->E[t->cur], &t->Hx[t->cur], &t->Hy[t->cur]};
  for (int k = 0; k < 3; ++k) {
    if (!dst[k]) continue;
    HIP_TRY(hipMemcpy(buf.data(), src[k]->p, buf.size(), hipMemcpyDeviceToHost));
    if (t->rs == 8) from_dev<double>(buf, cells, scale[k], dst[k]);
    else from_dev<float>(buf, cells, scale[k], dst[k]);
  }
  return MLN_OK;
}

void mln_tmz_free(mln_tmz *t) {
  if (!t) return;
  (void)hipStreamSynchronize(t->stream);
  delete t;
}

}  // extern "C"
