// pol2.hip -- the two-component solver of include/mln.h (mln_pol2_*): both
// transverse field components with H_I = -mu_z E_z - mu_y E_y.  Validation,
// the factors of the split interaction step (host, FP64), device state, the
// launch loop and the kernel instantiations of fwd_pol2.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "fwd_pol2.hpp"
#include "handle.hpp"

using namespace mln;

struct mln_pol2 {
  int N = 0, D = 0, q = 0;
  mln_grid grid{};
  mln_pol2_record rec{};
  hipStream_t stream = nullptr;
  int64_t nmed = 0, ld = 0, step = 0, nsnap = 0;
  int K = 0;      // steps per launch, 0: automatic (pol2_auto_steps)
  int lanes = 4;  // lanes per cell: 1 (K = 1: the one-step kernel, else the tile kernel) or 4 (quad
                  // kernel, N <= 3; the default there, 1 for N = 4, 6)
  int cus = 256;  // compute units of the device
  double amp_z = 0.0, amp_y = 0.0;
  double coef[5] = {0, 0, 0, 0, 0};  // ch, ca, cb, 1/dx, kmur
  std::vector<double> u0, src_host;
  DevBuf fac, src, u[2], Ez[2], Hy[2], Ey[2], G[2];
  int cur = 0;
};

namespace {

template <int N>
hipError_t launch_n(const Pol2Args &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.nx - 1 + 255) / 256);
  hipLaunchKernelGGL((fwd_pol2_kernel<N>), dim3(nb), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_tile_n(const Pol2Args &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.nx + a.owned - 1) / a.owned);
  hipLaunchKernelGGL((fwd_pol2_tile_kernel<N>), dim3(nb), dim3(kPol2TileW), 0, st, a);
  return hipGetLastError();
}

template <int N>
hipError_t launch_quad_n(const Pol2Args &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.nx + a.owned - 1) / a.owned);
  hipLaunchKernelGGL((fwd_pol2_quad_kernel<N>), dim3(nb), dim3(4 * kPol2QuadCells), 0, st, a);
  return hipGetLastError();
}

enum class Pol2Kernel { one_step, tile, quad };

// The largest steps per launch (at least 8) whose workgroups, one per
// compute unit, cover the grid: a step then lasts one workgroup's step on
// every unit, and more steps per launch only spread the launch cost
// further.  Grids larger than that: 12 (quad) or 16 steps per launch.
int pol2_auto_steps(const mln_pol2 *p) {
  const int w = p->lanes == 4 ? kPol2QuadCells : kPol2TileW;
  const int kmax = p->lanes == 4 ? kPol2QuadMaxSteps : kPol2MaxSteps;
  for (int k = kmax; k >= 8; --k) {
    const int64_t owned = w - 2 * k - 1;
    if ((p->grid.nx + owned - 1) / owned <= p->cus) return k;
  }
  return p->lanes == 4 ? 12 : 16;
}

// four lanes per cell: N = 2, 3 only (two components per lane)
hipError_t launch_pol2(int N, Pol2Kernel kind, const Pol2Args &a, hipStream_t st) {
  switch (N) {
    case 2:
      return kind == Pol2Kernel::quad ? launch_quad_n<2>(a, st)
             : kind == Pol2Kernel::tile ? launch_tile_n<2>(a, st) : launch_n<2>(a, st);
    case 3:
      return kind == Pol2Kernel::quad ? launch_quad_n<3>(a, st)
             : kind == Pol2Kernel::tile ? launch_tile_n<3>(a, st) : launch_n<3>(a, st);
    case 4:
      return kind == Pol2Kernel::quad ? hipErrorInvalidValue
             : kind == Pol2Kernel::tile ? launch_tile_n<4>(a, st) : launch_n<4>(a, st);
    case 6:
      return kind == Pol2Kernel::quad ? hipErrorInvalidValue
             : kind == Pol2Kernel::tile ? launch_tile_n<6>(a, st) : launch_n<6>(a, st);
    default: return hipErrorInvalidValue;
  }
}

size_t layout_size(int N) {
  switch (N) {
    case 2: return Pol2Layout<2>::size;
    case 3: return Pol2Layout<3>::size;
    case 4: return Pol2Layout<4>::size;
    case 6: return Pol2Layout<6>::size;
    default: return 0;
  }
}

// X^T Y for D x D row-major X, Y
std::vector<double> tmul(int D, const std::vector<double> &X, const std::vector<double> &Y) {
  std::vector<double> R((size_t)D * D, 0.0);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int k = 0; k < D; ++k) s += X[(size_t)k * D + i] * Y[(size_t)k * D + j];
      R[(size_t)i * D + j] = s;
    }
  return R;
}

// X^T v
std::vector<double> tvec(int D, const std::vector<double> &X, const std::vector<double> &v) {
  std::vector<double> r(D, 0.0);
  for (int i = 0; i < D; ++i)
    for (int k = 0; k < D; ++k) r[i] += X[(size_t)k * D + i] * v[k];
  return r;
}

// The factor block of fwd_pol2.hpp from the factors of the two dipoles (the
// field-free quantities A, c, popd, popc, d'_0 are the same in both).
std::vector<double> pol2_factors(const Factors &fz, const Factors &fy, double dt, std::vector<double> &u0) {
  const int N = fz.N, D = fz.D, Q = fz.q;
  const std::vector<double> &Ty = fy.T;
  std::vector<double> B = tmul(D, Ty, fz.T);  // T_y^T T_z
  std::vector<double> ATy((size_t)D * D, 0.0);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int k = 0; k < D; ++k) s += fz.A[(size_t)i * D + k] * Ty[(size_t)k * D + j];
      ATy[(size_t)i * D + j] = s;
    }
  std::vector<double> K = tmul(D, Ty, ATy);  // T_y^T A T_y
  std::vector<double> c = tvec(D, Ty, fz.c), wz = tvec(D, Ty, fz.w), wy = tvec(D, Ty, fy.w);
  u0 = tvec(D, Ty, fz.dprime0);
  std::vector<double> Bt((size_t)D * D);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) Bt[(size_t)i * D + j] = B[(size_t)j * D + i];
  std::vector<double> blk;
  blk.insert(blk.end(), B.begin(), B.end());
  if (N > 3) blk.insert(blk.end(), Bt.begin(), Bt.end());
  blk.insert(blk.end(), K.begin(), K.end());
  blk.insert(blk.end(), c.begin(), c.end());
  blk.insert(blk.end(), wz.begin(), wz.end());
  blk.insert(blk.end(), wy.begin(), wy.end());
  for (int p = 0; p < Q; ++p) blk.push_back(fy.theta[p] * (0.5 * dt));
  for (int p = 0; p < Q; ++p) blk.push_back(fz.theta[p] * dt);
  for (int a = 0; a < N; ++a)  // population rows in u-coordinates: popd[a,:] T_y
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
      for (int k = 0; k < D; ++k) s += fz.popd[(size_t)a * D + k] * Ty[(size_t)k * D + i];
      blk.push_back(s);
    }
  for (int a = 0; a < N; ++a) blk.push_back(fz.popc[a]);
  blk.push_back(fz.p0);
  blk.push_back(fy.p0);
  return blk;
}

int pol2_reset(mln_pol2 *p) {
  const int64_t nx = p->grid.nx;
  std::vector<double> ez(nx, 0.0), ey(nx, 0.0);
  ez[0] = p->amp_z * p->src_host[0];
  ey[0] = p->amp_y * p->src_host[0];
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(hipMemcpy(p->Ez[b].p, ez.data(), nx * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->Ey[b].p, ey.data(), nx * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(p->Hy[b].p, 0, p->Hy[b].bytes));
    HIP_TRY(hipMemset(p->G[b].p, 0, p->G[b].bytes));
  }
  std::vector<double> ub((size_t)p->D * p->ld, 0.0);
  for (int j = 0; j < p->D; ++j)
    for (int64_t c = 0; c < p->nmed; ++c) ub[(size_t)j * p->ld + c] = p->u0[j];
  HIP_TRY(hipMemcpy(p->u[0].p, ub.data(), ub.size() * sizeof(double), hipMemcpyHostToDevice));
  const double zero = 0.0;  // E at cell nx - 1 before the first step
  if (p->rec.probe_z_out) HIP_TRY(hipMemcpy(p->rec.probe_z_out, &zero, sizeof(double), hipMemcpyHostToDevice));
  if (p->rec.probe_y_out) HIP_TRY(hipMemcpy(p->rec.probe_y_out, &zero, sizeof(double), hipMemcpyHostToDevice));
  p->cur = 0;
  p->step = 0;
  return MLN_OK;
}

int pol2_steps(mln_pol2 *p, int64_t n) {
  const int K = p->K > 0 ? p->K : pol2_auto_steps(p);
  const Pol2Kernel kind = p->lanes == 4 ? Pol2Kernel::quad : K > 1 ? Pol2Kernel::tile : Pol2Kernel::one_step;
  for (int64_t s = 0; s < n;) {
    const int k = (int)std::min<int64_t>(K, n - s);
    Pol2Args a{};
    const int in = p->cur, out = 1 - p->cur;
    a.fac = (const double *)p->fac.p;
    a.Ezin = (const double *)p->Ez[in].p;
    a.Hyin = (const double *)p->Hy[in].p;
    a.Eyin = (const double *)p->Ey[in].p;
    a.Gin = (const double *)p->G[in].p;
    a.Ezout = (double *)p->Ez[out].p;
    a.Hyout = (double *)p->Hy[out].p;
    a.Eyout = (double *)p->Ey[out].p;
    a.Gout = (double *)p->G[out].p;
    a.uin = (const double *)p->u[in].p;
    a.uout = (double *)p->u[out].p;
    a.src = (const double *)p->src.p;
    a.nx = p->grid.nx;
    a.mb = p->grid.med_begin;
    a.me = p->grid.med_end;
    a.ld = p->ld;
    a.n0 = p->step;
    a.nsteps = k;
    a.halo = K;
    a.owned = (kind == Pol2Kernel::quad ? kPol2QuadCells : kPol2TileW) - 2 * K - 1;
    a.amp_z = p->amp_z;
    a.amp_y = p->amp_y;
    a.ch = p->coef[0];
    a.ca = p->coef[1];
    a.cb = p->coef[2];
    a.inv_dx = p->coef[3];
    a.kmur = p->coef[4];
    a.opaque0 = 0;
    // snapshot s is taken when step (s+1) snap_every - 1 completes
    const int64_t se = p->rec.snap_every;
    const int64_t m = se > 0 ? (p->step + se) / se : 0;  // the first snapshot at or after this step, plus one
    a.snap_every = se;
    a.snap_next = se > 0 ? m * se - 1 : -1;
    a.snap_i0 = se > 0 ? m - 1 : 0;
    a.ez_out = p->rec.ez_out;
    a.ey_out = p->rec.ey_out;
    a.pop_out = p->rec.pop_out;
    a.probe_z = p->rec.probe_z_out;
    a.probe_y = p->rec.probe_y_out;
    const hipError_t e = launch_pol2(p->N, kind, a, p->stream);
    if (e != hipSuccess) return set_err(MLN_EHIP, std::string("two-component launch: ") + hipGetErrorString(e));
    p->cur = 1 - p->cur;
    p->step += k;
    s += k;
  }
  return MLN_OK;
}

}  // namespace

extern "C" {

int mln_pol2_init(const mln_medium *medium, const double *dipole_y, const mln_grid *grid,
                  const mln_source *source, double amplitude_y, const mln_pol2_record *record, void *stream,
                  mln_pol2 **out) {
  if (!out) return set_err(MLN_EINVAL, "null output handle");
  *out = nullptr;
  if (!medium || !dipole_y || !grid || !source) return set_err(MLN_EINVAL, "need a medium, dipole_y, a grid and a source");
  const mln_grid &g = *grid;
  if (g.nx < 3 || g.nt < 0) return set_err(MLN_EINVAL, "need nx >= 3 and nt >= 0");
  if (!(g.dx > 0) || !(g.dt > 0) || !std::isfinite(g.dx) || !std::isfinite(g.dt))
    return set_err(MLN_EINVAL, "dx and dt must be positive");
  if (g.med_begin < 1 || g.med_end < g.med_begin || g.med_end > g.nx - 1)
    return set_err(MLN_EINVAL, "medium must satisfy 1 <= med_begin <= med_end <= nx-1");
  if (!(g.eps_r > 0) || !(g.mu_r > 0) || !(g.sigma >= 0))
    return set_err(MLN_EINVAL, "eps_r, mu_r must be > 0 and sigma >= 0");
  const double eps = kEps0 * g.eps_r, mu = kMu0 * g.mu_r;
  const double cl = 1.0 / std::sqrt(eps * mu);
  if (cl * g.dt / g.dx > 1.0 + 1e-12) return set_err(MLN_ECOURANT, "Courant number c dt/dx exceeds 1");
  if (!source->samples || source->n_samples < g.nt + 1) return set_err(MLN_EINVAL, "source needs nt+1 samples");
  if (!std::isfinite(source->amplitude) || !std::isfinite(amplitude_y))
    return set_err(MLN_EINVAL, "non-finite source amplitude");
  for (int64_t i = 0; i <= g.nt; ++i)
    if (!std::isfinite(source->samples[i])) return set_err(MLN_EINVAL, "non-finite source sample");

  std::unique_ptr<mln_pol2> p(new mln_pol2());
  std::string err;
  Factors fz, fy;
  int rc = build_factors(medium, g.dt, &fz, &err);
  if (rc) return set_err(rc, err);
  mln_medium my = *medium;
  my.dipole = dipole_y;
  rc = build_factors(&my, g.dt, &fy, &err);
  if (rc) return set_err(rc, std::string("dipole_y: ") + err);
  p->N = fz.N;
  p->D = fz.D;
  p->q = fz.q;
  if (layout_size(p->N) == 0) return set_err(MLN_ENOTSUPPORTED, "the two-component kernels are built for N = 2, 3, 4, 6");
  p->lanes = p->N <= 3 ? 4 : 1;
  p->grid = g;
  p->rec = record ? *record : mln_pol2_record{};
  if (p->rec.snap_every < 0) return set_err(MLN_EINVAL, "snap_every must be >= 0");
  p->nsnap = p->rec.snap_every > 0 ? g.nt / p->rec.snap_every : 0;
  if (p->nsnap == 0) {
    p->rec.ez_out = nullptr;
    p->rec.ey_out = nullptr;
    p->rec.pop_out = nullptr;
  }
  p->stream = (hipStream_t)stream;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      p->cus = cus;
  }
  p->amp_z = source->amplitude;
  p->amp_y = amplitude_y;
  p->nmed = g.med_end - g.med_begin;
  p->ld = std::max<int64_t>(1, (p->nmed + 63) / 64 * 64);
  // FDTD coefficients (Eq. maxwell, semi-implicit sigma), both components
  const double sg = g.sigma * g.dt / (2.0 * eps);
  p->coef[0] = g.dt / (mu * g.dx);
  p->coef[1] = (1.0 - sg) / (1.0 + sg);
  p->coef[2] = (g.dt / eps) / (1.0 + sg);
  p->coef[3] = 1.0 / g.dx;
  p->coef[4] = (cl * g.dt - g.dx) / (cl * g.dt + g.dx);
  std::vector<double> blk = pol2_factors(fz, fy, g.dt, p->u0);
  if (blk.size() != layout_size(p->N)) return set_err(MLN_EINVAL, "internal: factor block size");
  HIP_TRY(p->fac.alloc(blk.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(p->fac.p, blk.data(), blk.size() * sizeof(double), hipMemcpyHostToDevice));
  p->src_host.assign(source->samples, source->samples + g.nt + 1);
  HIP_TRY(p->src.alloc(p->src_host.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(p->src.p, p->src_host.data(), p->src_host.size() * sizeof(double), hipMemcpyHostToDevice));
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(p->Ez[b].alloc(g.nx * sizeof(double)));
    HIP_TRY(p->Ey[b].alloc(g.nx * sizeof(double)));
    HIP_TRY(p->Hy[b].alloc((g.nx - 1) * sizeof(double)));
    HIP_TRY(p->G[b].alloc((g.nx - 1) * sizeof(double)));
  }
  for (int b = 0; b < 2; ++b) HIP_TRY(p->u[b].alloc((size_t)p->D * p->ld * sizeof(double)));
  rc = pol2_reset(p.get());
  if (rc) return rc;
  *out = p.release();
  return MLN_OK;
}

int mln_pol2_configure(mln_pol2 *p, int steps_per_launch, int lanes_per_cell) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  if (lanes_per_cell != 1 && lanes_per_cell != 4) return set_err(MLN_EINVAL, "lanes_per_cell must be 1 or 4");
  if (lanes_per_cell == 4 && p->N > 3)
    return set_err(MLN_ENOTSUPPORTED, "four lanes per cell hold the Bloch vector for N <= 3 only");
  const int kmax = lanes_per_cell == 4 ? kPol2QuadMaxSteps : kPol2MaxSteps;
  if (steps_per_launch < 0 || steps_per_launch > kmax)
    return set_err(MLN_EINVAL, "steps_per_launch must be in 0.." + std::to_string(kmax) + " with " +
                                   std::to_string(lanes_per_cell) + " lane(s) per cell");
  p->K = steps_per_launch;
  p->lanes = lanes_per_cell;
  return MLN_OK;
}

int mln_pol2_step(mln_pol2 *p, int64_t n_steps) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  if (n_steps < 0) return set_err(MLN_EINVAL, "n_steps must be >= 0");
  return pol2_steps(p, std::min<int64_t>(n_steps, p->grid.nt - p->step));
}

int mln_pol2_run(mln_pol2 *p) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  const int rc = mln_pol2_step(p, p->grid.nt - p->step);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(p->stream));
  return MLN_OK;
}

int mln_pol2_reset(mln_pol2 *p) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(p->stream));
  return pol2_reset(p);
}

int mln_pol2_current_step(const mln_pol2 *p, int64_t *step) {
  if (!p || !step) return set_err(MLN_EINVAL, "null argument");
  *step = p->step;
  return MLN_OK;
}

int mln_pol2_get_fields(mln_pol2 *p, double *Ez, double *Hy, double *Ey, double *Hz) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  HIP_TRY(hipStreamSynchronize(p->stream));
  const int64_t nx = p->grid.nx;
  if (Ez) HIP_TRY(hipMemcpy(Ez, p->Ez[p->cur].p, nx * sizeof(double), hipMemcpyDeviceToHost));
  if (Ey) HIP_TRY(hipMemcpy(Ey, p->Ey[p->cur].p, nx * sizeof(double), hipMemcpyDeviceToHost));
  if (Hy) HIP_TRY(hipMemcpy(Hy, p->Hy[p->cur].p, (nx - 1) * sizeof(double), hipMemcpyDeviceToHost));
  if (Hz) {  // the kernel carries G = -H_z
    HIP_TRY(hipMemcpy(Hz, p->G[p->cur].p, (nx - 1) * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nx - 1; ++i) Hz[i] = -Hz[i];
  }
  return MLN_OK;
}

void mln_pol2_free(mln_pol2 *p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  delete p;
}

}  // extern "C"
