// pstd.hip -- the pseudo-spectral (PSTD) field solver of include/mln.h
// (mln_pstd_*): host set-up, launches and the kernel instantiations of
// fwd_pstd.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "fwd_pstd.hpp"
#include "handle.hpp"

using namespace mln;

namespace {

constexpr double kPi = 3.14159265358979323846;

// Largest cells-per-thread count built for N levels and TMAX threads per
// workgroup: a thread holds C cells of E and of the D-component state in
// registers (256 VGPRs per lane at 512 threads, 512 VGPRs and AGPRs at 256).
int pstd_max_cells(int N, int tmax) {
  switch (N) {
    case 2: return tmax == 256 ? 16 : 8;
    case 3: return tmax == 256 ? 16 : 8;
    case 4: return tmax == 256 ? 8 : 4;
    case 6: return tmax == 256 ? 4 : 2;
    default: return 0;
  }
}

template <int N, int C, int TMAX>
hipError_t launch_n(const PstdArgs &a, int n_inst, int threads, size_t lds, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute((const void *)fwd_pstd_kernel<N, C, TMAX>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((fwd_pstd_kernel<N, C, TMAX>), dim3((unsigned)n_inst), dim3(threads), lds, st, a);
  return hipGetLastError();
}

template <int N, int TMAX>
hipError_t launch_c(int C, const PstdArgs &a, int n_inst, int threads, size_t lds, hipStream_t st) {
  constexpr int cmax = N == 2 ? (TMAX == 256 ? 16 : 8)
                     : N == 3 ? (TMAX == 256 ? 16 : 8)
                     : N == 4 ? (TMAX == 256 ? 8 : 4)
                              : (TMAX == 256 ? 4 : 2);
  switch (C) {
    case 1: return launch_n<N, 1, TMAX>(a, n_inst, threads, lds, st);
    case 2: return launch_n<N, 2, TMAX>(a, n_inst, threads, lds, st);
    case 4:
      if constexpr (cmax >= 4) return launch_n<N, 4, TMAX>(a, n_inst, threads, lds, st);
      break;
    case 8:
      if constexpr (cmax >= 8) return launch_n<N, 8, TMAX>(a, n_inst, threads, lds, st);
      break;
    case 16:
      if constexpr (cmax >= 16) return launch_n<N, 16, TMAX>(a, n_inst, threads, lds, st);
      break;
  }
  return hipErrorInvalidValue;
}

template <int TMAX>
hipError_t launch_t(int N, int C, const PstdArgs &a, int n_inst, int threads, size_t lds, hipStream_t st) {
  switch (N) {
    case 2: return launch_c<2, TMAX>(C, a, n_inst, threads, lds, st);
    case 3: return launch_c<3, TMAX>(C, a, n_inst, threads, lds, st);
    case 4: return launch_c<4, TMAX>(C, a, n_inst, threads, lds, st);
    case 6: return launch_c<6, TMAX>(C, a, n_inst, threads, lds, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pstd(int N, int C, int tmax, const PstdArgs &a, int n_inst, int threads, size_t lds,
                       hipStream_t st) {
  if (threads > tmax) return hipErrorInvalidValue;
  return tmax == 256 ? launch_t<256>(N, C, a, n_inst, threads, lds, st)
                     : launch_t<512>(N, C, a, n_inst, threads, lds, st);
}

}  // namespace

struct mln_pstd {
  struct Inst {
    Factors f;
    DevBuf fac, pop, popc;
    FacDev<double> fd{};
    mln_record rec{};
    double *d_probe = nullptr, *d_e = nullptr, *d_pop = nullptr;
    DevBuf st_probe, st_e, st_pop;  // device staging for host outputs
  };
  int N = 0, n_inst = 0;
  mln_grid grid{};
  int C = 1, threads = 0, tmax = 256, log2m = 0;
  int n_cu = 256;  // compute units of the device the handle was created on
  size_t lds = 0;
  hipStream_t stream = nullptr;
  int64_t nmed = 0, ld = 0, step = 0;
  int spl = 256;  // time steps per launch
  int64_t snap_every = 0, nsnap = 0;
  double ca = 0, cb = 0, ah = 0, be = 0;
  std::vector<std::unique_ptr<Inst>> inst;
  DevBuf E, H, z, tab, dinst;
  std::vector<double> e_init, h_init, z_init;
};

namespace {

int pstd_reset(mln_pstd *p) {
  const int64_t nx = p->grid.nx;
  HIP_TRY(hipMemcpyAsync(p->E.p, p->e_init.data(), p->e_init.size() * sizeof(double), hipMemcpyHostToDevice,
                         p->stream));
  HIP_TRY(hipMemcpyAsync(p->H.p, p->h_init.data(), p->h_init.size() * sizeof(double), hipMemcpyHostToDevice,
                         p->stream));
  HIP_TRY(hipMemcpyAsync(p->z.p, p->z_init.data(), p->z_init.size() * sizeof(double), hipMemcpyHostToDevice,
                         p->stream));
  for (int i = 0; i < p->n_inst; ++i)
    if (p->inst[i]->d_probe)
      HIP_TRY(hipMemcpyAsync(p->inst[i]->d_probe, &p->e_init[(size_t)i * nx + nx - 1], sizeof(double),
                             hipMemcpyHostToDevice, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->step = 0;
  return MLN_OK;
}

int pstd_steps(mln_pstd *p, int64_t n) {
  PstdArgs a{};
  a.inst = (const PstdInst *)p->dinst.p;
  a.tab = (const double2 *)p->tab.p;
  a.nx = p->grid.nx;
  a.mb = p->grid.med_begin;
  a.me = p->grid.med_end;
  a.ld = p->ld;
  a.log2m = p->log2m;
  a.pt_size = pstd_pt_size(p->log2m);
  a.snap_every = p->snap_every;
  a.ca = p->ca;
  a.cb = p->cb;
  a.ah = p->ah;
  a.be = p->be;
  a.opaque0 = 0;
  while (n > 0) {
    const int k = (int)std::min<int64_t>(n, p->spl);
    a.step0 = p->step;
    a.nsteps = k;
    a.snap_next = -1;
    a.snap_i0 = 0;
    if (a.snap_every > 0) {  // first step n >= step0 with (n+1) % snap_every == 0
      const int64_t q = a.step0 / a.snap_every;
      a.snap_next = (q + 1) * a.snap_every - 1;
      a.snap_i0 = q;
    }
    hipError_t e = launch_pstd(p->N, p->C, p->tmax, a, p->n_inst, p->threads, p->lds, p->stream);
    if (e != hipSuccess) return set_err(MLN_EHIP, std::string("PSTD launch: ") + hipGetErrorString(e));
    p->step += k;
    n -= k;
  }
  return MLN_OK;
}

// Threads per workgroup: at most tmax (256 or 512), fewer on grids below
// that; C = nx / threads cells per thread.  Automatic (0), from measured
// step times: 512 where that shape is built (one problem steps fastest with
// the medium spread over more threads), except N = 6, whose 35-component
// state fits one thread's registers only at 256, and except batches of more
// problems than compute units on grids of at most 1024 cells, where two
// 256-thread workgroups share a compute unit (about 1.3x the throughput).
int set_shape(mln_pstd *p, int tmax) {
  if (tmax == 0) {
    const bool shared_cu = p->grid.nx <= 1024 && p->n_inst > p->n_cu;
    tmax = (p->N < 6 && !shared_cu && p->grid.nx <= 512 * pstd_max_cells(p->N, 512)) ? 512 : 256;
  }
  if (tmax != 256 && tmax != 512) return set_err(MLN_EINVAL, "PSTD threads per workgroup: 0, 256 or 512");
  const int64_t nx = p->grid.nx;
  const int threads = (int)std::min<int64_t>(nx, tmax);
  const int C = (int)(nx / threads);
  if (C > pstd_max_cells(p->N, tmax))
    return set_err(MLN_ENOTSUPPORTED, "PSTD grid of " + std::to_string((long long)nx) + " cells needs " +
                                          std::to_string(C) + " cells per thread at " + std::to_string(tmax) +
                                          " threads: more than are built for N = " + std::to_string(p->N));
  p->tmax = tmax;
  p->threads = threads;
  p->C = C;
  return MLN_OK;
}

}  // namespace

extern "C" {

int mln_pstd_init(int32_t n_inst, const mln_medium *media, const mln_grid *grid, const double *e_init,
                  const double *h_init, const mln_record *records, void *stream, mln_pstd **out) {
  if (!out) return set_err(MLN_EINVAL, "null output handle");
  *out = nullptr;
  if (n_inst < 1 || !media || !grid) return set_err(MLN_EINVAL, "need n_inst >= 1, media and a grid");
  const mln_grid &g = *grid;
  const int64_t nx = g.nx;
  if (nx < kPstdMinCells || (nx & (nx - 1)) != 0)
    return set_err(MLN_EINVAL, "PSTD grid: nx must be a power of two >= 64");
  if (g.nt < 0) return set_err(MLN_EINVAL, "nt must be >= 0");
  if (!(g.dx > 0) || !(g.dt > 0) || !std::isfinite(g.dx) || !std::isfinite(g.dt))
    return set_err(MLN_EINVAL, "dx and dt must be positive");
  if (g.med_begin < 1 || g.med_end < g.med_begin || g.med_end > nx - 1)
    return set_err(MLN_EINVAL, "medium must satisfy 1 <= med_begin <= med_end <= nx-1");
  if (!(g.eps_r > 0) || !(g.mu_r > 0) || !(g.sigma >= 0))
    return set_err(MLN_EINVAL, "eps_r, mu_r must be > 0 and sigma >= 0");
  const double eps = kEps0 * g.eps_r, mu = kMu0 * g.mu_r;
  const double cl = 1.0 / std::sqrt(eps * mu);
  const int64_t M = nx / 2;
  // leapfrog stability for the largest kept wavenumber: c kappa dt / 2 < 1
  const double kap_max = 2.0 * kPi * (double)(M - 1) / ((double)nx * g.dx);
  if (!(cl * kap_max * g.dt / 2.0 < 1.0))
    return set_err(MLN_ECOURANT, "PSTD leapfrog unstable: c dt kappa_max / 2 >= 1");
  const int N = media[0].n_levels;
  if (pstd_max_cells(N, 256) == 0) return set_err(MLN_ENOTSUPPORTED, "PSTD kernels are built for N = 2, 3, 4 and 6");
  for (int i = 1; i < n_inst; ++i)
    if (media[i].n_levels != N) return set_err(MLN_EINVAL, "all PSTD instances need the same level count");
  if (nx > 256 * pstd_max_cells(N, 256))
    return set_err(MLN_ENOTSUPPORTED, "PSTD grid too large for N = " + std::to_string(N) + ": nx <= " +
                                          std::to_string(256 * pstd_max_cells(N, 256)));
  int64_t se = 0;
  if (records) {
    se = records[0].snap_every;
    for (int i = 0; i < n_inst; ++i)
      if (records[i].snap_every != se) return set_err(MLN_EINVAL, "all records need the same snap_every");
    if (se < 0) return set_err(MLN_EINVAL, "snap_every must be >= 0");
  }
  auto ctx = [](int i) { return "instance " + std::to_string(i) + ": "; };
  if (e_init)
    for (int64_t i = 0; i < (int64_t)n_inst * nx; ++i)
      if (!std::isfinite(e_init[i])) return set_err(MLN_EINVAL, "non-finite initial E");
  if (h_init)
    for (int64_t i = 0; i < (int64_t)n_inst * nx; ++i)
      if (!std::isfinite(h_init[i])) return set_err(MLN_EINVAL, "non-finite initial H");

  std::unique_ptr<mln_pstd> p(new mln_pstd());
  int rc0 = 0;
  p->N = N;
  p->n_inst = n_inst;
  p->grid = g;
  {
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (cus > 0) p->n_cu = cus;
  }
  rc0 = set_shape(p.get(), 0);
  if (rc0) return rc0;
  p->log2m = 0;
  while ((int64_t(1) << p->log2m) < M) ++p->log2m;
  p->lds = (size_t)(2 * M + pstd_pt_size(p->log2m)) * sizeof(double2);
  p->stream = (hipStream_t)stream;
  p->nmed = g.med_end - g.med_begin;
  p->ld = std::max<int64_t>(1, (p->nmed + 63) / 64 * 64);
  p->snap_every = se;
  p->nsnap = se > 0 ? g.nt / se : 0;
  // field coefficients: semi-implicit conductivity as on the Yee grid
  const double sg = g.sigma * g.dt / (2.0 * eps);
  p->ca = (1.0 - sg) / (1.0 + sg);
  p->cb = (g.dt / eps) / (1.0 + sg);
  const double k0 = 2.0 * kPi / ((double)nx * g.dx);
  p->ah = (g.dt / mu) * k0;
  p->be = (p->cb / (double)M) * k0;
  const int D = N * N - 1;
  p->e_init.assign((size_t)n_inst * nx, 0.0);
  p->h_init.assign((size_t)n_inst * nx, 0.0);
  if (e_init) std::copy(e_init, e_init + (size_t)n_inst * nx, p->e_init.begin());
  if (h_init) std::copy(h_init, h_init + (size_t)n_inst * nx, p->h_init.begin());
  p->z_init.assign((size_t)n_inst * D * p->ld, 0.0);
  HIP_TRY(p->E.alloc((size_t)n_inst * nx * sizeof(double)));
  HIP_TRY(p->H.alloc((size_t)n_inst * nx * sizeof(double)));
  HIP_TRY(p->z.alloc((size_t)n_inst * D * p->ld * sizeof(double)));
  std::vector<PstdInst> hi(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    std::unique_ptr<mln_pstd::Inst> I(new mln_pstd::Inst());
    std::string err;
    int rc = build_factors(&media[i], g.dt, &I->f, &err);
    if (rc) return set_err(rc, ctx(i) + err);
    rc = upload_factors<double>(I->f, MLN_ROUTE_ROTATION, g.dt, I->fac, I->pop, I->popc, I->fd);
    if (rc) return rc;
    for (int j = 0; j < D; ++j)
      for (int64_t c = 0; c < p->nmed; ++c) p->z_init[((size_t)i * D + j) * p->ld + c] = I->f.y0[j];
    I->rec = records ? records[i] : mln_record{};
    const mln_record &r = I->rec;
    if (r.out_on_device) {
      I->d_probe = r.probe_out;
      I->d_e = r.e_out;
      I->d_pop = r.pop_out;
    } else {
      if (r.probe_out) {
        HIP_TRY(I->st_probe.alloc(sizeof(double) * (g.nt + 1)));
        I->d_probe = (double *)I->st_probe.p;
      }
      if (r.e_out && p->nsnap) {
        HIP_TRY(I->st_e.alloc(sizeof(double) * p->nsnap * nx));
        I->d_e = (double *)I->st_e.p;
      }
      if (r.pop_out && p->nsnap) {
        HIP_TRY(I->st_pop.alloc(sizeof(double) * p->nsnap * N * std::max<int64_t>(p->nmed, 1)));
        I->d_pop = (double *)I->st_pop.p;
      }
    }
    if (p->nsnap == 0) {
      I->d_e = nullptr;
      I->d_pop = nullptr;
    }
    PstdInst &d = hi[i];
    d.fac = I->fd;
    d.E = (double *)p->E.p + (size_t)i * nx;
    d.H = (double *)p->H.p + (size_t)i * nx;
    d.z = (double *)p->z.p + (size_t)i * D * p->ld;
    d.probe = I->d_probe;
    d.e_out = I->d_e;
    d.pop_out = I->d_pop;
    p->inst.push_back(std::move(I));
  }
  HIP_TRY(p->dinst.alloc(hi.size() * sizeof(PstdInst)));
  HIP_TRY(hipMemcpy(p->dinst.p, hi.data(), hi.size() * sizeof(PstdInst), hipMemcpyHostToDevice));
  // pass twiddles W_4h^j = exp(-2 pi i j / (4h)), j < h, for every radix-4
  // span h (at (h - h0) / 3); then per mode pair u (k = M/2 for u = 0, else
  // the bit reversal of 2u) exp(-2 pi i k / nx) and exp(-i pi k / nx)
  const int lm = p->log2m;
  const int pts = pstd_pt_size(lm);
  std::vector<double2> tab((size_t)pts + M);
  const int h0 = (lm & 1) ? 2 : 1;
  for (int h = h0; 4 * h <= M; h *= 4)
    for (int j = 0; j < h; ++j) {
      const double ph = 2.0 * kPi * (double)j / (4.0 * h);
      tab[(h - h0) / 3 + j] = make_double2(std::cos(ph), -std::sin(ph));
    }
  auto rev = [lm](int64_t v) {
    int64_t r = 0;
    for (int b = 0; b < lm; ++b) r |= ((v >> b) & 1) << (lm - 1 - b);
    return r;
  };
  for (int64_t u = 0; u < M / 2; ++u) {
    const int64_t k = u ? rev(2 * u) : M / 2;
    const double pw = 2.0 * kPi * (double)k / (double)nx, pe = kPi * (double)k / (double)nx;
    tab[pts + u] = make_double2(std::cos(pw), -std::sin(pw));
    tab[pts + M / 2 + u] = make_double2(std::cos(pe), -std::sin(pe));
  }
  HIP_TRY(p->tab.alloc(tab.size() * sizeof(double2)));
  HIP_TRY(hipMemcpy(p->tab.p, tab.data(), tab.size() * sizeof(double2), hipMemcpyHostToDevice));
  int rc = pstd_reset(p.get());
  if (rc) return rc;
  *out = p.release();
  return MLN_OK;
}

int mln_pstd_configure(mln_pstd *p, int32_t steps_per_launch, int32_t max_threads) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  if (steps_per_launch < 0) return set_err(MLN_EINVAL, "steps_per_launch must be >= 0");
  const int rc = set_shape(p, max_threads);
  if (rc) return rc;
  p->spl = steps_per_launch ? steps_per_launch : 256;
  return MLN_OK;
}

int mln_pstd_step(mln_pstd *p, int64_t n_steps) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  if (n_steps < 0) return set_err(MLN_EINVAL, "n_steps must be >= 0");
  return pstd_steps(p, std::min<int64_t>(n_steps, p->grid.nt - p->step));
}

int mln_pstd_run(mln_pstd *p) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  int rc = mln_pstd_step(p, p->grid.nt - p->step);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(p->stream));
  const int64_t nx = p->grid.nx;
  for (int i = 0; i < p->n_inst; ++i) {
    mln_pstd::Inst &I = *p->inst[i];
    if (I.rec.out_on_device) continue;
    if (I.st_probe.p)
      HIP_TRY(hipMemcpy(I.rec.probe_out, I.st_probe.p, sizeof(double) * (p->grid.nt + 1), hipMemcpyDeviceToHost));
    if (I.st_e.p)
      HIP_TRY(hipMemcpy(I.rec.e_out, I.st_e.p, sizeof(double) * p->nsnap * nx, hipMemcpyDeviceToHost));
    if (I.st_pop.p)
      HIP_TRY(hipMemcpy(I.rec.pop_out, I.st_pop.p, sizeof(double) * p->nsnap * p->N * p->nmed,
                        hipMemcpyDeviceToHost));
    if (I.rec.probe_out)
      for (int64_t n = 0; n <= p->grid.nt; ++n)
        if (!std::isfinite(I.rec.probe_out[n]))
          return set_err(MLN_ENONFINITE, "instance " + std::to_string(i) + ": non-finite probe value");
  }
  return MLN_OK;
}

int mln_pstd_reset(mln_pstd *p) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  return pstd_reset(p);
}

int mln_pstd_current_step(const mln_pstd *p, int64_t *step) {
  if (!p || !step) return set_err(MLN_EINVAL, "null argument");
  *step = p->step;
  return MLN_OK;
}

int mln_pstd_get_config(const mln_pstd *p, int32_t *threads, int32_t *cells_per_thread,
                        int32_t *steps_per_launch) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  if (threads) *threads = p->threads;
  if (cells_per_thread) *cells_per_thread = p->C;
  if (steps_per_launch) *steps_per_launch = p->spl;
  return MLN_OK;
}

int mln_pstd_get_fields(mln_pstd *p, int32_t inst, double *E, double *H) {
  if (!p) return set_err(MLN_EINVAL, "null handle");
  if (inst < 0 || inst >= p->n_inst) return set_err(MLN_EINVAL, "instance index out of range");
  const int64_t nx = p->grid.nx;
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (E)
    HIP_TRY(hipMemcpy(E, (double *)p->E.p + (size_t)inst * nx, nx * sizeof(double), hipMemcpyDeviceToHost));
  if (H)
    HIP_TRY(hipMemcpy(H, (double *)p->H.p + (size_t)inst * nx, nx * sizeof(double), hipMemcpyDeviceToHost));
  return MLN_OK;
}

void mln_pstd_free(mln_pstd *p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  delete p;
}

}  // extern "C"
