// setup.cpp -- one-time FP64 construction of everything the per-step kernels
// consume: the SU(N) adjoint representation of the medium (Sec. 3 of
// arXiv:1710.09799) and the matrix-exponential factors of Sec. 4.
//
// All of it runs once per medium on the host in double precision; the GPU
// only ever sees the finished factors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mln_internal.hpp"

namespace mln {
namespace {

const cplx kI(0.0, 1.0);

// ---------------------------------------------------------------- helpers

// C = A B for n x n complex row-major
void cmul(int n, const cplx *A, const cplx *B, cplx *C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cplx s = 0.0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      C[i * n + j] = s;
    }
}

// Tr{A B}
cplx ctrace2(int n, const cplx *A, const cplx *B) {
  cplx s = 0.0;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + i];
  return s;
}

// C = A B for real row-major (r x m)(m x c)
void rmul(int r, int m, int c, const double *A, const double *B, double *C) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < c; ++j) {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s += A[i * m + k] * B[k * c + j];
      C[i * c + j] = s;
    }
}

std::vector<double> transpose(int n, const std::vector<double> &A) {
  std::vector<double> T(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T[j * n + i] = A[i * n + j];
  return T;
}

std::vector<cplx> load_c(const double *p, int count) {
  std::vector<cplx> v(count);
  for (int i = 0; i < count; ++i) v[i] = cplx(p[2 * i], p[2 * i + 1]);
  return v;
}

double max_abs(const std::vector<cplx> &a) {
  double m = 0.0;
  for (auto &x : a) m = std::max(m, std::abs(x));
  return m;
}

// exp(X) for a real n x n matrix: scale to ||X||_1 <= 1/8, Taylor series
// summed until the terms stop contributing, then repeated squaring.
void expm_real(int n, const double *X, double *F) {
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(X[i * n + j]);
    nrm = std::max(nrm, s);
  }
  int sq = 0;
  while (std::ldexp(nrm, -sq) > 0.125) ++sq;
  std::vector<double> Y(n * n), term(n * n), tmp(n * n), sum(n * n, 0.0);
  for (int i = 0; i < n * n; ++i) Y[i] = std::ldexp(X[i], -sq);
  for (int i = 0; i < n; ++i) sum[i * n + i] = 1.0;
  term = sum;
  for (int k = 1; k < 40; ++k) {
    rmul(n, n, n, term.data(), Y.data(), tmp.data());
    double tn = 0.0, sn = 0.0;
    for (int i = 0; i < n * n; ++i) {
      term[i] = tmp[i] / k;
      sum[i] += term[i];
      tn = std::max(tn, std::fabs(term[i]));
      sn = std::max(sn, std::fabs(sum[i]));
    }
    if (tn <= 1e-20 * sn) break;
  }
  for (int s = 0; s < sq; ++s) {
    rmul(n, n, n, sum.data(), sum.data(), tmp.data());
    sum.swap(tmp);
  }
  std::memcpy(F, sum.data(), sizeof(double) * n * n);
}

// Hermitian eigen-decomposition A = V diag(m) V^+ by cyclic complex Jacobi
// rotations (each rotation: a phase that makes a_pq real, then a real Givens
// rotation that annihilates it).  Returns false if it does not converge.
bool herm_eig(int n, std::vector<cplx> A, std::vector<double> &m, std::vector<cplx> &V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  double total = 0.0;
  for (auto &x : A) total += std::norm(x);
  bool ok = false;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(A[p * n + q]);
    if (off <= 1e-34 * total || total == 0.0) { ok = true; break; }
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double r = std::abs(A[p * n + q]);
        if (r == 0.0) continue;
        cplx ph = A[p * n + q] / r;
        double al = A[p * n + p].real(), be = A[q * n + q].real();
        double tau = (be - al) / (2.0 * r);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        cplx wpp = c, wpq = s, wqp = -s * std::conj(ph), wqq = c * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // A <- A W
          cplx ap = A[k * n + p], aq = A[k * n + q];
          A[k * n + p] = ap * wpp + aq * wqp;
          A[k * n + q] = ap * wpq + aq * wqq;
          cplx vp = V[k * n + p], vq = V[k * n + q];
          V[k * n + p] = vp * wpp + vq * wqp;
          V[k * n + q] = vp * wpq + vq * wqq;
        }
        for (int k = 0; k < n; ++k) {  // A <- W^+ A
          cplx ap = A[p * n + k], aq = A[q * n + k];
          A[p * n + k] = std::conj(wpp) * ap + std::conj(wqp) * aq;
          A[q * n + k] = std::conj(wpq) * ap + std::conj(wqq) * aq;
        }
      }
  }
  m.resize(n);
  for (int i = 0; i < n; ++i) m[i] = A[i * n + i].real();
  return ok;
}

// ----------------------------------------------------------- the medium

struct Medium {
  int N;
  std::vector<cplx> h0, mu, rho0, relax;
  std::vector<std::vector<cplx>> jump;
  std::vector<double> rate;
  double deph = 0.0, Na = 0.0;
};

// G(X) (paper Eq. liouville): Lindblad channels + pure dephasing + optional
// general linear map on the row-major vectorisation of X.
void relax_map(const Medium &m, const cplx *X, cplx *out) {
  int n = m.N;
  std::vector<cplx> t1(n * n), t2(n * n), LL(n * n);
  for (int i = 0; i < n * n; ++i) out[i] = 0.0;
  for (size_t k = 0; k < m.jump.size(); ++k) {
    const cplx *L = m.jump[k].data();
    double r = m.rate[k];
    cmul(n, L, X, t1.data());  // L X
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        cplx s = 0.0;
        for (int j = 0; j < n; ++j) s += t1[a * n + j] * std::conj(L[b * n + j]);
        t2[a * n + b] = s;  // L X L^+
      }
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        cplx s = 0.0;
        for (int j = 0; j < n; ++j) s += std::conj(L[j * n + a]) * L[j * n + b];
        LL[a * n + b] = s;  // L^+ L
      }
    cmul(n, LL.data(), X, t1.data());
    for (int i = 0; i < n * n; ++i) out[i] += r * (t2[i] - 0.5 * t1[i]);
    cmul(n, X, LL.data(), t1.data());
    for (int i = 0; i < n * n; ++i) out[i] -= 0.5 * r * t1[i];
  }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (a != b) out[a * n + b] -= m.deph * X[a * n + b];
  if (!m.relax.empty()) {
    int n2 = n * n;
    for (int p = 0; p < n2; ++p) {
      cplx s = 0.0;
      for (int q = 0; q < n2; ++q) s += m.relax[p * n2 + q] * X[q];
      out[p] += s;
    }
  }
}

// SU(N) generators of Sec. 3: u_jk = t_jk + t_kj, v_jk = -i (t_jk - t_kj)
// for j < k (lexicographic), then w_l = -sqrt(2/(l(l+1))) (t_11 + .. + t_ll
// - l t_{l+1,l+1}), l = 1..N-1; all satisfy Tr{s_j s_k} = 2 delta_jk.
std::vector<cplx> make_generators(int N) {
  int D = N * N - 1, NN = N * N;
  std::vector<cplx> g(D * NN, 0.0);
  int idx = 0;
  for (int j = 0; j < N; ++j)
    for (int k = j + 1; k < N; ++k, ++idx) {
      g[idx * NN + j * N + k] = 1.0;
      g[idx * NN + k * N + j] = 1.0;
    }
  for (int j = 0; j < N; ++j)
    for (int k = j + 1; k < N; ++k, ++idx) {
      g[idx * NN + j * N + k] = -kI;
      g[idx * NN + k * N + j] = kI;
    }
  for (int l = 1; l <= N - 1; ++l, ++idx) {
    double f = -std::sqrt(2.0 / (l * (l + 1.0)));
    for (int a = 0; a < l; ++a) g[idx * NN + a * N + a] = f;
    g[idx * NN + l * N + l] = -l * f;
  }
  return g;
}

int fail(std::string *err, int code, const std::string &msg) {
  if (err) *err = msg;
  return code;
}

bool is_hermitian(int n, const std::vector<cplx> &A, double rel) {
  double scale = std::max(max_abs(A), 1e-300);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (std::abs(A[a * n + b] - std::conj(A[b * n + a])) > rel * scale) return false;
  return true;
}

bool finite_all(const double *p, int count) {
  for (int i = 0; i < count; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

int build_factors(const mln_medium *md, double dt, Factors *f, std::string *err) {
  if (!md || !f) return fail(err, MLN_EINVAL, "null medium or output");
  const int N = md->n_levels;
  if (N < 2 || N > 6) return fail(err, MLN_ENOTSUPPORTED, "n_levels must be in [2, 6]");
  if (!md->h0 || !md->dipole || !md->rho0) return fail(err, MLN_EINVAL, "h0, dipole and rho0 are required");
  if (md->n_jump < 0 || (md->n_jump > 0 && (!md->jump || !md->jump_rate)))
    return fail(err, MLN_EINVAL, "bad Lindblad channel arrays");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(err, MLN_EINVAL, "dt must be positive");
  if (!(md->density >= 0.0) || !std::isfinite(md->density)) return fail(err, MLN_EINVAL, "density must be >= 0");
  if (!(md->dephasing >= 0.0) || !std::isfinite(md->dephasing)) return fail(err, MLN_EINVAL, "dephasing must be >= 0");
  const int NN = N * N, D = NN - 1, q = N * (N - 1) / 2;
  if (!finite_all(md->h0, 2 * NN) || !finite_all(md->dipole, 2 * NN) || !finite_all(md->rho0, 2 * NN))
    return fail(err, MLN_EINVAL, "non-finite matrix entry");

  Medium m;
  m.N = N;
  m.h0 = load_c(md->h0, NN);
  m.mu = load_c(md->dipole, NN);
  m.rho0 = load_c(md->rho0, NN);
  m.deph = md->dephasing;
  m.Na = md->density;
  for (int k = 0; k < md->n_jump; ++k) {
    if (!finite_all(md->jump + 2 * NN * k, 2 * NN) || !(md->jump_rate[k] >= 0.0))
      return fail(err, MLN_EINVAL, "bad Lindblad channel");
    m.jump.push_back(load_c(md->jump + 2 * NN * k, NN));
    m.rate.push_back(md->jump_rate[k]);
  }
  if (md->relax_superop) {
    if (!finite_all(md->relax_superop, 2 * NN * NN)) return fail(err, MLN_EINVAL, "non-finite relax_superop");
    m.relax = load_c(md->relax_superop, NN * NN);
  }
  if (!is_hermitian(N, m.h0, 1e-12)) return fail(err, MLN_ENOTHERMITIAN, "h0 is not Hermitian");
  if (!is_hermitian(N, m.mu, 1e-12)) return fail(err, MLN_ENOTHERMITIAN, "dipole is not Hermitian");

  // rho0: Hermitian, unit trace, positive semidefinite
  {
    if (!is_hermitian(N, m.rho0, 1e-12)) return fail(err, MLN_EBADRHO, "rho0 is not Hermitian");
    cplx tr = 0.0;
    for (int a = 0; a < N; ++a) tr += m.rho0[a * N + a];
    if (std::abs(tr - 1.0) > 1e-12) return fail(err, MLN_EBADRHO, "rho0 does not have unit trace");
    std::vector<double> ev;
    std::vector<cplx> V;
    if (!herm_eig(N, m.rho0, ev, V)) return fail(err, MLN_ENUMERIC, "eigen-decomposition of rho0 failed");
    if (*std::min_element(ev.begin(), ev.end()) < -1e-12) return fail(err, MLN_EBADRHO, "rho0 is not positive semidefinite");
  }

  // Relaxation: trace preserving, Hermiticity preserving (so that the
  // adjoint representation stays real, Sec. 3).
  std::vector<cplx> X(NN), Y(NN);
  double gscale = m.deph;
  for (double r : m.rate) gscale = std::max(gscale, r);
  if (!m.relax.empty()) gscale = std::max(gscale, max_abs(m.relax));
  for (int p = 0; p < NN; ++p) {
    std::fill(X.begin(), X.end(), cplx(0.0));
    X[p] = 1.0;
    relax_map(m, X.data(), Y.data());
    cplx tr = 0.0;
    for (int a = 0; a < N; ++a) tr += Y[a * N + a];
    if (std::abs(tr) > 1e-12 * std::max(gscale, 1e-300))
      return fail(err, MLN_ENOTTRACEPRESERVING, "relaxation superoperator is not trace preserving");
  }

  Factors &F = *f;
  F = Factors();
  F.N = N;
  F.D = D;
  F.q = q;
  F.gen = make_generators(N);
  const cplx *s = F.gen.data();

  // Eq. elems2: m_jk = (i/2hbar) Tr{H0 [s_j, s_k]} + 1/2 Tr{G(s_k) s_j},
  //             u_jk = -(i/2hbar) Tr{mu [s_j, s_k]};  d_eq (Sec. 3); v (Eq. comp_mu)
  F.M.assign(D * D, 0.0);
  F.U.assign(D * D, 0.0);
  F.deq.assign(D, 0.0);
  F.v.assign(D, 0.0);
  F.d0.assign(D, 0.0);
  std::vector<cplx> C(NN), Gs(D * NN);
  for (int k = 0; k < D; ++k) relax_map(m, s + k * NN, Gs.data() + k * NN);
  double imag_worst = 0.0, mscale = 0.0, hscale = max_abs(m.h0) / kHbar;
  for (int j = 0; j < D; ++j)
    for (int k = 0; k < D; ++k) {
      std::vector<cplx> sjsk(NN), sksj(NN);
      cmul(N, s + j * NN, s + k * NN, sjsk.data());
      cmul(N, s + k * NN, s + j * NN, sksj.data());
      for (int i = 0; i < NN; ++i) C[i] = sjsk[i] - sksj[i];
      cplx mh = kI / (2.0 * kHbar) * ctrace2(N, m.h0.data(), C.data());
      cplx gj = 0.5 * ctrace2(N, Gs.data() + k * NN, s + j * NN);
      cplx uj = -kI / (2.0 * kHbar) * ctrace2(N, m.mu.data(), C.data());
      F.M[j * D + k] = (mh + gj).real();
      F.U[j * D + k] = uj.real();
      imag_worst = std::max(imag_worst, std::fabs(gj.imag()));
      mscale = std::max(mscale, std::abs(gj));
    }
  if (imag_worst > 1e-9 * std::max(std::max(mscale, gscale), 1e-300))
    return fail(err, MLN_EINVAL, "relaxation superoperator does not preserve Hermiticity");
  (void)hscale;
  {
    std::vector<cplx> Id(NN, 0.0), GI(NN);
    for (int a = 0; a < N; ++a) Id[a * N + a] = 1.0;
    relax_map(m, Id.data(), GI.data());
    for (int j = 0; j < D; ++j) {
      F.deq[j] = (ctrace2(N, GI.data(), s + j * NN) / double(N)).real();
      F.v[j] = ctrace2(N, m.mu.data(), s + j * NN).real();
      F.d0[j] = ctrace2(N, m.rho0.data(), s + j * NN).real();
    }
  }

  // L1 half step, exact for any (also singular) M: exp of the augmented
  // matrix [[M, d_eq], [0, 0]] dt/2 = [[A0, b0], [0, 1]], which equals the
  // Sec. 4.1 form A0 (d + d_in) - d_in when M is invertible.
  {
    int n1 = D + 1;
    std::vector<double> Xa(n1 * n1, 0.0), Fa(n1 * n1);
    for (int j = 0; j < D; ++j) {
      for (int k = 0; k < D; ++k) Xa[j * n1 + k] = F.M[j * D + k] * 0.5 * dt;
      Xa[j * n1 + D] = F.deq[j] * 0.5 * dt;
    }
    expm_real(n1, Xa.data(), Fa.data());
    F.A0.assign(D * D, 0.0);
    F.b0.assign(D, 0.0);
    for (int j = 0; j < D; ++j) {
      for (int k = 0; k < D; ++k) F.A0[j * D + k] = Fa[j * n1 + k];
      F.b0[j] = Fa[j * n1 + D];
    }
    if (!finite_all(F.A0.data(), D * D) || !finite_all(F.b0.data(), D))
      return fail(err, MLN_ENUMERIC, "non-finite half-step propagator");
  }

  // Factorisation of U (Sec. 4.2).  U is the adjoint-representation image
  // of rho -> (i/hbar)[mu, rho]; in the eigenbasis mu = V diag(m) V^+ that map
  // turns each coherence rho~_ab by the rate (m_a - m_b)/hbar and leaves the
  // populations alone.  O_jk = 1/2 Tr{s_j V^+ s_k V} is the (orthogonal)
  // change of Bloch basis to that frame; reordering its rows so that
  // (u_ab, v_ab) sit next to each other gives T^T, with T^T U T block
  // diagonal.  This yields exactly the eigenvector pairs the paper pairs into
  // T, also when eigenvalues of U are degenerate.
  {
    std::vector<double> mev;
    std::vector<cplx> V;
    if (!herm_eig(N, m.mu, mev, V)) return fail(err, MLN_ENUMERIC, "eigen-decomposition of the dipole failed");
    std::vector<cplx> Vh(NN), t1(NN), sk(NN);
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) Vh[a * N + b] = std::conj(V[b * N + a]);
    std::vector<double> O(D * D);
    for (int k = 0; k < D; ++k) {
      cmul(N, Vh.data(), s + k * NN, t1.data());
      cmul(N, t1.data(), V.data(), sk.data());  // V^+ s_k V
      for (int j = 0; j < D; ++j) O[j * D + k] = 0.5 * ctrace2(N, s + j * NN, sk.data()).real();
    }
    std::vector<double> Tt(D * D);
    for (int p = 0; p < q; ++p)
      for (int k = 0; k < D; ++k) {
        Tt[(2 * p) * D + k] = O[p * D + k];
        Tt[(2 * p + 1) * D + k] = O[(q + p) * D + k];
      }
    for (int l = 2 * q; l < D; ++l)
      for (int k = 0; k < D; ++k) Tt[l * D + k] = O[l * D + k];
    F.T = transpose(D, Tt);
    // orthogonality check
    std::vector<double> chk(D * D);
    rmul(D, D, D, Tt.data(), F.T.data(), chk.data());
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j)
        if (std::fabs(chk[i * D + j] - (i == j ? 1.0 : 0.0)) > 1e-12)
          return fail(err, MLN_ENUMERIC, "Bloch basis change is not orthogonal");
    std::vector<double> B(D * D), tmp(D * D);
    rmul(D, D, D, Tt.data(), F.U.data(), tmp.data());
    rmul(D, D, D, tmp.data(), F.T.data(), B.data());
    double us = 0.0;
    for (double x : F.U) us = std::max(us, std::fabs(x));
    F.theta.assign(q, 0.0);
    for (int p = 0; p < q; ++p) F.theta[p] = B[(2 * p) * D + 2 * p + 1];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) {
        double want = 0.0;
        if (i / 2 == j / 2 && i < 2 * q && j < 2 * q && i != j) want = (i < j) ? F.theta[i / 2] : -F.theta[i / 2];
        if (std::fabs(B[i * D + j] - want) > 1e-10 * std::max(us, 1e-300))
          return fail(err, MLN_ENUMERIC, "U is not block diagonal in the dipole eigenbasis");
      }
  }

  // Route D (Eq. exp2): U = R Lambda R^+, eigenvector pairs (t_a +- i t_b)/sqrt2
  // with eigenvalues +-i theta; null directions keep eigenvalue 0.
  F.R.assign(D * D, 0.0);
  F.lam.assign(D, 0.0);
  {
    const double r2 = 1.0 / std::sqrt(2.0);
    for (int p = 0; p < q; ++p) {
      for (int i = 0; i < D; ++i) {
        double ta = F.T[i * D + 2 * p], tb = F.T[i * D + 2 * p + 1];
        F.R[i * D + 2 * p] = r2 * cplx(ta, tb);
        F.R[i * D + 2 * p + 1] = r2 * cplx(ta, -tb);
      }
      F.lam[2 * p] = cplx(0.0, F.theta[p]);
      F.lam[2 * p + 1] = cplx(0.0, -F.theta[p]);
    }
    for (int l = 2 * q; l < D; ++l)
      for (int i = 0; i < D; ++i) F.R[i * D + l] = F.T[i * D + l];
  }

  // Route R (generalised Rodrigues, Sec. 4.2) with S_i = T J_i T^T so that
  // U = sum_i theta_i S_i and exp(U x) = I + sum sin(theta_i x) S_i
  // + (1 - cos(theta_i x)) S_i^2.
  F.S.assign(q * D * D, 0.0);
  F.S2.assign(q * D * D, 0.0);
  for (int p = 0; p < q; ++p)
    for (int r = 0; r < D; ++r)
      for (int c = 0; c < D; ++c) {
        double ar = F.T[r * D + 2 * p], br = F.T[r * D + 2 * p + 1];
        double ac = F.T[c * D + 2 * p], bc = F.T[c * D + 2 * p + 1];
        F.S[(p * D + r) * D + c] = ar * bc - br * ac;
        F.S2[(p * D + r) * D + c] = -(ar * ac + br * bc);
      }

  // Full-step quantities.  With the state d' taken after the first half step,
  // one time step is d'' = A_I d', d'_next = A d'' + c with A = A0^2 and
  // c = (A0 + I) b0, and dP/dt = 1/2 N_a v^T (M (A0 d'' + b0) + d_eq).
  F.A.assign(D * D, 0.0);
  rmul(D, D, D, F.A0.data(), F.A0.data(), F.A.data());
  F.c.assign(D, 0.0);
  for (int i = 0; i < D; ++i) {
    double acc = F.b0[i];
    for (int k = 0; k < D; ++k) acc += F.A0[i * D + k] * F.b0[k];
    F.c[i] = acc;
  }
  {
    std::vector<double> MA0(D * D);
    rmul(D, D, D, F.M.data(), F.A0.data(), MA0.data());
    F.w.assign(D, 0.0);
    for (int j = 0; j < D; ++j) {
      double acc = 0.0;
      for (int k = 0; k < D; ++k) acc += MA0[k * D + j] * F.v[k];
      F.w[j] = 0.5 * m.Na * acc;
    }
    double acc = 0.0;
    for (int k = 0; k < D; ++k) {
      double mb = F.deq[k];
      for (int j = 0; j < D; ++j) mb += F.M[k * D + j] * F.b0[j];
      acc += F.v[k] * mb;
    }
    F.p0 = 0.5 * m.Na * acc;
  }
  {
    std::vector<double> Tt = transpose(D, F.T), tmp(D * D);
    rmul(D, D, D, Tt.data(), F.A.data(), tmp.data());
    F.K.assign(D * D, 0.0);
    rmul(D, D, D, tmp.data(), F.T.data(), F.K.data());
    F.cz.assign(D, 0.0);
    F.wz.assign(D, 0.0);
    rmul(D, D, 1, Tt.data(), F.c.data(), F.cz.data());
    rmul(D, D, 1, Tt.data(), F.w.data(), F.wz.data());
  }
  // populations of d^{n+1/2} = A0 d'' + b0 (Eq. comp_rho, diagonal part)
  F.popd.assign(N * D, 0.0);
  F.popz.assign(N * D, 0.0);
  F.popc.assign(N, 1.0 / N);
  for (int a = 0; a < N; ++a) {
    for (int k = 0; k < D; ++k) {
      double sd = s[k * NN + a * N + a].real();
      F.popc[a] += 0.5 * sd * F.b0[k];
      for (int j = 0; j < D; ++j) F.popd[a * D + j] += 0.5 * sd * F.A0[k * D + j];
    }
  }
  rmul(N, D, D, F.popd.data(), F.T.data(), F.popz.data());
  // initial state after the first half step of step 0
  F.dprime0.assign(D, 0.0);
  for (int i = 0; i < D; ++i) {
    double acc = F.b0[i];
    for (int k = 0; k < D; ++k) acc += F.A0[i * D + k] * F.d0[k];
    F.dprime0[i] = acc;
  }
  F.z0.assign(D, 0.0);
  {
    std::vector<double> Tt = transpose(D, F.T);
    rmul(D, D, 1, Tt.data(), F.dprime0.data(), F.z0.data());
  }
  // reference state of the rotation route
  {
    auto residual = [&](const std::vector<double> &z) {  // max |K z + cz - z|
      double r = 0.0;
      for (int i = 0; i < D; ++i) {
        double acc = F.cz[i] - z[i];
        for (int j = 0; j < D; ++j) acc += F.K[i * D + j] * z[j];
        r = std::max(r, std::fabs(acc));
      }
      return r;
    };
    double kn = 0.0, cn = 0.0, zn0 = 0.0;
    for (double x : F.K) kn = std::max(kn, std::fabs(x));
    for (double x : F.cz) cn = std::max(cn, std::fabs(x));
    for (double x : F.z0) zn0 = std::max(zn0, std::fabs(x));
    // solve (I - K) zr = cz by Gaussian elimination with partial pivoting
    std::vector<double> Am(D * D), b = F.cz;
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) Am[i * D + j] = (i == j ? 1.0 : 0.0) - F.K[i * D + j];
    bool ok = true;
    double amax = 0.0;
    for (double x : Am) amax = std::max(amax, std::fabs(x));
    for (int k = 0; k < D && ok; ++k) {
      int p = k;
      for (int i = k + 1; i < D; ++i)
        if (std::fabs(Am[i * D + k]) > std::fabs(Am[p * D + k])) p = i;
      if (std::fabs(Am[p * D + k]) <= 1e-10 * amax) { ok = false; break; }
      if (p != k) {
        for (int j = 0; j < D; ++j) std::swap(Am[k * D + j], Am[p * D + j]);
        std::swap(b[k], b[p]);
      }
      for (int i = k + 1; i < D; ++i) {
        double fct = Am[i * D + k] / Am[k * D + k];
        for (int j = k; j < D; ++j) Am[i * D + j] -= fct * Am[k * D + j];
        b[i] -= fct * b[k];
      }
    }
    std::vector<double> zr(D, 0.0);
    if (ok) {
      for (int k = D - 1; k >= 0; --k) {
        double acc = b[k];
        for (int j = k + 1; j < D; ++j) acc -= Am[k * D + j] * zr[j];
        zr[k] = acc / Am[k * D + k];
      }
      double zn = 0.0;
      for (double x : zr) zn = std::max(zn, std::fabs(x));
      ok = std::isfinite(zn) && zn <= 4.0 && residual(zr) <= 1e-13 * (kn * zn + cn + 1e-300);
    }
    // Prefer the initial state itself when it is a fixed point (the usual
    // case: the medium starts at rest), so that y starts at exactly zero.
    const bool z0_fixed = residual(F.z0) <= 1e-13 * (kn * zn0 + cn + 1e-300);
    const bool stationary = ok || z0_fixed;
    if (z0_fixed) {
      F.zr = F.z0;
    } else if (ok) {
      F.zr = zr;
    } else {
      F.zr.assign(D, 0.0);
    }
    F.rz.assign(D, 0.0);
    F.pr = 0.0;
    if (!stationary) {
      F.rz = F.cz;
      F.pr = F.p0;
    }
    F.y0.assign(D, 0.0);
    for (int i = 0; i < D; ++i) F.y0[i] = F.z0[i] - F.zr[i];
    F.popcy = F.popc;
    for (int a = 0; a < N; ++a)
      for (int j = 0; j < D; ++j) F.popcy[a] += F.popz[a * D + j] * F.zr[j];
  }
  return MLN_OK;
}

}  // namespace mln

// ===================================================================
// Chain rule of the adjoint run: from gradients with respect to the
// d-coordinate step quantities (A = exp(M dt), c, w, p0, U, d'_0) to
// gradients with respect to the physical inputs.  Every physical input enters
// M, U, v, d_eq linearly (Sec. 3, Eqs. elems1/elems2/comp_mu), so their
// directional derivatives are the adjoint-representation images of the
// perturbation itself; the only non-linear step is the augmented exponential,
// whose directional (Frechet) derivative is the upper-right block of
// exp([[X, dX], [0, X]]) (Higham, Functions of Matrices, Sec. 10.6).
namespace mln {
namespace {

// R_jk = 1/2 Tr{map(s_k) s_j},  r_j = 1/N Tr{map(I) s_j}
template <class Map>
void adj_rep(int N, const std::vector<cplx> &gen, Map map, std::vector<double> &R, std::vector<double> &r) {
  const int NN = N * N, D = NN - 1;
  std::vector<cplx> Y(NN), Id(NN, 0.0);
  R.assign(D * D, 0.0);
  r.assign(D, 0.0);
  for (int k = 0; k < D; ++k) {
    map(gen.data() + k * NN, Y.data());
    for (int j = 0; j < D; ++j) R[j * D + k] = 0.5 * ctrace2(N, Y.data(), gen.data() + j * NN).real();
  }
  for (int a = 0; a < N; ++a) Id[a * N + a] = 1.0;
  map(Id.data(), Y.data());
  for (int j = 0; j < D; ++j) r[j] = (ctrace2(N, Y.data(), gen.data() + j * NN) / double(N)).real();
}

// -(i/hbar)[X, Y] for a Hermitian direction X
void commutator_map(int N, const std::vector<cplx> &X, double sign, const cplx *Y, cplx *out) {
  std::vector<cplx> a(N * N), b(N * N);
  cmul(N, X.data(), Y, a.data());
  cmul(N, Y, X.data(), b.data());
  for (int i = 0; i < N * N; ++i) out[i] = sign * (-kI / kHbar) * (a[i] - b[i]);
}

double dotv(const std::vector<double> &a, const double *b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

}  // namespace

int chain_rule(const mln_medium *md, double dt, const double *gA, const double *gc, const double *gw,
               double gp0, const double *gU, const double *gd0, mln_grads *out, std::string *err) {
  Factors F;
  int rc = build_factors(md, dt, &F, err);
  if (rc) return rc;
  if (!out) return fail(err, MLN_EINVAL, "null gradient output");
  const int N = F.N, D = F.D, NN = N * N, n1 = D + 1;
  const double Na = md->density;
  Medium m;
  m.N = N;
  m.deph = 0.0;
  std::vector<double> MA0(D * D), Mb0de(D), A0T(D * D);
  rmul(D, D, D, F.M.data(), F.A0.data(), MA0.data());
  for (int k = 0; k < D; ++k) {
    double s = F.deq[k];
    for (int j = 0; j < D; ++j) s += F.M[k * D + j] * F.b0[j];
    Mb0de[k] = s;
  }
  // exp of the augmented matrix and of its block-doubled version
  std::vector<double> Xa(n1 * n1, 0.0);
  for (int j = 0; j < D; ++j) {
    for (int k = 0; k < D; ++k) Xa[j * n1 + k] = F.M[j * D + k] * 0.5 * dt;
    Xa[j * n1 + D] = F.deq[j] * 0.5 * dt;
  }
  // directional derivative of J for one perturbation (dM, dU, dv, ddeq)
  auto directional = [&](const std::vector<double> &dM, const std::vector<double> &dU,
                         const std::vector<double> &dv, const std::vector<double> &ddeq,
                         double dNa) -> double {
    std::vector<double> dA0(D * D, 0.0), db0(D, 0.0);
    bool lin = false;
    for (double x : dM) lin |= x != 0.0;
    for (double x : ddeq) lin |= x != 0.0;
    if (lin) {
      // L(X, .) is linear: scale the direction to the size of X so that the
      // block exponential is not dominated by it, and scale back afterwards.
      double xmax = 0.0, emax = 0.0;
      for (double x : Xa) xmax = std::max(xmax, std::fabs(x));
      for (double x : dM) emax = std::max(emax, std::fabs(x) * 0.5 * dt);
      for (double x : ddeq) emax = std::max(emax, std::fabs(x) * 0.5 * dt);
      const double alpha = emax / std::max(xmax, 1e-30 * emax);
      const int n2 = 2 * n1;
      std::vector<double> Z(n2 * n2, 0.0), FZ(n2 * n2);
      for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
          Z[i * n2 + j] = Xa[i * n1 + j];
          Z[(n1 + i) * n2 + n1 + j] = Xa[i * n1 + j];
        }
      for (int j = 0; j < D; ++j) {
        for (int k = 0; k < D; ++k) Z[j * n2 + n1 + k] = dM[j * D + k] * 0.5 * dt / alpha;
        Z[j * n2 + n1 + D] = ddeq[j] * 0.5 * dt / alpha;
      }
      expm_real(n2, Z.data(), FZ.data());
      for (int j = 0; j < D; ++j) {
        for (int k = 0; k < D; ++k) dA0[j * D + k] = FZ[j * n2 + n1 + k] * alpha;
        db0[j] = FZ[j * n2 + n1 + D] * alpha;
      }
    }
    std::vector<double> dA(D * D), t1(D * D), t2(D * D);
    rmul(D, D, D, dA0.data(), F.A0.data(), t1.data());
    rmul(D, D, D, F.A0.data(), dA0.data(), t2.data());
    for (int i = 0; i < D * D; ++i) dA[i] = t1[i] + t2[i];
    std::vector<double> dc(D), dw(D), dd0(D);
    for (int i = 0; i < D; ++i) {
      double s = db0[i];
      for (int k = 0; k < D; ++k) s += dA0[i * D + k] * F.b0[k] + F.A0[i * D + k] * db0[k];
      dc[i] = s;
      double s2 = db0[i];
      for (int k = 0; k < D; ++k) s2 += dA0[i * D + k] * F.d0[k];
      dd0[i] = s2;
    }
    // w = 1/2 Na (M A0)^T v
    std::vector<double> dMA0(D * D), t3(D * D);
    rmul(D, D, D, dM.data(), F.A0.data(), dMA0.data());
    rmul(D, D, D, F.M.data(), dA0.data(), t3.data());
    double dp0 = 0.0;
    for (int j = 0; j < D; ++j) {
      double s = 0.0, s0 = 0.0;
      for (int k = 0; k < D; ++k) {
        s += (dMA0[k * D + j] + t3[k * D + j]) * F.v[k] + MA0[k * D + j] * dv[k];
        s0 += MA0[k * D + j] * F.v[k];
      }
      dw[j] = 0.5 * Na * s + 0.5 * dNa * s0;
    }
    {
      double s = 0.0, s0 = 0.0;
      for (int k = 0; k < D; ++k) {
        double inner = ddeq[k];
        for (int j = 0; j < D; ++j) inner += dM[k * D + j] * F.b0[j] + F.M[k * D + j] * db0[j];
        s += dv[k] * Mb0de[k] + F.v[k] * inner;
        s0 += F.v[k] * Mb0de[k];
      }
      dp0 = 0.5 * Na * s + 0.5 * dNa * s0;
    }
    double J = 0.0;
    for (int i = 0; i < D * D; ++i) J += gA[i] * dA[i] + gU[i] * dU[i];
    for (int i = 0; i < D; ++i) J += gc[i] * dc[i] + gw[i] * dw[i] + gd0[i] * dd0[i];
    J += gp0 * dp0;
    return J;
  };
  const std::vector<double> zDD(D * D, 0.0), zD(D, 0.0);
  std::vector<double> R, r;
  // Hermitian directions |a><b| + |b><a| (real) and i|a><b| - i|b><a| (imaginary)
  auto herm_dir = [&](int a, int b, bool imag) {
    std::vector<cplx> X(NN, 0.0);
    if (a == b) {
      X[a * N + a] = 1.0;
    } else if (!imag) {
      X[a * N + b] = 1.0;
      X[b * N + a] = 1.0;
    } else {
      X[a * N + b] = kI;
      X[b * N + a] = -kI;
    }
    return X;
  };
  for (int a = 0; a < N; ++a)
    for (int b = a; b < N; ++b)
      for (int im = 0; im < (a == b ? 1 : 2); ++im) {
        std::vector<cplx> X = herm_dir(a, b, im == 1);
        double jh = 0.0, jm = 0.0;
        if (out->d_h0) {
          adj_rep(N, F.gen, [&](const cplx *Y, cplx *o) { commutator_map(N, X, 1.0, Y, o); }, R, r);
          jh = directional(R, zDD, zD, zD, 0.0);
        }
        if (out->d_dipole) {
          std::vector<double> dU, dv(D);
          // U is the image of rho -> -(i/hbar)[-mu, rho]
          adj_rep(N, F.gen, [&](const cplx *Y, cplx *o) { commutator_map(N, X, -1.0, Y, o); }, dU, r);
          for (int k = 0; k < D; ++k) dv[k] = ctrace2(N, X.data(), F.gen.data() + k * NN).real();
          jm = directional(zDD, dU, dv, zD, 0.0);
        }
        auto put = [&](double *dst, double val) {
          if (!dst) return;
          if (a == b) {
            dst[2 * (a * N + a)] = val;
            dst[2 * (a * N + a) + 1] = 0.0;
          } else if (im == 0) {
            dst[2 * (a * N + b)] = val;
            dst[2 * (b * N + a)] = val;
          } else {
            dst[2 * (a * N + b) + 1] = val;
            dst[2 * (b * N + a) + 1] = -val;
          }
        };
        put(out->d_h0, jh);
        put(out->d_dipole, jm);
      }
  if (out->d_jump_rate)
    for (int k = 0; k < md->n_jump; ++k) {
      Medium one;
      one.N = N;
      one.jump.push_back(load_c(md->jump + 2 * NN * k, NN));
      one.rate.push_back(1.0);
      adj_rep(N, F.gen, [&](const cplx *Y, cplx *o) { relax_map(one, Y, o); }, R, r);
      out->d_jump_rate[k] = directional(R, zDD, zD, r, 0.0);
    }
  if (out->d_dephasing) {
    Medium one;
    one.N = N;
    one.deph = 1.0;
    adj_rep(N, F.gen, [&](const cplx *Y, cplx *o) { relax_map(one, Y, o); }, R, r);
    *out->d_dephasing = directional(R, zDD, zD, r, 0.0);
  }
  if (out->d_density) *out->d_density = directional(zDD, zDD, zD, zD, 1.0);
  return MLN_OK;
}

}  // namespace mln
