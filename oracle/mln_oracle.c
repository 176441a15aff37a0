/*
 * mln_oracle.c -- plain FP64 CPU reference for the Maxwell-Liouville-von
 * Neumann (MLN) system of Riesch & Jirauschek, arXiv:1710.09799.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark call this code.  It shares no source,
 * header, table or helper with the GPU library; the only thing the two sides
 * have in common is the seeded input description (medium, grid, source
 * samples) produced in Python.
 *
 * What it computes (deliberately the slow, obvious way):
 *   * the FULL complex N x N density matrix of every medium cell -- no
 *     adjoint / Bloch-vector representation anywhere;
 *   * the field-free generator L0 + G (Sec. 2, Eq. liouville) as an
 *     N^2 x N^2 superoperator S acting on the row-major vectorisation of rho,
 *     built by applying the map to every basis matrix |c><d|;
 *   * the symmetric Strang splitting of Sec. 4.1 (Eqs. for d', d'', d^{n+1/2})
 *     carried out on rho:  half step exp(S dt/2), full interaction step
 *     rho -> W rho W^+ with W = exp(+i mu E^n dt / hbar) (the exact flow of
 *     -i/hbar [-mu E, rho] for a field frozen at the midpoint value E^n),
 *     half step exp(S dt/2);
 *   * every matrix exponential by ONE generic scaling-and-squaring diagonal
 *     Pade approximant [6/6] (Moler & Van Loan, "Nineteen dubious ways",
 *     Sec. 3: with ||X||_1 <= 1/2 the [6/6] backward error is below 3.4e-16),
 *     LU with partial pivoting, no structure exploited;
 *   * the polarisation derivative from Eq. polarization2,
 *     dP/dt = N_a Re Tr{ mu (L0(rho) + G(rho)) }, evaluated on rho^{n+1/2};
 *   * the 1-D Yee FDTD update of Eq. maxwell on the staggered grid of Fig. 1;
 *   * the FP64 adjoint of that discrete map (orc_grad): reverse mode through
 *     every step, matrix-exponential derivatives from the block identity for
 *     the Frechet derivative, gradients with respect to H0, the dipole
 *     matrix, the jump and dephasing rates, N_a and the source amplitude;
 *   * a pseudo-spectral (PSTD) field solver on a periodic grid
 *     (orc_pstd_run): the same leapfrog and medium step with the spatial
 *     derivatives taken from direct DFT sums;
 *   * the same medium step on a two-dimensional TMz Yee grid (orc_run2d),
 *     the extension past the one-dimensional models the paper restricts
 *     itself to (Conclusion);
 *   * both transverse field components with an interaction Hamiltonian
 *     -mu_z E_z - mu_y E_y (orc_run_pol2), the extension past the single
 *     component and fixed interaction form the paper keeps (Sec. 2,
 *     Conclusion).
 *
 * Readings of points the paper leaves open (same on the GPU side, but written
 * independently there):
 *   * hard source E(cell 0, step n) = amp * src[n];
 *   * first-order Mur absorbing boundary at cell nx-1 with coefficient
 *     (c dt - dx)/(c dt + dx), c = 1/sqrt(eps mu);
 *   * conductivity handled semi-implicitly (average of E^n and E^{n+1});
 *   * the medium occupies cells [med_begin, med_end), 1 <= begin <= end <= nx-1;
 *   * snapshot s records E^{(s+1) k} and the populations of rho^{(s+1)k - 1/2}
 *     for k = snap_every; the probe records E at cell nx-1 for steps 0..nt.
 *
 * Physical constants: CODATA 2018.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cx;

#define ORC_HBAR 1.054571817e-34
#define ORC_C0 299792458.0
#define ORC_EPS0 8.8541878128e-12
#define ORC_MU0 1.25663706212e-6

#define PADE_Q 6

void orc_constants(double *out)
{
    out[0] = ORC_HBAR;
    out[1] = ORC_C0;
    out[2] = ORC_EPS0;
    out[3] = ORC_MU0;
}

/* ----------------------------------------------------------------------- */
/* dense complex linear algebra, row-major n x n                            */

static void mat_mul(int n, const cx *A, const cx *B, cx *C)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cx s = 0;
            for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
            C[i * n + j] = s;
        }
}

/* Solve A X = B for X (n x n right-hand sides), Gaussian elimination with
 * partial pivoting.  A and B are overwritten; X is returned in B. */
static int lu_solve(int n, cx *A, cx *B)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = cabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (cabs(A[i * n + k]) > best) { best = cabs(A[i * n + k]); p = i; }
        if (best == 0.0) return -1;
        if (p != k)
            for (int j = 0; j < n; ++j) {
                cx t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t;
                t = B[k * n + j]; B[k * n + j] = B[p * n + j]; B[p * n + j] = t;
            }
        for (int i = k + 1; i < n; ++i) {
            cx f = A[i * n + k] / A[k * n + k];
            if (f == 0) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int j = 0; j < n; ++j) B[i * n + j] -= f * B[k * n + j];
        }
    }
    for (int k = n - 1; k >= 0; --k)
        for (int j = 0; j < n; ++j) {
            cx s = B[k * n + j];
            for (int i = k + 1; i < n; ++i) s -= A[k * n + i] * B[i * n + j];
            B[k * n + j] = s / A[k * n + k];
        }
    return 0;
}

static double fact(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Coefficient c_k of the diagonal [q/q] Pade numerator of exp:
 * c_k = (2q-k)! q! / ((2q)! k! (q-k)!)   (Moler & Van Loan, Sec. 3). */
double orc_pade_coef(int q, int k)
{
    return fact(2 * q - k) * fact(q) / (fact(2 * q) * fact(k) * fact(q - k));
}

/* F = exp(A) for a general complex n x n matrix.  work: 5 n^2 complex. */
static int expm_work(int n, const cx *A, cx *F, cx *work)
{
    cx *X = work, *P = work + n * n, *T = work + 2 * n * n;
    cx *Nm = work + 3 * n * n, *Dm = work + 4 * n * n;
    double nrm = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += cabs(A[i * n + j]);
        if (s > nrm) nrm = s;
    }
    int sq = 0;
    double scale = 1.0;
    while (nrm * scale > 0.5) { scale *= 0.5; ++sq; }
    for (int i = 0; i < n * n; ++i) X[i] = A[i] * scale;
    /* P = X^k, accumulated powers */
    for (int i = 0; i < n * n; ++i) { P[i] = 0; Nm[i] = 0; Dm[i] = 0; }
    for (int i = 0; i < n; ++i) { P[i * n + i] = 1; }
    for (int k = 0; k <= PADE_Q; ++k) {
        double c = orc_pade_coef(PADE_Q, k);
        double sg = (k % 2) ? -1.0 : 1.0;
        for (int i = 0; i < n * n; ++i) { Nm[i] += c * P[i]; Dm[i] += sg * c * P[i]; }
        if (k < PADE_Q) {
            mat_mul(n, P, X, T);
            memcpy(P, T, sizeof(cx) * n * n);
        }
    }
    if (lu_solve(n, Dm, Nm)) return -1;
    for (int s = 0; s < sq; ++s) {
        mat_mul(n, Nm, Nm, T);
        memcpy(Nm, T, sizeof(cx) * n * n);
    }
    memcpy(F, Nm, sizeof(cx) * n * n);
    return 0;
}

/* exported for the oracle's own pin tests: interleaved (re, im) arrays */
int orc_expm(int n, const double *A, double *F)
{
    cx *w = (cx *)malloc(sizeof(cx) * (size_t)n * n * 7);
    cx *a = w + 5 * n * n, *f = w + 6 * n * n;
    for (int i = 0; i < n * n; ++i) a[i] = A[2 * i] + I * A[2 * i + 1];
    int rc = expm_work(n, a, f, w);
    for (int i = 0; i < n * n; ++i) { F[2 * i] = creal(f[i]); F[2 * i + 1] = cimag(f[i]); }
    free(w);
    return rc;
}

/* ----------------------------------------------------------------------- */
/* the quantum medium                                                       */

typedef struct {
    int n;
    cx *h0, *mu;              /* n x n */
    int n_jump;
    cx *jump;                 /* n_jump x n x n */
    double *rate;
    double dephasing;
    cx *relax;                /* n^2 x n^2 or NULL */
    cx *S;                    /* n^2 x n^2 superoperator of L0 + G */
    cx *E0;                   /* exp(S dt/2) */
} medium_t;

static cx *load_cx(const double *p, int count)
{
    if (!p) return NULL;
    cx *o = (cx *)malloc(sizeof(cx) * count);
    for (int i = 0; i < count; ++i) o[i] = p[2 * i] + I * p[2 * i + 1];
    return o;
}

/* out = -(i/hbar)[H0, X] + sum_k r_k (L X L^+ - 1/2 L^+L X - 1/2 X L^+L)
 *       - dephasing * offdiag(X) + R vec(X)              (paper Eq. liouville) */
static void field_free_map(const medium_t *m, const cx *X, cx *out, cx *t1, cx *t2)
{
    int n = m->n;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            cx s = 0;
            for (int k = 0; k < n; ++k)
                s += m->h0[a * n + k] * X[k * n + b] - X[a * n + k] * m->h0[k * n + b];
            out[a * n + b] = -I / ORC_HBAR * s;
        }
    for (int j = 0; j < m->n_jump; ++j) {
        const cx *L = m->jump + (size_t)j * n * n;
        double r = m->rate[j];
        /* t1 = L X, t2 = (L X) L^+ */
        mat_mul(n, L, X, t1);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k) s += t1[a * n + k] * conj(L[b * n + k]);
                t2[a * n + b] = s;
            }
        for (int a = 0; a < n * n; ++a) out[a] += r * t2[a];
        /* t1 = L^+ L */
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k) s += conj(L[k * n + a]) * L[k * n + b];
                t1[a * n + b] = s;
            }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k)
                    s += t1[a * n + k] * X[k * n + b] + X[a * n + k] * t1[k * n + b];
                out[a * n + b] -= 0.5 * r * s;
            }
    }
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            if (a != b) out[a * n + b] -= m->dephasing * X[a * n + b];
    if (m->relax) {
        int n2 = n * n;
        for (int p = 0; p < n2; ++p) {
            cx s = 0;
            for (int q = 0; q < n2; ++q) s += m->relax[p * n2 + q] * X[q];
            out[p] += s;
        }
    }
}

static int medium_init(medium_t *m, int n, const double *h0, const double *mu, int n_jump,
                       const double *jump, const double *rate, double deph,
                       const double *relax, double dt)
{
    memset(m, 0, sizeof(*m));
    m->n = n;
    m->h0 = load_cx(h0, n * n);
    m->mu = load_cx(mu, n * n);
    m->n_jump = n_jump;
    m->jump = n_jump ? load_cx(jump, n_jump * n * n) : NULL;
    m->rate = (double *)malloc(sizeof(double) * (n_jump ? n_jump : 1));
    for (int j = 0; j < n_jump; ++j) m->rate[j] = rate[j];
    m->dephasing = deph;
    m->relax = relax ? load_cx(relax, n * n * n * n) : NULL;
    int n2 = n * n;
    m->S = (cx *)calloc((size_t)n2 * n2, sizeof(cx));
    m->E0 = (cx *)calloc((size_t)n2 * n2, sizeof(cx));
    cx *X = (cx *)calloc(n2, sizeof(cx)), *Y = (cx *)calloc(n2, sizeof(cx));
    cx *t1 = (cx *)calloc(n2, sizeof(cx)), *t2 = (cx *)calloc(n2, sizeof(cx));
    for (int q = 0; q < n2; ++q) {
        memset(X, 0, sizeof(cx) * n2);
        X[q] = 1.0;
        field_free_map(m, X, Y, t1, t2);
        for (int p = 0; p < n2; ++p) m->S[p * n2 + q] = Y[p];
    }
    cx *A = (cx *)malloc(sizeof(cx) * n2 * n2), *w = (cx *)malloc(sizeof(cx) * 5 * n2 * n2);
    for (int i = 0; i < n2 * n2; ++i) A[i] = m->S[i] * (0.5 * dt);
    int rc = expm_work(n2, A, m->E0, w);
    free(A); free(w); free(X); free(Y); free(t1); free(t2);
    return rc;
}

static void medium_free(medium_t *m)
{
    free(m->h0); free(m->mu); free(m->jump); free(m->rate); free(m->relax);
    free(m->S); free(m->E0);
}

/* exported for tests: S (n^2 x n^2, interleaved) and exp(S dt/2) */
int orc_superop(int n, const double *h0, const double *mu, int n_jump, const double *jump,
                const double *rate, double deph, const double *relax, double dt,
                double *S_out, double *E0_out)
{
    medium_t m;
    int rc = medium_init(&m, n, h0, mu, n_jump, jump, rate, deph, relax, dt);
    int n4 = n * n * n * n;
    for (int i = 0; i < n4; ++i) {
        if (S_out) { S_out[2 * i] = creal(m.S[i]); S_out[2 * i + 1] = cimag(m.S[i]); }
        if (E0_out) { E0_out[2 * i] = creal(m.E0[i]); E0_out[2 * i + 1] = cimag(m.E0[i]); }
    }
    medium_free(&m);
    return rc;
}

/* per-thread scratch for one cell update */
typedef struct {
    cx *v, *w, *W, *Wa, *t, *ex;
} cell_ws_t;

static void ws_alloc(cell_ws_t *s, int n)
{
    int n2 = n * n;
    s->v = (cx *)malloc(sizeof(cx) * n2);
    s->w = (cx *)malloc(sizeof(cx) * n2);
    s->W = (cx *)malloc(sizeof(cx) * n2);
    s->Wa = (cx *)malloc(sizeof(cx) * n2);
    s->t = (cx *)malloc(sizeof(cx) * n2);
    s->ex = (cx *)malloc(sizeof(cx) * 5 * n2);
}

static void ws_free(cell_ws_t *s)
{
    free(s->v); free(s->w); free(s->W); free(s->Wa); free(s->t); free(s->ex);
}

/* y = M x for the n^2 x n^2 matrix M on vec(rho) */
static void super_apply(int n2, const cx *M, const cx *x, cx *y)
{
    for (int p = 0; p < n2; ++p) {
        cx s = 0;
        for (int q = 0; q < n2; ++q) s += M[p * n2 + q] * x[q];
        y[p] = s;
    }
}

/* One Strang step of Sec. 4.1 on the density matrix rho (in place), field E
 * frozen at the midpoint.  Returns dP/dt = N_a Re Tr{mu (L0+G)(rho^{n+1/2})}. */
static double cell_step(const medium_t *m, cx *rho, double E, double dt, double Na, cell_ws_t *s)
{
    int n = m->n, n2 = n * n;
    super_apply(n2, m->E0, rho, s->v);                       /* rho'  */
    for (int i = 0; i < n2; ++i) s->Wa[i] = (I * dt * E / ORC_HBAR) * m->mu[i];
    expm_work(n, s->Wa, s->W, s->ex);                         /* W = exp(i mu E dt/hbar) */
    mat_mul(n, s->W, s->v, s->t);
    for (int a = 0; a < n; ++a)                               /* rho'' = W rho' W^+ */
        for (int b = 0; b < n; ++b) {
            cx acc = 0;
            for (int k = 0; k < n; ++k) acc += s->t[a * n + k] * conj(s->W[b * n + k]);
            s->w[a * n + b] = acc;
        }
    super_apply(n2, m->E0, s->w, rho);                        /* rho^{n+1/2} */
    super_apply(n2, m->S, rho, s->v);                         /* (L0 + G)(rho) */
    cx tr = 0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) tr += m->mu[a * n + b] * s->v[b * n + a];
    return Na * creal(tr);
}

/* min eigenvalue of a Hermitian matrix: cyclic Jacobi on the real symmetric
 * embedding [[Re, -Im], [Im, Re]] (every eigenvalue of rho appears twice). */
static double herm_min_eig(int n, const cx *A)
{
    int m = 2 * n;
    double *B = (double *)malloc(sizeof(double) * m * m);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double re = 0.5 * (creal(A[a * n + b]) + creal(A[b * n + a]));
            double im = 0.5 * (cimag(A[a * n + b]) - cimag(A[b * n + a]));
            B[a * m + b] = re;
            B[(a + n) * m + (b + n)] = re;
            B[a * m + (b + n)] = -im;
            B[(a + n) * m + b] = im;
        }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) off += B[p * m + q] * B[p * m + q];
        if (off < 1e-40) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = B[p * m + q];
                if (fabs(apq) < 1e-300) continue;
                double tau = (B[q * m + q] - B[p * m + p]) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < m; ++k) {   /* columns */
                    double bkp = B[k * m + p], bkq = B[k * m + q];
                    B[k * m + p] = c * bkp - sn * bkq;
                    B[k * m + q] = sn * bkp + c * bkq;
                }
                for (int k = 0; k < m; ++k) {   /* rows */
                    double bpk = B[p * m + k], bqk = B[q * m + k];
                    B[p * m + k] = c * bpk - sn * bqk;
                    B[q * m + k] = sn * bpk + c * bqk;
                }
            }
    }
    double mn = B[0];
    for (int i = 1; i < m; ++i) if (B[i * m + i] < mn) mn = B[i * m + i];
    free(B);
    return mn;
}

double orc_min_eig(int n, const double *A)
{
    cx *a = load_cx(A, n * n);
    double r = herm_min_eig(n, a);
    free(a);
    return r;
}

/* diagnostics: [0] max |Tr rho - 1|, [1] max |rho - rho^+|, [2] min eigenvalue,
 * [3] max |Tr rho^2 - Tr rho0^2| */
static void check_rho(int n, const cx *rho, double pur0, double *diag)
{
    cx tr = 0, pur = 0;
    double herm = 0.0;
    for (int a = 0; a < n; ++a) {
        tr += rho[a * n + a];
        for (int b = 0; b < n; ++b) {
            double d = cabs(rho[a * n + b] - conj(rho[b * n + a]));
            if (d > herm) herm = d;
            pur += rho[a * n + b] * rho[b * n + a];
        }
    }
    double e = cabs(tr - 1.0);
    double ev = herm_min_eig(n, rho);
    double pd = fabs(creal(pur) - pur0);
#pragma omp critical(orc_diag)
    {
        if (e > diag[0]) diag[0] = e;
        if (herm > diag[1]) diag[1] = herm;
        if (ev < diag[2]) diag[2] = ev;
        if (pd > diag[3]) diag[3] = pd;
    }
}

static double purity_of(int n, const cx *r)
{
    cx p = 0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) p += r[a * n + b] * r[b * n + a];
    return creal(p);
}

/* ----------------------------------------------------------------------- */
/* coupled Maxwell + Liouville run                                          */

int orc_run(int n, const double *h0, const double *mu, int n_jump, const double *jump,
            const double *rate, double deph, const double *relax, const double *rho0,
            double Na, int64_t nx, int64_t nt, double dx, double dt, int64_t mb, int64_t me,
            double eps_r, double mu_r, double sigma, const double *src, double amp,
            const double *e_init, const double *h_init,
            int64_t snap_every, double *e_snap, double *pop_snap, double *probe,
            double *h_out, double *diag, int nthreads)
{
    if (n < 2 || nx < 3 || nt < 0 || mb < 1 || me < mb || me > nx - 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    medium_t m;
    if (medium_init(&m, n, h0, mu, n_jump, jump, rate, deph, relax, dt)) return -2;
    int n2 = n * n;
    int64_t nmed = me - mb;
    cx *rho = (cx *)malloc(sizeof(cx) * (size_t)(nmed ? nmed : 1) * n2);
    cx *r0 = load_cx(rho0, n2);
    for (int64_t c = 0; c < nmed; ++c) memcpy(rho + c * n2, r0, sizeof(cx) * n2);
    double pur0 = purity_of(n, r0);
    double *E = (double *)calloc(nx, sizeof(double));
    double *H = (double *)calloc(nx, sizeof(double));
    double *P = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double eps = ORC_EPS0 * eps_r, muu = ORC_MU0 * mu_r;
    double cl = 1.0 / sqrt(eps * muu);
    double kmur = (cl * dt - dx) / (cl * dt + dx);
    double sg = sigma * dt / (2.0 * eps);
    double ca = (1.0 - sg) / (1.0 + sg), cb = (dt / eps) / (1.0 + sg);
    double ch = dt / (muu * dx);
    E[0] = amp * src[0];
    /* optional initial fields: E^0 on every cell (including the source cell)
     * and H^{-1/2} on the nx - 1 faces */
    if (e_init) memcpy(E, e_init, sizeof(double) * nx);
    if (h_init) memcpy(H, h_init, sizeof(double) * (nx - 1));
    if (probe) probe[0] = E[nx - 1];
    if (diag) { diag[0] = 0; diag[1] = 0; diag[2] = 1e300; diag[3] = 0; }
    for (int64_t t = 0; t < nt; ++t) {
        for (int64_t i = 0; i + 1 < nx; ++i) H[i] += ch * (E[i + 1] - E[i]);
#pragma omp parallel
        {
            cell_ws_t ws;
            ws_alloc(&ws, n);
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nmed; ++c)
                P[c] = cell_step(&m, rho + c * n2, E[mb + c], dt, Na, &ws);
            ws_free(&ws);
        }
        double e_nm2 = E[nx - 2], e_nm1 = E[nx - 1];
        for (int64_t i = 1; i + 1 < nx; ++i) {
            double dp = (i >= mb && i < me) ? P[i - mb] : 0.0;
            E[i] = ca * E[i] + cb * (-dp + (H[i] - H[i - 1]) / dx);
        }
        E[0] = amp * src[t + 1];
        E[nx - 1] = e_nm2 + kmur * (E[nx - 2] - e_nm1);
        if (probe) probe[t + 1] = E[nx - 1];
        if (snap_every > 0 && (t + 1) % snap_every == 0) {
            int64_t s = (t + 1) / snap_every - 1;
            if (e_snap) memcpy(e_snap + s * nx, E, sizeof(double) * nx);
            for (int64_t c = 0; c < nmed; ++c) {
                const cx *r = rho + c * n2;
                if (pop_snap)
                    for (int a = 0; a < n; ++a)
                        pop_snap[(s * n + a) * nmed + c] = creal(r[a * n + a]);
                if (diag) check_rho(n, r, pur0, diag);
            }
        }
    }
    if (h_out) memcpy(h_out, H, sizeof(double) * (nx - 1));   /* H^{nt-1/2} */
    free(rho); free(r0); free(E); free(H); free(P);
    medium_free(&m);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* two transverse field components: H_I = -mu_z E_z - mu_y E_y              */
/*
 * The paper keeps one field component and the interaction -mu E_z (Sec. 2)
 * and names the fixed interaction form as a limitation (Conclusion).  For a
 * wave along x both transverse components take part: Maxwell's equations
 * split into two independent Yee pairs, (E_z, H_y) as in orc_run and
 * (E_y, G) with G = -H_z, which obeys the same update in the same form,
 *   G_i += dt/(mu dx) (E_y(i+1) - E_y(i)),
 *   E_y(i) = ca E_y(i) + cb (-dP_y/dt + (G_i - G_{i-1})/dx),
 * and the medium couples them through H_I = -mu_z E_z - mu_y E_y.
 * Reading of the Strang step of Sec. 4.1 for two components: the
 * interaction factor is itself split symmetrically, so that each factor
 * keeps a fixed generator (the property the paper's exponential routes
 * rely on):  rho'' = W rho' W^+ with W = W_y W_z W_y,
 * W_y = exp(+i mu_y E_y^n dt / (2 hbar)), W_z = exp(+i mu_z E_z^n dt / hbar)
 * (second order in dt like the step around it; exact when mu_y and mu_z
 * commute).  dP_k/dt = N_a Re Tr{mu_k (L0 + G)(rho^{n+1/2})}, k = z, y.
 * Sources E_z(0) = amp_z src[n], E_y(0) = amp_y src[n]; the Mur boundary of
 * orc_run on both components.  Records as orc_run for each component
 * (ez_snap / ey_snap, probe_z / probe_y) and the populations once; optional
 * initial fields (E^0 on every cell, H^{-1/2} and G^{-1/2} on the nx - 1
 * faces); hy_out and g_out receive H^{nt-1/2} and G^{nt-1/2}.
 */
static double cell_step_pol2(const medium_t *m, const cx *muy, cx *rho, double Ez, double Ey, double dt,
                             double Na, cell_ws_t *s, cx *Wy, cx *Wz, double *dpy)
{
    int n = m->n, n2 = n * n;
    super_apply(n2, m->E0, rho, s->v);                        /* rho' */
    for (int i = 0; i < n2; ++i) s->Wa[i] = (I * (0.5 * dt) * Ey / ORC_HBAR) * muy[i];
    expm_work(n, s->Wa, Wy, s->ex);                            /* W_y */
    for (int i = 0; i < n2; ++i) s->Wa[i] = (I * dt * Ez / ORC_HBAR) * m->mu[i];
    expm_work(n, s->Wa, Wz, s->ex);                            /* W_z */
    mat_mul(n, Wz, Wy, s->t);
    mat_mul(n, Wy, s->t, s->W);                                /* W = W_y W_z W_y */
    mat_mul(n, s->W, s->v, s->t);
    for (int a = 0; a < n; ++a)                                /* rho'' = W rho' W^+ */
        for (int b = 0; b < n; ++b) {
            cx acc = 0;
            for (int k = 0; k < n; ++k) acc += s->t[a * n + k] * conj(s->W[b * n + k]);
            s->w[a * n + b] = acc;
        }
    super_apply(n2, m->E0, s->w, rho);                         /* rho^{n+1/2} */
    super_apply(n2, m->S, rho, s->v);                          /* (L0 + G)(rho) */
    cx trz = 0, tr_y = 0;
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            trz += m->mu[a * n + b] * s->v[b * n + a];
            tr_y += muy[a * n + b] * s->v[b * n + a];
        }
    *dpy = Na * creal(tr_y);
    return Na * creal(trz);
}

/* one Yee pair: H on the faces, then E with the polarisation current */
static void yee_pair_h(int64_t nx, double ch, const double *E, double *H)
{
    for (int64_t i = 0; i + 1 < nx; ++i) H[i] += ch * (E[i + 1] - E[i]);
}

static void yee_pair_e(int64_t nx, int64_t mb, int64_t me, double ca, double cb, double dx, double kmur,
                       double e0_next, const double *P, const double *H, double *E)
{
    double e_nm2 = E[nx - 2], e_nm1 = E[nx - 1];
    for (int64_t i = 1; i + 1 < nx; ++i) {
        double dp = (i >= mb && i < me) ? P[i - mb] : 0.0;
        E[i] = ca * E[i] + cb * (-dp + (H[i] - H[i - 1]) / dx);
    }
    E[0] = e0_next;
    E[nx - 1] = e_nm2 + kmur * (E[nx - 2] - e_nm1);
}

int orc_run_pol2(int n, const double *h0, const double *mu_z, const double *mu_y, int n_jump,
                 const double *jump, const double *rate, double deph, const double *relax,
                 const double *rho0, double Na, int64_t nx, int64_t nt, double dx, double dt, int64_t mb,
                 int64_t me, double eps_r, double mu_r, double sigma, const double *src, double amp_z,
                 double amp_y, const double *ez_init, const double *hy_init, const double *ey_init,
                 const double *g_init, int64_t snap_every, double *ez_snap, double *ey_snap, double *pop_snap,
                 double *probe_z, double *probe_y, double *hy_out, double *g_out, int nthreads)
{
    if (n < 2 || nx < 3 || nt < 0 || mb < 1 || me < mb || me > nx - 1 || !mu_y) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    medium_t m;
    if (medium_init(&m, n, h0, mu_z, n_jump, jump, rate, deph, relax, dt)) return -2;
    int n2 = n * n;
    int64_t nmed = me - mb;
    cx *muy = load_cx(mu_y, n2);
    cx *rho = (cx *)malloc(sizeof(cx) * (size_t)(nmed ? nmed : 1) * n2);
    cx *r0 = load_cx(rho0, n2);
    for (int64_t c = 0; c < nmed; ++c) memcpy(rho + c * n2, r0, sizeof(cx) * n2);
    double *Ez = (double *)calloc(nx, sizeof(double)), *Hy = (double *)calloc(nx, sizeof(double));
    double *Ey = (double *)calloc(nx, sizeof(double)), *G = (double *)calloc(nx, sizeof(double));
    double *Pz = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double *Py = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double eps = ORC_EPS0 * eps_r, muu = ORC_MU0 * mu_r;
    double cl = 1.0 / sqrt(eps * muu);
    double kmur = (cl * dt - dx) / (cl * dt + dx);
    double sg = sigma * dt / (2.0 * eps);
    double ca = (1.0 - sg) / (1.0 + sg), cb = (dt / eps) / (1.0 + sg);
    double ch = dt / (muu * dx);
    Ez[0] = amp_z * src[0];
    Ey[0] = amp_y * src[0];
    if (ez_init) memcpy(Ez, ez_init, sizeof(double) * nx);
    if (ey_init) memcpy(Ey, ey_init, sizeof(double) * nx);
    if (hy_init) memcpy(Hy, hy_init, sizeof(double) * (nx - 1));
    if (g_init) memcpy(G, g_init, sizeof(double) * (nx - 1));
    if (probe_z) probe_z[0] = Ez[nx - 1];
    if (probe_y) probe_y[0] = Ey[nx - 1];
    for (int64_t t = 0; t < nt; ++t) {
        yee_pair_h(nx, ch, Ez, Hy);
        yee_pair_h(nx, ch, Ey, G);
#pragma omp parallel
        {
            cell_ws_t ws;
            ws_alloc(&ws, n);
            cx *Wy = (cx *)malloc(sizeof(cx) * n2), *Wz = (cx *)malloc(sizeof(cx) * n2);
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nmed; ++c)
                Pz[c] = cell_step_pol2(&m, muy, rho + c * n2, Ez[mb + c], Ey[mb + c], dt, Na, &ws, Wy, Wz,
                                       Py + c);
            free(Wy); free(Wz);
            ws_free(&ws);
        }
        yee_pair_e(nx, mb, me, ca, cb, dx, kmur, amp_z * src[t + 1], Pz, Hy, Ez);
        yee_pair_e(nx, mb, me, ca, cb, dx, kmur, amp_y * src[t + 1], Py, G, Ey);
        if (probe_z) probe_z[t + 1] = Ez[nx - 1];
        if (probe_y) probe_y[t + 1] = Ey[nx - 1];
        if (snap_every > 0 && (t + 1) % snap_every == 0) {
            int64_t s = (t + 1) / snap_every - 1;
            if (ez_snap) memcpy(ez_snap + s * nx, Ez, sizeof(double) * nx);
            if (ey_snap) memcpy(ey_snap + s * nx, Ey, sizeof(double) * nx);
            if (pop_snap)
                for (int64_t c = 0; c < nmed; ++c)
                    for (int a = 0; a < n; ++a)
                        pop_snap[(s * n + a) * nmed + c] = creal(rho[c * n2 + a * n + a]);
        }
    }
    if (hy_out) memcpy(hy_out, Hy, sizeof(double) * (nx - 1));
    if (g_out) memcpy(g_out, G, sizeof(double) * (nx - 1));
    free(muy); free(rho); free(r0); free(Ez); free(Hy); free(Ey); free(G); free(Pz); free(Py);
    medium_free(&m);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* two-dimensional TMz run: the same medium step on a 2-D Yee grid           */
/*
 * The paper restricts itself to one spatial dimension (Conclusion); this is
 * the same scheme on the 2-D transverse-magnetic Yee grid (E_z at cell
 * centres (i, j), H_x at (i, j + 1/2), H_y at (i + 1/2, j), all arrays row
 * major with index j * nx + i) with the medium step of every cell unchanged:
 *   H_x += -dt/(mu dy) (E_z(i, j+1) - E_z(i, j))      (every column, j + 1
 *                                                        taken modulo ny)
 *   H_y += dt/(mu dx) (E_z(i+1, j) - E_z(i, j))        (i = 0 .. nx-2)
 *   medium cells: Strang step with E_z(i, j), dP/dt  (as in orc_run)
 *   E_z = ca E_z + cb (-dP/dt + (H_y(i) - H_y(i-1))/dx
 *                             - (H_x(j) - H_x(j-1))/dy)  (i = 1 .. nx-2)
 * Boundaries: periodic in y; a hard source column E_z(0, j) =
 * amp * src[n] * prof[j]; a first-order Mur boundary (normal incidence, the
 * coefficient of orc_run) on column nx-1.  The medium fills the rectangle
 * [mx0, mx1) x [my0, my1) with 1 <= mx0 <= mx1 <= nx-1, 0 <= my0 <= my1 <=
 * ny; its cells are numbered row major within the rectangle.  Records:
 * snapshot s holds E_z^{(s+1)k} (ny x nx) and the populations of
 * rho^{(s+1)k-1/2} ([s][a][cell]); probe[n * ny + j] = E_z^n(nx-1, j).
 * Optional initial fields replace the zero fields (ez_init including the
 * source column); hx_out and hy_out receive H^{nt-1/2}.
 */
int orc_run2d(int n, const double *h0, const double *mu, int n_jump, const double *jump,
              const double *rate, double deph, const double *relax, const double *rho0,
              double Na, int64_t nx, int64_t ny, int64_t nt, double dx, double dy, double dt,
              int64_t mx0, int64_t mx1, int64_t my0, int64_t my1,
              double eps_r, double mu_r, double sigma, const double *src, double amp,
              const double *prof, const double *ez_init, const double *hx_init,
              const double *hy_init, int64_t snap_every, double *e_snap, double *pop_snap,
              double *probe, double *hx_out, double *hy_out, double *diag, int nthreads)
{
    if (n < 2 || nx < 3 || ny < 1 || nt < 0 || mx0 < 1 || mx1 < mx0 || mx1 > nx - 1 ||
        my0 < 0 || my1 < my0 || my1 > ny)
        return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    medium_t m;
    if (medium_init(&m, n, h0, mu, n_jump, jump, rate, deph, relax, dt)) return -2;
    int n2 = n * n;
    int64_t mw = mx1 - mx0, nmed = mw * (my1 - my0), ncell = nx * ny;
    cx *rho = (cx *)malloc(sizeof(cx) * (size_t)(nmed ? nmed : 1) * n2);
    cx *r0 = load_cx(rho0, n2);
    for (int64_t c = 0; c < nmed; ++c) memcpy(rho + c * n2, r0, sizeof(cx) * n2);
    double pur0 = purity_of(n, r0);
    double *E = (double *)calloc(ncell, sizeof(double));
    double *Hx = (double *)calloc(ncell, sizeof(double));
    double *Hy = (double *)calloc(ncell, sizeof(double));
    double *P = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double *eo = (double *)malloc(sizeof(double) * 2 * ny);  /* E(nx-2), E(nx-1) before the step */
    double eps = ORC_EPS0 * eps_r, muu = ORC_MU0 * mu_r;
    double cl = 1.0 / sqrt(eps * muu);
    double kmur = (cl * dt - dx) / (cl * dt + dx);
    double sg = sigma * dt / (2.0 * eps);
    double ca = (1.0 - sg) / (1.0 + sg), cb = (dt / eps) / (1.0 + sg);
    double chx = dt / (muu * dx), chy = dt / (muu * dy);
    for (int64_t j = 0; j < ny; ++j) E[j * nx] = amp * src[0] * prof[j];
    if (ez_init) memcpy(E, ez_init, sizeof(double) * ncell);
    if (hx_init) memcpy(Hx, hx_init, sizeof(double) * ncell);
    if (hy_init) memcpy(Hy, hy_init, sizeof(double) * ncell);
    if (probe)
        for (int64_t j = 0; j < ny; ++j) probe[j] = E[j * nx + nx - 1];
    if (diag) { diag[0] = 0; diag[1] = 0; diag[2] = 1e300; diag[3] = 0; }
    for (int64_t t = 0; t < nt; ++t) {
        for (int64_t j = 0; j < ny; ++j) {
            int64_t jp = (j + 1) % ny;
            for (int64_t i = 0; i < nx; ++i) Hx[j * nx + i] -= chy * (E[jp * nx + i] - E[j * nx + i]);
            for (int64_t i = 0; i + 1 < nx; ++i) Hy[j * nx + i] += chx * (E[j * nx + i + 1] - E[j * nx + i]);
        }
#pragma omp parallel
        {
            cell_ws_t ws;
            ws_alloc(&ws, n);
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nmed; ++c) {
                int64_t i = mx0 + c % mw, j = my0 + c / mw;
                P[c] = cell_step(&m, rho + c * n2, E[j * nx + i], dt, Na, &ws);
            }
            ws_free(&ws);
        }
        for (int64_t j = 0; j < ny; ++j) {
            eo[2 * j] = E[j * nx + nx - 2];
            eo[2 * j + 1] = E[j * nx + nx - 1];
        }
        for (int64_t j = 0; j < ny; ++j) {
            int64_t jm = (j + ny - 1) % ny;
            for (int64_t i = 1; i + 1 < nx; ++i) {
                double dp = 0.0;
                if (i >= mx0 && i < mx1 && j >= my0 && j < my1) dp = P[(j - my0) * mw + (i - mx0)];
                double curl = (Hy[j * nx + i] - Hy[j * nx + i - 1]) / dx -
                              (Hx[j * nx + i] - Hx[jm * nx + i]) / dy;
                E[j * nx + i] = ca * E[j * nx + i] + cb * (-dp + curl);
            }
        }
        for (int64_t j = 0; j < ny; ++j) {
            E[j * nx] = amp * src[t + 1] * prof[j];
            E[j * nx + nx - 1] = eo[2 * j] + kmur * (E[j * nx + nx - 2] - eo[2 * j + 1]);
        }
        if (probe)
            for (int64_t j = 0; j < ny; ++j) probe[(t + 1) * ny + j] = E[j * nx + nx - 1];
        if (snap_every > 0 && (t + 1) % snap_every == 0) {
            int64_t s = (t + 1) / snap_every - 1;
            if (e_snap) memcpy(e_snap + s * ncell, E, sizeof(double) * ncell);
            for (int64_t c = 0; c < nmed; ++c) {
                const cx *r = rho + c * n2;
                if (pop_snap)
                    for (int a = 0; a < n; ++a)
                        pop_snap[(s * n + a) * nmed + c] = creal(r[a * n + a]);
                if (diag) check_rho(n, r, pur0, diag);
            }
        }
    }
    if (hx_out) memcpy(hx_out, Hx, sizeof(double) * ncell);
    if (hy_out) memcpy(hy_out, Hy, sizeof(double) * ncell);
    free(rho); free(r0); free(E); free(Hx); free(Hy); free(P); free(eo);
    medium_free(&m);
    return 0;
}

/* Prescribed-field mode (no FDTD): cell c sees E = efield[t * ncell + c] at
 * step t.  Records the populations of rho^{t+1/2} and dP/dt per step, and the
 * final density matrices. */
int orc_bloch(int n, const double *h0, const double *mu, int n_jump, const double *jump,
              const double *rate, double deph, const double *relax, const double *rho0,
              double Na, int64_t ncell, int64_t nt, double dt, const double *efield,
              double *pop, double *dp, double *rho_final, double *diag, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    medium_t m;
    if (medium_init(&m, n, h0, mu, n_jump, jump, rate, deph, relax, dt)) return -2;
    int n2 = n * n;
    cx *r0 = load_cx(rho0, n2);
    double pur0 = purity_of(n, r0);
    if (diag) { diag[0] = 0; diag[1] = 0; diag[2] = 1e300; diag[3] = 0; }
#pragma omp parallel
    {
        cell_ws_t ws;
        ws_alloc(&ws, n);
        cx *rho = (cx *)malloc(sizeof(cx) * n2);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < ncell; ++c) {
            memcpy(rho, r0, sizeof(cx) * n2);
            for (int64_t t = 0; t < nt; ++t) {
                double p = cell_step(&m, rho, efield[t * ncell + c], dt, Na, &ws);
                if (dp) dp[t * ncell + c] = p;
                if (pop)
                    for (int a = 0; a < n; ++a) pop[(t * n + a) * ncell + c] = creal(rho[a * n + a]);
            }
            if (diag) check_rho(n, rho, pur0, diag);
            if (rho_final)
                for (int i = 0; i < n2; ++i) {
                    rho_final[(c * n2 + i) * 2] = creal(rho[i]);
                    rho_final[(c * n2 + i) * 2 + 1] = cimag(rho[i]);
                }
        }
        free(rho);
        ws_free(&ws);
    }
    free(r0);
    medium_free(&m);
    return 0;
}

/* ----------------------------------------------------------------------- */
/* FP64 adjoint of orc_run (reverse mode through the steps above)           */
/*
 * For J(probe) with g[n] = dJ/dprobe[n], the gradients with respect to the
 * physical inputs.  Reverse mode over the exact discrete map of orc_run:
 * the forward pass stores rho before every cell step and the field the cell
 * saw; the reverse pass walks the steps backwards.  Conventions: for a
 * complex quantity z the adjoint is Z = dJ/dRe z + i dJ/dIm z, so a linear
 * map y = A x gives X += A^H Y, and <X, Y> = Re tr(X^H Y).  The derivative
 * of a matrix exponential enters through the adjoint of its Frechet
 * derivative, L(A, .)^* = L(A^H, .), evaluated by the block identity
 * exp([[B, C], [0, B]]) = [[e^B, L(B, C)], [0, e^B]] (Higham, Functions of
 * Matrices, 2008) with the same generic Pade exponential.  The field-free
 * generator is linear in H0, the jump rates and the dephasing rate, so their
 * gradients are inner products of the accumulated dJ/dS with the
 * superoperators of the derivative maps, built by applying each map to the
 * basis matrices.  Everything is recomputed the slow, obvious way.
 */

/* out = L(A^H, G) for n x n complex A, G.  L is linear in G, so G enters the
 * block scaled to the 1-norm of A (otherwise a large G would set the
 * scaling of the block exponential and its many squarings) and the result is
 * scaled back. */
static int frechet_adj(int n, const cx *A, const cx *G, cx *out)
{
    int m = 2 * n;
    double an = 0.0, gn = 0.0;
    for (int j = 0; j < n; ++j) {
        double sa = 0.0, sg = 0.0;
        for (int i = 0; i < n; ++i) { sa += cabs(A[i * n + j]); sg += cabs(G[i * n + j]); }
        if (sa > an) an = sa;
        if (sg > gn) gn = sg;
    }
    if (gn == 0.0) {
        for (int i = 0; i < n * n; ++i) out[i] = 0.0;
        return 0;
    }
    /* G enters as (G / |G|_1) * s and the result is scaled back by
     * |G|_1 / s, with s = max(|A|_1, 1/4): dividing first keeps a G near
     * the bottom of the double range (an adjoint that has barely reached a
     * cell) from overflowing the factor s / |G|_1, and the floor on s keeps
     * G out of the subnormal range when A is tiny (a cell the field has
     * barely reached, E ~ 1e-300), where it would lose its significant
     * digits; the block's norm stays below 1/2 + |A|_1 either way */
    double an1 = an > 0.25 ? an : 0.25;
    cx *B = (cx *)calloc((size_t)m * m, sizeof(cx));
    cx *F = (cx *)malloc(sizeof(cx) * m * m);
    cx *w = (cx *)malloc(sizeof(cx) * 5 * m * m);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cx ah = conj(A[j * n + i]);
            B[i * m + j] = ah;
            B[(n + i) * m + n + j] = ah;
            B[i * m + n + j] = (G[i * n + j] / gn) * an1;
        }
    int rc = expm_work(m, B, F, w);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) out[i * n + j] = (F[i * m + n + j] / an1) * gn;
    free(B); free(F); free(w);
    return rc;
}

/* the derivative maps of the field-free generator */
enum { DM_COMM = 0, DM_JUMP = 1, DM_DEPH = 2 };

/* Y = (d generator / d theta)(X) for: DM_COMM -(i/hbar)[K, X];
 * DM_JUMP L X L^+ - 1/2 {L^+ L, X}; DM_DEPH -offdiag(X). */
static void deriv_map(int kind, int n, const cx *K, const cx *X, cx *Y, cx *t1, cx *t2)
{
    if (kind == DM_COMM) {
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k) s += K[a * n + k] * X[k * n + b] - X[a * n + k] * K[k * n + b];
                Y[a * n + b] = -I / ORC_HBAR * s;
            }
    } else if (kind == DM_JUMP) {
        mat_mul(n, K, X, t1);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k) s += t1[a * n + k] * conj(K[b * n + k]);
                Y[a * n + b] = s;
            }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k) s += conj(K[k * n + a]) * K[k * n + b];
                t2[a * n + b] = s;
            }
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                cx s = 0;
                for (int k = 0; k < n; ++k) s += t2[a * n + k] * X[k * n + b] + X[a * n + k] * t2[k * n + b];
                Y[a * n + b] -= 0.5 * s;
            }
    } else {
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) Y[a * n + b] = (a == b) ? 0.0 : -X[a * n + b];
    }
}

/* <GS, dS> where dS is the superoperator of the derivative map */
static double super_inner(int kind, int n, const cx *K, const cx *GS)
{
    int n2 = n * n;
    cx *X = (cx *)calloc(n2, sizeof(cx)), *Y = (cx *)malloc(sizeof(cx) * n2);
    cx *t1 = (cx *)malloc(sizeof(cx) * n2), *t2 = (cx *)malloc(sizeof(cx) * n2);
    double acc = 0.0;
    for (int q = 0; q < n2; ++q) {
        memset(X, 0, sizeof(cx) * n2);
        X[q] = 1.0;
        deriv_map(kind, n, K, X, Y, t1, t2);
        for (int p = 0; p < n2; ++p) acc += creal(conj(GS[p * n2 + q]) * Y[p]);
    }
    free(X); free(Y); free(t1); free(t2);
    return acc;
}

/* gradient of a Hermitian matrix input from the unconstrained adjoint G:
 * off-diagonal a < b: G_ab + conj(G_ba) (real and imaginary perturbation of
 * the pair), conjugate below the diagonal; diagonal: Re G_aa */
static void herm_grad(int n, const cx *G, double *out)
{
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            cx v = (a == b) ? creal(G[a * n + a]) : (a < b ? G[a * n + b] + conj(G[b * n + a])
                                                           : conj(G[b * n + a] + conj(G[a * n + b])));
            out[2 * (a * n + b)] = creal(v);
            out[2 * (a * n + b) + 1] = cimag(v);
        }
}

int orc_grad(int n, const double *h0, const double *mu, int n_jump, const double *jump,
             const double *rate, double deph, const double *relax, const double *rho0,
             double Na, int64_t nx, int64_t nt, double dx, double dt, int64_t mb, int64_t me,
             double eps_r, double mu_r, double sigma, const double *src, double amp,
             const double *gprobe, double *g_h0, double *g_mu, double *g_rate, double *g_deph,
             double *g_amp, double *g_Na, int nthreads)
{
    if (n < 2 || nx < 3 || nt < 0 || mb < 1 || me < mb || me > nx - 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    medium_t m;
    if (medium_init(&m, n, h0, mu, n_jump, jump, rate, deph, relax, dt)) return -2;
    int n2 = n * n;
    int64_t nmed = me - mb;
    /* the trajectory: rho before every step, the field each cell saw */
    size_t need = (size_t)nt * (size_t)(nmed ? nmed : 1) * n2;
    if (need > ((size_t)1 << 27)) { medium_free(&m); return -3; }  /* 2 GiB of history */
    cx *hist = (cx *)malloc(sizeof(cx) * (need ? need : 1));
    double *ehist = (double *)malloc(sizeof(double) * (size_t)(nt ? nt : 1) * (nmed ? nmed : 1));
    cx *rho = (cx *)malloc(sizeof(cx) * (size_t)(nmed ? nmed : 1) * n2);
    cx *r0 = load_cx(rho0, n2);
    for (int64_t c = 0; c < nmed; ++c) memcpy(rho + c * n2, r0, sizeof(cx) * n2);
    double *E = (double *)calloc(nx, sizeof(double));
    double *H = (double *)calloc(nx, sizeof(double));
    double *P = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double eps = ORC_EPS0 * eps_r, muu = ORC_MU0 * mu_r;
    double cl = 1.0 / sqrt(eps * muu);
    double kmur = (cl * dt - dx) / (cl * dt + dx);
    double sg = sigma * dt / (2.0 * eps);
    double ca = (1.0 - sg) / (1.0 + sg), cb = (dt / eps) / (1.0 + sg);
    double ch = dt / (muu * dx);
    E[0] = amp * src[0];
    for (int64_t t = 0; t < nt; ++t) {
        for (int64_t i = 0; i + 1 < nx; ++i) H[i] += ch * (E[i + 1] - E[i]);
        memcpy(hist + (size_t)t * nmed * n2, rho, sizeof(cx) * nmed * n2);
        for (int64_t c = 0; c < nmed; ++c) ehist[t * nmed + c] = E[mb + c];
#pragma omp parallel
        {
            cell_ws_t ws;
            ws_alloc(&ws, n);
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nmed; ++c)
                P[c] = cell_step(&m, rho + c * n2, E[mb + c], dt, Na, &ws);
            ws_free(&ws);
        }
        double e_nm2 = E[nx - 2], e_nm1 = E[nx - 1];
        for (int64_t i = 1; i + 1 < nx; ++i) {
            double dp = (i >= mb && i < me) ? P[i - mb] : 0.0;
            E[i] = ca * E[i] + cb * (-dp + (H[i] - H[i - 1]) / dx);
        }
        E[0] = amp * src[t + 1];
        E[nx - 1] = e_nm2 + kmur * (E[nx - 2] - e_nm1);
    }

    /* reverse sweep */
    double *lE = (double *)calloc(nx, sizeof(double)), *lEo = (double *)calloc(nx, sizeof(double));
    double *lH = (double *)calloc(nx, sizeof(double));
    double *lP = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double *lEc = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    cx *lrho = (cx *)calloc((size_t)(nmed ? nmed : 1) * n2, sizeof(cx));
    cx *mu_cx = m.mu;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    /* per-thread accumulators: dJ/dE0 (n2 x n2), dJ/dS (n2 x n2), dJ/dmu (n x n), dJ/dNa */
    cx *accE0 = (cx *)calloc((size_t)nth * n2 * n2, sizeof(cx));
    cx *accS = (cx *)calloc((size_t)nth * n2 * n2, sizeof(cx));
    cx *accMu = (cx *)calloc((size_t)nth * n2, sizeof(cx));
    double *accNa = (double *)calloc(nth, sizeof(double));
    double gamp = 0.0;
    double alpha = dt / ORC_HBAR;
    for (int64_t t = nt - 1; t >= 0; --t) {
        /* lE holds dJ/dE after step t; the probe of step t+1 */
        lE[nx - 1] += gprobe[t + 1];
        memset(lEo, 0, sizeof(double) * nx);
        /* Mur boundary: E[nx-1] = E_old[nx-2] + kmur (E_new[nx-2] - E_old[nx-1]) */
        double bnd = lE[nx - 1];
        lE[nx - 2] += kmur * bnd;
        lEo[nx - 2] += bnd;
        lEo[nx - 1] -= kmur * bnd;
        /* source */
        gamp += lE[0] * src[t + 1];
        /* interior E update (H after this step's H update) */
        for (int64_t i = 1; i + 1 < nx; ++i) {
            double l = lE[i];
            lEo[i] += ca * l;
            lH[i] += cb / dx * l;
            lH[i - 1] -= cb / dx * l;
            if (i >= mb && i < me) lP[i - mb] = -cb * l;
        }
        /* cell steps */
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            cx *aE0 = accE0 + (size_t)tid * n2 * n2, *aS = accS + (size_t)tid * n2 * n2;
            cx *aMu = accMu + (size_t)tid * n2;
            cx *v = (cx *)malloc(sizeof(cx) * n2), *w = (cx *)malloc(sizeof(cx) * n2);
            cx *rn = (cx *)malloc(sizeof(cx) * n2), *y = (cx *)malloc(sizeof(cx) * n2);
            cx *W = (cx *)malloc(sizeof(cx) * n2), *X = (cx *)malloc(sizeof(cx) * n2);
            cx *t1 = (cx *)malloc(sizeof(cx) * n2), *t2 = (cx *)malloc(sizeof(cx) * n2);
            cx *lw = (cx *)malloc(sizeof(cx) * n2), *lv = (cx *)malloc(sizeof(cx) * n2);
            cx *GW = (cx *)malloc(sizeof(cx) * n2), *GX = (cx *)malloc(sizeof(cx) * n2);
            cx *ex = (cx *)malloc(sizeof(cx) * 5 * n2);
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nmed; ++c) {
                const cx *ro = hist + ((size_t)t * nmed + c) * n2;
                double Ec = ehist[t * nmed + c];
                cx *L = lrho + (size_t)c * n2;  /* dJ/drho after this step */
                /* recompute the step */
                super_apply(n2, m.E0, ro, v);
                for (int i = 0; i < n2; ++i) X[i] = (I * alpha * Ec) * mu_cx[i];
                expm_work(n, X, W, ex);
                mat_mul(n, W, v, t1);
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        cx s = 0;
                        for (int k = 0; k < n; ++k) s += t1[a * n + k] * conj(W[b * n + k]);
                        w[a * n + b] = s;
                    }
                super_apply(n2, m.E0, w, rn);
                super_apply(n2, m.S, rn, y);
                /* P = Na Re <vec mu, S rho_new> */
                double lp = lP[c];
                double ptr = 0.0;
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) ptr += creal(mu_cx[a * n + b] * y[b * n + a]);
                accNa[tid] += lp * ptr;
                /* dJ/drho_new += lp Na S^H vec(mu); dJ/dS += lp Na vec(mu) rho_new^H */
                for (int q = 0; q < n2; ++q) {
                    cx s = 0;
                    for (int p = 0; p < n2; ++p) s += conj(m.S[p * n2 + q]) * mu_cx[p];
                    L[q] += lp * Na * s;
                }
                for (int p = 0; p < n2; ++p)
                    for (int q = 0; q < n2; ++q) aS[p * n2 + q] += lp * Na * mu_cx[p] * conj(rn[q]);
                /* dJ/dmu from P: conj(y_ba) */
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) aMu[a * n + b] += lp * Na * conj(y[b * n + a]);
                /* rho_new = E0 w */
                for (int q = 0; q < n2; ++q) {
                    cx s = 0;
                    for (int p = 0; p < n2; ++p) s += conj(m.E0[p * n2 + q]) * L[p];
                    lw[q] = s;
                }
                for (int p = 0; p < n2; ++p)
                    for (int q = 0; q < n2; ++q) aE0[p * n2 + q] += L[p] * conj(w[q]);
                /* w = W v W^+ : lv = W^+ lw W; GW = lw W v^H + lw^H W v */
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        cx s = 0;
                        for (int k = 0; k < n; ++k) s += conj(W[k * n + a]) * lw[k * n + b];
                        t1[a * n + b] = s;
                    }
                mat_mul(n, t1, W, lv);
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        cx s = 0;
                        for (int k = 0; k < n; ++k) s += W[a * n + k] * conj(v[b * n + k]);
                        t1[a * n + b] = s;  /* W v^H */
                    }
                mat_mul(n, lw, t1, GW);
                mat_mul(n, W, v, t1);       /* W v */
                for (int a = 0; a < n; ++a)
                    for (int b = 0; b < n; ++b) {
                        cx s = 0;
                        for (int k = 0; k < n; ++k) s += conj(lw[k * n + a]) * t1[k * n + b];
                        GW[a * n + b] += s;
                    }
                /* W = exp(X), X = i alpha E mu */
                frechet_adj(n, X, GW, GX);
                double le = 0.0;
                for (int i = 0; i < n2; ++i) {
                    le += creal(conj(GX[i]) * (I * alpha) * mu_cx[i]);
                    aMu[i] += GX[i] * conj(I * alpha * Ec);
                }
                lEc[c] = le;
                /* v = E0 rho_old */
                for (int q = 0; q < n2; ++q) {
                    cx s = 0;
                    for (int p = 0; p < n2; ++p) s += conj(m.E0[p * n2 + q]) * lv[p];
                    t2[q] = s;
                }
                for (int p = 0; p < n2; ++p)
                    for (int q = 0; q < n2; ++q) aE0[p * n2 + q] += lv[p] * conj(ro[q]);
                memcpy(L, t2, sizeof(cx) * n2);
            }
            free(v); free(w); free(rn); free(y); free(W); free(X); free(t1); free(t2);
            free(lw); free(lv); free(GW); free(GX); free(ex);
        }
        for (int64_t c = 0; c < nmed; ++c) lEo[mb + c] += lEc[c];
        /* H update: H_i += ch (E_old[i+1] - E_old[i]) */
        for (int64_t i = 0; i + 1 < nx; ++i) {
            lEo[i + 1] += ch * lH[i];
            lEo[i] -= ch * lH[i];
        }
        memcpy(lE, lEo, sizeof(double) * nx);
    }
    /* initial field: E[0] = amp src[0] */
    gamp += lE[0] * src[0];

    /* reduce the per-thread accumulators */
    for (int th = 1; th < nth; ++th) {
        for (int i = 0; i < n2 * n2; ++i) {
            accE0[i] += accE0[(size_t)th * n2 * n2 + i];
            accS[i] += accS[(size_t)th * n2 * n2 + i];
        }
        for (int i = 0; i < n2; ++i) accMu[i] += accMu[(size_t)th * n2 + i];
        accNa[0] += accNa[th];
    }
    /* E0 = exp(S dt/2): dJ/dS += dt/2 L((S dt/2)^H, dJ/dE0) */
    cx *A = (cx *)malloc(sizeof(cx) * n2 * n2), *GA = (cx *)malloc(sizeof(cx) * n2 * n2);
    for (int i = 0; i < n2 * n2; ++i) A[i] = m.S[i] * (0.5 * dt);
    int rc = frechet_adj(n2, A, accE0, GA);
    for (int i = 0; i < n2 * n2; ++i) accS[i] += 0.5 * dt * GA[i];
    /* parameters of the field-free generator */
    cx *K = (cx *)calloc(n2, sizeof(cx));
    cx *GH = (cx *)calloc(n2, sizeof(cx));
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            if (a == b) {
                memset(K, 0, sizeof(cx) * n2);
                K[a * n + a] = 1.0;
                GH[a * n + a] = super_inner(DM_COMM, n, K, accS);
            } else {
                memset(K, 0, sizeof(cx) * n2);
                K[a * n + b] = 1.0; K[b * n + a] = 1.0;
                double gr = super_inner(DM_COMM, n, K, accS);
                memset(K, 0, sizeof(cx) * n2);
                K[a * n + b] = I; K[b * n + a] = -I;
                double gi = super_inner(DM_COMM, n, K, accS);
                GH[a * n + b] = gr + I * gi;
                GH[b * n + a] = gr - I * gi;
            }
        }
    if (g_h0)
        for (int i = 0; i < n2; ++i) { g_h0[2 * i] = creal(GH[i]); g_h0[2 * i + 1] = cimag(GH[i]); }
    if (g_rate)
        for (int j = 0; j < n_jump; ++j) g_rate[j] = super_inner(DM_JUMP, n, m.jump + (size_t)j * n2, accS);
    if (g_deph) *g_deph = super_inner(DM_DEPH, n, NULL, accS);
    if (g_mu) herm_grad(n, accMu, g_mu);
    if (g_amp) *g_amp = gamp;
    if (g_Na) *g_Na = accNa[0];
    free(A); free(GA); free(K); free(GH);
    free(accE0); free(accS); free(accMu); free(accNa);
    free(lE); free(lEo); free(lH); free(lP); free(lEc); free(lrho);
    free(hist); free(ehist); free(rho); free(r0); free(E); free(H); free(P);
    medium_free(&m);
    return rc ? -4 : 0;
}

/* ----------------------------------------------------------------------- */
/* pseudo-spectral time-domain (PSTD) field solver                          */
/*
 * The paper notes that its Liouville treatment combines with a PSTD field
 * solver as well as with FDTD (Introduction; Sec. 4).  Reading taken here:
 * the staggered leapfrog of the Yee scheme in time (E at integer steps, H at
 * half steps), the spatial derivatives spectral on a periodic grid of nx
 * cells, the half-cell staggering of H realised by the shift factor
 * exp(+-i kappa dx/2) of every Fourier mode, the Nyquist mode of an even nx
 * dropped.  A run is an initial-value problem: E at step 0 and H at step
 * -1/2 are given (e_init, h_init), the grid is periodic with no absorbing
 * boundary, the probe is cell nx - 1, and the medium coupling is exactly as
 * in orc_run.  A hard source at cell 0 (src != NULL) is optional: a sample
 * forced on a spectral grid radiates both ways and leaves a jump in H whose
 * Gibbs error spoils the method's convergence, so it serves comparisons
 * only.  The derivatives are direct DFT sums (O(nx^2) per derivative): the
 * definition, no FFT.
 */

/* out[j] = d/dx of the periodic band-limited interpolant of f (samples at
 * x_i = i dx), evaluated at x_j + shift (shift = +dx/2 or -dx/2). */
static void spectral_derivative(int64_t nx, double dx, const double *f, double shift, double *out,
                                double *re, double *im)
{
    const double tw = 2.0 * 3.14159265358979323846 / (double)nx;
    int64_t kmax = (nx - 1) / 2;  /* modes -kmax..kmax; the Nyquist mode is dropped */
    for (int64_t k = 0; k <= kmax; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t i = 0; i < nx; ++i) {
            double a = tw * (double)((k * i) % nx);
            sr += f[i] * cos(a);
            si -= f[i] * sin(a);
        }
        re[k] = sr;
        im[k] = si;
    }
    for (int64_t j = 0; j < nx; ++j) {
        double acc = 0.0;
        for (int64_t k = 1; k <= kmax; ++k) {
            /* the pair (k, -k) of a real signal: 2 Re{ i kappa e^{i kappa (x_j + shift)} F_k } / nx */
            double kappa = tw * (double)k / dx;
            double ph = tw * (double)((k * j) % nx) + kappa * shift;
            double c = cos(ph), s = sin(ph);
            /* i kappa (re + i im)(c + i s) -> real part: -kappa (re s + im c) */
            acc += -kappa * (re[k] * s + im[k] * c);
        }
        out[j] = 2.0 * acc / (double)nx;
    }
}

int orc_pstd_run(int n, const double *h0, const double *mu, int n_jump, const double *jump,
                 const double *rate, double deph, const double *relax, const double *rho0,
                 double Na, int64_t nx, int64_t nt, double dx, double dt, int64_t mb, int64_t me,
                 double eps_r, double mu_r, double sigma, const double *src, double amp,
                 const double *e_init, const double *h_init,
                 int64_t snap_every, double *e_snap, double *pop_snap, double *probe, double *h_final,
                 int nthreads)
{
    if (n < 2 || nx < 3 || nt < 0 || mb < 1 || me < mb || me > nx - 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    medium_t m;
    if (medium_init(&m, n, h0, mu, n_jump, jump, rate, deph, relax, dt)) return -2;
    int n2 = n * n;
    int64_t nmed = me - mb;
    cx *rho = (cx *)malloc(sizeof(cx) * (size_t)(nmed ? nmed : 1) * n2);
    cx *r0 = load_cx(rho0, n2);
    for (int64_t c = 0; c < nmed; ++c) memcpy(rho + c * n2, r0, sizeof(cx) * n2);
    double *E = (double *)calloc(nx, sizeof(double));
    double *H = (double *)calloc(nx, sizeof(double));
    double *D = (double *)calloc(nx, sizeof(double));
    double *re = (double *)calloc(nx, sizeof(double)), *im = (double *)calloc(nx, sizeof(double));
    double *P = (double *)calloc(nmed ? nmed : 1, sizeof(double));
    double eps = ORC_EPS0 * eps_r, muu = ORC_MU0 * mu_r;
    double sg = sigma * dt / (2.0 * eps);
    double ca = (1.0 - sg) / (1.0 + sg), cb = (dt / eps) / (1.0 + sg);
    double chp = dt / muu;
    if (e_init) memcpy(E, e_init, sizeof(double) * nx);
    if (h_init) memcpy(H, h_init, sizeof(double) * nx);
    if (!e_init && src) E[0] = amp * src[0];
    if (probe) probe[0] = E[nx - 1];
    for (int64_t t = 0; t < nt; ++t) {
        /* H at x_i + dx/2 */
        spectral_derivative(nx, dx, E, 0.5 * dx, D, re, im);
        for (int64_t i = 0; i < nx; ++i) H[i] += chp * D[i];
#pragma omp parallel
        {
            cell_ws_t ws;
            ws_alloc(&ws, n);
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nmed; ++c)
                P[c] = cell_step(&m, rho + c * n2, E[mb + c], dt, Na, &ws);
            ws_free(&ws);
        }
        /* dH/dx at x_i: the samples of H sit half a cell to the right */
        spectral_derivative(nx, dx, H, -0.5 * dx, D, re, im);
        for (int64_t i = 0; i < nx; ++i) {
            double dp = (i >= mb && i < me) ? P[i - mb] : 0.0;
            E[i] = ca * E[i] + cb * (-dp + D[i]);
        }
        if (src) E[0] = amp * src[t + 1];
        if (probe) probe[t + 1] = E[nx - 1];
        if (snap_every > 0 && (t + 1) % snap_every == 0) {
            int64_t s = (t + 1) / snap_every - 1;
            if (e_snap) memcpy(e_snap + s * nx, E, sizeof(double) * nx);
            if (pop_snap)
                for (int64_t c = 0; c < nmed; ++c)
                    for (int a = 0; a < n; ++a)
                        pop_snap[(s * n + a) * nmed + c] = creal(rho[c * n2 + a * n + a]);
        }
    }
    if (h_final) memcpy(h_final, H, sizeof(double) * nx);
    free(rho); free(r0); free(E); free(H); free(D); free(re); free(im); free(P);
    medium_free(&m);
    return 0;
}

/* exported for the pins: the spectral derivative itself */
void orc_spectral_derivative(int64_t nx, double dx, const double *f, double shift, double *out)
{
    double *re = (double *)calloc(nx, sizeof(double)), *im = (double *)calloc(nx, sizeof(double));
    spectral_derivative(nx, dx, f, shift, out, re, im);
    free(re); free(im);
}
