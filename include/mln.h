/*
 * mln.h -- C ABI of the MI355X (gfx950) Maxwell-Liouville-von Neumann solver.
 *
 * Method: Riesch & Jirauschek, "Numerical Method for the Maxwell-Liouville-von
 * Neumann Equations using Efficient Matrix Exponential Computations",
 * arXiv:1710.09799.  The density matrix of every medium cell is carried as a
 * real Bloch vector d in R^(N^2-1) in the SU(N) adjoint representation
 * (Sec. 3, Eq. comp_rho), advanced by the symmetric Strang splitting of
 * Sec. 4.1 (half step exp(M dt/2), full step exp(U E^n dt), half step
 * exp(M dt/2)), and coupled to a 1-D Yee FDTD update of E_z / H_y
 * (Sec. 2, Eq. maxwell; Fig. 1) through the polarisation derivative
 * dP/dt = 1/2 N_a v^T (M d + d_eq) (Sec. 3, last equation).
 *
 * Conventions shared by every call:
 *   * Every entry point returns int: 0 (MLN_OK) or a negative MLN_E* code.
 *     No C++ exception crosses this boundary.  mln_last_error() returns a
 *     human-readable message for the last failure on the calling thread.
 *   * Complex N x N matrices are row-major arrays of 2*N*N doubles with real
 *     and imaginary parts interleaved.
 *   * SI units: J, C m, s, m, V/m, 1/m^3.
 *   * Inputs are copied during the call; the caller may free them afterwards.
 *   * Output buffers are owned by the caller.  They are device pointers when
 *     mln_record.out_on_device = 1 (e.g. the data_ptr() of a torch tensor on
 *     the GPU), host pointers otherwise.
 *   * All device work is enqueued on the HIP stream given in mln_options
 *     (NULL = the default stream).  A handle must not be used from two host
 *     threads at once.
 */
#ifndef MLN_H
#define MLN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define MLN_OK 0
#define MLN_EINVAL (-1)              /* null pointer, size or range error          */
#define MLN_ENOTHERMITIAN (-2)       /* H0 or mu not Hermitian (1e-12 relative)    */
#define MLN_ENOTTRACEPRESERVING (-3) /* Tr G(X) != 0 for some X: the adjoint
                                        representation needs trace preservation
                                        (Sec. 3, Eq. comp_rho)                     */
#define MLN_ECOURANT (-4)            /* c dt / dx > 1: explicit Yee update unstable */
#define MLN_EBADRHO (-5)             /* rho0 not Hermitian, not trace 1 or not PSD  */
#define MLN_ENOMEM (-6)              /* device or host allocation failed            */
#define MLN_EHIP (-7)                /* a HIP runtime call failed                   */
#define MLN_ENOTSUPPORTED (-8)       /* level count / precision / route not built   */
#define MLN_ENONFINITE (-9)          /* NaN or Inf seen in the recorded output      */
#define MLN_ESTATE (-10)             /* call not valid in the handle's state        */
#define MLN_ENUMERIC (-11)           /* a one-time factorisation failed to converge */

/* mln_options.ckpt_every: keep the whole forward tape instead of checkpoints */
#define MLN_TAPE_ALL (-1)

/* ---- enumerations ------------------------------------------------------ */
typedef enum {
  MLN_FP64 = 0,           /* state, factors and arithmetic in double precision          */
  MLN_FP32 = 1,           /* plain single precision; the rotation route carries the
                             deviation from the rest state (about 2e-6 on 1e4 steps,
                             1.5e-5 in the populations after 1e5 steps), the other
                             routes carry d itself (about 1e-4)                        */
  MLN_FP32_COMP = 2,      /* single precision with a compensated (two-float) Bloch-vector
                             state and two-float factors; E and H in plain FP32, whose
                             rounding accumulates along long propagation paths (2.6e-5
                             in the six-level probe after 2e5 steps, 4.9e-5 in the
                             30000-cell problems of the 64-problem sweep): past ~1e5
                             steps or ~2e4 cells use MLN_FP32_COMP_FIELDS for 1e-5   */
  MLN_FP32_BF16SPLIT = 3, /* compensated FP32 state and fields; the shared-factor
                             transform runs on MFMA with three-part BF16 splits of both
                             operands and six products (~2^-24 relative), FP32
                             accumulation; N = 4, 6                                     */
  MLN_FP32_BF16X3 = 4,    /* as MLN_FP32_BF16SPLIT with two-part splits and three
                             products (~2^-16 relative).  Outside the split-BF16
                             tolerance of 1e-4 on long runs: the six-level workload
                             (50000 cells, 2e5 steps) ends 4.9e-4 away from the FP64
                             path in the probe field (1e-5 after 2e4 steps; bound
                             stated for such runs: 1e-3); use MLN_FP32_BF16SPLIT
                             where 1e-4 must hold past ~5e4 steps                     */
  MLN_FP32_COMP_FIELDS = 5, /* as MLN_FP32_COMP, and E, H and the source samples are
                             two-float pairs as well (for runs of 1e5 steps and more,
                             where FP32 rounding of the fields accumulates); workgroup
                             and four-lanes-per-cell kernels                            */
  MLN_FP32_FIELDS = 6     /* plain single-precision state (the deviation from the rest
                             state, as MLN_FP32) with E, H and the source samples as
                             two-float pairs: the fields' rounding, which dominates
                             plain FP32's field error on long propagation paths, is
                             removed at a fraction of the compensated state's cost.
                             The state's rounding remains: worst deviation from FP64
                             1.4e-5 (E and populations) over the 64-problem sweep of
                             20000 steps at 1.47x the FP64 batch rate; 1.6e-5 in the
                             populations after 1e5 steps (use MLN_FP32_COMP_FIELDS
                             where 1e-5 must hold).  Rotation route, N <= 3,
                             workgroup and four-lanes-per-cell kernels and the batch */
} mln_precision;

typedef enum {
  MLN_ROUTE_ROTATION = 0, /* fused form of the generalised Rodrigues route: 2x2 rotations
                             in the eigenbasis of U, the two half steps merged into one
                             shared D x D factor                                         */
  MLN_ROUTE_DIAG = 1,     /* Sec. 4.2 first route: A_I = R exp(Lambda E dt) R^+          */
  MLN_ROUTE_RODRIGUES = 2, /* Sec. 4.2 second route: A_I = I + sum sin S_i + (1-cos) S_i^2 */
  MLN_ROUTE_PADE = 3       /* the generic route the paper compares against (Sec. 4.2, Sec.
                              5.3): exp(U E dt) by a scaled diagonal Pade approximant every
                              step (degree 3, 5 or 7 from the 1-norm), applied to d by one
                              linear solve; FP64 or plain FP32.  N <= 3: one cell per
                              thread; N = 4, 6: one wavefront per cell, 512 threads per
                              workgroup, default tile 128 and 8 steps per launch (a
                              tile whose LDS need exceeds 160 KB gives MLN_EINVAL)       */
} mln_route;

/* ---- problem description ---------------------------------------------- */

/* The quantum medium: Sec. 2 (Eq. liouville, H = H0 - mu E_z) and the test
 * systems of Sec. 5.  The relaxation superoperator G is the sum of
 *   * Lindblad channels: G(rho) += rate_k (L_k rho L_k^+ - 1/2 {L_k^+ L_k, rho}),
 *   * pure dephasing:    G(rho)_ab -= dephasing * rho_ab for a != b,
 *   * a general linear map given as an N^2 x N^2 complex matrix acting on the
 *     row-major vectorisation of rho (NULL if unused).
 * G must be trace preserving.  N = n_levels; the GPU kernels are built for
 * N = 2, 3, 4 and 6 (mln_setup_factors accepts 2 <= N <= 6). */
typedef struct {
  int32_t n_levels;
  const double *h0;            /* N*N complex, Hermitian [J]                       */
  const double *dipole;        /* N*N complex, Hermitian [C m]                     */
  int32_t n_jump;              /* number of Lindblad channels (>= 0)               */
  const double *jump;          /* n_jump * N*N complex                             */
  const double *jump_rate;     /* n_jump rates [1/s]                               */
  double dephasing;            /* [1/s]                                            */
  const double *relax_superop; /* N^2*N^2 complex, or NULL                         */
  const double *rho0;          /* N*N complex initial density matrix               */
  double density;              /* N_a [1/m^3]                                      */
} mln_medium;

/* 1-D Yee grid (Fig. 1): E_z on cells 0..nx-1 at integer steps, H_y on the
 * nx-1 faces at half-integer steps, the medium on cells [med_begin, med_end)
 * with 1 <= med_begin <= med_end <= nx-1.  Cell 0 is a hard source, cell nx-1
 * a first-order Mur absorbing boundary and the probe. */
typedef struct {
  int64_t nx, nt;
  double dx, dt;
  int64_t med_begin, med_end;
  double eps_r, mu_r, sigma;   /* relative permittivity / permeability, conductivity */
} mln_grid;

/* E_z(cell 0, step n) = amplitude * samples[n] for n = 0..nt (n_samples >= nt+1). */
typedef struct {
  const double *samples;
  int64_t n_samples;
  double amplitude;
} mln_source;

/* What the run records (all float64).  Snapshot s = 0 .. nt/snap_every - 1 is
 * taken when step (s+1)*snap_every - 1 completes: E at every cell
 * (e_out[s*nx + i]) and the populations rho_aa of d^{n+1/2} on every medium
 * cell (pop_out[(s*N + a)*n_med + c]).  The probe holds E at cell nx-1 for
 * steps 0..nt (probe_out[n]).  Any pointer may be NULL. */
typedef struct {
  int64_t snap_every;          /* 0: no snapshots                                  */
  double *pop_out;
  double *e_out;
  double *probe_out;
  int32_t out_on_device;       /* 1: the pointers above are device pointers        */
} mln_record;

typedef struct {
  int32_t precision;           /* mln_precision                                    */
  int32_t route;               /* mln_route                                        */
  int32_t steps_per_launch;    /* time steps fused into one launch (0 = automatic) */
  int32_t tile;                /* cells per workgroup tile (0 = automatic)         */
  void *stream;                /* hipStream_t, NULL = default stream               */
  int32_t ckpt_every;          /* > 0: mln_run keeps a full-state checkpoint every
                                  ckpt_every steps so that mln_grad can run; 0: off;
                                  MLN_TAPE_ALL: mln_run keeps the whole forward
                                  tape (the state z' and E of every medium cell
                                  and step, (N^2) x cells x nt reals, e.g. 18 GB
                                  for 10000 cells x 50000 steps in FP32) in device
                                  memory, so that mln_grad needs no recomputation
                                  (MLN_ENOMEM if it does not fit)                 */
  int32_t variant;             /* forward kernel: 0 automatic, 1 workgroup tile
                                  (one cell per thread, LDS exchange), 2 wavefront
                                  tile (rotation route; tile/64 cells per lane),
                                  3 quad tile (rotation route, N <= 3; four lanes
                                  per cell, tile = cells per workgroup), 4
                                  streamed (rotation route, FP64 / FP32 /
                                  compensated FP32: one time step per launch,
                                  one thread per cell, tile 0 or 256, steps per
                                  launch 0 or 1; state, E and H read from and
                                  written to device memory every step), 5 quad
                                  tile with the shared-factor product on the
                                  matrix cores (rotation route, N <= 3, FP64 /
                                  FP32 / compensated modes; the 16 cells of a
                                  wavefront as one 16 x 8 by 8 x 16 product per
                                  step, Sec. 4.1 fused half steps; tile as for
                                  3, a multiple of 16).
                                  Automatic: quad for N <= 3 on grids below 1e5
                                  cells (latency-bound sizes), workgroup tile on
                                  larger ones; N = 4: wavefront tile; N = 6:
                                  workgroup tile; split-BF16 precisions: quad    */
} mln_options;

/* Gradients of a scalar objective J with respect to the physical inputs (any
 * pointer may be NULL).  Hermitian N x N inputs use one complex number per
 * entry: for a < b, d[a*N+b] = dJ/dRe(X_ab) + i dJ/dIm(X_ab) under the
 * Hermitian perturbation that changes X_ab and X_ba together (d[b*N+a] is its
 * conjugate); d[a*N+a] = dJ/dX_aa. */
typedef struct {
  double *d_h0;                /* N*N complex (level energies: the diagonal)       */
  double *d_dipole;            /* N*N complex                                      */
  double *d_jump_rate;         /* n_jump                                           */
  double *d_dephasing;         /* 1                                                */
  double *d_amplitude;         /* 1 (source amplitude)                             */
  double *d_density;           /* 1 (N_a)                                          */
} mln_grads;

typedef struct mln_handle mln_handle;

/* ---- lifecycle and forward propagation -------------------------------- */

/* Validate the problem, build the one-time FP64 factors (Sec. 3 generators,
 * M, U, v, d_eq; A0 = exp(M dt/2) and its inhomogeneous part from one
 * augmented exponential; the factorisation of U for the chosen route,
 * Sec. 4.2), upload them and set the initial state (d from rho0, E = H = 0,
 * E at cell 0 = amplitude*samples[0]).  Allocates all device memory the handle
 * needs.  Errors: MLN_EINVAL, MLN_ENOTHERMITIAN, MLN_ENOTTRACEPRESERVING,
 * MLN_ECOURANT, MLN_EBADRHO, MLN_ENOTSUPPORTED, MLN_ENOMEM, MLN_EHIP,
 * MLN_ENUMERIC.  On error *out is set to NULL. */
int mln_init(const mln_medium *medium, const mln_grid *grid, const mln_source *source,
             const mln_record *record, const mln_options *options, mln_handle **out);

/* Advance n_steps time steps (clamped to the steps left), enqueued on the
 * handle's stream; returns without waiting.  Allocates nothing. */
int mln_step(mln_handle *h, int64_t n_steps);

/* Advance to step nt, wait for the stream, copy host-side records and check
 * the recorded output for NaN/Inf (MLN_ENONFINITE).  From step 0 without
 * checkpoints or tape (and unless mln_use_graph(h, 0)), the launches of the
 * whole run are replayed as one HIP graph, captured on the first such call
 * (on a private stream; kernel nodes only) and rebuilt after mln_configure /
 * mln_tune. */
int mln_run(mln_handle *h);

/* on = 1 (default): mln_run from step 0 replays the graph described above;
 * on = 0: its launches are enqueued one by one. */
int mln_use_graph(mln_handle *h, int32_t on);

/* Return to the initial state (step 0) without rebuilding factors. */
int mln_reset(mln_handle *h);

/* Current step index (number of completed time steps). */
int mln_current_step(const mln_handle *h, int64_t *step);

/* The kernel configuration the handle runs: variant (1 workgroup tile, 2
 * wavefront tile, 3 four lanes per cell, 4 streamed, 5 four lanes per cell
 * with the matrix-core product; the automatic choice resolved),
 * cells per tile and time steps per launch.  Any pointer may be NULL. */
int mln_get_config(const mln_handle *h, int32_t *variant, int32_t *tile, int32_t *steps_per_launch);

/* Change the kernel configuration (same meaning and rules as the variant,
 * tile and steps_per_launch options of mln_init; 0 = automatic / default)
 * of a handle at step 0.  On error the configuration is unchanged.
 * Errors: MLN_ESTATE (not at step 0), MLN_EINVAL, MLN_ENOTSUPPORTED. */
int mln_configure(mln_handle *h, int32_t variant, int32_t tile, int32_t steps_per_launch);

/* Autotuner for one problem: time every kernel configuration the handle's
 * level count, precision and route allow (variants 1-5, several tile shapes)
 * on the problem itself, about trial_steps steps each from step 0 with
 * nothing recorded (HIP events on the handle's stream), keep the fastest per
 * time step and return the handle to step 0 with it.  The choice is returned
 * in *variant, *tile and *steps_per_launch (any may be NULL).  Candidates
 * that need more steps than the run has are skipped.  Synchronises.
 * Errors: MLN_ESTATE (not at step 0), MLN_EINVAL, MLN_EHIP. */
int mln_tune(mln_handle *h, int32_t trial_steps, int32_t *variant, int32_t *tile, int32_t *steps_per_launch);

/* Copy the current fields to host arrays E[nx] (step n) and H[nx-1]
 * (step n-1/2).  Synchronises the stream. */
int mln_get_fields(mln_handle *h, double *E, double *H);

/* The physical state after the completed steps (mln_current_step), host
 * arrays; any pointer may be NULL.  Synchronises.
 *   E         nx values, E at the current step (Sec. 2, Fig. 1)
 *   H         nx - 1 values, H_{i+1/2} half a step earlier
 *   rho_diag  N x nmed populations rho_aa = 1/N + (1/2) sum_l d_l (s_l)_aa
 *             (Eq. comp_rho) of every medium cell, row a = level
 * The device carries each cell's state after the first L1 half step of the
 * next step (Sec. 4.1); the Bloch vector is recovered in FP64 as
 * d = A0^-1 (d' - b0). */
int mln_get_state(const mln_handle *h, double *E, double *H, double *rho_diag);

/* The Bloch vectors d (Sec. 3: rho = 1/N + (1/2) sum_l d_l s_l, generators
 * as mln_setup_factors returns them) of every medium cell after the
 * completed steps: D x nmed host array, row l = component.  Synchronises. */
int mln_get_bloch(const mln_handle *h, double *d);

/* Replace the state at the current step (the step counter is unchanged):
 * E (nx), H (nx - 1) and Bloch vectors d (D x nmed, as
 * mln_get_bloch returns them), host arrays; NULL leaves that part as it is.
 * The values are converted to the handle's precision; d is not checked for
 * positivity.  Invalidates the checkpoints of mln_grad until the next run
 * from step 0.  MLN_EINVAL on non-finite input.  Synchronises. */
int mln_set_state(mln_handle *h, const double *E, const double *H, const double *d);

/* Opaque full-state checkpoint (fields, Bloch state, step counter).
 * mln_state_bytes gives the size; save/load copy to/from a host buffer and
 * synchronise.  A loaded state continues bit-identically. */
int mln_state_bytes(const mln_handle *h, int64_t *bytes);
int mln_save_state(mln_handle *h, void *host_buf);
int mln_load_state(mln_handle *h, const void *host_buf);

/* Prescribed-field mode (no FDTD, used by the tests): medium cell c sees
 * E = efield[t*n_med + c] at step t for t = 0..n_steps-1, starting from
 * rho0.  Records the populations of d^{t+1/2} (pop_out[(t*N + a)*n_med + c])
 * and dP/dt (dp_out[t*n_med + c]); either may be NULL.  efield, pop_out and
 * dp_out are device pointers if out_on_device was set at init, else host
 * pointers.  Synchronises.  Does not touch the coupled-run state. */
int mln_bloch_only(mln_handle *h, const double *efield, int64_t n_steps, double *pop_out,
                   double *dp_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as mln_bloch_only, with the same kernels, that allocates
 * nothing.  mln_bloch_only stages the initial Bloch state in a device buffer
 * it allocates per call; this variant stages it in a library-owned device
 * array of MLN_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends;
 * its address is looked up once per device at mln_init).  efield, pop_out
 * and dp_out must be DEVICE pointers whatever out_on_device says (no host
 * staging); pop_out and dp_out may be NULL.  The scratch is shared by every
 * call on one GPU and keeps the last call's contents (each call overwrites
 * what it reads): calls that overlap in time on one GPU (other host threads,
 * other streams) race and must be serialised by the caller.  Errors:
 * MLN_EINVAL (null pointer, negative n_steps, or an initial state larger
 * than the scratch), MLN_ESTATE, MLN_EHIP.  Synchronises the handle's
 * stream. */
#define MLN_NOALLOC_SCRATCH_BYTES 4096
int mln_bloch_only_noalloc(mln_handle *h, const double *efield, int64_t n_steps, double *pop_out,
                           double *dp_out);

/* Vector-Jacobian product of the whole run (the adjoint, reverse-time pass):
 * given g[n] = dJ/dprobe[n] for n = 0..nt (host array), fill *out with
 * dJ/d(inputs).  Needs a handle created with ckpt_every > 0 or MLN_TAPE_ALL
 * on which mln_run has completed from step 0; with checkpoints the forward
 * state is rebuilt segment by segment from them (recomputation, which leaves
 * the forward buffers in an intermediate state: mln_reset before stepping
 * again), with the whole tape in memory nothing is recomputed (and mln_grad
 * may be called again for another dJ_dprobe); each segment is swept backwards
 * by the reverse kernel, which accumulates the parameter gradients on the GPU.
 * With two or more checkpoint intervals the rebuild of the next segment runs
 * on a second stream the handle creates (non-blocking, default priority) into
 * a second segment tape while the current one is reversed, ordered by events;
 * the call waits for both streams before it returns.  The
 * final chain rule through exp(M dt/2) runs on the host in FP64.  Supported
 * for the rotation route, FP64 and FP32 (plain or compensated), N <= 3.
 * Errors: MLN_ESTATE (no completed checkpointed run), MLN_ENOTSUPPORTED.
 * Synchronises. */
int mln_grad(mln_handle *h, const double *dJ_dprobe, mln_grads *out);

/* Tiling of mln_grad's reverse kernel.  variant 0 (default): automatic
 * (after a four-lanes-per-cell forward kernel: 128-cell tiles and the
 * largest even step count up to 48 that keeps the tiles within the compute
 * units, 16 where none does; 64-cell tiles and 16 steps for the FP64
 * three-level reverse step; 256 cells and 16 steps after the streamed
 * forward kernel; otherwise the forward kernel's tiling); 1: one thread per cell, tile a multiple of 64 in [64,
 * 256]; 3: four lanes per cell, tile a multiple of 16 in [16, 128].  tile 0:
 * 256 (variant 1) or 128; steps_per_launch 0: tile/4; the halo is
 * steps_per_launch cells on each side, so 2 steps_per_launch < tile.  The
 * tape is read by cell, so the reverse tiling is independent of the forward
 * one; every tiling gives the same gradient to rounding.  Errors:
 * MLN_EINVAL, MLN_ENOTSUPPORTED (route or N the adjoint does not cover). */
int mln_configure_adjoint(mln_handle *h, int32_t variant, int32_t tile, int32_t steps_per_launch);

void mln_free(mln_handle *h);

const char *mln_strerror(int code);
const char *mln_last_error(void);

/* ---- many independent problems in one launch sequence ----------------- */

/* A batch advances n_inst independent problems in lockstep: parameter
 * sweeps over media, densities, dipoles and grid lengths, each problem
 * being the single-medium problem of Sec. 2 with its own Bloch-vector
 * propagation (Sec. 3, 4.1).  Every launch covers one chunk of time steps for
 * all problems: workgroup g is tile t of problem i according to a table on
 * the device, two- and three-level problems share the launch, and the tiles
 * are one-cell-per-thread (variant 1, the default) or four-lanes-per-cell
 * (variant 3) tiles of the rotation route.
 *   media, grids, sources  arrays of n_inst descriptors (as for mln_init);
 *                          every grid has the same dt and nt; N = 2 or 3
 *   records                array of n_inst recordings, or NULL (none)
 *   options                precision MLN_FP64, MLN_FP32, MLN_FP32_COMP,
 *                          MLN_FP32_COMP_FIELDS or MLN_FP32_FIELDS;
 *                          route MLN_ROUTE_ROTATION; variant 0 (= 1), 1 or
 *                          3; ckpt_every 0; tile / steps_per_launch as for
 *                          mln_init (0: 256 cells for variant 1, 128 for
 *                          variant 3; 16 steps); stream shared by all problems
 * Each problem gets its own handle (device state, factors, recording), owned
 * by the batch; mln_batch_instance lends it out (do not mln_free it).
 * Errors: those of mln_init (prefixed with the problem index in
 * mln_last_error), MLN_EINVAL (unequal dt or nt), MLN_ENOTSUPPORTED. */
typedef struct mln_batch mln_batch;
int mln_init_batch(int32_t n_inst, const mln_medium *media, const mln_grid *grids,
                   const mln_source *sources, const mln_record *records,
                   const mln_options *options, mln_batch **out);

/* Autotuner: time every candidate (kernel variant 1 or 3, cells per tile,
 * steps per launch) on the batch itself over about trial_steps steps (HIP
 * events on the batch's stream), keep the fastest per time step, and reset
 * the batch to step 0.  The choice is returned in *variant, *tile and
 * *steps_per_launch (any may be NULL).  Synchronises. */
int mln_batch_tune(mln_batch *b, int32_t trial_steps, int32_t *variant, int32_t *tile,
                   int32_t *steps_per_launch);

/* Set the kernel variant (1: one cell per thread, tile a multiple of 64 in
 * [64, 256]; 3: four lanes per cell, tile a multiple of 16 in [32, 256]) and
 * tile shape explicitly (batch at step 0) / read them back together with the
 * number of workgroups of one launch. */
int mln_batch_configure(mln_batch *b, int32_t variant, int32_t tile, int32_t steps_per_launch);
int mln_batch_get_config(const mln_batch *b, int32_t *variant, int32_t *tile,
                         int32_t *steps_per_launch, int64_t *workgroups);

/* on = 1 (default): mln_batch_run from step 0 replays one HIP graph holding
 * every launch of the run (captured on first use, rebuilt after a change of
 * tile shape); on = 0: launches are enqueued one by one. */
int mln_batch_use_graph(mln_batch *b, int32_t on);

/* Advance every problem by n_steps (clipped at nt); asynchronous. */
int mln_batch_step(mln_batch *b, int64_t n_steps);
/* Run every problem to nt and deliver the recordings; synchronises.
 * MLN_ESTATE if a problem was stepped on its own since the last reset. */
int mln_batch_run(mln_batch *b);
/* Back to step 0 for every problem; synchronises. */
int mln_batch_reset(mln_batch *b);
/* Borrow the handle of problem i (for mln_get_fields, mln_save_state, ...). */
int mln_batch_instance(mln_batch *b, int32_t i, mln_handle **h);
void mln_batch_free(mln_batch *b);

/* ---- pseudo-spectral (PSTD) field solver ------------------------------- */
/* The paper names PSTD as a field solver that its Liouville treatment combines
 * with, as well as FDTD (Introduction; Sec. 4).  Here: the staggered leapfrog
 * of the Yee scheme in time (E at steps n, H at n + 1/2), the spatial
 * derivatives spectral on a periodic grid of nx cells -- every Fourier mode
 * of wavenumber kappa multiplied by i kappa exp(+-i kappa dx / 2), the sign
 * giving the half-cell offset of H (x_i + dx/2) from E (x_i = i dx), the
 * Nyquist mode dropped -- and the medium advanced by the rotation route in
 * FP64, exactly as the Yee kernels do (Sec. 4.1, Eq. maxwell with the
 * derivatives replaced).
 *
 * A run is an initial-value problem: E at step 0 and H at step -1/2 are
 * given; there is no source and no absorbing boundary (the grid is a ring);
 * the probe is E at cell nx - 1, with probe[0] = E at step 0.  n_inst
 * independent problems share the grid and advance together, one workgroup
 * each; they may differ in medium (same level count) and initial fields.
 *
 *   media    n_inst media, all with the same n_levels N in {2, 3, 4, 6}
 *   grid     nx a power of two, 64 <= nx <= 4096, 4096, 2048, 1024 for
 *            N = 2, 3, 4, 6; nt >= 0; medium cells [med_begin, med_end) with
 *            1 <= med_begin <= med_end <= nx - 1; eps_r, mu_r, sigma as on
 *            the Yee grid (conductivity semi-implicit).  Stability needs
 *            c dt kappa_max / 2 < 1 with kappa_max = 2 pi (nx/2 - 1) / (nx dx),
 *            c = 1 / sqrt(eps mu): else MLN_ECOURANT
 *   e_init   n_inst x nx host array (row i: instance i), or NULL for zero
 *   h_init   n_inst x nx host array of H at step -1/2, or NULL for zero
 *   records  n_inst records (all with the same snap_every), or NULL: per
 *            instance probe_out (nt + 1), e_out (nsnap x nx) and pop_out
 *            (nsnap x N x nmed) as in mln_init, nsnap = nt / snap_every
 *   stream   hipStream_t for all device work, NULL = the default stream
 * Inputs are copied; the record buffers stay owned by the caller.  Errors:
 * MLN_EINVAL (null or out-of-range arguments, non-finite initial fields,
 * mixed level counts or snap_every), MLN_ENOTSUPPORTED (N or nx outside the
 * built set), MLN_ECOURANT, the medium errors of mln_init, MLN_ENOMEM and
 * MLN_EHIP.  On error *out is set to NULL. */
typedef struct mln_pstd mln_pstd;
int mln_pstd_init(int32_t n_inst, const mln_medium *media, const mln_grid *grid, const double *e_init,
                  const double *h_init, const mln_record *records, void *stream, mln_pstd **out);

/* Launch shape: time steps fused into one launch (0 = 256) and the most
 * threads a workgroup may have (0 = automatic, 256 or 512; a grid of nx
 * cells then runs min(nx, max_threads) threads of nx / threads cells each).
 * 256 threads hold every built grid size in registers; 512 build up to half
 * as many cells per thread (MLN_ENOTSUPPORTED beyond).  Automatic: 512
 * where built for N <= 4 (it steps one problem fastest), else 256; and 256
 * for batches of more problems than the device has compute units on grids
 * of at most 1024 cells, where two workgroups then share a compute unit. */
int mln_pstd_configure(mln_pstd *p, int32_t steps_per_launch, int32_t max_threads);

/* Launch shape: threads per workgroup (nx / cells_per_thread), cells per
 * thread and steps per launch.  Any pointer may be NULL. */
int mln_pstd_get_config(const mln_pstd *p, int32_t *threads, int32_t *cells_per_thread,
                        int32_t *steps_per_launch);

/* Advance n_steps (clamped to the steps left), enqueued on the stream;
 * returns without waiting.  Allocates nothing. */
int mln_pstd_step(mln_pstd *p, int64_t n_steps);

/* Advance to step nt, wait, copy host-side records and check every probe for
 * NaN/Inf (MLN_ENONFINITE). */
int mln_pstd_run(mln_pstd *p);

/* Back to the initial fields and medium state (step 0).  Synchronises. */
int mln_pstd_reset(mln_pstd *p);

int mln_pstd_current_step(const mln_pstd *p, int64_t *step);

/* E (at the current step) and H (half a step earlier) of instance `inst`
 * into host arrays of nx values (either may be NULL).  Synchronises. */
int mln_pstd_get_fields(mln_pstd *p, int32_t inst, double *E, double *H);

void mln_pstd_free(mln_pstd *p);

/* ---- two-dimensional TMz grid ------------------------------------------ */
/* The paper's models are one-dimensional (Conclusion names the restriction).
 * Here the same medium step (the rotation route of Sec. 4.1-4.2, every
 * medium cell as in mln_init) sits on the 2-D transverse-magnetic Yee grid:
 * E_z at cell centres (i, j), H_x at (i, j + 1/2), H_y at (i + 1/2, j),
 * the 2-D form of Eq. maxwell
 *   H_x -= dt/(mu dy) dE_z/dy,  H_y += dt/(mu dx) dE_z/dx,
 *   E_z  = ca E_z + cb (-dP/dt + dH_y/dx - dH_x/dy)   (semi-implicit sigma),
 * periodic in y, a hard source column E_z(0, j) = amplitude * samples[n] *
 * profile[j], a first-order Mur boundary (normal incidence) on column nx-1.
 * Every field array is ny x nx, row major (index j * nx + i); H_y on column
 * nx-1 is unused.
 *
 *   medium   N in {2, 3, 4, 6}; the same medium in every medium cell
 *   grid     nx >= 3, ny >= 1, nt >= 0, dx, dy, dt > 0; the medium fills the
 *            rectangle [mx0, mx1) x [my0, my1) with 1 <= mx0 <= mx1 <= nx-1,
 *            0 <= my0 <= my1 <= ny (its nmed cells numbered row major);
 *            eps_r, mu_r > 0, sigma >= 0.  Stability needs
 *            c dt sqrt(1/dx^2 + 1/dy^2) <= 1, c = 1/sqrt(eps mu): else
 *            MLN_ECOURANT
 *   source   samples[0..nt] (n >= nt + 1), amplitude, profile[0..ny-1]
 *   record   DEVICE pointers (FP64), each may be NULL: probe_out
 *            ((nt + 1) x ny: E_z(nx-1, j) at step n at [n * ny + j]),
 *            e_out (nsnap x ny x nx), pop_out (nsnap x N x nmed: rho_aa of
 *            d^{n+1/2} as in mln_init), nsnap = nt / snap_every (0: none)
 *   precision MLN_FP64, MLN_FP32 or MLN_FP32_COMP (MLN_ENOTSUPPORTED else)
 *   stream   hipStream_t for all device work, NULL = the default stream
 * One kernel launch per time step (64 x 4 cells per workgroup, the Bloch
 * state streamed from and to device memory each step).  Inputs are copied;
 * records stay owned by the caller.  Errors: MLN_EINVAL, MLN_ECOURANT,
 * MLN_ENOTSUPPORTED, the medium errors of mln_init, MLN_ENOMEM, MLN_EHIP;
 * on error *out is set to NULL. */
typedef struct {
  int64_t nx, ny, nt;
  double dx, dy, dt;
  int64_t mx0, mx1, my0, my1;
  double eps_r, mu_r, sigma;
} mln_tmz_grid;
typedef struct {
  const double *samples;
  int64_t n;
  double amplitude;
  const double *profile;
} mln_tmz_source;
typedef struct {
  int64_t snap_every;
  double *pop_out, *e_out, *probe_out;
} mln_tmz_record;
typedef struct mln_tmz mln_tmz;
int mln_tmz_init(const mln_medium *medium, const mln_tmz_grid *grid, const mln_tmz_source *source,
                 const mln_tmz_record *record, int32_t precision, void *stream, mln_tmz **out);
/* Advance min(n_steps, nt - current step) steps; asynchronous on the stream. */
int mln_tmz_step(mln_tmz *t, int64_t n_steps);
/* The remaining steps, then synchronise. */
int mln_tmz_run(mln_tmz *t);
/* Back to step 0 (initial fields and state); synchronises. */
int mln_tmz_reset(mln_tmz *t);
int mln_tmz_current_step(const mln_tmz *t, int64_t *step);
/* Replace E_z (at the current step n) and/or H_x, H_y (at n - 1/2): host
 * arrays of ny x nx values, each may be NULL; non-finite values give
 * MLN_EINVAL.  At step 0 the probe's first row is rewritten from the new
 * E_z.  Synchronises. */
int mln_tmz_set_fields(mln_tmz *t, const double *Ez, const double *Hx, const double *Hy);
/* E_z at the current step and H_x, H_y half a step earlier, into host arrays
 * of ny x nx values (each may be NULL).  Synchronises. */
int mln_tmz_get_fields(mln_tmz *t, double *Ez, double *Hx, double *Hy);
void mln_tmz_free(mln_tmz *t);

/* ---- both transverse field components ---------------------------------- */
/* The paper keeps E_z and the interaction -mu E_z only (Sec. 2) and names the
 * fixed interaction form as a limitation (Conclusion).  Here a wave along x
 * carries both transverse components and the interaction Hamiltonian is
 * H_I = -mu_z E_z - mu_y E_y: two independent Yee pairs, (E_z, H_y) as in
 * mln_init and (E_y, H_z) (Eq. maxwell for the other polarisation), coupled
 * through the medium, dP_k/dt = N_a Re Tr{mu_k (L0 + G)(rho)} for k = z, y.
 * The interaction factor of the Strang step (Sec. 4.1) is split
 * symmetrically, exp(U_y E_y dt/2) exp(U_z E_z dt) exp(U_y E_y dt/2), so that
 * every factor keeps a fixed generator and the rotation form of the
 * exponential routes (Sec. 4.2); second order like the step around it, and
 * exact when mu_y and mu_z commute.
 *
 *   medium      as mln_init; its dipole couples to E_z; N in {2, 3, 4, 6}
 *   dipole_y    N*N complex Hermitian, couples to E_y (all zero: E_y is
 *               free vacuum propagation of its source)
 *   grid        as mln_init (both components share it, the host medium and
 *               the Mur boundary at cell nx-1)
 *   source      E_z(cell 0, step n) = amplitude * samples[n],
 *               E_y(cell 0, step n) = amplitude_y * samples[n]
 *   record      DEVICE pointers (FP64), each may be NULL: ez_out, ey_out
 *               (nsnap x nx), pop_out (nsnap x N x n_med: rho_aa of
 *               d^{n+1/2}), probe_z_out, probe_y_out (E at cell nx-1 for
 *               steps 0..nt); snapshot s taken when step (s+1) snap_every - 1
 *               completes
 *   stream      hipStream_t for all device work, NULL = the default stream
 * FP64; the step costs three D x D products.  Temporal blocking: a
 * workgroup keeps both field pairs of its window in LDS and the Bloch
 * vectors in registers for K steps per launch and recomputes a halo of K
 * cells on its right and K + 1 on its left (the Mur cell depends on two
 * cells to its left).  Default: four lanes per cell (N = 2, 3; one thread
 * per cell for N = 4, 6, whose factors are read with scalar loads), K the
 * largest whose workgroups fit one per compute unit (at least 8), else 12
 * (four lanes) or 16 (mln_pol2_configure).  Inputs are copied.  Errors:
 * MLN_EINVAL, MLN_ECOURANT, MLN_ENOTSUPPORTED (N not in {2, 3, 4, 6}), the
 * medium errors of mln_init (also for dipole_y), MLN_ENOMEM, MLN_EHIP; on
 * error *out is set to NULL. */
typedef struct {
  int64_t snap_every;
  double *ez_out, *ey_out, *pop_out, *probe_z_out, *probe_y_out;
} mln_pol2_record;
typedef struct mln_pol2 mln_pol2;
int mln_pol2_init(const mln_medium *medium, const double *dipole_y, const mln_grid *grid,
                  const mln_source *source, double amplitude_y, const mln_pol2_record *record, void *stream,
                  mln_pol2 **out);
/* Kernel shape: steps per launch K and lanes per cell (default 0 and 4 for
 * N <= 3, 0 and 1 for N = 4, 6).
 * K = 0: automatic, the largest K (at least 8) for which the workgroups fit
 * one per compute unit, else 12 (four lanes) or 16 (one lane).
 *   lanes_per_cell 1: K in 0..64, one thread per cell.  K = 1: one launch
 *     per step, every field and Bloch vector read from and written to device
 *     memory each step; K > 1: blocked, 256-cell windows, 256 - 2 K - 1
 *     owned cells per workgroup.
 *   lanes_per_cell 4 (N <= 3): K in 0..48.  Blocked, 128-cell windows of
 *     four lanes per cell (512 threads), 128 - 2 K - 1 owned cells: lane r
 *     holds components 2r, 2r+1 of the Bloch vector, so each lane forms two
 *     rows of each of the three products.
 * The results do not depend on the shape beyond rounding (the same steps
 * per cell; with four lanes dP/dt and the populations are summed in
 * another order).  Takes effect with the next launch.  Errors: MLN_EINVAL
 * (p NULL, lanes not 1 or 4, K out of range), MLN_ENOTSUPPORTED (four lanes
 * with N = 4, 6). */
int mln_pol2_configure(mln_pol2 *p, int steps_per_launch, int lanes_per_cell);
/* Advance min(n_steps, nt - current step) steps; asynchronous on the stream. */
int mln_pol2_step(mln_pol2 *p, int64_t n_steps);
/* The remaining steps, then synchronise. */
int mln_pol2_run(mln_pol2 *p);
/* Back to step 0 (initial fields and state); synchronises. */
int mln_pol2_reset(mln_pol2 *p);
int mln_pol2_current_step(const mln_pol2 *p, int64_t *step);
/* E_z, E_y at the current step and H_y, H_z half a step earlier into host
 * arrays (nx values for E, nx - 1 for H; each may be NULL).  Synchronises. */
int mln_pol2_get_fields(mln_pol2 *p, double *Ez, double *Hy, double *Ey, double *Hz);
void mln_pol2_free(mln_pol2 *p);

/* ---- one-time factors (host only, no GPU needed) ---------------------- */

/* The FP64 quantities built once per medium and time step.  D = N^2-1,
 * q = N(N-1)/2.  Any pointer may be NULL.
 *   gen    D*N*N complex  SU(N) generators s_j: all u_jk, then all v_jk
 *                         (pairs j<k in lexicographic order), then
 *                         w_1..w_{N-1} (Sec. 3)
 *   M, U   D*D            Eq. elems2 (row-major, m_jk, u_jk)
 *   deq, v, d0  D         d_eq (Sec. 3), dipole vector (Eq. comp_mu), d(rho0)
 *   A0, b0 D*D, D         d -> A0 d + b0 is the exact half step of L1
 *                         (Sec. 4.1); b0 = (A0 - I) M^-1 d_eq when M is
 *                         invertible, and is defined for singular M as well
 *   T      D*D            orthogonal; T^T U T is block diagonal with q blocks
 *                         theta_i [[0,1],[-1,0]] followed by zeros
 *   theta  q              rotation rates of U's eigenvalue pairs +-i theta_i
 *   R      D*D complex    route-D eigenvectors (U = R Lambda R^+)
 *   lam    D complex      route-D eigenvalues (purely imaginary)
 *   S      q*D*D          route-R matrices S_i with U = sum theta_i S_i
 *   K, c   D*D, D         fused factor T^T A0^2 T and T^T (A0 + I) b0
 *   w, p0  D, 1           dP/dt = w . z'' + p0 in T-coordinates
 */
typedef struct {
  double *gen, *M, *U, *deq, *v, *d0, *A0, *b0, *T, *theta, *R, *lam, *S, *K, *c, *w, *p0;
} mln_factors;

int mln_setup_factors(const mln_medium *medium, double dt, mln_factors *out);

/* Host-only chain rule used by mln_grad, exposed for testing: given the
 * gradients of J with respect to the d-coordinate step quantities
 * gA = dJ/dA (D*D, A = exp(M dt)), gc = dJ/dc (D, c = (A0 + I) b0),
 * gw = dJ/dw (D, dP/dt = w . d'' + p0), gp0 = dJ/dp0, gU = dJ/dU (D*D) and
 * gd0 = dJ/dd'_0 (D, d'_0 = A0 d(rho0) + b0), fill d_h0, d_dipole,
 * d_jump_rate, d_dephasing and d_density of *out (d_amplitude untouched). */
int mln_chain_rule(const mln_medium *medium, double dt, const double *gA, const double *gc,
                   const double *gw, double gp0, const double *gU, const double *gd0,
                   mln_grads *out);

/* Library version (major*10000 + minor*100 + patch). */
int mln_version(void);

/* Diagnostic for the measurement (no problem involved): the time per step,
 * in microseconds, of `workgroups` workgroups of `threads` lanes (a multiple
 * of 64 up to 1024) that per step write one value per lane to LDS, pass one
 * workgroup barrier, read two neighbours back and run a chain of `chain` (0,
 * 32, 64 or 128) dependent FP32 FMAs -- the floor under any tile kernel's
 * step at that launch shape.  Runs `steps` and 2 `steps` steps on the
 * default stream and reports the difference per step (launch overhead
 * removed).  Allocates a small device buffer; synchronises. */
int mln_measure_step_floor(int32_t workgroups, int32_t threads, int32_t steps, int32_t chain,
                           double *us_per_step);

/* Diagnostic: the vector FMA rate of the device in TFLOP/s (fp64 = 0: FP32,
 * else FP64), from 16 independent chains of plain (not packed) FMAs per lane
 * on 32 workgroups of 256 lanes per compute unit; the peak the kernels'
 * vector code can reach at the clock under load.  Synchronises. */
int mln_measure_fma_rate(int32_t fp64, double *tflops);

#ifdef __cplusplus
}
#endif

#endif /* MLN_H */
