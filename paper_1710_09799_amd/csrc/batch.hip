// batch.hip -- many independent problems in one lockstep launch sequence:
// the batched ABI of include/mln.h (mln_init_batch and mln_batch_*), its
// tile autotuner and the HIP-graph capture of a whole run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "fwd_batch.hpp"
#include "handle.hpp"

using namespace mln;

namespace mln {

template <typename Real, bool COMP, bool CF>
void launch_block_batch(bool many, dim3 grid, dim3 block, const BatchInst<Real> *inst, const BatchTile *tiles,
                        int64_t step0, int nsteps, int slot, hipStream_t st) {
  if (many)
    hipLaunchKernelGGL((fwd_block_batch_kernel<Real, COMP, CF>), grid, block, 0, st, inst, tiles, step0, nsteps,
                       slot);
  else
    hipLaunchKernelGGL((fwd_block_batch_kernel_few<Real, COMP, CF>), grid, block, 0, st, inst, tiles, step0,
                       nsteps, slot);
}

// quad = true: four lanes per cell (4 W threads per workgroup); false: one
// cell per thread (W threads), compiled for seven wavefronts per SIMD when
// the launch has many tiles (many_tiles).
template <typename Real>
hipError_t launch_fwd_batch(bool quad, bool comp, bool cf, int W, const BatchInst<Real> *inst,
                            const BatchTile *tiles, int64_t nblocks, int64_t step0, int nsteps, int slot,
                            hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  const dim3 grid((unsigned)nblocks), block(quad ? 4 * W : W);
  const bool many = many_tiles(nblocks);
  if (cf && !comp) {
    // plain single-precision state, float-float fields
    if constexpr (std::is_same<Real, float>::value) {
      if (quad)
        hipLaunchKernelGGL((fwd_quad_batch_kernel<float, false, true>), grid, block, 0, st, inst, tiles, step0, nsteps,
                           slot);
      else
        launch_block_batch<float, false, true>(many, grid, block, inst, tiles, step0, nsteps, slot, st);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (comp) {
    if constexpr (std::is_same<Real, float>::value) {
      if (quad && cf)
        hipLaunchKernelGGL((fwd_quad_batch_kernel<float, true, true>), grid, block, 0, st, inst, tiles, step0,
                           nsteps, slot);
      else if (quad)
        hipLaunchKernelGGL((fwd_quad_batch_kernel<float, true, false>), grid, block, 0, st, inst, tiles, step0,
                           nsteps, slot);
      else if (cf)
        launch_block_batch<float, true, true>(many, grid, block, inst, tiles, step0, nsteps, slot, st);
      else
        launch_block_batch<float, true, false>(many, grid, block, inst, tiles, step0, nsteps, slot, st);
    } else {
      return hipErrorInvalidValue;
    }
  } else if (quad) {
    hipLaunchKernelGGL((fwd_quad_batch_kernel<Real, false, false>), grid, block, 0, st, inst, tiles, step0, nsteps,
                       slot);
  } else {
    launch_block_batch<Real, false, false>(many, grid, block, inst, tiles, step0, nsteps, slot, st);
  }
  return hipGetLastError();
}

}  // namespace mln

struct mln_batch {
  std::vector<mln_handle *> inst;  // owned
  int prec = MLN_FP32;
  bool comp = false, cf = false;     // compensated state / fields
  hipStream_t stream = nullptr;       // the caller's stream
  hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
  int variant = 3;                    // 3: four lanes per cell, 1: one cell per thread
  int W = 0, halo = 0;
  int64_t nt = 0, step = 0, nblocks = 0;
  int cur = 0;
  mln::DevBuf dinst, dtiles;
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~mln_batch() {
    drop_graph();
    for (mln_handle *h : inst) mln_free(h);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

namespace {

bool valid_tiling(int variant, int W, int K) {
  if (K < 1 || 2 * K >= W || K > kMaxStepsPerLaunch) return false;
  if (variant == 3) return W >= 32 && W <= kMaxQuadTile && W % 16 == 0;
  if (variant == 1) return W >= 64 && W <= kMaxTile && W % 64 == 0;
  return false;
}

template <typename Real>
int upload_tables(mln_batch *b) {
  std::vector<BatchInst<Real>> hi(b->inst.size());
  std::vector<BatchTile> tiles;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    mln_handle *h = b->inst[i];
    const FacDev<Real> &fd = [&]() -> const FacDev<Real> & {
      if constexpr (std::is_same<Real, double>::value)
        return h->fd;
      else
        return h->ff;
    }();
    const int keep = h->cur;
    for (int s = 0; s < 2; ++s) {
      h->cur = s;
      hi[i].a[s] = make_args<Real>(h, fd, 0, 0, true);
    }
    h->cur = keep;
    hi[i].n_levels = h->f.N;
    for (int64_t t = 0; t < h->ntiles; ++t) tiles.push_back(BatchTile{(int32_t)i, (int32_t)t});
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(b->dinst.alloc(hi.size() * sizeof(BatchInst<Real>)));
  HIP_TRY(hipMemcpy(b->dinst.p, hi.data(), hi.size() * sizeof(BatchInst<Real>), hipMemcpyHostToDevice));
  HIP_TRY(b->dtiles.alloc(std::max<size_t>(tiles.size(), 1) * sizeof(BatchTile)));
  if (!tiles.empty())
    HIP_TRY(hipMemcpy(b->dtiles.p, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice));
  b->nblocks = (int64_t)tiles.size();
  return MLN_OK;
}

// Set the kernel and tile shape of every problem and rebuild the device tables.
int configure(mln_batch *b, int variant, int W, int K) {
  if (!valid_tiling(variant, W, K))
    return set_err(MLN_EINVAL,
                   "batch tiling: variant 3 (tile a multiple of 16 in [32, 256]) or 1 (a multiple of 64 in "
                   "[64, 256]), 2 steps_per_launch < tile, steps_per_launch <= 128");
  int64_t blocks = 0;
  for (mln_handle *h : b->inst) blocks += (h->grid.nx + (W - 2 * K) - 1) / (W - 2 * K);
  if (blocks > 0x7fffffff) return set_err(MLN_EINVAL, "too many workgroups for one launch");
  for (mln_handle *h : b->inst) {
    h->quad = variant == 3;
    h->wave = false;
    h->W = W;
    h->halo = K;
    h->owned = W - 2 * K;
    h->ntiles = (h->grid.nx + h->owned - 1) / h->owned;
  }
  b->variant = variant;
  b->W = W;
  b->halo = K;
  b->drop_graph();
  return b->prec == MLN_FP64 ? upload_tables<double>(b) : upload_tables<float>(b);
}

int enqueue(mln_batch *b, int64_t step0, int k, int slot, hipStream_t st) {
  hipError_t e;
  const bool quad = b->variant == 3;
  if (b->prec == MLN_FP64)
    e = launch_fwd_batch<double>(quad, false, false, b->W, (const BatchInst<double> *)b->dinst.p,
                                 (const BatchTile *)b->dtiles.p, b->nblocks, step0, k, slot, st);
  else
    e = launch_fwd_batch<float>(quad, b->comp, b->cf, b->W, (const BatchInst<float> *)b->dinst.p,
                                (const BatchTile *)b->dtiles.p, b->nblocks, step0, k, slot, st);
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
  return MLN_OK;
}

// Every problem must sit at the batch's step and ping-pong slot (a problem
// stepped on its own through its handle leaves the lockstep).
int check_lockstep(const mln_batch *b) {
  for (const mln_handle *h : b->inst)
    if (h->step != b->step || h->cur != b->cur)
      return set_err(MLN_ESTATE, "a problem of the batch was stepped on its own; mln_batch_reset first");
  return MLN_OK;
}

void advance(mln_batch *b, int64_t k, int launches) {
  b->step += k;
  if (launches & 1) b->cur = 1 - b->cur;
  for (mln_handle *h : b->inst) {
    h->step = b->step;
    h->cur = b->cur;
  }
}

int step_eager(mln_batch *b, int64_t n) {
  int64_t done = 0;
  int launches = 0, slot = b->cur;
  while (done < n) {
    const int k = (int)std::min<int64_t>(n - done, b->halo);
    int rc = enqueue(b, b->step + done, k, slot, b->stream);
    if (rc) return rc;
    slot = 1 - slot;
    done += k;
    ++launches;
  }
  advance(b, n, launches);
  return MLN_OK;
}

// Capture the launch sequence of a whole run (steps 0..nt, from slot 0).
int capture_run(mln_batch *b) {
  if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  int slot = 0, rc = MLN_OK;
  for (int64_t s = 0; s < b->nt && rc == MLN_OK;) {
    const int k = (int)std::min<int64_t>(b->nt - s, b->halo);
    rc = enqueue(b, s, k, slot, b->cap_stream);
    slot = 1 - slot;
    s += k;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return set_err(MLN_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  b->graph = g;
  HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return MLN_OK;
}

}  // namespace

extern "C" {

int mln_init_batch(int32_t n_inst, const mln_medium *media, const mln_grid *grids, const mln_source *sources,
                   const mln_record *records, const mln_options *options, mln_batch **out) {
  if (!out) return set_err(MLN_EINVAL, "null output");
  *out = nullptr;
  if (n_inst < 1 || !media || !grids || !sources) return set_err(MLN_EINVAL, "need n_inst >= 1 problems");
  mln_options opt{};
  if (options) opt = *options;
  if (opt.precision != MLN_FP64 && opt.precision != MLN_FP32 && opt.precision != MLN_FP32_COMP &&
      opt.precision != MLN_FP32_COMP_FIELDS && opt.precision != MLN_FP32_FIELDS)
    return set_err(MLN_ENOTSUPPORTED, "batched launch: FP64, FP32 or compensated FP32");
  if (opt.route != MLN_ROUTE_ROTATION) return set_err(MLN_ENOTSUPPORTED, "batched launch: rotation route only");
  if (opt.variant != 0 && opt.variant != 1 && opt.variant != 3)
    return set_err(MLN_ENOTSUPPORTED, "batched launch: one-cell-per-thread or four-lanes-per-cell tiles");
  if (opt.ckpt_every != 0) return set_err(MLN_ENOTSUPPORTED, "batched launch: no checkpoints");
  const int variant = opt.variant == 0 ? 1 : opt.variant;
  const int W = opt.tile > 0 ? opt.tile : (variant == 3 ? 128 : 256);
  const int K = opt.steps_per_launch > 0 ? opt.steps_per_launch : 16;
  if (!valid_tiling(variant, W, K))
    return set_err(MLN_EINVAL, "batch tiling: variant 3 (tile a multiple of 16 in [32, 256]) or 1 (a multiple "
                               "of 64 in [64, 256]), 2 steps_per_launch < tile, steps_per_launch <= 128");
  for (int32_t i = 0; i < n_inst; ++i) {
    if (media[i].n_levels != 2 && media[i].n_levels != 3)
      return set_err(MLN_ENOTSUPPORTED, "batched launch: N = 2 or 3 levels");
    if (grids[i].dt != grids[0].dt || grids[i].nt != grids[0].nt)
      return set_err(MLN_EINVAL, "batched problems advance in lockstep: equal dt and nt");
  }
  std::unique_ptr<mln_batch> b(new mln_batch());
  b->prec = opt.precision;
  b->comp = opt.precision == MLN_FP32_COMP || opt.precision == MLN_FP32_COMP_FIELDS;
  b->cf = opt.precision == MLN_FP32_COMP_FIELDS || opt.precision == MLN_FP32_FIELDS;
  b->stream = (hipStream_t)opt.stream;
  b->nt = grids[0].nt;
  mln_options o = opt;
  o.variant = variant;
  o.tile = W;
  o.steps_per_launch = K;
  for (int32_t i = 0; i < n_inst; ++i) {
    mln_handle *h = nullptr;
    int rc = mln_init(&media[i], &grids[i], &sources[i], records ? &records[i] : nullptr, &o, &h);
    if (rc) {
      std::string m = "problem " + std::to_string(i) + ": " + mln_last_error();
      return set_err(rc, m);
    }
    b->inst.push_back(h);
  }
  int rc = configure(b.get(), variant, W, K);
  if (rc) return rc;
  *out = b.release();
  return MLN_OK;
}

int mln_batch_configure(mln_batch *b, int32_t variant, int32_t tile, int32_t steps_per_launch) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  if (b->step != 0) return set_err(MLN_ESTATE, "configure a batch at step 0 (mln_batch_reset)");
  return configure(b, variant, tile, steps_per_launch);
}

int mln_batch_get_config(const mln_batch *b, int32_t *variant, int32_t *tile, int32_t *steps_per_launch,
                         int64_t *workgroups) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  if (variant) *variant = b->variant;
  if (tile) *tile = b->W;
  if (steps_per_launch) *steps_per_launch = b->halo;
  if (workgroups) *workgroups = b->nblocks;
  return MLN_OK;
}

int mln_batch_use_graph(mln_batch *b, int32_t on) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  b->use_graph = on != 0;
  return MLN_OK;
}

int mln_batch_reset(mln_batch *b) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  for (mln_handle *h : b->inst) {
    int rc = reset_state(h);
    if (rc) return rc;
  }
  b->step = 0;
  b->cur = 0;
  return MLN_OK;
}

int mln_batch_step(mln_batch *b, int64_t n_steps) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  if (n_steps < 0) return set_err(MLN_EINVAL, "n_steps must be >= 0");
  int rc = check_lockstep(b);
  if (rc) return rc;
  return step_eager(b, std::min<int64_t>(n_steps, b->nt - b->step));
}

int mln_batch_run(mln_batch *b) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  int rc = check_lockstep(b);
  if (rc) return rc;
  if (b->use_graph && b->step == 0 && b->cur == 0 && b->nt > 0 && b->nblocks > 0) {
    if (!b->exec) {
      rc = capture_run(b);
      if (rc) return rc;
    }
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    const int64_t launches = (b->nt + b->halo - 1) / b->halo;
    advance(b, b->nt, (int)(launches & 1));
  } else {
    rc = step_eager(b, b->nt - b->step);
    if (rc) return rc;
  }
  for (mln_handle *h : b->inst) {
    rc = finish_run(h);
    if (rc) return rc;
  }
  return MLN_OK;
}

int mln_batch_tune(mln_batch *b, int32_t trial_steps, int32_t *variant, int32_t *tile, int32_t *steps_per_launch) {
  if (!b) return set_err(MLN_EINVAL, "null batch");
  if (trial_steps < 1) return set_err(MLN_EINVAL, "trial_steps must be >= 1");
  // (variant, cells per tile, steps per launch)
  static const int cand[][3] = {{3, 64, 8},   {3, 64, 16},  {3, 96, 16},  {3, 128, 8},  {3, 128, 16},
                                {3, 128, 32}, {3, 192, 16}, {3, 192, 32}, {3, 256, 16}, {3, 256, 32},
                                {3, 256, 64}, {1, 128, 16}, {1, 128, 32}, {1, 192, 16}, {1, 192, 32},
                                {1, 256, 16}, {1, 256, 32}, {1, 256, 64}};
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best = INFINITY;
  int bv = b->variant, bw = b->W, bk = b->halo, rc = MLN_OK;
  const int64_t nt = b->nt;
  for (const auto &c : cand) {
    if (!valid_tiling(c[0], c[1], c[2])) continue;
    // whole launches only, at least two, and within the run length
    int64_t steps = std::max<int64_t>(2 * c[2], (trial_steps + c[2] - 1) / c[2] * c[2]);
    if (steps + c[2] > nt) continue;
    if ((rc = configure(b, c[0], c[1], c[2])) || (rc = mln_batch_reset(b))) break;
    if ((rc = step_eager(b, c[2]))) break;  // warm-up launch
    if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = set_err(MLN_EHIP, "event record"); break; }
    if ((rc = step_eager(b, steps))) break;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = set_err(MLN_EHIP, "event synchronize");
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double per_step = ms / (double)steps;
    if (per_step < best) {
      best = per_step;
      bv = c[0];
      bw = c[1];
      bk = c[2];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = configure(b, bv, bw, bk)) || (rc = mln_batch_reset(b))) return rc;
  if (variant) *variant = bv;
  if (tile) *tile = bw;
  if (steps_per_launch) *steps_per_launch = bk;
  return MLN_OK;
}

int mln_batch_instance(mln_batch *b, int32_t i, mln_handle **h) {
  if (!b || !h) return set_err(MLN_EINVAL, "null argument");
  if (i < 0 || i >= (int32_t)b->inst.size()) return set_err(MLN_EINVAL, "instance index out of range");
  *h = b->inst[i];
  return MLN_OK;
}

void mln_batch_free(mln_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  delete b;
}

}  // extern "C"
