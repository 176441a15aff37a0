// fwd_batch.hpp -- one launch that advances many independent problems.
//
// Every workgroup is one tile of one problem.  A table in device memory maps
// the workgroup index to (problem, tile); the problem's arguments (buffers,
// factors, grid, recording) live in device memory too, one copy per
// ping-pong slot, so a launch carries only the step range and the slot.
// Two- and three-level problems share a launch: the workgroup branches once,
// uniformly, to the tile of its level count -- four lanes per cell, or one
// cell per thread (the better choice once the batch fills the chip).  All
// problems advance in lockstep with one time step, so the launch sequence of
// a whole run is fixed and can be captured in a HIP graph.
#pragma once

#include "fwd_quad.hpp"

namespace mln {

// The arguments of this workgroup's problem for the launch's step range.
template <typename Real>
__device__ __forceinline__ FwdArgs<Real> batch_args(const BatchInst<Real> &bi, int64_t step0, int nsteps, int slot) {
  FwdArgs<Real> a = bi.a[slot];
  a.step0 = step0;
  a.nsteps = nsteps;
  a.snap_next = -1;
  a.snap_i0 = 0;
  if (a.snap_every > 0) {  // first step n >= step0 with (n+1) % snap_every == 0
    const int64_t k = step0 / a.snap_every;
    a.snap_next = (k + 1) * a.snap_every - 1;
    a.snap_i0 = k;
  }
  return a;
}

template <typename Real, bool COMP, bool CF>
__global__ void __launch_bounds__(1024)
    fwd_quad_batch_kernel(const BatchInst<Real> *__restrict__ inst, const BatchTile *__restrict__ tiles,
                          int64_t step0, int nsteps, int slot) {
  const BatchTile bt = tiles[blockIdx.x];
  const BatchInst<Real> &bi = inst[bt.inst];
  const FwdArgs<Real> a = batch_args(bi, step0, nsteps, slot);
  if (bi.n_levels == 2)
    quad_tile<2, Real, COMP, CF>(a, bt.tile);
  else
    quad_tile<3, Real, COMP, CF>(a, bt.tile);
}

// Compiled for seven wavefronts per SIMD: the default register budget held
// 3-4 (115 to 135 VGPRs) and left the vector units half idle.  Measured on
// the 64-problem sweep (tile 256, 16 steps per launch), cell-updates/s
// against the default budget: FP64 1.04e11 / 8.78e10, FP32 1.64e11 /
// 1.50e11, compensated state 9.27e10 / 8.58e10, compensated state and
// fields 8.50e10 / 6.61e10, compensated fields 1.46e11 / 1.29e11; five, six
// and eight wavefronts were slower than seven.  The budget costs spills
// (12-156 B per lane, some inside the step loop); the added wavefronts
// more than pay for them when there are many tiles (many_tiles).
template <typename Real, bool COMP, bool CF>
__device__ __forceinline__ void block_batch_tile(const BatchInst<Real> *__restrict__ inst,
                                                 const BatchTile *__restrict__ tiles, int64_t step0, int nsteps,
                                                 int slot) {
  const BatchTile bt = tiles[blockIdx.x];
  const BatchInst<Real> &bi = inst[bt.inst];
  const FwdArgs<Real> a = batch_args(bi, step0, nsteps, slot);
  if (bi.n_levels == 2)
    block_tile<2, Real, ROUTE_ROT, COMP, CF>(a, bt.tile);
  else
    block_tile<3, Real, ROUTE_ROT, COMP, CF>(a, bt.tile);
}
template <typename Real, bool COMP, bool CF>
__global__ void __launch_bounds__(kMaxTile) __attribute__((amdgpu_waves_per_eu(7, 8)))
    fwd_block_batch_kernel(const BatchInst<Real> *__restrict__ inst, const BatchTile *__restrict__ tiles,
                           int64_t step0, int nsteps, int slot) {
  block_batch_tile<Real, COMP, CF>(inst, tiles, step0, nsteps, slot);
}
// the default register budget, for batches of few tiles
template <typename Real, bool COMP, bool CF>
__global__ void __launch_bounds__(kMaxTile)
    fwd_block_batch_kernel_few(const BatchInst<Real> *__restrict__ inst, const BatchTile *__restrict__ tiles,
                               int64_t step0, int nsteps, int slot) {
  block_batch_tile<Real, COMP, CF>(inst, tiles, step0, nsteps, slot);
}

}  // namespace mln
