// fwd_batch.hpp -- one launch that advances many independent problems.
//
// Every workgroup is one tile of one problem.  A table in device memory maps
// the workgroup index to (problem, tile); the problem's arguments (buffers,
// factors, grid, recording) live in device memory too, one copy per
// ping-pong slot, so a launch carries only the step range and the slot.
// Two- and three-level problems share a launch: the workgroup branches once,
// uniformly, to the four-lanes-per-cell tile of its level count.  All problems
// advance in lockstep with one time step, so the launch sequence of a whole
// run is fixed and can be captured in a HIP graph.
#pragma once

#include "fwd_quad.hpp"

namespace mln {

template <typename Real, bool COMP, bool CF>
__global__ void __launch_bounds__(1024)
    fwd_quad_batch_kernel(const BatchInst<Real> *__restrict__ inst, const BatchTile *__restrict__ tiles,
                          int64_t step0, int nsteps, int slot) {
  const BatchTile bt = tiles[blockIdx.x];
  const BatchInst<Real> &bi = inst[bt.inst];
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
  if (bi.n_levels == 2)
    quad_tile<2, Real, COMP, CF>(a, bt.tile);
  else
    quad_tile<3, Real, COMP, CF>(a, bt.tile);
}

}  // namespace mln
