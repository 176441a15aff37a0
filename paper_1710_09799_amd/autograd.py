"""torch.autograd.Function over the coupled solver.

``LadderTransmission.apply(params, problem, precision, ckpt_every)`` runs the
forward simulation on the GPU and returns the probe trace E(cell nx-1, step n)
for n = 0..nt.  ``params`` is a float64 CPU tensor of a ladder medium:

    [E_0, ..., E_{N-1},          level energies [J]
     mu_01, ..., mu_{N-2,N-1},   nearest-neighbour real dipole elements [C m]
     gamma,                      Lindblad decay rate of every |a><a+1| channel
     gamma_phi,                  pure-dephasing rate
     amplitude]                  source amplitude [V/m]

The backward pass is the library's adjoint (reverse-time) kernel with
checkpoint recomputation (mln_grad); it returns dJ/dparams for any upstream
gradient dJ/dprobe.  Only the rotation route is differentiable.
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import mln
from . import workloads as W


def ladder_problem(template, params):
    """Copy of ``template`` whose medium is the ladder described by params."""
    p = np.asarray(params, dtype=np.float64)
    n = template.medium.n_levels
    energies = p[:n]
    dip = p[n:2 * n - 1]
    gamma, gphi, amp = p[2 * n - 1], p[2 * n], p[2 * n + 1]
    prob = copy.copy(template)
    med = W.ladder_medium(energies, dip, density=template.medium.density, decay=0.0,
                          dephasing=gphi)
    med.rho0 = template.medium.rho0.copy()
    for a in range(n - 1):
        L = np.zeros((n, n), dtype=np.complex128)
        L[a, a + 1] = 1.0
        med.jumps.append(L)
        med.jump_rates.append(float(gamma))
    prob.medium = med
    prob.source = W.Source(samples=template.source.samples, amplitude=float(amp))
    return prob


def ladder_params(problem):
    med = problem.medium
    n = med.n_levels
    e = np.real(np.diag(med.h0))
    dip = [med.dipole[a, a + 1].real for a in range(n - 1)]
    gamma = med.jump_rates[0] if med.jump_rates else 0.0
    return np.concatenate([e, dip, [gamma, med.dephasing, problem.source.amplitude]])


def grads_to_ladder(g, n):
    """Map the library's physical gradients to the ladder parameter vector."""
    de = [g["d_h0"][a, a].real for a in range(n)]
    dd = [g["d_dipole"][a, a + 1].real for a in range(n - 1)]
    return np.concatenate([de, dd, [float(np.sum(g["d_jump_rate"])), g["d_dephasing"],
                                    g["d_amplitude"]]])


class LadderTransmission(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, template, precision="fp32c", ckpt_every=500):
        prob = ladder_problem(template, params.detach().cpu().numpy())
        solver = mln.Solver(prob, precision=precision, ckpt_every=ckpt_every)
        out = solver.run()
        ctx.solver = solver
        ctx.n = prob.medium.n_levels
        return out["probe"].clone()

    @staticmethod
    def backward(ctx, grad_probe):
        g = ctx.solver.grad(grad_probe.detach().double().cpu().numpy())
        ctx.solver.close()
        return torch.tensor(grads_to_ladder(g, ctx.n), dtype=torch.float64), None, None, None
