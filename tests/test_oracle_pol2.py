"""Pins of the oracle's two-component run (orc_run_pol2): both transverse
field components, E_z with its Yee partner H_y and E_y with G = -H_z,
coupled to the medium through H_I = -mu_z E_z - mu_y E_y, with the
interaction factor of the Strang step split symmetrically (y half, z, y
half).  The pins are properties of the equations, not copies of the update
lines:

* no second dipole and no second source: every recorded value equals the
  one-component run (orc_run) bit for bit, and E_y stays zero;
* a second dipole of zero with a second source: E_y is the free vacuum
  propagation of its source, the one-component run of an empty medium;
* equal dipoles and equal sources: the two generators commute, so the split
  is exact, and the pair (E_y, E_z) is the one-component run with dipole
  sqrt(2) mu and source sqrt(2) s rotated by 45 degrees (E_y = E_z =
  E' / sqrt(2), the same populations); this fixes both polarisation currents
  and the weight of each component in the interaction;
* dipoles that do not commute (mu_z on the 0-1 transition, mu_y on 1-2 of a
  ladder) and pulses in both components crossing a coherent slab: the field
  energy of both pairs plus N_a Tr(rho H0) is conserved to O(dt^2).
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1710_09799_amd import workloads as W


def _yee_energy(e, h_minus, dx, dt, eps, mu):
    h_plus = h_minus + dt / (mu * dx) * np.diff(e)
    return dx * (0.5 * eps * np.sum(e ** 2) + 0.5 * mu * np.sum(h_minus * h_plus))


def _problem(nx=260, nt=700, seed=3, n=3):
    p = W.random_problem(n, seed, nx=nx, nt=nt)
    return p


def test_without_second_component_equals_single_run(orc):
    p = _problem()
    n = p.medium.n_levels
    one = orc.run(p, snap_every=70)
    two = orc.run_pol2(p, np.zeros((n, n)), 0.0, snap_every=70)
    assert np.array_equal(two["probe_z"], one["probe"])
    assert np.array_equal(two["ez_snap"], one["e_snap"])
    assert np.array_equal(two["pop"], one["pop"])
    assert np.array_equal(two["hy"], one["h"])
    assert not np.any(two["ey_snap"]) and not np.any(two["probe_y"]) and not np.any(two["g"])


def test_second_source_without_second_dipole_is_free_propagation(orc):
    p = _problem()
    n = p.medium.n_levels
    two = orc.run_pol2(p, np.zeros((n, n)), 0.7, snap_every=70)
    vac = W.Problem("vac", W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0),
                    W.Grid(nx=p.grid.nx, nt=p.grid.nt, dx=p.grid.dx, dt=p.grid.dt, med_begin=1, med_end=1),
                    W.Source(p.source.samples, 0.7))
    ref = orc.run(vac, snap_every=70)
    assert np.array_equal(two["probe_y"], ref["probe"])
    assert np.array_equal(two["ey_snap"], ref["e_snap"])
    assert np.array_equal(two["g"], ref["h"])


@pytest.mark.parametrize("n,seed", [(2, 5), (3, 3)])
def test_equal_dipoles_are_a_rotated_single_run(orc, n, seed):
    check_equal_dipoles(orc, n, seed)


def check_equal_dipoles(orc, n=3, seed=3):
    p = _problem(n=n, seed=seed)
    mu = np.asarray(p.medium.dipole)
    two = orc.run_pol2(p, mu, p.source.amplitude, snap_every=70)
    assert np.array_equal(two["ez_snap"], two["ey_snap"]) and np.array_equal(two["probe_z"], two["probe_y"])
    rot = W.Problem(p.name, dataclasses.replace(p.medium, dipole=math.sqrt(2.0) * mu), p.grid,
                    W.Source(p.source.samples, math.sqrt(2.0) * p.source.amplitude))
    one = orc.run(rot, snap_every=70)
    scale = np.max(np.abs(one["e_snap"]))
    assert np.max(np.abs(math.sqrt(2.0) * two["ez_snap"] - one["e_snap"])) < 1e-12 * scale
    assert np.max(np.abs(math.sqrt(2.0) * two["probe_z"] - one["probe"])) < 1e-12 * scale
    assert np.max(np.abs(two["pop"] - one["pop"])) < 1e-12


def _two_component_energy_drift(orc, courant):
    """Pulses in both components (E_z resonant with the 0-1 transition, E_y
    with 1-2) cross a coherent three-level slab whose dipoles do not
    commute; the run is closed (zero hard source, nothing reaches the
    absorbing end).  Returns (change of the total energy) / (energy the
    medium took up)."""
    c = orc.constants()
    hb, eps, mu = c["hbar"], c["eps0"], c["mu0"]
    c0 = 1.0 / math.sqrt(eps * mu)
    dx = W.LAMBDA0 / 20
    dt = courant * dx / c0
    nx, mb, me, na = 1400, 500, 575, 1e25
    sig_t, d = 10e-15, 1e-29
    w1, w2 = W.OMEGA0, 1.1 * W.OMEGA0
    amp = 0.5 * math.pi * hb / (d * sig_t * math.sqrt(2 * math.pi))
    nt = int(round(560 * dx / (c0 * dt)))
    med = W.ladder_medium([0.0, hb * w1, hb * (w1 + w2)], [d, 0.0], density=na)
    muy = np.zeros((3, 3), dtype=np.complex128)
    muy[1, 2] = muy[2, 1] = d
    ez0, hy0 = W.moving_pulse(nx, dx, dt, 260 * dx, c0 * sig_t, w1, amp)
    ey0, g0 = W.moving_pulse(nx, dx, dt, 250 * dx, c0 * sig_t, w2, amp)
    hy0, g0 = hy0[: nx - 1], g0[: nx - 1]
    grid = W.Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=mb, med_end=me)
    prob = W.Problem("coh2", med, grid, W.Source(np.zeros(nt + 1), 0.0))
    out = orc.run_pol2(prob, muy, 0.0, snap_every=nt, init=dict(ez=ez0, hy=hy0, ey=ey0, g=g0))
    ez1, ey1 = out["ez_snap"][0], out["ey_snap"][0]
    assert np.max(np.abs(ez1[-80:])) < 1e-9 * amp and np.max(np.abs(ey1[-80:])) < 1e-9 * amp
    levels = np.real(np.diag(med.h0))
    w_med = na * dx * np.sum(levels[:, None] * out["pop"][0])
    w0 = _yee_energy(ez0, hy0, dx, dt, eps, mu) + _yee_energy(ey0, g0, dx, dt, eps, mu)
    w1_ = _yee_energy(ez1, out["hy"], dx, dt, eps, mu) + _yee_energy(ey1, out["g"], dx, dt, eps, mu) + w_med
    # both transitions took part: population reached the top level
    assert np.max(out["pop"][0][2]) > 1e-3
    assert w_med > 0.05 * w0
    return (w1_ - w0) / w_med


def test_noncommuting_dipoles_conserve_energy_to_second_order(orc):
    check_noncommuting_energy(orc)


def check_noncommuting_energy(orc):
    d1 = _two_component_energy_drift(orc, 0.5)
    d2 = _two_component_energy_drift(orc, 0.25)
    print(f"energy drift {d1:.3e} {d2:.3e}")
    assert abs(d1) < 0.02
    assert abs(d2) < abs(d1) / 3.0
