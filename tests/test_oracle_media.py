"""Pins of the oracle's coupled Yee run (orc_run) where a medium or a
non-vacuum host is present: the feedback of the polarisation current into
the field (Sec. 2, Eq. maxwell, with dP/dt of Eq. polarization2), the
semi-implicit conductivity, and the permittivity and permeability of the
host.  Each pin is a closed form or a conservation law of the discrete
scheme, not a second copy of the oracle's update lines:

* energy balance: without relaxation the field energy plus the level energy
  N_a Tr(rho H0) is a constant of the coupled equations; the leapfrog keeps
  it to O(dt^2).  A polarisation term with the wrong sign or weight, or a
  wrong density factor, leaves an O(1) error;
* a CW wave in a conducting host: attenuation, phase advance and impedance
  follow the dispersion relation of the semi-implicit Yee scheme, derived
  below from the update equations written as difference quotients;
* the magic time step in a dielectric / magnetic host (c_h dt = dx with
  c_h = 1/sqrt(eps mu)): exact translation of E, and H = -E / Z with
  Z = sqrt(mu / eps), which tells eps_r and mu_r apart (the speed alone
  does not).
"""
import math

import numpy as np
import pytest

from paper_1710_09799_amd import workloads as W


def _yee_energy(e, h_minus, dx, dt, eps, mu):
    """Discrete field energy of the 1-D Yee scheme at integer step n:
    dx sum (eps E_i^2 / 2 + mu H_{i+1/2}^{n-1/2} H_{i+1/2}^{n+1/2} / 2), with
    H^{n+1/2} = H^{n-1/2} + dt/(mu dx) (E_{i+1} - E_i).  It is conserved
    exactly in vacuum between perfectly conducting ends."""
    h_plus = h_minus + dt / (mu * dx) * np.diff(e)
    return dx * (0.5 * eps * np.sum(e ** 2) + 0.5 * mu * np.sum(h_minus * h_plus))


def _coherent_yee_energy_drift(orc, courant, mutate=None):
    """A pi pulse given as initial fields crosses a coherent two-level slab
    (no relaxation).  Cell 0 is the (zero) hard source, i.e. a perfect
    conductor; the run stops before any field reaches the absorbing end.
    Returns (change of field + level energy) / (energy the medium took up)."""
    c = orc.constants()
    hb, eps, mu = c["hbar"], c["eps0"], c["mu0"]
    c0 = 1.0 / math.sqrt(eps * mu)
    dx = W.LAMBDA0 / 20
    dt = courant * dx / c0
    nx, mb, me, na = 1400, 500, 575, 1e25
    sig_t, d = 10e-15, 1e-29
    amp = math.pi * hb / (d * sig_t * math.sqrt(2 * math.pi))
    nt = int(round(560 * dx / (c0 * dt)))
    med = W.ladder_medium([0.0, hb * W.OMEGA0], [d], density=na)
    if mutate is not None:
        med = mutate(med)
    e0, h0 = W.moving_pulse(nx, dx, dt, 260 * dx, c0 * sig_t, W.OMEGA0, amp)
    h0 = h0[: nx - 1]
    grid = W.Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=mb, med_end=me)
    out = orc.run(W.Problem("coh", med, grid, W.Source(np.zeros(nt + 1), 0.0)),
                  snap_every=nt, e_init=e0, h_init=h0)
    e1 = out["e_snap"][0]
    # nothing reached the absorbing boundary: the run is closed
    assert np.max(np.abs(e1[-80:])) < 1e-9 * amp
    assert np.max(np.abs(out["probe"])) < 1e-9 * amp
    levels = np.real(np.diag(med.h0))
    w_med = na * dx * np.sum(levels[:, None] * out["pop"][0])
    w0 = _yee_energy(e0, h0, dx, dt, eps, mu)
    w1 = _yee_energy(e1, out["h"], dx, dt, eps, mu) + w_med
    assert w_med > 0.1 * w0  # the slab takes up a sizeable part of the pulse
    return (w1 - w0) / w_med


def test_yee_vacuum_energy_is_exact(orc):
    """Empty medium: the discrete energy is conserved to rounding."""
    c = orc.constants()
    eps, mu = c["eps0"], c["mu0"]
    c0 = 1.0 / math.sqrt(eps * mu)
    dx = W.LAMBDA0 / 20
    dt = 0.5 * dx / c0
    nx, nt = 600, 500
    e0, h0 = W.moving_pulse(nx, dx, dt, 150 * dx, 20 * dx, W.OMEGA0, 1e8)
    h0 = h0[: nx - 1]
    med = W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0)
    grid = W.Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=1, med_end=1)
    out = orc.run(W.Problem("vac", med, grid, W.Source(np.zeros(nt + 1), 0.0)),
                  snap_every=nt, e_init=e0, h_init=h0)
    w0 = _yee_energy(e0, h0, dx, dt, eps, mu)
    w1 = _yee_energy(out["e_snap"][0], out["h"], dx, dt, eps, mu)
    assert abs(w1 - w0) < 1e-12 * w0


def test_yee_coherent_medium_conserves_energy_to_second_order(orc):
    """Field energy plus N_a Tr(rho H0) over a pulse crossing a coherent
    slab: the drift is small and falls by about four when dt halves."""
    check_coherent_energy(orc)


def check_coherent_energy(orc):
    d1 = _coherent_yee_energy_drift(orc, 0.5)
    d2 = _coherent_yee_energy_drift(orc, 0.25)
    assert abs(d1) < 0.02
    assert abs(d2) < abs(d1) / 3.0


def _lossy_k(omega, dx, dt, eps, mu, sigma):
    """Complex wavenumber of E ~ exp(i(omega t - k x)) in the semi-implicit
    lossy Yee scheme.  With the updates
        mu (H^{n+1/2} - H^{n-1/2}) / dt = (E_{i+1} - E_i) / dx,
        eps (E^{n+1} - E^n) / dt + sigma (E^{n+1} + E^n) / 2
            = (H_{i+1/2} - H_{i-1/2}) / dx,
    a plane wave gives
        sin^2(k dx/2) = eps mu (dx/dt)^2 sin^2(w dt/2)
                        - i (mu sigma dx^2 / (2 dt)) sin(w dt/2) cos(w dt/2)
    (Im k < 0: decay towards +x)."""
    s, co = math.sin(omega * dt / 2), math.cos(omega * dt / 2)
    rhs = eps * mu * (dx / dt) ** 2 * s * s - 1j * (mu * sigma * dx * dx / (2 * dt)) * s * co
    return 2.0 / dx * np.arcsin(np.sqrt(rhs + 0j))


def _cw_fit(orc, eps_r, mu_r, sigma, courant=0.5, nx=1600, nt=3000):
    """Drive a CW wave, switched on smoothly over eight periods, into a host
    (eps_r, mu_r, sigma) that fills the grid; return (measured k, predicted k,
    max relative H mismatch).  The wave front stays short of the far end, so
    nothing is reflected; the smooth switch-on keeps the zero-frequency part
    of the drive (which a conductor turns into a static H) negligible."""
    c = orc.constants()
    eps, mu = c["eps0"] * eps_r, c["mu0"] * mu_r
    ch = 1.0 / math.sqrt(eps * mu)
    dx = W.DX0
    dt = courant * dx / ch
    w = W.OMEGA0
    t = np.arange(nt + 1) * dt
    t_on = 16 * math.pi / w
    ramp = np.where(t < t_on, 0.5 - 0.5 * np.cos(math.pi * t / t_on), 1.0)
    med = W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0)
    grid = W.Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=1, med_end=1,
                  eps_r=eps_r, mu_r=mu_r, sigma=sigma)
    out = orc.run(W.Problem("host", med, grid, W.Source(ramp * np.sin(w * t), 1.0)),
                  snap_every=1)
    e_n, e_p = out["e_snap"][-1], out["e_snap"][-2]
    i = np.arange(10, 140)
    # E^n_i = a_i cos(theta_i), E^{n-1}_i = a_i cos(theta_i - w dt)
    z = e_n[i] + 1j * (e_p[i] - e_n[i] * math.cos(w * dt)) / math.sin(w * dt)
    x = i * dx
    im_k = np.polyfit(x, np.log(np.abs(z)), 1)[0]
    re_k = -np.polyfit(x, np.unwrap(np.angle(z)), 1)[0]
    k = _lossy_k(w, dx, dt, eps, mu, sigma)
    # impedance: H^{n-1/2}_{i+1/2} = Re(z_i e^{-i w dt/2} e^{-i k dx/2} B/A)
    ratio = -(dt / mu) * np.sin(k * dx / 2) / (dx * math.sin(w * dt / 2))
    h_pred = np.real(z * np.exp(-0.5j * w * dt) * np.exp(-0.5j * k * dx) * ratio)
    h_err = np.max(np.abs(out["h"][i] - h_pred)) / np.max(np.abs(h_pred))
    return re_k + 1j * im_k, k, h_err


@pytest.mark.parametrize("eps_r,mu_r,sigma", [
    (1.0, 1.0, 2.0e3),
    (2.25, 1.0, 3.0e3),
    (1.0, 2.25, 0.0),
    (2.25, 1.0, 0.0),
    (1.5, 1.8, 1.0e3),
])
def test_cw_wave_follows_the_lossy_yee_dispersion(orc, eps_r, mu_r, sigma):
    """Phase advance, attenuation and E/H ratio of a CW wave in a host medium
    match the semi-implicit lossy Yee dispersion relation.  A conductivity
    term with half its weight, or eps_r and mu_r exchanged, fails."""
    check_cw_dispersion(orc, eps_r, mu_r, sigma)


def check_cw_dispersion(orc, eps_r, mu_r, sigma):
    k_meas, k, h_err = _cw_fit(orc, eps_r, mu_r, sigma)
    assert abs(k_meas.real - k.real) < 1e-6 * abs(k.real)
    if sigma > 0:
        assert k.imag < 0
        assert abs(k_meas.imag - k.imag) < 2e-5 * abs(k.imag)
        # the residual H error is the static H a conductor keeps from the
        # switch-on (its zero-frequency part)
        assert h_err < 2e-4
    else:
        assert abs(k_meas.imag) < 1e-8 * abs(k.real)
        assert h_err < 1e-6


@pytest.mark.parametrize("eps_r,mu_r", [(2.25, 1.0), (1.0, 2.25), (4.0, 0.5)])
def test_magic_time_step_in_a_host_medium(orc, eps_r, mu_r):
    """c_h dt = dx in a host with c_h = 1/sqrt(eps mu): E^n_i = a s[n - i]
    exactly (the Mur coefficient vanishes, so the probe sees s[n - (nx-1)]),
    and H^{n-1/2}_{i+1/2} = -(a / Z) s[n - 1 - i] with Z = sqrt(mu / eps)."""
    check_magic_step_in_host(orc, eps_r, mu_r)


def check_magic_step_in_host(orc, eps_r, mu_r):
    c = orc.constants()
    eps, mu = c["eps0"] * eps_r, c["mu0"] * mu_r
    nx, nt, dx = 60, 150, 1e-7
    dt = dx * math.sqrt(eps * mu)
    rng = np.random.default_rng(7)
    s = rng.normal(size=nt + 1)
    a = 1.7
    med = W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0)
    grid = W.Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=1, med_end=1, eps_r=eps_r, mu_r=mu_r)
    out = orc.run(W.Problem("host", med, grid, W.Source(s, a)), snap_every=nt)
    i = np.arange(nx - 1)
    want = np.where(i <= nt, a * s[np.clip(nt - i, 0, None)], 0.0)
    assert np.max(np.abs(out["e_snap"][0][: nx - 1] - want)) < 1e-12 * a * np.abs(s).max()
    k = np.arange(nt + 1) - (nx - 1)
    want_p = np.where(k >= 0, a * s[np.clip(k, 0, None)], 0.0)
    assert np.max(np.abs(out["probe"] - want_p)) < 1e-12 * a * np.abs(s).max()
    z = math.sqrt(mu / eps)
    j = np.arange(nx - 1)
    want_h = -(a / z) * np.where(nt - 1 - j >= 0, s[np.clip(nt - 1 - j, 0, None)], 0.0)
    assert np.max(np.abs(out["h"] - want_h)) < 1e-12 * (a / z) * np.abs(s).max()


def test_host_parameters_change_the_coupled_run(orc):
    """The host media used by the GPU parity cases change the oracle's
    coupled run far beyond every parity tolerance (so those cases do test
    the host parameters)."""
    def prob(sigma, eps_r, mu_r):
        p = W.random_problem(3, 12, nx=203, nt=360)
        p.grid.sigma, p.grid.eps_r, p.grid.mu_r = sigma, eps_r, mu_r
        return p
    vac = orc.run(prob(0.0, 1.0, 1.0), snap_every=40)
    for host in [(2.0e3, 1.0, 1.0), (0.0, 2.25, 1.0), (0.0, 1.0, 2.25), (1.0e3, 1.5, 1.8)]:
        ref = orc.run(prob(*host), snap_every=40)
        d = np.max(np.abs(ref["e_snap"] - vac["e_snap"])) / np.max(np.abs(vac["e_snap"]))
        assert d > 1e-2, host
