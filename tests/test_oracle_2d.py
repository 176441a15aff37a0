"""Pins of the oracle's two-dimensional TMz run (orc_run2d), the extension of
the scheme past the one-dimensional models the paper restricts itself to
(Conclusion).  Each is a property of the discrete 2-D scheme that does not
repeat its update lines:

* a problem uniform in y is the one-dimensional problem in every row: the
  2-D run equals the (separately pinned) 1-D run row by row, and H_x stays 0;
* a single transverse Fourier mode cos(k_y y) driven at omega propagates in x
  with the wavenumber of the 2-D Yee dispersion relation
  sin^2(w dt/2)/(c dt)^2 = sin^2(k_x dx/2)/dx^2 + sin^2(k_y dy/2)/dy^2 and
  keeps its transverse shape;
* without relaxation the 2-D field energy plus N_a Tr(rho H0) is conserved
  to O(dt^2) while a beam crosses a coherent slab of finite width.
"""
import math

import numpy as np
import pytest

from paper_1710_09799_amd import workloads as W


def _as_1d(p2):
    g = p2.grid
    grid = W.Grid(nx=g.nx, nt=g.nt, dx=g.dx, dt=g.dt, med_begin=g.mx0, med_end=g.mx1,
                  eps_r=g.eps_r, mu_r=g.mu_r, sigma=g.sigma)
    return W.Problem(p2.name + "_1d", p2.medium, grid, W.Source(p2.source.samples, p2.source.amplitude))


@pytest.mark.parametrize("n,seed,host", [(2, 1, (0.0, 1.0, 1.0)), (3, 2, (1e3, 2.25, 1.0)),
                                         (4, 3, (0.0, 1.0, 1.5))])
def test_uniform_in_y_equals_the_1d_run(orc, n, seed, host):
    nx, ny, nt = 90, 7, 260
    p2 = W.random_problem_2d(n, seed, nx=nx, ny=ny, nt=nt, rect=(20, 70, 0, ny))
    p2.grid.sigma, p2.grid.eps_r, p2.grid.mu_r = host
    p2.source = W.Source2D(p2.source.samples, p2.source.amplitude, np.ones(ny))
    r2 = orc.run2d(p2, snap_every=65)
    r1 = orc.run(_as_1d(p2), snap_every=65)
    scale = np.max(np.abs(r1["e_snap"]))
    assert scale > 0.01 * p2.source.amplitude
    for j in range(ny):
        assert np.max(np.abs(r2["e_snap"][:, j, :] - r1["e_snap"])) <= 1e-14 * scale
        assert np.max(np.abs(r2["probe"][:, j] - r1["probe"])) <= 1e-14 * scale
        assert np.max(np.abs(r2["hy"][j, : nx - 1] - r1["h"])) <= 1e-14 * np.max(np.abs(r1["h"]))
    mw = 50
    pop2 = r2["pop"].reshape(r2["pop"].shape[0], n, ny, mw)
    for j in range(ny):
        assert np.max(np.abs(pop2[:, :, j, :] - r1["pop"])) <= 1e-14
    assert np.max(np.abs(r2["hx"])) == 0.0


def _mode_kx(orc, ny, m, dy_cells, nt, nx=1600):
    c = orc.constants()
    c0 = 1.0 / math.sqrt(c["eps0"] * c["mu0"])
    dx = W.DX0
    dy = dy_cells * dx
    dt = 0.5 * dx / c0
    w = W.OMEGA0
    ky = 2 * math.pi * m / (ny * dy)
    prof = np.cos(ky * np.arange(ny) * dy)
    t = np.arange(nt + 1) * dt
    t_on = 16 * math.pi / w
    ramp = np.where(t < t_on, 0.5 - 0.5 * np.cos(math.pi * t / t_on), 1.0)
    med = W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0)
    snaps = []
    for steps in (nt - 1, nt):
        grid = W.Grid2D(nx=nx, ny=ny, nt=steps, dx=dx, dy=dy, dt=dt, mx0=1, mx1=1, my0=0, my1=0)
        out = orc.run2d(W.Problem2D("mode", med, grid, W.Source2D(ramp * np.sin(w * t), 1.0, prof)),
                        snap_every=steps)
        snaps.append(out["e_snap"][0])
    e_p, e_n = snaps
    # the transverse shape is kept exactly
    assert np.max(np.abs(e_n - e_n[0][None, :] * prof[:, None])) <= 1e-12 * np.max(np.abs(e_n))
    i = np.arange(10, 200)
    z = e_n[0, i] + 1j * (e_p[0, i] - e_n[0, i] * math.cos(w * dt)) / math.sin(w * dt)
    kx_meas = -np.polyfit(i * dx, np.unwrap(np.angle(z)), 1)[0]
    rhs = (math.sin(w * dt / 2) / (c0 * dt)) ** 2 - (math.sin(ky * dy / 2) / dy) ** 2
    kx = 2.0 / dx * math.asin(dx * math.sqrt(rhs))
    return kx_meas, kx, math.sqrt(max(0.0, (w / c0) ** 2 - ky ** 2))


@pytest.mark.parametrize("ny,m,dy_cells", [(40, 1, 3.0), (80, 2, 1.5), (30, 0, 1.0)])
def test_transverse_mode_follows_the_2d_yee_dispersion(orc, ny, m, dy_cells):
    check_mode(orc, ny, m, dy_cells)


def check_mode(orc, ny, m, dy_cells):
    kx_meas, kx, kx_cont = _mode_kx(orc, ny, m, dy_cells, 3000)
    # (a guided mode near its cut-off settles slowly after the switch-on)
    assert abs(kx_meas - kx) < 5e-6 * kx
    if m > 0:
        # the transverse wavenumber matters far beyond the tolerance: the
        # 1-D (k_y = 0) wavenumber at the same omega, dt = dx / (2 c)
        w, dx = W.OMEGA0, W.DX0
        dt = 0.5 * dx / W.C0
        free = 2.0 / dx * math.asin(dx / (W.C0 * dt) * math.sin(w * dt / 2))
        assert abs(free - kx) > 1e-2 * kx
    assert abs(kx - kx_cont) < 0.02 * kx_cont  # close to the continuum value


def _beam_energy_drift(orc, courant):
    c = orc.constants()
    hb, eps, mu = c["hbar"], c["eps0"], c["mu0"]
    c0 = 1.0 / math.sqrt(eps * mu)
    dx = dy = W.LAMBDA0 / 20
    dt = courant * dx / c0
    nx, ny = 800, 64
    mx0, mx1, my0, my1 = 370, 430, 16, 48
    na, d, sig_t = 4e25, 1e-29, 6e-15
    amp = 1.5 * math.pi * hb / (d * sig_t * math.sqrt(2 * math.pi))
    nt = int(round(330 * dx / (c0 * dt)))
    med = W.ladder_medium([0.0, hb * W.OMEGA0], [d], density=na)
    e1, h1 = W.moving_pulse(nx, dx, dt, 200 * dx, c0 * sig_t, W.OMEGA0, amp)
    prof = W.gaussian_profile(ny, ny / 2, ny / 5)
    ez0 = prof[:, None] * e1[None, :]
    hy0 = prof[:, None] * h1[None, :]
    hy0[:, nx - 1] = 0.0
    hx0 = np.zeros((ny, nx))
    grid = W.Grid2D(nx=nx, ny=ny, nt=nt, dx=dx, dy=dy, dt=dt, mx0=mx0, mx1=mx1, my0=my0, my1=my1)
    out = orc.run2d(W.Problem2D("beam", med, grid, W.Source2D(np.zeros(nt + 1), 0.0, np.zeros(ny))),
                    snap_every=nt, ez_init=ez0, hx_init=hx0, hy_init=hy0)
    chx, chy = dt / (mu * dx), dt / (mu * dy)

    def energy(ez, hx, hy):
        hxp = hx - chy * (np.roll(ez, -1, axis=0) - ez)
        hyp = hy.copy()
        hyp[:, :-1] += chx * np.diff(ez, axis=1)
        return dx * dy * np.sum(0.5 * eps * ez ** 2 + 0.5 * mu * (hx * hxp + hy * hyp))

    e_end = out["e_snap"][0]
    assert np.max(np.abs(e_end[:, -60:])) < 1e-9 * amp  # nothing reached the absorbing end
    w_med = na * dx * dy * np.sum(hb * W.OMEGA0 * out["pop"][0][1])
    w0 = energy(ez0, hx0, hy0)
    w1 = energy(e_end, out["hx"], out["hy"]) + w_med
    assert w_med > 0.02 * w0
    return (w1 - w0) / w_med


@pytest.mark.slow
def test_beam_through_coherent_slab_conserves_energy_to_second_order(orc):
    check_beam_energy(orc)


def check_beam_energy(orc):
    # measured: 1.9e-3 at 0.35 of the 1-D Courant number, 5.8e-4 at half dt
    d1 = _beam_energy_drift(orc, 0.35)
    d2 = _beam_energy_drift(orc, 0.175)
    assert abs(d1) < 0.01
    assert abs(d2) < abs(d1) / 2.5


def test_2d_vacuum_energy_is_exact(orc):
    """Empty medium, initial beam, perfectly conducting source column,
    periodic y: the discrete 2-D energy holds to rounding."""
    c = orc.constants()
    eps, mu = c["eps0"], c["mu0"]
    c0 = 1.0 / math.sqrt(eps * mu)
    dx = dy = W.LAMBDA0 / 20
    dt = 0.4 * dx / c0
    nx, ny, nt = 300, 32, 200
    e1, h1 = W.moving_pulse(nx, dx, dt, 100 * dx, 12 * dx, W.OMEGA0, 1e8)
    prof = W.gaussian_profile(ny, ny / 2, ny / 6)
    ez0, hy0 = prof[:, None] * e1[None, :], prof[:, None] * h1[None, :]
    hy0[:, nx - 1] = 0.0
    hx0 = np.zeros((ny, nx))
    med = W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0)
    grid = W.Grid2D(nx=nx, ny=ny, nt=nt, dx=dx, dy=dy, dt=dt, mx0=1, mx1=1, my0=0, my1=0)
    out = orc.run2d(W.Problem2D("vac", med, grid, W.Source2D(np.zeros(nt + 1), 0.0, np.zeros(ny))),
                    snap_every=nt, ez_init=ez0, hx_init=hx0, hy_init=hy0)
    chx, chy = dt / (mu * dx), dt / (mu * dy)

    def energy(ez, hx, hy):
        hxp = hx - chy * (np.roll(ez, -1, axis=0) - ez)
        hyp = hy.copy()
        hyp[:, :-1] += chx * np.diff(ez, axis=1)
        return np.sum(0.5 * eps * ez ** 2 + 0.5 * mu * (hx * hxp + hy * hyp))

    w0 = energy(ez0, hx0, hy0)
    w1 = energy(out["e_snap"][0], out["hx"], out["hy"])
    assert np.max(np.abs(out["hx"])) > 1e-3 * np.max(np.abs(hy0))  # the beam diffracts
    assert abs(w1 - w0) < 1e-12 * w0
