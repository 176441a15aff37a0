"""Seeded synthetic inputs for the Maxwell-Liouville-von Neumann solver.

This module only *describes* problems: the quantum medium (level energies,
dipole operator, relaxation channels, initial density matrix, particle
density), the 1-D grid and the sampled source pulse.  It contains none of the
method's arithmetic (no generators, no Bloch vectors, no exponentials, no
field updates), so that both the GPU path and the independent FP64 checker
can consume exactly the same inputs.

Physical set-up follows the two-level and three-level test systems of the
paper (Sec. 5.1, Sec. 5.2: Hamiltonian H = H0 - mu E_z, relaxation
superoperator G, ground-state initial condition, Courant number 0.5).  The
concrete sizes are synthetic stand-ins for the paper's literature test cases,
whose pulse parameters and reference curves are not part of the paper text.

Units: SI throughout (J, C m, s, m, V/m, 1/m^3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# CODATA 2018 exact / recommended values (used here only to size pulses and
# grids; each solver carries its own copy of the constants it computes with).
HBAR = 1.054571817e-34
C0 = 299792458.0
E_CHARGE = 1.602176634e-19
H_PLANCK = 6.62607015e-34
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6


@dataclasses.dataclass
class Medium:
    """An N-level quantum medium (paper Sec. 2, Eq. liouville).

    h0        : (N, N) complex Hermitian, field-free Hamiltonian [J]
    dipole    : (N, N) complex Hermitian dipole operator mu [C m]; the
                interaction Hamiltonian is -mu E_z
    jumps     : list of (N, N) complex Lindblad operators L_k (unit norm
                convention: G(rho) += rate_k (L rho L^+ - {L^+ L, rho}/2))
    jump_rates: rates of the Lindblad channels [1/s]
    dephasing : pure-dephasing rate applied to every off-diagonal element
    relax_superop: optional (N^2, N^2) complex matrix acting on the
                row-major vectorisation of rho, added to G
    rho0      : (N, N) complex initial density matrix
    density   : particle density N_a [1/m^3]
    """

    h0: np.ndarray
    dipole: np.ndarray
    rho0: np.ndarray
    density: float
    jumps: List[np.ndarray] = dataclasses.field(default_factory=list)
    jump_rates: List[float] = dataclasses.field(default_factory=list)
    dephasing: float = 0.0
    relax_superop: Optional[np.ndarray] = None

    @property
    def n_levels(self) -> int:
        return int(self.h0.shape[0])


@dataclasses.dataclass
class Grid:
    """1-D Yee grid (paper Sec. 4, Fig. 1).

    E_z lives on cells 0..nx-1 (integer time steps), H_y on the nx-1 faces
    between them (half-integer steps).  The medium occupies cells
    [med_begin, med_end), strictly inside the domain.  Cell 0 carries the
    hard source, cell nx-1 a first-order Mur absorbing boundary and the
    probe.
    """

    nx: int
    nt: int
    dx: float
    dt: float
    med_begin: int
    med_end: int
    eps_r: float = 1.0
    mu_r: float = 1.0
    sigma: float = 0.0

    @property
    def n_med(self) -> int:
        return self.med_end - self.med_begin


@dataclasses.dataclass
class Source:
    """Hard source: E_z(cell 0, step n) = amplitude * samples[n], n = 0..nt."""

    samples: np.ndarray
    amplitude: float


@dataclasses.dataclass
class Problem:
    name: str
    medium: Medium
    grid: Grid
    source: Source


# ---------------------------------------------------------------------------
# building blocks


def ladder_medium(energies, dipoles, density, decay=0.0, dephasing=0.0):
    """Ladder system: diagonal H0, real nearest-neighbour dipoles, downward
    Lindblad decay |a><a+1| at one shared rate, ground-state start."""
    n = len(energies)
    h0 = np.diag(np.asarray(energies, dtype=np.complex128))
    mu = np.zeros((n, n), dtype=np.complex128)
    for a, m in enumerate(dipoles):
        mu[a, a + 1] = m
        mu[a + 1, a] = m
    jumps, rates = [], []
    if decay > 0.0:
        for a in range(n - 1):
            L = np.zeros((n, n), dtype=np.complex128)
            L[a, a + 1] = 1.0
            jumps.append(L)
            rates.append(decay)
    rho0 = np.zeros((n, n), dtype=np.complex128)
    rho0[0, 0] = 1.0
    return Medium(h0=h0, dipole=mu, rho0=rho0, density=density, jumps=jumps,
                  jump_rates=rates, dephasing=dephasing)


def sech_pulse(nt, dt, omega, tau, t0):
    t = np.arange(nt + 1, dtype=np.float64) * dt
    return (1.0 / np.cosh((t - t0) / tau)) * np.sin(omega * (t - t0))


def gauss_pulse(nt, dt, omega, sigma_t, t0):
    t = np.arange(nt + 1, dtype=np.float64) * dt
    return np.exp(-0.5 * ((t - t0) / sigma_t) ** 2) * np.sin(omega * (t - t0))


def moving_pulse(nx, dx, dt, x0, sigma_x, omega, amplitude, eps_r=1.0, mu_r=1.0):
    """Initial fields of a Gaussian-envelope pulse moving towards larger x on
    a periodic grid of nx cells: E at x_i = i dx and time 0, H at
    x_i + dx/2 and time -dt/2, from the vacuum relation H = -sqrt(eps/mu) E
    of such a wave (the fields of a pulse in the staggered leapfrog, whose
    own dispersion differs from c by O((omega dt)^2)).  x0 is the centre,
    sigma_x the envelope's standard deviation, omega the carrier frequency.
    Returns (E, H), two float64 arrays of nx values."""
    eps, mu = EPS0 * eps_r, MU0 * mu_r
    c = 1.0 / math.sqrt(eps * mu)
    L = nx * dx

    def field(x):
        u = (x - x0 + 0.5 * L) % L - 0.5 * L  # periodic distance from the centre
        return amplitude * np.exp(-0.5 * (u / sigma_x) ** 2) * np.sin(omega / c * u)

    x = np.arange(nx, dtype=np.float64) * dx
    e = field(x)
    h = -math.sqrt(eps / mu) * field(x + 0.5 * dx + 0.5 * c * dt)
    return e, h


def cw_wave(nt, dt, omega):
    t = np.arange(nt + 1, dtype=np.float64) * dt
    return np.sin(omega * t)


# reference optical frequency of the synthetic two- and three-level cases
OMEGA0 = 2.0 * math.pi * 2e14
LAMBDA0 = 2.0 * math.pi * C0 / OMEGA0
DX0 = LAMBDA0 / 40.0
DT0 = 0.5 * DX0 / C0          # Courant number 0.5


def two_level(nx=2000, nt=10000, name="two_level_2pi_sech"):
    """N=2 self-induced-transparency set-up: ground state, no relaxation,
    medium in the central half, 2-pi sech pulse (100 fs envelope FWHM)."""
    mu12 = 1e-29
    med = ladder_medium([-0.5 * HBAR * OMEGA0, 0.5 * HBAR * OMEGA0], [mu12],
                        density=1e24)
    tau = 100e-15 / (2.0 * math.acosh(2.0))
    e0 = 2.0 * HBAR / (mu12 * tau)          # area (mu/hbar) E0 pi tau = 2 pi
    grid = Grid(nx=nx, nt=nt, dx=DX0, dt=DT0, med_begin=nx // 4,
                med_end=nx // 4 + nx // 2)
    src = Source(samples=sech_pulse(nt, DT0, OMEGA0, tau, 6.0 * tau), amplitude=e0)
    return Problem(name, med, grid, src)


def sit_paper(nt=None, nx=32768, medium_from=1024, tau=10e-15, name="sit_paper_grid"):
    """The paper's two-level self-induced-transparency test case (Sec. 5.1)
    on the grid it prints: 32768 cells over 150 um (4.578 nm), Courant 0.5
    (7.635e-18 s), run to 187.5 fs (24559 steps; nt overrides);
    H0 = hbar w12 diag(-1/2, 1/2) with w12 = 4 pi 1e14 /s, mu12 = 1e-29 C m,
    the printed relaxation superoperator with T1 = T2 = 1e-10 s (the garbled
    unit read as seconds), ground-state start.  The paper leaves the density,
    the medium's extent and the pulse to its reference; stand-ins: N_a = 1e24
    /m^3, the medium from cell medium_from to the last cell, a 2-pi sech pulse
    of tau = 10 fs (area (mu/hbar) E0 pi tau = 2 pi) at w12, centred at 6 tau,
    injected at cell 0."""
    w12 = 4.0 * math.pi * 1e14
    mu12 = 1e-29
    t1 = t2 = 1e-10
    med = ladder_medium([-0.5 * HBAR * w12, 0.5 * HBAR * w12], [mu12], density=1e24)
    # printed superoperator on row-major vec(rho), index 2a + b:
    # G11 = rho22/T1, G12 = -rho12/T2, G21 = -rho21/T2, G22 = -rho22/T1
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0, 3] = 1.0 / t1
    g[1, 1] = -1.0 / t2
    g[2, 2] = -1.0 / t2
    g[3, 3] = -1.0 / t1
    med.relax_superop = g
    dx = 150e-6 / 32768
    dt = 0.5 * dx / C0
    if nt is None:
        nt = int(round(187.5e-15 / dt))
    grid = Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=medium_from, med_end=nx - 1)
    e0 = 2.0 * HBAR / (mu12 * tau)
    src = Source(samples=sech_pulse(nt, dt, w12, tau, 6.0 * tau), amplitude=e0)
    return Problem(name, med, grid, src)


def song_paper(nt=None, nx=32768, medium_from=1024, tau=10e-15, area=0.5 * math.pi, name="song_paper_grid"):
    """The paper's three-level test case (Sec. 5.2) on the grid of its
    two-level case (32768 cells of 4.578 nm, Courant 0.5, 7.635e-18 s, run to
    187.5 fs; nt overrides): H0 = hbar diag(0, w2, w3) with w2 = 2.372e15 and
    w3 = 2.417e15 /s (the printed exponent is lost; 1e15 because the case runs
    on the two-level grid, made for w ~ 1.3e15 /s, and it puts the two
    transitions near 794 and 779 nm), a V system: dipole mu12 = 1.48e-29 C m
    between levels 1 and 2 and gamma mu12 (gamma = sqrt 2) between 1 and 3,
    the printed relaxation superoperator with T1 = 1e-10 s, ground-state
    start.  The paper leaves density, medium extent and pulse to its
    reference; stand-ins: N_a = 1e24 /m^3, the medium from cell medium_from to
    the last cell, a sech pulse of tau = 10 fs at the mean transition
    frequency (its spectrum covers both lines) with pulse area `area` on the
    1-2 transition, centred at 6 tau, injected at cell 0."""
    w2, w3 = 2.372e15, 2.417e15
    mu12, gamma = 1.48e-29, math.sqrt(2.0)
    t1 = 1e-10
    h0 = np.diag(np.array([0.0, HBAR * w2, HBAR * w3], dtype=np.complex128))
    mu = np.zeros((3, 3), dtype=np.complex128)
    mu[0, 1] = mu[1, 0] = mu12
    mu[0, 2] = mu[2, 0] = gamma * mu12
    rho0 = np.zeros((3, 3), dtype=np.complex128)
    rho0[0, 0] = 1.0
    med = Medium(h0=h0, dipole=mu, rho0=rho0, density=1e24)
    # printed superoperator (1/T1) x [[g/3, -r12, -r13], [-r21, g/3 - (r22 -
    # r11), -r23], [-r31, -r32, g/3 - (r33 - r11)]], g = r33 + r22 - 2 r11, on
    # the row-major vec(rho) (index 3a + b)
    g = np.zeros((9, 9), dtype=np.complex128)
    g[0, [0, 4, 8]] = [-2.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0]
    g[4, [0, 4, 8]] = [1.0 / 3.0, -2.0 / 3.0, 1.0 / 3.0]
    g[8, [0, 4, 8]] = [1.0 / 3.0, 1.0 / 3.0, -2.0 / 3.0]
    for k in (1, 2, 3, 5, 6, 7):
        g[k, k] = -1.0
    med.relax_superop = g / t1
    dx = 150e-6 / 32768
    dt = 0.5 * dx / C0
    if nt is None:
        nt = int(round(187.5e-15 / dt))
    grid = Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=medium_from, med_end=nx - 1)
    e0 = area * HBAR / (mu12 * math.pi * tau)
    src = Source(samples=sech_pulse(nt, dt, 0.5 * (w2 + w3), tau, 6.0 * tau), amplitude=e0)
    return Problem(name, med, grid, src)


def three_level(nx=20000, nt=100000, name="three_level_ladder_pi_gauss"):
    """N=3 ladder: energies hbar*omega0*{0, 1.0, 2.1}, mu01=1e-29,
    mu12=0.8e-29, Lindblad decay 1e12/s, pure dephasing 5e12/s, medium fills
    cells [1, nx-1), Gaussian pi pulse with 200 fs envelope FWHM at omega0."""
    mu01 = 1e-29
    med = ladder_medium([0.0, HBAR * OMEGA0, 2.1 * HBAR * OMEGA0], [mu01, 0.8e-29],
                        density=1e24, decay=1e12, dephasing=5e12)
    sig = 200e-15 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    e0 = math.pi * HBAR / (mu01 * sig * math.sqrt(2.0 * math.pi))
    grid = Grid(nx=nx, nt=nt, dx=DX0, dt=DT0, med_begin=1, med_end=nx - 1)
    src = Source(samples=gauss_pulse(nt, DT0, OMEGA0, sig, 600e-15), amplitude=e0)
    return Problem(name, med, grid, src)


def cross_ladder(nx=20000, nt=20000, name="three_level_cross_polarised_ladder"):
    """The three-level ladder of three_level() with its two transitions
    coupled to different field components: mu01 (1e-29) to E_z and mu12
    (0.8e-29) to E_y (dipoles that do not commute); the pi pulse of
    three_level() drives E_z, the same waveform at 0.6 of its amplitude E_y.
    Returns (problem, dipole_y, amplitude_y) for the two-component solver."""
    p = three_level(nx=nx, nt=nt, name=name)
    h0 = np.real(np.diag(p.medium.h0))
    p.medium = ladder_medium(list(h0), [1e-29, 0.0], density=1e24, decay=1e12, dephasing=5e12)
    muy = np.zeros((3, 3), dtype=np.complex128)
    muy[1, 2] = muy[2, 1] = 0.8e-29
    return p, muy, 0.6 * p.source.amplitude


# A spectral grid resolves a wave with far fewer cells than the Yee grid.
DX_PSTD = LAMBDA0 / 8.0
DT_PSTD = 0.5 * DX_PSTD / C0  # Courant number 0.5 (PSTD leapfrog limit ~2/pi)


def pstd_three_level(nx=2048, nt=8192, name="pstd_three_level_ring"):
    """The three-level ladder medium of three_level() on a periodic grid for
    the pseudo-spectral solver: nx cells of lambda0/8 (a ring nx/8
    wavelengths long), the medium in cells [nx/4, 3nx/4), a Gaussian pi pulse
    of 50 fs envelope FWHM as the initial field, centred at nx/8 and moving
    towards the medium; nt steps at Courant number 0.5 (nt = 4 nx is two
    round trips).  Returns (problem, e_init, h_init)."""
    mu01 = 1e-29
    med = ladder_medium([0.0, HBAR * OMEGA0, 2.1 * HBAR * OMEGA0], [mu01, 0.8e-29],
                        density=1e24, decay=1e12, dephasing=5e12)
    sig = 50e-15 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    amp = math.pi * HBAR / (mu01 * sig * math.sqrt(2.0 * math.pi))
    grid = Grid(nx=nx, nt=nt, dx=DX_PSTD, dt=DT_PSTD, med_begin=nx // 4, med_end=3 * nx // 4)
    e0, h0 = moving_pulse(nx, DX_PSTD, DT_PSTD, (nx // 8) * DX_PSTD, C0 * sig, OMEGA0, amp)
    return Problem(name, med, grid, Source(np.zeros(nt + 1), 0.0)), e0, h0


def pstd_random(n, seed, nx=64, nt=200, med=None, density=1e25):
    """Short PSTD run on a ring of nx cells of lambda0/8: random N-level
    medium (random_medium with the given density) in cells [med) (default
    [nx/4, 3nx/4)), a Gaussian pulse (envelope ~8 cells, random amplitude
    near a pi pulse) centred at nx/8 moving towards it.  Returns (problem,
    e_init, h_init)."""
    rng = np.random.default_rng(seed + 11)
    medium = random_medium(n, seed, density=density)
    b, e = (nx // 4, 3 * nx // 4) if med is None else med
    grid = Grid(nx=nx, nt=nt, dx=DX_PSTD, dt=DT_PSTD, med_begin=b, med_end=e)
    sig_x = 8.0 * DX_PSTD * float(rng.uniform(0.8, 1.2))
    amp = float(rng.uniform(2e9, 6e9))
    e0, h0 = moving_pulse(nx, DX_PSTD, DT_PSTD, (nx // 8) * DX_PSTD, sig_x, OMEGA0, amp)
    return Problem(f"pstd_random_n{n}_s{seed}", medium, grid, Source(np.zeros(nt + 1), 0.0)), e0, h0


def six_level(nx=50000, nt=200000, seed=1710, name="six_level_qcl_cw"):
    """N=6 QCL-like region: energies U[0,60] meV (sorted), tridiagonal real
    dipoles U[1,5] nm*e, one Lindblad channel |a><b| per pair a<b with
    log-uniform rate in [1e11, 1e13]/s, CW drive at the level-1 -> level-2
    transition (0-based) with 1e6 V/m."""
    rng = np.random.default_rng(seed)
    ev = np.sort(rng.uniform(0.0, 60e-3, size=6)) * E_CHARGE
    dip = rng.uniform(1.0, 5.0, size=5) * 1e-9 * E_CHARGE
    rates = 10.0 ** rng.uniform(11.0, 13.0, size=15)
    med = ladder_medium(ev, dip, density=1e22)
    k = 0
    for a in range(6):
        for b in range(a + 1, 6):
            L = np.zeros((6, 6), dtype=np.complex128)
            L[a, b] = 1.0
            med.jumps.append(L)
            med.jump_rates.append(float(rates[k]))
            k += 1
    lam = H_PLANCK * C0 / (60e-3 * E_CHARGE)
    dx = lam / 40.0
    dt = 0.5 * dx / C0
    w21 = (ev[2] - ev[1]) / HBAR
    grid = Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=1, med_end=nx - 1)
    src = Source(samples=cw_wave(nt, dt, w21), amplitude=1e6)
    return Problem(name, med, grid, src)


def adjoint_case(nx=10000, nt=50000, name="three_level_adjoint"):
    """Three-level ladder medium and pulse on a shorter grid, used for the
    transmitted-energy gradient runs."""
    p = three_level(nx=nx, nt=nt, name=name)
    return p


def batched_sweep(n_inst=64, nt=20000, seed=9799, nx_range=(1000, 30000)):
    """Independent instances, half two-level and half three-level, with
    per-instance grid length, detuning, density and dipole strength."""
    rng = np.random.default_rng(seed)
    kinds = np.array([2] * (n_inst // 2) + [3] * (n_inst - n_inst // 2))
    rng.shuffle(kinds)
    out = []
    for i, kind in enumerate(kinds):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        det = rng.uniform(-0.05, 0.05)
        dens = 10.0 ** rng.uniform(23.0, 25.0)
        mu01 = 10.0 ** rng.uniform(math.log10(0.5e-29), math.log10(2e-29))
        if kind == 2:
            p = two_level(nx=nx, nt=nt, name=f"inst{i}_n2")
            e = np.diag(p.medium.h0).real * (1.0 + det)
            p.medium = ladder_medium(e, [mu01], density=dens)
        else:
            p = three_level(nx=nx, nt=nt, name=f"inst{i}_n3")
            e = np.diag(p.medium.h0).real * (1.0 + det)
            p.medium = ladder_medium(e, [mu01, 0.8 * mu01], density=dens,
                                     decay=1e12, dephasing=5e12)
        out.append(p)
    return out


# ---------------------------------------------------------------------------
# small random problems for brute-force parity


def random_hermitian(rng, n, scale):
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    return 0.5 * scale * (a + a.conj().T)


def random_density(rng, n, pure=False):
    if pure:
        psi = rng.normal(size=n) + 1j * rng.normal(size=n)
        psi /= np.linalg.norm(psi)
        return np.outer(psi, psi.conj())
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    r = a @ a.conj().T
    return r / np.trace(r).real


def random_medium(n, seed, relax=True, density=1e24, dipole_scale=1e-29,
                  complex_dipole=True):
    """Random N-level medium of the same physical scale as the ladder cases:
    level spacings around hbar*omega0, dipoles around 1e-29 C m, a few random
    Lindblad channels and a dephasing rate near 1e12/s."""
    rng = np.random.default_rng(seed)
    ev = np.sort(rng.uniform(0.0, 2.0 * n, size=n)) * HBAR * OMEGA0 * 0.5
    h0 = np.diag(ev).astype(np.complex128)
    h0 = h0 + random_hermitian(rng, n, 0.05 * HBAR * OMEGA0)
    mu = random_hermitian(rng, n, dipole_scale)
    if not complex_dipole:
        mu = mu.real.astype(np.complex128)
    med = Medium(h0=h0, dipole=mu, rho0=random_density(rng, n), density=density)
    if relax:
        for _ in range(n):
            L = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
            L /= np.linalg.norm(L)
            med.jumps.append(L)
            med.jump_rates.append(float(10.0 ** rng.uniform(11.0, 12.5)))
        med.dephasing = float(10.0 ** rng.uniform(11.0, 12.5))
    return med


def random_problem(n, seed, nx=48, nt=300, relax=True, med=None):
    """Short coupled run on a small grid with a strong resonant pulse, so that
    every cell of the medium sees a field within a few hundred steps."""
    rng = np.random.default_rng(seed + 7)
    medium = random_medium(n, seed, relax=relax)
    b, e = (1, nx - 1) if med is None else med
    grid = Grid(nx=nx, nt=nt, dx=DX0, dt=DT0, med_begin=b, med_end=e)
    sig = 20 * DT0 * float(rng.uniform(1.0, 2.0))
    src = Source(samples=gauss_pulse(nt, DT0, OMEGA0, sig, 4.0 * sig),
                 amplitude=float(rng.uniform(1e9, 3e9)))
    return Problem(f"random_n{n}_s{seed}", medium, grid, src)


def random_dipole(n, seed, scale):
    """A random N x N complex Hermitian dipole operator whose largest entry is
    `scale` [C m] (the second dipole of the two-component runs: it does not
    commute with a random first one)."""
    rng = np.random.default_rng(seed + 29)
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    h = 0.5 * (a + a.conj().T)
    return scale * h / np.max(np.abs(h))


# ---------------------------------------------------------------------------
# two-dimensional (TMz) problems: the paper's scheme is one-dimensional
# (Conclusion names the restriction); these extend the grid to x-y with the
# same medium step in every cell


@dataclasses.dataclass
class Grid2D:
    """2-D TMz Yee grid: E_z at cell centres (i, j), H_x at (i, j + 1/2),
    H_y at (i + 1/2, j); arrays row major (index j * nx + i).  Periodic in y;
    column 0 carries the hard source (amplitude * samples[n] * profile[j]),
    column nx-1 a first-order Mur boundary and the probe.  The medium fills
    the rectangle [mx0, mx1) x [my0, my1), 1 <= mx0 <= mx1 <= nx-1."""

    nx: int
    ny: int
    nt: int
    dx: float
    dy: float
    dt: float
    mx0: int
    mx1: int
    my0: int
    my1: int
    eps_r: float = 1.0
    mu_r: float = 1.0
    sigma: float = 0.0

    @property
    def n_med(self) -> int:
        return (self.mx1 - self.mx0) * (self.my1 - self.my0)


@dataclasses.dataclass
class Source2D:
    """Hard source column: E_z(0, j, step n) = amplitude * samples[n] * profile[j]."""

    samples: np.ndarray
    amplitude: float
    profile: np.ndarray


@dataclasses.dataclass
class Problem2D:
    name: str
    medium: Medium
    grid: Grid2D
    source: Source2D


def gaussian_profile(ny, centre, width):
    """Transverse beam profile exp(-((j - centre) / width)^2 / 2), periodic
    distance in j."""
    j = np.arange(ny, dtype=np.float64)
    u = (j - centre + 0.5 * ny) % ny - 0.5 * ny
    return np.exp(-0.5 * (u / width) ** 2)


def three_level_2d(nx=2048, ny=512, nt=4096, name="three_level_2d_beam"):
    """The three-level ladder medium of three_level() on a 2-D grid of
    nx x ny square cells of lambda0/40 (Courant number c dt/dx = 0.5, 0.71 of
    the 2-D stability limit), the medium on columns [nx/8, 7nx/8) over the
    full height; a Gaussian beam (profile width ny/8 cells, centred) carrying
    a Gaussian pulse of 50 fs envelope FWHM at omega0, centred at 3 FWHM,
    with the pi-pulse amplitude of the 1-D case for that width."""
    mu01 = 1e-29
    med = ladder_medium([0.0, HBAR * OMEGA0, 2.1 * HBAR * OMEGA0], [mu01, 0.8e-29],
                        density=1e24, decay=1e12, dephasing=5e12)
    sig = 50e-15 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    e0 = math.pi * HBAR / (mu01 * sig * math.sqrt(2.0 * math.pi))
    grid = Grid2D(nx=nx, ny=ny, nt=nt, dx=DX0, dy=DX0, dt=DT0, mx0=nx // 8, mx1=7 * nx // 8,
                  my0=0, my1=ny)
    src = Source2D(samples=gauss_pulse(nt, DT0, OMEGA0, sig, 150e-15), amplitude=e0,
                   profile=gaussian_profile(ny, ny / 2, ny / 8))
    return Problem2D(name, med, grid, src)


def random_problem_2d(n, seed, nx=64, ny=24, nt=200, relax=True, rect=None):
    """Short 2-D run: random medium (random_medium) on a rectangle (default
    [nx/4, 3nx/4) x [ny/4, 3ny/4)), a random transverse profile and a strong
    resonant pulse, so that the medium sees a field within the run."""
    rng = np.random.default_rng(seed + 13)
    medium = random_medium(n, seed, relax=relax)
    x0, x1, y0, y1 = rect if rect is not None else (nx // 4, 3 * nx // 4, ny // 4, 3 * ny // 4)
    grid = Grid2D(nx=nx, ny=ny, nt=nt, dx=DX0, dy=DX0 * float(rng.uniform(0.8, 1.25)), dt=DT0,
                  mx0=x0, mx1=x1, my0=y0, my1=y1)
    sig = 15 * DT0 * float(rng.uniform(1.0, 1.5))
    prof = 0.5 + rng.uniform(0.0, 1.0, size=ny)
    src = Source2D(samples=gauss_pulse(nt, DT0, OMEGA0, sig, 4.0 * sig),
                   amplitude=float(rng.uniform(1e9, 3e9)), profile=prof)
    return Problem2D(f"random2d_n{n}_s{seed}", medium, grid, src)
