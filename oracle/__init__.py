"""FP64 CPU reference solver (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps ``mln_oracle.c`` -- a plain density-matrix
integrator with generic Pade exponentials that shares no code with the GPU
library -- through ctypes.  See the header of ``mln_oracle.c`` for what it
computes and which passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mln_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libmln_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O3 -fopenmp, no host-specific ISA so the
    library also runs on other x86-64 hosts)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = bind(_LIB)
    return _lib


def bind(path):
    """Load an oracle library from ``path`` and declare its entry points (the
    tests also use it to load deliberately broken copies built on the CPU and
    check that the pins reject them)."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    L.orc_run.restype = ctypes.c_int
    L.orc_run.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp,
                          ctypes.c_double, i64, i64, ctypes.c_double, ctypes.c_double, i64, i64,
                          ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double,
                          dp, dp, i64, dp, dp, dp, dp, dp, ctypes.c_int]
    L.orc_run_pol2.restype = ctypes.c_int
    L.orc_run_pol2.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp,
                               ctypes.c_double, i64, i64, ctypes.c_double, ctypes.c_double, i64, i64,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double,
                               ctypes.c_double, dp, dp, dp, dp, i64, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
    L.orc_bloch.restype = ctypes.c_int
    L.orc_bloch.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp,
                            ctypes.c_double, i64, i64, ctypes.c_double, dp, dp, dp, dp, dp,
                            ctypes.c_int]
    L.orc_grad.restype = ctypes.c_int
    L.orc_grad.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp,
                           ctypes.c_double, i64, i64, ctypes.c_double, ctypes.c_double, i64, i64,
                           ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double,
                           dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
    L.orc_pstd_run.restype = ctypes.c_int
    L.orc_pstd_run.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp,
                               ctypes.c_double, i64, i64, ctypes.c_double, ctypes.c_double, i64, i64,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, ctypes.c_double,
                               dp, dp, i64, dp, dp, dp, dp, ctypes.c_int]
    L.orc_run2d.restype = ctypes.c_int
    L.orc_run2d.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp, dp,
                            ctypes.c_double, i64, i64, i64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, i64, i64, i64, i64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, dp, ctypes.c_double, dp, dp, dp, dp, i64, dp, dp, dp,
                            dp, dp, dp, ctypes.c_int]
    L.orc_spectral_derivative.restype = None
    L.orc_spectral_derivative.argtypes = [i64, ctypes.c_double, dp, ctypes.c_double, dp]
    L.orc_expm.restype = ctypes.c_int
    L.orc_expm.argtypes = [ctypes.c_int, dp, dp]
    L.orc_superop.restype = ctypes.c_int
    L.orc_superop.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int, dp, dp, ctypes.c_double, dp,
                              ctypes.c_double, dp, dp]
    L.orc_pade_coef.restype = ctypes.c_double
    L.orc_pade_coef.argtypes = [ctypes.c_int, ctypes.c_int]
    L.orc_min_eig.restype = ctypes.c_double
    L.orc_min_eig.argtypes = [ctypes.c_int, dp]
    L.orc_constants.restype = None
    L.orc_constants.argtypes = [dp]
    return L


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cx(a):
    """complex array -> contiguous interleaved float64 view"""
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


def constants():
    out = np.zeros(4)
    lib().orc_constants(_p(out))
    return dict(hbar=out[0], c0=out[1], eps0=out[2], mu0=out[3])


def expm(a):
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    rc = lib().orc_expm(n, _p(_cx(a)), _p(out.view(np.float64)))
    if rc:
        raise RuntimeError("oracle expm failed")
    return out


def pade_coef(q, k):
    return lib().orc_pade_coef(q, k)


def min_eig(a):
    a = np.asarray(a, dtype=np.complex128)
    return lib().orc_min_eig(a.shape[0], _p(_cx(a)))


def _medium_args(med):
    n = med.n_levels
    nj = len(med.jumps)
    jumps = _cx(np.array(med.jumps).reshape(nj, n, n)) if nj else None
    rates = np.ascontiguousarray(np.array(med.jump_rates, dtype=np.float64)) if nj else None
    relax = _cx(med.relax_superop) if med.relax_superop is not None else None
    return n, _cx(med.h0), _cx(med.dipole), nj, jumps, rates, float(med.dephasing), relax, \
        _cx(med.rho0)


def superop(med, dt):
    n, h0, mu, nj, jumps, rates, deph, relax, _ = _medium_args(med)
    S = np.zeros((n * n, n * n), dtype=np.complex128)
    E0 = np.zeros((n * n, n * n), dtype=np.complex128)
    rc = lib().orc_superop(n, _p(h0), _p(mu), nj, _p(jumps), _p(rates), deph, _p(relax), dt,
                           _p(S.view(np.float64)), _p(E0.view(np.float64)))
    if rc:
        raise RuntimeError("oracle superop failed")
    return S, E0


def run(problem, snap_every=0, nthreads=0, nt=None, e_init=None, h_init=None):
    """Coupled FDTD + density-matrix run.  e_init (nx values, E^0 including
    the source cell) and h_init (nx - 1 values, H^{-1/2} on the faces
    (i + 1/2) dx) replace the zero initial fields.  Returns dict with 'probe'
    (nt+1), 'e_snap' (nsnap, nx), 'pop' (nsnap, N, n_med), 'h' (H^{nt-1/2},
    nx - 1 values) and 'diag'."""
    med, g, src = problem.medium, problem.grid, problem.source
    nt = g.nt if nt is None else nt
    n, h0, mu, nj, jumps, rates, deph, relax, rho0 = _medium_args(med)
    nsnap = nt // snap_every if snap_every > 0 else 0
    probe = np.zeros(nt + 1)
    e_snap = np.zeros((max(nsnap, 1), g.nx))
    pop = np.zeros((max(nsnap, 1), n, max(g.n_med, 1)))
    hfin = np.zeros(g.nx - 1)
    diag = np.zeros(4)
    samples = np.ascontiguousarray(src.samples[: nt + 1], dtype=np.float64)
    ei = None if e_init is None else np.ascontiguousarray(e_init, dtype=np.float64)
    hi = None if h_init is None else np.ascontiguousarray(h_init, dtype=np.float64)
    if ei is not None and ei.shape != (g.nx,):
        raise ValueError("e_init must have nx values")
    if hi is not None and hi.shape != (g.nx - 1,):
        raise ValueError("h_init must have nx - 1 values")
    rc = lib().orc_run(n, _p(h0), _p(mu), nj, _p(jumps), _p(rates), deph, _p(relax), _p(rho0),
                       float(med.density), g.nx, nt, g.dx, g.dt, g.med_begin, g.med_end,
                       g.eps_r, g.mu_r, g.sigma, _p(samples), float(src.amplitude),
                       _p(ei), _p(hi), snap_every, _p(e_snap), _p(pop), _p(probe), _p(hfin),
                       _p(diag), nthreads)
    if rc:
        raise RuntimeError(f"oracle run failed ({rc})")
    return dict(probe=probe, e_snap=e_snap[:nsnap], pop=pop[:nsnap, :, : g.n_med], h=hfin,
                diag=dict(trace=diag[0], herm=diag[1], min_eig=diag[2], purity=diag[3]))


def run_pol2(problem, dipole_y, amplitude_y, snap_every=0, nthreads=0, nt=None, init=None):
    """Both transverse field components (orc_run_pol2): the medium's dipole
    couples to E_z, dipole_y (N x N Hermitian) to E_y; the source waveform
    drives E_z with the problem's amplitude and E_y with amplitude_y.  init:
    optional dict of initial fields 'ez', 'ey' (nx values) and 'hy', 'g'
    (nx - 1 values, g = -H_z).  Returns 'probe_z', 'probe_y' (nt+1),
    'ez_snap', 'ey_snap' (nsnap, nx), 'pop' (nsnap, N, n_med), 'hy', 'g'."""
    med, g, src = problem.medium, problem.grid, problem.source
    nt = g.nt if nt is None else nt
    n, h0, mu, nj, jumps, rates, deph, relax, rho0 = _medium_args(med)
    muy = _cx(np.asarray(dipole_y, dtype=np.complex128).reshape(n, n))
    nsnap = nt // snap_every if snap_every > 0 else 0
    probe_z, probe_y = np.zeros(nt + 1), np.zeros(nt + 1)
    ez_snap, ey_snap = np.zeros((max(nsnap, 1), g.nx)), np.zeros((max(nsnap, 1), g.nx))
    pop = np.zeros((max(nsnap, 1), n, max(g.n_med, 1)))
    hy, gf = np.zeros(g.nx - 1), np.zeros(g.nx - 1)
    samples = np.ascontiguousarray(src.samples[: nt + 1], dtype=np.float64)
    init = init or {}
    fields = {}
    for key, size in (("ez", g.nx), ("hy", g.nx - 1), ("ey", g.nx), ("g", g.nx - 1)):
        v = init.get(key)
        if v is not None:
            v = np.ascontiguousarray(v, dtype=np.float64)
            if v.shape != (size,):
                raise ValueError(f"initial field {key} must have {size} values")
        fields[key] = v
    rc = lib().orc_run_pol2(n, _p(h0), _p(mu), _p(muy), nj, _p(jumps), _p(rates), deph, _p(relax), _p(rho0),
                            float(med.density), g.nx, nt, g.dx, g.dt, g.med_begin, g.med_end,
                            g.eps_r, g.mu_r, g.sigma, _p(samples), float(src.amplitude), float(amplitude_y),
                            _p(fields["ez"]), _p(fields["hy"]), _p(fields["ey"]), _p(fields["g"]),
                            snap_every, _p(ez_snap), _p(ey_snap), _p(pop), _p(probe_z), _p(probe_y),
                            _p(hy), _p(gf), nthreads)
    if rc:
        raise RuntimeError(f"oracle two-component run failed ({rc})")
    return dict(probe_z=probe_z, probe_y=probe_y, ez_snap=ez_snap[:nsnap], ey_snap=ey_snap[:nsnap],
                pop=pop[:nsnap, :, : g.n_med], hy=hy, g=gf)


def bloch(med, efield, dt, nthreads=0):
    """Prescribed-field mode: efield[t, c] drives cell c at step t.  Returns
    'pop' (nt, N, ncell), 'dp' (nt, ncell), 'rho' (ncell, N, N), 'diag'."""
    efield = np.ascontiguousarray(np.atleast_2d(np.asarray(efield, dtype=np.float64)))
    nt, ncell = efield.shape
    n, h0, mu, nj, jumps, rates, deph, relax, rho0 = _medium_args(med)
    pop = np.zeros((nt, n, ncell))
    dp = np.zeros((nt, ncell))
    rho = np.zeros((ncell, n, n), dtype=np.complex128)
    diag = np.zeros(4)
    rc = lib().orc_bloch(n, _p(h0), _p(mu), nj, _p(jumps), _p(rates), deph, _p(relax), _p(rho0),
                         float(med.density), ncell, nt, dt, _p(efield), _p(pop), _p(dp),
                         _p(rho.view(np.float64)), _p(diag), nthreads)
    if rc:
        raise RuntimeError(f"oracle bloch failed ({rc})")
    return dict(pop=pop, dp=dp, rho=rho,
                diag=dict(trace=diag[0], herm=diag[1], min_eig=diag[2], purity=diag[3]))


def grad(problem, dJ_dprobe, nthreads=0):
    """FP64 adjoint of ``run``: gradients of J with respect to the physical
    inputs, given g[n] = dJ/dprobe[n] (n = 0..nt).  Same conventions as the
    library's mln_grads: Hermitian inputs (H0, dipole) as N x N complex arrays
    where, for a < b, d[a, b] = dJ/dRe X_ab + i dJ/dIm X_ab under the Hermitian
    perturbation of the pair (d[b, a] its conjugate) and d[a, a] = dJ/dX_aa.
    Stores the whole trajectory: for small problems only."""
    med, g, src = problem.medium, problem.grid, problem.source
    n, h0, mu, nj, jumps, rates, deph, relax, rho0 = _medium_args(med)
    gp = np.ascontiguousarray(np.asarray(dJ_dprobe, dtype=np.float64))
    if gp.shape != (g.nt + 1,):
        raise ValueError("dJ_dprobe must have nt + 1 entries")
    samples = np.ascontiguousarray(src.samples[: g.nt + 1], dtype=np.float64)
    gh = np.zeros((n, n), dtype=np.complex128)
    gm = np.zeros((n, n), dtype=np.complex128)
    gr = np.zeros(max(nj, 1))
    gd, ga, gn = np.zeros(1), np.zeros(1), np.zeros(1)
    rc = lib().orc_grad(n, _p(h0), _p(mu), nj, _p(jumps), _p(rates), deph, _p(relax), _p(rho0),
                        float(med.density), g.nx, g.nt, g.dx, g.dt, g.med_begin, g.med_end,
                        g.eps_r, g.mu_r, g.sigma, _p(samples), float(src.amplitude), _p(gp),
                        _p(gh.view(np.float64)), _p(gm.view(np.float64)), _p(gr), _p(gd), _p(ga), _p(gn),
                        nthreads)
    if rc:
        raise RuntimeError(f"oracle adjoint failed ({rc})")
    return dict(d_h0=gh, d_dipole=gm, d_jump_rate=gr[:nj], d_dephasing=float(gd[0]),
                d_amplitude=float(ga[0]), d_density=float(gn[0]))


def pstd_run(problem, snap_every=0, nthreads=0, nt=None, e_init=None, h_init=None, hard_source=False):
    """Coupled run with the pseudo-spectral field solver on a periodic grid
    (see orc_pstd_run).  e_init / h_init (nx values each; H[i] sits at
    (i + 1/2) dx) replace the zero initial fields and the initial source
    sample; hard_source=True forces cell 0 to the source as run() does.  Returns 'probe', 'e_snap',
    'pop' as run() does, and 'h' (the final H)."""
    med, g, src = problem.medium, problem.grid, problem.source
    nt = g.nt if nt is None else nt
    n, h0, mu, nj, jumps, rates, deph, relax, rho0 = _medium_args(med)
    nsnap = nt // snap_every if snap_every > 0 else 0
    probe = np.zeros(nt + 1)
    e_snap = np.zeros((max(nsnap, 1), g.nx))
    pop = np.zeros((max(nsnap, 1), n, max(g.n_med, 1)))
    hfin = np.zeros(g.nx)
    samples = np.ascontiguousarray(src.samples[: nt + 1], dtype=np.float64)
    ei = None if e_init is None else np.ascontiguousarray(e_init, dtype=np.float64)
    hi = None if h_init is None else np.ascontiguousarray(h_init, dtype=np.float64)
    rc = lib().orc_pstd_run(n, _p(h0), _p(mu), nj, _p(jumps), _p(rates), deph, _p(relax), _p(rho0),
                            float(med.density), g.nx, nt, g.dx, g.dt, g.med_begin, g.med_end,
                            g.eps_r, g.mu_r, g.sigma, _p(samples) if hard_source else None,
                            float(src.amplitude), _p(ei), _p(hi),
                            snap_every, _p(e_snap), _p(pop), _p(probe), _p(hfin), nthreads)
    if rc:
        raise RuntimeError(f"oracle pstd run failed ({rc})")
    return dict(probe=probe, e_snap=e_snap[:nsnap], pop=pop[:nsnap, :, : g.n_med], h=hfin)


def spectral_derivative(f, dx, shift):
    """d/dx of the periodic band-limited interpolant of f at x_i + shift."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    lib().orc_spectral_derivative(len(f), float(dx), _p(f), float(shift), _p(out))
    return out


def run2d(problem, snap_every=0, nthreads=0, nt=None, ez_init=None, hx_init=None, hy_init=None):
    """Coupled run on the 2-D TMz Yee grid (see orc_run2d).  Initial fields
    are (ny, nx) arrays.  Returns 'probe' (nt+1, ny), 'e_snap' (nsnap, ny,
    nx), 'pop' (nsnap, N, n_med), 'hx' and 'hy' (ny, nx: H^{nt-1/2}), 'diag'."""
    med, g, src = problem.medium, problem.grid, problem.source
    nt = g.nt if nt is None else nt
    n, h0, mu, nj, jumps, rates, deph, relax, rho0 = _medium_args(med)
    nsnap = nt // snap_every if snap_every > 0 else 0
    probe = np.zeros((nt + 1, g.ny))
    e_snap = np.zeros((max(nsnap, 1), g.ny, g.nx))
    pop = np.zeros((max(nsnap, 1), n, max(g.n_med, 1)))
    hx = np.zeros((g.ny, g.nx))
    hy = np.zeros((g.ny, g.nx))
    diag = np.zeros(4)
    samples = np.ascontiguousarray(src.samples[: nt + 1], dtype=np.float64)
    prof = np.ascontiguousarray(src.profile, dtype=np.float64)
    if prof.shape != (g.ny,):
        raise ValueError("profile must have ny values")
    inits = []
    for a in (ez_init, hx_init, hy_init):
        if a is not None:
            a = np.ascontiguousarray(a, dtype=np.float64)
            if a.shape != (g.ny, g.nx):
                raise ValueError("initial fields must be (ny, nx) arrays")
        inits.append(a)
    rc = lib().orc_run2d(n, _p(h0), _p(mu), nj, _p(jumps), _p(rates), deph, _p(relax), _p(rho0),
                         float(med.density), g.nx, g.ny, nt, g.dx, g.dy, g.dt, g.mx0, g.mx1, g.my0,
                         g.my1, g.eps_r, g.mu_r, g.sigma, _p(samples), float(src.amplitude), _p(prof),
                         _p(inits[0]), _p(inits[1]), _p(inits[2]), snap_every, _p(e_snap), _p(pop),
                         _p(probe), _p(hx), _p(hy), _p(diag), nthreads)
    if rc:
        raise RuntimeError(f"oracle 2-D run failed ({rc})")
    return dict(probe=probe, e_snap=e_snap[:nsnap], pop=pop[:nsnap, :, : g.n_med], hx=hx, hy=hy,
                diag=dict(trace=diag[0], herm=diag[1], min_eig=diag[2], purity=diag[3]))
