"""Thin Python binding of the C ABI in ``include/mln.h`` (argument marshalling
only: every step of the time integration runs in the HIP kernels of
``libmln.so``).  PyTorch provides the device memory for the recorded outputs
and the HIP stream the library enqueues on.

The binding never falls back to another implementation: if ``libmln.so`` is
missing or a call fails, it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmln.so")

PRECISIONS = {"fp64": 0, "fp32": 1, "fp32c": 2, "bf16x6": 3, "bf16x3": 4, "fp32cf": 5, "fp32f": 6}
ROUTES = {"rotation": 0, "diag": 1, "rodrigues": 2, "pade": 3}
VARIANTS = {"auto": 0, "block": 1, "wave": 2, "quad": 3, "stream": 4, "quad_mfma": 5}
TAPE_ALL = -1  # ckpt_every: keep the whole forward tape in device memory (Solver(ckpt_every="tape"))
_VARIANT_NAMES = {1: "block", 2: "wave", 3: "quad", 4: "stream", 5: "quad_mfma"}

_dp = ctypes.POINTER(ctypes.c_double)


class MLNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mln error {code}: {msg}")
        self.code = code


class _Medium(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("h0", _dp), ("dipole", _dp),
                ("n_jump", ctypes.c_int32), ("jump", _dp), ("jump_rate", _dp),
                ("dephasing", ctypes.c_double), ("relax_superop", _dp), ("rho0", _dp),
                ("density", ctypes.c_double)]


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("nt", ctypes.c_int64), ("dx", ctypes.c_double),
                ("dt", ctypes.c_double), ("med_begin", ctypes.c_int64), ("med_end", ctypes.c_int64),
                ("eps_r", ctypes.c_double), ("mu_r", ctypes.c_double), ("sigma", ctypes.c_double)]


class _Source(ctypes.Structure):
    _fields_ = [("samples", _dp), ("n_samples", ctypes.c_int64), ("amplitude", ctypes.c_double)]


class _Record(ctypes.Structure):
    _fields_ = [("snap_every", ctypes.c_int64), ("pop_out", _dp), ("e_out", _dp),
                ("probe_out", _dp), ("out_on_device", ctypes.c_int32)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("route", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("ckpt_every", ctypes.c_int32), ("variant", ctypes.c_int32)]


class _TmzGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nt", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("mx0", ctypes.c_int64), ("mx1", ctypes.c_int64), ("my0", ctypes.c_int64),
                ("my1", ctypes.c_int64), ("eps_r", ctypes.c_double), ("mu_r", ctypes.c_double),
                ("sigma", ctypes.c_double)]


class _TmzSource(ctypes.Structure):
    _fields_ = [("samples", _dp), ("n_samples", ctypes.c_int64), ("amplitude", ctypes.c_double),
                ("profile", _dp)]


class _TmzRecord(ctypes.Structure):
    _fields_ = [("snap_every", ctypes.c_int64), ("pop_out", _dp), ("e_out", _dp), ("probe_out", _dp)]


class _Pol2Record(ctypes.Structure):
    _fields_ = [("snap_every", ctypes.c_int64), ("ez_out", _dp), ("ey_out", _dp), ("pop_out", _dp),
                ("probe_z_out", _dp), ("probe_y_out", _dp)]


class _Grads(ctypes.Structure):
    _fields_ = [(n, _dp) for n in ("d_h0", "d_dipole", "d_jump_rate", "d_dephasing", "d_amplitude",
                                   "d_density")]


class _Factors(ctypes.Structure):
    _fields_ = [(n, _dp) for n in ("gen", "M", "U", "deq", "v", "d0", "A0", "b0", "T", "theta",
                                   "R", "lam", "S", "K", "c", "w", "p0")]


# every symbol include/mln.h declares
EXPORTS = ["mln_init", "mln_step", "mln_run", "mln_use_graph", "mln_reset", "mln_current_step", "mln_get_config", "mln_configure", "mln_tune",
           "mln_configure_adjoint", "mln_get_fields", "mln_get_state", "mln_get_bloch", "mln_set_state",
           "mln_state_bytes", "mln_save_state", "mln_load_state", "mln_bloch_only", "mln_bloch_only_noalloc", "mln_free",
           "mln_strerror", "mln_last_error", "mln_setup_factors", "mln_version", "mln_grad",
           "mln_chain_rule", "mln_init_batch", "mln_batch_tune", "mln_batch_configure",
           "mln_batch_get_config", "mln_batch_use_graph", "mln_batch_step", "mln_batch_run",
           "mln_batch_reset", "mln_batch_instance", "mln_batch_free", "mln_measure_step_floor",
           "mln_measure_fma_rate", "mln_pstd_init", "mln_pstd_configure", "mln_pstd_get_config",
           "mln_pstd_step", "mln_pstd_run", "mln_pstd_reset", "mln_pstd_current_step", "mln_pstd_get_fields",
           "mln_pstd_free", "mln_tmz_init", "mln_tmz_step", "mln_tmz_run", "mln_tmz_reset",
           "mln_tmz_current_step", "mln_tmz_set_fields", "mln_tmz_get_fields", "mln_tmz_free",
           "mln_pol2_init", "mln_pol2_configure", "mln_pol2_step", "mln_pol2_run", "mln_pol2_reset", "mln_pol2_current_step",
           "mln_pol2_get_fields", "mln_pol2_free"]

_lib = None


def load():
    """Load libmln.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_1710_09799_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "mln_init": ([ctypes.POINTER(_Medium), ctypes.POINTER(_Grid), ctypes.POINTER(_Source),
                      ctypes.POINTER(_Record), ctypes.POINTER(_Options), ctypes.POINTER(P)], ctypes.c_int),
        "mln_step": ([P, ctypes.c_int64], ctypes.c_int),
        "mln_run": ([P], ctypes.c_int),
        "mln_use_graph": ([P, ctypes.c_int32], ctypes.c_int),
        "mln_reset": ([P], ctypes.c_int),
        "mln_current_step": ([P, i64p], ctypes.c_int),
        "mln_get_config": ([P, i32p, i32p, i32p], ctypes.c_int),
        "mln_configure": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "mln_tune": ([P, ctypes.c_int32, i32p, i32p, i32p], ctypes.c_int),
        "mln_configure_adjoint": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "mln_get_fields": ([P, _dp, _dp], ctypes.c_int),
        "mln_get_state": ([P, _dp, _dp, _dp], ctypes.c_int),
        "mln_get_bloch": ([P, _dp], ctypes.c_int),
        "mln_set_state": ([P, _dp, _dp, _dp], ctypes.c_int),
        "mln_state_bytes": ([P, i64p], ctypes.c_int),
        "mln_save_state": ([P, P], ctypes.c_int),
        "mln_load_state": ([P, P], ctypes.c_int),
        "mln_bloch_only": ([P, _dp, ctypes.c_int64, _dp, _dp], ctypes.c_int),
        "mln_bloch_only_noalloc": ([P, _dp, ctypes.c_int64, _dp, _dp], ctypes.c_int),
        "mln_free": ([P], None),
        "mln_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "mln_last_error": ([], ctypes.c_char_p),
        "mln_setup_factors": ([ctypes.POINTER(_Medium), ctypes.c_double, ctypes.POINTER(_Factors)],
                              ctypes.c_int),
        "mln_version": ([], ctypes.c_int),
        "mln_grad": ([P, _dp, ctypes.POINTER(_Grads)], ctypes.c_int),
        "mln_chain_rule": ([ctypes.POINTER(_Medium), ctypes.c_double, _dp, _dp, _dp, ctypes.c_double,
                            _dp, _dp, ctypes.POINTER(_Grads)], ctypes.c_int),
        "mln_init_batch": ([ctypes.c_int32, ctypes.POINTER(_Medium), ctypes.POINTER(_Grid),
                            ctypes.POINTER(_Source), ctypes.POINTER(_Record), ctypes.POINTER(_Options),
                            ctypes.POINTER(P)], ctypes.c_int),
        "mln_batch_tune": ([P, ctypes.c_int32, i32p, i32p, i32p], ctypes.c_int),
        "mln_batch_configure": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "mln_batch_get_config": ([P, i32p, i32p, i32p, i64p], ctypes.c_int),
        "mln_batch_use_graph": ([P, ctypes.c_int32], ctypes.c_int),
        "mln_batch_step": ([P, ctypes.c_int64], ctypes.c_int),
        "mln_batch_run": ([P], ctypes.c_int),
        "mln_batch_reset": ([P], ctypes.c_int),
        "mln_batch_instance": ([P, ctypes.c_int32, ctypes.POINTER(P)], ctypes.c_int),
        "mln_batch_free": ([P], None),
        "mln_measure_step_floor": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "mln_measure_fma_rate": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "mln_pstd_init": ([ctypes.c_int32, ctypes.POINTER(_Medium), ctypes.POINTER(_Grid), _dp, _dp,
                           ctypes.POINTER(_Record), P, ctypes.POINTER(P)], ctypes.c_int),
        "mln_pstd_configure": ([P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "mln_pstd_get_config": ([P, i32p, i32p, i32p], ctypes.c_int),
        "mln_pstd_step": ([P, ctypes.c_int64], ctypes.c_int),
        "mln_pstd_run": ([P], ctypes.c_int),
        "mln_pstd_reset": ([P], ctypes.c_int),
        "mln_pstd_current_step": ([P, i64p], ctypes.c_int),
        "mln_pstd_get_fields": ([P, ctypes.c_int32, _dp, _dp], ctypes.c_int),
        "mln_pstd_free": ([P], None),
        "mln_tmz_init": ([ctypes.POINTER(_Medium), ctypes.POINTER(_TmzGrid), ctypes.POINTER(_TmzSource),
                          ctypes.POINTER(_TmzRecord), ctypes.c_int32, P, ctypes.POINTER(P)], ctypes.c_int),
        "mln_tmz_step": ([P, ctypes.c_int64], ctypes.c_int),
        "mln_tmz_run": ([P], ctypes.c_int),
        "mln_tmz_reset": ([P], ctypes.c_int),
        "mln_tmz_current_step": ([P, i64p], ctypes.c_int),
        "mln_tmz_set_fields": ([P, _dp, _dp, _dp], ctypes.c_int),
        "mln_tmz_get_fields": ([P, _dp, _dp, _dp], ctypes.c_int),
        "mln_tmz_free": ([P], None),
        "mln_pol2_init": ([ctypes.POINTER(_Medium), _dp, ctypes.POINTER(_Grid), ctypes.POINTER(_Source),
                           ctypes.c_double, ctypes.POINTER(_Pol2Record), P, ctypes.POINTER(P)], ctypes.c_int),
        "mln_pol2_configure": ([P, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "mln_pol2_step": ([P, ctypes.c_int64], ctypes.c_int),
        "mln_pol2_run": ([P], ctypes.c_int),
        "mln_pol2_reset": ([P], ctypes.c_int),
        "mln_pol2_current_step": ([P, i64p], ctypes.c_int),
        "mln_pol2_get_fields": ([P, _dp, _dp, _dp, _dp], ctypes.c_int),
        "mln_pol2_free": ([P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        L = load()
        raise MLNError(rc, L.mln_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _cx(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


class _MediumArgs:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, med):
        n = med.n_levels
        self.h0 = _cx(med.h0)
        self.mu = _cx(med.dipole)
        self.rho0 = _cx(med.rho0)
        nj = len(med.jumps)
        self.jump = _cx(np.array(med.jumps).reshape(nj, n, n)) if nj else None
        self.rate = np.ascontiguousarray(np.array(med.jump_rates, dtype=np.float64)) if nj else None
        self.relax = _cx(med.relax_superop) if med.relax_superop is not None else None
        self.s = _Medium(n, _ptr(self.h0), _ptr(self.mu), nj, _ptr(self.jump), _ptr(self.rate),
                         float(med.dephasing), _ptr(self.relax), _ptr(self.rho0), float(med.density))


def setup_factors(medium, dt):
    """Host-only FP64 factors (no GPU needed).  Returns a dict of numpy arrays."""
    L = load()
    n = medium.n_levels
    D, q = n * n - 1, n * (n - 1) // 2
    out = dict(gen=np.zeros((D, n, n), complex), M=np.zeros((D, D)), U=np.zeros((D, D)),
               deq=np.zeros(D), v=np.zeros(D), d0=np.zeros(D), A0=np.zeros((D, D)), b0=np.zeros(D),
               T=np.zeros((D, D)), theta=np.zeros(q), R=np.zeros((D, D), complex),
               lam=np.zeros(D, complex), S=np.zeros((q, D, D)), K=np.zeros((D, D)), c=np.zeros(D),
               w=np.zeros(D), p0=np.zeros(1))
    ptrs = {k: (v.view(np.float64) if np.iscomplexobj(v) else v).ctypes.data_as(_dp) for k, v in out.items()}
    fs = _Factors(**ptrs)
    ma = _MediumArgs(medium)
    _check(L.mln_setup_factors(ctypes.byref(ma.s), float(dt), ctypes.byref(fs)))
    out["p0"] = float(out["p0"][0])
    return out


def _new_grads(n, n_jump):
    g = dict(d_h0=np.zeros((n, n), complex), d_dipole=np.zeros((n, n), complex),
             d_jump_rate=np.zeros(max(n_jump, 1)), d_dephasing=np.zeros(1), d_amplitude=np.zeros(1),
             d_density=np.zeros(1))
    ptrs = {k: (v.view(np.float64) if np.iscomplexobj(v) else v).ctypes.data_as(_dp) for k, v in g.items()}
    return g, _Grads(**ptrs)


def _finish_grads(g, n_jump):
    g["d_jump_rate"] = g["d_jump_rate"][:n_jump]
    for k in ("d_dephasing", "d_amplitude", "d_density"):
        g[k] = float(g[k][0])
    return g


def chain_rule(medium, dt, gA, gc, gw, gp0, gU, gd0):
    """Host-only chain rule (see mln_chain_rule in include/mln.h)."""
    L = load()
    n = medium.n_levels
    g, gs = _new_grads(n, len(medium.jumps))
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (gA, gc, gw, gU, gd0)]
    ma = _MediumArgs(medium)
    _check(L.mln_chain_rule(ctypes.byref(ma.s), float(dt), _ptr(arr[0]), _ptr(arr[1]), _ptr(arr[2]),
                            float(gp0), _ptr(arr[3]), _ptr(arr[4]), ctypes.byref(gs)))
    return _finish_grads(g, len(medium.jumps))


class Solver:
    """One coupled simulation on the GPU.

    Outputs (torch float64 tensors on the device) after run():
      probe (nt+1,), e_snap (nsnap, nx), pop (nsnap, N, n_med).
    """

    def __init__(self, problem, precision="fp64", route="rotation", snap_every=0,
                 steps_per_launch=0, tile=0, record_probe=True, record_pop=True, record_e=True,
                 ckpt_every=0, variant="auto"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Solver needs a HIP device")
        L = load()
        self.problem = problem
        med, g, src = problem.medium, problem.grid, problem.source
        n = med.n_levels
        self.nsnap = g.nt // snap_every if snap_every > 0 else 0
        dev = torch.device("cuda")
        self.probe = torch.zeros(g.nt + 1, dtype=torch.float64, device=dev) if record_probe else None
        self.e_snap = (torch.zeros((self.nsnap, g.nx), dtype=torch.float64, device=dev)
                       if (record_e and self.nsnap) else None)
        self.pop = (torch.zeros((self.nsnap, n, g.n_med), dtype=torch.float64, device=dev)
                    if (record_pop and self.nsnap) else None)
        self._ma = _MediumArgs(med)
        self._samples = np.ascontiguousarray(src.samples, dtype=np.float64)
        gs = _Grid(g.nx, g.nt, g.dx, g.dt, g.med_begin, g.med_end, g.eps_r, g.mu_r, g.sigma)
        ss = _Source(_ptr(self._samples), len(self._samples), float(src.amplitude))

        def dptr(t):
            return ctypes.cast(ctypes.c_void_p(t.data_ptr()), _dp) if t is not None else None

        rs = _Record(snap_every, dptr(self.pop), dptr(self.e_snap), dptr(self.probe), 1)
        self.stream = torch.cuda.current_stream()
        if ckpt_every == "tape":
            ckpt_every = TAPE_ALL
        os_ = _Options(PRECISIONS[precision], ROUTES[route], steps_per_launch, tile,
                       ctypes.c_void_p(self.stream.cuda_stream), ckpt_every, VARIANTS[variant])
        h = ctypes.c_void_p()
        _check(L.mln_init(ctypes.byref(self._ma.s), ctypes.byref(gs), ctypes.byref(ss),
                          ctypes.byref(rs), ctypes.byref(os_), ctypes.byref(h)))
        self._h = h
        self._L = L

    def step(self, n):
        _check(self._L.mln_step(self._h, int(n)))

    def run(self):
        _check(self._L.mln_run(self._h))
        return self.outputs()

    def reset(self):
        _check(self._L.mln_reset(self._h))

    def use_graph(self, on=True):
        """run() from step 0 replays one HIP graph of the run's launches (on,
        the default) or enqueues them one by one."""
        _check(self._L.mln_use_graph(self._h, 1 if on else 0))

    def current_step(self):
        v = ctypes.c_int64()
        _check(self._L.mln_current_step(self._h, ctypes.byref(v)))
        return v.value

    def config(self):
        """The kernel the handle runs: variant ("block", "wave" or "quad"),
        tile and steps per launch."""
        v, w, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._L.mln_get_config(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(k)))
        return {"variant": _VARIANT_NAMES[v.value], "tile": w.value, "steps_per_launch": k.value}

    def configure(self, variant="auto", tile=0, steps_per_launch=0):
        """Change the kernel configuration (at step 0)."""
        _check(self._L.mln_configure(self._h, VARIANTS[variant], int(tile), int(steps_per_launch)))

    def configure_adjoint(self, variant="auto", tile=0, steps_per_launch=0):
        """Tiling of grad()'s reverse kernel: "auto", "block" or "quad", cells
        per tile, steps per launch."""
        _check(self._L.mln_configure_adjoint(self._h, VARIANTS[variant], int(tile), int(steps_per_launch)))

    def tune(self, trial_steps=256):
        """Autotune the kernel configuration on this problem (at step 0); the
        handle keeps the fastest.  Returns config()."""
        v, w, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._L.mln_tune(self._h, int(trial_steps), ctypes.byref(v), ctypes.byref(w), ctypes.byref(k)))
        return self.config()

    def outputs(self):
        return dict(probe=self.probe, e_snap=self.e_snap, pop=self.pop)

    def fields(self):
        nx = self.problem.grid.nx
        E = np.zeros(nx)
        H = np.zeros(nx - 1)
        _check(self._L.mln_get_fields(self._h, _ptr(E), _ptr(H)))
        return E, H

    def state(self):
        """E (nx), H (nx - 1) and the populations (N x nmed) after the
        completed steps (mln_get_state)."""
        g, n = self.problem.grid, self.problem.medium.n_levels
        E, H = np.zeros(g.nx), np.zeros(g.nx - 1)
        pop = np.zeros((n, g.n_med))
        _check(self._L.mln_get_state(self._h, _ptr(E), _ptr(H), _ptr(pop)))
        return E, H, pop

    def bloch(self):
        """Bloch vectors (D x nmed) of every medium cell (mln_get_bloch)."""
        n = self.problem.medium.n_levels
        d = np.zeros((n * n - 1, self.problem.grid.n_med))
        _check(self._L.mln_get_bloch(self._h, _ptr(d)))
        return d

    def set_state(self, E=None, H=None, d=None):
        """Replace E (nx), H (nx - 1) and/or the Bloch vectors (D x nmed) at
        the current step (mln_set_state)."""
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (E, H, d)]
        g, n = self.problem.grid, self.problem.medium.n_levels
        for a, shape in zip(arrs, ((g.nx,), (g.nx - 1,), (n * n - 1, g.n_med))):
            if a is not None and a.shape != shape:
                raise ValueError(f"expected shape {shape}, got {a.shape}")
        _check(self._L.mln_set_state(self._h, *(_ptr(a) for a in arrs)))

    def save_state(self):
        nb = ctypes.c_int64()
        _check(self._L.mln_state_bytes(self._h, ctypes.byref(nb)))
        buf = np.zeros(nb.value, dtype=np.uint8)
        _check(self._L.mln_save_state(self._h, buf.ctypes.data_as(ctypes.c_void_p)))
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(self._L.mln_load_state(self._h, buf.ctypes.data_as(ctypes.c_void_p)))

    def bloch_only(self, efield):
        """Prescribed field efield (nt, n_med) as a torch float64 device tensor."""
        import torch
        efield = efield.contiguous()
        nt, nc = efield.shape
        n = self.problem.medium.n_levels
        pop = torch.zeros((nt, n, nc), dtype=torch.float64, device=efield.device)
        dp = torch.zeros((nt, nc), dtype=torch.float64, device=efield.device)
        cast = lambda t: ctypes.cast(ctypes.c_void_p(t.data_ptr()), _dp)
        _check(self._L.mln_bloch_only(self._h, cast(efield), nt, cast(pop), cast(dp)))
        return dict(pop=pop, dp=dp)

    def bloch_only_noalloc(self, efield, pop=None, dp=None):
        """mln_bloch_only_noalloc: as bloch_only, writing into caller-owned
        device tensors pop (nt, N, n_med) and dp (nt, n_med) (float64; either
        may be None) with no device allocation inside the library."""
        import torch
        efield = efield.contiguous()
        nt = efield.shape[0]
        n, nc = self.problem.medium.n_levels, self.problem.grid.n_med
        for t, shape in ((efield, (nt, nc)), (pop, (nt, n, nc)), (dp, (nt, nc))):
            if t is None:
                continue
            if tuple(t.shape) != shape or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"expected a contiguous float64 device tensor of shape {shape}")
        cast = lambda t: ctypes.cast(ctypes.c_void_p(t.data_ptr()), _dp) if t is not None else None
        _check(self._L.mln_bloch_only_noalloc(self._h, cast(efield), nt, cast(pop), cast(dp)))
        return dict(pop=pop, dp=dp)

    def grad(self, dJ_dprobe):
        """Adjoint pass (needs ckpt_every > 0 and a completed run()).  dJ_dprobe:
        host array of nt+1 values.  Returns the gradient dict of mln_grads."""
        med = self.problem.medium
        g, gs = _new_grads(med.n_levels, len(med.jumps))
        gp = np.ascontiguousarray(np.asarray(dJ_dprobe, dtype=np.float64))
        if gp.shape != (self.problem.grid.nt + 1,):
            raise ValueError("dJ_dprobe must have nt+1 entries")
        _check(self._L.mln_grad(self._h, _ptr(gp), ctypes.byref(gs)))
        return _finish_grads(g, len(med.jumps))

    def close(self):
        if getattr(self, "_h", None):
            self._L.mln_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dptr(t):
    return ctypes.cast(ctypes.c_void_p(t.data_ptr()), _dp) if t is not None else None


class Batch:
    """Many independent problems (N = 2 or 3, equal dt and nt) advanced in
    lockstep by one launch per chunk of time steps (mln_init_batch).

    outputs(i) gives problem i's recordings (torch float64 device tensors), as
    Solver.outputs() does.
    """

    def __init__(self, problems, precision="fp32c", snap_every=0, steps_per_launch=0, tile=0,
                 record_probe=True, record_pop=True, record_e=True, graph=True, variant="auto"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Batch needs a HIP device")
        L = load()
        self._L = L
        self.problems = list(problems)
        n = len(self.problems)
        dev = torch.device("cuda")
        self._keep = []
        meds = (_Medium * n)()
        grids = (_Grid * n)()
        srcs = (_Source * n)()
        recs = (_Record * n)()
        self._out = []
        for i, p in enumerate(self.problems):
            g = p.grid
            nsnap = g.nt // snap_every if snap_every > 0 else 0
            o = dict(probe=torch.zeros(g.nt + 1, dtype=torch.float64, device=dev) if record_probe else None,
                     e_snap=(torch.zeros((nsnap, g.nx), dtype=torch.float64, device=dev)
                             if (record_e and nsnap) else None),
                     pop=(torch.zeros((nsnap, p.medium.n_levels, g.n_med), dtype=torch.float64, device=dev)
                          if (record_pop and nsnap) else None))
            self._out.append(o)
            ma = _MediumArgs(p.medium)
            smp = np.ascontiguousarray(p.source.samples, dtype=np.float64)
            self._keep += [ma, smp]
            meds[i] = ma.s
            grids[i] = _Grid(g.nx, g.nt, g.dx, g.dt, g.med_begin, g.med_end, g.eps_r, g.mu_r, g.sigma)
            srcs[i] = _Source(_ptr(smp), len(smp), float(p.source.amplitude))
            recs[i] = _Record(snap_every, _dptr(o["pop"]), _dptr(o["e_snap"]), _dptr(o["probe"]), 1)
        self.stream = torch.cuda.current_stream()
        opt = _Options(PRECISIONS[precision], ROUTES["rotation"], steps_per_launch, tile,
                       ctypes.c_void_p(self.stream.cuda_stream), 0, VARIANTS[variant])
        h = ctypes.c_void_p()
        _check(L.mln_init_batch(n, meds, grids, srcs, recs, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h
        self.use_graph(graph)

    def tune(self, trial_steps=256):
        """Autotune (kernel variant, tile, steps per launch); returns them."""
        v, w, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._L.mln_batch_tune(self._h, int(trial_steps), ctypes.byref(v), ctypes.byref(w),
                                      ctypes.byref(k)))
        return _VARIANT_NAMES[v.value], w.value, k.value

    def configure(self, variant, tile, steps_per_launch):
        _check(self._L.mln_batch_configure(self._h, VARIANTS[variant], int(tile), int(steps_per_launch)))

    def config(self):
        v, w, k, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(self._L.mln_batch_get_config(self._h, ctypes.byref(v), ctypes.byref(w), ctypes.byref(k),
                                            ctypes.byref(nb)))
        return dict(variant=_VARIANT_NAMES[v.value], tile=w.value, steps_per_launch=k.value, workgroups=nb.value)

    def use_graph(self, on):
        _check(self._L.mln_batch_use_graph(self._h, 1 if on else 0))

    def step(self, n):
        _check(self._L.mln_batch_step(self._h, int(n)))

    def run(self):
        _check(self._L.mln_batch_run(self._h))
        return self._out

    def reset(self):
        _check(self._L.mln_batch_reset(self._h))

    def outputs(self, i):
        return self._out[i]

    def close(self):
        if getattr(self, "_h", None):
            self._L.mln_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pstd:
    """Problems on a periodic grid with the pseudo-spectral field solver
    (mln_pstd_init): all share problems[0].grid and differ in medium (same
    level count) and initial fields.  e_init / h_init: E at step 0 and H at
    step -1/2, shape (nx,) for all problems or (n, nx), None for zero.  The
    problems' sources are not used (a PSTD run has none).  outputs(i) gives
    problem i's recordings as torch float64 device tensors."""

    def __init__(self, problems, e_init=None, h_init=None, snap_every=0, steps_per_launch=0, max_threads=0,
                 record_probe=True, record_pop=True, record_e=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Pstd needs a HIP device")
        L = load()
        self._L = L
        self.problems = list(problems)
        n = len(self.problems)
        g = self.problems[0].grid
        self.grid = g
        dev = torch.device("cuda")

        def rows(a):
            if a is None:
                return None
            a = np.asarray(a, dtype=np.float64)
            a = np.broadcast_to(a, (n, g.nx)) if a.ndim == 1 else a
            if a.shape != (n, g.nx):
                raise ValueError(f"initial fields need shape ({g.nx},) or ({n}, {g.nx})")
            return np.ascontiguousarray(a)

        self._e0, self._h0 = rows(e_init), rows(h_init)
        nsnap = g.nt // snap_every if snap_every > 0 else 0
        meds = (_Medium * n)()
        recs = (_Record * n)()
        self._keep = []
        self._out = []
        for i, p in enumerate(self.problems):
            o = dict(probe=torch.zeros(g.nt + 1, dtype=torch.float64, device=dev) if record_probe else None,
                     e_snap=(torch.zeros((nsnap, g.nx), dtype=torch.float64, device=dev)
                             if (record_e and nsnap) else None),
                     pop=(torch.zeros((nsnap, p.medium.n_levels, g.n_med), dtype=torch.float64, device=dev)
                          if (record_pop and nsnap) else None))
            self._out.append(o)
            ma = _MediumArgs(p.medium)
            self._keep.append(ma)
            meds[i] = ma.s
            recs[i] = _Record(snap_every, _dptr(o["pop"]), _dptr(o["e_snap"]), _dptr(o["probe"]), 1)
        grid = _Grid(g.nx, g.nt, g.dx, g.dt, g.med_begin, g.med_end, g.eps_r, g.mu_r, g.sigma)
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.mln_pstd_init(n, meds, ctypes.byref(grid), _ptr(self._e0), _ptr(self._h0), recs,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        if steps_per_launch or max_threads:
            self.configure(steps_per_launch, max_threads)

    def configure(self, steps_per_launch=0, max_threads=0):
        """Steps per launch (0 = 256) and the most threads per workgroup
        (0 = automatic, 256 or 512)."""
        _check(self._L.mln_pstd_configure(self._h, int(steps_per_launch), int(max_threads)))

    def config(self):
        t, c, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._L.mln_pstd_get_config(self._h, ctypes.byref(t), ctypes.byref(c), ctypes.byref(k)))
        return dict(threads=t.value, cells_per_thread=c.value, steps_per_launch=k.value)

    def step(self, n):
        _check(self._L.mln_pstd_step(self._h, int(n)))

    def run(self):
        _check(self._L.mln_pstd_run(self._h))
        return self._out

    def reset(self):
        _check(self._L.mln_pstd_reset(self._h))

    def current_step(self):
        s = ctypes.c_int64()
        _check(self._L.mln_pstd_current_step(self._h, ctypes.byref(s)))
        return s.value

    def fields(self, i=0):
        E = np.zeros(self.grid.nx)
        H = np.zeros(self.grid.nx)
        _check(self._L.mln_pstd_get_fields(self._h, int(i), _ptr(E), _ptr(H)))
        return E, H

    def outputs(self, i):
        return self._out[i]

    def close(self):
        if getattr(self, "_h", None):
            self._L.mln_pstd_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pol2:
    """Both transverse field components (mln_pol2_init): the problem's dipole
    couples to E_z, dipole_y (N x N Hermitian) to E_y; the source waveform
    drives E_z with the problem's amplitude and E_y with amplitude_y.  FP64,
    N = 2, 3, 4, 6.  Outputs (torch float64 device tensors) after run(): probe_z,
    probe_y (nt+1), ez_snap, ey_snap (nsnap, nx), pop (nsnap, N, n_med).
    steps_per_launch, lanes_per_cell: mln_pol2_configure (None: the library's
    defaults)."""

    def __init__(self, problem, dipole_y, amplitude_y, snap_every=0, record_probe=True, record_pop=True,
                 record_e=True, steps_per_launch=None, lanes_per_cell=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Pol2 needs a HIP device")
        L = load()
        self._L = L
        self.problem = problem
        med, g, src = problem.medium, problem.grid, problem.source
        n = med.n_levels
        nsnap = g.nt // snap_every if snap_every > 0 else 0
        dev = torch.device("cuda")
        z = lambda shape, on: torch.zeros(shape, dtype=torch.float64, device=dev) if on else None
        self.probe_z = z((g.nt + 1,), record_probe)
        self.probe_y = z((g.nt + 1,), record_probe)
        self.ez_snap = z((nsnap, g.nx), record_e and nsnap)
        self.ey_snap = z((nsnap, g.nx), record_e and nsnap)
        self.pop = z((nsnap, n, g.n_med), record_pop and nsnap)
        self._ma = _MediumArgs(med)
        self._muy = _cx(np.asarray(dipole_y, dtype=np.complex128).reshape(n, n))
        self._samples = np.ascontiguousarray(src.samples, dtype=np.float64)
        gs = _Grid(g.nx, g.nt, g.dx, g.dt, g.med_begin, g.med_end, g.eps_r, g.mu_r, g.sigma)
        ss = _Source(_ptr(self._samples), len(self._samples), float(src.amplitude))
        rs = _Pol2Record(snap_every, _dptr(self.ez_snap), _dptr(self.ey_snap), _dptr(self.pop),
                         _dptr(self.probe_z), _dptr(self.probe_y))
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.mln_pol2_init(ctypes.byref(self._ma.s), _ptr(self._muy), ctypes.byref(gs), ctypes.byref(ss),
                               float(amplitude_y), ctypes.byref(rs), ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(h)))
        self._h = h
        if steps_per_launch is not None or lanes_per_cell is not None:
            self.configure(0 if steps_per_launch is None else steps_per_launch, lanes_per_cell)

    def configure(self, steps_per_launch=0, lanes_per_cell=None):
        """mln_pol2_configure; lanes_per_cell None: the library's default for
        the level count (4 for N <= 3, 1 for N = 4, 6)."""
        if lanes_per_cell is None:
            lanes_per_cell = 4 if self.problem.medium.n_levels <= 3 else 1
        _check(self._L.mln_pol2_configure(self._h, int(steps_per_launch), int(lanes_per_cell)))

    def step(self, n):
        _check(self._L.mln_pol2_step(self._h, int(n)))

    def run(self):
        _check(self._L.mln_pol2_run(self._h))
        return self.outputs()

    def reset(self):
        _check(self._L.mln_pol2_reset(self._h))

    def current_step(self):
        s = ctypes.c_int64()
        _check(self._L.mln_pol2_current_step(self._h, ctypes.byref(s)))
        return s.value

    def outputs(self):
        return dict(probe_z=self.probe_z, probe_y=self.probe_y, ez_snap=self.ez_snap, ey_snap=self.ey_snap,
                    pop=self.pop)

    def fields(self):
        """E_z, H_y, E_y, H_z (E at the current step, H half a step earlier)."""
        g = self.problem.grid
        out = [np.zeros(g.nx), np.zeros(g.nx - 1), np.zeros(g.nx), np.zeros(g.nx - 1)]
        _check(self._L.mln_pol2_get_fields(self._h, *(_ptr(a) for a in out)))
        return tuple(out)

    def close(self):
        if getattr(self, "_h", None):
            self._L.mln_pol2_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tmz:
    """One problem on the two-dimensional TMz grid (mln_tmz_init): a
    workloads.Problem2D.  Outputs (torch float64 device tensors) after run():
    probe (nt+1, ny), e_snap (nsnap, ny, nx), pop (nsnap, N, n_med)."""

    def __init__(self, problem, precision="fp64", snap_every=0, record_probe=True, record_pop=True,
                 record_e=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Tmz needs a HIP device")
        L = load()
        self._L = L
        self.problem = problem
        med, g, src = problem.medium, problem.grid, problem.source
        n = med.n_levels
        nsnap = g.nt // snap_every if snap_every > 0 else 0
        dev = torch.device("cuda")
        self.probe = torch.zeros((g.nt + 1, g.ny), dtype=torch.float64, device=dev) if record_probe else None
        self.e_snap = (torch.zeros((nsnap, g.ny, g.nx), dtype=torch.float64, device=dev)
                       if (record_e and nsnap) else None)
        self.pop = (torch.zeros((nsnap, n, g.n_med), dtype=torch.float64, device=dev)
                    if (record_pop and nsnap) else None)
        self._ma = _MediumArgs(med)
        self._samples = np.ascontiguousarray(src.samples, dtype=np.float64)
        self._prof = np.ascontiguousarray(src.profile, dtype=np.float64)
        if self._prof.shape != (g.ny,):
            raise ValueError("the source profile needs ny values")
        gs = _TmzGrid(g.nx, g.ny, g.nt, g.dx, g.dy, g.dt, g.mx0, g.mx1, g.my0, g.my1, g.eps_r, g.mu_r,
                      g.sigma)
        ss = _TmzSource(_ptr(self._samples), len(self._samples), float(src.amplitude), _ptr(self._prof))
        rs = _TmzRecord(snap_every, _dptr(self.pop), _dptr(self.e_snap), _dptr(self.probe))
        self.stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.mln_tmz_init(ctypes.byref(self._ma.s), ctypes.byref(gs), ctypes.byref(ss), ctypes.byref(rs),
                              PRECISIONS[precision], ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h

    def step(self, n):
        _check(self._L.mln_tmz_step(self._h, int(n)))

    def run(self):
        _check(self._L.mln_tmz_run(self._h))
        return self.outputs()

    def reset(self):
        _check(self._L.mln_tmz_reset(self._h))

    def current_step(self):
        s = ctypes.c_int64()
        _check(self._L.mln_tmz_current_step(self._h, ctypes.byref(s)))
        return s.value

    def outputs(self):
        return dict(probe=self.probe, e_snap=self.e_snap, pop=self.pop)

    def set_fields(self, Ez=None, Hx=None, Hy=None):
        g = self.problem.grid
        arrs = []
        for a in (Ez, Hx, Hy):
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != (g.ny, g.nx):
                    raise ValueError(f"fields need shape ({g.ny}, {g.nx})")
            arrs.append(a)
        _check(self._L.mln_tmz_set_fields(self._h, *(_ptr(a) for a in arrs)))

    def fields(self):
        """E_z (current step), H_x and H_y (half a step earlier), (ny, nx) each."""
        g = self.problem.grid
        out = [np.zeros((g.ny, g.nx)) for _ in range(3)]
        _check(self._L.mln_tmz_get_fields(self._h, *(_ptr(a) for a in out)))
        return tuple(out)

    def close(self):
        if getattr(self, "_h", None):
            self._L.mln_tmz_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tmz_run(problem, precision="fp64", snap_every=0, ez_init=None, hx_init=None, hy_init=None, **kw):
    """Convenience: one 2-D problem run to the end (optionally from given
    initial fields); outputs as numpy arrays plus the final 'ez', 'hx', 'hy'."""
    s = Tmz(problem, precision=precision, snap_every=snap_every, **kw)
    if ez_init is not None or hx_init is not None or hy_init is not None:
        s.set_fields(ez_init, hx_init, hy_init)
    out = s.run()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["ez"], res["hx"], res["hy"] = s.fields()
    s.close()
    return res


def pstd_run(problem, e_init=None, h_init=None, snap_every=0, **kw):
    """Convenience: one PSTD problem run to the end; outputs as numpy arrays
    plus the final fields 'e' and 'h'."""
    s = Pstd([problem], e_init=e_init, h_init=h_init, snap_every=snap_every, **kw)
    out = s.run()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out[0].items()}
    res["e"], res["h"] = s.fields(0)
    s.close()
    return res


def run(problem, **kw):
    """Convenience: build, run to the end, return outputs as numpy arrays."""
    s = Solver(problem, **kw)
    out = s.run()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    s.close()
    return res


def step_floor(workgroups, threads, steps=2000, chain=0):
    """mln_measure_step_floor: microseconds per step of an LDS exchange, a
    workgroup barrier and `chain` dependent FMAs at this launch shape."""
    L = load()
    us = ctypes.c_double()
    _check(L.mln_measure_step_floor(int(workgroups), int(threads), int(steps), int(chain), ctypes.byref(us)))
    return us.value


def fma_rate(fp64=False):
    """mln_measure_fma_rate: achieved plain-FMA TFLOP/s (FP32 or FP64)."""
    L = load()
    v = ctypes.c_double()
    _check(L.mln_measure_fma_rate(1 if fp64 else 0, ctypes.byref(v)))
    return v.value
