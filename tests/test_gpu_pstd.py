"""Pseudo-spectral (PSTD) field solver on the GPU (mln_pstd_*): element-by-
element parity with the FP64 oracle's PSTD run (direct DFT derivatives,
density-matrix medium) for N = 2, 3, 4, 6 and every cells-per-thread shape
of the one-workgroup kernel, with launch chunks that do not divide the run,
snapshots across launches, media that start and end at arbitrary cells,
batches of different media and initial fields, and the exact single-mode
vacuum solution of the leapfrog at the largest grid."""
import math

import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-10  # FP64 throughout: FFT vs direct DFT sums differ by rounding only

_REFS = {}


def _oracle_run(orc, p, se, e0, h0):
    """The oracle's run of a case, computed once for both launch shapes."""
    key = (p.name, p.grid.nx, p.grid.nt, p.grid.med_begin, p.grid.med_end, se)
    if key not in _REFS:
        _REFS[key] = orc.pstd_run(p, snap_every=se, e_init=e0, h_init=h0)
    return _REFS[key]


def _check(got, ref, h_final=None):
    # E errors relative to the largest field anywhere (the probe cell can sit
    # far from the pulse, where E is rounding noise of the pulse's size)
    scale = max(np.max(np.abs(ref["probe"])), np.max(np.abs(ref["e_snap"])))
    errs = {"probe": np.max(np.abs(got["probe"] - ref["probe"])) / scale}
    if ref["e_snap"] is not None and ref["e_snap"].size:
        errs["e_snap"] = np.max(np.abs(got["e_snap"] - ref["e_snap"])) / scale
    if ref["pop"] is not None and ref["pop"].size:
        errs["pop"] = np.max(np.abs(got["pop"] - ref["pop"]))
    if h_final is not None:
        errs["h"] = np.max(np.abs(h_final - ref["h"])) / np.max(np.abs(ref["h"]))
    print("  errors", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < TOL, (k, v)


# (N, nx, nt, steps per launch, medium range or None): nx 64..512 run one
# cell per thread, 1024 two, 2048 four, 4096 eight; on the large grids the
# medium sits under the initial pulse so that the few steps the oracle can
# afford still couple it strongly
CASES = [
    (2, 64, 200, 64, None), (3, 64, 200, 37, None), (4, 64, 120, 50, None), (6, 64, 80, 33, None),
    (2, 512, 120, 256, (40, 301)), (3, 256, 150, 41, (17, 200)),
    (2, 1024, 40, 13, (100, 250)), (3, 1024, 40, 9, (101, 233)), (6, 1024, 12, 5, (110, 150)),
    (2, 2048, 24, 7, (230, 420)), (3, 2048, 24, 10, (231, 399)), (4, 2048, 16, 6, (240, 300)),
    (2, 4096, 12, 5, (490, 700)), (3, 4096, 12, 4, (500, 611)),
]


# 512-thread workgroups build half as many cells per thread as 256
_MAX512 = {2: 4096, 3: 4096, 4: 2048, 6: 1024}


@pytest.mark.parametrize("tmax", [256, 512])
@pytest.mark.parametrize("n,nx,nt,spl,med", CASES)
def test_pstd_matches_oracle(orc, n, nx, nt, spl, med, tmax):
    if tmax == 512 and nx > _MAX512[n]:
        pytest.skip("not built for 512 threads")
    print(f"[case] pstd N={n} nx={nx} nt={nt} spl={spl} med={med} threads<={tmax}", flush=True)
    p, e0, h0 = W.pstd_random(n, 3 + n, nx=nx, nt=nt, med=med)
    se = max(1, nt // 4)
    ref = _oracle_run(orc, p, se, e0, h0)
    s = mln.Pstd([p], e_init=e0, h_init=h0, snap_every=se, steps_per_launch=spl, max_threads=tmax)
    cfg = s.config()
    assert cfg["threads"] * cfg["cells_per_thread"] == nx and cfg["threads"] == min(nx, tmax)
    out = {k: (v.cpu().numpy() if v is not None else None) for k, v in s.run()[0].items()}
    e, h = s.fields(0)
    s.close()
    _check(out, ref, h_final=h)
    assert np.array_equal(out["probe"][-1], e[-1])


def test_pstd_batch_of_media_and_fields(orc):
    """Three problems with different media and initial fields in one launch;
    each matches its own oracle run."""
    nx, nt = 256, 160
    items = [W.pstd_random(3, seed, nx=nx, nt=nt, med=(30 + 7 * seed, 180 + 5 * seed)) for seed in (1, 2, 3)]
    # one grid for all: the medium range of the first problem
    g = items[0][0].grid
    probs = [W.Problem(p.name, p.medium, g, p.source) for p, _, _ in items]
    e0 = np.stack([it[1] for it in items])
    h0 = np.stack([it[2] * (1.0 + 0.1 * i) for i, it in enumerate(items)])
    s = mln.Pstd(probs, e_init=e0, h_init=h0, snap_every=40, steps_per_launch=50)
    outs = [{k: (v.cpu().numpy() if v is not None else None) for k, v in o.items()} for o in s.run()]
    fields = [s.fields(i) for i in range(3)]
    s.close()
    for i, p in enumerate(probs):
        print(f"[case] batch instance {i}", flush=True)
        ref = orc.pstd_run(p, snap_every=40, e_init=e0[i], h_init=h0[i])
        _check(outs[i], ref, h_final=fields[i][1])


def test_pstd_reset_repeats_bitwise_and_chunking_changes_rounding_only():
    """A reset run with the same launch chunks repeats bit for bit.  Other
    chunks (steps in pieces, another steps-per-launch) agree to rounding: H
    returns to real space at the end of every launch, so the chunking only
    moves where that rounding happens."""
    p, e0, h0 = W.pstd_random(2, 9, nx=128, nt=300)
    s = mln.Pstd([p], e_init=e0, h_init=h0, snap_every=30, steps_per_launch=64)

    def grab():
        return {k: v.cpu().numpy().copy() for k, v in s.outputs(0).items()}, s.fields(0)

    s.run()
    first, f1 = grab()
    s.reset()
    assert s.current_step() == 0
    s.run()
    again, f2 = grab()
    for k in first:
        assert np.array_equal(first[k], again[k]), k
    assert np.array_equal(f1[0], f2[0]) and np.array_equal(f1[1], f2[1])
    s.reset()
    s.step(37)
    s.step(101)
    assert s.current_step() == 138
    s.configure(17, 512)
    assert s.config()["threads"] == 128
    s.run()
    pieces, f3 = grab()
    s.close()
    scale = np.max(np.abs(first["e_snap"]))
    assert np.max(np.abs(pieces["e_snap"] - first["e_snap"])) < 1e-12 * scale
    assert np.max(np.abs(pieces["probe"] - first["probe"])) < 1e-12 * scale
    assert np.max(np.abs(pieces["pop"] - first["pop"])) < 1e-12
    assert np.max(np.abs(f3[1] - f1[1])) < 1e-12 * np.max(np.abs(f1[1]))


@pytest.mark.parametrize("m", [1, 37, 1000])
def test_pstd_single_mode_exact_at_the_largest_grid(orc, m):
    """Vacuum (a medium of zero density), E = A cos(kappa x) with its exact
    leapfrog partner H: after nt steps E = A cos(kappa x - omega nt dt) with
    sin(omega dt / 2) = c kappa dt / 2, at nx = 4096 and 2000 steps."""
    c = orc.constants()
    nx, nt = 4096, 2000
    dx = W.DX_PSTD
    c0 = 1.0 / math.sqrt(c["eps0"] * c["mu0"])
    dt = 0.5 * dx / c0
    kap = 2 * math.pi * m / (nx * dx)
    w = 2.0 / dt * math.asin(c0 * kap * dt / 2.0)
    A = 2.0e9
    B = -dt * A * kap / (2.0 * c["mu0"] * math.sin(w * dt / 2.0))
    x = np.arange(nx) * dx
    e0 = A * np.cos(kap * x)
    h0 = B * np.cos(kap * (x + 0.5 * dx) + w * dt / 2.0)
    med = W.ladder_medium([0.0, 1e-19], [1e-29], density=0.0)
    p = W.Problem("vac", med, W.Grid(nx=nx, nt=nt, dx=dx, dt=dt, med_begin=1, med_end=2),
                  W.Source(np.zeros(nt + 1), 0.0))
    out = mln.pstd_run(p, e_init=e0, h_init=h0, snap_every=nt)
    want_e = A * np.cos(kap * x - w * nt * dt)
    want_h = B * np.cos(kap * (x + 0.5 * dx) - w * (nt - 0.5) * dt)
    err_e = np.max(np.abs(out["e_snap"][0] - want_e)) / A
    err_h = np.max(np.abs(out["h"] - want_h)) / abs(B)
    print(f"[case] single mode m={m}: err_E={err_e:.2e} err_H={err_h:.2e}", flush=True)
    assert err_e < 1e-9 and err_h < 1e-9
    n = np.arange(nt + 1)
    assert np.max(np.abs(out["probe"] - A * np.cos(kap * x[-1] - w * n * dt))) < 1e-9 * A


def test_pstd_bench_workload_full_size(orc):
    """The bench's ring (three-level ladder, 2048 cells, 8192 steps, default
    launch shape): its first 40 steps element by element against the oracle
    on the full ring, and over the whole run the properties that hold at any
    size (populations in [0, 1] summing to 1, finite fields and probe)."""
    p, e0, h0 = W.pstd_three_level()
    g = p.grid
    short = W.Problem(p.name, p.medium, W.Grid(nx=g.nx, nt=40, dx=g.dx, dt=g.dt, med_begin=g.med_begin,
                                              med_end=g.med_end), p.source)
    ref = orc.pstd_run(short, snap_every=10, e_init=e0, h_init=h0)
    s = mln.Pstd([short], e_init=e0, h_init=h0, snap_every=10)
    out = {k: (v.cpu().numpy() if v is not None else None) for k, v in s.run()[0].items()}
    s.close()
    print("[case] bench ring, first 40 steps", flush=True)
    _check(out, ref)
    print("[case] bench ring, full run", flush=True)
    full = mln.pstd_run(p, e_init=e0, h_init=h0, snap_every=g.nt // 4)
    pop = full["pop"]
    assert np.all(np.isfinite(full["probe"])) and np.all(np.isfinite(full["e"])) and np.all(np.isfinite(full["h"]))
    assert pop.min() > -1e-12 and pop.max() < 1 + 1e-12
    assert np.max(np.abs(pop.sum(axis=1) - 1.0)) < 1e-12
    # the pi pulse inverts the medium where it passes; the upper levels decay
    # (1 ps) over the 2.6 ps run, so the inversion shows in the early snapshots
    mins = pop[:, 0].min(axis=1)
    print("  lowest ground-state population per snapshot:", np.round(mins, 3), flush=True)
    assert mins.min() < 0.5


def test_pstd_automatic_launch_shape():
    """One problem runs 512-thread workgroups where built (N <= 4); N = 6 runs
    256; a batch of more problems than compute units on a grid of at most
    1024 cells runs 256 (two workgroups share a compute unit)."""
    import torch
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for n, nx, ninst, want in ((3, 1024, 1, 512), (2, 4096, 1, 512), (6, 512, 1, 256),
                               (3, 1024, n_cu + 1, 256), (3, 2048, n_cu + 1, 512)):
        items = [W.pstd_random(n, 1, nx=nx, nt=4) for _ in range(1)]
        p, e0, h0 = items[0]
        s = mln.Pstd([p] * ninst, e_init=e0, h_init=h0, record_pop=False, record_e=False, record_probe=False)
        got = s.config()["threads"]
        s.close()
        assert got == min(nx, want), (n, nx, ninst, got)


def test_pstd_empty_medium_matches_oracle(orc):
    """A ring with an empty medium range (med_begin == med_end) propagates the
    initial pulse as the oracle does."""
    p, e0, h0 = W.pstd_random(3, 4, nx=256, nt=120, med=(100, 100))
    ref = orc.pstd_run(p, snap_every=40, e_init=e0, h_init=h0)
    out = mln.pstd_run(p, e_init=e0, h_init=h0, snap_every=40)
    assert out["pop"] is None or out["pop"].size == 0
    ref["pop"] = None
    _check(out, ref, h_final=out["h"])
