"""GPU parity of the two-component solver (mln_pol2_*, both transverse field
components with H_I = -mu_z E_z - mu_y E_y and the interaction factor split
y half / z / y half) against the oracle's orc_run_pol2, through the C ABI.

Bars: FP64 1e-10 on E_z, E_y (snapshots and probes, relative to the largest
value) and the populations.  Cases: random media with a random second dipole
that does not commute with the first, several workgroups with a ragged last
one; edge geometries; a lossy / dielectric host; the exact reductions (no
second component: the one-component GPU run; equal dipoles and sources: the
one-component run with sqrt(2) mu and sqrt(2) s, rotated by 45 degrees);
reset and stepping in pieces; field read-back; errors; N = 4 and 6 (one
thread per cell, factors through scalar loads).  Kernels: the
blocked four-lanes-per-cell kernel at its default (automatic steps per
launch) in every case, and each kernel shape against the oracle and against
the one-step kernel
(ragged last workgroups down to a single owned cell, run lengths and
snapshot intervals that are not multiples of it).
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _np(d):
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in d.items()}


def _errs(got, ref):
    out = {}
    for comp in ("z", "y"):
        e = np.concatenate([got[f"e{comp}_snap"].ravel(), got[f"probe_{comp}"]])
        er = np.concatenate([ref[f"e{comp}_snap"].ravel(), ref[f"probe_{comp}"]])
        out[comp] = np.max(np.abs(e - er)) / max(np.max(np.abs(er)), 1e-300)
    out["pop"] = np.max(np.abs(got["pop"] - ref["pop"])) if ref["pop"].size else 0.0
    return out


def _problem(n, seed, nx=600, nt=420, med=None, host=None):
    p = W.random_problem(n, seed, nx=nx, nt=nt, med=med)
    if host is not None:
        p.grid.sigma, p.grid.eps_r, p.grid.mu_r = host
    muy = W.random_dipole(n, seed, float(np.max(np.abs(p.medium.dipole))))
    return p, muy


def _run(p, muy, amp_y, snap, steps_per_launch=None, lanes_per_cell=None):
    s = mln.Pol2(p, muy, amp_y, snap_every=snap, steps_per_launch=steps_per_launch, lanes_per_cell=lanes_per_cell)
    out = _np(s.run())
    s.close()
    return out


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (3, 7)])
def test_pol2_matches_oracle(orc, n, seed):
    p, muy = _problem(n, seed)
    amp_y = 0.8 * p.source.amplitude
    _case("pol2_random", n=n, seed=seed)
    ref = orc.run_pol2(p, muy, amp_y, snap_every=42)
    got = _run(p, muy, amp_y, 42)
    e = _errs(got, ref)
    print(f"  err_Ez={e['z']:.2e} err_Ey={e['y']:.2e} err_pop={e['pop']:.2e}", flush=True)
    assert e["z"] < 1e-10 and e["y"] < 1e-10 and e["pop"] < 1e-10
    # the second component does take part: E_y inside the medium is not free
    free = orc.run_pol2(p, np.zeros_like(muy), amp_y, snap_every=42)
    assert np.max(np.abs(ref["ey_snap"] - free["ey_snap"])) > 1e-5 * np.max(np.abs(free["ey_snap"]))


@pytest.mark.parametrize("geom", [dict(nx=300, mb=150, me=151), dict(nx=257, mb=1, me=256),
                                  dict(nx=260, mb=100, me=100), dict(nx=3, mb=1, me=2)])
def test_pol2_edge_geometries(orc, geom):
    p, muy = _problem(3, 4, nx=geom["nx"], nt=240, med=(geom["mb"], geom["me"]))
    _case("pol2_edge", **geom)
    ref = orc.run_pol2(p, muy, 0.5 * p.source.amplitude, snap_every=30)
    got = _run(p, muy, 0.5 * p.source.amplitude, 30)
    e = _errs(got, ref)
    print(f"  err_Ez={e['z']:.2e} err_Ey={e['y']:.2e} err_pop={e['pop']:.2e}", flush=True)
    assert e["z"] < 1e-10 and e["y"] < 1e-10 and e["pop"] < 1e-10


@pytest.mark.parametrize("host", [(2.0e3, 1.0, 1.0), (1.0e3, 1.5, 1.8)])
def test_pol2_host_media(orc, host):
    p, muy = _problem(3, 5, nx=400, nt=300, host=host)
    _case("pol2_host", host=host)
    ref = orc.run_pol2(p, muy, 1.2 * p.source.amplitude, snap_every=50)
    got = _run(p, muy, 1.2 * p.source.amplitude, 50)
    e = _errs(got, ref)
    print(f"  err_Ez={e['z']:.2e} err_Ey={e['y']:.2e} err_pop={e['pop']:.2e}", flush=True)
    assert e["z"] < 1e-10 and e["y"] < 1e-10 and e["pop"] < 1e-10


# nx against the cells a workgroup owns, 256 - 2 K - 1 with one lane per
# cell: 447 = 2 x 223 + 1 and 448 leave one and two cells to the last
# workgroup at K = 16; 600 with K = 64 gives four workgroups of 127 and a
# fifth of 92, 130 one of 127 and one of 3.  With four lanes 128 - 2 K - 1:
# 191 = 2 x 95 + 1 at K = 16, 160 = 2 x 79 + 2 at K = 24, 600 at K = 48
# gives nineteen of 31 and one of 11.
@pytest.mark.parametrize("k,lanes,nx,nt", [(1, 1, 600, 420), (2, 1, 600, 420), (7, 1, 509, 333),
                                           (16, 1, 447, 420), (16, 1, 448, 421), (64, 1, 600, 420),
                                           (64, 1, 130, 300), (1, 4, 300, 200), (5, 4, 509, 333),
                                           (16, 4, 191, 420), (24, 4, 160, 421), (48, 4, 600, 420)])
def test_pol2_steps_per_launch(orc, k, lanes, nx, nt):
    p, muy = _problem(3, 9, nx=nx, nt=nt, med=(3, nx - 2))
    amp_y = 0.7 * p.source.amplitude
    _case("pol2_steps_per_launch", k=k, lanes=lanes, nx=nx, nt=nt)
    ref = orc.run_pol2(p, muy, amp_y, snap_every=37)
    got = _run(p, muy, amp_y, 37, steps_per_launch=k, lanes_per_cell=lanes)
    e = _errs(got, ref)
    print(f"  err_Ez={e['z']:.2e} err_Ey={e['y']:.2e} err_pop={e['pop']:.2e}", flush=True)
    assert e["z"] < 1e-10 and e["y"] < 1e-10 and e["pop"] < 1e-10
    if k > 1 or lanes > 1:  # the one-step kernel takes the same steps per cell
        one = _run(p, muy, amp_y, 37, steps_per_launch=1, lanes_per_cell=1)
        d = _errs(got, one)
        print(f"  vs one-step kernel: {d['z']:.2e} {d['y']:.2e} {d['pop']:.2e}", flush=True)
        assert d["z"] < 1e-13 and d["y"] < 1e-13 and d["pop"] < 1e-13


# N = 4, 6: one thread per cell, the factors read with scalar loads; the
# one-step kernel, the blocked kernel at its default and at 7 steps per
# launch over several workgroups (600 cells: 241 owned per workgroup)
@pytest.mark.parametrize("n,seed", [(4, 11), (6, 12)])
@pytest.mark.parametrize("k", [1, 0, 7])
def test_pol2_four_and_six_levels(orc, n, seed, k):
    p, muy = _problem(n, seed, nx=600, nt=260, med=(2, 590))
    amp_y = 0.9 * p.source.amplitude
    _case("pol2_n46", n=n, seed=seed, k=k)
    ref = orc.run_pol2(p, muy, amp_y, snap_every=26)
    got = _run(p, muy, amp_y, 26, steps_per_launch=k)
    e = _errs(got, ref)
    print(f"  err_Ez={e['z']:.2e} err_Ey={e['y']:.2e} err_pop={e['pop']:.2e}", flush=True)
    assert e["z"] < 1e-10 and e["y"] < 1e-10 and e["pop"] < 1e-10
    free = orc.run_pol2(p, np.zeros_like(muy), amp_y, snap_every=26)
    assert np.max(np.abs(ref["ey_snap"] - free["ey_snap"])) > 1e-5 * np.max(np.abs(free["ey_snap"]))


def test_pol2_configure_between_steps(orc):
    """Changing the steps per launch mid-run (and stepping in odd pieces)
    leaves the run as it was."""
    p, muy = _problem(2, 10, nx=700, nt=310)
    amp_y = 0.9 * p.source.amplitude
    _case("pol2_configure_between_steps")
    s = mln.Pol2(p, muy, amp_y, snap_every=31)
    for k, lanes, n in ((16, 1, 5), (1, 1, 3), (12, 4, 40), (64, 1, 70), (3, 1, 11), (1, 4, 2), (48, 4, 60),
                        (0, 1, 20), (0, 4, 1000)):
        s.configure(k, lanes)
        s.step(n)
    assert s.current_step() == p.grid.nt
    got = _np(s.outputs())
    for bad in ((65, 1), (-3, 1), (-1, 4), (49, 4), (16, 2), (16, 0)):
        with pytest.raises(mln.MLNError) as e:
            s.configure(*bad)
        assert e.value.code == -1
    s.close()
    ref = orc.run_pol2(p, muy, amp_y, snap_every=31)
    e = _errs(got, ref)
    assert e["z"] < 1e-10 and e["y"] < 1e-10 and e["pop"] < 1e-10


def test_pol2_without_second_component_is_the_single_run():
    p, _ = _problem(3, 3)
    n = p.medium.n_levels
    _case("pol2_reduces_to_single")
    got = _run(p, np.zeros((n, n)), 0.0, 42)
    one = _np(mln.run(p, precision="fp64", snap_every=42))
    scale = np.max(np.abs(one["e_snap"]))
    assert np.max(np.abs(got["ez_snap"] - one["e_snap"])) < 1e-12 * scale
    assert np.max(np.abs(got["probe_z"] - one["probe"])) < 1e-12 * scale
    assert np.max(np.abs(got["pop"] - one["pop"])) < 1e-12
    assert not np.any(got["ey_snap"]) and not np.any(got["probe_y"])


def test_pol2_equal_dipoles_is_a_rotated_single_run():
    p, _ = _problem(3, 6)
    mu = np.asarray(p.medium.dipole)
    _case("pol2_equal_dipoles")
    got = _run(p, mu, p.source.amplitude, 42)
    rot = W.Problem(p.name, dataclasses.replace(p.medium, dipole=math.sqrt(2.0) * mu), p.grid,
                    W.Source(p.source.samples, math.sqrt(2.0) * p.source.amplitude))
    one = _np(mln.run(rot, precision="fp64", snap_every=42))
    scale = np.max(np.abs(one["e_snap"]))
    for comp in ("z", "y"):
        assert np.max(np.abs(math.sqrt(2.0) * got[f"e{comp}_snap"] - one["e_snap"])) < 1e-11 * scale
        assert np.max(np.abs(math.sqrt(2.0) * got[f"probe_{comp}"] - one["probe"])) < 1e-11 * scale
    assert np.max(np.abs(got["pop"] - one["pop"])) < 1e-11


def test_pol2_reset_steps_and_fields(orc):
    p, muy = _problem(2, 8, nx=300, nt=200)
    amp_y = 0.6 * p.source.amplitude
    _case("pol2_reset_steps")
    s = mln.Pol2(p, muy, amp_y, snap_every=25)
    first = _np(s.run())
    Ez, Hy, Ey, Hz = s.fields()
    s.reset()
    assert s.current_step() == 0
    s.step(77)
    s.step(1000)  # clamped to the run length
    assert s.current_step() == p.grid.nt
    second = _np(s.outputs())
    s.close()
    for k in first:
        assert np.array_equal(first[k], second[k]), k
    ref = orc.run_pol2(p, muy, amp_y, snap_every=25)
    scale = np.max(np.abs(ref["ez_snap"]))
    assert np.max(np.abs(Ez - ref["ez_snap"][-1])) < 1e-10 * scale
    assert np.max(np.abs(Ey - ref["ey_snap"][-1])) < 1e-10 * max(np.max(np.abs(ref["ey_snap"])), 1e-300)
    hs = np.max(np.abs(ref["hy"]))
    assert np.max(np.abs(Hy - ref["hy"])) < 1e-10 * hs
    assert np.max(np.abs(Hz + ref["g"])) < 1e-10 * max(np.max(np.abs(ref["g"])), 1e-300)


def test_pol2_errors():
    p, muy = _problem(3, 2, nx=100, nt=50)
    bad = muy.copy()
    bad[0, 1] += 1e-30  # not Hermitian
    with pytest.raises(mln.MLNError) as e:
        mln.Pol2(p, bad, 1.0)
    assert e.value.code == -2
    p5 = W.random_problem(5, 3, nx=100, nt=50)
    with pytest.raises(mln.MLNError) as e:
        mln.Pol2(p5, W.random_dipole(5, 3, 1e-29), 1.0)
    assert e.value.code == -8
    p4 = W.random_problem(4, 3, nx=100, nt=50)
    s4 = mln.Pol2(p4, W.random_dipole(4, 3, 1e-29), 1.0)
    with pytest.raises(mln.MLNError) as e:
        s4.configure(16, 4)  # four lanes hold the Bloch vector for N <= 3 only
    assert e.value.code == -8
    s4.close()
    p.grid.dt *= 3.0  # Courant number above one
    with pytest.raises(mln.MLNError) as e:
        mln.Pol2(p, muy, 1.0)
    assert e.value.code == -4
