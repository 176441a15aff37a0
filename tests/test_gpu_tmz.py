"""GPU parity of the two-dimensional TMz solver (mln_tmz_*) against the
oracle's 2-D run, through the C ABI: every recorded E_z snapshot, the probe
column, the populations and the final H_x, H_y.

err_E = max |E - E_oracle| / max |E_oracle| over snapshots and probe;
err_pop = max |rho_aa - rho_aa_oracle|; err_H = max |H - H_oracle| of the
final H_x, H_y relative to max |E_oracle| / Z (Z = sqrt(mu / eps), the
magnetic field of a plane wave at the peak electric field: the final H alone
can be small once the pulse has left).
Tolerances: FP64 1e-10, single precision 1e-5.
"""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32c": 1e-5, "fp32": 1e-5}


def _errs(got, ref, eps_r=1.0, mu_r=1.0):
    e = np.concatenate([got["e_snap"].ravel(), got["probe"].ravel()])
    er = np.concatenate([ref["e_snap"].ravel(), ref["probe"].ravel()])
    err_e = np.max(np.abs(e - er)) / np.max(np.abs(er))
    err_p = np.max(np.abs(got["pop"] - ref["pop"])) if ref["pop"].size else 0.0
    hs = np.max(np.abs(er)) * np.sqrt(W.EPS0 * eps_r / (W.MU0 * mu_r))
    err_h = max(np.max(np.abs(got["hx"] - ref["hx"])), np.max(np.abs(got["hy"][:, :-1] - ref["hy"][:, :-1]))) / hs
    return err_e, err_p, err_h


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module")
def refs(orc):
    cache = {}

    def get(key, problem, snap):
        if key not in cache:
            cache[key] = orc.run2d(problem, snap_every=snap)
        return cache[key]
    return get


SHAPES = [(70, 5), (131, 24), (64, 8)]


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (4, 3), (6, 4)])
@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32"])
def test_tmz_random_media(refs, n, seed, nx, ny, precision):
    """Random media with relaxation on a rectangle inside grids that span
    several workgroups with ragged last tiles in x and y."""
    p = W.random_problem_2d(n, seed, nx=nx, ny=ny, nt=240)
    _case("tmz_random", n=n, nx=nx, ny=ny, precision=precision)
    ref = refs((n, seed, nx, ny), p, 40)
    got = mln.tmz_run(p, precision=precision, snap_every=40)
    ee, ep, eh = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e} err_H={eh:.2e}", flush=True)
    tol = TOL[precision]
    assert ee < tol and ep < tol and eh < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("geom", [
    dict(nx=3, ny=6, rect=(1, 2, 0, 6)),      # one interior column: medium and Mur writer at once
    dict(nx=40, ny=1, rect=(5, 39, 0, 1)),    # one row: y wraps onto itself; medium up to nx-1
    dict(nx=50, ny=9, rect=(10, 10, 2, 7)),   # empty medium
    dict(nx=66, ny=7, rect=(1, 65, 0, 7)),    # medium over every interior cell
    dict(nx=65, ny=13, rect=(64, 64, 0, 13)),  # last column alone in its workgroup, no medium
])
def test_tmz_edge_geometries(orc, precision, geom):
    nx, ny = geom["nx"], geom["ny"]
    p = W.random_problem_2d(3, 9, nx=nx, ny=ny, nt=150, rect=geom["rect"])
    _case("tmz_edge", precision=precision, **geom)
    ref = orc.run2d(p, snap_every=30)
    got = mln.tmz_run(p, precision=precision, snap_every=30)
    ee, ep, eh = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e} err_H={eh:.2e}", flush=True)
    tol = TOL[precision]
    assert ee < tol and ep < tol and eh < tol


@pytest.mark.parametrize("host", [(2.0e3, 1.0, 1.0), (0.0, 2.25, 1.0), (1.0e3, 1.5, 1.8)])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_tmz_host_media(orc, host, precision):
    p = W.random_problem_2d(3, 5, nx=100, ny=12, nt=200)
    p.grid.sigma, p.grid.eps_r, p.grid.mu_r = host
    _case("tmz_host", host=host, precision=precision)
    ref = orc.run2d(p, snap_every=50)
    got = mln.tmz_run(p, precision=precision, snap_every=50)
    ee, ep, eh = _errs(got, ref, host[1], host[2])
    print(f"  err_E={ee:.2e} err_pop={ep:.2e} err_H={eh:.2e}", flush=True)
    tol = TOL[precision]
    assert ee < tol and ep < tol and eh < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_tmz_uniform_in_y_equals_the_1d_gpu_run(precision):
    """A y-uniform problem on the 2-D grid is the 1-D problem in every row."""
    nx, ny, nt = 150, 6, 300
    p2 = W.random_problem_2d(3, 11, nx=nx, ny=ny, nt=nt, rect=(30, 120, 0, ny))
    p2.source = W.Source2D(p2.source.samples, p2.source.amplitude, np.ones(ny))
    g = p2.grid
    p1 = W.Problem("row", p2.medium, W.Grid(nx=nx, nt=nt, dx=g.dx, dt=g.dt, med_begin=30, med_end=120),
                   W.Source(p2.source.samples, p2.source.amplitude))
    r2 = mln.tmz_run(p2, precision=precision, snap_every=50)
    r1 = mln.run(p1, precision=precision, snap_every=50, variant="block")
    scale = np.max(np.abs(r1["e_snap"]))
    tol = 1e-14 if precision == "fp64" else 1e-6
    for j in range(ny):
        assert np.max(np.abs(r2["e_snap"][:, j, :] - r1["e_snap"])) <= tol * scale
        assert np.max(np.abs(r2["probe"][:, j] - r1["probe"])) <= tol * scale
    assert np.max(np.abs(r2["hx"])) == 0.0


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32"])
def test_tmz_initial_fields_and_readback(orc, precision):
    """A beam given as initial fields (set at step 0), zero source: records
    and the final fields read back (the single-precision H is carried
    rescaled on the device) against the oracle from the same fields; a
    set/get round trip returns the fields."""
    nx, ny, nt = 200, 16, 240
    p = W.random_problem_2d(2, 21, nx=nx, ny=ny, nt=nt, rect=(90, 150, 3, 13))
    p.source = W.Source2D(np.zeros(nt + 1), 0.0, np.zeros(ny))
    g = p.grid
    e1, h1 = W.moving_pulse(nx, g.dx, g.dt, 50 * g.dx, 10 * g.dx, W.OMEGA0, 2e9)
    prof = W.gaussian_profile(ny, ny / 2, ny / 5)
    ez0, hy0 = prof[:, None] * e1[None, :], prof[:, None] * h1[None, :]
    ez0[:, 0] = 0.0
    ez0[:, -1] = 0.0
    hy0[:, -1] = 0.0
    hx0 = 1e-3 * np.roll(hy0, 1, axis=0)
    _case("tmz_initial_fields", precision=precision)
    s = mln.Tmz(p, precision=precision, snap_every=40)
    s.set_fields(ez0, hx0, hy0)
    e_b, hx_b, hy_b = s.fields()
    rt = 0.0 if precision == "fp64" else 2e-7
    assert np.max(np.abs(e_b - ez0)) <= rt * np.max(np.abs(ez0))
    assert np.max(np.abs(hy_b - hy0)) <= rt * np.max(np.abs(hy0))
    assert np.max(np.abs(hx_b - hx0)) <= rt * np.max(np.abs(hx0))
    out = {k: v.cpu().numpy() for k, v in s.run().items()}
    out["ez"], out["hx"], out["hy"] = s.fields()
    s.close()
    ref = orc.run2d(p, snap_every=40, ez_init=ez0, hx_init=hx0, hy_init=hy0)
    ee, ep, eh = _errs(out, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e} err_H={eh:.2e}", flush=True)
    tol = TOL[precision]
    assert ee < tol and ep < tol and eh < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_tmz_beam_workload_reduced(orc, precision):
    """The 2-D beam workload's physics (three-level ladder, Gaussian beam,
    50 fs pi pulse) on a 256 x 64 grid for 3000 steps: the pulse crosses
    into the medium."""
    p = W.three_level_2d(nx=256, ny=64, nt=3000)
    _case("tmz_beam_reduced", precision=precision)
    ref = orc.run2d(p, snap_every=500)
    got = mln.tmz_run(p, precision=precision, snap_every=500)
    ee, ep, eh = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e} err_H={eh:.2e}", flush=True)
    tol = TOL[precision]
    assert ee < tol and ep < tol and eh < tol
    assert np.max(ref["pop"][:, 1:]) > 1e-3  # the medium was excited


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_tmz_beam_workload_full_size(precision):
    """The full 2048 x 512 grid for all 4096 steps in the benchmark's
    configuration: populations in [0, 1] summing to one, finite fields, and
    in compensated FP32 within 1e-5 of the FP64 run (which the reduced
    workload ties to the oracle)."""
    p = W.three_level_2d()
    _case("tmz_beam_full", precision=precision)
    got = mln.tmz_run(p, precision=precision, snap_every=2048, record_e=False)
    pop = got["pop"]
    assert np.all(np.isfinite(pop)) and pop.min() > -1e-6 and pop.max() < 1 + 1e-6
    assert np.max(np.abs(pop.sum(axis=1) - 1.0)) < 1e-6
    assert np.all(np.isfinite(got["ez"]))
    assert np.max(pop[:, 1:]) > 1e-3
    if precision == "fp32c":
        ref = mln.tmz_run(p, precision="fp64", snap_every=2048, record_e=False)
        err = np.max(np.abs(got["probe"] - ref["probe"])) / np.max(np.abs(ref["probe"]))
        err_p = np.max(np.abs(got["pop"] - ref["pop"]))
        print(f"  fp32c vs fp64 full size: err_probe={err:.2e} err_pop={err_p:.2e}", flush=True)
        assert err < 1e-5 and err_p < 1e-5


def test_tmz_rejects_bad_input():
    p = W.random_problem_2d(3, 1, nx=40, ny=4, nt=10)
    p.grid.dt = 2.0 * p.grid.dx / W.C0  # beyond the 2-D Courant limit
    with pytest.raises(mln.MLNError) as e:
        mln.Tmz(p)
    assert e.value.code == -4
    p = W.random_problem_2d(3, 1, nx=40, ny=4, nt=10, rect=(0, 5, 0, 4))
    with pytest.raises(mln.MLNError) as e:
        mln.Tmz(p)
    assert e.value.code == -1
    p = W.random_problem_2d(3, 1, nx=40, ny=4, nt=10)
    with pytest.raises(mln.MLNError) as e:
        mln.Tmz(p, precision="bf16x6")
    assert e.value.code == -8
