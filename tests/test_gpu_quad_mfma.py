"""GPU parity of the four-lanes-per-cell kernel with its shared-factor
product on the matrix cores (variant "quad_mfma"), through the C ABI.

The product z <- (K - I) y'' + c of the fused half steps (Sec. 4.1) runs as
two 16x16x4 MFMA instructions per wavefront and step, so its rounding order
differs from the DPP kernel's FMA chain: the comparisons are with the FP64
oracle at the usual bars (FP64 1e-10, FP32 modes 1e-5), and between the two
kernels in FP64 (both within rounding of each other).

err_E = max |E - E_oracle| / max |E_oracle| over snapshots and probe;
err_pop = max |rho_aa - rho_aa_oracle|.
"""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32c": 1e-5, "fp32cf": 1e-5, "fp32": 1e-5, "fp32f": 1e-5}


def _errs(got, ref):
    e = np.concatenate([got["e_snap"].ravel(), got["probe"].ravel()])
    er = np.concatenate([ref["e_snap"].ravel(), ref["probe"].ravel()])
    err_e = np.max(np.abs(e - er)) / np.max(np.abs(er))
    err_p = np.max(np.abs(got["pop"] - ref["pop"])) if ref["pop"].size else 0.0
    return err_e, err_p


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module")
def refs(orc):
    cache = {}

    def get(key, problem, snap):
        if key not in cache:
            cache[key] = orc.run(problem, snap_every=snap)
        return cache[key]
    return get


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (3, 7)])
@pytest.mark.parametrize("tile,k", [(32, 8), (128, 20), (256, 63), (80, 20), (48, 11)])
@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32cf", "fp32", "fp32f"])
def test_quad_mfma_random_media(refs, n, seed, tile, k, precision):
    """Random media with complex dipoles and general Lindblad channels on 203
    cells (several tiles, ragged last tile), snapshots across launches."""
    p = W.random_problem(n, seed, nx=203, nt=360)
    _case("quad_mfma_random", n=n, seed=seed, tile=tile, k=k, precision=precision)
    ref = refs((n, seed), p, 40)
    got = mln.run(p, precision=precision, snap_every=40, variant="quad_mfma", tile=tile, steps_per_launch=k)
    ee, ep = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < TOL[precision] and ep < TOL[precision]


@pytest.mark.parametrize("host", [(2.0e3, 1.0, 1.0), (1.0e3, 1.5, 1.8)])
@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_quad_mfma_host_media(orc, host, precision):
    p = W.random_problem(3, 5, nx=203, nt=360)
    p.grid.sigma, p.grid.eps_r, p.grid.mu_r = host
    _case("quad_mfma_host", host=host, precision=precision)
    ref = orc.run(p, snap_every=40)
    got = mln.run(p, precision=precision, snap_every=40, variant="quad_mfma", tile=64, steps_per_launch=16)
    ee, ep = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < TOL[precision] and ep < TOL[precision]


@pytest.mark.parametrize("geom", [dict(nx=40, mb=1, me=39), dict(nx=300, mb=150, me=151),
                                  dict(nx=130, mb=64, me=128)])
def test_quad_mfma_edge_media(orc, geom):
    """The medium over every interior cell, a single medium cell, a medium
    ending at a tile border: the per-cell selection around the uniform
    matrix-core product."""
    p = W.random_problem(3, 4, nx=geom["nx"], nt=240)
    p.grid.med_begin, p.grid.med_end = geom["mb"], geom["me"]
    _case("quad_mfma_edge", **geom)
    ref = orc.run(p, snap_every=30)
    got = mln.run(p, precision="fp64", snap_every=30, variant="quad_mfma", tile=32, steps_per_launch=8)
    ee, ep = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < 1e-10 and ep < 1e-10


def test_quad_mfma_equals_dpp_kernel_fp64():
    """The three-level ladder on 2000 cells for 4000 steps: the matrix-core
    kernel and the DPP kernel agree to FP64 rounding."""
    p = W.three_level(nx=2000, nt=4000)
    _case("quad_mfma_vs_quad")
    a = mln.run(p, precision="fp64", snap_every=500, variant="quad_mfma", tile=128, steps_per_launch=20)
    b = mln.run(p, precision="fp64", snap_every=500, variant="quad", tile=128, steps_per_launch=20)
    ee, ep = _errs(a, b)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < 1e-12 and ep < 1e-12


@pytest.mark.slow
def test_quad_mfma_three_level_full_grid_through_pulse(orc):
    """The full 20000-cell grid in the benchmark's shape (128 cells, 20 steps
    per launch) in compensated FP32 against the oracle for 12000 steps (the pi
    pulse has entered the medium)."""
    p = W.three_level()
    p.grid.nt = 12000
    _case("quad_mfma_three_level_full")
    ref = orc.run(p, snap_every=3000)
    got = mln.run(p, precision="fp32c", snap_every=3000, variant="quad_mfma", tile=128, steps_per_launch=20)
    ee, ep = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < 1e-5 and ep < 1e-5


def test_quad_mfma_full_length_against_fp64():
    """The whole three-level workload (20000 cells, 1e5 steps) in compensated
    FP32 on the matrix-core kernel against the FP64 DPP kernel (which the
    parity suite ties to the oracle): the full-length deviation stays within
    the FP32 bar."""
    p = W.three_level()
    _case("quad_mfma_full_length")
    a = mln.run(p, precision="fp32c", snap_every=20000, variant="quad_mfma", tile=128, steps_per_launch=20)
    b = mln.run(p, precision="fp64", snap_every=20000, variant="quad", tile=128, steps_per_launch=20)
    ee, ep = _errs(a, b)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < 1e-5 and ep < 1e-5


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-4)])
def test_quad_mfma_adjoint_matches_dpp_forward(precision, tol):
    """mln_grad after a matrix-core forward run (checkpoints recomputed with
    it) against mln_grad after the DPP forward run: the reverse kernel is the
    same, so the gradients agree to the forward kernels' rounding."""
    p = W.three_level(nx=160, nt=700)
    p.medium.density = 1e25
    t = np.arange(p.grid.nt + 1) * p.grid.dt
    sig = 30 * p.grid.dt
    p.source = W.Source(np.exp(-0.5 * ((t - 5 * sig) / sig) ** 2) * np.sin(W.OMEGA0 * (t - 5 * sig)), 2e9)
    _case("quad_mfma_adjoint", precision=precision)
    gs = []
    for variant in ("quad_mfma", "quad"):
        s = mln.Solver(p, precision=precision, ckpt_every=64, variant=variant, tile=64, steps_per_launch=16)
        probe = s.run()["probe"].cpu().numpy()
        gs.append(s.grad(2.0 * p.grid.dt * probe))
        s.close()
    for key in gs[0]:
        a, b = np.asarray(gs[0][key]), np.asarray(gs[1][key])
        scale = max(np.max(np.abs(b)), 1e-300)
        print(f"  {key}: {np.max(np.abs(a - b)) / scale:.2e}", flush=True)
        assert np.max(np.abs(a - b)) <= tol * scale


def test_quad_mfma_config_and_errors():
    p = W.random_problem(3, 2, nx=203, nt=50)
    s = mln.Solver(p, precision="fp32c", variant="quad_mfma", tile=64, steps_per_launch=8)
    assert s.config() == {"variant": "quad_mfma", "tile": 64, "steps_per_launch": 8}
    with pytest.raises(mln.MLNError):
        s.configure("quad_mfma", tile=72)  # not a multiple of 16
    assert s.config()["variant"] == "quad_mfma"
    s.close()
    p6 = W.random_problem(6, 4, nx=203, nt=50)
    with pytest.raises(mln.MLNError) as e:
        mln.Solver(p6, precision="fp64", variant="quad_mfma")
    assert e.value.code == -8
