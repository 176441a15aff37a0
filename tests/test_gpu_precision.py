"""Reduced-precision paths against the FP64 oracle.

Tolerances: single precision ("fp32"; compensated "fp32c": two-float Bloch
vectors and factors; "fp32cf": E and H as two-float pairs as well; "fp32f":
plain single-precision state with two-float E and H) must meet
1e-5 on err_E and err_pop (the FP32 target); plain single precision on the
diagonalisation and Rodrigues routes, which carry d rather than its deviation
from the rest state, is held to a looser bound that documents its drift
(factor rounding accumulates over the near-identity steps); split-BF16 meets
1e-4.
"""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu


def _errs(got, ref):
    e = np.concatenate([got["e_snap"].ravel(), got["probe"].ravel()])
    er = np.concatenate([ref["e_snap"].ravel(), ref["probe"].ravel()])
    return (np.max(np.abs(e - er)) / np.max(np.abs(er)),
            np.max(np.abs(got["pop"] - ref["pop"])) if ref["pop"].size else 0.0)


@pytest.fixture(scope="module")
def three_level_ref(orc):
    p = W.three_level(nx=2000, nt=10000)
    return p, orc.run(p, snap_every=500)


@pytest.fixture(scope="module")
def two_level_ref(orc):
    p = W.two_level()
    return p, orc.run(p, snap_every=1000)


@pytest.mark.parametrize("precision,variant", [("fp32c", "auto"), ("fp32cf", "quad"), ("fp32cf", "block"),
                                               ("fp32f", "quad"), ("fp32f", "block")])
def test_fp32c_three_level(three_level_ref, precision, variant):
    p, ref = three_level_ref
    got = mln.run(p, precision=precision, variant=variant, snap_every=500)
    ee, ep = _errs(got, ref)
    print(f"{precision} {variant} three_level err_E={ee:.3e} err_pop={ep:.3e}")
    assert ee < 1e-5 and ep < 1e-5


def test_fp32c_two_level(two_level_ref):
    p, ref = two_level_ref
    got = mln.run(p, precision="fp32c", snap_every=1000)
    ee, ep = _errs(got, ref)
    print(f"fp32c two_level err_E={ee:.3e} err_pop={ep:.3e}")
    assert ee < 1e-5 and ep < 1e-5


@pytest.mark.parametrize("route,variant,tol", [("rotation", "quad", 1e-5), ("rotation", "block", 1e-5),
                                               ("diag", "block", 1e-3), ("rodrigues", "block", 1e-3),
                                               ("pade", "block", 1e-3)])
def test_fp32_plain_three_level(three_level_ref, route, variant, tol):
    """Plain single precision.  The rotation route carries the deviation from
    the (exact) rest state, so the rounding of the factors acts on the
    excitation only and the FP32 tolerance holds; the diagonalisation,
    Rodrigues and per-step Pade routes carry d itself and are held to the
    documented 1e-3."""
    p, ref = three_level_ref
    got = mln.run(p, precision="fp32", route=route, variant=variant, snap_every=500)
    ee, ep = _errs(got, ref)
    print(f"fp32 {route} {variant} three_level err_E={ee:.3e} err_pop={ep:.3e}")
    assert ee < tol and ep < tol


def test_fp32_plain_two_level(two_level_ref):
    p, ref = two_level_ref
    got = mln.run(p, precision="fp32", snap_every=1000)
    ee, ep = _errs(got, ref)
    print(f"fp32 two_level err_E={ee:.3e} err_pop={ep:.3e}")
    assert ee < 1e-5 and ep < 1e-5


@pytest.mark.parametrize("precision", ["fp32c", "fp32cf"])
def test_fp32c_small_random(orc, precision):
    for n, seed in ((2, 1), (3, 2), (4, 3), (6, 4)):
        p = W.random_problem(n, seed, nx=203, nt=360)
        ref = orc.run(p, snap_every=40)
        got = mln.run(p, precision=precision, snap_every=40, tile=64, steps_per_launch=8)
        ee, ep = _errs(got, ref)
        print(f"{precision} random n={n} err_E={ee:.3e} err_pop={ep:.3e}")
        assert ee < 1e-5 and ep < 1e-5


def test_fp32c_bloch_only(orc):
    import torch
    med = W.random_medium(3, 60)
    rng = np.random.default_rng(1)
    nt, nc = 4000, 16
    f = rng.uniform(-3e9, 3e9, size=(nt, nc))
    grid = W.Grid(nx=nc + 2, nt=1, dx=W.DX0, dt=W.DT0, med_begin=1, med_end=nc + 1)
    prob = W.Problem("b", med, grid, W.Source(np.zeros(2), 0.0))
    ref = orc.bloch(med, f, W.DT0)
    s = mln.Solver(prob, precision="fp32c")
    out = s.bloch_only(torch.tensor(f, device="cuda"))
    err = np.max(np.abs(out["pop"].cpu().numpy() - ref["pop"]))
    print(f"fp32c bloch err_pop={err:.3e}")
    assert err < 1e-5


@pytest.fixture(scope="module")
def six_level_ref(orc):
    p = W.six_level(nx=1000, nt=20000)
    return p, orc.run(p, snap_every=2000)


@pytest.mark.parametrize("precision,variant,tol", [("fp64", "block", 1e-10), ("fp64", "wave", 1e-10),
                                                   ("fp32c", "block", 1e-5), ("fp32cf", "block", 1e-5),
                                                   ("fp32", "block", 1e-5),
                                                   ("bf16x6", "block", 1e-4), ("bf16x3", "block", 1e-4),
                                                   ("bf16x6", "quad", 1e-4), ("bf16x3", "quad", 1e-4)])
def test_six_level_reduced(six_level_ref, precision, variant, tol):
    """Six-level (N = 6, D = 35) region at 1000 cells x 20000 steps: CW drive,
    15 Lindblad channels, every recorded E and population."""
    p, ref = six_level_ref
    kw = dict(tile=64, steps_per_launch=16) if variant == "wave" else {}
    got = mln.run(p, precision=precision, variant=variant, snap_every=2000, **kw)
    ee, ep = _errs(got, ref)
    print(f"six_level {precision} {variant} err_E={ee:.3e} err_pop={ep:.3e}")
    assert ee < tol and ep < tol


@pytest.mark.parametrize("variant", ["block", "quad"])
@pytest.mark.parametrize("precision", ["bf16x6", "bf16x3"])
@pytest.mark.parametrize("n,seed", [(4, 3), (6, 4)])
@pytest.mark.parametrize("tile,k", [(64, 8), (128, 32), (256, 50)])
def test_split_bf16_mfma_small_random(orc, precision, n, seed, tile, k, variant):
    """Shared-factor transform on the matrix cores (split-BF16, FP32
    accumulation) for random media, several tiles and a ragged last tile,
    one cell per thread and four lanes per cell; split-BF16 tolerance 1e-4."""
    p = W.random_problem(n, seed, nx=203, nt=360)
    ref = orc.run(p, snap_every=40)
    got = mln.run(p, precision=precision, variant=variant, snap_every=40, tile=tile, steps_per_launch=k)
    ee, ep = _errs(got, ref)
    print(f"{precision} {variant} random n={n} tile={tile} err_E={ee:.3e} err_pop={ep:.3e}")
    assert ee < 1e-4 and ep < 1e-4


def test_compensated_fields_long_run():
    """Over 1e5 steps of continuous drive the FP32 rounding of E and H
    accumulates; with two-float fields the deviation from the FP64 path (which
    matches the oracle to 1e-10) stays below the FP32 tolerance and below the
    plain-field deviation."""
    p = W.six_level(nx=600, nt=100000)
    ref = mln.run(p, precision="fp64", record_pop=False, record_e=False)["probe"]
    errs = {}
    for prec in ("fp32c", "fp32cf", "bf16x6"):
        got = mln.run(p, precision=prec, record_pop=False, record_e=False)["probe"]
        errs[prec] = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("long-run deviation from FP64:", errs)
    assert errs["fp32cf"] < 1e-5
    assert errs["fp32cf"] < errs["fp32c"]
    assert errs["bf16x6"] < 1e-4


def test_wave_kernel_rejects_compensated_fields():
    p = W.random_problem(4, 3, nx=100, nt=50)
    with pytest.raises(mln.MLNError) as e:
        mln.Solver(p, precision="fp32cf", variant="wave", tile=64, steps_per_launch=8)
    assert e.value.code == -8


def test_plain_state_compensated_fields_limits():
    """MLN_FP32_FIELDS is built for the rotation route and N <= 3; it runs on
    the workgroup and four-lanes-per-cell kernels (the automatic choice is
    the DPP quad kernel) and not on the wavefront or streamed kernels."""
    p6 = W.random_problem(6, 3, nx=100, nt=50)
    with pytest.raises(mln.MLNError) as e:
        mln.Solver(p6, precision="fp32f")
    assert e.value.code == -8
    p3 = W.random_problem(3, 3, nx=100, nt=50)
    with pytest.raises(mln.MLNError) as e:
        mln.Solver(p3, precision="fp32f", route="diag")
    assert e.value.code == -8
    for variant in ("wave", "stream"):
        with pytest.raises(mln.MLNError) as e:
            mln.Solver(p3, precision="fp32f", variant=variant)
        assert e.value.code == -8
    s = mln.Solver(p3, precision="fp32f")
    assert s.config()["variant"] == "quad"
    s.close()


@pytest.mark.slow
def test_six_level_full_size():
    """The six-level workload at full size (50000 cells, 200000 steps) in the
    benchmark's launch configurations.  The oracle cannot run it; the FP64 GPU
    path (matched to the oracle to 1e-10 on the reduced six-level shape) is
    the reference: split-BF16 (six products) within its 1e-4 bound and
    compensated fields within 1e-5 on the probe; split-BF16 with three
    products within the 1e-3 its header entry states for runs this long
    (measured 4.9e-4, outside the 1e-4 split-BF16 tolerance); populations of
    every run in [0, 1] and summing to one."""
    p = W.six_level()
    nt = p.grid.nt
    kw = dict(tile=256, steps_per_launch=16, snap_every=nt // 2, record_e=False)
    ref = mln.run(p, precision="fp64", variant="block", **kw)
    for prec, tol in (("bf16x6", 1e-4), ("fp32cf", 1e-5), ("bf16x3", 1e-3)):
        got = mln.run(p, precision=prec, **kw)
        err = np.max(np.abs(got["probe"] - ref["probe"])) / np.max(np.abs(ref["probe"]))
        print(f"six-level full size {prec}: probe deviation from FP64 {err:.2e}")
        assert err < tol
        for out in (got, ref):
            pop = out["pop"]
            assert np.all(np.isfinite(pop)) and pop.min() > -1e-6 and pop.max() < 1 + 1e-6
            assert np.max(np.abs(pop.sum(axis=1) - 1.0)) < 1e-6
