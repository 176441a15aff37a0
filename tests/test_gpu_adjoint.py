"""The adjoint (reverse-time) pass against finite differences.

Objective: J = dt * sum_n E_probe[n]^2 (energy of the transmitted field at the
right boundary), so dJ/dprobe[n] = 2 dt E_probe[n].
"""
import math

import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W
from paper_1710_09799_amd.autograd import ladder_params, ladder_problem, grads_to_ladder

pytestmark = pytest.mark.gpu


def _J(probe, dt):
    return dt * float(np.sum(probe ** 2))


def _small_ladder(n, nx=160, nt=700):
    """Short three-level (or two-level) ladder run whose transmitted field is
    reshaped by the medium."""
    p = W.three_level(nx=nx, nt=nt) if n == 3 else W.two_level(nx=nx, nt=nt)
    if n == 2:
        p.medium = W.ladder_medium(np.real(np.diag(p.medium.h0)), [1e-29], density=1e25,
                                   decay=1e12, dephasing=5e12)
    else:
        p.medium.density = 1e25
    t = np.arange(nt + 1) * p.grid.dt
    sig = 30 * p.grid.dt
    p.source = W.Source(np.exp(-0.5 * ((t - 5 * sig) / sig) ** 2) * np.sin(W.OMEGA0 * (t - 5 * sig)), 2e9)
    return p


def _run_J(prob, precision="fp64"):
    out = mln.run(prob, precision=precision)
    return _J(out["probe"], prob.grid.dt)


def _grad(prob, precision="fp64", ckpt=64):
    s = mln.Solver(prob, precision=precision, ckpt_every=ckpt)
    out = s.run()
    probe = out["probe"].cpu().numpy()
    J = _J(probe, prob.grid.dt)
    g = s.grad(2.0 * prob.grid.dt * probe)
    s.close()
    return J, g


def _fd_ladder(prob, runner, h=1e-6, richardson=False):
    """Central differences in each ladder parameter (relative step h; energy
    steps relative to the level spacing).  With richardson=True, steps h and
    2h are combined to cancel the O(h^2) term."""
    x0 = ladder_params(prob)
    n = prob.medium.n_levels
    scale = np.abs(x0).copy()
    spacing = np.max(np.abs(np.diff(x0[:n])))
    scale[:n] = spacing

    def cd(i, hh):
        xp, xm = x0.copy(), x0.copy()
        xp[i] += hh * scale[i]
        xm[i] -= hh * scale[i]
        return (runner(ladder_problem(prob, xp)) - runner(ladder_problem(prob, xm))) / (2 * hh * scale[i])
    out = []
    for i in range(len(x0)):
        if richardson:
            out.append((4.0 * cd(i, h) - cd(i, 2 * h)) / 3.0)
        else:
            out.append(cd(i, h))
    return np.array(out), scale


def _compare(ga, fd, scale, tol_scale, tol_rel):
    """|a - b| <= tol_scale * max_j |b_j| + tol_rel |b| for the gradients
    expressed per relative parameter change (a = g * scale)."""
    a, b = ga * scale, fd * scale
    big = np.max(np.abs(b))
    for i in range(len(a)):
        print(i, a[i], b[i])
        assert abs(a[i] - b[i]) <= tol_scale * big + tol_rel * abs(b[i]), (i, a[i], b[i], big)


@pytest.mark.parametrize("n", [2, 3])
def test_fp64_adjoint_matches_fd_of_gpu_forward(n):
    """Central differences with the h = 1e-6 relative step of the workload
    description, and a Richardson-extrapolated h = 1e-4 difference that is
    not limited by round-off for the weakly coupled parameters."""
    prob = _small_ladder(n)
    print(f"[case] adjoint fp64 n={n}", flush=True)
    J, g = _grad(prob)
    ga = grads_to_ladder(g, n)
    fd, scale = _fd_ladder(prob, _run_J)
    _compare(ga, fd, scale, 1e-6, 1e-5)
    fdr, _ = _fd_ladder(prob, _run_J, h=1e-4, richardson=True)
    _compare(ga, fdr, scale, 1e-8, 1e-6)


def test_fp64_adjoint_matches_fd_of_oracle(orc):
    """Independent check: finite differences of the FP64 density-matrix
    oracle (Richardson-extrapolated, h = 1e-4)."""
    n = 3
    prob = _small_ladder(n, nx=120, nt=500)
    J, g = _grad(prob, ckpt=50)
    ga = grads_to_ladder(g, n)

    def orc_J(p):
        return _J(orc.run(p)["probe"], p.grid.dt)
    fd, scale = _fd_ladder(prob, orc_J, h=1e-4, richardson=True)
    _compare(ga, fd, scale, 1e-8, 1e-6)


def _cmp_oracle_adjoint(g, ref, tol_group, tol_rel):
    worst = 0.0
    for k in ("d_h0", "d_dipole", "d_jump_rate", "d_dephasing", "d_amplitude", "d_density"):
        a = np.atleast_1d(np.asarray(g[k]))
        b = np.atleast_1d(np.asarray(ref[k]))
        big = np.max(np.abs(b))
        err = np.abs(a - b)
        print(f"  {k:12s} max|ref| {big:.3e} max err / max|ref| {np.max(err) / big:.2e}")
        assert np.all(err <= tol_group * big + tol_rel * np.abs(b)), (k, a, b)
        worst = max(worst, np.max(err) / big)
    return worst


@pytest.mark.parametrize("kind", ["ladder3", "random2", "random3"])
def test_fp64_adjoint_matches_oracle_adjoint(orc, kind):
    """The GPU adjoint against the oracle's own FP64 adjoint (reverse mode
    through the full density-matrix scheme, no Bloch representation): every
    physical gradient the library returns, for the transmitted-field energy.
    Both are exact adjoints of discretisations that agree to round-off, so
    they agree far below the finite-difference tolerance."""
    if kind == "ladder3":
        prob = _small_ladder(3, nx=120, nt=500)
    else:
        n = int(kind[-1])
        prob = W.random_problem(n, 40 + n, nx=64, nt=300)
        prob.medium.density = 1e25
    print(f"[case] oracle adjoint {kind}", flush=True)
    s = mln.Solver(prob, precision="fp64", ckpt_every=50)
    probe = s.run()["probe"].cpu().numpy()
    g = s.grad(2.0 * prob.grid.dt * probe)
    s.close()
    ref = orc.grad(prob, 2.0 * prob.grid.dt * orc.run(prob)["probe"])
    _cmp_oracle_adjoint(g, ref, 1e-10, 1e-8)


def test_adjoint_invariants():
    """Shifting every level energy by the same amount changes nothing
    (commutator with the identity vanishes, Eq. liouville): the energy
    gradients sum to zero.  J is quadratic in the source amplitude when the
    medium is absent: a dJ/da = 2 J."""
    prob = _small_ladder(3)
    J, g = _grad(prob)
    de = np.real(np.diag(g["d_h0"]))
    assert abs(de.sum()) <= 1e-8 * np.abs(de).max()
    vac = _small_ladder(3)
    vac.medium.density = 0.0
    J0, g0 = _grad(vac)
    a = vac.source.amplitude
    assert abs(a * g0["d_amplitude"] - 2 * J0) <= 1e-10 * J0


@pytest.mark.parametrize("ckpt", [1, 7, 64, 700])
def test_checkpoint_interval_does_not_change_gradient(ckpt):
    prob = _small_ladder(3, nt=700)
    _, g1 = _grad(prob, ckpt=ckpt)
    _, g2 = _grad(prob, ckpt=100)
    a, b = grads_to_ladder(g1, 3), grads_to_ladder(g2, 3)
    assert np.max(np.abs(a - b) / (np.abs(b) + 1e-300 + 1e-6 * np.abs(b).max())) < 1e-9


@pytest.mark.parametrize("precision", ["fp32c", "fp32cf", "fp32f", "fp32"])
def test_fp32_adjoint_close_to_fp64(precision):
    """The single-precision modes' gradients (the reverse step runs in FP32
    on the tape the forward kernel wrote; with float-float fields the tape
    holds the high part of E) against FP64."""
    prob = _small_ladder(3, nt=2000)
    _, g64 = _grad(prob, "fp64", ckpt=200)
    _, g32 = _grad(prob, precision, ckpt=200)
    a, b = grads_to_ladder(g32, 3), grads_to_ladder(g64, 3)
    scale = ladder_params(prob)
    scale[:3] = np.max(np.abs(np.diff(scale[:3])))
    rel = np.abs(a - b) * np.abs(scale) / np.max(np.abs(b * scale))
    print("fp32 vs fp64 adjoint rel", rel)
    assert np.max(rel) < 1e-3


def test_torch_autograd_function():
    import torch
    from paper_1710_09799_amd.autograd import LadderTransmission
    prob = _small_ladder(3, nt=500)
    x = torch.tensor(ladder_params(prob), dtype=torch.float64, requires_grad=True)
    probe = LadderTransmission.apply(x, prob, "fp64", 50)
    J = prob.grid.dt * (probe ** 2).sum()
    J.backward()
    _, g = _grad(prob, ckpt=50)
    want = grads_to_ladder(g, 3)
    assert np.allclose(x.grad.numpy(), want, rtol=1e-10, atol=0)


def test_grad_state_errors():
    prob = _small_ladder(2, nt=100)
    s = mln.Solver(prob, precision="fp64")
    s.run()
    with pytest.raises(mln.MLNError) as e:
        s.grad(np.zeros(101))
    assert e.value.code == -10
    s2 = mln.Solver(prob, precision="fp64", ckpt_every=10)
    s2.step(50)
    with pytest.raises(mln.MLNError) as e:
        s2.grad(np.zeros(101))
    assert e.value.code == -10


@pytest.mark.slow
def test_adjoint_case_full_size():
    """The adjoint workload at full size (three-level ladder, 10000 cells,
    50000 steps, checkpoints every 500): the FP64 gradient of the transmitted
    energy against central differences with the h = 1e-6 relative step (FP64
    forward runs), and the compensated-FP32 gradient (the measured
    configuration) against the FP64 one."""
    prob = W.adjoint_case()
    print("[case] adjoint case full size", flush=True)
    J, g64 = _grad(prob, "fp64", ckpt=500)
    ga = grads_to_ladder(g64, 3)
    fd, scale = _fd_ladder(prob, _run_J)
    _compare(ga, fd, scale, 1e-6, 1e-5)
    _, g32 = _grad(prob, "fp32c", ckpt=500)
    a = grads_to_ladder(g32, 3) * scale
    b = ga * scale
    rel = np.abs(a - b) / np.max(np.abs(b))
    print("fp32c vs fp64 gradient, relative to the largest:", rel)
    assert np.max(rel) < 1e-3


def _p5_problem():
    """The adjoint workload cut to 1000 cells x 5000 steps (checkpoints every
    500 steps).  Its Gaussian pi pulse (200 fs envelope FWHM) is centred at
    step 2500 instead of 600 fs so that the transmitted pulse reaches the
    probe inside the shorter run (it arrives about 2000 steps after it
    leaves the source)."""
    nx, nt = 1000, 5000
    p = W.adjoint_case(nx=nx, nt=nt)
    sig = 200e-15 / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    p.source = W.Source(W.gauss_pulse(nt, W.DT0, W.OMEGA0, sig, 2500 * W.DT0), p.source.amplitude)
    return p


@pytest.mark.slow
def test_p5_adjoint_matches_oracle_adjoint(orc):
    """The reduced adjoint workload (1000 cells x 5000 steps, checkpoints
    every 500): the GPU's FP64 gradient of the transmitted energy against the
    oracle's FP64 adjoint on every gradient group (1e-10 of the group's
    largest entry), and the compensated-FP32 gradient within 1e-3."""
    prob = _p5_problem()
    print("[case] P5 adjoint vs oracle adjoint (1000 x 5000)", flush=True)
    ref_probe = orc.run(prob)["probe"]
    assert np.max(np.abs(ref_probe)) > 0.3 * prob.source.amplitude  # the pulse arrived
    ref = orc.grad(prob, 2.0 * prob.grid.dt * ref_probe)
    for precision, tol in (("fp64", 1e-10), ("fp32c", 1e-3)):
        s = mln.Solver(prob, precision=precision, ckpt_every=500)
        probe = s.run()["probe"].cpu().numpy()
        g = s.grad(2.0 * prob.grid.dt * probe)
        s.close()
        print(f"  {precision}", flush=True)
        worst = _cmp_oracle_adjoint(g, ref, tol, 0.0 if precision != "fp64" else 1e-8)
        print(f"  {precision} worst group error {worst:.2e}", flush=True)


@pytest.mark.parametrize("precision", ["fp64", "fp32c", "fp32cf"])
def test_whole_tape_equals_checkpoints(precision):
    """ckpt_every = MLN_TAPE_ALL keeps the forward tape of every step in device
    memory: the gradient equals the checkpointed one (same values recorded,
    without recomputation), a second mln_grad for another objective works
    without rerunning, and mln_set_state invalidates the tape."""
    prob = _small_ladder(3, nx=160, nt=700)
    print(f"[case] whole tape {precision}", flush=True)
    _, gc = _grad(prob, precision, ckpt=64)
    s = mln.Solver(prob, precision=precision, ckpt_every="tape")
    probe = s.run()["probe"].cpu().numpy()
    gt = s.grad(2.0 * prob.grid.dt * probe)
    a, b = grads_to_ladder(gt, 3), grads_to_ladder(gc, 3)
    # the tapes are the same; the reverse launches group the steps
    # differently (one segment against 64-step segments), which changes the
    # rounding of the single-precision per-launch sums
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.max(np.abs(a - b) / (np.abs(b) + 1e-300 + 1e-9 * np.abs(b).max())) < tol
    # another objective on the same run: J' = dt sum probe (linear), twice
    g1 = grads_to_ladder(s.grad(np.full(prob.grid.nt + 1, prob.grid.dt)), 3)
    g2 = grads_to_ladder(s.grad(np.full(prob.grid.nt + 1, prob.grid.dt)), 3)
    assert np.array_equal(g1, g2)
    assert not np.allclose(g1, a)
    E, H, _ = s.state()
    s.set_state(E=E)
    with pytest.raises(mln.MLNError) as e:
        s.grad(2.0 * prob.grid.dt * probe)
    assert e.value.code == -10
    s.reset()
    s.run()
    g3 = grads_to_ladder(s.grad(2.0 * prob.grid.dt * probe), 3)
    assert np.array_equal(g3, a)
    s.close()


@pytest.mark.parametrize("precision,variant", [("fp64", "quad"), ("fp32c", "quad_mfma"), ("fp32", "block")])
def test_overlapped_rebuild_is_deterministic(precision, variant):
    """With several checkpoint intervals mln_grad rebuilds segment k-1 on a
    second stream while segment k is reversed: the gradient is the same bit
    for bit on every call (a missing dependency between the two streams would
    read a tape buffer before or while it is rewritten), and equal to the
    one-segment pass (nothing overlapped) to rounding."""
    prob = _small_ladder(3, nx=400, nt=1500)
    print(f"[case] overlap {precision} {variant}", flush=True)
    s = mln.Solver(prob, precision=precision, ckpt_every=96, variant=variant)
    gs = []
    for _ in range(3):
        s.reset()
        probe = s.run()["probe"].cpu().numpy()
        gs.append(grads_to_ladder(s.grad(2.0 * prob.grid.dt * probe), 3))
    s.close()
    assert np.array_equal(gs[0], gs[1]) and np.array_equal(gs[0], gs[2])
    s1 = mln.Solver(prob, precision=precision, ckpt_every=prob.grid.nt, variant=variant)
    probe = s1.run()["probe"].cpu().numpy()
    g1 = grads_to_ladder(s1.grad(2.0 * prob.grid.dt * probe), 3)
    s1.close()
    tol = 1e-9 if precision == "fp64" else 1e-4
    assert np.max(np.abs(gs[0] - g1) / (np.abs(g1) + 1e-300 + 1e-6 * np.abs(g1).max())) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_reverse_tiling_does_not_change_gradient(precision):
    """mln_configure_adjoint: the reverse kernel's tiling is independent of
    the forward one (the tape is read by cell); every tiling, on both
    reverse kernels, gives the automatic tiling's gradient to rounding, with
    checkpoints and with the whole tape."""
    prob = _small_ladder(3, nx=300, nt=900)
    print(f"[case] reverse tiling {precision}", flush=True)
    tol = 1e-11 if precision == "fp64" else 2e-5
    for ck in (128, "tape"):
        s = mln.Solver(prob, precision=precision, ckpt_every=ck)
        probe = s.run()["probe"].cpu().numpy()
        gp = 2.0 * prob.grid.dt * probe
        ref = grads_to_ladder(s.grad(gp), 3)
        for variant, tile, k in (("quad", 128, 44), ("quad", 64, 16), ("quad", 32, 7), ("quad", 128, 1),
                                 ("block", 256, 16), ("block", 64, 31)):
            if ck != "tape":
                s.reset()
                s.run()
            s.configure_adjoint(variant, tile, k)
            g = grads_to_ladder(s.grad(gp), 3)
            dev = np.max(np.abs(g - ref) / (np.abs(ref) + 1e-300 + 1e-6 * np.abs(ref).max()))
            print(f"  ckpt={ck} {variant} tile={tile} k={k}: {dev:.2e}", flush=True)
            assert dev < tol
        s.configure_adjoint("auto")
        s.close()


def test_configure_adjoint_errors():
    prob = _small_ladder(3, nx=160, nt=300)
    s = mln.Solver(prob, precision="fp64", ckpt_every=50)
    for args in (("quad", 72, 8), ("quad", 256, 8), ("quad", 64, 32), ("block", 96, 8), ("block", 256, 200),
                 ("wave", 64, 8), ("auto", 64, 0)):
        with pytest.raises(mln.MLNError) as e:
            s.configure_adjoint(*args)
        assert e.value.code == -1, args
    s.configure_adjoint("quad", 0, 0)  # tile 128, 32 steps
    s.configure_adjoint("block")  # tile 256, 64 steps
    s.configure_adjoint()
    s.close()
    p6 = W.random_problem(6, 3, nx=100, nt=50)
    s6 = mln.Solver(p6, precision="fp64")
    with pytest.raises(mln.MLNError) as e:
        s6.configure_adjoint("quad", 64, 8)
    assert e.value.code == -8
    s6.close()
