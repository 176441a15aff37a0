"""The streamed one-step kernel of the 1-D grid (variant "stream": one launch
per time step, one thread per cell, state and fields through device memory)
against the oracle: every recorded E and population, FP64 at 1e-10 and the
single-precision modes at 1e-5; its checkpointed adjoint against the
oracle's FP64 adjoint."""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu


def _errs(got, ref):
    e = np.concatenate([got["e_snap"].ravel(), got["probe"].ravel()])
    er = np.concatenate([ref["e_snap"].ravel(), ref["probe"].ravel()])
    return np.max(np.abs(e - er)) / np.max(np.abs(er)), np.max(np.abs(got["pop"] - ref["pop"]))


@pytest.fixture(scope="module")
def refs(orc):
    cache = {}

    def get(key, p, snap):
        if key not in cache:
            cache[key] = orc.run(p, snap_every=snap)
        return cache[key]
    return get


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2), (4, 3), (6, 4)])
@pytest.mark.parametrize("nx", [203, 513, 3])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-5), ("fp32", 1e-5)])
def test_stream_random_media(refs, n, seed, nx, precision, tol):
    p = W.random_problem(n, seed, nx=nx, nt=360)
    print(f"[case] stream n={n} nx={nx} {precision}", flush=True)
    ref = refs((n, seed, nx), p, 40)
    got = mln.run(p, precision=precision, snap_every=40, variant="stream")
    ee, ep = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < tol and ep < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32c", 1e-5)])
def test_stream_two_level_full(orc, precision, tol):
    p = W.two_level()
    print(f"[case] stream two-level full {precision}", flush=True)
    ref = orc.run(p, snap_every=1000)
    got = mln.run(p, precision=precision, snap_every=1000, variant="stream")
    ee, ep = _errs(got, ref)
    print(f"  err_E={ee:.2e} err_pop={ep:.2e}", flush=True)
    assert ee < tol and ep < tol


def test_stream_host_medium_and_state(orc):
    p = W.random_problem(3, 8, nx=150, nt=200)
    p.grid.sigma, p.grid.eps_r, p.grid.mu_r = 1e3, 1.5, 1.8
    ref = orc.run(p, snap_every=50)
    s = mln.Solver(p, precision="fp64", snap_every=50, variant="stream")
    got = {k: v.cpu().numpy() for k, v in s.run().items()}
    _, H, _ = s.state()
    assert s.config()["variant"] == "stream"
    s.close()
    ee, ep = _errs(got, ref)
    assert ee < 1e-10 and ep < 1e-10
    assert np.max(np.abs(H - ref["h"])) < 1e-10 * np.max(np.abs(ref["h"]))


def test_stream_adjoint_matches_oracle_adjoint(orc):
    """The checkpointed adjoint recomputes segments with the handle's forward
    kernel (here the streamed one, which writes the tape) and reverses them
    with the one-cell-per-thread reverse kernel: every gradient group against
    the oracle's FP64 adjoint (1e-10 of the group's largest entry), as for
    the other forward kernels."""
    nt = 500
    p = W.three_level(nx=120, nt=nt)
    p.medium.density = 1e25
    # a short strong pulse that crosses the grid within the run (the
    # workload's own pulse peaks only after 9600 steps)
    t = np.arange(nt + 1) * p.grid.dt
    sig = 30 * p.grid.dt
    p.source = W.Source(np.exp(-0.5 * ((t - 5 * sig) / sig) ** 2) * np.sin(W.OMEGA0 * (t - 5 * sig)), 2e9)
    s = mln.Solver(p, precision="fp64", ckpt_every=50, variant="stream")
    probe = s.run()["probe"].cpu().numpy()
    g = s.grad(2.0 * p.grid.dt * probe)
    s.close()
    ref = orc.grad(p, 2.0 * p.grid.dt * orc.run(p)["probe"])
    for k in ("d_h0", "d_dipole", "d_jump_rate", "d_dephasing", "d_amplitude", "d_density"):
        a, b = np.atleast_1d(np.asarray(g[k])), np.atleast_1d(np.asarray(ref[k]))
        big = np.max(np.abs(b))
        err = np.max(np.abs(a - b)) / big
        print(f"  {k:12s} max err / max|ref| {err:.2e}", flush=True)
        assert np.all(np.abs(a - b) <= 1e-10 * big + 1e-8 * np.abs(b)), k


def test_stream_rejects_unsupported():
    p = W.random_problem(3, 1, nx=60, nt=20)
    for kw in (dict(precision="fp32cf"), dict(route="diag"), dict(steps_per_launch=4)):
        with pytest.raises(mln.MLNError):
            mln.Solver(p, variant="stream", **kw)
