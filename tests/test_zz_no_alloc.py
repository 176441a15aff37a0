"""mln_bloch_only_noalloc (the entry point for callers that cannot allocate
device memory) against mln_bloch_only on the same handle and input: the same
kernels, so the outputs agree bit for bit; two handles of different level
counts, precisions and sizes called in a row (the second smaller), and the
first again with fewer steps, so that a result depending on what an earlier
call left in the shared scratch would show.  The FP64 case is also held to
the oracle's prescribed-field run at 1e-10."""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu


def _solver(n, seed, ncell, precision):
    med = W.random_medium(n, seed)
    grid = W.Grid(nx=ncell + 2, nt=1, dx=W.DX0, dt=W.DT0, med_begin=1, med_end=ncell + 1)
    prob = W.Problem("b", med, grid, W.Source(np.zeros(2), 0.0))
    return prob, mln.Solver(prob, precision=precision)


def _both(s, prob, f):
    import torch
    n, nc = prob.medium.n_levels, prob.grid.n_med
    e = torch.tensor(f, device="cuda")
    ref = s.bloch_only(e)
    pop = torch.full((f.shape[0], n, nc), float("nan"), dtype=torch.float64, device="cuda")
    dp = torch.full((f.shape[0], nc), float("nan"), dtype=torch.float64, device="cuda")
    got = s.bloch_only_noalloc(e, pop, dp)
    return ({k: v.cpu().numpy() for k, v in ref.items()}, {k: v.cpu().numpy() for k, v in got.items()})


def test_noalloc_matches_bloch_only_on_calls_in_a_row(orc):
    rng = np.random.default_rng(3)
    print("[case] noalloc: N=3 fp64 201 cells x 300 steps", flush=True)
    pa, sa = _solver(3, 31, 201, "fp64")
    fa = rng.uniform(-3e9, 3e9, size=(300, 201))
    ref, got = _both(sa, pa, fa)
    assert np.array_equal(got["pop"], ref["pop"]) and np.array_equal(got["dp"], ref["dp"])
    o = orc.bloch(pa.medium, fa, W.DT0)
    assert np.max(np.abs(got["pop"] - o["pop"])) < 1e-10
    assert np.max(np.abs(got["dp"] - o["dp"])) < 1e-10 * np.max(np.abs(o["dp"]))

    print("[case] noalloc: N=2 fp32c 50 cells x 120 steps (smaller, second call)", flush=True)
    pb, sb = _solver(2, 32, 50, "fp32c")
    fb = rng.uniform(-3e9, 3e9, size=(120, 50))
    ref, got = _both(sb, pb, fb)
    assert np.array_equal(got["pop"], ref["pop"]) and np.array_equal(got["dp"], ref["dp"])
    ob = orc.bloch(pb.medium, fb, W.DT0)
    assert np.max(np.abs(got["pop"] - ob["pop"])) < 1e-5

    print("[case] noalloc: N=3 fp64 again, 77 steps", flush=True)
    ref, got = _both(sa, pa, fa[:77])
    assert np.array_equal(got["pop"], ref["pop"]) and np.array_equal(got["dp"], ref["dp"])
    sa.close()
    sb.close()


def test_noalloc_six_level_split_bf16():
    rng = np.random.default_rng(4)
    print("[case] noalloc: N=6 bf16x6 and fp64 64 cells x 100 steps", flush=True)
    for precision in ("bf16x6", "fp64"):
        p, s = _solver(6, 33, 64, precision)
        f = rng.uniform(-3e9, 3e9, size=(100, 64))
        ref, got = _both(s, p, f)
        assert np.array_equal(got["pop"], ref["pop"]) and np.array_equal(got["dp"], ref["dp"])
        s.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    p, s = _solver(2, 34, 10, "fp64")
    L = mln.load()
    assert L.mln_bloch_only_noalloc(s._h, None, 5, None, None) == -1
    e = torch.zeros((5, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        s.bloch_only_noalloc(e, torch.zeros((5, 3, 10), dtype=torch.float64, device="cuda"))
    s.close()
