"""mln_run's HIP-graph replay of a whole run against the same launches
enqueued one by one (mln_use_graph(h, 0)), through the C ABI.

The graph holds the same kernels with the same arguments, so every recorded
value (snapshots, probe, populations) and the final fields must be equal bit
for bit.  Each replay is checked, with other eager work on the device and
host synchronisation between replays, after a change of kernel
configuration (the graph is rebuilt), and for the streamed one-step kernel.
"""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _outputs(s):
    out = {k: v.cpu().numpy().copy() for k, v in s.run().items() if v is not None}
    out["fields"] = s.fields()
    return out


def _same(a, b, rtol=0.0):
    for k in a:
        pairs = zip(a[k], b[k]) if k == "fields" else [(a[k], b[k])]
        for x, y in pairs:
            if rtol == 0.0:
                assert np.array_equal(x, y), k
            else:
                assert np.max(np.abs(x - y)) <= rtol * max(np.max(np.abs(x)), 1e-300), k


@pytest.mark.parametrize("n,precision,variant,tile,k", [
    (3, "fp32c", "quad_mfma", 128, 20), (3, "fp64", "quad", 64, 16), (2, "fp32", "block", 256, 32),
    (3, "fp32cf", "quad", 128, 20), (2, "fp64", "stream", 0, 0)])
def test_graph_replays_equal_eager(n, precision, variant, tile, k):
    p = W.random_problem(n, 3, nx=203, nt=410)
    _case("graph_vs_eager", n=n, precision=precision, variant=variant, tile=tile, k=k)
    s = mln.Solver(p, precision=precision, snap_every=40, variant=variant, tile=tile, steps_per_launch=k)
    s.use_graph(False)
    eager = _outputs(s)
    s.use_graph(True)
    other = W.random_problem(2, 9, nx=100, nt=50)
    for rep in range(3):
        s.reset()
        got = _outputs(s)
        _same(eager, got)
        mln.run(other, precision="fp64", snap_every=10)  # eager work between replays
    s.close()


def test_graph_rebuilt_after_configure():
    p = W.random_problem(3, 4, nx=203, nt=300)
    _case("graph_configure")
    s = mln.Solver(p, precision="fp32c", snap_every=30, variant="quad", tile=128, steps_per_launch=20)
    first = _outputs(s)
    s.reset()
    s.configure("quad_mfma", tile=64, steps_per_launch=12)
    s.use_graph(False)
    eager = _outputs(s)
    s.reset()
    s.use_graph(True)
    graph = _outputs(s)
    _same(eager, graph)
    # a different kernel: equal to rounding, not bit for bit
    assert np.max(np.abs(graph["probe"] - first["probe"])) <= 1e-5 * np.max(np.abs(first["probe"]))
    s.close()


def test_run_after_partial_steps_is_eager_and_correct():
    p = W.random_problem(3, 5, nx=203, nt=300)
    _case("graph_partial")
    s = mln.Solver(p, precision="fp64", snap_every=30, variant="quad", tile=64, steps_per_launch=16)
    full = _outputs(s)
    s.reset()
    s.step(37)
    rest = _outputs(s)  # mln_run from step 37: launches enqueued one by one
    _same(full, rest, rtol=1e-13)
    s.close()
