"""State access at the boundary (mln_get_state, mln_get_bloch,
mln_set_state): the physical state after the completed steps -- fields,
populations (Eq. comp_rho) and Bloch vectors (Sec. 3) recovered from the
carried half-stepped state -- against the oracle's density matrix run, and a
state written into a second handle continuing the run of the first."""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W

pytestmark = pytest.mark.gpu


def _bloch_of(rho, gen):
    # d_l = Tr(rho s_l) (Tr s_l s_m = 2 delta_lm, rho = 1/N + d.s / 2)
    return np.real(np.einsum("ab,lba->l", rho, gen))


@pytest.mark.parametrize("precision,route", [("fp64", "rotation"), ("fp64", "diag"), ("fp64", "rodrigues"),
                                             ("fp64", "pade"), ("fp32c", "rotation"),
                                             ("bf16x6", "rotation")])
@pytest.mark.parametrize("n", [2, 3, 6])
def test_state_after_steps_matches_oracle(orc, precision, route, n):
    if precision == "bf16x6" and n != 6:
        pytest.skip("split-BF16 kernels are built for N = 4, 6")
    tol = 1e-10 if precision == "fp64" else (1e-5 if precision == "fp32c" else 1e-4)
    print(f"[case] state N={n} {precision} {route}", flush=True)
    p = W.random_problem(n, 40 + n, nx=90, nt=160)
    k = 100
    ref = orc.run(p, snap_every=k)  # populations and E after step k
    s = mln.Solver(p, precision=precision, route=route)
    E0, H0, pop0 = s.state()
    d0 = s.bloch()
    gen = mln.setup_factors(p.medium, p.grid.dt)["gen"]
    want = _bloch_of(p.medium.rho0, gen)
    assert np.max(np.abs(d0 - want[:, None])) < (1e-13 if precision == "fp64" else 1e-6)
    assert np.max(np.abs(pop0 - np.real(np.diag(p.medium.rho0))[:, None])) < (1e-13 if precision == "fp64" else 1e-6)
    assert E0[0] == pytest.approx(p.source.amplitude * p.source.samples[0]) and np.all(H0 == 0)
    s.step(k)
    E, H, pop = s.state()
    s.close()
    escale = np.max(np.abs(ref["e_snap"]))
    err_e = np.max(np.abs(E - ref["e_snap"][0])) / escale
    err_p = np.max(np.abs(pop - ref["pop"][0]))
    print(f"  err_E={err_e:.2e} err_pop={err_p:.2e}", flush=True)
    assert err_e < tol and err_p < tol


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32c", 1e-5), ("fp32cf", 1e-5)])
def test_set_state_continues_another_run(precision, tol):
    """Run A for k steps; handle B (same problem) advanced k steps on its own,
    then given A's E, H and Bloch vectors: both continue to the end and record
    the same probe and snapshots (up to the rounding of the FP64 conversion
    of the carried state)."""
    p = W.random_problem(3, 7, nx=200, nt=400)
    k = 150
    a = mln.Solver(p, precision=precision, snap_every=50)
    b = mln.Solver(p, precision=precision, snap_every=50)
    a.step(k)
    E, H, _ = a.state()
    d = a.bloch()
    # B diverges first: a different state written at step 0 and stepped k
    b.set_state(E=np.zeros(p.grid.nx), d=np.zeros_like(d))
    b.step(k)
    b.set_state(E=E, H=H, d=d)
    Eb, Hb, _ = b.state()
    assert np.max(np.abs(Eb - E)) <= 1e-7 * np.max(np.abs(E)) if precision != "fp64" else np.array_equal(Eb, E)
    oa = {kk: v.cpu().numpy() for kk, v in a.run().items() if v is not None}
    ob = {kk: v.cpu().numpy() for kk, v in b.run().items() if v is not None}
    a.close()
    b.close()
    scale = np.max(np.abs(oa["e_snap"]))
    err_e = max(np.max(np.abs(ob["e_snap"][3:] - oa["e_snap"][3:])), np.max(np.abs(ob["probe"][k + 1:] - oa["probe"][k + 1:]))) / scale
    err_p = np.max(np.abs(ob["pop"][3:] - oa["pop"][3:]))
    print(f"[case] set_state {precision}: err_E={err_e:.2e} err_pop={err_p:.2e}", flush=True)
    assert err_e < tol and err_p < tol


def test_set_state_rejects_non_finite():
    p = W.random_problem(2, 1, nx=64, nt=20)
    s = mln.Solver(p)
    E = np.zeros(p.grid.nx)
    E[5] = np.nan
    with pytest.raises(mln.MLNError):
        s.set_state(E=E)
    s.close()


def test_state_of_a_batch_instance(orc):
    """mln_get_state on the handle of one problem of a batch (mln_batch_instance)
    after the batch has stepped: populations and E against the oracle."""
    import ctypes
    probs = [W.random_problem(2, 5, nx=150, nt=200), W.random_problem(3, 6, nx=230, nt=200)]
    k = 120
    b = mln.Batch(probs, precision="fp64", variant="block", tile=128, steps_per_launch=8, graph=False)
    b.step(k)
    L = mln.load()
    for i, p in enumerate(probs):
        h = ctypes.c_void_p()
        assert L.mln_batch_instance(b._h, i, ctypes.byref(h)) == 0
        g, n = p.grid, p.medium.n_levels
        E, H = np.zeros(g.nx), np.zeros(g.nx - 1)
        pop = np.zeros((n, g.n_med))
        assert L.mln_get_state(h, mln._ptr(E), mln._ptr(H), mln._ptr(pop)) == 0
        ref = orc.run(p, snap_every=k)
        err_e = np.max(np.abs(E - ref["e_snap"][0])) / np.max(np.abs(ref["e_snap"]))
        err_p = np.max(np.abs(pop - ref["pop"][0]))
        print(f"[case] batch instance {i}: err_E={err_e:.2e} err_pop={err_p:.2e}", flush=True)
        assert err_e < 1e-10 and err_p < 1e-10
    b.close()
