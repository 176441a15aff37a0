"""The paper's test cases as set up here.  Two-level (Sec. 5.1): the grid
arithmetic matches the printed spacing, step and snapshot time, and the
printed relaxation superoperator is the Lindblad form it stands for (decay
of the upper level at 1/T1, coherences at 1/T2 in total).  Three-level
(Sec. 5.2): the same grid, transitions the grid resolves, a V system with
the printed dipole ratio, and the printed relaxation superoperator's
action."""
import numpy as np
import pytest

from paper_1710_09799_amd import workloads as W


def test_sit_grid_matches_printed_values():
    p = W.sit_paper()
    g = p.grid
    assert g.nx == 32768
    assert round(g.dx * 1e9, 3) == 4.578          # nm
    assert round(g.dt * 1e18, 3) == 7.635          # 1e-18 s
    assert abs(g.nt * g.dt - 187.5e-15) < 0.5 * g.dt
    assert abs(W.C0 * g.dt / g.dx - 0.5) < 1e-12


def _lindblad_superop(L, rate):
    # vec row-major: vec(A X B) = (A kron B^T) vec(X)
    n = L.shape[0]
    I = np.eye(n)
    LdL = L.conj().T @ L
    return rate * (np.kron(L, L.conj()) - 0.5 * np.kron(LdL, I) - 0.5 * np.kron(I, LdL.T))


def test_sit_relaxation_is_decay_plus_dephasing():
    g = W.sit_paper().medium.relax_superop
    t1 = t2 = 1e-10
    L = np.array([[0, 1], [0, 0]], dtype=complex)  # |1><2|: upper level decays
    deph = np.zeros((4, 4), dtype=complex)
    deph[1, 1] = deph[2, 2] = -(1.0 / t2 - 0.5 / t1)
    want = _lindblad_superop(L, 1.0 / t1) + deph
    assert np.max(np.abs(g - want)) <= 1e-6  # rates ~1e10 /s: relative 1e-16
    # trace preservation: sum over the diagonal outputs vanishes for every input
    assert np.max(np.abs(g[0] + g[3])) == 0.0


# The paper's three-level test case (Sec. 5.2) on the same grid


def test_song_grid_and_transitions():
    """Same grid as the two-level case; the transition frequencies (exponent
    read as 1e15) lie near 794 and 779 nm and are resolved by the grid."""
    p = W.song_paper()
    s = W.sit_paper()
    assert (p.grid.nx, p.grid.dx, p.grid.dt, p.grid.nt) == (s.grid.nx, s.grid.dx, s.grid.dt, s.grid.nt)
    ev = np.real(np.diag(p.medium.h0)) / W.HBAR
    w2, w3 = ev[1] - ev[0], ev[2] - ev[0]
    assert abs(w2 - 2.372e15) < 1e3 and abs(w3 - 2.417e15) < 1e3
    lam2, lam3 = 2 * np.pi * W.C0 / w2, 2 * np.pi * W.C0 / w3
    assert 790e-9 < lam2 < 800e-9 and 775e-9 < lam3 < 785e-9
    assert 2 * np.pi / w3 / p.grid.dt > 300 and lam3 / p.grid.dx > 150


def test_song_dipoles_form_a_v_system():
    mu = W.song_paper().medium.dipole
    assert mu[1, 2] == 0 and mu[0, 0] == mu[1, 1] == mu[2, 2] == 0
    assert np.allclose(mu, mu.conj().T)
    assert abs(mu[0, 2] / mu[0, 1] - np.sqrt(2.0)) < 1e-15


def _apply(g, rho):
    return (g @ rho.reshape(-1)).reshape(rho.shape)


def test_song_relaxation_as_printed():
    """The stored superoperator acting on density matrices: coherences decay
    at 1/T1, trace and Hermiticity are preserved, the ground state relaxes
    with diagonal rates (-2/3, 1/3, 1/3)/T1, and the one density matrix it
    leaves unchanged is the maximally mixed state (the printed form, read as
    it stands)."""
    g = W.song_paper().medium.relax_superop
    t1 = 1e-10
    rng = np.random.default_rng(5)
    a = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    rho = a @ a.conj().T
    rho /= np.trace(rho)
    d = _apply(g, rho)
    assert abs(np.trace(d)) < 1e-6  # rates ~1e10 /s
    assert np.max(np.abs(d - d.conj().T)) < 1e-6
    for i, j in ((0, 1), (0, 2), (1, 2)):
        assert abs(d[i, j] + rho[i, j] / t1) < 1e-6 * abs(rho[i, j] / t1)
    dg = _apply(g, np.diag([1.0, 0.0, 0.0]).astype(complex))
    assert np.allclose(np.real(np.diag(dg)) * t1, [-2 / 3, 1 / 3, 1 / 3], atol=1e-15)
    # null space among Hermitian unit-trace matrices: I / 3 only
    w, v = np.linalg.eig(g)
    null = v[:, np.abs(w) < 1e-3 / t1]
    assert null.shape[1] == 1
    m = null[:, 0].reshape(3, 3)
    m = m / np.trace(m)
    assert np.allclose(m, np.eye(3) / 3, atol=1e-12)
