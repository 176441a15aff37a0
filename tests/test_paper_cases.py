"""The paper's two-level test case (Sec. 5.1) as set up here: the grid
arithmetic matches the printed spacing, step and snapshot time, and the
printed relaxation superoperator is the Lindblad form it stands for (decay
of the upper level at 1/T1, coherences at 1/T2 in total)."""
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
