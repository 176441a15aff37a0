"""CPU test of the host chain rule used by the adjoint (mln_chain_rule): for a
random linear functional J of the step quantities (A = exp(M dt), c, w, p0,
U, d'_0), the chain-rule gradient with respect to every physical input equals
central finite differences of J through the host factor construction."""
import numpy as np
import pytest

from paper_1710_09799_amd import mln
from paper_1710_09799_amd import workloads as W


def _quantities(med, dt):
    f = mln.setup_factors(med, dt)
    A0, b0 = f["A0"], f["b0"]
    A = A0 @ A0
    c = A0 @ b0 + b0
    w = 0.5 * med.density * (f["M"] @ A0).T @ f["v"]
    p0 = 0.5 * med.density * f["v"] @ (f["M"] @ b0 + f["deq"])
    d0p = A0 @ f["d0"] + b0
    return A, c, w, p0, f["U"], d0p


def _J(med, dt, R):
    A, c, w, p0, U, d0p = _quantities(med, dt)
    return (np.sum(R[0] * A) + R[1] @ c + R[2] @ w + R[3] * p0 + np.sum(R[4] * U) + R[5] @ d0p)


def _copy(med):
    return W.Medium(h0=med.h0.copy(), dipole=med.dipole.copy(), rho0=med.rho0.copy(),
                    density=med.density, jumps=[j.copy() for j in med.jumps],
                    jump_rates=list(med.jump_rates), dephasing=med.dephasing)


@pytest.mark.parametrize("n,seed", [(2, 1), (3, 2)])
def test_chain_rule_matches_finite_differences(n, seed):
    med = W.random_medium(n, seed)
    dt = W.DT0
    D = n * n - 1
    rng = np.random.default_rng(seed)
    A, c, w, p0, U, d0p = _quantities(med, dt)
    # scale the random weights so every term contributes comparably
    R = [rng.normal(size=(D, D)) / np.abs(A).max(), rng.normal(size=D) / max(np.abs(c).max(), 1e-300),
         rng.normal(size=D) / np.abs(w).max(), rng.normal() / abs(p0), rng.normal(size=(D, D)) / np.abs(U).max(),
         rng.normal(size=D) / np.abs(d0p).max()]
    g = mln.chain_rule(med, dt, R[0], R[1], R[2], R[3], R[4], R[5])

    def fd(setter, scale):
        h = 1e-5 * scale
        mp, mm = _copy(med), _copy(med)
        setter(mp, +h)
        setter(mm, -h)
        return (_J(mp, dt, R) - _J(mm, dt, R)) / (2 * h)

    def check(got, want, what):
        assert abs(got - want) <= 1e-6 * max(abs(want), 1e-3 * scale_ref), (what, got, want)

    scale_ref = 1.0
    eh = np.abs(med.h0).max()
    for a in range(n):
        for b in range(a, n):
            def s_re(m, h, a=a, b=b):
                m.h0[a, b] += h
                if a != b:
                    m.h0[b, a] += h
            want = fd(s_re, eh)
            scale_ref = max(abs(want) * eh, 1e-300) / eh
            check(g["d_h0"][a, b].real, want, ("h0 re", a, b))
            if a != b:
                def s_im(m, h, a=a, b=b):
                    m.h0[a, b] += 1j * h
                    m.h0[b, a] -= 1j * h
                check(g["d_h0"][a, b].imag, fd(s_im, eh), ("h0 im", a, b))
                assert g["d_h0"][b, a] == np.conj(g["d_h0"][a, b])
    em = np.abs(med.dipole).max()
    for a in range(n):
        for b in range(a, n):
            def m_re(m, h, a=a, b=b):
                m.dipole[a, b] += h
                if a != b:
                    m.dipole[b, a] += h
            want = fd(m_re, em)
            scale_ref = abs(want) + 1e-300
            check(g["d_dipole"][a, b].real, want, ("mu re", a, b))
            if a != b:
                def m_im(m, h, a=a, b=b):
                    m.dipole[a, b] += 1j * h
                    m.dipole[b, a] -= 1j * h
                check(g["d_dipole"][a, b].imag, fd(m_im, em), ("mu im", a, b))
    for k in range(len(med.jumps)):
        def r_k(m, h, k=k):
            m.jump_rates[k] += h
        want = fd(r_k, med.jump_rates[k])
        scale_ref = abs(want) + 1e-300
        check(g["d_jump_rate"][k], want, ("rate", k))

    def deph(m, h):
        m.dephasing += h
    want = fd(deph, med.dephasing)
    scale_ref = abs(want) + 1e-300
    check(g["d_dephasing"], want, "dephasing")

    def dens(m, h):
        m.density += h
    want = fd(dens, med.density)
    scale_ref = abs(want) + 1e-300
    check(g["d_density"], want, "density")
