"""The oracle's pins reject plausible mistakes in its coupled Yee run.

Each case copies the oracle's C source, plants one mistake in the coupled
run (orc_run: the first occurrence of the line in the file), builds the copy
with gcc into a temporary directory, loads it in place of the real oracle
and runs the pin that covers that part.  The pin must fail.  The mistakes
are those a reading of Sec. 2 (Eq. maxwell) and Eq. polarization2 could make
the same way on both the oracle's and the GPU's side, so parity alone would
not catch them:

* the polarisation current fed back with the wrong sign, or twice;
* the density N_a dropped by half in dP/dt;
* the semi-implicit conductivity with half its weight;
* eps_r and mu_r exchanged;
* the Mur coefficient taken with the vacuum speed of light in a host medium;
* in the two-dimensional run: H_x updated with the wrong sign, dx and dy
  exchanged in the H coefficients, the y direction not wrapped, and the
  polarisation current fed back with the wrong sign;
* in the two-component run: the E_y polarisation current with the wrong
  sign, the y factors of the split interaction with the full angle, and the
  y dipole driven by E_z.

Everything here runs on the CPU.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_2d as M2
import test_oracle_media as M
import test_oracle_pol2 as MP

MUTANTS = {
    "feedback_sign": ("E[i] = ca * E[i] + cb * (-dp + (H[i] - H[i - 1]) / dx);",
                      "E[i] = ca * E[i] + cb * (dp + (H[i] - H[i - 1]) / dx);",
                      lambda: M.check_coherent_energy(oracle)),
    "feedback_twice": ("E[i] = ca * E[i] + cb * (-dp + (H[i] - H[i - 1]) / dx);",
                       "E[i] = ca * E[i] + cb * (-2.0 * dp + (H[i] - H[i - 1]) / dx);",
                       lambda: M.check_coherent_energy(oracle)),
    "density_half": ("P[c] = cell_step(&m, rho + c * n2, E[mb + c], dt, Na, &ws);",
                     "P[c] = cell_step(&m, rho + c * n2, E[mb + c], dt, 0.5 * Na, &ws);",
                     lambda: M.check_coherent_energy(oracle)),
    "sigma_quarter": ("double sg = sigma * dt / (2.0 * eps);",
                      "double sg = sigma * dt / (4.0 * eps);",
                      lambda: M.check_cw_dispersion(oracle, 2.25, 1.0, 3.0e3)),
    "eps_mu_exchanged": ("double eps = ORC_EPS0 * eps_r, muu = ORC_MU0 * mu_r;",
                         "double eps = ORC_EPS0 * mu_r, muu = ORC_MU0 * eps_r;",
                         lambda: M.check_magic_step_in_host(oracle, 2.25, 1.0)),
    "mur_vacuum_speed": ("double cl = 1.0 / sqrt(eps * muu);",
                         "double cl = 1.0 / sqrt(ORC_EPS0 * ORC_MU0);",
                         lambda: M.check_magic_step_in_host(oracle, 2.25, 1.0)),
    # the two-dimensional run
    "2d_hx_sign": ("Hx[j * nx + i] -= chy * (E[jp * nx + i] - E[j * nx + i]);",
                   "Hx[j * nx + i] += chy * (E[jp * nx + i] - E[j * nx + i]);",
                   lambda: M2.check_mode(oracle, 40, 1, 3.0)),
    "2d_dx_dy_exchanged": ("double chx = dt / (muu * dx), chy = dt / (muu * dy);",
                           "double chx = dt / (muu * dy), chy = dt / (muu * dx);",
                           lambda: M2.check_mode(oracle, 40, 1, 3.0)),
    "2d_no_wrap": ("int64_t jm = (j + ny - 1) % ny;",
                   "int64_t jm = j > 0 ? j - 1 : 0;",
                   lambda: M2.check_mode(oracle, 40, 1, 3.0)),
    "2d_feedback_sign": ("E[j * nx + i] = ca * E[j * nx + i] + cb * (-dp + curl);",
                         "E[j * nx + i] = ca * E[j * nx + i] + cb * (dp + curl);",
                         lambda: M2.check_beam_energy(oracle)),
    # the two-component run
    "pol2_y_feedback_sign": ("*dpy = Na * creal(tr_y);", "*dpy = -Na * creal(tr_y);",
                             lambda: MP.check_equal_dipoles(oracle)),
    "pol2_y_full_angle": ("s->Wa[i] = (I * (0.5 * dt) * Ey / ORC_HBAR) * muy[i];",
                          "s->Wa[i] = (I * dt * Ey / ORC_HBAR) * muy[i];",
                          lambda: MP.check_equal_dipoles(oracle)),
    "pol2_y_driven_by_ez": ("Pz[c] = cell_step_pol2(&m, muy, rho + c * n2, Ez[mb + c], Ey[mb + c], dt, Na, &ws, Wy, Wz,",
                            "Pz[c] = cell_step_pol2(&m, muy, rho + c * n2, Ez[mb + c], Ez[mb + c], dt, Na, &ws, Wy, Wz,",
                            lambda: MP.check_noncommuting_energy(oracle)),
}


def _build_mutant(tmp_path, name, old, new):
    src = open(oracle._SRC).read()
    assert old in src, f"mutation site of {name} not found"
    mutated = src.replace(old, new, 1)
    c_file = tmp_path / f"orc_{name}.c"
    so_file = tmp_path / f"liborc_{name}.so"
    c_file.write_text(mutated)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                           "-o", str(so_file), str(c_file), "-lm"])
    return str(so_file)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_rejects_planted_mistake(tmp_path, name):
    old, new, pin = MUTANTS[name]
    real = oracle.lib()
    pin()  # the pin passes on the real oracle
    path = _build_mutant(tmp_path, name, old, new)
    oracle._lib = oracle.bind(path)
    try:
        with pytest.raises(AssertionError):
            pin()
    finally:
        oracle._lib = real
        os.remove(path)
