"""The oracle pins reject plausible mistakes.

Each case plants one mistake in a copy of the oracle source (a dropped term, a
flipped sign, a wrong index or weight), builds it into a temporary library, and
runs the pin suite against it in a subprocess: the suite must fail.  Nothing here
touches the GPU or the product library.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "phx_oracle.c")

MUTATIONS = {
    "kinetic_sign": ("cplx h = -(p->hbar * p->hbar / (2.0 * p->mass))", "cplx h = (p->hbar * p->hbar / (2.0 * p->mass))"),
    "kinetic_mass": ("(2.0 * p->mass)) * laplacian", "(p->mass)) * laplacian"),
    "laplacian_y_index": ("at(p, f, i, j + 1) + at(p, f, i, j - 1)", "at(p, f, i, j + 1) + at(p, f, i, j + 1)"),
    "periodic_wrap": ("i = ((i % p->nx) + p->nx) % p->nx;", "i = 0;"),
    "zero_ghost": ("if (p->bc_x == ORC_BC_ZERO) return 0.0;", "if (p->bc_x == ORC_BC_ZERO) i = i < 0 ? 0 : p->nx - 1;"),
    "nonlinear_sign": ("(pot + p->g * rho +", "(pot - p->g * rho +"),
    "cross_interaction_dropped": ("+ p->g_x * rho_o", "+ 0.0 * rho_o"),
    "tetm_mixed_sign": ("- 2.0 * sgn * I * d_xy(p, po, i, j));", "+ 2.0 * sgn * I * d_xy(p, po, i, j));"),
    "tetm_dyy_sign": ("h += p->delta_lt * (d_xx(p, po, i, j) - d_yy(p, po, i, j)", "h += p->delta_lt * (d_xx(p, po, i, j) + d_yy(p, po, i, j)"),
    "gain_dropped": ("0.5 * (p->R * nn - p->gamma_c) * v;", "0.5 * (-p->gamma_c) * v;"),
    "loss_factor": ("0.5 * (p->R * nn - p->gamma_c) * v;", "(p->R * nn - p->gamma_c) * v;"),
    "reservoir_depletion": ("(p->gamma_r + p->R * rho) * nn;", "(p->gamma_r + rho) * nn;"),
    "rk4_stage_offset": ("const double a[4] = {0.0, 0.5, 0.5, 1.0};", "const double a[4] = {0.0, 0.5, 1.0, 1.0};"),
    "rk4_weight": ("(k[0][q] + 2.0 * k[1][q] + 2.0 * k[2][q] + k[3][q])", "(k[0][q] + 2.0 * k[1][q] + k[2][q] + 2.0 * k[3][q])"),
    "dp_bhat_coeff": ("393.0 / 640.0", "393.0 / 641.0"),
    "dp_a_coeff": ("-355.0 / 33.0", "-355.0 / 34.0"),
    "kinetic_energy_ghost_link": ("const int ilo = (p->bc_x == ORC_BC_ZERO) ? -1 : 0;", "const int ilo = 0;"),
    "energy_int_half": ("o->e_int = 0.5 * p->g * dA * s_int;", "o->e_int = p->g * dA * s_int;"),
}

# Mistakes in the stochastic part, checked by the noise pins.
NOISE_MUTATIONS = {
    "philox_multiplier": ("M1 = 0xCD9E8D57u", "M1 = 0xCD9E8D59u"),
    "philox_weyl": ("W1 = 0xBB67AE85u", "W1 = 0xBB67AE87u"),
    "philox_rounds": ("round < 10; ++round", "round < 7; ++round"),
    "philox_word_order": ("n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0",
                          "n0 = hi0 ^ c1 ^ k0, n1 = lo0, n2 = hi1 ^ c3 ^ k1, n3 = lo1"),
    "counter_component_cell_swapped": ("ctr[4] = {q >> 1, s,", "ctr[4] = {s, q >> 1,"),
    "pair_shares_words": ("const uint32_t *w = x + 2 * (q & 1);", "const uint32_t *w = x;"),
    "pair_index_not_halved": ("ctr[4] = {q >> 1, s,", "ctr[4] = {q, s,"),
    "box_muller_radius": ("sqrt(-2.0 * log(u1))", "sqrt(-log(u1))"),
    "box_muller_same_angle": ("out[1] = r * sin(two_pi * u2);", "out[1] = r * cos(two_pi * u2);"),
    "noise_cell_area": ("nu * (p->R * nn + p->gamma_c) * dt / (4.0 * dV)", "nu * (p->R * nn + p->gamma_c) * dt / (4.0)"),
    "noise_half": ("* dt / (4.0 * dV);", "* dt / (2.0 * dV);"),
    "noise_gain_dropped": ("nu * (p->R * nn + p->gamma_c)", "nu * (p->gamma_c)"),
    "noise_real_only": ("(xi[0] + I * xi[1])", "(xi[0] + I * xi[0])"),
    "noise_step_index": ("orc_noise(p, psi, n, dt, nu, seed, step0 + k);", "orc_noise(p, psi, n, dt, nu, seed, step0);"),
}


# Mistakes in the coherent drive, checked by the drive pins.
DRIVE_MUTATIONS = {
    "drive_sign": ("f_psi[q] += -(I / p->hbar) * (p->E[q] * phase);", "f_psi[q] += (I / p->hbar) * (p->E[q] * phase);"),
    "drive_phase_sign": ("cexp(-I * p->omega * t)", "cexp(I * p->omega * t)"),
    "drive_hbar_dropped": ("-(I / p->hbar) * (p->E[q] * phase)", "-(I) * (p->E[q] * phase)"),
    "rk4_stage_time": ("rhs_at(p, y, yn, V, P, t + a[s] * dt, k[s], kn[s]);", "rhs_at(p, y, yn, V, P, t, k[s], kn[s]);"),
    "rk4_step_time": ("const double t = p->t0 + (double)step * dt;", "const double t = p->t0;"),
    "dp_node": ("3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0", "3.0 / 10.0, 4.0 / 5.0, 7.0 / 9.0"),
    "dp_attempt_time": ("pt.t0 = ctrl->t;", "pt.t0 = p->t0;"),
    "observables_undriven": ("rhs_at(p, psi, n, V, P, p->t0, fp, fn);", "orc_rhs(p, psi, n, V, P, fp, fn);"),
    "noisy_loop_drive_time": ("pk.t0 = p->t0 + (double)k * dt;", "pk.t0 = p->t0;"),
}


# Mistakes in the imaginary-time propagation, checked by its pins.
IMAG_MUTATIONS = {
    "imag_rotation_sign": ("k[s][q] *= -I;", "k[s][q] *= I;"),
    "imag_rotation_dropped": ("k[s][q] *= -I;", "k[s][q] *= 1.0;"),
    "imag_norm_target": ("const double scale = sqrt(N0 / total_norm(p, psi));",
                         "const double scale = sqrt(1.0 / total_norm(p, psi));"),
    "imag_weights": ("(k[0][q] + 2.0 * k[1][q] + 2.0 * k[2][q] + k[3][q]) * dt;\n        const double scale",
                     "(k[0][q] + 2.0 * k[1][q] + k[2][q] + 2.0 * k[3][q]) * dt;\n        const double scale"),
    "imag_stage_argument": ("                arg = y;", "                arg = psi;"),
}


# Mistakes in the observables that only the dynamics fix, checked by their pins.
OBS_MUTATIONS = {
    "tetm_energy_factor_two": ("s_tetm += 2.0 * creal(conj(pp[k]) * jp);", "s_tetm += creal(conj(pp[k]) * jp);"),
    "tetm_energy_mixed_sign": ("- 2.0 * I * d_xy(p, pm, i, j));", "+ 2.0 * I * d_xy(p, pm, i, j));"),
    "tetm_energy_dyy_sign": ("(d_xx(p, pm, i, j) - d_yy(p, pm, i, j)", "(d_xx(p, pm, i, j) + d_yy(p, pm, i, j)"),
    "cross_energy_zero": ("o->e_cross = p->g_x * dA * s_cross;", "o->e_cross = 0.0 * dA * s_cross;"),
    "cross_energy_half": ("o->e_cross = p->g_x * dA * s_cross;", "o->e_cross = 0.5 * p->g_x * dA * s_cross;"),
    "reservoir_energy_half": ("o->e_res = p->g_r * dA * s_res;", "o->e_res = 0.5 * p->g_r * dA * s_res;"),
    "reservoir_total_area": ("o->reservoir = dA * s_nr;", "o->reservoir = s_nr;"),
    "energy_sum_drops_tetm": ("o->e_cross + o->e_tetm + o->e_res;", "o->e_cross + o->e_res;"),
}


def _run_pins_on_mutant(old, new, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor {old!r} no longer in the oracle source"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new, 1))
    lib = oracle.compile_library(str(mutated), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, PHX_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", pins)],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


@pytest.mark.parametrize("name", sorted(NOISE_MUTATIONS))
def test_noise_pins_reject_planted_mistake(name, tmp_path):
    old, new = NOISE_MUTATIONS[name]
    r = _run_pins_on_mutant(old, new, "test_oracle_noise_pins.py", tmp_path)
    assert r.returncode != 0, f"noise pins passed with planted mistake {name}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(DRIVE_MUTATIONS))
def test_drive_pins_reject_planted_mistake(name, tmp_path):
    old, new = DRIVE_MUTATIONS[name]
    r = _run_pins_on_mutant(old, new, "test_oracle_drive_pins.py", tmp_path)
    assert r.returncode != 0, f"drive pins passed with planted mistake {name}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(IMAG_MUTATIONS))
def test_imag_pins_reject_planted_mistake(name, tmp_path):
    old, new = IMAG_MUTATIONS[name]
    r = _run_pins_on_mutant(old, new, "test_oracle_imag_pins.py", tmp_path)
    assert r.returncode != 0, f"imaginary-time pins passed with planted mistake {name}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path):
    old, new = MUTATIONS[name]
    r = _run_pins_on_mutant(old, new, "test_oracle_pins.py", tmp_path)
    assert r.returncode != 0, f"pins passed with planted mistake {name}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(OBS_MUTATIONS))
def test_observable_pins_reject_planted_mistake(name, tmp_path):
    old, new = OBS_MUTATIONS[name]
    r = _run_pins_on_mutant(old, new, "test_oracle_observable_pins.py", tmp_path)
    assert r.returncode != 0, f"observable pins passed with planted mistake {name}:\n{r.stdout[-2000:]}"
