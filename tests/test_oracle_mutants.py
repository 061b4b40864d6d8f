"""Planted mistakes in a copy of the oracle: every one must fail a pin.

Each case copies ``oracle/oracle.c``, replaces one expression with a
plausible mistake (a flipped sign, a dropped factor or term, a shifted index,
a wrong time level, a transposed operand), builds the copy with the oracle's
own build recipe, and runs the pins that should catch it against that build
through a separate instance of the oracle's ctypes wrapper.  A case passes
when at least one of its pins fails; an unmodified copy, built and loaded the
same way, passes all of them (the control case at the end).  This is what
makes the pins a check of the oracle rather than a restatement of it.
"""
import importlib.util
import os

import pytest

import test_oracle_adjoint as ta
import test_oracle_cpml as tc
import test_oracle_fields as tf
import test_oracle_particles as tp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
WRAPPER = os.path.join(ROOT, "oracle", "pic_oracle.py")

CAVITY = lambda m: tf.test_pec_cavity_mode_is_exact_discrete_eigenmode(m, (1, 2, 1))  # noqa: E731
CAVITY2 = lambda m: tf.test_pec_cavity_mode_is_exact_discrete_eigenmode(m, (2, 1, 3))  # noqa: E731
PLANE = lambda m: tf.test_periodic_plane_wave_phase_advance(m)  # noqa: E731
MATRIX_P = lambda m: tf.test_step_matrix_equals_incidence_assembly(m, (True, False, True))  # noqa: E731
PLASMA = lambda m: tf.test_lossless_plasma_oscillation_closed_form(m)  # noqa: E731
DAMPED = lambda m: tf.test_damped_drude_mode_follows_eq6_eq8_recurrence(m)  # noqa: E731
COLLIDE = lambda m: tf.test_collisional_damping_and_frequency(m)  # noqa: E731
ROTATE = lambda m: tp.test_boris_pure_magnetic_rotation(m)  # noqa: E731
IMPULSE = lambda m: tp.test_boris_pure_electric_impulse(m)  # noqa: E731
GATHER = lambda m: tp.test_gather_is_exact_on_affine_fields(m)  # noqa: E731
FREE = lambda m: tp.test_free_particle_moves_at_u_over_gamma(m)  # noqa: E731
DEPOSIT = lambda m: tp.test_single_move_deposit_conserves_charge(m, (0.7, -0.4, 0.25))  # noqa: E731
GAUSS_METAL = lambda m: tp.test_gauss_law_with_metal_polarization(m)  # noqa: E731
PROBE = lambda m: tp.test_probe_dft_of_exact_cavity_mode(m)  # noqa: E731
TRANSPOSE = lambda m: [ta.test_adjoint_step_is_transpose_blockwise(m, c) for c in range(len(ta.CASES))]  # noqa: E731
FD = lambda m: ta.test_gradient_matches_central_differences(m)  # noqa: E731
CPML = lambda m: tp.test_cpml_reflection_below_minus_40_db(m)  # noqa: E731
UNIFORM = lambda m: tc.test_uniform_cpml_every_axis_and_polarisation(m)  # noqa: E731
KENERGY = lambda m: tc.test_kappa_graded_layers_conserve_the_weighted_yee_energy(m)  # noqa: E731
KERNEL = lambda m: tc.test_cpml_coefficients_are_the_recursive_convolution_of_the_kernel(m)  # noqa: E731
DIAG = lambda m: tc.test_diagnostics_by_hand(m)  # noqa: E731

# (name, original text, planted mistake, pins expected to catch it)
MUTANTS = [
    ("H curl: sign of the z difference in Hx",
     "AT(Hx, i, j, k) -= ch * (dy - dz);", "AT(Hx, i, j, k) -= ch * (dy + dz);", [CAVITY, MATRIX_P]),
    ("E curl: x and y differences swapped in Ez",
     "AT(Ez, i, j, k) += ce * (dx - dy) -", "AT(Ez, i, j, k) += ce * (dy - dx) -", [CAVITY2, MATRIX_P]),
    ("periodic wrap: Ex reads H at j instead of j - 1",
     "int jm = wrap(s, 1, j - 1), km = wrap(s, 2, k - 1);\n                double dy = AT(Hz, i, j, k) - AT(Hz, i, jm, k);",
     "int jm = wrap(s, 1, j), km = wrap(s, 2, k - 1);\n                double dy = AT(Hz, i, j, k) - AT(Hz, i, jm, k);",
     [PLANE, MATRIX_P]),
    ("Eq. 6: factor 2 dropped from cb",
     "*cb = 2.0 * dt * OR_EPS0 * wp * wp / (2.0 + g * dt);",
     "*cb = dt * OR_EPS0 * wp * wp / (2.0 + g * dt);", [PLASMA, DAMPED]),
    ("Eq. 6: sign of the damping term in ca",
     "*ca = (2.0 - g * dt) / (2.0 + g * dt);", "*ca = (2.0 + g * dt) / (2.0 - g * dt);", [COLLIDE, DAMPED]),
    ("Eq. 6: J driven by the updated E instead of E^n",
     "AT(s->cb[0], i, j, k) * AT(Ex, i, j, k);",
     "AT(s->cb[0], i, j, k) * (AT(Ex, i, j, k) + ce * (dy - dz));", [DAMPED, MATRIX_P]),
    ("Eq. 8: polarization current dropped from Ez",
     "AT(Ez, i, j, k) += ce * (dx - dy) - cj * (jn + AT(s->Jb[2], i, j, k));",
     "AT(Ez, i, j, k) += ce * (dx - dy) - cj * AT(s->Jb[2], i, j, k);", [GAUSS_METAL, MATRIX_P]),
    ("Boris: rotation factor 2 / (1 + t^2) halved",
     "sv[a] = 2.0 * t[a] / (1.0 + t2);", "sv[a] = t[a] / (1.0 + t2);", [ROTATE]),
    ("Boris: second half kick dropped",
     "for (int a = 0; a < 3; ++a) u[a] = uq[a] + h * E[a];", "for (int a = 0; a < 3; ++a) u[a] = uq[a];",
     [IMPULSE]),
    ("move: non-relativistic velocity u instead of u / gamma",
     "X1[a] = (pos[a] + s->dt * u[a] / g) / dx;", "X1[a] = (pos[a] + s->dt * u[a]) / dx;", [FREE]),
    ("gather: E component sampled on the node lattice",
     "oe[c] = 0.5;", "oe[c] = 0.0;", [GATHER]),
    ("gather: B from the new H level only",
     "B[c] = OR_MU0 * 0.5 * (interp(s, &s->Hprev[c], oh, X) + interp(s, &s->H[c], oh, X));",
     "B[c] = OR_MU0 * interp(s, &s->H[c], oh, X);", [GATHER]),
    ("Esirkepov: transverse weight dS dS' / 3 written as / 4 in Jx",
     "acc += dS[0][m] * (S0[1][b] * S0[2][c] + 0.5 * dS[1][b] * S0[2][c] +\n"
     "                                   0.5 * S0[1][b] * dS[2][c] + dS[1][b] * dS[2][c] / 3.0);",
     "acc += dS[0][m] * (S0[1][b] * S0[2][c] + 0.5 * dS[1][b] * S0[2][c] +\n"
     "                                   0.5 * S0[1][b] * dS[2][c] + dS[1][b] * dS[2][c] / 4.0);",
     [DEPOSIT]),
    ("deposit: current prefactor off by a factor dx",
     "const double f = -qw / (s->dt * s->dx * s->dx);", "const double f = -qw / (s->dt * s->dx);",
     [DEPOSIT]),
    ("probe DFT: sign of the phase",
     "s->fim[p * s->nfreq + f] -= s->dt * ez * sin(th);", "s->fim[p * s->nfreq + f] += s->dt * ez * sin(th);",
     [PROBE]),
    ("probe DFT: phase one step early",
     "const double t = (double)s->step * s->dt;", "const double t = (double)(s->step - 1) * s->dt;", [PROBE]),
    ("adjoint: Drude factor ca dropped from the J adjoint",
     "AT(s->Ja[c], i, j, k) = AT(s->ca[c], i, j, k) * jt;", "AT(s->Ja[c], i, j, k) = jt;", [TRANSPOSE, FD]),
    ("adjoint: sign of the shifted face's weight",
     "AT(s->Ha[a2], m1[0], m1[1], m1[2]) -= t1;", "AT(s->Ha[a2], m1[0], m1[1], m1[2]) += t1;", [TRANSPOSE]),
    ("gradient: cb's factor taken from J instead of E^n",
     "gcb[q] += jt * En[q];", "gcb[q] += jt * Jn[q];", [FD]),
    ("CPML: sign of the memory coefficient c",
     "*c = (sig > 0.0) ? sig * (*b - 1.0) /", "*c = (sig > 0.0) ? sig * (1.0 - *b) /", [CPML, KERNEL]),
    ("CPML: conductivity grading reversed (largest at the interface)",
     "const double sig = smax * pow(r, m);", "const double sig = smax * pow(1.0 - r, m);", [CPML, KERNEL]),
    ("CPML: memory used before its update (Hz, x derivative)",
     "*p = s->bH[0][i] * *p + s->cH[0][i] * dx;\n                    dx = dx / s->kH[0][i] + *p;\n"
     "                }\n                if (s->lH[1][j]) {\n                    double *p = &AT(s->psiH[2][1]",
     "const double old_ = *p;\n                    *p = s->bH[0][i] * *p + s->cH[0][i] * dx;\n"
     "                    dx = dx / s->kH[0][i] + old_;\n"
     "                }\n                if (s->lH[1][j]) {\n                    double *p = &AT(s->psiH[2][1]",
     [UNIFORM]),
    ("CPML: 1/kappa applied to the memory as well (Ey, z derivative)",
     "double *p = &AT(s->psiE[1][2], i, j, k);\n                    *p = s->bE[2][k] * *p + s->cE[2][k] * dz;\n"
     "                    dz = dz / s->kE[2][k] + *p;",
     "double *p = &AT(s->psiE[1][2], i, j, k);\n                    *p = s->bE[2][k] * *p + s->cE[2][k] * dz;\n"
     "                    dz = (dz + *p) / s->kE[2][k];",
     [UNIFORM]),
    ("CPML: H-type coefficients sampled at the nodes instead of the half nodes",
     "cpml_coeff(s, a, i + 0.5, pml,", "cpml_coeff(s, a, (double)i, pml,", [KENERGY, KERNEL]),
    ("diagnostics: periodic copies counted in the field energy",
     "if (s->bc[a] == OR_PERIODIC && id[a] == s->n[a]) dup = 1;",
     "if (s->bc[a] == OR_PERIODIC && id[a] > s->n[a]) dup = 1;", [DIAG]),
]


def _wrapper_for(lib, tag):
    """A separate instance of the oracle's ctypes wrapper bound to `lib`."""
    spec = importlib.util.spec_from_file_location(f"pic_oracle_planted_{tag}", WRAPPER)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.LIB_PATH = lib
    return mod


@pytest.mark.parametrize("case", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(case, tmp_path):
    from oracle import build as obuild

    name, old, new, pins = MUTANTS[case]
    src = open(SRC).read()
    assert src.count(old) == 1, f"pattern of '{name}' must occur once in oracle.c"
    path = tmp_path / "oracle_planted.c"
    path.write_text(src.replace(old, new))
    lib = obuild.build(src=str(path), lib=str(tmp_path / "liboracle_planted.so"))
    mod = _wrapper_for(lib, case)
    caught = []
    for pin in pins:
        try:
            pin(mod)
        except AssertionError:
            caught.append(pin)
    assert caught, f"no pin fails with the planted mistake: {name}"


def test_unmodified_copy_passes_every_pin(tmp_path):
    """Control for the harness: the same copy, build and wrapper instance
    without a planted mistake passes every pin the cases use."""
    from oracle import build as obuild

    path = tmp_path / "oracle_copy.c"
    path.write_text(open(SRC).read())
    lib = obuild.build(src=str(path), lib=str(tmp_path / "liboracle_copy.so"))
    mod = _wrapper_for(lib, "control")
    pins = []
    for _, _, _, ps in MUTANTS:
        pins += [p for p in ps if p not in pins]
    for pin in pins:
        pin(mod)
