"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of the oracle source (a dropped factor,
a flipped sign, an index off by one), builds it with gcc into a temporary
directory, and checks that at least one pin fails on it.  Runs on the CPU only.
"""
import importlib.util
import os
import subprocess
import sys

import numpy as np
import pytest

from tests import test_oracle_dense as TD
from tests import test_oracle_dispersion as TP
from tests import test_oracle_energy_sum as TE
from tests import test_oracle_invariants as TI
from tests import test_oracle_witness as TW
from tests import test_oracle_yee as TY

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "tete_oracle.c")
PY = os.path.join(os.path.dirname(HERE), "oracle", "oracle.py")

MUTANTS = {
    # S3 with alpha instead of 2 alpha
    "ez_half_weight": ("upd_ez(g, m, f, 2.0 * a, jz);", "upd_ez(g, m, f, a, jz);",
                       [lambda o: TD.test_ten_updates_equal_dense_scheme(o, 0)]),
    # S4/S5 left out (TM group half-updated)
    "no_second_h_half": ("    upd_hx(g, m, f, a);                /* S4", "    (void)0;                /* S4",
                         [lambda o: TD.test_ten_updates_equal_dense_scheme(o, 0),
                          lambda o: TI.test_energy_conserved_without_current(o, False)]),
    # wrong sign of P_z e_y in S1/S4
    "hx_pz_sign": ("f[HX][idx(g, i, j, k)] += a * m[HX][idx(g, i, j, k)] * (pz_ey - py_ez);",
                   "f[HX][idx(g, i, j, k)] += a * m[HX][idx(g, i, j, k)] * (-pz_ey - py_ez);",
                   [lambda o: TP.test_one_step_eigenvalues_follow_27(o)]),
    # transposed difference taken forward instead of backward in S6/S9
    "ex_pyt_index": ("double pyt_hz = at(g, f, HZ, i, j - 1, k) - at(g, f, HZ, i, j, k);",
                     "double pyt_hz = at(g, f, HZ, i, j, k) - at(g, f, HZ, i, j + 1, k);",
                     [lambda o: TD.test_ten_updates_equal_dense_scheme(o, 0)]),
    # cross term of W^{n,e} with the wrong sign
    "energy_cross_sign": ("return 0.5 * total(&sq) - 0.5 * a * a * (total(&r0) + total(&r1)) + a * total(&lc);",
                          "return 0.5 * total(&sq) - 0.5 * a * a * (total(&r0) + total(&r1)) - a * total(&lc);",
                          [lambda o: TD.test_energy_is_half_yQy(o, 0)]),
    # energy R-term with + alpha^2 (the sign the paper prints)
    "energy_r_sign": ("return 0.5 * total(&sq) - 0.5 * a * a * (total(&r0) + total(&r1)) + a * total(&lc);",
                      "return 0.5 * total(&sq) + 0.5 * a * a * (total(&r0) + total(&r1)) + a * total(&lc);",
                      [lambda o: TD.test_energy_is_half_yQy(o, 0)]),
    # energy summed without the compensation (a plain running sum)
    "energy_plain_sum": ("static double total(const orc_sum* a) { return a->s + a->c; }",
                         "static double total(const orc_sum* a) { return a->s; }",
                         [lambda o: TE.test_energy_sum_is_exactly_rounded_to_a_few_ulp(o)]),
    # charge with (I + alpha^2 r_0)
    "charge_r_sign": ("return e0 / kap - a * a * r;", "return e0 / kap + a * a * r;",
                      [lambda o: TI.test_gauss_law_moving_bunch(o)]),
    # current with the sign printed in the scaled forms
    "current_sign": ("(pyt_hx - pxt_hy - src);", "(pyt_hx - pxt_hy + src);",
                     [lambda o: TI.test_gauss_law_moving_bunch(o)]),
    # bunch one cell late
    "bunch_late": ("int mm = k - n + b->M;", "int mm = k - n + 1 + b->M;",
                   [lambda o: TI.test_gauss_law_moving_bunch(o)]),
    # wake sample taken one step early
    "wake_index": ("int jj = n - k - b->M;", "int jj = n - k - b->M + 1;",
                   [lambda o: TI.test_wake_energy_identity(o)]),
    # staircase rule misses one adjacent cell
    "pec_rule": ("cell_is_pec(g, cell_pec, i, j - 1, k) || cell_is_pec(g, cell_pec, i, j, k);\n        m[EX]",
                 "cell_is_pec(g, cell_pec, i, j, k);\n        m[EX]",
                 [lambda o: TI.test_staircase_pec_edges_are_cell_edges(o)]),
    # Yee: half the time step in the updates
    "yee_half_step": ("    const double dt = g->cdt;\n    upd_ex(g, m, f, dt, NULL);",
                      "    const double dt = 0.5 * g->cdt;\n    upd_ex(g, m, f, dt, NULL);",
                      [lambda o: TY.test_yee_eigenvalues_follow_9(o),
                       lambda o: TY.test_yee_transversely_uniform_pulse(o)]),
    # Yee: h updated before e (the order of (7) reversed)
    "yee_h_first": ("    upd_ex(g, m, f, dt, NULL);          /* e_x^{n+1/2} */\n"
                    "    upd_ey(g, m, f, dt, NULL);          /* e_y^{n+1/2} */\n"
                    "    upd_ez(g, m, f, dt, jz);            /* e_z^{n+1/2} */\n",
                    "    upd_hx(g, m, f, dt);\n    upd_hy(g, m, f, dt);\n    upd_hz(g, m, f, dt);\n"
                    "    upd_ex(g, m, f, dt, NULL);          /* e_x^{n+1/2} */\n"
                    "    upd_ey(g, m, f, dt, NULL);          /* e_y^{n+1/2} */\n"
                    "    upd_ez(g, m, f, dt, jz);            /* e_z^{n+1/2} */\n    return;\n",
                    [lambda o: TY.test_yee_transversely_uniform_pulse(o),
                     lambda o: TY.test_yee_leapfrog_invariant_conserved(o)]),
    # Yee invariant with |e^{n+1/2}|^2 instead of the cross product
    "yee_invariant_square": ("if (kap > 0.0) s += fo[c][idx(g, i, j, k)] * fn[c][idx(g, i, j, k)] / kap;",
                             "if (kap > 0.0) s += fn[c][idx(g, i, j, k)] * fn[c][idx(g, i, j, k)] / kap;",
                             [lambda o: TY.test_yee_leapfrog_invariant_conserved(o)]),
}


def _load_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new)
    c = tmp_path / (name + ".c")
    c.write_text(src)
    so = tmp_path / (name + ".so")
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    spec = importlib.util.spec_from_file_location("oracle_mutant_" + name, PY)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    mod.LIB = str(so)
    mod._lib = None
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new, pins = MUTANTS[name]
    mod = _load_mutant(tmp_path, name, old, new)
    caught = 0
    for pin in pins:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, FloatingPointError, ValueError, np.linalg.LinAlgError):
            caught += 1
    assert caught >= 1, "no pin caught mutant %s" % name


# ---- the r-z oracle (Python): each mutant is a list of (old, new) first-occurrence edits
from tests import test_oracle_rz as TZ

RZ_SRC = os.path.join(os.path.dirname(HERE), "oracle", "rz_oracle.py")

RZ_MUTANTS = {
    # the implicit factors with the subscripts as printed (swapped between e_z and h_z)
    "rz_printed_factor_order": ([('m["ez"] * m["hr"])                 # S3', 'm["hz"] * m["er"])                 # S3'),
                                 ('m["hz"] * m["er"])                 # S8', 'm["ez"] * m["hr"])                 # S8')],
                                [lambda z: TZ.test_rz_energy_conserved(z, 1)]),
    # azimuthal coupling of h_r with the wrong sign
    "rz_hr_m_sign": ([('(-pz(f["ephi"]) + M * f["ez"])', '(-pz(f["ephi"]) - M * f["ez"])')],
                     [lambda z: TZ.test_rz_energy_conserved(z, 1),
                      lambda z: TZ.test_rz_tm_modes_converge_second_order(z, 1)]),
    # on-axis dual facet taken as dr^2 / 4
    "rz_axis_area": ([("dz / (dr * dr / 8.0)", "dz / (dr * dr / 4.0)")],
                     [lambda z: TZ.test_rz_facets_tile_the_cross_section(z)]),
    # kappa_r at the node radius instead of r_{j+1/2}
    "rz_kappa_r_radius": ([('m["er"] = dr / (rh * dz)', 'm["er"] = dr / (np.maximum(r, dr) * dz)')],
                          [lambda z: TZ.test_rz_modes_with_z_variation(z, "TE", 1, 1)]),
    # current with the sign printed in (24)
    "rz_current_sign": ([('- M * f["hr"] - Jz)', '- M * f["hr"] + Jz)')],
                        [lambda z: TZ.test_rz_gauss_law_ring_bunch(z, 1, 3, 1.0)]),
    # radial difference of h_z in the energy taken forward
    "rz_energy_r1": ([('m["ephi"] * prs(f["hz"]) ** 2', 'm["ephi"] * pr(f["hz"]) ** 2')],
                     [lambda z: TZ.test_rz_energy_conserved(z, 1)]),
    # charge with + alpha^2
    "rz_charge_alpha": ([("ez * _inv(m[\"ez\"]) - a * a * rz", "ez * _inv(m[\"ez\"]) + a * a * rz")],
                        [lambda z: TZ.test_rz_gauss_law_ring_bunch(z, 1, 3, 1.0)]),
    # wake sample one step early
    "rz_wake_index": ([("jj = n - k - bunch.M", "jj = n - k - bunch.M + 1")],
                      [lambda z: TZ.test_rz_wake_energy_identity(z, 1)]),
    # Yee with half the step
    "rz_yee_half_step": ([("    dt = g.cdt\n    M = g.m", "    dt = 0.5 * g.cdt\n    M = g.m")],
                         [lambda z: TZ.test_rz_stability_independent_of_m(z)]),
    # the axis treated as a wall
    "rz_axis_wall": ([("cell[0, :] = cell[1, :]", "cell[0, :] = True")],
                     [lambda z: TZ.test_rz_tm_modes_converge_second_order(z, 0)]),
    # Panofsky-Wenzel with a one-sided sum instead of the trapezoid
    "rz_pw_rule": ([("np.cumsum(0.5 * (D[1:] + D[:-1]))", "np.cumsum(D[1:])")],
                   [lambda z: TZ.test_rz_transverse_wake_matches_lorentz_force(z)]),
}


def _load_rz_mutant(tmp_path, name, edits):
    src = open(RZ_SRC).read()
    for old, new in edits:
        assert src.count(old) >= 1, (name, old)
        src = src.replace(old, new, 1)
    p = tmp_path / (name + ".py")
    p.write_text(src)
    spec = importlib.util.spec_from_file_location("rz_mutant_" + name, str(p))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(RZ_MUTANTS))
def test_rz_pins_catch_planted_mistake(tmp_path, name):
    edits, pins = RZ_MUTANTS[name]
    mod = _load_rz_mutant(tmp_path, name, edits)
    caught = 0
    for pin in pins:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, FloatingPointError, ValueError, np.linalg.LinAlgError):
            caught += 1
    assert caught >= 1, "no pin caught mutant %s" % name


# ---- the implicit oracle (Python), same harness as the r-z one
from tests import test_oracle_implicit as TIM

IM_SRC = os.path.join(os.path.dirname(HERE), "oracle", "implicit_oracle.py")

IM_MUTANTS = {
    # transverse coupling of e_z to h_y with the wrong sign
    "imp_t0_sign": ([('(EZ, HY, "pxt", -1.0, "ka")', '(EZ, HY, "pxt", +1.0, "ka")')],
                    [lambda z: TIM.test_implicit_eigenvalues_follow_the_dispersion_relation(z),
                     lambda z: TIM.test_implicit_energy_law(z)]),
    # the explicit half of the transverse operator dropped (backward Euler in T_0)
    "imp_no_mean_t0": ([("self.P0 = (I + self.a * self.T0).tocsr()", "self.P0 = I.tocsr()"),
                        ("self.lu0 = spla.splu((I - self.a * self.T0).tocsc())",
                         "self.lu0 = spla.splu((I - 2 * self.a * self.T0).tocsc())")],
                       [lambda z: TIM.test_implicit_eigenvalues_follow_the_dispersion_relation(z)]),
    # coupling -L^T with the wrong sign on e_x
    "imp_lt_sign": ([('(EX, HY, "pzt", +1.0, "ka")', '(EX, HY, "pzt", -1.0, "ka")')],
                    [lambda z: TIM.test_implicit_transversely_uniform_pulse(z),
                     lambda z: TIM.test_implicit_energy_law(z)]),
    # current with the sign printed in the scaled forms
    "imp_current_sign": ([("rhs[2 * self.n:] -= dt", "rhs[2 * self.n:] += dt")],
                         [lambda z: TIM.test_implicit_gauss_law(z)]),
    # energy cross term with the wrong sign
    "imp_energy_cross": ([("return s + a * float(lc)", "return s - a * float(lc)")],
                         [lambda z: TIM.test_implicit_energy_law(z)]),
    # charge without the time average of the transverse fluxes
    "imp_charge_no_mean": ([("dx = 0.5 * (d(fo, EX) + d(fn, EX))", "dx = d(fn, EX)")],
                           [lambda z: TIM.test_implicit_gauss_law(z)]),
}


def _load_im_mutant(tmp_path, name, edits):
    src = open(IM_SRC).read()
    for old, new in edits:
        assert src.count(old) >= 1, (name, old)
        src = src.replace(old, new, 1)
    p = tmp_path / (name + ".py")
    p.write_text(src)
    spec = importlib.util.spec_from_file_location("im_mutant_" + name, str(p))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(IM_MUTANTS))
def test_implicit_pins_catch_planted_mistake(tmp_path, name):
    edits, pins = IM_MUTANTS[name]
    mod = _load_im_mutant(tmp_path, name, edits)
    caught = 0
    for pin in pins:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, FloatingPointError, ValueError, np.linalg.LinAlgError, RuntimeError):
            caught += 1
    assert caught >= 1, "no pin caught mutant %s" % name


WO_SRC = os.path.join(os.path.dirname(HERE), "oracle", "witness_oracle.py")

WO_MUTANTS = {
    # the quadrature one sample late
    "wo_time_index": ([("js = n - k - bunch.M", "js = n + 1 - k - bunch.M")],
                      [lambda w: TW.test_centre_line_is_the_bunch_line_wake(w),
                       lambda w: TW.test_witness_causality(w)]),
    # only the new level of e_z in the quadrature
    "wo_no_average": ([("-0.5 * (old[l][ok] + new[ok])", "-1.0 * new[ok]")],
                      [lambda w: TW.test_centre_line_is_the_bunch_line_wake(w)]),
    # the -x and +x neighbours swapped
    "wo_swapped_x": ([("OFFSETS = ((0, 0), (-1, 0), (1, 0),", "OFFSETS = ((0, 0), (1, 0), (-1, 0),")],
                     [lambda w: TW.test_transverse_wake_matches_lorentz_force(w)]),
    # a neighbour line two cells out
    "wo_far_y": ([("(0, -1), (0, 1))", "(0, -2), (0, 1))")],
                 [lambda w: TW.test_mirror_symmetry_of_off_axis_wakes(w),
                  lambda w: TW.test_transverse_wake_matches_lorentz_force(w)]),
    # one-cell difference taken as the centred one
    "wo_half_width": ([("(W[2] - W[1]) / (2.0 * dx)", "(W[2] - W[1]) / dx")],
                      [lambda w: TW.test_transverse_wake_matches_lorentz_force(w)]),
    # rectangle rule instead of the trapezoid, one sample late
    "wo_rectangle": ([("out[1:] = np.cumsum(0.5 * (D[1:] + D[:-1])) * ds", "out[1:] = np.cumsum(D[:-1]) * ds")],
                     [lambda w: TW.test_transverse_wake_matches_lorentz_force(w)]),
}


@pytest.mark.parametrize("name", sorted(WO_MUTANTS))
def test_witness_pins_catch_planted_mistake(tmp_path, name):
    edits, pins = WO_MUTANTS[name]
    src = open(WO_SRC).read()
    for old, new in edits:
        assert src.count(old) >= 1, (name, old)
        src = src.replace(old, new, 1)
    p = tmp_path / (name + ".py")
    p.write_text(src)
    spec = importlib.util.spec_from_file_location("wo_mutant_" + name, str(p))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    caught = 0
    for pin in pins:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, FloatingPointError, ValueError):
            caught += 1
    assert caught >= 1, "no pin caught mutant %s" % name


# ---- the open-pipe oracle (Python), same harness
from tests import test_oracle_pipe as TPI
from tests import test_oracle_pipe_closed as TPC

PI_SRC = os.path.join(os.path.dirname(HERE), "oracle", "pipe_oracle.py")

PI_MUTANTS = {
    # h taken at the same time level as e (no half-step stagger)
    "pipe_h_stagger": ([("Fh = profile(lam, M, g.cdt, k + 1 - n0)", "Fh = profile(lam, M, g.cdt, k - n0)")],
                       [lambda p: TPI.test_self_field_moves_one_cell_per_step(p, 5, 7, 1.0)]),
    # the x and y weights of the cross-section's operator swapped
    "pipe_weights_swapped": ([("wx, wy = g.dy / g.dx, g.dx / g.dy", "wx, wy = g.dx / g.dy, g.dy / g.dx")],
                             [lambda p: TPI.test_potential_matches_discrete_sine_series(p)]),
    # the profile's mean tied to half the current
    "pipe_profile_half": ([("F[q] = 2.0 * cur - F[q + 1]", "F[q] = cur - F[q + 1]")],
                          [lambda p: TPI.test_self_field_node_charges_are_the_bunch(p),
                           lambda p: TPC.test_3d_step_out_open_pipes_equal_closed_box_limit(p)]),
    # h_y with the wrong sign
    "pipe_hy_sign": ([('f["hy"][:-1, :, :-1] = ((g.dy / g.dx) * Ex)', 'f["hy"][:-1, :, :-1] = (-(g.dy / g.dx) * Ex)')],
                     [lambda p: TPI.test_self_field_moves_one_cell_per_step(p, 5, 7, 1.0)]),
    # the bunch cells one cell late in the profile
    "pipe_cell_offset": ([("cur = lam[q + 2 * M] / dtau if q >= -2 * M else 0.0",
                           "cur = lam[q + 2 * M - 1] / dtau if q >= -2 * M + 1 else 0.0")],
                         [lambda p: TPI.test_self_field_node_charges_are_the_bunch(p)]),
    # r-z: the azimuthal term of the radial problem left out
    "rz_pipe_no_m2": ([("diag = (rm + rp) / g.dr + (g.m * g.m * g.dr / (j * g.dr) if j > 0 else 0.0)",
                        "diag = (rm + rp) / g.dr")],
                      [lambda p: TPI.test_rz_self_field_moves_one_cell_per_step(p, 1, 4)]),
    # r-z: h_r with the wrong sign
    "rz_pipe_hr_sign": ([("hr = np.where(j > 0, (g.dr / (j * g.dr)) * Ep, 0.0)",
                          "hr = np.where(j > 0, -(g.dr / (j * g.dr)) * Ep, 0.0)")],
                        [lambda p: TPI.test_rz_self_field_moves_one_cell_per_step(p, 1, 4)]),
    # r-z: h_phi tied to e_r at the node radius instead of r_{j+1/2}
    "rz_pipe_hphi_radius": ([("((j + 0.5) * g.dr / g.dr)", "((j + 0.0) * g.dr / g.dr)")],
                            [lambda p: TPI.test_rz_self_field_moves_one_cell_per_step(p, 0, 0),
                             lambda p: TPC.test_rz_step_out_open_pipes_equal_closed_box_limit(p)]),
}


@pytest.mark.parametrize("name", sorted(PI_MUTANTS))
def test_pipe_pins_catch_planted_mistake(tmp_path, name):
    edits, pins = PI_MUTANTS[name]
    src = open(PI_SRC).read()
    for old, new in edits:
        assert src.count(old) >= 1, (name, old)
        src = src.replace(old, new, 1)
    p = tmp_path / (name + ".py")
    p.write_text(src)
    spec = importlib.util.spec_from_file_location("pi_mutant_" + name, str(p))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    caught = 0
    for pin in pins:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except (AssertionError, FloatingPointError, ValueError):
            caught += 1
    assert caught >= 1, "no pin caught mutant %s" % name
