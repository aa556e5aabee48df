"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a copy of the oracle -- a dropped term,
a flipped sign, a transposed operand, a wrong index, window or tie rule, the wrong
Jacobi partner, a wrong control rule -- builds it, and runs the pins that must
catch it against that build (through UCAC_ORACLE_LIB, in a child pytest).  The
test fails if a mutant passes its pins: every mistake listed here is caught by at
least one pin that does not use the oracle as its own reference.  Mistakes in the
network oracle (oracle/mlp.py) are planted in-process by replacing its functions.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ucac_oracle.c")

CTRL = "tests/test_oracle_control.py"
BLK = "tests/test_oracle_blocks.py"
DPT = "tests/test_oracle_dp.py"
SOL = "tests/test_oracle_solve.py"
ADP = "tests/test_oracle_adapt.py"
UCW = "tests/test_oracle_ucwarm.py"

# (name, text in the oracle, replacement, occurrence, pins that must fail)
MUTATIONS = [
    # reported objective (eq:uc-acopf cost)
    ("objective_no_startup", "P->csu[g] * S->usu[k] + ", "", 0, [f"{CTRL}::test_objective_matches_cost_definition"]),
    ("objective_no_kappa1", "obj += P->k2[g] * p * p + P->k1[g] * p;", "obj += P->k2[g] * p * p;", 0,
     [f"{CTRL}::test_objective_matches_cost_definition"]),
    ("objective_no_noload", "obj += P->cnl[g] * S->uon[k] + ", "obj += ", 0,
     [f"{CTRL}::test_objective_matches_cost_definition"]),
    ("objective_no_shutdown", " + P->csd[g] * S->usd[k];", ";", 0,
     [f"{CTRL}::test_objective_matches_cost_definition"]),
    ("cost_units_kappa2", "net->gen_c2[g] * base * base", "net->gen_c2[g] * base", 0,
     [f"{CTRL}::test_objective_matches_cost_definition", f"{SOL}::test_single_bus_economic_dispatch"]),
    # residuals and the inner/outer control (Alg. alg:basic, step:outer)
    ("rd_bus_duplicates_only", "S->sc[SC_RD] = fmax(fmax(d_va, d_fl), fmax(fmax(d_pb, d_qb), d_ub));",
     "S->sc[SC_RD] = d_va;", 0, [f"{CTRL}::test_residuals_recomputed_from_two_states"]),
    ("rin_without_z_lines", "rin = fmax(rin, fabs(a[r] + z));", "rin = fmax(rin, fabs(a[r]));", 0,
     [f"{CTRL}::test_residuals_recomputed_from_two_states"]),
    ("rp_with_z_units", "rp = fmax(rp, fabs(a[r]));", "rp = fmax(rp, fabs(a[r] + z));", 1,
     [f"{CTRL}::test_residuals_on_plain_trajectory"]),
    ("inner_rule_uses_rp", "if (fmax(S->sc[SC_RIN], S->sc[SC_RD]) <= eps_inner(P)",
     "if (fmax(S->sc[SC_RP], S->sc[SC_RD]) <= eps_inner(P)", 0, [f"{CTRL}::test_inner_loop_exit_rule"]),
    ("inner_eps_decays_4k", "P->par.eps_in0 * pow(2.0, -k)", "P->par.eps_in0 * pow(4.0, -k)", 0,
     [f"{CTRL}::test_inner_loop_exit_rule"]),
    ("inner_eps_floor_tol", "fmax(0.5 * P->par.tol,", "fmax(P->par.tol,", 0, [f"{CTRL}::test_inner_loop_exit_rule"]),
    ("max_inner_off_by_one", "S->sc[SC_LIN] >= (double)P->par.max_inner", "S->sc[SC_LIN] > (double)P->par.max_inner", 0,
     [f"{CTRL}::test_inner_loop_exit_rule"]),
    ("beta_rule_reversed", "if (S->sc[SC_ZINF] > P->par.theta * S->sc[SC_ZPREV])",
     "if (S->sc[SC_ZINF] < P->par.theta * S->sc[SC_ZPREV])", 0, [f"{SOL}::test_beta_rule_trace"]),
    ("lambda_update_sign", "S->lB[r][k] + beta * S->zB[r][k]", "S->lB[r][k] - beta * S->zB[r][k]", 0,
     [f"{BLK}::test_outer_update_lambda"]),
    ("z_update_without_lambda", "double z = -(S->lG[r][k] + S->yG[r][k] + rho * a[r])", "double z = -(S->yG[r][k] + rho * a[r])",
     0, [f"{CTRL}::test_z_update_with_nonzero_lambda"]),
    ("z_update_beta_dropped", "double z = -(S->lB[r][k] + S->yB[r][k] + rho * a[r]) / (beta + rho);",
     "double z = -(S->lB[r][k] + S->yB[r][k] + rho * a[r]) / rho;", 0, [f"{CTRL}::test_z_update_with_nonzero_lambda"]),
    ("y_update_without_z", "S->yB[r][k] += rho * (a[r] + z);", "S->yB[r][k] += rho * a[r];", 0,
     [f"{BLK}::test_z_and_y_updates"]),
    # the UC dynamic program (Alg. dp_algo)
    ("dp_tie_switches", "if (c_stay <= c_switch)", "if (c_stay < c_switch)", 0, [f"{DPT}::test_ties_stay"]),
    ("dp_window_too_long", "int until = t + hold - 1 < T ? t + hold - 1 : T;", "int until = t + hold < T ? t + hold : T;", 0,
     [f"{DPT}::test_dp_matches_brute_force"]),
    ("dp_min_up_down_swapped", "const int hold = alt ? m->TU : m->TD;", "const int hold = alt ? m->TD : m->TU;", 0,
     [f"{DPT}::test_dp_matches_brute_force"]),
    ("dp_initial_hold_ignored", "int hold = u0 ? Lg : Fg;", "int hold = 0;", 0, [f"{DPT}::test_dp_matches_brute_force"]),
    ("uc_cost_su_sd_swapped", "u[1] = (s - sp) > 0 ? (s - sp) : 0;", "u[1] = (sp - s) > 0 ? (sp - s) : 0;", 0,
     [f"{DPT}::test_uc_cost_terms", f"{DPT}::test_su_sd_reduction_exact"]),
    ("uc_cost_half_rho_dropped", "L += y[k] * r + 0.5 * rho * r * r;", "L += y[k] * r + rho * r * r;", 0,
     [f"{DPT}::test_uc_cost_terms"]),
    # line model and the line subproblem
    ("admittance_full_charging", "adm[1] = bs + 0.5 * b;", "adm[1] = bs + b;", 0, [f"{BLK}::test_flows_match_complex_power"]),
    ("flow_q_sign", "case 1: *a = -adm[1];", "case 1: *a = adm[1];", 0, [f"{BLK}::test_flows_match_complex_power"]),
    ("branch_grad_v2_factor", "g[0] += b->rho_va * r4 * 2.0 * x[0];", "g[0] += b->rho_va * r4 * x[0];", 0,
     [f"{BLK}::test_branch_objective_and_derivatives"]),
    ("branch_hessian_drop_term", "H[0][0] += b->rho_va * (4.0 * x[0] * x[0] + 2.0 * r4);",
     "H[0][0] += b->rho_va * (4.0 * x[0] * x[0]);", 0, [f"{BLK}::test_branch_objective_and_derivatives"]),
    ("branch_phr_sign", "double t = b->nu[m] + b->mu * h;", "double t = b->nu[m] - b->mu * h;", 0,
     [f"{BLK}::test_branch_objective_and_derivatives"]),
    ("nu_update_forgets_nu", "S->nuf[k] = fmax(0.0, b.nu[0] + b.mu * hf);", "S->nuf[k] = fmax(0.0, b.mu * hf);", 0,
     [f"{BLK}::test_line_limits_active"]),
    ("branch_target_sign", "b.c[r] = xb[r] - S->zB[r][k] - S->yB[r][k] / rho;", "b.c[r] = xb[r] + S->zB[r][k] - S->yB[r][k] / rho;",
     0, [f"{BLK}::test_line_block_stationary"]),
    # generator, relaxed-commitment and bus blocks
    ("gen_ramp_down_sign", "double e5 = -pb_prev + d->rd * uon", "double e5 = -pb_prev - d->rd * uon", 0,
     [f"{BLK}::test_generator_block_kkt_random"]),
    ("gen_c1_slack_side", "{e1, e2, e5, e6}, {1, 0, 1, 0}", "{e1, e2, e5, e6}, {0, 1, 1, 0}", 0,
     [f"{BLK}::test_generator_block_kkt_random"]),
    ("ubar_b_sign", "return clampd((u->rho_uc * u->h3 - u->rho_c", "return clampd((u->rho_uc * u->h3 + u->rho_c", 0,
     [f"{BLK}::test_ubar_block_kkt"]),
    ("ubar_su_next_period", "u.h2 = S->usu[kn] + S->zG[RG_U2][kn]", "u.h2 = S->usu[k] + S->zG[RG_U2][kn]", 0,
     [f"{BLK}::test_ubar_block_kkt_with_start_ups"]),
    ("ubar_su_first_period_u0", "(h6 - P->ru[g] * (double)P->u0[g])", "(h6)", 0, [f"{BLK}::test_ubar_block_kkt"]),
    ("bus_flow_target_sign", "M11 += 1.0 / rpq; aTt += -tauP;", "M11 += 1.0 / rpq; aTt += tauP;", 0,
     [f"{BLK}::test_bus_block_kkt"]),
    ("bus_new_ubar_partner", "- P->ru[g] * X->ubon[k] - P->su[g] * X->ubsu[kn]", "- P->ru[g] * S->ubon[k] - P->su[g] * X->ubsu[kn]",
     0, [f"{BLK}::test_bus_block_kkt"]),
    ("bus_shunt_sign", "double aw = Ww > 0.0 ? -P->gs[i] : 0.0", "double aw = Ww > 0.0 ? P->gs[i] : 0.0", 0,
     [f"{BLK}::test_bus_block_with_shunts_and_ramp_rows"]),
    ("bus_reference_angle", "S->thb[bi] = (i == P->ref || Wt == 0.0)", "S->thb[bi] = (Wt == 0.0)", 0,
     [f"{SOL}::test_ac_power_flow_residual_at_convergence", f"{BLK}::test_bus_block_kkt"]),
    # residual balancing of the penalty classes
    ("adapt_direction_swapped", "S->sc[rho_slot[c]] = rho * tau;", "S->sc[rho_slot[c]] = rho / tau;", 0,
     [f"{ADP}::test_decisions_follow_the_rule"]),
    ("adapt_dual_not_normalised", "double sd = rho * dx_c[c] / y_c[c];", "double sd = rho * dx_c[c];", 0,
     [f"{ADP}::test_decisions_follow_the_rule"]),
    ("adapt_voltage_rows_as_power", "static int class_branch(int r) { return r < 4 ? CL_PQ : CL_VA; }",
     "static int class_branch(int r) { return r < 6 ? CL_PQ : CL_VA; }", 0, [f"{ADP}::test_decisions_follow_the_rule"]),
    ("adapt_coupling_change_without_pbar", "d_va, fmax(d_pb, d_ub), d_ub};", "d_va, d_ub, d_ub};", 0,
     [f"{ADP}::test_decisions_follow_the_rule"]),
    ("adapt_noise_floor_removed", "if (!(rin_c[c] > ADAPT_NOISE || sd > ADAPT_NOISE)) continue;", "", 0,
     [f"{ADP}::test_rounding_level_class_keeps_its_penalty"]),
    ("adapt_span_ignored", "rho * tau <= rho0[c] * span", "1", 0, [f"{ADP}::test_limits"]),
    ("adapt_cap_off_by_one", "S->sc[cnt_slot[c]] >= (double)P->par.adapt_max", "S->sc[cnt_slot[c]] > (double)P->par.adapt_max",
     0, [f"{ADP}::test_limits"]),
    ("adapt_wrong_iteration", "fmod(S->sc[SC_ITER], (double)P->par.adapt_every)",
     "fmod(S->sc[SC_ITER] + 1.0, (double)P->par.adapt_every)", 0, [f"{ADP}::test_decisions_follow_the_rule"]),
    ("adapt_penalty_not_used", "static double rho_va(const orc_problem *P) { return P->st.sc[SC_RHO_VA]; }",
     "static double rho_va(const orc_problem *P) { return P->par.rho_va; }", 0,
     [f"{ADP}::test_equals_penalties_set_by_hand"]),
    # UC warm start (the multiperiod ACOPF, then the commitments from its generation levels)
    ("ucwarm_threshold_full_pmin", "u[k] = P->st.p[k] >= 0.5 * P->pmin[g] ? 1 : 0;", "u[k] = P->st.p[k] >= P->pmin[g] ? 1 : 0;", 0,
     [f"{UCW}::test_rounding_and_restart"]),
    ("relax_keeps_min_generation_row", "{d->relax ? 0.0 : rc, rc, rc, rc}", "{rc, rc, rc, rc}", 0,
     [f"{UCW}::test_relaxed_run_is_the_multiperiod_acopf"]),
    ("relax_runs_the_dp", "if (P->par.relax_uc) return; /* the multiperiod ACOPF has no commitment decisions */", "", 0,
     [f"{UCW}::test_relaxed_run_is_the_multiperiod_acopf"]),
    ("relax_updates_every_row", "if (P->par.relax_uc && (r == RG_C1 || r >= RG_U1)) continue;", "", 0,
     [f"{UCW}::test_relaxed_run_is_the_multiperiod_acopf"]),
    ("ucwarm_restart_keeps_relaxed_state", "  P->par = saved;\n  init_state_u(P, u);", "  P->par = saved;", 0,
     [f"{UCW}::test_rounding_and_restart"]),
    # cold start
    ("cold_start_v_bound", "double x[4] = {0.5 * (P->vmin[i] + P->vmax[i]),", "double x[4] = {P->vmax[i],", 0,
     [f"{BLK}::test_initial_state_cold_start"]),
]


def _mutate(text, old, new, occurrence):
    pos = -1
    for _ in range(occurrence + 1):
        pos = text.find(old, pos + 1)
        if pos < 0:
            raise AssertionError(f"mutation anchor not found: {old!r}")
    return text[:pos] + new + text[pos + len(old):]


def _run_case(case, tmpdir):
    name, old, new, occ, targets = case
    src = _mutate(open(SRC).read(), old, new, occ)
    csrc = os.path.join(tmpdir, f"{name}.c")
    lib = os.path.join(tmpdir, f"lib_{name}.so")
    with open(csrc, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
                           "-fopenmp", "-o", lib, csrc, "-lm"])
    env = dict(os.environ, UCAC_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + targets,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-400:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    text = open(SRC).read()
    for name, old, new, occ, _ in MUTATIONS:
        _mutate(text, old, new, occ)  # every anchor exists
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        results = list(ex.map(lambda c: _run_case(c, str(tmp_path)), MUTATIONS))
    survived = [(name, out) for name, rc, out in results if rc != 1]
    assert not survived, survived


def test_unmutated_oracle_passes_the_same_pins(tmp_path):
    """The child runs are meaningful: the same pins pass on an unmutated copy."""
    targets = sorted({t for *_, ts in MUTATIONS for t in ts})
    name, rc, out = _run_case(("unmutated", "#include <math.h>", "#include <math.h>", 0, targets), str(tmp_path))
    assert rc == 0, out


# ---- the network oracle --------------------------------------------------------

def test_adam_with_swapped_betas_fails_its_pin(monkeypatch):
    from oracle import mlp
    from tests import test_oracle_mlp as pins
    good = mlp.adam

    def swapped(vec, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        return good(vec, g, m, v, t, lr, b1=b2, b2=b1, eps=eps)

    monkeypatch.setattr(mlp, "adam", swapped)
    with pytest.raises(AssertionError):
        pins.test_adam_later_steps_closed_form()


def test_backprop_without_silu_derivative_fails_its_pin(monkeypatch):
    from oracle import mlp
    from tests import test_oracle_mlp as pins
    monkeypatch.setattr(mlp, "dsilu", lambda z: 1.0 / (1.0 + np.exp(-z)))
    with pytest.raises(AssertionError):
        pins.test_backprop_matches_finite_differences()
