"""Whole-solve pins of the oracle: convergence on the 9-bus ring, AC power-flow
residuals of the converged duplicates, a single-bus economic dispatch in closed
form, the beta rule of step:outer, determinism and bit-exact resume."""
import numpy as np
import pytest

import oracle
from paper_2310_13145_amd import synth
from tests import ucrows


@pytest.fixture(scope="module")
def solved9():
    inst = synth.config_instance(0)
    o = oracle.Oracle(inst)
    rc, iters = o.solve(tol=1e-4, max_iters=5000)
    return inst, o, rc, iters


def test_ring9_converges(solved9):
    inst, o, rc, iters = solved9
    S = o.state()
    assert rc == 0 and S["converged"] == 1.0
    assert S["r_p"] <= 1e-4 and S["r_d"] <= 1e-4
    # r_p is the max-norm of the coupling-row violations, recomputed from the rows
    rows = ucrows.line_rows(inst, S) + list(ucrows.gen_rows(inst, S).values())
    assert max(np.abs(r).max() for r in rows) == pytest.approx(S["r_p"], rel=1e-12)


def test_ac_power_flow_residual_at_convergence(solved9):
    """Bus injections of the AC network at (sqrt(wbar), thetabar) match the dispatched
    pbar, qbar minus load up to a constant times the tolerance."""
    inst, o, rc, iters = solved9
    S = o.state()
    N, G, T = inst["n_bus"], inst["n_gen"], inst["T"]
    wb = S["wb"].reshape(T, N); thb = S["thb"].reshape(T, N)
    pb = S["pb"].reshape(T, G); qb = S["qb"].reshape(T, G)
    worst = 0.0
    for t in range(T):
        Sinj = ucrows.ybus_injections(inst, np.sqrt(wb[t]), thb[t])
        Pg = np.zeros(N); Qg = np.zeros(N)
        np.add.at(Pg, inst["gen_bus"], pb[t]); np.add.at(Qg, inst["gen_bus"], qb[t])
        worst = max(worst, np.abs(Sinj.real - (Pg - inst["load_p"][t])).max(),
                    np.abs(Sinj.imag - (Qg - inst["load_q"][t])).max())
    assert worst <= 50 * 1e-4


def test_single_bus_economic_dispatch():
    """No network, slack ramps, unit windows: the converged dispatch is the
    equal-marginal-cost dispatch of the committed units (bisection on the price)."""
    inst = dict(n_bus=1, n_line=0, n_gen=3, T=4, ref_bus=0, base_mva=100.0,
                line_from=np.zeros(0, np.int32), line_to=np.zeros(0, np.int32),
                line_r=np.zeros(0), line_x=np.zeros(0), line_b=np.zeros(0), line_rate=np.zeros(0),
                bus_gs=np.zeros(1), bus_bs=np.zeros(1), bus_vmin=np.full(1, 0.9), bus_vmax=np.full(1, 1.1),
                load_p=np.array([[2.0], [2.4], [3.1], [2.2]]), load_q=np.array([[0.6], [0.7], [0.9], [0.65]]),
                gen_bus=np.zeros(3, np.int32),
                gen_pmin=np.array([0.2, 0.3, 0.1]), gen_pmax=np.array([1.0, 1.5, 2.0]),
                gen_qmin=np.array([-0.5, -0.5, -0.5]), gen_qmax=np.array([1.0, 1.0, 1.0]),
                gen_c2=np.array([0.05, 0.02, 0.08]), gen_c1=np.array([20.0, 25.0, 15.0]),
                gen_cnl=np.zeros(3), gen_csu=np.zeros(3), gen_csd=np.zeros(3),
                gen_ru=np.full(3, 10.0), gen_rd=np.full(3, 10.0), gen_su=np.full(3, 10.0), gen_sd=np.full(3, 10.0),
                gen_min_up=np.ones(3, np.int32), gen_min_dn=np.ones(3, np.int32),
                gen_u0=np.ones(3, np.int32), gen_init_on=np.zeros(3, np.int32), gen_init_off=np.zeros(3, np.int32),
                gen_p0=np.array([0.5, 0.8, 0.9]))
    o = oracle.Oracle(inst)
    rc, iters = o.solve(tol=1e-6, max_iters=20000)
    assert rc == 0
    S = o.state()
    p = S["p"].reshape(4, 3); u = S["uon"].reshape(4, 3)
    k2, k1 = inst["gen_c2"] * 1e4, inst["gen_c1"] * 100
    for t in range(4):
        on = u[t] > 0.5
        lo = np.where(on, inst["gen_pmin"], 0.0); hi = np.where(on, inst["gen_pmax"], 0.0)
        disp = lambda lam: np.clip((lam - k1) / (2 * k2), lo, hi)
        a, b = 0.0, 1e5
        for _ in range(200):
            m = 0.5 * (a + b)
            a, b = (m, b) if disp(m).sum() < inst["load_p"][t, 0] else (a, m)
        np.testing.assert_allclose(p[t], disp(0.5 * (a + b)), atol=1e-3)


def test_beta_rule_trace():
    """beta grows by tau exactly when ||z^k||_inf > theta ||z^{k-1}||_inf (step:outer)."""
    inst = synth.config_instance(0)
    o = oracle.Oracle(inst)
    par = o.params
    prev = o.state()
    seen = 0
    for _ in range(1500):
        o.step(1)
        S = o.state()
        if S["k_outer"] != prev["k_outer"]:
            seen += 1
            grow = S["z_inf"] > par.theta * prev["znorm_prev"]
            want = min(par.tau * prev["beta"], par.beta_max) if grow else prev["beta"]
            assert S["beta"] == want
            assert S["znorm_prev"] == S["z_inf"]
            assert S["l_inner"] == 0
        prev = S
    assert seen >= 3


def test_deterministic_and_resume_bit_exact():
    inst = synth.small_instance(14, 20, 5, 5, seed=77)
    a = oracle.Oracle(inst)
    a.step(40)
    mid = a.get_state()
    a.step(25)
    b = oracle.Oracle(inst)
    b.set_state(mid)
    b.step(25)
    np.testing.assert_array_equal(a.get_state(), b.get_state())
    c = oracle.Oracle(inst)
    c.step(65)
    np.testing.assert_array_equal(a.get_state(), c.get_state())


def test_thread_count_invariance():
    """The oracle's parallel loops give the same iterate bit for bit on one thread and
    on every host thread (the items of each block are independent; the residuals are
    maxima)."""
    inst = synth.small_instance(30, 45, 8, 12, seed=33)
    states = []
    for n in (1, max(2, oracle.max_threads()), 3):
        oracle.set_threads(n)
        o = oracle.Oracle(inst)
        o.step(60)
        states.append(o.get_state())
    oracle.set_threads(0)
    for s in states[1:]:
        np.testing.assert_array_equal(states[0], s)
