"""Pins of the oracle's UC warm start (Sec. IV-A: commitments from the generation levels
of a multiperiod ACOPF solved first):

* the relaxed run is the multiperiod ACOPF: no commitment decision is taken (u and
  its duplicate stay at the cold start), the commitment rows and the
  minimum-generation row carry no multiplier, generation may fall below the
  minimum output but stays in [0, P-bar], and at its tolerance the bus-side point
  satisfies the AC power-flow equations (mismatch of a Y-bus evaluation) and the
  ramp limits;
* the rounding: a unit is on in a period exactly when its relaxed generation there
  is at least half its minimum output, recomputed from a separate relaxed run;
* the restart: everything but the commitments, their duplicates and the slacks is
  the cold start, start-ups and shut-downs follow from the commitments' changes,
  and the slacks are the feasible values for the new commitments.
"""
import numpy as np

import oracle
from paper_2310_13145_amd import synth
from tests import ucrows

COMMIT_ARRAYS = ("uon", "usu", "usd", "ubon", "ubsu", "ubsd", "s1", "s2", "s3", "s4", "s5", "s6")


def relaxed(inst, tol, max_iters):
    o = oracle.Oracle(inst, relax_uc=1)
    rc, it = o.solve(tol, max_iters)
    return o, rc, it


def test_relaxed_run_is_the_multiperiod_acopf():
    inst = synth.config_instance(1)
    # a no-load cost far above the commitment rows' penalty: a dynamic program run on
    # these tables would switch every unit off, so a run that takes no commitment
    # decision is visible
    inst["gen_cnl"] = np.full(inst["n_gen"], 1e6)
    tol = 1e-4
    o, rc, it = relaxed(inst, tol, 6000)
    assert rc == 0
    S = o.state()
    G, T, N = inst["n_gen"], inst["T"], inst["n_bus"]
    cold = oracle.Oracle(inst).state()
    for k in ("uon", "usu", "usd", "ubon", "ubsu", "ubsd"):
        np.testing.assert_array_equal(S[k], cold[k], err_msg=k)
    for r in (2, 8, 9, 10):  # C1, U1, U2, U3
        assert not np.any(S[f"zG{r}"]) and not np.any(S[f"yG{r}"]) and not np.any(S[f"lG{r}"])
    p = S["p"].reshape(T, G)
    pmin, pmax = inst["gen_pmin"], inst["gen_pmax"]
    assert np.all(p >= 0.0) and np.all(p <= pmax + 1e-12)
    below = (p < pmin - 1e-6) & (p > 1e-6)
    assert np.sum(below) > 0  # units below their minimum output: the relaxation is used
    # generator stationarity without the minimum-generation row: d/dp of the cost plus
    # the multipliers of the rows p enters (G1, C2, C5, C6, each with coefficient +1)
    # vanishes up to the penalty terms rho (a + z) of those rows
    base = inst["base_mva"]
    k2, k1 = inst["gen_c2"] * base * base, inst["gen_c1"] * base
    y = {r: S[f"yG{r}"].reshape(T, G) for r in (0, 3, 6, 7)}
    stat = 2.0 * k2 * p + k1 + y[0] + y[3] + y[6] + y[7]
    bound = 4 * o.params.rho_cpl * S["r_in"] + 1e-6
    assert np.all(np.abs(stat[below]) <= bound), (np.max(np.abs(stat[below])), bound)
    # the AC power flow at the bus-side point
    wb, thb = S["wb"].reshape(T, N), S["thb"].reshape(T, N)
    pb, qb = S["pb"].reshape(T, G), S["qb"].reshape(T, G)
    worst = 0.0
    for t in range(T):
        inj = ucrows.ybus_injections(inst, np.sqrt(wb[t]), thb[t])
        Pg = np.zeros(N); Qg = np.zeros(N)
        np.add.at(Pg, inst["gen_bus"], pb[t]); np.add.at(Qg, inst["gen_bus"], qb[t])
        worst = max(worst, np.max(np.abs(Pg - inst["load_p"][t] - inj.real)),
                    np.max(np.abs(Qg - inst["load_q"][t] - inj.imag)))
    assert worst <= 50 * tol, worst
    # the ramp limits between consecutive periods (all units on)
    dp = np.diff(np.vstack([inst["gen_p0"], pb]), axis=0)
    assert np.all(dp <= inst["gen_ru"] + 50 * tol) and np.all(-dp <= inst["gen_rd"] + 50 * tol)


def test_rounding_and_restart():
    inst = synth.config_instance(1)
    G, T = inst["n_gen"], inst["T"]
    tol, mi = 1e-3, 3000
    ref, rc_ref, it_ref = relaxed(inst, tol, mi)
    p = ref.state()["p"].reshape(T, G)
    u = (p >= 0.5 * inst["gen_pmin"]).astype(float)
    assert 0 < u.sum() < u.size  # some units off, some on

    o = oracle.Oracle(inst)
    rc, it = o.uc_warmstart(tol, mi)
    assert (rc, it) == (rc_ref, it_ref)
    S = o.state()
    cold = oracle.Oracle(inst).state()
    for name, arr in cold.items():
        if name in COMMIT_ARRAYS:
            continue
        np.testing.assert_array_equal(np.asarray(S[name]), np.asarray(arr), err_msg=name)
    np.testing.assert_array_equal(S["uon"].reshape(T, G), u)
    prev = np.vstack([inst["gen_u0"][None, :].astype(float), u[:-1]])
    np.testing.assert_array_equal(S["usu"].reshape(T, G), (u > prev).astype(float))
    np.testing.assert_array_equal(S["usd"].reshape(T, G), (u < prev).astype(float))
    for a, b in (("ubon", "uon"), ("ubsu", "usu"), ("ubsd", "usd")):
        np.testing.assert_array_equal(S[a], S[b])
    # slacks: the feasible values for the new commitments, so that rows C1-C6 are
    # satisfied or off only by the sign their slack cannot absorb
    rows = ucrows.gen_rows(inst, S)
    for name, sgn in (("C1", 1), ("C2", -1), ("C3", 1), ("C4", -1), ("C5", 1), ("C6", -1)):
        r = rows[name]
        s = S[f"s{int(name[1])}"].reshape(T, G)
        # a row with -s (C1, C3, C5) is zero where its slack is positive and negative
        # otherwise; a row with +s (C2, C4, C6) is zero there and positive otherwise
        assert np.all(np.abs(r[s > 0]) <= 1e-12), name
        assert np.all(sgn * r[s == 0] <= 1e-12), name
