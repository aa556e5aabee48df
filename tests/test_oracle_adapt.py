"""Pins of the oracle's residual balancing of the penalty classes (the remedy the
paper's conclusion names for the method's sensitivity to rho_pq, rho_va, rho_uc),
each against quantities recomputed from saved states with code that shares nothing
with the oracle:

* with balancing off the penalties in force stay the configured ones;
* every decision equals the balancing rule applied to the class residuals
  recomputed from the two states around the deciding iteration (rows from their
  definitions, duplicate changes from the raw arrays), with both directions, every
  class and a class at the rounding level (which keeps its penalty) exercised;
* the new penalties enter the next iteration exactly as the same penalties set by
  hand would (a run with balancing equals a run without it whose penalties are
  changed by hand at the same iterations to the same values);
* the limits: at most adapt_max changes per class, and every penalty within
  [rho0 / span, rho0 * span].
"""
import numpy as np
import pytest

import oracle
from paper_2310_13145_amd import synth
from tests import ucrows

CLASSES = ("pq", "va", "cpl", "uc")
# duplicates contained in each class's rows
CLASS_DUPS = {"pq": ("Pbf", "Qbf", "Pbt", "Qbt", "pb", "qb"), "va": ("wb", "thb"),
              "cpl": ("pb", "ubon", "ubsu", "ubsd"), "uc": ("ubon", "ubsu", "ubsd")}
LINE_ROW_CLASS = ["pq"] * 4 + ["va"] * 4
NOISE = 1e-9  # residuals at or below this on both sides are rounding noise: no decision
GEN_ROW_CLASS = ["pq", "pq"] + ["cpl"] * 6 + ["uc"] * 3


def instance():
    inst = synth.small_instance(14, 20, 5, 6, seed=83)
    inst["gen_cnl"] = np.full(5, 40.0)
    return inst


def class_residuals(inst, S0, S1):
    """Per class: max |a_r + z_r| and max |y_r| over its rows in state S1, and the
    largest change of the duplicates in its rows from S0 to S1."""
    T, L, G = inst["T"], inst["n_line"], inst["n_gen"]
    lr = ucrows.line_rows(inst, S1)
    gr = ucrows.gen_rows(inst, S1)
    rin = {c: 0.0 for c in CLASSES}
    ymax = {c: 0.0 for c in CLASSES}
    for r in range(8):
        c = LINE_ROW_CLASS[r]
        rin[c] = max(rin[c], float(np.max(np.abs(lr[r] + np.reshape(S1[f"zB{r}"], (T, L))))))
        ymax[c] = max(ymax[c], float(np.max(np.abs(S1[f"yB{r}"]))))
    for r, name in enumerate(ucrows.GEN_ROWS):
        c = GEN_ROW_CLASS[r]
        rin[c] = max(rin[c], float(np.max(np.abs(gr[name] + np.reshape(S1[f"zG{r}"], (T, G))))))
        ymax[c] = max(ymax[c], float(np.max(np.abs(S1[f"yG{r}"]))))
    dx = {c: max(float(np.max(np.abs(np.asarray(S1[d]) - np.asarray(S0[d])))) for d in CLASS_DUPS[c])
          for c in CLASSES}
    return rin, dx, ymax


def test_off_keeps_the_configured_penalties():
    inst = instance()
    o = oracle.Oracle(inst)
    p = o.params
    for _ in range(40):
        o.step(1)
        S = o.state()
        assert (S["rho_pq"], S["rho_va"], S["rho_cpl"], S["rho_uc"]) == (p.rho_pq, p.rho_va, p.rho_cpl, p.rho_uc)
        assert S["nchg_pq"] == S["nchg_va"] == S["nchg_cpl"] == S["nchg_uc"] == 0.0


def _check_decisions(inst, mu, tau, K, n_iters, **over):
    """Run the oracle with balancing and check every decision against the rule applied
    to recomputed class residuals; return the set of (class, kind) events seen."""
    o = oracle.Oracle(inst, adapt_every=K, adapt_mu=mu, adapt_tau=tau, **over)
    hit = set()
    prev = o.state()
    checked = 0
    for it in range(1, n_iters + 1):
        o.step(1)
        S = o.state()
        if it % K == 0:
            rin, dx, ymax = class_residuals(inst, prev, S)
            for c in CLASSES:
                rho0, rho1 = prev[f"rho_{c}"], S[f"rho_{c}"]
                if ymax[c] == 0.0:
                    assert rho1 == rho0, (it, c)
                    continue
                sd = rho0 * dx[c] / ymax[c]
                if rin[c] <= NOISE and sd <= NOISE:
                    assert rho1 == rho0, (it, c, "rounding-level residuals decide nothing")
                    hit.add((c, "noise"))
                    continue
                # a decision this close to the threshold may differ in the last bit of a
                # recomputed residual: skip it
                if abs(rin[c] - mu * sd) <= 1e-9 * max(rin[c], mu * sd) or \
                        abs(sd - mu * rin[c]) <= 1e-9 * max(sd, mu * rin[c]):
                    continue
                if rin[c] > mu * sd:
                    assert rho1 == rho0 * tau, (it, c, rin[c], sd)
                    hit.add((c, "up"))
                elif sd > mu * rin[c]:
                    assert rho1 == rho0 / tau, (it, c, rin[c], sd)
                    hit.add((c, "down"))
                else:
                    assert rho1 == rho0, (it, c, rin[c], sd)
                    hit.add((c, "keep"))
                checked += 1
        else:
            for c in CLASSES:
                assert S[f"rho_{c}"] == prev[f"rho_{c}"], (it, c)
        prev = S
    assert checked > 0
    return hit


def test_decisions_follow_the_rule():
    """adapt_every = 3 with a small imbalance factor on a 14-bus mesh: decisions in
    both directions in every class within 150 iterations."""
    hit = _check_decisions(instance(), 1.5, 2.0, 3, 150, adapt_max=1000, adapt_span=1e6)
    assert {"up", "down"} <= {d for _, d in hit}, hit
    assert {c for c, d in hit if d in ("up", "down")} == set(CLASSES), hit


def test_rounding_level_class_keeps_its_penalty():
    """The 118-bus workload with mu = 10, tau = 2 and a decision after every 50th
    iteration: once the commitments equal their binary duplicates, the commitment
    rows' residuals are rounding noise, and that class keeps its penalty."""
    hit = _check_decisions(synth.config_instance(1), 10.0, 2.0, 50, 450)
    assert ("uc", "noise") in hit, hit


def test_equals_penalties_set_by_hand():
    """The penalties a balancing run chooses, set by hand at the same iterations in a
    run without balancing, give the same iterate bit for bit."""
    inst = instance()
    a = oracle.Oracle(inst, adapt_every=2, adapt_mu=2.0)
    b = oracle.Oracle(inst)
    changes = 0
    for it in range(80):
        Sa = a.state()
        cur = {f"rho_{c}": Sa[f"rho_{c}"] for c in CLASSES}
        Sb = b.state()
        if any(Sb[k] != v for k, v in cur.items()):
            b.set_params(**cur)
            changes += 1
        a.step(1)
        b.step(1)
    assert changes >= 5
    fa, fb = a.state(), b.state()
    for name, arr in fa.items():
        if name.startswith("nchg") or np.isscalar(arr) and name.startswith("rho"):
            continue
        np.testing.assert_array_equal(np.asarray(arr), np.asarray(fb[name]), err_msg=name)


@pytest.mark.parametrize("span,cap", [(2.0, 1000), (1e6, 3)])
def test_limits(span, cap):
    inst = instance()
    o = oracle.Oracle(inst, adapt_every=1, adapt_mu=1.2, adapt_span=span, adapt_max=cap)
    p = o.params
    rho0 = {"pq": p.rho_pq, "va": p.rho_va, "cpl": p.rho_cpl, "uc": p.rho_uc}
    counts = {c: 0 for c in CLASSES}
    prev = o.state()
    for _ in range(120):
        o.step(1)
        S = o.state()
        for c in CLASSES:
            assert rho0[c] / span <= S[f"rho_{c}"] <= rho0[c] * span
            if S[f"rho_{c}"] != prev[f"rho_{c}"]:
                counts[c] += 1
            assert S[f"nchg_{c}"] == counts[c] <= cap
        prev = S
    if cap == 3:
        assert max(counts.values()) == 3
