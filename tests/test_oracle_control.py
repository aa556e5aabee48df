"""Pins of the oracle's control quantities against their definitions, recomputed
from saved states with code that shares nothing with the oracle:

* the reported objective, the cost of eq:uc-acopf (quadratic generation cost plus the
  no-load, start-up and shut-down costs of f^UC) on arbitrary states with every cost
  coefficient nonzero;
* the dual residual r_d (largest change of any bus-side duplicate across one inner
  iteration), the inner residual r_in (max |A x + B xbar + z|), the primal residual
  r_p (max |A x + B xbar|, the primal infeasibility of Sec. IV-D) and ||z||_inf, each
  against two consecutive states, with every duplicate array in turn holding the
  largest change;
* the inner-loop exit of Alg. alg:basic: step:outer runs exactly when
  max(r_in, r_d) <= max(tol/2, eps_in0 2^-k) or when the inner loop reaches
  max_inner iterations, on whole trajectories with both kinds of exit.
"""
import numpy as np
import pytest

import oracle
from paper_2310_13145_amd import synth
from tests import ucrows

DUPLICATES = ("wb", "thb", "Pbf", "Qbf", "Pbt", "Qbt", "pb", "qb", "ubon", "ubsu", "ubsd")


def costed_instance():
    """14-bus mesh with every cost term of f^UC nonzero and two units starting off."""
    inst = synth.small_instance(14, 20, 5, 5, seed=81)
    rng = np.random.default_rng(21)
    inst["gen_cnl"] = rng.uniform(50.0, 150.0, 5)
    inst["gen_csd"] = rng.uniform(20.0, 80.0, 5)
    inst["gen_u0"] = np.array([0, 1, 1, 0, 1], np.int32)
    return inst


def objective_from_definition(inst, S):
    """sum over (t, g) of c2 P^2 + c1 P (P in MW) + C_nl u_on + C_su u_su + C_sd u_sd."""
    G, T = inst["n_gen"], inst["T"]
    base = inst["base_mva"]
    total = 0.0
    for t in range(T):
        for g in range(G):
            k = t * G + g
            mw = S["p"][k] * base
            total += inst["gen_c2"][g] * mw * mw + inst["gen_c1"][g] * mw
            total += inst["gen_cnl"][g] * S["uon"][k] + inst["gen_csu"][g] * S["usu"][k]
            total += inst["gen_csd"][g] * S["usd"][k]
    return total


def test_objective_matches_cost_definition():
    inst = costed_instance()
    o = oracle.Oracle(inst)
    o.step(30)
    assert o.objective() == pytest.approx(objective_from_definition(inst, o.state()), rel=1e-12)
    # arbitrary states: every term of the cost enters with its own coefficient
    rng = np.random.default_rng(22)
    flat = o.get_state()
    for _ in range(20):
        S = oracle.unpack_state(flat.copy(), *o.dims)
        TG = inst["T"] * inst["n_gen"]
        buf = flat.copy()
        lay = oracle.state_layout(*o.dims)
        off = 0
        for name, n in lay:
            if name == "p":
                buf[off:off + n] = rng.uniform(0.0, 3.0, n)
            elif name in ("uon", "usu", "usd"):
                buf[off:off + n] = rng.integers(0, 2, n)
            off += n
        o.set_state(buf)
        S = oracle.unpack_state(buf, *o.dims)
        assert len(S["p"]) == TG
        assert o.objective() == pytest.approx(objective_from_definition(inst, S), rel=1e-12)


def residuals_from_states(inst, params, S0, S1):
    rb, rg = ucrows.rhos(params)
    a_line = ucrows.line_rows(inst, S1)
    a_gen = ucrows.gen_rows(inst, S1)
    rp = rin = zinf = 0.0
    for kind, rows in (("B", a_line), ("G", [a_gen[n] for n in ucrows.GEN_ROWS])):
        for r, a in enumerate(rows):
            z = np.asarray(S1[f"z{kind}{r}"]).reshape(a.shape)
            rp = max(rp, float(np.abs(a).max(initial=0.0)))
            rin = max(rin, float(np.abs(a + z).max(initial=0.0)))
            zinf = max(zinf, float(np.abs(z).max(initial=0.0)))
    rd = max(float(np.abs(np.asarray(S1[k]) - np.asarray(S0[k])).max(initial=0.0)) for k in DUPLICATES)
    argmax = max(DUPLICATES, key=lambda k: np.abs(np.asarray(S1[k]) - np.asarray(S0[k])).max(initial=0.0))
    return rp, rin, rd, zinf, argmax


@pytest.mark.parametrize("which", DUPLICATES)
def test_residuals_recomputed_from_two_states(which):
    """Perturb one duplicate array of a mid-run state so that it holds the largest
    change of the next iteration; r_d must see it, and r_p, r_in, ||z|| must equal
    the maxima recomputed from the rows of the new state."""
    inst = costed_instance()
    o = oracle.Oracle(inst)
    o.step(25)
    flat = o.get_state()
    off = 0
    for name, n in oracle.state_layout(*o.dims):
        if name == which:
            flat[off:off + n] += 3.0 + np.linspace(0.0, 1.0, n)
        off += n
    o.set_state(flat)
    S0 = o.state()
    o.step(1)
    S1 = o.state()
    rp, rin, rd, zinf, argmax = residuals_from_states(inst, o.params, S0, S1)
    assert argmax == which
    assert S1["r_d"] == rd
    assert S1["r_p"] == pytest.approx(rp, rel=1e-13, abs=1e-15)
    assert S1["r_in"] == pytest.approx(rin, rel=1e-13, abs=1e-15)
    assert S1["z_inf"] == pytest.approx(zinf, rel=1e-13, abs=1e-15)


def test_residuals_on_plain_trajectory():
    inst = synth.config_instance(0)
    o = oracle.Oracle(inst)
    S0 = o.state()
    for _ in range(40):
        o.step(1)
        S1 = o.state()
        rp, rin, rd, zinf, _ = residuals_from_states(inst, o.params, S0, S1)
        assert S1["r_d"] == rd
        assert S1["r_p"] == pytest.approx(rp, rel=1e-13, abs=1e-15)
        assert S1["r_in"] == pytest.approx(rin, rel=1e-13, abs=1e-15)
        S0 = S1


@pytest.mark.parametrize("max_inner", [1000, 7])
def test_inner_loop_exit_rule(max_inner):
    """step:outer runs after inner iteration l of outer iteration k exactly when
    max(r_in, r_d) <= max(tol / 2, eps_in0 * 2^-k) or l reaches max_inner."""
    inst = synth.config_instance(0)
    o = oracle.Oracle(inst, max_inner=max_inner)
    par = o.params
    prev = o.state()
    by_tol = by_count = 0
    near = 0
    for _ in range(1200):
        o.step(1)
        S = o.state()
        k = prev["k_outer"]
        eps = max(0.5 * par.tol, par.eps_in0 * 2.0 ** (-k))
        small = max(S["r_in"], S["r_d"]) <= eps
        full = prev["l_inner"] + 1 >= max_inner
        advanced = S["k_outer"] == k + 1
        assert S["k_outer"] in (k, k + 1)
        assert advanced == (small or full), (S["iter"], k, S["r_in"], S["r_d"], eps)
        if advanced:
            assert S["l_inner"] == 0
            by_tol += small
            by_count += full and not small
        else:
            assert S["l_inner"] == prev["l_inner"] + 1
        # iterations where r_p and r_in fall on opposite sides of the threshold
        near += (max(S["r_p"], S["r_d"]) <= eps) != small
        prev = S
    assert by_tol >= 2
    if max_inner < 100:
        assert by_count >= 20
    else:
        assert near >= 1


def test_z_update_with_nonzero_lambda():
    """step:z minimises lambda z + beta/2 z^2 + y (a + z) + rho/2 (a + z)^2 row by row,
    so lambda + beta z + y_old + rho (a + z) = 0; with step:y that is
    lambda + beta z + y_new = 0.  Checked with random outer multipliers on every row
    (the early iterations of a run still have lambda = 0)."""
    inst = costed_instance()
    o = oracle.Oracle(inst)
    o.step(25)
    flat = o.get_state()
    rng = np.random.default_rng(23)
    off = 0
    for name, n in oracle.state_layout(*o.dims):
        if name.startswith("lB") or name.startswith("lG"):
            flat[off:off + n] = rng.normal(scale=300.0, size=n)
        off += n
    o.set_state(flat)
    S0 = o.state()
    o.step(1)
    S1 = o.state()
    assert S1["k_outer"] == S0["k_outer"]
    rb, rg = ucrows.rhos(o.params)
    beta = S0["beta"]
    rows = {"B": ucrows.line_rows(inst, S1), "G": [ucrows.gen_rows(inst, S1)[n] for n in ucrows.GEN_ROWS]}
    for kind, rho in (("B", rb), ("G", rg)):
        for r, a in enumerate(rows[kind]):
            lam, z = np.asarray(S0[f"l{kind}{r}"]), np.asarray(S1[f"z{kind}{r}"])
            y0, y1 = np.asarray(S0[f"y{kind}{r}"]), np.asarray(S1[f"y{kind}{r}"])
            scale = max(1.0, np.abs(lam).max(), np.abs(y1).max())
            np.testing.assert_allclose(lam + beta * z + y0 + rho[r] * (a.ravel() + z), 0.0, atol=1e-10 * scale)
            np.testing.assert_allclose(lam + beta * z + y1, 0.0, atol=1e-10 * scale)
