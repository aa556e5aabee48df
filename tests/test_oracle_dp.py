"""Pins of the oracle's UC dynamic program (Sec. III-B, Alg. dp_algo) against brute
force over the feasible set set:UC written out from its constraints."""
import itertools

import numpy as np
import pytest

import oracle


def feasible(u, su, sd, u0, Lg, Fg, TU, TD):
    """set:UC for one generator, 1-based periods; the state equation is also
    applied at t = 1 with the given u_0 (the initial state is data)."""
    T = len(u)
    if any(1 - u[t] for t in range(min(Lg, T))):          # uc_initial_on
        return False
    if any(u[t] for t in range(min(Fg, T))):              # uc_initial_off
        return False
    for t in range(T):                                    # uc_acopf_gen_state
        prev = u0 if t == 0 else u[t - 1]
        if prev - u[t] + su[t] - sd[t] != 0:
            return False
    for t in range(TU, T + 1):                            # uc_minup, t = TU..T
        if sum(su[i - 1] for i in range(t - TU + 1, t + 1)) > u[t - 1]:
            return False
    for t in range(TD, T + 1):                            # uc_mindn
        if sum(sd[i - 1] for i in range(t - TD + 1, t + 1)) > 1 - u[t - 1]:
            return False
    return True


def brute_force_reduced(Ltab, u0, Lg, Fg, TU, TD):
    T = Ltab.shape[0]
    best, arg = np.inf, []
    for u in itertools.product((0, 1), repeat=T):
        su = [max(0, u[t] - (u0 if t == 0 else u[t - 1])) for t in range(T)]
        sd = [max(0, (u0 if t == 0 else u[t - 1]) - u[t]) for t in range(T)]
        if not feasible(u, su, sd, u0, Lg, Fg, TU, TD):
            continue
        c = sum(Ltab[t, u0 if t == 0 else u[t - 1], u[t]] for t in range(T))
        if c < best - 1e-12:
            best, arg = c, [u]
        elif abs(c - best) <= 1e-12:
            arg.append(u)
    return best, arg


@pytest.mark.parametrize("seed", range(60))
def test_dp_matches_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    T = int(rng.integers(4, 13))
    TU, TD = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    T = max(T, TU, TD)  # the windows of set:UC cover every switch only when T >= T^U, T^D
    u0 = int(rng.integers(0, 2))
    hold = int(rng.integers(0, 4)) if rng.random() < 0.4 else 0
    Lg, Fg = (hold, 0) if u0 == 1 else (0, hold)
    Ltab = rng.normal(size=(T, 2, 2))
    cost, u = oracle.dp(Ltab, u0, Lg, Fg, TU, TD)
    best, args = brute_force_reduced(Ltab, u0, Lg, Fg, TU, TD)
    assert cost == pytest.approx(best, rel=1e-12, abs=1e-12)
    su = [max(0, u[t] - (u0 if t == 0 else u[t - 1])) for t in range(T)]
    sd = [max(0, (u0 if t == 0 else u[t - 1]) - u[t]) for t in range(T)]
    assert feasible(list(u), su, sd, u0, Lg, Fg, TU, TD)
    recomputed = sum(Ltab[t, u0 if t == 0 else u[t - 1], u[t]] for t in range(T))
    assert recomputed == pytest.approx(cost, rel=1e-12, abs=1e-12)
    if len(args) == 1:
        assert tuple(int(v) for v in u) == args[0]


def test_su_sd_reduction_exact():
    """Optimising over (u_on, u_su, u_sd) in {0,1}^{3T} under set:UC with independent
    per-variable costs equals optimising over u_on with u_su, u_sd inferred."""
    rng = np.random.default_rng(7)
    for trial in range(40):
        T = 4
        TU, TD = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        u0 = int(rng.integers(0, 2))
        w = rng.normal(size=(T, 3, 2))  # cost of variable k at value 0/1, arbitrary sign
        best_full = np.inf
        for bits in itertools.product((0, 1), repeat=3 * T):
            u, su, sd = bits[:T], bits[T:2 * T], bits[2 * T:]
            if not feasible(u, su, sd, u0, 0, 0, TU, TD):
                continue
            c = sum(w[t, 0, u[t]] + w[t, 1, su[t]] + w[t, 2, sd[t]] for t in range(T))
            best_full = min(best_full, c)
        Ltab = np.zeros((T, 2, 2))
        for t in range(T):
            for sp in (0, 1):
                for s in (0, 1):
                    Ltab[t, sp, s] = w[t, 0, s] + w[t, 1, max(0, s - sp)] + w[t, 2, max(0, sp - s)]
        cost, _ = oracle.dp(Ltab, u0, 0, 0, TU, TD)
        assert cost == pytest.approx(best_full, abs=1e-12)


@pytest.mark.parametrize("u0", [0, 1])
def test_ties_stay(u0):
    """With every transition equally costly, the stay-on-ties rule keeps u_0."""
    T = 8
    cost, u = oracle.dp(np.ones((T, 2, 2)), u0, 0, 0, 2, 3)
    assert cost == T
    assert list(u) == [u0] * T


def test_switch_block_truncated_at_horizon():
    """A start-up in the last period holds only to T (A8 reading)."""
    T = 5
    L = np.zeros((T, 2, 2))
    L[:, 0, 0] = 1.0           # staying off costs 1 per period
    L[:, 1, 1] = 0.5           # staying on costs 0.5
    L[:4, 0, 1] = 10.0         # starting up is expensive except in the last period
    L[4, 0, 1] = 0.0
    cost, u = oracle.dp(L, 0, 0, 0, 3, 1)
    best, args = brute_force_reduced(L, 0, 0, 0, 3, 1)
    assert cost == pytest.approx(best)
    assert list(u) == [0, 0, 0, 0, 1]


def test_uc_cost_terms():
    """L^UC(s', s) = commitment costs + y(u - ubar + z) + rho/2 (u - ubar + z)^2 summed
    over on/su/sd with su/sd inferred from (s', s)."""
    ub, z, y = [0.3, 0.2, 0.1], [0.01, -0.02, 0.03], [5.0, -4.0, 3.0]
    rho = 7.0
    for sp in (0, 1):
        for s in (0, 1):
            u = [s, max(0, s - sp), max(0, sp - s)]
            want = 2.0 * s + 11.0 * u[1] + 13.0 * u[2]
            for k in range(3):
                r = u[k] - ub[k] + z[k]
                want += y[k] * r + rho / 2 * r * r
            got = oracle.uc_cost(2.0, 11.0, 13.0, rho, sp, s, ub, z, y)
            assert got == pytest.approx(want, rel=1e-14)
