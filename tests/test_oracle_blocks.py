"""Pins of the oracle's continuous blocks: line flows against complex power,
analytic derivatives against finite differences, a separable closed form of the
line subproblem, and first-order optimality (KKT) of every block update checked
on states before/after one oracle iteration with the Lagrangian assembled from the
paper's row definitions (tests/ucrows.py)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2310_13145_amd import synth
from tests import ucrows

TWO_PI = 2 * np.pi


def complex_flows(r, x, b, xv):
    """S_ij = V_i conj(I_ij), S_ji = V_j conj(I_ji) for the pi model."""
    vi, vj, ti, tj = xv
    Vi, Vj = vi * np.exp(1j * ti), vj * np.exp(1j * tj)
    ys = 1 / (r + 1j * x)
    Iij = ys * (Vi - Vj) + 0.5j * b * Vi
    Iji = ys * (Vj - Vi) + 0.5j * b * Vj
    Sij, Sji = Vi * np.conj(Iij), Vj * np.conj(Iji)
    return np.array([Sij.real, Sij.imag, Sji.real, Sji.imag])


def random_branch(rng, rho_pq=5e3, rho_va=1e4, rate=None, nu=(0.0, 0.0)):
    r, x, b = rng.uniform(0.005, 0.03), rng.uniform(0.05, 0.2), rng.uniform(0, 0.2)
    adm = oracle.line_admittance(r, x, b)
    xs = np.array([rng.uniform(0.92, 1.08), rng.uniform(0.92, 1.08), rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4)])
    f = complex_flows(r, x, b, xs)
    c = np.concatenate([f + rng.normal(scale=0.05, size=4), [xs[0] ** 2 + rng.normal(scale=0.01), xs[1] ** 2 + rng.normal(scale=0.01)],
                        xs[2:] + rng.normal(scale=0.02, size=2)])
    rate = rng.uniform(1.5, 3.0) if rate is None else rate
    v = np.concatenate([adm, [rate], [0.9, 0.9, -TWO_PI, -TWO_PI], [1.1, 1.1, TWO_PI, TWO_PI], c, [rho_pq, rho_va, rho_pq], list(nu)])
    return v, (r, x, b)


def F_numpy(v, rxb, xv):
    """Line subproblem objective from its definition with complex-power flows."""
    f = complex_flows(*rxb, xv)
    c, rate = v[17:25], v[8]
    rho_pq, rho_va, mu, nu = v[25], v[26], v[27], v[28:30]
    F = 0.5 * rho_pq * np.sum((f - c[:4]) ** 2)
    F += 0.5 * rho_va * ((xv[0] ** 2 - c[4]) ** 2 + (xv[1] ** 2 - c[5]) ** 2 + (xv[2] - c[6]) ** 2 + (xv[3] - c[7]) ** 2)
    for m in range(2):
        h = f[2 * m] ** 2 + f[2 * m + 1] ** 2 - rate ** 2
        F += (max(0.0, nu[m] + mu * h) ** 2 - nu[m] ** 2) / (2 * mu)
    return F


def test_flows_match_complex_power():
    rng = np.random.default_rng(3)
    for _ in range(200):
        r, x, b = rng.uniform(0.005, 0.03), rng.uniform(0.05, 0.2), rng.uniform(0, 0.2)
        xv = np.array([rng.uniform(0.9, 1.1), rng.uniform(0.9, 1.1), rng.uniform(-3, 3), rng.uniform(-3, 3)])
        got = oracle.line_flows(oracle.line_admittance(r, x, b), xv)
        np.testing.assert_allclose(got, complex_flows(r, x, b, xv), rtol=1e-12, atol=1e-12)


def test_branch_objective_and_derivatives():
    rng = np.random.default_rng(4)
    for trial in range(60):
        # small rating so that the PHR term is active in some trials
        v, rxb = random_branch(rng, rate=rng.choice([0.3, 2.0]), nu=(rng.uniform(0, 50), 0.0))
        xv = np.array([rng.uniform(0.92, 1.08), rng.uniform(0.92, 1.08), rng.uniform(-0.4, 0.4), rng.uniform(-0.4, 0.4)])
        F, g, H = oracle.branch_eval(v, xv)
        assert F == pytest.approx(F_numpy(v, rxb, xv), rel=1e-11, abs=1e-9)
        assert F == pytest.approx(oracle.branch_F(v, xv), rel=1e-13, abs=1e-12)
        h = 1e-6
        for i in range(4):
            e = np.zeros(4); e[i] = h
            Fp, gp, _ = oracle.branch_eval(v, xv + e)
            Fm, gm, _ = oracle.branch_eval(v, xv - e)
            assert g[i] == pytest.approx((Fp - Fm) / (2 * h), rel=1e-5, abs=1e-4 * max(1.0, abs(F)) )
            np.testing.assert_allclose(H[:, i], (gp - gm) / (2 * h), rtol=1e-5, atol=1e-3 * max(1.0, np.abs(H).max()) * 1e-3)
        np.testing.assert_allclose(H, H.T, rtol=1e-13, atol=1e-9)


def test_branch_separable_closed_form():
    """rho_pq = 0 and no limit: the problem separates into (v^2 - c)^2 and (th - c)^2."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        v, _ = random_branch(rng, rho_pq=0.0, rate=1e6)
        v[27] = 1.0  # mu (unused: the limit is far)
        x, it, _ = oracle.branch_solve(v, [1.0, 1.0, 0.0, 0.0], max_iter=100, gtol=1e-10)
        c = v[17:25]
        want = [np.clip(np.sqrt(max(c[4], 0)), 0.9, 1.1), np.clip(np.sqrt(max(c[5], 0)), 0.9, 1.1), c[6], c[7]]
        np.testing.assert_allclose(x, want, rtol=1e-10, atol=1e-10)


def test_branch_solve_is_stationary_and_minimal():
    rng = np.random.default_rng(6)
    from scipy.optimize import minimize
    for trial in range(40):
        v, rxb = random_branch(rng, rate=rng.choice([0.5, 2.5]))
        gtol = 1e-8
        x, it, cg = oracle.branch_solve(v, [1.0, 1.0, 0.0, 0.0], max_iter=50, gtol=gtol)
        F, g, H = oracle.branch_eval(v, x)
        lo, hi = v[9:13], v[13:17]
        free = ~(((x <= lo) & (g > 0)) | ((x >= hi) & (g < 0)))
        assert it < 50
        Hf = H[np.ix_(free, free)]
        # the method stops at the gradient tolerance, or where its step falls below
        # 1e-15 (1 + |x|_inf): there the free-set Newton step is below the resolution
        # of x, and the gradient may sit at its rounding level just above gtol
        pg = np.max(np.abs(g[free]))
        step = np.max(np.abs(np.linalg.solve(Hf, g[free])))
        assert pg <= gtol or step <= 2e-15 * (1.0 + np.max(np.abs(x))), (trial, pg, step)
        assert np.linalg.eigvalsh(Hf).min() >= -1e-6 * np.abs(Hf).max()
        # no better point nearby (generic bounded quasi-Newton from the oracle's answer)
        res = minimize(lambda xx: F_numpy(v, rxb, xx), x, method="L-BFGS-B", bounds=list(zip(lo, hi)),
                       options=dict(ftol=1e-15, gtol=1e-12))
        assert res.fun >= F - 1e-9 * max(1.0, abs(F))


@pytest.mark.parametrize("hold", [False, True])
def test_branch_trial_projected_search(hold):
    """One trial point of the line Newton where the free Hessian is positive definite
    and the Newton step lies inside the region (Steihaug's step is the Newton step
    there).  A step that stays in the box is taken whole.  One that leaves it is
    projected; if that projection fails the model's sufficient-decrease test
    (q(s) <= 0.01 g.s), the trial stops where the ray x + alpha d first reaches a bound
    it is moving towards (TRON's projected search, found here by bisection on alpha),
    with that variable exactly on its bound and, where the trial lies on the ray, the
    model strictly decreased.  The
    sample holds projections whose model value lies in (0.01 g.s, 0]: a decrease, but
    too small, so they are searched, and free variables on a bound that the Newton step
    pushes outwards: with the hold step (taken from warm starts) those are held on the
    bound and the step solved without them (TRON's subspace step holds every variable
    on a bound); without it they are projected like the others.  (The variable that sets alpha is also placed on
    its bound explicitly, a guard: x + alpha d lands on it exactly in every case seen.)"""
    rng = np.random.default_rng(11)
    seen = {"inside": 0, "clip": 0, "search": 0, "small_decrease": 0, "held": 0}
    for trial in range(8000):
        v, _ = random_branch(rng, rate=rng.choice([0.5, 2.5]))
        v[9:11] = 0.95
        v[13:15] = 1.05
        lo, hi = v[9:13], v[13:17]
        x = np.array([rng.choice([0.951, 1.049]) + rng.normal(scale=0.002), rng.uniform(0.96, 1.04),
                      rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)])
        x = np.clip(x, lo, hi)
        F, g, H = oracle.branch_eval(v, x)
        fr = ~(((x <= lo) & (g > 0)) | ((x >= hi) & (g < 0)))
        Hf = H[np.ix_(fr, fr)]
        if np.linalg.eigvalsh(Hf).min() <= 0:
            continue
        # (CG and the direct solve below agree to about 1e-12 on these Hessians; the
        # three cases differ at the scale of the step)
        d = np.zeros(4)
        d[fr] = -np.linalg.solve(Hf, g[fr])
        # a free variable on a bound that the step pushes outwards is held there and the
        # step solved again without it
        held = fr & (((x <= lo) & (d < 0)) | ((x >= hi) & (d > 0))) & hold
        if held.any():
            fr = fr & ~held
            Hf = H[np.ix_(fr, fr)]
            if np.linalg.eigvalsh(Hf).min() <= 0:
                continue
            d = np.zeros(4)
            d[fr] = -np.linalg.solve(Hf, g[fr])
        delta = 10.0
        if np.linalg.norm(d) >= 0.5 * delta:
            continue
        seen["held"] += int(held.any())
        xt, q = oracle.branch_trial(v, x, delta, hold)
        model = lambda st: g @ st + 0.5 * st @ H @ st
        xd = x + d
        if not np.any((xd < lo) | (xd > hi)):
            seen["inside"] += 1
            np.testing.assert_allclose(xt, xd, rtol=0, atol=1e-9)
            continue
        sc = np.clip(xd, lo, hi) - x
        if model(sc) <= 0.01 * (g @ sc):
            seen["clip"] += 1
            np.testing.assert_allclose(xt, x + sc, rtol=0, atol=1e-9)
            continue
        seen["search"] += 1
        seen["small_decrease"] += model(sc) <= 0.0
        # components that move towards a bound they are not on
        mv = ((d > 0) & (x < hi)) | ((d < 0) & (x > lo))
        inside = lambda a: np.all(((x + a * d) >= lo - 1e-300) | ~mv) and np.all(((x + a * d) <= hi) | ~mv)
        a0, a1 = 0.0, 1.0
        for _ in range(200):
            am = 0.5 * (a0 + a1)
            a0, a1 = (am, a1) if inside(am) else (a0, am)
        expect = np.clip(x + a0 * d, lo, hi)
        np.testing.assert_allclose(xt, expect, rtol=0, atol=1e-9)
        on = [(i, xt[i] == (hi[i] if d[i] > 0 else lo[i])) for i in range(4) if mv[i]]
        assert any(hit for _, hit in on), (trial, xt, lo, hi)
        assert q == pytest.approx(model(xt - x), rel=1e-9, abs=1e-12)
        # the model decreases along the ray; where a variable on a bound is pushed
        # outwards its projection leaves the ray, and the ratio test decides as before
        if not np.any(((d > 0) & (x >= hi)) | ((d < 0) & (x <= lo))):
            assert model(xt - x) < 0.0
    if not hold:
        seen.pop("held")
    assert min(seen.values()) >= 3, seen


# --------------------------------------------------------------------------------
# block optimality on states around one oracle iteration
# --------------------------------------------------------------------------------

def mesh_instance():
    inst = synth.make_instance(14, 20, 5, 5, seed=77)
    return inst


@pytest.fixture(scope="module", params=["ring9", "mesh14"])
def states(request):
    inst = synth.config_instance(0) if request.param == "ring9" else mesh_instance()
    o = oracle.Oracle(inst)
    o.step(25)
    S0 = o.state()
    o.step(1)
    S1 = o.state()
    return inst, o.params, S0, S1


def lagrangian_grad(inst, params, base, var, rows_fn, zkey, ykey, rho_list):
    """Gradient of sum_r y_r (a_r + z_r) + rho_r/2 (a_r + z_r)^2 w.r.t. each entry of
    state array `var`, with rows linear in that variable (exact differences)."""
    a0 = rows_fn(inst, base)
    z = [np.asarray(base[f"{zkey}{r}"]).reshape(a0[r].shape) for r in range(len(a0))]
    y = [np.asarray(base[f"{ykey}{r}"]).reshape(a0[r].shape) for r in range(len(a0))]
    grad = np.zeros(len(base[var]))
    for k in range(len(base[var])):
        pert = dict(base)
        arr = np.array(base[var], dtype=float)
        arr[k] += 1.0
        pert[var] = arr
        a1 = rows_fn(inst, pert)
        for r in range(len(a0)):
            da = a1[r] - a0[r]
            if np.any(da):
                grad[k] += np.sum((y[r] + rho_list[r] * (a0[r] + z[r])) * da)
    return grad


def gen_rows_list(inst, S):
    d = ucrows.gen_rows(inst, S)
    return [d[n] for n in ucrows.GEN_ROWS]


def mixed(S_new, S_old, new_keys):
    out = dict(S_old)
    for k in new_keys:
        out[k] = S_new[k]
    return out


def kkt_box(x, g, lo, hi, scale):
    tol = 1e-9 * scale
    at_lo = x <= lo + 1e-13
    at_hi = x >= hi - 1e-13
    inner = ~(at_lo | at_hi)
    assert np.all(np.abs(g[inner]) <= tol), np.abs(g[inner]).max()
    assert np.all(g[at_lo & ~at_hi] >= -tol)
    assert np.all(g[at_hi & ~at_lo] <= tol)


def test_generator_block_kkt(states):
    inst, par, S0, S1 = states
    _, rg = ucrows.rhos(par)
    T, G = inst["T"], inst["n_gen"]
    gen_vars = ["p", "q", "s1", "s2", "s3", "s4", "s5", "s6"]
    base = mixed(S1, S0, gen_vars)  # new x_gen, everything else as at the start of the iteration
    k2 = np.tile(inst["gen_c2"] * 1e4, T)
    k1 = np.tile(inst["gen_c1"] * 100, T)
    qlo = np.tile(np.minimum(0, inst["gen_qmin"]), T)
    qhi = np.tile(np.maximum(0, inst["gen_qmax"]), T)
    for var in gen_vars:
        g = lagrangian_grad(inst, par, base, var, gen_rows_list, "zG", "yG", rg)
        x = np.asarray(base[var])
        if var == "p":
            g = g + 2 * k2 * x + k1
            lo, hi = np.zeros_like(x), np.tile(inst["gen_pmax"], T)
        elif var == "q":
            lo, hi = qlo, qhi
        else:
            lo, hi = np.zeros_like(x), np.full_like(x, np.inf)
        kkt_box(x, g, lo, hi, scale=max(par.rho_pq, par.rho_cpl))


def test_ubar_block_kkt(states):
    inst, par, S0, S1 = states
    _, rg = ucrows.rhos(par)
    x_keys = ["p", "q", "s1", "s2", "s3", "s4", "s5", "s6", "uon", "usu", "usd"]
    base = mixed(S1, S0, x_keys + ["ubon", "ubsu", "ubsd"])  # old pbar (Jacobi)
    for var in ("ubon", "ubsu", "ubsd"):
        g = lagrangian_grad(inst, par, base, var, gen_rows_list, "zG", "yG", rg)
        x = np.asarray(base[var])
        kkt_box(x, g, np.zeros_like(x), np.ones_like(x), scale=par.rho_uc)


def test_bus_block_kkt(states):
    """Stationarity: the gradient of the bus-block Lagrangian terms lies in the span of
    the balance constraints' gradients (least squares residual ~ 0), and the balance
    equations (uc_acopf_p_balance, uc_acopf_q_balance) hold."""
    inst, par, S0, S1 = states
    rb, rg = ucrows.rhos(par)
    N, L, G, T = inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"]
    x_keys = ["vf", "vt", "thf", "tht", "pf", "qf", "pt", "qt", "p", "q", "s1", "s2", "s3", "s4", "s5", "s6", "uon", "usu", "usd"]
    bus_keys = ["wb", "thb", "Pbf", "Qbf", "Pbt", "Qbt", "pb", "qb"]
    base = mixed(S1, S0, x_keys + bus_keys)  # old ubar (Jacobi)
    grads = {}
    for var in bus_keys:
        gl = lagrangian_grad(inst, par, base, var, ucrows.line_rows, "zB", "yB", rb)
        gg = lagrangian_grad(inst, par, base, var, gen_rows_list, "zG", "yG", rg)
        grads[var] = gl + gg
    fr, to, gb = inst["line_from"], inst["line_to"], inst["gen_bus"]
    sh = lambda k, n: np.asarray(base[k]).reshape(T, n)
    for t in range(T):
        # balance residuals
        Pbal = np.zeros(N); Qbal = np.zeros(N)
        np.add.at(Pbal, gb, sh("pb", G)[t]); np.add.at(Qbal, gb, sh("qb", G)[t])
        np.add.at(Pbal, fr, -sh("Pbf", L)[t]); np.add.at(Pbal, to, -sh("Pbt", L)[t])
        np.add.at(Qbal, fr, -sh("Qbf", L)[t]); np.add.at(Qbal, to, -sh("Qbt", L)[t])
        Pbal -= inst["bus_gs"] * sh("wb", N)[t]; Qbal += inst["bus_bs"] * sh("wb", N)[t]
        np.testing.assert_allclose(Pbal, inst["load_p"][t], atol=1e-11)
        np.testing.assert_allclose(Qbal, inst["load_q"][t], atol=1e-11)
    for t in range(T):
        for i in range(N):
            # variables of bus i at period t and their constraint coefficients
            entries = []
            for l in np.where(fr == i)[0]:
                entries += [("Pbf", t * L + l, -1, 0), ("Qbf", t * L + l, 0, -1)]
            for l in np.where(to == i)[0]:
                entries += [("Pbt", t * L + l, -1, 0), ("Qbt", t * L + l, 0, -1)]
            for g in np.where(gb == i)[0]:
                entries += [("pb", t * G + g, 1, 0), ("qb", t * G + g, 0, 1)]
            entries += [("wb", t * N + i, -inst["bus_gs"][i], inst["bus_bs"][i])]
            gvec = np.array([grads[k][idx] for k, idx, _, _ in entries])
            A = np.array([[a, b] for _, _, a, b in entries])
            mu, *_ = np.linalg.lstsq(A, gvec, rcond=None)
            assert np.abs(gvec - A @ mu).max() <= 1e-8 * max(par.rho_pq, par.rho_va)
            th = grads["thb"][t * N + i]
            if i != inst["ref_bus"]:
                assert abs(th) <= 1e-8 * par.rho_va
            else:
                assert base["thb"][t * N + i] == 0.0


def test_uc_block_is_optimal(states):
    """The DP's commitments minimise the UC-block Lagrangian over set:UC (brute force)."""
    inst, par, S0, S1 = states
    T, G = inst["T"], inst["n_gen"]
    from tests.test_oracle_dp import feasible
    sh = lambda k: np.asarray(S0[k]).reshape(T, G)
    ub = [sh("ubon"), sh("ubsu"), sh("ubsd")]
    z = [sh("zG8"), sh("zG9"), sh("zG10")]
    y = [sh("yG8"), sh("yG9"), sh("yG10")]
    got = np.asarray(S1["uon"]).reshape(T, G)
    for g in range(G):
        u0, TU, TD = int(inst["gen_u0"][g]), int(inst["gen_min_up"][g]), int(inst["gen_min_dn"][g])
        best, best_u = np.inf, None
        def cost(u):
            c = 0.0
            for t in range(T):
                prev = u0 if t == 0 else u[t - 1]
                uu = [u[t], max(0, u[t] - prev), max(0, prev - u[t])]
                c += inst["gen_cnl"][g] * uu[0] + inst["gen_csu"][g] * uu[1] + inst["gen_csd"][g] * uu[2]
                for k in range(3):
                    r = uu[k] - ub[k][t, g] + z[k][t, g]
                    c += y[k][t, g] * r + par.rho_uc / 2 * r * r
            return c
        for u in itertools.product((0, 1), repeat=T):
            su = [max(0, u[t] - (u0 if t == 0 else u[t - 1])) for t in range(T)]
            sd = [max(0, (u0 if t == 0 else u[t - 1]) - u[t]) for t in range(T)]
            if not feasible(u, su, sd, u0, int(inst["gen_init_on"][g]), int(inst["gen_init_off"][g]), TU, TD):
                continue
            c = cost(u)
            if c < best:
                best, best_u = c, u
        assert cost(tuple(int(v) for v in got[:, g])) == pytest.approx(best, rel=1e-12, abs=1e-9)


def test_line_block_stationary(states):
    inst, par, S0, S1 = states
    N, L, T = inst["n_bus"], inst["n_line"], inst["T"]
    fr, to = inst["line_from"], inst["line_to"]
    rb, _ = ucrows.rhos(par)
    gtol = 1e-12 * max(1, par.rho_pq, par.rho_va)
    for t in range(T):
        for l in range(L):
            k = t * L + l
            xb = [S0["Pbf"][k], S0["Qbf"][k], S0["Pbt"][k], S0["Qbt"][k],
                  S0["wb"][t * N + fr[l]], S0["wb"][t * N + to[l]], S0["thb"][t * N + fr[l]], S0["thb"][t * N + to[l]]]
            c = [xb[r] - S0[f"zB{r}"][k] - S0[f"yB{r}"][k] / rb[r] for r in range(8)]
            adm = oracle.line_admittance(inst["line_r"][l], inst["line_x"][l], inst["line_b"][l])
            lo = [inst["bus_vmin"][fr[l]], inst["bus_vmin"][to[l]], -TWO_PI, -TWO_PI]
            hi = [inst["bus_vmax"][fr[l]], inst["bus_vmax"][to[l]], TWO_PI, TWO_PI]
            v = np.concatenate([adm, [inst["line_rate"][l]], lo, hi, c, [par.rho_pq, par.rho_va, par.mu_line, S0["nuf"][k], S0["nut"][k]]])
            x = np.array([S1["vf"][k], S1["vt"][k], S1["thf"][k], S1["tht"][k]])
            F, g, H = oracle.branch_eval(v, x)
            free = ~(((x <= lo) & (g > 0)) | ((x >= hi) & (g < 0)))
            assert np.abs(g[free]).max(initial=0) <= gtol * 1.0001
            f = complex_flows(inst["line_r"][l], inst["line_x"][l], inst["line_b"][l], x)
            np.testing.assert_allclose([S1["pf"][k], S1["qf"][k], S1["pt"][k], S1["qt"][k]], f, rtol=1e-12, atol=1e-12)
            hf = f[0] ** 2 + f[1] ** 2 - inst["line_rate"][l] ** 2
            assert S1["nuf"][k] == pytest.approx(max(0.0, S0["nuf"][k] + par.mu_line * hf), rel=1e-12, abs=1e-12)


def test_z_and_y_updates(states):
    """step:z makes dL/dz = lambda + beta z + y + rho (a + z) vanish; step:y then gives
    y_new = y_old + rho (a + z), so lambda + beta z + y_new = 0 row by row."""
    inst, par, S0, S1 = states
    rb, rg = ucrows.rhos(par)
    beta = S0["beta"]
    a_line = ucrows.line_rows(inst, S1)
    a_gen = gen_rows_list(inst, S1)
    for kind, a_list, rho in (("B", a_line, rb), ("G", a_gen, rg)):
        for r in range(len(a_list)):
            z, y1, y0, lam = (np.asarray(S1[f"z{kind}{r}"]), np.asarray(S1[f"y{kind}{r}"]),
                              np.asarray(S0[f"y{kind}{r}"]), np.asarray(S1[f"l{kind}{r}"]))
            lam0 = np.asarray(S0[f"l{kind}{r}"])
            a = a_list[r].ravel()
            np.testing.assert_allclose(y1, y0 + rho[r] * (a + z), rtol=1e-12, atol=1e-9)
            if S1["k_outer"] == S0["k_outer"]:
                np.testing.assert_allclose(lam0 + beta * z + y1, 0.0, atol=1e-9 * max(1.0, np.abs(y1).max()))


# --------------------------------------------------------------------------------
# pins that switch on features the synthetic workloads leave off
# --------------------------------------------------------------------------------

def gen_block_objective_grad(data, rho, xin, z, y, v):
    """Gradient of the generator-block objective (cost + Lagrangian terms of rows
    G1, G2, C1..C6) w.r.t. (p, q, s1..s6), from the row definitions."""
    k2, k1, pmax, qlo, qhi, Plo, Pup, Qlo, Qup, RU, RD, SU, SD = data
    pb, qb, pbp, uon, uonp, usu, usd = xin
    p, q, s1, s2, s3, s4, s5, s6 = v
    rows = [  # (a_r, d a_r / d (p, q, s1..s6))
        (p - pb, [1, 0, 0, 0, 0, 0, 0, 0]),
        (q - qb, [0, 1, 0, 0, 0, 0, 0, 0]),
        (p - s1 - Plo * uon, [1, 0, -1, 0, 0, 0, 0, 0]),
        (p + s2 - Pup * uon, [1, 0, 0, 1, 0, 0, 0, 0]),
        (q - s3 - Qlo * uon, [0, 1, 0, 0, -1, 0, 0, 0]),
        (q + s4 - Qup * uon, [0, 1, 0, 0, 0, 1, 0, 0]),
        (p - pbp - s5 + RD * uon + SD * usd, [1, 0, 0, 0, 0, 0, -1, 0]),
        (p - pbp + s6 - RU * uonp - SU * usu, [1, 0, 0, 0, 0, 0, 0, 1]),
    ]
    rr = [rho[0], rho[0]] + [rho[1]] * 6
    g = np.zeros(8)
    g[0] += 2 * k2 * p + k1
    for r, (a, da) in enumerate(rows):
        g += (y[r] + rr[r] * (a + z[r])) * np.array(da, float)
    return g


def test_generator_block_kkt_random():
    """Random multipliers and duplicates so that every slack row binds somewhere."""
    rng = np.random.default_rng(11)
    active = np.zeros(8, bool)
    for trial in range(400):
        Pup = rng.uniform(1, 3)
        data = [rng.uniform(100, 1000), rng.uniform(1000, 4000), Pup, -0.3 * Pup, 0.6 * Pup,
                0.2 * Pup, Pup, -0.3 * Pup, 0.6 * Pup, 0.5 * Pup, 0.5 * Pup, 0.5 * Pup, 0.5 * Pup]
        rho = [5e3, rng.choice([5e3, 5e4])]
        xin = [rng.uniform(0, Pup), rng.uniform(-0.3, 0.6) * Pup, rng.uniform(0, Pup), rng.uniform(0, 1),
               rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0, 1)]
        z = rng.normal(scale=0.3, size=8)
        y = rng.normal(scale=2000, size=8)
        v = oracle.gen_solve(data, rho, xin, z, y)
        g = gen_block_objective_grad(data, rho, xin, z, y, v)
        lo = np.array([0, data[3] if data[3] < 0 else 0] + [0] * 6, float)
        hi = np.array([data[2], max(0, data[4])] + [np.inf] * 6)
        kkt_box(v, g, lo, hi, scale=1e5)
        active |= v > 1e-12
    assert active[2:].all()  # every slack was positive in some trial


def test_bus_block_with_shunts_and_ramp_rows():
    """Bus KKT on a mesh with shunts (the G^s, B^s terms of the balance equations)."""
    inst = synth.small_instance(14, 20, 5, 5, seed=78)
    rng = np.random.default_rng(12)
    inst["bus_gs"] = rng.uniform(0.0, 0.05, 14)
    inst["bus_bs"] = rng.uniform(-0.2, 0.2, 14)
    o = oracle.Oracle(inst)
    o.step(20)
    S0 = o.state(); o.step(1); S1 = o.state()
    test_bus_block_kkt((inst, o.params, S0, S1))


def test_ubar_block_kkt_with_start_ups():
    """Relaxed-commitment KKT where units start up in the horizon (u_su = 1 at the
    first period of the units that begin off), so the U2 rows of t + 1 matter."""
    inst = synth.small_instance(14, 20, 5, 5, seed=81)
    inst["gen_u0"] = np.array([0, 1, 1, 0, 1], np.int32)
    o = oracle.Oracle(inst)
    o.step(20)
    S0 = o.state(); o.step(1); S1 = o.state()
    assert S1["usu"].max() == 1.0
    test_ubar_block_kkt((inst, o.params, S0, S1))


def test_line_limits_active():
    """Tight ratings make the PHR term active; the line block stays stationary and
    nu follows nu <- max(0, nu + mu h) at each end."""
    inst = synth.small_instance(14, 20, 5, 5, seed=79)
    inst["line_rate"] = inst["line_rate"] * 0.15
    o = oracle.Oracle(inst)
    o.step(30)
    S0 = o.state(); o.step(1); S1 = o.state()
    assert (S1["nuf"] > 0).sum() > 0 and (S1["nut"] > 0).sum() > 0
    test_line_block_stationary((inst, o.params, S0, S1))


def test_outer_update_lambda():
    """step:outer: lambda <- clamp(lambda + beta z) at the iteration that ends an inner loop."""
    inst = synth.config_instance(0)
    o = oracle.Oracle(inst)
    prev = o.state()
    for _ in range(2000):
        o.step(1)
        S = o.state()
        if S["k_outer"] != prev["k_outer"]:
            for kind, nr in (("B", 8), ("G", 11)):
                for r in range(nr):
                    want = np.clip(prev[f"l{kind}{r}"] + prev["beta"] * S[f"z{kind}{r}"], -1e12, 1e12)
                    np.testing.assert_allclose(S[f"l{kind}{r}"], want, rtol=1e-14, atol=0)
            return
        prev = S
    pytest.fail("no outer update")


def test_initial_state_cold_start():
    """Cold start: v mid-bounds, angles 0, flows from voltages, duplicates equal to the
    originals, all committed, slacks at their feasible projection, multipliers 0."""
    inst = synth.small_instance(14, 20, 5, 5, seed=80)
    inst["gen_u0"] = np.array([0, 1, 0, 1, 1], np.int32)  # two units start up in period 1
    o = oracle.Oracle(inst)
    S = o.state()
    T, G = inst["T"], inst["n_gen"]
    fr, to = inst["line_from"], inst["line_to"]
    vm = 0.5 * (inst["bus_vmin"] + inst["bus_vmax"])
    assert np.all(S["vf"].reshape(T, -1) == vm[fr]) and np.all(S["thf"] == 0) and np.all(S["tht"] == 0)
    for l in range(inst["n_line"]):
        f = complex_flows(inst["line_r"][l], inst["line_x"][l], inst["line_b"][l], [vm[fr[l]], vm[to[l]], 0, 0])
        np.testing.assert_allclose([S["pf"][l], S["qf"][l], S["pt"][l], S["qt"][l]], f, rtol=1e-12, atol=1e-14)
    np.testing.assert_array_equal(S["Pbf"], S["pf"]); np.testing.assert_array_equal(S["pb"], S["p"])
    assert np.all(S["uon"] == 1) and np.all(S["ubon"] == 1)
    assert np.array_equal(S["usu"].reshape(T, G)[0], 1 - inst["gen_u0"]) and np.all(S["usu"].reshape(T, G)[1:] == 0)
    rows = ucrows.gen_rows(inst, S)
    for name, sign in (("C1", -1), ("C2", 1), ("C3", -1), ("C4", 1), ("C5", -1), ("C6", 1)):
        a = rows[name]
        # a "-s" row is satisfied or negative with s = 0; a "+s" row is satisfied or positive
        assert np.all(a * sign >= -1e-15)
        s = S[f"s{name[1]}"].reshape(T, G)
        assert np.all(s >= 0)
        assert np.all((np.abs(a) <= 1e-15) | (s == 0))
    for k in ("zB0", "yB0", "lG5", "nuf"):
        assert np.all(S[k] == 0)
    assert S["beta"] == o.params.beta0
