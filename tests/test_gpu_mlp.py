"""Learned warm start on the GPU against the FP64 oracle of the network
(oracle/mlp.py, BF16 rounding emulated at the kernels' rounding points), the
pair logging against host-computed inputs and solutions, and the learned start
inside the ADMM against the plain method.

Tolerances: the kernels accumulate in FP32 where the oracle uses FP64, so a
hidden activation can land on the other side of a BF16 rounding boundary (one
BF16 ulp, 2^-8 relative).  Such flips are rare and each moves an output by about
2^-8 |a| |w|; outputs are compared at 1e-2 absolute on unit-scale values and
2e-3 in relative L2 norm.  Gradients are compared element by element: every entry
of a parameter block within 2^-5 of that block's largest entry (a flipped BF16
operand changes one product of a sum by 2^-8 of its size, and a block's entries
are sums of at most a few hundred such products of comparable size) plus 2^-6 of
the entry itself, and the whole block within 1e-2 in relative L2 norm.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as om
from paper_2310_13145_amd import synth, ucac

pytestmark = pytest.mark.gpu


def _feats(rng, n):
    """Inputs on the scale of the real features (unit order, a few larger)."""
    return rng.normal(0.0, 1.0, (n, om.N_IN)) * rng.uniform(0.2, 2.0, om.N_IN)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [1, 64, 257, 1000])
def test_forward_matches_oracle(n):
    print(f"[mlp] forward n={n}", flush=True)
    rng = np.random.default_rng(100 + n)
    vec = om.init_params(7)
    vec[om.N_H * om.N_IN:om.N_H * om.N_IN + om.N_H] = rng.normal(0, 0.1, om.N_H)  # nonzero b1
    X = _feats(rng, n).astype(np.float32)
    net = ucac.WarmStartNet(seed=1)
    net.set_weights(vec.astype(np.float32))
    y = net.forward(X)
    ref, _ = om.forward(vec.astype(np.float32).astype(np.float64), X.astype(np.float64), rounding=True)
    assert y.shape == (n, 4)
    assert np.max(np.abs(y - ref)) <= 1e-2, np.max(np.abs(y - ref))
    assert _rel(y, ref) <= 2e-3
    # and far from the unrounded network's outputs only by BF16 effects
    ref64, _ = om.forward(vec, X.astype(np.float64), rounding=False)
    assert _rel(y, ref64) <= 5e-2
    net.close()


def test_forward_empty_and_weights_roundtrip():
    net = ucac.WarmStartNet(seed=3)
    w = net.get_weights()
    assert w.shape == (ucac.MLP_PARAMS,) and np.all(np.isfinite(w))
    ref = om.init_params(0)  # same distribution: bounds 1/sqrt(fan_in), zero biases
    P = om.unpack(w.astype(np.float64))
    assert np.all(np.abs(P["W1"]) <= 1 / np.sqrt(20) + 1e-7) and np.all(P["b1"] == 0) and np.all(P["b3"] == 0)
    assert ref.size == w.size
    assert net.forward(np.zeros((0, 20), np.float32)).shape == (0, 4)
    with pytest.raises(ucac.UcacError):
        net.set_weights(np.zeros(10, np.float32))
    net.close()


@pytest.mark.parametrize("n", [64, 300])
def test_gradient_matches_oracle(n):
    print(f"[mlp] gradient n={n}", flush=True)
    rng = np.random.default_rng(200 + n)
    vec = om.init_params(11)
    vec += rng.normal(0, 0.02, vec.size)  # nonzero biases everywhere
    vec32 = vec.astype(np.float32)
    X = _feats(rng, n).astype(np.float32)
    Y = rng.normal(0, 0.5, (n, 4)).astype(np.float32)
    net = ucac.WarmStartNet()
    net.set_weights(vec32)
    g, ls = net.grad(X, Y)
    gr, lr_ = om.grad(vec32.astype(np.float64), X.astype(np.float64), Y.astype(np.float64), rounding=True)
    assert abs(ls - lr_) <= 1e-2 * lr_
    P, R = om.unpack(g.astype(np.float64)), om.unpack(gr)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert _rel(P[k], R[k]) <= 1e-2, (k, _rel(P[k], R[k]))
        scale = np.abs(R[k]).max()
        err = np.abs(P[k] - R[k])
        bound = 2.0 ** -5 * scale + 2.0 ** -6 * np.abs(R[k])
        assert np.all(err <= bound), (k, float((err / scale).max()), np.unravel_index(np.argmax(err - bound), err.shape))
    # the weights are unchanged by a gradient evaluation
    np.testing.assert_array_equal(net.get_weights(), vec32)
    net.close()


def test_adam_step_matches_formula():
    """One full-batch Adam step: new weights = old - lr * m_hat / (sqrt(v_hat) + eps)
    with the device's own gradient (bias-corrected, t = 1)."""
    rng = np.random.default_rng(5)
    n, lr = 256, 1e-3
    vec32 = om.init_params(2).astype(np.float32)
    X = _feats(rng, n).astype(np.float32)
    Y = rng.normal(0, 0.5, (n, 4)).astype(np.float32)
    net = ucac.WarmStartNet()
    net.set_weights(vec32)
    g, _ = net.grad(X, Y)
    net.train(X, Y, epochs=1, batch=n, lr=lr, seed=1)
    w1 = net.get_weights().astype(np.float64)
    ref, _, _ = om.adam(vec32.astype(np.float64), g.astype(np.float64), np.zeros(g.size), np.zeros(g.size), 1, lr)
    big = np.abs(g) > 1e-5
    assert big.sum() > 0.9 * g.size
    assert np.max(np.abs(w1 - ref)[big]) <= 1e-3 * lr + 1e-7
    assert np.max(np.abs(w1 - vec32)) <= lr * (1 + 1e-3) + 1e-7
    net.close()


def test_adam_later_steps_match_oracle():
    """Three full-batch Adam steps in a row (t = 1, 2, 3, moments carried across
    calls): each step's new weights equal the oracle's Adam update applied to the
    device's own gradient at the weights of that step, with the oracle's moments
    accumulated over the same gradients.  From t = 2 on the update depends on
    beta1 and beta2 separately."""
    rng = np.random.default_rng(6)
    n, lr = 256, 1e-3
    vec32 = om.init_params(12).astype(np.float32)
    X = _feats(rng, n).astype(np.float32)
    Y = rng.normal(0, 0.5, (n, 4)).astype(np.float32)
    net = ucac.WarmStartNet()
    net.set_weights(vec32)
    w = vec32.astype(np.float64)
    m = np.zeros(w.size); v = np.zeros(w.size)
    for t in (1, 2, 3):
        print(f"[mlp] adam step t={t}", flush=True)
        g, _ = net.grad(X, Y)
        g = g.astype(np.float64)
        net.train(X, Y, epochs=1, batch=n, lr=lr, seed=t)
        w_dev = net.get_weights().astype(np.float64)
        ref, m, v = om.adam(w, g, m, v, t, lr)
        big = np.abs(g) > 1e-5
        assert big.sum() > 0.9 * g.size
        assert np.max(np.abs(w_dev - ref)[big]) <= 2e-3 * lr + 1e-7, (t, np.max(np.abs(w_dev - ref)[big]))
        w = w_dev
    net.close()


def test_training_fits_a_teacher():
    """Pairs from a fixed teacher network: Adam on the device lowers the loss well
    below that of the starting network, and the oracle agrees on the trained
    network's loss."""
    rng = np.random.default_rng(9)
    n = 4096
    teacher = om.init_params(123)
    X = _feats(rng, n).astype(np.float32)
    Y, _ = om.forward(teacher, X.astype(np.float64), rounding=False)
    Y = Y.astype(np.float32)
    net = ucac.WarmStartNet(seed=4)
    l0 = om.loss(net.get_weights().astype(np.float64), X, Y)
    last = net.train(X, Y, epochs=30, batch=128, lr=3e-3, seed=2)
    w = net.get_weights().astype(np.float64)
    l1 = om.loss(w, X.astype(np.float64), Y.astype(np.float64), rounding=True)
    print(f"[mlp] teacher loss {l0:.3e} -> {l1:.3e} (device last pass {last:.3e})", flush=True)
    assert l1 < 0.1 * l0
    assert abs(last - l1) <= 0.5 * l1 + 1e-6
    net.close()


def _expected_features(inst, p, s0):
    """The 20 inputs of every line solve of an iteration started from state s0 (host FP64)."""
    N, L, G, T = inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"]
    st = ucac.split_state(s0, N, L, G, T)
    adm = np.array([oracle.line_admittance(inst["line_r"][l], inst["line_x"][l], inst["line_b"][l]) for l in range(L)])
    fr, to = inst["line_from"], inst["line_to"]
    f = np.zeros((T, L, 20))
    rho = [p.rho_pq] * 4 + [p.rho_va] * 4
    wb, thb = st["wb"].reshape(T, N), st["thb"].reshape(T, N)
    xb = [st["Pbf"], st["Qbf"], st["Pbt"], st["Qbt"], wb[:, fr], wb[:, to], thb[:, fr], thb[:, to]]
    c = [xb[r].reshape(T, L) - st[f"zB{r}"].reshape(T, L) - st[f"yB{r}"].reshape(T, L) / rho[r] for r in range(8)]
    rate = inst["line_rate"]
    f[..., 0] = 0.1 * adm[:, 0]
    f[..., 1] = 0.05 * adm[:, 3]
    f[..., 2] = 10.0 * (adm[:, 1] + adm[:, 3])
    f[..., 3] = rate / 3.0
    for r in range(4):
        f[..., 4 + r] = c[r]
    f[..., 8] = c[4] - 1.0
    f[..., 9] = c[5] - 1.0
    f[..., 10] = 5.0 * (c[6] - c[7])
    f[..., 11] = st["nuf"].reshape(T, L) / p.mu_line
    f[..., 12] = st["nut"].reshape(T, L) / p.mu_line
    f[..., 13] = inst["bus_vmin"][fr] - 1.0
    f[..., 14] = inst["bus_vmax"][fr] - 1.0
    f[..., 15] = inst["bus_vmin"][to] - 1.0
    f[..., 16] = inst["bus_vmax"][to] - 1.0
    f[..., 17] = np.log10(p.rho_pq) - 4.0
    f[..., 18] = np.log10(p.rho_va) - 4.0
    f[..., 19] = (c[0] ** 2 + c[1] ** 2 - rate ** 2) / rate ** 2
    return f.reshape(T * L, 20), c


def _sort_rows(a, keys):
    order = np.lexsort(tuple(a[:, k] for k in reversed(keys)))
    return a[order]


def test_log_pairs_inputs_and_solutions():
    """One logged iteration: the inputs match the host computation from the starting
    state and the targets match the solution the iteration left in the state."""
    inst = synth.config_instance(1)
    N, L, G, T = inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"]
    g = ucac.Solver(inst)
    g.step(30)
    s0 = g.get_state()
    feats, targs = g.log_pairs(1, stride=1)
    s1 = g.get_state()
    assert feats.shape == (T * L, 20) and targs.shape == (T * L, 4)
    ef, c = _expected_features(inst, g.params, s0)
    st1 = ucac.split_state(s1, N, L, G, T)
    et = np.stack([st1["vf"] - 1.0, st1["vt"] - 1.0, 10.0 * (st1["thf"] - c[6].ravel()),
                   10.0 * (st1["tht"] - c[7].ravel())], axis=1)
    # rows come back in completion order: compare as sorted sets of (input, target) rows
    got = _sort_rows(np.hstack([feats, targs]).astype(np.float64), [4, 5, 6, 7])
    exp = _sort_rows(np.hstack([ef.astype(np.float32), et.astype(np.float32)]).astype(np.float64), [4, 5, 6, 7])
    np.testing.assert_allclose(got, exp, rtol=1e-5, atol=1e-6)
    # a logging run is an ordinary iteration: it matches the unlogged one bit for bit
    h = ucac.Solver(inst)
    h.step(31)
    np.testing.assert_array_equal(h.get_state(), s1)
    # stride and capacity
    f2, t2 = g.log_pairs(4, stride=4)
    assert f2.shape[0] == T * L  # each solve logged once over four iterations
    f3, _ = g.log_pairs(2, stride=1, cap=100)
    assert f3.shape[0] == 100
    g.close(), h.close()


def test_learned_start_random_net_same_iterates():
    """With an untrained network the learned start still reaches the same iterates as
    the oracle's flat-start method (Newton converges to the same point to its
    tolerance; lanes that do not converge fall back to the flat start)."""
    from test_gpu_parity import compare
    inst = synth.config_instance(1)
    g = ucac.Solver(inst)
    net = ucac.WarmStartNet(seed=8)
    g.set_warmstart(net.get_weights())
    o = oracle.Oracle(inst)
    g.branch_counters(reset=True)
    for k in range(5):
        g.step(10)
        o.step(10)
        compare(g.get_state(), o.get_state(), inst, 1e-8, f"learned random net, iteration {10 * (k + 1)}")
    cnt = g.branch_counters()
    print(f"[mlp] random-net counters {cnt}", flush=True)
    # back to the plain start
    g.set_warmstart(None)
    g.step(5)
    o.step(5)
    compare(g.get_state(), o.get_state(), inst, 1e-8, "after reverting to flat start")
    with pytest.raises(ucac.UcacError):
        g.set_warmstart(np.full(ucac.MLP_PARAMS, np.nan, np.float32))
    with pytest.raises(ucac.UcacError):
        g.set_warmstart(np.zeros(5, np.float32))
    g.close(), net.close()


def test_trained_net_cuts_newton_work():
    """Train on pairs logged from other seeds of the same distribution, then on a
    fresh instance: the learned start needs fewer Newton iterations than the flat
    start, and the iterates still match the oracle."""
    from test_gpu_parity import compare
    X, Y = [], []
    for seed in (1, 2):
        inst_tr = synth.small_instance(118, 186, 54, 24, seed=500 + seed)
        s = ucac.Solver(inst_tr)
        f, t = s.log_pairs(300, stride=10)
        X.append(f), Y.append(t)
        s.close()
    X, Y = np.vstack(X), np.vstack(Y)
    net = ucac.WarmStartNet(seed=0)
    l0 = net.train(X, Y, epochs=1, batch=256, lr=1e-3, seed=0)
    l1 = net.train(X, Y, epochs=15, batch=256, lr=1e-3, seed=1)
    print(f"[mlp] trained on {X.shape[0]} pairs: loss {l0:.3e} -> {l1:.3e}", flush=True)
    assert l1 < 0.5 * l0
    inst = synth.config_instance(1)
    plain = ucac.Solver(inst)
    learned = ucac.Solver(inst)
    learned.set_warmstart(net.get_weights())
    plain.step(100), learned.step(100)
    plain.branch_counters(reset=True), learned.branch_counters(reset=True)
    plain.step(100), learned.step(100)
    cp, cl = plain.branch_counters(), learned.branch_counters()
    print(f"[mlp] newton iterations per 100 ADMM iterations: flat {cp['newton']}, learned {cl['newton']} "
          f"(fallbacks {cl['fallbacks']})", flush=True)
    assert cl["newton"] < cp["newton"]
    o = oracle.Oracle(inst)
    o.step(200)
    compare(learned.get_state(), o.get_state(), inst, 1e-8, "trained learned start, 200 iterations")
    plain.close(), learned.close(), net.close()


def test_line_start_points_match_oracle_network():
    """The network inside the ADMM (the learned-start kernel that predicts each line
    solve's Newton start): its decoded start points equal the FP64 oracle network
    (BF16 rounding at the kernel's rounding points) applied to the host-computed
    inputs of the same iteration, decoded the same way (v = 1 + y0, 1 + y1;
    theta = angle target + y2 / 10, + y3 / 10), within the forward pass's tolerance."""
    inst = synth.config_instance(1)
    N, L, G, T = inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"]
    g = ucac.Solver(inst)
    g.step(30)
    s0 = g.get_state()
    rng = np.random.default_rng(31)
    vec = om.init_params(17)
    vec += rng.normal(0, 0.05, vec.size)  # nonzero biases, outputs away from zero
    w = vec.astype(np.float32)
    g.set_warmstart(w)
    g.step(1)
    x0 = g.line_starts().astype(np.float64)
    ef, c = _expected_features(inst, g.params, s0)
    y, _ = om.forward(w.astype(np.float64), ef.astype(np.float32).astype(np.float64), rounding=True)
    ref = np.stack([1.0 + y[:, 0], 1.0 + y[:, 1], c[6].ravel() + 0.1 * y[:, 2], c[7].ravel() + 0.1 * y[:, 3]])
    err_v = np.max(np.abs(x0[:2] - ref[:2]))
    err_t = np.max(np.abs(x0[2:] - ref[2:]))
    print(f"[mlp] start points vs oracle network: |dv| {err_v:.2e}, |dtheta| {err_t:.2e}", flush=True)
    assert err_v <= 1e-2 and err_t <= 1e-3
    raw = np.stack([x0[0] - 1.0, x0[1] - 1.0, 10.0 * (x0[2] - c[6].ravel()), 10.0 * (x0[3] - c[7].ravel())], axis=1)
    assert _rel(raw, y) <= 2e-3
    g.close()
