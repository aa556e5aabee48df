"""Row definitions of the extended UC-ACOPF problem, written from the paper for the
tests (eq:uc-acopf-ext with the slack rows, the component consensus rows, and the
augmented Lagrangian L_{beta,rho} of Sec. III).  Used only to check block
optimality and invariants of the oracle with generic solvers; it implements no
block solver."""
import numpy as np

GEN_ROWS = ["G1", "G2", "C1", "C2", "C3", "C4", "C5", "C6", "U1", "U2", "U3"]


def gen_rows(inst, S):
    """a_r of the generator-side rows, each [T, G], from a state dict S."""
    G, T = inst["n_gen"], inst["T"]
    sh = lambda a: np.asarray(a).reshape(T, G)
    p, q = sh(S["p"]), sh(S["q"])
    s = [sh(S[f"s{k}"]) for k in range(1, 7)]
    pb, qb = sh(S["pb"]), sh(S["qb"])
    ub, ubsu, ubsd = sh(S["ubon"]), sh(S["ubsu"]), sh(S["ubsd"])
    pbp = np.vstack([inst["gen_p0"][None, :], pb[:-1]])
    ubp = np.vstack([inst["gen_u0"][None, :].astype(float), ub[:-1]])
    return {
        "G1": p - pb, "G2": q - qb,
        "C1": p - s[0] - inst["gen_pmin"] * ub,
        "C2": p + s[1] - inst["gen_pmax"] * ub,
        "C3": q - s[2] - inst["gen_qmin"] * ub,
        "C4": q + s[3] - inst["gen_qmax"] * ub,
        "C5": p - pbp - s[4] + inst["gen_rd"] * ub + inst["gen_sd"] * ubsd,
        "C6": p - pbp + s[5] - inst["gen_ru"] * ubp - inst["gen_su"] * ubsu,
        "U1": sh(S["uon"]) - ub, "U2": sh(S["usu"]) - ubsu, "U3": sh(S["usd"]) - ubsd,
    }


def line_rows(inst, S):
    N, L, T = inst["n_bus"], inst["n_line"], inst["T"]
    fr, to = inst["line_from"], inst["line_to"]
    sh = lambda a, n: np.asarray(a).reshape(T, n)
    wb, thb = sh(S["wb"], N), sh(S["thb"], N)
    return [
        sh(S["pf"], L) - sh(S["Pbf"], L), sh(S["qf"], L) - sh(S["Qbf"], L),
        sh(S["pt"], L) - sh(S["Pbt"], L), sh(S["qt"], L) - sh(S["Qbt"], L),
        sh(S["vf"], L) ** 2 - wb[:, fr], sh(S["vt"], L) ** 2 - wb[:, to],
        sh(S["thf"], L) - thb[:, fr], sh(S["tht"], L) - thb[:, to],
    ]


def rhos(params):
    rb = [params.rho_pq] * 4 + [params.rho_va] * 4
    rg = [params.rho_pq] * 2 + [params.rho_cpl] * 6 + [params.rho_uc] * 3
    return rb, rg


def ybus_injections(inst, vm, va):
    """Complex injections S_i = V_i conj((Y V)_i) of the pi-model network (the
    standard power-flow definition, independent of the W-form rows)."""
    N = inst["n_bus"]
    r, x, b = inst["line_r"], inst["line_x"], inst["line_b"]
    ys = 1.0 / (r + 1j * x)
    Y = np.zeros((N, N), complex)
    for l, (i, j) in enumerate(zip(inst["line_from"], inst["line_to"])):
        Y[i, i] += ys[l] + 0.5j * b[l]
        Y[j, j] += ys[l] + 0.5j * b[l]
        Y[i, j] -= ys[l]
        Y[j, i] -= ys[l]
    Y[np.arange(N), np.arange(N)] += inst["bus_gs"] + 1j * inst["bus_bs"]
    V = vm * np.exp(1j * va)
    return V * np.conj(Y @ V)
