"""FP64 CPU oracle for the UC-ACOPF two-level ADMM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library behind
``include/ucac.h``) never calls it and shares no code with it.

The C source (``ucac_oracle.c``) is plain FP64 code that follows the paper's
formulation and iteration order (an OpenMP parallel for over the independent
items of each block, with results that do not depend on the thread count); this
module only marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ucac_oracle.c")
# UCAC_ORACLE_LIB points the tests at another build of the same source (used to
# check on the CPU that the pins catch mistakes planted in a copy of the oracle).
_LIB = os.environ.get("UCAC_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))

NRB = 8   # line rows: Pf Qf Pt Qt Wf Wt Thf Tht
NRG = 11  # generator rows: G1 G2 C1..C6 U1 U2 U3
SCALARS = ["beta", "znorm_prev", "k_outer", "l_inner", "iter", "r_p", "r_in", "r_d", "z_inf", "converged",
           "rho_pq", "rho_va", "rho_cpl", "rho_uc", "nchg_pq", "nchg_va", "nchg_cpl", "nchg_uc"]


def build(verbose=False):
    """Compile the oracle with plain IEEE FP64 semantics (no contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-Wall", "-o", _LIB, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return _LIB


class _Net(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("n_line", C.c_int32), ("n_gen", C.c_int32), ("T", C.c_int32),
        ("ref_bus", C.c_int32), ("base_mva", C.c_double),
        ("line_from", C.c_void_p), ("line_to", C.c_void_p),
        ("line_r", C.c_void_p), ("line_x", C.c_void_p), ("line_b", C.c_void_p), ("line_rate", C.c_void_p),
        ("bus_gs", C.c_void_p), ("bus_bs", C.c_void_p), ("bus_vmin", C.c_void_p), ("bus_vmax", C.c_void_p),
        ("load_p", C.c_void_p), ("load_q", C.c_void_p),
        ("gen_bus", C.c_void_p),
        ("gen_pmin", C.c_void_p), ("gen_pmax", C.c_void_p), ("gen_qmin", C.c_void_p), ("gen_qmax", C.c_void_p),
        ("gen_c2", C.c_void_p), ("gen_c1", C.c_void_p), ("gen_cnl", C.c_void_p), ("gen_csu", C.c_void_p),
        ("gen_csd", C.c_void_p),
        ("gen_ru", C.c_void_p), ("gen_rd", C.c_void_p), ("gen_su", C.c_void_p), ("gen_sd", C.c_void_p),
        ("gen_min_up", C.c_void_p), ("gen_min_dn", C.c_void_p), ("gen_u0", C.c_void_p),
        ("gen_init_on", C.c_void_p), ("gen_init_off", C.c_void_p),
        ("gen_p0", C.c_void_p),
    ]


class Params(C.Structure):
    _fields_ = [
        ("rho_pq", C.c_double), ("rho_va", C.c_double), ("rho_uc", C.c_double), ("rho_cpl", C.c_double),
        ("beta0", C.c_double), ("tau", C.c_double), ("theta", C.c_double), ("lambda_max", C.c_double),
        ("beta_max", C.c_double), ("mu_line", C.c_double),
        ("newton_max_iter", C.c_int32), ("newton_gtol", C.c_double),
        ("max_inner", C.c_int32), ("eps_in0", C.c_double), ("tol", C.c_double),
        ("warm_start", C.c_int32),
        ("adapt_every", C.c_int32), ("adapt_mu", C.c_double), ("adapt_tau", C.c_double),
        ("adapt_max", C.c_int32), ("adapt_span", C.c_double),
        ("relax_uc", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if "UCAC_ORACLE_LIB" not in os.environ and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LIB)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(_Net), C.POINTER(Params)]
        L.orc_destroy.argtypes = [vp]
        L.orc_params_default.argtypes = [C.POINTER(Params)]
        L.orc_step.argtypes = [vp, C.c_int]
        L.orc_solve.argtypes = [vp, C.c_double, C.c_int, ip]
        L.orc_solve.restype = C.c_int
        L.orc_uc_warmstart.argtypes = [vp, C.c_double, C.c_int, ip]
        L.orc_uc_warmstart.restype = C.c_int
        L.orc_state_size.argtypes = [vp]
        L.orc_state_size.restype = C.c_size_t
        L.orc_get_state.argtypes = [vp, vp]
        L.orc_set_state.argtypes = [vp, vp]
        L.orc_reset.argtypes = [vp]
        L.orc_set_params.argtypes = [vp, C.POINTER(Params)]
        L.orc_get_branch_iters.argtypes = [vp, vp]
        L.orc_objective.argtypes = [vp]
        L.orc_objective.restype = C.c_double
        L.orc_dp.argtypes = [C.c_int, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp]
        L.orc_dp.restype = C.c_double
        L.orc_uc_cost.argtypes = [C.c_double] * 4 + [C.c_int, C.c_int, vp, vp, vp]
        L.orc_uc_cost.restype = C.c_double
        L.orc_gen_solve.argtypes = [vp] * 6
        L.orc_ubar_solve.argtypes = [vp, vp]
        L.orc_branch_eval.argtypes = [vp, vp, vp, vp]
        L.orc_branch_eval.restype = C.c_double
        L.orc_branch_F.argtypes = [vp, vp]
        L.orc_branch_F.restype = C.c_double
        L.orc_branch_solve.argtypes = [vp, vp, C.c_int, C.c_double, C.c_int, ip]
        L.orc_branch_solve.restype = C.c_int
        L.orc_branch_trial.argtypes = [vp, vp, C.c_double, C.c_int, vp]
        L.orc_branch_trial.restype = C.c_double
        L.orc_line_admittance.argtypes = [C.c_double, C.c_double, C.c_double, vp]
        L.orc_line_flows.argtypes = [vp, vp, vp]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def set_threads(n):
    """Threads of the oracle's parallel loops (0: the OpenMP default)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


def default_params(**over):
    p = Params()
    lib().orc_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def state_layout(n_bus, n_line, n_gen, T):
    """(name, count) pairs of the flat FP64 state, in order."""
    TL, TG, TN = T * n_line, T * n_gen, T * n_bus
    lay = [(n, TL) for n in ("vf", "vt", "thf", "tht", "pf", "qf", "pt", "qt", "nuf", "nut")]
    lay += [(n, TG) for n in ("p", "q", "s1", "s2", "s3", "s4", "s5", "s6", "uon", "usu", "usd")]
    lay += [(n, TN) for n in ("wb", "thb")]
    lay += [(n, TL) for n in ("Pbf", "Qbf", "Pbt", "Qbt")]
    lay += [(n, TG) for n in ("pb", "qb", "ubon", "ubsu", "ubsd")]
    for kind in ("zB", "yB", "lB"):
        lay += [(f"{kind}{r}", TL) for r in range(NRB)]
    for kind in ("zG", "yG", "lG"):
        lay += [(f"{kind}{r}", TG) for r in range(NRG)]
    lay += [("scalars", len(SCALARS))]
    return lay


def unpack_state(flat, n_bus, n_line, n_gen, T):
    out, off = {}, 0
    for name, n in state_layout(n_bus, n_line, n_gen, T):
        out[name] = flat[off:off + n]
        off += n
    assert off == len(flat)
    sc = out.pop("scalars")
    for i, s in enumerate(SCALARS):
        out[s] = float(sc[i])
    return out


class Oracle:
    """One UC-ACOPF instance held by the FP64 oracle."""

    def __init__(self, inst, params=None, **over):
        self.inst = inst
        self._keep = {}
        net = _Net()
        for name, _ in _Net._fields_:
            v = inst[name]
            if isinstance(v, np.ndarray):
                want = np.int32 if v.dtype.kind in "iu" else np.float64
                a = np.ascontiguousarray(v, dtype=want)
                self._keep[name] = a
                setattr(net, name, a.ctypes.data)
            else:
                setattr(net, name, v)
        self.params = params if params is not None else default_params(**over)
        self.h = lib().orc_create(C.byref(net), C.byref(self.params))
        self.dims = (inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"])

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_params(self, **over):
        for k, v in over.items():
            setattr(self.params, k, v)
        lib().orc_set_params(self.h, C.byref(self.params))

    def step(self, n=1):
        lib().orc_step(self.h, int(n))

    def solve(self, tol=1e-4, max_iters=10000):
        it = C.c_int32(0)
        rc = lib().orc_solve(self.h, tol, int(max_iters), C.byref(it))
        return rc, it.value

    def uc_warmstart(self, tol=1e-3, max_iters=2000):
        """UC warm start: relaxed multiperiod ACOPF, commitments rounded from its
        generation levels, then the cold start with those commitments."""
        it = C.c_int32(0)
        rc = lib().orc_uc_warmstart(self.h, float(tol), int(max_iters), C.byref(it))
        return rc, it.value

    def state_size(self):
        return int(lib().orc_state_size(self.h))

    def get_state(self):
        buf = np.empty(self.state_size(), dtype=np.float64)
        lib().orc_get_state(self.h, _ptr(buf))
        return buf

    def set_state(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float64)
        assert flat.size == self.state_size()
        lib().orc_set_state(self.h, _ptr(flat))

    def state(self):
        return unpack_state(self.get_state(), *self.dims)

    def reset(self):
        lib().orc_reset(self.h)

    def objective(self):
        return float(lib().orc_objective(self.h))

    def branch_iters(self):
        n, L, G, T = self.dims
        out = np.empty(T * L, dtype=np.int32)
        lib().orc_get_branch_iters(self.h, _ptr(out))
        return out


# ---- single-item entry points --------------------------------------------------

def dp(Ltab, u0, Lg, Fg, TU, TD):
    """Ltab: array [T, 2, 2] indexed [t, s_prev, s]."""
    Ltab = np.ascontiguousarray(Ltab, dtype=np.float64)
    T = Ltab.shape[0]
    u = np.zeros(T, dtype=np.int8)
    cost = lib().orc_dp(T, _ptr(Ltab), int(u0), int(Lg), int(Fg), int(TU), int(TD), _ptr(u))
    return cost, u


def uc_cost(cnl, csu, csd, rho, sp, s, ub, z, y):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (ub, z, y)]
    return lib().orc_uc_cost(cnl, csu, csd, rho, int(sp), int(s), *[_ptr(v) for v in a])


def gen_solve(data, rho, xin, z, y):
    arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (data, rho, xin, z, y)]
    out = np.zeros(8)
    lib().orc_gen_solve(*[_ptr(v) for v in arrs], _ptr(out))
    return out


def ubar_solve(v):
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_ubar_solve(_ptr(v), _ptr(out))
    return out


def branch_eval(v, x):
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.zeros(4)
    H = np.zeros(16)
    F = lib().orc_branch_eval(_ptr(v), _ptr(x), _ptr(g), _ptr(H))
    return F, g, H.reshape(4, 4)


def branch_F(v, x):
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().orc_branch_F(_ptr(v), _ptr(x))


def branch_solve(v, x0, max_iter=50, gtol=1e-8, hold=False):
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.array(x0, dtype=np.float64)
    cg = C.c_int32(0)
    it = lib().orc_branch_solve(_ptr(v), _ptr(x), int(max_iter), float(gtol), int(bool(hold)), C.byref(cg))
    return x, it, cg.value


def branch_trial(v, x, delta, hold=False):
    """Trial point of one projected trust-region Newton iteration from x (gradient,
    Hessian and free set taken at x) and the model value q(xt - x); hold: the hold
    step of warm starts (a free variable on a bound that the step pushes outwards is
    held there and the step solved again)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    xt = np.zeros(4)
    q = lib().orc_branch_trial(_ptr(v), _ptr(x), float(delta), int(bool(hold)), _ptr(xt))
    return xt, q


def line_admittance(r, x, b):
    out = np.zeros(8)
    lib().orc_line_admittance(r, x, b, _ptr(out))
    return out


def line_flows(adm, x):
    adm = np.ascontiguousarray(adm, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.zeros(4)
    lib().orc_line_flows(_ptr(adm), _ptr(x), _ptr(f))
    return f
