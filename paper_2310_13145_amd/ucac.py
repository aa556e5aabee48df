"""ctypes binding of the HIP library behind include/ucac.h.

Argument marshalling only: every step of the iteration runs in the library's HIP
kernels.  The functions keep the C names (ucac_create, ucac_step, ...); `Solver`
is a small convenience wrapper around one handle.  PyTorch, when present, only
supplies the HIP stream (``Solver.use_torch_stream``).

Importing this module never builds anything; if the shared library is missing
it raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libucac.so")
# iterations per chunk of ucac_solve (SOLVE_CHUNK in csrc/ucac_api.hip): the solve runs
# chunks from a snapshot and replays the one that reaches the tolerance
SOLVE_CHUNK = 64

UCAC_OK, UCAC_NOT_CONVERGED = 0, 1
UCAC_E_INVAL, UCAC_E_NOMEM, UCAC_E_DEVICE, UCAC_E_STATE, UCAC_E_NUMERIC = -1, -2, -3, -4, -5


class UcacError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ucac error {code}: {msg}")
        self.code = code


class ucac_network(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("n_line", C.c_int32), ("n_gen", C.c_int32), ("T", C.c_int32),
        ("ref_bus", C.c_int32), ("base_mva", C.c_double),
        ("line_from", C.c_void_p), ("line_to", C.c_void_p),
        ("line_r", C.c_void_p), ("line_x", C.c_void_p), ("line_b", C.c_void_p), ("line_rate", C.c_void_p),
        ("bus_gs", C.c_void_p), ("bus_bs", C.c_void_p), ("bus_vmin", C.c_void_p), ("bus_vmax", C.c_void_p),
        ("load_p", C.c_void_p), ("load_q", C.c_void_p),
        ("gen_bus", C.c_void_p),
        ("gen_pmin", C.c_void_p), ("gen_pmax", C.c_void_p), ("gen_qmin", C.c_void_p), ("gen_qmax", C.c_void_p),
        ("gen_c2", C.c_void_p), ("gen_c1", C.c_void_p),
        ("gen_cnl", C.c_void_p), ("gen_csu", C.c_void_p), ("gen_csd", C.c_void_p),
        ("gen_ru", C.c_void_p), ("gen_rd", C.c_void_p), ("gen_su", C.c_void_p), ("gen_sd", C.c_void_p),
        ("gen_min_up", C.c_void_p), ("gen_min_dn", C.c_void_p), ("gen_u0", C.c_void_p),
        ("gen_init_on", C.c_void_p), ("gen_init_off", C.c_void_p),
        ("gen_p0", C.c_void_p),
    ]


class ucac_params(C.Structure):
    _fields_ = [
        ("rho_pq", C.c_double), ("rho_va", C.c_double), ("rho_uc", C.c_double), ("rho_cpl", C.c_double),
        ("beta0", C.c_double), ("tau", C.c_double), ("theta", C.c_double), ("lambda_max", C.c_double),
        ("beta_max", C.c_double), ("mu_line", C.c_double),
        ("newton_max_iter", C.c_int32), ("newton_gtol", C.c_double),
        ("max_inner", C.c_int32), ("eps_in0", C.c_double), ("tol", C.c_double),
        ("warm_start", C.c_int32), ("device", C.c_int32),
        ("adapt_every", C.c_int32), ("adapt_mu", C.c_double), ("adapt_tau", C.c_double),
        ("adapt_max", C.c_int32), ("adapt_span", C.c_double),
    ]


class ucac_batch_config(C.Structure):
    _fields_ = [("dp_lanes", C.c_int32), ("branch_block", C.c_int32), ("order", C.c_int32)]


BATCH_CANDIDATES = [(dl, bb, od) for od in (0, 1) for bb in (256, 64) for dl in (64, 16)]

_INT_FIELDS = {"line_from", "line_to", "gen_bus", "gen_min_up", "gen_min_dn", "gen_u0", "gen_init_on", "gen_init_off"}

_lib = None


def lib():
    """Load libucac.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, ip = C.c_void_p, C.POINTER(C.c_int32)
        dp = C.POINTER(C.c_double)
        L.ucac_params_default.argtypes = [C.POINTER(ucac_params)]
        L.ucac_params_default.restype = None
        L.ucac_create.argtypes = [C.POINTER(ucac_network), C.POINTER(ucac_params), C.POINTER(vp)]
        L.ucac_set_stream.argtypes = [vp, vp]
        L.ucac_step.argtypes = [vp, C.c_int32]
        L.ucac_solve.argtypes = [vp, C.c_double, C.c_int32, ip]
        L.ucac_residuals.argtypes = [vp, dp, dp, dp, dp]
        L.ucac_uc_warmstart.argtypes = [vp, C.c_double, C.c_int32, ip]
        L.ucac_get_solution.argtypes = [vp] * 8
        L.ucac_get_state.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
        L.ucac_set_state.argtypes = [vp, vp, C.c_size_t]
        L.ucac_get_branch_iters.argtypes = [vp, vp]
        L.ucac_get_line_starts.argtypes = [vp, vp]
        L.ucac_last_error.argtypes = [vp]
        L.ucac_last_error.restype = C.c_char_p
        L.ucac_destroy.argtypes = [vp]
        L.ucac_destroy.restype = None
        L.ucac_kernel_times.argtypes = [vp, C.c_int32, vp, C.c_int32]
        L.ucac_branch_counters.argtypes = [vp, vp, C.c_int32]
        L.ucac_solve_milestones.argtypes = [vp, vp]
        fp, i64p = C.POINTER(C.c_float), C.POINTER(C.c_int64)
        L.ucac_set_warmstart.argtypes = [vp, vp, C.c_size_t]
        L.ucac_set_params.argtypes = [vp, C.POINTER(ucac_params)]
        L.ucac_set_params.restype = C.c_int
        L.ucac_log_pairs.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, C.c_int64, i64p]
        L.ucac_mlp_create.argtypes = [C.c_int32, C.c_uint64, C.POINTER(vp)]
        L.ucac_mlp_set_weights.argtypes = [vp, vp, C.c_size_t]
        L.ucac_mlp_get_weights.argtypes = [vp, vp, C.c_size_t]
        L.ucac_mlp_forward.argtypes = [vp, vp, C.c_int64, vp]
        L.ucac_mlp_grad.argtypes = [vp, vp, vp, C.c_int64, vp, dp]
        L.ucac_mlp_train.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_uint64, dp]
        L.ucac_mlp_grad_noalloc.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
        L.ucac_mlp_last_error.argtypes = [vp]
        L.ucac_mlp_last_error.restype = C.c_char_p
        L.ucac_mlp_destroy.argtypes = [vp]
        L.ucac_mlp_destroy.restype = None
        L.ucac_dp_batch.argtypes = [C.c_int32, C.c_int32] + [vp] * 8 + [C.c_int32, vp]
        L.ucac_dp_batch.restype = C.c_int
        L.ucac_batch_create.argtypes = [C.POINTER(ucac_network), C.c_int32, C.POINTER(ucac_params), C.POINTER(vp)]
        L.ucac_batch_size.argtypes = [vp]
        L.ucac_batch_size.restype = C.c_int32
        L.ucac_batch_member.argtypes = [vp, C.c_int32, C.POINTER(vp)]
        L.ucac_batch_step.argtypes = [vp, C.c_int32]
        L.ucac_batch_solve.argtypes = [vp, C.c_double, C.c_int32, vp, vp]
        L.ucac_batch_autotune.argtypes = [vp, C.c_int32, C.POINTER(ucac_batch_config), vp, C.c_int32]
        L.ucac_batch_set_config.argtypes = [vp, C.POINTER(ucac_batch_config)]
        L.ucac_batch_get_config.argtypes = [vp, C.POINTER(ucac_batch_config)]
        L.ucac_batch_last_error.argtypes = [vp]
        L.ucac_batch_last_error.restype = C.c_char_p
        L.ucac_batch_destroy.argtypes = [vp]
        L.ucac_batch_destroy.restype = None
        for name in ("ucac_create", "ucac_set_stream", "ucac_step", "ucac_solve", "ucac_residuals", "ucac_uc_warmstart",
                     "ucac_get_solution", "ucac_get_state", "ucac_set_state", "ucac_get_branch_iters",
                     "ucac_get_line_starts",
                     "ucac_kernel_times", "ucac_branch_counters", "ucac_solve_milestones",
                     "ucac_set_warmstart", "ucac_log_pairs", "ucac_mlp_create", "ucac_mlp_set_weights",
                     "ucac_mlp_get_weights", "ucac_mlp_forward", "ucac_mlp_grad", "ucac_mlp_train",
                     "ucac_mlp_grad_noalloc",
                     "ucac_batch_create", "ucac_batch_member", "ucac_batch_step", "ucac_batch_solve",
                     "ucac_batch_autotune", "ucac_batch_set_config", "ucac_batch_get_config"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def ucac_params_default(**over) -> ucac_params:
    p = ucac_params()
    lib().ucac_params_default(C.byref(p))
    for k, v in over.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def make_network(inst):
    """ucac_network view of an instance dict; returns (struct, keep-alive arrays)."""
    net = ucac_network()
    keep = []
    for name, _ in ucac_network._fields_:
        v = inst[name]
        if name in ("n_bus", "n_line", "n_gen", "T", "ref_bus", "base_mva"):
            setattr(net, name, v)
            continue
        a = np.ascontiguousarray(v, dtype=np.int32 if name in _INT_FIELDS else np.float64)
        keep.append(a)
        setattr(net, name, a.ctypes.data if a.size else None)
    return net, keep


NRB, NRG = 8, 11
SCALARS = ("beta", "znorm_prev", "k_outer", "l_inner", "iter", "r_p", "r_in", "r_d", "z_inf", "converged",
           "rho_pq", "rho_va", "rho_cpl", "rho_uc", "nchg_pq", "nchg_va", "nchg_cpl", "nchg_uc")


def state_layout(n_bus, n_line, n_gen, T):
    """(name, count) pairs of the flat FP64 state of ucac_get_state, in order."""
    TL, TG, TN = T * n_line, T * n_gen, T * n_bus
    out = [(k, TL) for k in ("vf", "vt", "thf", "tht", "pf", "qf", "pt", "qt", "nuf", "nut")]
    out += [(k, TG) for k in ("p", "q", "s1", "s2", "s3", "s4", "s5", "s6", "uon", "usu", "usd")]
    out += [(k, TN) for k in ("wb", "thb")]
    out += [(k, TL) for k in ("Pbf", "Qbf", "Pbt", "Qbt")]
    out += [(k, TG) for k in ("pb", "qb", "ubon", "ubsu", "ubsd")]
    for kind in ("zB", "yB", "lB"):
        out += [(f"{kind}{r}", TL) for r in range(NRB)]
    for kind in ("zG", "yG", "lG"):
        out += [(f"{kind}{r}", TG) for r in range(NRG)]
    out.append(("scalars", len(SCALARS)))
    return out


def split_state(flat, n_bus, n_line, n_gen, T):
    """Named views of a flat state."""
    out, off = {}, 0
    for name, n in state_layout(n_bus, n_line, n_gen, T):
        out[name] = flat[off:off + n]
        off += n
    if off != len(flat):
        raise ValueError("state size does not match the instance dimensions")
    sc = out.pop("scalars")
    for i, k in enumerate(SCALARS):
        out[k] = float(sc[i])
    return out


def ucac_last_error(h=None) -> str:
    s = lib().ucac_last_error(h)
    return s.decode() if s else ""


def _check(rc, h=None, ok=(UCAC_OK,)):
    if rc not in ok:
        raise UcacError(rc, ucac_last_error(h))
    return rc


def ucac_create(inst, params: ucac_params):
    net, keep = make_network(inst)
    h = C.c_void_p()
    rc = lib().ucac_create(C.byref(net), C.byref(params), C.byref(h))
    _check(rc, None)
    return h


def ucac_set_stream(h, stream_ptr):
    return _check(lib().ucac_set_stream(h, C.c_void_p(stream_ptr) if stream_ptr else None), h)


def ucac_step(h, n_iters):
    return _check(lib().ucac_step(h, int(n_iters)), h)


def ucac_solve(h, tol, max_iters):
    it = C.c_int32(0)
    rc = _check(lib().ucac_solve(h, float(tol), int(max_iters), C.byref(it)), h, ok=(UCAC_OK, UCAC_NOT_CONVERGED))
    return rc, it.value


def ucac_residuals(h):
    out = [C.c_double() for _ in range(4)]
    _check(lib().ucac_residuals(h, *[C.byref(o) for o in out]), h)
    return tuple(o.value for o in out)


def ucac_get_solution(h, n_bus, n_gen, T):
    p = np.empty((T, n_gen)); q = np.empty((T, n_gen))
    u = [np.empty((T, n_gen), np.int8) for _ in range(3)]
    vm = np.empty((T, n_bus)); va = np.empty((T, n_bus))
    _check(lib().ucac_get_solution(h, _ptr(p), _ptr(q), _ptr(u[0]), _ptr(u[1]), _ptr(u[2]), _ptr(vm), _ptr(va)), h)
    return dict(p=p, q=q, u_on=u[0], u_su=u[1], u_sd=u[2], vm=vm, va=va)


def ucac_get_state(h):
    n = C.c_size_t(0)
    _check(lib().ucac_get_state(h, None, C.byref(n)), h)
    buf = np.empty(n.value // 8, dtype=np.float64)
    _check(lib().ucac_get_state(h, _ptr(buf), C.byref(n)), h)
    return buf


def ucac_set_state(h, buf):
    buf = np.ascontiguousarray(buf, dtype=np.float64)
    return _check(lib().ucac_set_state(h, _ptr(buf), buf.nbytes), h)


def ucac_get_branch_iters(h, n_line, T):
    out = np.empty(T * n_line, dtype=np.int32)
    _check(lib().ucac_get_branch_iters(h, _ptr(out)), h)
    return out


def ucac_get_line_starts(h, n_line, T):
    """The learned start's predicted points of the last learned-start iteration:
    [4][T * n_line] (v_i, v_j, theta_i, theta_j), FP32."""
    out = np.empty((4, T * n_line), dtype=np.float32)
    _check(lib().ucac_get_line_starts(h, _ptr(out)), h)
    return out


KERNELS = ("units", "branch", "bus", "post", "finalize")


def ucac_kernel_times(h, n_iters):
    """n_iters iterations launched kernel by kernel with HIP events; mean ms per kernel
    between event records, and "<kernel>_dispatch": its mean from its dispatch's own
    begin and end timestamps."""
    K = len(KERNELS)
    out = np.zeros(2 * K)
    _check(lib().ucac_kernel_times(h, int(n_iters), _ptr(out), len(out)), h)
    d = dict(zip(KERNELS, out[:K].tolist()))
    d.update({f"{k}_dispatch": float(out[K + i]) for i, k in enumerate(KERNELS)})
    return d


def ucac_branch_counters(h, reset=False):
    out = np.zeros(7, dtype=np.uint64)
    _check(lib().ucac_branch_counters(h, _ptr(out), int(bool(reset))), h)
    return dict(evals=int(out[0]), rejected=int(out[1]), cg=int(out[2]), newton=int(out[3]), fallbacks=int(out[4]),
                direct=int(out[5]), searches=int(out[6]))


MLP_PARAMS = 5764
MLP_IN, MLP_OUT = 20, 4
MLP_NOALLOC_MAX = 16384


def ucac_set_warmstart(h, weights):
    """Use the learned Newton start with these FP32 weights (None: back to the configured start)."""
    if weights is None:
        _check(lib().ucac_set_warmstart(h, None, 0), h)
        return
    w = np.ascontiguousarray(weights, dtype=np.float32)
    _check(lib().ucac_set_warmstart(h, _ptr(w), w.size), h)


def ucac_log_pairs(h, n_iters, stride, cap):
    """Run n_iters inner iterations and return the logged (features [m, 20], targets [m, 4])."""
    f = np.zeros((max(cap, 0), MLP_IN), dtype=np.float32)
    t = np.zeros((max(cap, 0), MLP_OUT), dtype=np.float32)
    n = C.c_int64(0)
    _check(lib().ucac_log_pairs(h, int(n_iters), int(stride), _ptr(f), _ptr(t), int(cap), C.byref(n)), h)
    return f[:n.value], t[:n.value]


def _mcheck(rc, m):
    if rc != UCAC_OK:
        s = lib().ucac_mlp_last_error(m)
        raise UcacError(rc, s.decode() if s else "")
    return rc


class WarmStartNet:
    """The learned line warm-start network on one GPU (FP32 master weights, BF16 copies)."""

    def __init__(self, seed=0, device=0):
        m = C.c_void_p()
        _mcheck(lib().ucac_mlp_create(int(device), int(seed) & (2**64 - 1), C.byref(m)), None)
        self.m = m

    def close(self):
        if getattr(self, "m", None):
            lib().ucac_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self):
        w = np.zeros(MLP_PARAMS, dtype=np.float32)
        _mcheck(lib().ucac_mlp_get_weights(self.m, _ptr(w), w.size), self.m)
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _mcheck(lib().ucac_mlp_set_weights(self.m, _ptr(w), w.size), self.m)

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, MLP_IN)
        y = np.zeros((x.shape[0], MLP_OUT), dtype=np.float32)
        _mcheck(lib().ucac_mlp_forward(self.m, _ptr(x), x.shape[0], _ptr(y)), self.m)
        return y

    def grad(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, MLP_IN)
        t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1, MLP_OUT)
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        ls = C.c_double(0.0)
        _mcheck(lib().ucac_mlp_grad(self.m, _ptr(x), _ptr(t), x.shape[0], _ptr(g), C.byref(ls)), self.m)
        return g, ls.value

    def grad_noalloc(self, x, t, grad, loss, stream=None):
        """ucac_mlp_grad_noalloc on device tensors the caller owns: x [n, 20] and t [n, 4]
        float32, grad [MLP_PARAMS] float32 and loss [1] float64 (written: the sum of
        squared errors).  Enqueued on `stream` (a torch stream; default: the current one)."""
        import torch
        n = int(x.shape[0])
        for a, shape, dt in ((x, (n, MLP_IN), torch.float32), (t, (n, MLP_OUT), torch.float32),
                             (grad, (MLP_PARAMS,), torch.float32), (loss, (1,), torch.float64)):
            if tuple(a.shape) != shape or a.dtype != dt or not a.is_cuda or not a.is_contiguous():
                raise ValueError(f"expected a contiguous {dt} cuda tensor of shape {shape}, got {a.dtype} "
                                 f"{tuple(a.shape)} on {a.device}")
        st = (stream or torch.cuda.current_stream(x.device)).cuda_stream
        _mcheck(lib().ucac_mlp_grad_noalloc(self.m, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()), n,
                                            C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()),
                                            C.c_void_p(st)), self.m)

    def train(self, x, t, epochs=10, batch=256, lr=1e-3, seed=0):
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, MLP_IN)
        t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1, MLP_OUT)
        ls = C.c_double(0.0)
        _mcheck(lib().ucac_mlp_train(self.m, _ptr(x), _ptr(t), x.shape[0], int(epochs), int(batch), float(lr),
                                     int(seed) & (2**64 - 1), C.byref(ls)), self.m)
        return ls.value


def ucac_solve_milestones(h):
    """First iteration of the last solve/step call with r_p, r_d <= 1e-2, 1e-3, 1e-4 (-1: never)."""
    out = np.zeros(3, dtype=np.int32)
    _check(lib().ucac_solve_milestones(h, _ptr(out)), h)
    return {"1e-2": int(out[0]), "1e-3": int(out[1]), "1e-4": int(out[2])}


def ucac_destroy(h):
    if h:
        lib().ucac_destroy(h)


class Solver:
    """One UC-ACOPF instance resident on the GPU."""

    def __init__(self, inst, params: ucac_params | None = None, **over):
        self.inst = inst
        self.params = params if params is not None else ucac_params_default(**over)
        self.dims = (inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"])
        self.h = ucac_create(inst, self.params)

    def close(self):
        if getattr(self, "h", None):
            ucac_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def use_torch_stream(self):
        import torch
        ucac_set_stream(self.h, torch.cuda.current_stream().cuda_stream)

    def step(self, n=1):
        ucac_step(self.h, n)

    def solve(self, tol=1e-4, max_iters=20000):
        return ucac_solve(self.h, tol, max_iters)

    def uc_warmstart(self, tol=1e-3, max_iters=2000):
        """UC warm start: the multiperiod ACOPF solved first, commitments from its
        generation levels, then the cold start with them; (status, iterations)."""
        it = C.c_int32(0)
        rc = lib().ucac_uc_warmstart(self.h, float(tol), int(max_iters), C.byref(it))
        _check(rc, self.h, ok=(UCAC_OK, UCAC_NOT_CONVERGED))
        return rc, it.value

    def residuals(self):
        return ucac_residuals(self.h)

    def solution(self):
        N, L, G, T = self.dims
        return ucac_get_solution(self.h, N, G, T)

    def get_state(self):
        return ucac_get_state(self.h)

    def set_state(self, buf):
        ucac_set_state(self.h, buf)

    def milestones(self):
        return ucac_solve_milestones(self.h)

    def kernel_times(self, n_iters):
        return ucac_kernel_times(self.h, n_iters)

    def branch_counters(self, reset=False):
        return ucac_branch_counters(self.h, reset)

    def branch_iters(self):
        N, L, G, T = self.dims
        return ucac_get_branch_iters(self.h, L, T)

    def set_warmstart(self, weights):
        ucac_set_warmstart(self.h, weights)

    def line_starts(self):
        N, L, G, T = self.dims
        return ucac_get_line_starts(self.h, L, T)

    def set_params(self, **over):
        """Change parameters from the next iteration on (iterate and multipliers kept)."""
        p = ucac_params()
        C.memmove(C.byref(p), C.byref(self.params), C.sizeof(ucac_params))
        for k, v in over.items():
            if not hasattr(p, k):
                raise KeyError(k)
            setattr(p, k, v)
        _check(lib().ucac_set_params(self.h, C.byref(p)), self.h)
        self.params = p

    def log_pairs(self, n_iters, stride=1, cap=None):
        N, L, G, T = self.dims
        if cap is None:
            cap = n_iters * ((L * T + stride - 1) // stride)
        return ucac_log_pairs(self.h, n_iters, stride, cap)


def _bcheck(rc, b, ok=(UCAC_OK,)):
    if rc not in ok:
        msg = lib().ucac_batch_last_error(b)
        raise UcacError(rc, msg.decode() if msg else "")
    return rc


class Member(Solver):
    """View of one member of a Batch (the batch owns the handle)."""

    def __init__(self, batch, k):
        inst = batch.insts[k]
        self.inst = inst
        self.params = batch.params
        self.dims = (inst["n_bus"], inst["n_line"], inst["n_gen"], inst["T"])
        h = C.c_void_p()
        _bcheck(lib().ucac_batch_member(batch.b, int(k), C.byref(h)), batch.b)
        self.h = h
        self._batch = batch  # keeps the owner alive

    def close(self):
        self.h = None  # owned by the batch


class Batch:
    """Many independent instances advanced by one grouped launch per kernel."""

    def __init__(self, insts, params: ucac_params | None = None, **over):
        self.insts = list(insts)
        self.params = params if params is not None else ucac_params_default(**over)
        nets, self._keep = [], []
        for inst in self.insts:
            net, keep = make_network(inst)
            nets.append(net)
            self._keep.append(keep)
        arr = (ucac_network * len(nets))(*nets)
        b = C.c_void_p()
        _bcheck(lib().ucac_batch_create(arr, len(nets), C.byref(self.params), C.byref(b)), None)
        self.b = b

    def __len__(self):
        return len(self.insts)

    def close(self):
        if getattr(self, "b", None):
            lib().ucac_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def member(self, k):
        return Member(self, k)

    def step(self, n=1):
        _bcheck(lib().ucac_batch_step(self.b, int(n)), self.b)

    def solve(self, tol=1e-4, max_iters=20000):
        n = len(self.insts)
        iters = np.zeros(n, dtype=np.int32)
        conv = np.zeros(n, dtype=np.int32)
        rc = _bcheck(lib().ucac_batch_solve(self.b, float(tol), int(max_iters), _ptr(iters), _ptr(conv)), self.b,
                     ok=(UCAC_OK, UCAC_NOT_CONVERGED))
        return rc, iters, conv.astype(bool)

    def autotune(self, iters=10):
        c = ucac_batch_config()
        ms = np.zeros(len(BATCH_CANDIDATES))
        _bcheck(lib().ucac_batch_autotune(self.b, int(iters), C.byref(c), _ptr(ms), len(ms)), self.b)
        return (c.dp_lanes, c.branch_block, c.order), dict(zip(BATCH_CANDIDATES, ms.tolist()))

    def set_config(self, dp_lanes=64, branch_block=256, order=0):
        c = ucac_batch_config(dp_lanes, branch_block, order)
        _bcheck(lib().ucac_batch_set_config(self.b, C.byref(c)), self.b)

    def config(self):
        c = ucac_batch_config()
        _bcheck(lib().ucac_batch_get_config(self.b, C.byref(c)), self.b)
        return (c.dp_lanes, c.branch_block, c.order)


def ucac_dp_batch(tab, min_up, min_dn, u0, hold_on, hold_off, lanes_per_unit=64, stream=None):
    """G unit-commitment DPs on device tensors: tab [G, T, 2, 2] float64 (cuda),
    the five int32 [G] tensors; returns (u_on [G, T] int8, cost [G] float64) on the
    same device.  Enqueued on `stream` (a torch stream; default: the current one)."""
    import torch
    G, T = int(tab.shape[0]), int(tab.shape[1])
    dev = tab.device
    ints = [x.to(device=dev, dtype=torch.int32).contiguous() for x in (min_up, min_dn, u0, hold_on, hold_off)]
    tab = tab.to(dtype=torch.float64).contiguous()
    u = torch.empty((G, T), dtype=torch.int8, device=dev)
    cost = torch.empty(G, dtype=torch.float64, device=dev)
    st = (stream or torch.cuda.current_stream(dev)).cuda_stream
    rc = lib().ucac_dp_batch(G, T, C.c_void_p(tab.data_ptr()), *[C.c_void_p(x.data_ptr()) for x in ints],
                             C.c_void_p(u.data_ptr()), C.c_void_p(cost.data_ptr()), int(lanes_per_unit), C.c_void_p(st))
    _check(rc, None)
    return u, cost
