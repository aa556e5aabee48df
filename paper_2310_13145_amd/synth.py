"""Seeded synthetic UC-ACOPF instances.

This module only draws network, generator and load data; it holds none of the
method's arithmetic (no admittances, no costs in per-unit, no subproblem maths).
Both the FP64 oracle and the HIP library consume the dictionaries it returns.

The paper's experiments use MATPOWER IEEE cases with an ISO-NE demand profile
(Section IV-B).  That data is not available here, so every workload is a seeded
stand-in with the parameter distributions below:

* topology: a ring plus chords (9-bus case) or a planar Delaunay mesh made
  connected by its Euclidean minimum spanning tree and then filled with Delaunay
  edges drawn uniformly at random up to the requested line count;
* lines: r ~ U(0.005, 0.03), x ~ U(0.05, 0.2), b ~ U(0, 0.2), rating ~ U(1.5, 3) p.u.;
* generators at distinct random buses: c2 ~ U(0.01, 0.1) $/MW^2h, c1 ~ U(10, 40) $/MWh,
  start-up cost ~ U(100, 500) $, Pmax ~ U(1, 3) p.u., Pmin = 0.2 Pmax,
  ramp and start-up/shut-down ramps 0.5 Pmax per period, min up/down ~ U{2, 3},
  reactive capability Qmax = 0.6 Pmax, Qmin = -0.6 Pmax (a unit absorbs as much as
  it produces: the lines' charging b ~ U(0, 0.2) supplies about 0.1 p.u. per line,
  far more than the light load's reactive demand, and with Qmin = -0.3 Pmax the
  units cannot absorb the surplus within the voltage bounds in the light periods
  of the 2000-bus mesh), initially on at p0 = 0.5 Pmax;
* loads on round(2N/3) random buses, base ~ U(0.5, 1.5) rescaled so the base
  total is 30 % of the installed capacity (a light load, the same motive as the
  paper's demand discount; at 40 % and above the random placement of units and
  loads leaves some periods of the 118-bus mesh without a feasible AC operating
  point), a daily sinusoid of +-20 % with a random phase, and Q = 0.3 P.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2310131450

# name -> (buses, lines, generators, periods)
CONFIGS = {
    0: dict(name="ring9_T6", n_bus=9, n_line=12, n_gen=3, T=6),
    1: dict(name="mesh118_T24", n_bus=118, n_line=186, n_gen=54, T=24),
    2: dict(name="mesh2000_T24", n_bus=2000, n_line=3200, n_gen=500, T=24),
    4: dict(name="mesh10000_T48", n_bus=10000, n_line=13000, n_gen=2500, T=48),
}


def _ring_with_chords(rng, n, n_line):
    edges = [(i, (i + 1) % n) for i in range(n)]
    have = {tuple(sorted(e)) for e in edges}
    while len(edges) < n_line:
        i, j = rng.choice(n, size=2, replace=False)
        key = (min(i, j), max(i, j))
        if key in have or (j - i) % n in (1, n - 1):
            continue
        have.add(key)
        edges.append((int(i), int(j)))
    return np.array(edges, dtype=np.int64)


def _delaunay_mesh(rng, n, n_line):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial import Delaunay

    pts = rng.random((n, 2))
    tri = Delaunay(pts)
    cand = set()
    for s in tri.simplices:
        for a in range(3):
            i, j = int(s[a]), int(s[(a + 1) % 3])
            cand.add((min(i, j), max(i, j)))
    cand = sorted(cand)
    length = np.array([np.hypot(*(pts[i] - pts[j])) for i, j in cand])
    if n_line > len(cand):
        raise ValueError(f"{n_line} lines requested but the mesh has {len(cand)} edges")
    ii = np.array([e[0] for e in cand])
    jj = np.array([e[1] for e in cand])
    w = coo_matrix((length, (ii, jj)), shape=(n, n)).tocsr()
    mst = minimum_spanning_tree(w).tocoo()
    chosen = {(min(a, b), max(a, b)) for a, b in zip(mst.row.tolist(), mst.col.tolist())}
    if len(chosen) != n - 1:
        raise RuntimeError("Delaunay graph is not connected")
    # the remaining lines are Delaunay edges drawn uniformly at random: adding the
    # shortest ones instead only thickens dense clusters and leaves long tree-like
    # corridors (a 2000-bus mesh then has diameter ~180 and a DC dispatch overloads
    # ~190 lines by up to 5x); random edges give diameter ~50 and a loadable grid
    for k in rng.permutation(len(cand)):
        if len(chosen) >= n_line:
            break
        chosen.add(cand[k])
    edges = sorted(chosen)
    # random orientation so that "from" is not always the lower index
    out = []
    for i, j in edges:
        out.append((i, j) if rng.random() < 0.5 else (j, i))
    return np.array(out, dtype=np.int64)


def make_instance(n_bus, n_line, n_gen, T, seed, ring=False, load_frac=0.3):
    """Return a dict of numpy arrays laid out as the library's network struct."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = _ring_with_chords(rng, n_bus, n_line) if ring else _delaunay_mesh(rng, n_bus, n_line)
    L = len(edges)
    line_r = rng.uniform(0.005, 0.03, L)
    line_x = rng.uniform(0.05, 0.2, L)
    line_b = rng.uniform(0.0, 0.2, L)
    line_rate = rng.uniform(1.5, 3.0, L)

    gen_bus = rng.choice(n_bus, size=n_gen, replace=False)
    pmax = rng.uniform(1.0, 3.0, n_gen)
    c2 = rng.uniform(0.01, 0.1, n_gen)
    c1 = rng.uniform(10.0, 40.0, n_gen)
    csu = rng.uniform(100.0, 500.0, n_gen)
    tu = rng.integers(2, 4, n_gen)
    td = rng.integers(2, 4, n_gen)

    n_load = int(round(2 * n_bus / 3))
    load_bus = rng.choice(n_bus, size=n_load, replace=False)
    base = rng.uniform(0.5, 1.5, n_load)
    base *= load_frac * pmax.sum() / base.sum()
    phase = rng.uniform(0.0, 24.0)
    load_p = np.zeros((T, n_bus))
    for t in range(T):
        load_p[t, load_bus] = base * (1.0 + 0.2 * math.sin(2.0 * math.pi * (t + phase) / 24.0))
    load_q = 0.3 * load_p

    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    return dict(
        n_bus=n_bus, n_line=L, n_gen=n_gen, T=T, ref_bus=0, base_mva=100.0,
        line_from=i32(edges[:, 0]), line_to=i32(edges[:, 1]),
        line_r=f64(line_r), line_x=f64(line_x), line_b=f64(line_b), line_rate=f64(line_rate),
        bus_gs=f64(np.zeros(n_bus)), bus_bs=f64(np.zeros(n_bus)),
        bus_vmin=f64(np.full(n_bus, 0.9)), bus_vmax=f64(np.full(n_bus, 1.1)),
        load_p=f64(load_p), load_q=f64(load_q),
        gen_bus=i32(gen_bus),
        gen_pmin=f64(0.2 * pmax), gen_pmax=f64(pmax),
        gen_qmin=f64(-0.6 * pmax), gen_qmax=f64(0.6 * pmax),
        gen_c2=f64(c2), gen_c1=f64(c1), gen_cnl=f64(np.zeros(n_gen)),
        gen_csu=f64(csu), gen_csd=f64(np.zeros(n_gen)),
        gen_ru=f64(0.5 * pmax), gen_rd=f64(0.5 * pmax),
        gen_su=f64(0.5 * pmax), gen_sd=f64(0.5 * pmax),
        gen_min_up=i32(tu), gen_min_dn=i32(td),
        gen_u0=i32(np.ones(n_gen)), gen_init_on=i32(np.zeros(n_gen)),
        gen_init_off=i32(np.zeros(n_gen)),
        gen_p0=f64(0.5 * pmax),
    )


def config_instance(cfg_id: int, instance: int = 0):
    """Instance of a named workload (0: 9-bus T=6, 1: 118-bus T=24, 2: 2000-bus T=24,
    4: 10000-bus T=48; 3: one member of the 64-instance batch)."""
    if cfg_id == 3:
        return batch_member(instance)
    c = CONFIGS[cfg_id]
    return make_instance(c["n_bus"], c["n_line"], c["n_gen"], c["T"], SEED_BASE + cfg_id,
                         ring=(cfg_id == 0))


def training_instance(cfg_id: int, k: int):
    """Instance k of the same shape and distributions as workload cfg_id, drawn from a
    seed that no evaluation workload uses (training data for the learned start)."""
    c = CONFIGS[cfg_id]
    return make_instance(c["n_bus"], c["n_line"], c["n_gen"], c["T"], SEED_BASE + 100_000 + 1000 * cfg_id + k,
                         ring=(cfg_id == 0))


def batch_member(k: int):
    """Member k of the uneven 64-instance batch: N ~ logU[30, 2000], L = round(1.5 N),
    G = round(0.25 N), T uniform in {12, 24, 48}."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 3 + 1000 * (k + 1)))
    n = int(round(math.exp(rng.uniform(math.log(30.0), math.log(2000.0)))))
    T = int(rng.choice([12, 24, 48]))
    return make_instance(n, int(round(1.5 * n)), max(1, int(round(0.25 * n))), T,
                         SEED_BASE + 3 + k)


def batch_instances(n: int = 64):
    return [batch_member(k) for k in range(n)]


def small_instance(n_bus, n_line, n_gen, T, seed):
    """Tiny seeded instance for tests (ring topology below 12 buses, mesh above)."""
    return make_instance(n_bus, n_line, n_gen, T, seed, ring=(n_bus < 12))
