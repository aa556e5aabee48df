"""The C-ABI library: it builds, loads and exports every symbol include/ucac.h
declares; input validation rejects bad networks before any device work; the
state format agrees with the oracle's.  No GPU compute here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2310_13145_amd import synth, ucac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ucac.LIB_PATH):
        from paper_2310_13145_amd import build
        build.build()
    return ucac.lib()


def header_functions():
    text = open(os.path.join(ROOT, "include", "ucac.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ucac_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_params_default(lib):
    p = ucac.ucac_params_default()
    assert (p.rho_pq, p.rho_va, p.rho_uc, p.rho_cpl) == (5e3, 1e4, 1e5, 5e3)
    assert (p.tau, p.theta, p.beta0) == (6.0, 0.8, 1e5)
    assert p.newton_max_iter == 50 and p.warm_start == 0


def _bad(mut):
    inst = synth.small_instance(9, 12, 3, 4, seed=5)
    mut(inst)
    net, keep = ucac.make_network(inst)
    h = C.c_void_p()
    rc = ucac.lib().ucac_create(C.byref(net), C.byref(ucac.ucac_params_default()), C.byref(h))
    return rc, ucac.ucac_last_error(None)


@pytest.mark.parametrize("mut,needle", [
    (lambda d: d["line_from"].__setitem__(0, 99), "bad end buses"),
    (lambda d: d["line_to"].__setitem__(1, d["line_from"][1]), "bad end buses"),
    (lambda d: d["line_x"].__setitem__(2, np.nan), "non-finite"),
    (lambda d: (d["line_r"].__setitem__(0, 0.0), d["line_x"].__setitem__(0, 0.0)), "zero impedance"),
    (lambda d: d["gen_pmin"].__setitem__(0, 10.0), "pmin > pmax"),
    (lambda d: d["gen_min_up"].__setitem__(1, 0), "min up/down"),
    (lambda d: d["gen_u0"].__setitem__(2, 3), "u0"),
    (lambda d: d["bus_vmin"].__setitem__(3, 1.2), "voltage bounds"),
    (lambda d: d["load_p"].__setitem__((0, 0), np.inf), "non-finite load"),
    (lambda d: d.__setitem__("ref_bus", 9), "ref_bus"),
    (lambda d: d.__setitem__("T", 0), "bad sizes"),
])
def test_validation_rejects(lib, mut, needle):
    rc, msg = _bad(mut)
    assert rc == ucac.UCAC_E_INVAL
    assert needle in msg


def test_isolated_bus_rejected(lib):
    def mut(d):
        # reroute every line of bus 4 away from it; bus 4 keeps no line and no unit
        for l in range(d["n_line"]):
            for end in ("line_from", "line_to"):
                if d[end][l] == 4:
                    other = d["line_to"][l] if end == "line_from" else d["line_from"][l]
                    d[end][l] = 5 if other != 5 else 6
        d["gen_bus"][d["gen_bus"] == 4] = 7
    rc, msg = _bad(mut)
    assert rc == ucac.UCAC_E_INVAL and ("neither a line nor a generator" in msg or "bad end buses" in msg)


def test_state_format_matches_oracle():
    import oracle
    for dims in [(9, 12, 3, 6), (118, 186, 54, 24), (1, 0, 3, 4)]:
        assert ucac.state_layout(*dims) == [(n, c) for n, c in oracle.state_layout(*dims)]
    inst = synth.config_instance(0)
    o = oracle.Oracle(inst)
    assert o.state_size() == sum(c for _, c in ucac.state_layout(9, 12, 3, 6))


def test_batch_validation(lib):
    """Batch arguments and member networks are checked before any device work."""
    good = synth.small_instance(9, 12, 3, 6, seed=5)
    bad = synth.small_instance(9, 12, 3, 6, seed=6)
    bad["gen_pmin"] = bad["gen_pmax"] + 1.0
    with pytest.raises(ucac.UcacError) as e:
        ucac.Batch([bad, good])
    assert e.value.code == ucac.UCAC_E_INVAL and "member 0" in str(e.value) and "pmin > pmax" in str(e.value)
    with pytest.raises(ucac.UcacError) as e:
        ucac.Batch([good], warm_start=2)
    assert e.value.code == ucac.UCAC_E_INVAL
    b = C.c_void_p()
    p = ucac.ucac_params_default()
    assert lib.ucac_batch_create(None, 0, C.byref(p), C.byref(b)) == ucac.UCAC_E_INVAL
    assert ucac.BATCH_CANDIDATES[0] == (64, 256, 0) and len(ucac.BATCH_CANDIDATES) == 8


def test_dp_batch_validation(lib):
    """Argument checks of the standalone DP happen before any device work."""
    assert lib.ucac_dp_batch(-1, 24, *([None] * 8), 64, None) == ucac.UCAC_E_INVAL
    assert lib.ucac_dp_batch(10, 0, *([None] * 8), 64, None) == ucac.UCAC_E_INVAL
    assert lib.ucac_dp_batch(10, 24, *([None] * 8), 32, None) == ucac.UCAC_E_INVAL
    assert lib.ucac_dp_batch(10, 24, *([None] * 8), 64, None) == ucac.UCAC_E_INVAL  # null pointers
    assert "null" in ucac.ucac_last_error(None)
    assert lib.ucac_dp_batch(0, 24, *([None] * 8), 64, None) == ucac.UCAC_OK  # nothing to do


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises at once: there is no CPU path
    to fall back to, and creating a solver fails rather than running anything else."""
    monkeypatch.setattr(ucac, "_lib", None)
    monkeypatch.setattr(ucac, "LIB_PATH", str(tmp_path / "libucac.so"))
    with pytest.raises(ImportError, match="missing"):
        ucac.lib()
    with pytest.raises(ImportError, match="missing"):
        ucac.Solver(synth.small_instance(9, 12, 3, 2, seed=1))
