"""Batched execution on the GPU: every member of a batch computes, bit for bit,
what the same instance computes alone (same kernels, same arithmetic; the batch
only changes which block runs which member), under every mapping the tuner can
choose, across a tuning run, and in solve mode where members stop at different
iterations.  One member is also checked against the FP64 oracle directly."""
import numpy as np
import pytest

import oracle
from paper_2310_13145_amd import synth, ucac

pytestmark = pytest.mark.gpu


def members():
    """Uneven sizes and horizons (ring, meshes; T = 6 ... 48)."""
    return [
        synth.config_instance(0),                         # 9 buses, T = 6
        synth.small_instance(14, 20, 5, 12, seed=901),
        synth.small_instance(30, 45, 8, 24, seed=902),
        synth.config_instance(1),                         # 118 buses, T = 24
        synth.small_instance(60, 90, 15, 48, seed=903),
    ]


def _single_states(insts, n_iters):
    out = []
    for inst in insts:
        s = ucac.Solver(inst)
        s.step(n_iters)
        out.append(s.get_state())
        s.close()
    return out


def test_members_match_single_instances():
    insts = members()
    print(f"[batch] {len(insts)} members, sizes {[i['n_bus'] for i in insts]}", flush=True)
    ref = _single_states(insts, 30)
    b = ucac.Batch(insts)
    b.step(30)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.member(k).get_state(), ref[k], err_msg=f"member {k}")
    b.close()


def test_members_match_across_graph_sizes():
    """85 batch iterations in one call (graphs of 64, 16, 4 and 1) against each member
    run alone in single steps."""
    insts = members()[:3]
    ref = []
    for inst in insts:
        s = ucac.Solver(inst)
        for _ in range(85):
            s.step(1)
        ref.append(s.get_state())
        s.close()
    b = ucac.Batch(insts)
    b.step(85)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.member(k).get_state(), ref[k], err_msg=f"member {k}")
    b.close()


@pytest.mark.parametrize("cfg", ucac.BATCH_CANDIDATES)
def test_every_mapping_bit_identical(cfg):
    insts = members()
    ref = _single_states(insts, 12)
    b = ucac.Batch(insts)
    b.set_config(*cfg)
    assert b.config() == cfg
    b.step(12)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.member(k).get_state(), ref[k], err_msg=f"member {k}, config {cfg}")
    b.close()


@pytest.mark.parametrize("cfg", [(16, 256, 1), (64, 64, 0)])
def test_long_horizon_member_bit_identical(cfg):
    """A member with a long horizon sets the unit side's units per block for the whole
    batch (sized by the longest horizon); every member still computes what it does
    alone."""
    insts = [synth.small_instance(9, 12, 3, 6, seed=501), synth.small_instance(14, 20, 5, 160, seed=502),
             synth.small_instance(30, 45, 8, 24, seed=503)]
    print(f"[batch] long-horizon members, T = {[i['T'] for i in insts]}, config {cfg}", flush=True)
    ref = _single_states(insts, 10)
    b = ucac.Batch(insts)
    b.set_config(*cfg)
    b.step(10)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.member(k).get_state(), ref[k], err_msg=f"member {k}, config {cfg}")
    b.close()


def test_autotune_keeps_iterate():
    insts = members()
    ref = _single_states(insts, 20)
    b = ucac.Batch(insts)
    b.step(10)
    chosen, times = b.autotune(iters=5)
    print(f"[batch] tuned {chosen}: {times}", flush=True)
    assert chosen in ucac.BATCH_CANDIDATES and b.config() == chosen
    assert all(v > 0 for v in times.values())
    b.step(10)
    for k in range(len(insts)):
        np.testing.assert_array_equal(b.member(k).get_state(), ref[k], err_msg=f"member {k} after tuning")
    b.close()


def test_solve_stops_members_independently():
    insts = members()[:4]
    single = []
    for inst in insts:
        s = ucac.Solver(inst)
        rc, it = s.solve(1e-3, 3000)
        single.append((rc == ucac.UCAC_OK, it, s.get_state()))
        s.close()
    b = ucac.Batch(insts)
    rc, iters, conv = b.solve(1e-3, 3000)
    print(f"[batch] solve iters {iters.tolist()} converged {conv.tolist()} single {[x[1] for x in single]}", flush=True)
    for k in range(len(insts)):
        assert conv[k] == single[k][0] and iters[k] == single[k][1], k
        np.testing.assert_array_equal(b.member(k).get_state(), single[k][2], err_msg=f"member {k}")
    assert len(set(iters.tolist())) > 1  # the members really stopped at different iterations
    b.close()


def test_member_against_oracle():
    from test_gpu_parity import compare
    insts = members()
    b = ucac.Batch(insts)
    b.set_config(16, 64, 1)
    b.step(50)
    for k in (1, 4):
        o = oracle.Oracle(insts[k])
        o.step(50)
        compare(b.member(k).get_state(), o.get_state(), insts[k], 1e-8, f"batch member {k}")
    b.close()


def test_full_batch_sampled():
    """The 64-instance uneven batch (30 to 2000 buses, T in {12, 24, 48}): sampled
    members match their single-instance runs after tuning."""
    insts = synth.batch_instances(64)
    b = ucac.Batch(insts)
    chosen, _ = b.autotune(iters=3)
    b.step(5)
    for k in (0, 21, 63):
        s = ucac.Solver(insts[k])
        s.step(5)
        np.testing.assert_array_equal(b.member(k).get_state(), s.get_state(), err_msg=f"member {k}, config {chosen}")
        s.close()
    b.close()
