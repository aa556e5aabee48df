"""The standalone UC dynamic program (Alg. dp_algo) on the GPU against the FP64
oracle's DP, unit by unit: schedules and optimal costs bit for bit (the recursion
is plain IEEE additions in a fixed order on both sides), on random tables, on
integer tables full of exact ties (the stay-on-ties rule), and on the horizons of
the paper's DP experiment."""
import numpy as np
import pytest
import torch

import oracle
from paper_2310_13145_amd import ucac

pytestmark = pytest.mark.gpu


def _case(G, T, seed, ties=False):
    rng = np.random.default_rng(seed)
    if ties:
        tab = rng.integers(0, 4, size=(G, T, 2, 2)).astype(np.float64)
    else:
        tab = rng.normal(0.0, 1.0, size=(G, T, 2, 2)) * rng.uniform(0.1, 10.0, size=(G, 1, 1, 1))
    tu = rng.integers(1, 7, G).astype(np.int32)
    td = rng.integers(1, 7, G).astype(np.int32)
    u0 = rng.integers(0, 2, G).astype(np.int32)
    lon = np.where(u0 == 1, rng.integers(0, 6, G), 0).astype(np.int32)
    loff = np.where(u0 == 0, rng.integers(0, 6, G), 0).astype(np.int32)
    return tab, tu, td, u0, lon, loff


def _run(case, lanes):
    tab, tu, td, u0, lon, loff = case
    dev = torch.device("cuda:0")
    t = [torch.from_numpy(x).to(dev) for x in (tab, tu, td, u0, lon, loff)]
    u, cost = ucac.ucac_dp_batch(*t, lanes_per_unit=lanes)
    torch.cuda.synchronize()
    return u.cpu().numpy(), cost.cpu().numpy()


def _check(case, u, cost):
    tab, tu, td, u0, lon, loff = case
    for g in range(tab.shape[0]):
        c, uo = oracle.dp(tab[g], u0[g], lon[g], loff[g], tu[g], td[g])
        assert c == cost[g], (g, c, cost[g])
        np.testing.assert_array_equal(u[g], uo, err_msg=f"unit {g}")


@pytest.mark.parametrize("T", [1, 6, 24, 48, 168])
@pytest.mark.parametrize("lanes", [64, 16])
def test_random_tables_bit_exact(T, lanes):
    print(f"[dp] T={T} lanes={lanes}", flush=True)
    case = _case(97, T, seed=1000 + T + lanes)
    u, cost = _run(case, lanes)
    _check(case, u, cost)


@pytest.mark.parametrize("lanes", [64, 16])
def test_ties_bit_exact(lanes):
    case = _case(200, 24, seed=7 + lanes, ties=True)
    u, cost = _run(case, lanes)
    _check(case, u, cost)


def test_sizes_and_errors():
    dev = torch.device("cuda:0")
    case = _case(0, 24, seed=3)
    u, cost = ucac.ucac_dp_batch(*[torch.from_numpy(x).to(dev) for x in case])
    assert u.shape == (0, 24) and cost.shape == (0,)
    big = _case(4, 400, seed=4)
    with pytest.raises(ucac.UcacError) as e:
        ucac.ucac_dp_batch(*[torch.from_numpy(x).to(dev) for x in big], lanes_per_unit=16)
    assert e.value.code == ucac.UCAC_E_INVAL and "LDS" in str(e.value)
    u, cost = _run(big, 64)  # one unit per block fits
    _check(big, u, cost)
