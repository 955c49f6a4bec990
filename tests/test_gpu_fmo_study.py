"""GPU: the paper's FMO model (Table 1, trapping at BChl 3 and 4) through
heom_efficiency against the FP64 oracle at a fixed horizon, and one point of
the trapping-time protocol (run to the 1e-5 population criterion, depth
raised until the trapping time is stable)."""
import sys

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import fmo_study, heom, workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    heom.library()
    yield


@pytest.mark.parametrize("site", [1, 6])
def test_table1_efficiency_and_trapping_time_against_oracle(site):
    sys_ = workloads.fmo_table1(lam=55.0, gamma_inv_fs=166.0)
    rho0 = workloads.site_state(7, site)
    dt, steps = 2.5, 800  # 2 ps
    _say(f"case: FMO Table 1 lambda 55 depth 3 site {site} to 2 ps")
    h = heom.Hierarchy(sys_, 3)
    r = heom.efficiency(h, rho0, dt, dt * steps)
    ref = oracle.propagate(sys_, 3, rho0, dt, steps, record_every=steps)
    p_trap, p_rec, q = ref["scalars"]
    assert abs(r["eta"] - p_trap) <= 1e-10 * p_trap
    t_mean = dt * steps * p_trap - q  # int t dP_trap, by parts
    assert abs(r["mean_trap_time_fs"] - t_mean) <= 1e-10 * t_mean
    assert abs(r["p_recomb"] - p_rec) <= 1e-10 * p_rec


def test_trapping_protocol_point():
    _say("case: trapping protocol, lambda 35, site 1, depths 2..4")
    rows = fmo_study.trapping_scan([35.0], sites=(1,), depth0=2, max_depth=4, tol_ps=0.02)
    r = rows[0]
    assert 0.5 < r["eta"] < 1.0 and r["p_remaining"] < 1e-5
    assert 1.0 < r["trap_time_ps"] < 30.0 and r["t_max_ps"] > r["trap_time_ps"]
    assert r["depth"] in (3, 4)
    assert abs(r["eta"] + r["p_recomb"] + r["p_remaining"] - 1.0) < 1e-9
