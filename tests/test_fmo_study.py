"""Host-side checks of the FMO study module: the Table 1 input matches its
fixture, the depth-convergence protocol stops where the paper's criterion
says, and the Gibbs reference has the textbook limits."""
import math
import os

import numpy as np

import oracle.dense
from paper_1012_4382_amd import fmo_study, workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_table1_model_matches_fixture_and_paper_rates():
    H = np.loadtxt(os.path.join(GOLDEN, "fmo_table1_cm.txt"))
    assert np.array_equal(workloads.FMO_TABLE1_H, H)
    s = workloads.fmo_table1()
    assert np.array_equal(s["trap_per_ps"], [0, 0, 0.4, 0.4, 0, 0, 0])
    assert np.allclose(s["rec_per_ps"], 1 / 250.0)
    assert workloads.fmo_table1(sinks=False)["trap_per_ps"] is None


def test_converge_depth_stops_at_the_criterion():
    calls = []

    def run(depth):  # trapping time converging geometrically in the depth
        calls.append(depth)
        return {"mean_trap_time_fs": 6000.0 + 800.0 / 2 ** depth, "eta": 0.9,
                "t_end_fs": 1.0, "p_recomb": 0.0, "p_remaining": 0.0}

    r = fmo_study.converge_depth(run, 3, 20.0, 12)
    # |t(D+1) - t(D)| = 400 / 2^D: 25 (4->5), 12.5 (5->6), 6.25 (6->7): two
    # changes in a row within 20 fs end the search at depth 7.
    assert r["converged"] and r["depth"] == 7 and calls == [3, 4, 5, 6, 7]
    assert r["delta_fs"] == 400.0 / 2 ** 6
    r = fmo_study.converge_depth(run, 3, 1e-9, 5)
    assert not r["converged"] and r["depth"] == 5

    # A chance agreement of two shallow depths does not end the search.
    seq = {3: 7000.0, 4: 7005.0, 5: 6500.0, 6: 6490.0, 7: 6485.0}
    r = fmo_study.converge_depth(lambda d: {"mean_trap_time_fs": seq[d]}, 3, 20.0, 7)
    assert r["converged"] and r["depth"] == 7


def test_gibbs_populations_limits():
    assert math.isclose(fmo_study.KB_CM_PER_K, oracle.dense.KB_CM_PER_K, rel_tol=1e-15)
    E = np.array([0.0, 100.0, 250.0])
    p = fmo_study.gibbs_populations(np.diag(E), 300.0)
    w = np.exp(-E / (fmo_study.KB_CM_PER_K * 300.0))
    assert np.allclose(p, w / w.sum(), rtol=1e-14)
    g = fmo_study.gibbs_populations(workloads.FMO_TABLE1_H, 300.0)
    assert abs(g.sum() - 1.0) < 1e-14 and np.all(g > 0)
    assert np.allclose(fmo_study.gibbs_populations(workloads.FMO_TABLE1_H, 1e9), 1 / 7, atol=1e-6)
