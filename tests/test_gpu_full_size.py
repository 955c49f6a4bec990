"""GPU parity at the largest sizes of the workloads, on the full state.

The benchmark's HBM-resident shape (7 sites, depth 16: 245157 ADOs, the
paper's largest hierarchy) and the serving workload's largest request (24
sites, depth 4: 20475 ADOs) are propagated for two RK4 steps by the launch
configuration the benchmark uses (the autotuned LDS-tiled kernels), and every
ADO, matched by multi-index, is compared with the FP64 oracle.  After two
steps every ADO up to tier 8 is nonzero, and at depth 4 all of them are.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import heom, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


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


def _compare_full_state(sys_, depth, rho0, steps, dt=1.0):
    h = heom.Hierarchy(sys_, depth)
    _, sinks, ws = heom.propagate(h, rho0, dt, steps, record_every=steps)
    sig, sc = heom.read_state(h, ws)
    ref = oracle.propagate(sys_, depth, rho0, dt, steps, record_every=steps, want_state=True)
    osig, osc = ref["state"]
    multi, _, _ = h.tables()
    omulti = oracle.enumerate_ados(sys_, depth)
    index = {tuple(int(v) for v in r): i for i, r in enumerate(omulti)}
    perm = np.array([index[tuple(int(v) for v in r)] for r in multi])
    assert len(set(perm.tolist())) == h.n_ados == len(omulti)
    want = osig[perm]
    scale = float(np.max(np.abs(want)))
    err = float(np.max(np.abs(sig - want)))
    assert err <= FP64_TOL * scale, (err, scale)
    assert np.max(np.abs(sc - osc)) <= FP64_TOL
    # Nonzero deep tiers: the comparison is not between zeros.
    tiers = np.sum(multi, axis=1)
    deepest = int(np.max(tiers[np.max(np.abs(sig), axis=(1, 2)) > 0]))
    return h.n_ados, deepest


def test_depth16_full_state_two_steps():
    w = workloads.fmo_like(seed=0, site=1, depth=16)
    _say("case: N=7 depth 16 (245157 ADOs), 2 steps, full state vs oracle")
    n, deepest = _compare_full_state(w["system"], 16, w["rho0"], 2)
    assert n == 245157 and deepest == 8


def test_24site_depth4_full_state_two_steps():
    w = next(r for r in workloads.serving_trace(200)
             if r["system"]["H"].shape[0] == 24 and r["depth"] == 4)
    _say("case: 24-site ring depth 4 (20475 ADOs), 2 steps, full state vs oracle")
    n, deepest = _compare_full_state(w["system"], 4, w["rho0"], 2)
    assert n == 20475 and deepest == 4
