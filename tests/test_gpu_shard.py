"""GPU: a hierarchy split over ranks (the one-GPU part of sharding).

Each rank's share runs as an instance of its own with remapped neighbour
tables; before every RK4 stage a copy kernel fills each rank's halo slots
from the ranks that own those ADOs.  The split launch must reproduce the
unsplit launch bitwise: every ADO is computed by the same kernel from the
same inputs.  The unsplit launch itself is checked against the oracle by
test_gpu_parity.py and test_gpu_full_size.py.
"""
import sys

import numpy as np
import pytest

from paper_1012_4382_amd import heom, workloads

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


@pytest.mark.parametrize("depth,ranks,steps", [(8, 8, 200), (16, 8, 4), (5, 3, 64)])
def test_split_equals_unsplit_bitwise(depth, ranks, steps):
    w = workloads.fmo_like(seed=1, site=6, depth=depth)
    _say(f"case: N=7 depth {depth} split over {ranks} ranks, {steps} steps")
    h = heom.Hierarchy(w["system"], depth)
    rho, sinks, ws = heom.propagate(h, w["rho0"], 1.0, steps, record_every=2)
    s = heom.Shard(h, ranks)
    rho_s, sinks_s, ws_s = heom.propagate_sharded(s, w["rho0"], 1.0, steps, record_every=2)
    assert np.array_equal(rho_s, rho)
    assert np.array_equal(sinks_s, sinks)
    sig, sc = heom.read_state(h, ws)
    sig_s, sc_s = heom.read_state_sharded(s, ws_s)
    assert np.array_equal(sig_s, sig) and np.array_equal(sc_s, sc)
    assert all(s.info(r)["n_halo"] > 0 for r in range(ranks))
    s.close()


def test_split_matsubara_resume_and_no_graph():
    """One Matsubara term per bath (14 modes), 4 ranks: a split run continued
    (HEOM_RESUME) and launched without graphs equals the unsplit straight run."""
    w = workloads.sweep_instance(2)  # depth 5, 11628 ADOs
    _say("case: sweep instance 2 (K=1, depth 5) over 4 ranks, 100 + 60 steps, resume")
    h = heom.Hierarchy(w["system"], w["depth"])
    rho, sinks, _ = heom.propagate(h, w["rho0"], 1.0, 160, record_every=160)
    s = heom.Shard(h, 4)
    _, _, ws = heom.propagate_sharded(s, w["rho0"], 1.0, 100, record_every=100)
    rho_s, sinks_s, _ = heom.propagate_sharded(s, None, 1.0, 60, record_every=60, workspace=ws,
                                               resume=True, graphs=False)
    assert np.array_equal(rho_s[-1], rho[-1])
    assert np.array_equal(sinks_s, sinks)
    s.close()
