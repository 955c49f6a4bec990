"""GPU: the two forms of the neighbour tables in one launch.

The stage kernels stage an instance's neighbour tables as 16-bit offsets from
the ADO's own index where every neighbour lies within 32767 ADOs, else as the
32-bit indices; the choice is per instance, so one batched launch can hold
both.  A 7-site depth-14 hierarchy (116280 ADOs, neighbours up to 38760 ADOs
apart: 32-bit) and a depth-5 one (792 ADOs: 16-bit) run together and alone;
the batch must equal the solo runs bitwise (records and sinks), and the small
one must match the FP64 oracle.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import heom, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU (run with -m 'not gpu' on CPU)")
    heom.library()
    yield


def _max_offset(h):
    _, up, down = h.tables()
    i = np.arange(h.n_ados)[:, None]
    du = np.where(up >= 0, up - i, 0)
    dd = np.where(down >= 0, down - i, 0)
    return int(max(np.abs(du).max(), np.abs(dd).max()))


def test_batch_mixes_16_and_32_bit_tables():
    big = workloads.fmo_like(seed=0, site=1, depth=14)
    small = workloads.fmo_like(seed=1, site=6, depth=5)
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in (big, small)]
    assert _max_offset(hs[0]) > 32767 >= _max_offset(hs[1])
    r0 = [big["rho0"], small["rho0"]]
    print(f"case: batch of {hs[0].n_ados} + {hs[1].n_ados} ADOs, 40 steps, records every 10",
          flush=True)
    sys.stdout.flush()
    rho_b, sinks_b, _ = heom.propagate_batch(hs, r0, 1.0, 40, record_every=10)
    for k, h in enumerate(hs):
        rho_1, sinks_1, _ = heom.propagate(h, r0[k], 1.0, 40, record_every=10)
        assert np.array_equal(rho_b[k], rho_1), k
        assert np.array_equal(np.asarray(sinks_b)[k], sinks_1), k
    ref = oracle.propagate(small["system"], 5, small["rho0"], 1.0, 40, record_every=10)
    err = np.max(np.abs(rho_b[1] - ref["rho"])) / np.max(np.abs(ref["rho"]))
    assert err <= FP64_TOL
    for h in hs:
        h.close()
