"""The allocation-free entry point heom_advance_slots_noalloc against
heom_advance_slots, through the C-ABI.

Both advance their own copies of the same runs (separate workspaces) and must
agree bitwise: they share the kernels, and the allocation-free call only
places its launch descriptors and work list in the library's static device
array.  Two calls in a row, the second with a smaller input (fewer slots, and
one continued run), check that a call leaves nothing behind that the next one
depends on.  Host-side rejections (oversized scratch, tables not resident)
need no kernel.
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


def _runs():
    trace = workloads.serving_trace(200)
    pick = [next(r for r in trace if r["system"]["H"].shape[0] == N and r["depth"] == D)
            for N, D in ((7, 4), (24, 2), (2, 3), (12, 2))]
    fmo = workloads.fmo_like(seed=2, site=6, depth=3)
    return [(r["system"], r["depth"], r["rho0"]) for r in pick] + \
        [(fmo["system"], 3, fmo["rho0"])]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_advance_slots_two_calls(precision):
    runs = _runs()
    hs = [heom.Hierarchy(s, d) for s, d, _ in runs]
    r0 = [r for _, _, r in runs]
    prec = heom.PRECISIONS[precision]
    ws_ref = [heom.allocate_workspace(h.workspace_bytes[prec]) for h in hs]
    ws_na = [heom.allocate_workspace(h.workspace_bytes[prec]) for h in hs]
    scratch = heom.allocate_workspace(heom.slots_scratch_bytes(hs))
    # Call 1: every run starts (the allocating call first: it uploads the
    # neighbour tables, which the allocation-free call requires).
    _say(f"case: noalloc vs advance_slots, 5 slots (N=7/24/2/12/7), start, 70 steps {precision}")
    rho_a, sk_a = heom.advance_slots(hs, ws_ref, [True] * 5, r0, 1.0, 70, scratch,
                                     precision=precision)
    rho_b, sk_b = heom.advance_slots_noalloc(hs, ws_na, [True] * 5, r0, 1.0, 70,
                                             precision=precision)
    for k in range(5):
        assert np.array_equal(rho_a[k], rho_b[k]), k
        assert np.array_equal(sk_a[k], sk_b[k]), k
    assert np.all(np.isfinite(sk_b)) and sk_b[:, 0].max() > 0
    p_trap_70 = sk_b[3, 0]
    # Call 2, smaller: two slots, one continued and one started afresh.
    sub = [3, 0]
    _say(f"case: noalloc vs advance_slots, 2 slots (continue N=12, restart N=7), 40 steps "
         f"{precision}")
    args = ([hs[k] for k in sub], None, [False, True], [None, r0[0]], 1.0, 40)
    rho_a, sk_a = heom.advance_slots(args[0], [ws_ref[k] for k in sub], *args[2:], scratch,
                                     precision=precision)
    rho_b, sk_b = heom.advance_slots_noalloc(args[0], [ws_na[k] for k in sub], *args[2:],
                                             precision=precision)
    for k in range(2):
        assert np.array_equal(rho_a[k], rho_b[k]), k
        assert np.array_equal(sk_a[k], sk_b[k]), k
    # The continued run really continued (its trapped population grew).
    assert sk_b[0, 0] > p_trap_70 > 0


def test_noalloc_host_rejections():
    """Rejected on the host, before any launch: a hierarchy whose tables are
    not on the device yet, and slots beyond the static scratch."""
    w = workloads.fmo_like(seed=3, site=1, depth=2)
    h = heom.Hierarchy(w["system"], 2)  # fresh handle: no device tables yet
    ws = heom.allocate_workspace(h.workspace_bytes[heom.HEOM_FP64])
    with pytest.raises(heom.HeomError) as e:
        heom.advance_slots_noalloc([h], [ws], [True], [w["rho0"]], 1.0, 10)
    assert e.value.status == heom.HEOM_E_UNSUPPORTED and "tables" in str(e.value)
    # 24-site depth 6 (593775 ADOs) in 8 slots needs more than 2 MiB of scratch.
    big = next(r for r in workloads.serving_trace(200) if r["system"]["H"].shape[0] == 24)
    hb = heom.Hierarchy(big["system"], 6)
    hs = [hb] * 8
    assert heom.slots_scratch_bytes(hs) > 2 << 20
    fake = [ws] * 8  # never dereferenced: the size check comes first
    with pytest.raises(heom.HeomError) as e:
        heom.advance_slots_noalloc(hs, fake, [True] * 8, [big["rho0"]] * 8, 1.0, 10)
    assert e.value.status == heom.HEOM_E_WORKSPACE and "static scratch" in str(e.value)
