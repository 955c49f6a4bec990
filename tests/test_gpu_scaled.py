"""GPU: the scaled hierarchy and its filter against the oracle.

The scaled hierarchy holds sigma_n / w_n with w_n = sqrt(prod_m n_m! |c_m|^n_m)
(the introduction's scaled HEOM); its stages run on the tile kernel (launch
shape 0, N <= 12) or the wide kernel with coupling weights by mode and
occupation, and the two agree bitwise.  The oracle propagates the same
scaled equations (pinned in test_oracle_pins.py against the similarity
transform of the dense generator and against the unscaled oracle).

Bars: FP64 1e-10 relative on sigma_0 over the trajectory and per tier on the
full scaled state; FP32-mixed 1e-5 absolute on populations and P_trap.  With
the filter, an ADO whose largest entry lies within rounding of the threshold
can be kept on one side and zeroed on the other (the GPU's nested RK4 and the
oracle's classic RK4 round differently), so filtered runs are compared at
1e-10 relative plus the threshold, and their counts of nonzero ADOs within 1 %.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import heom, workloads
from tiers import assert_tiers, match_oracle_order

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-5


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


def _three_sites(seed=2):
    w = workloads.fmo_like(seed=seed, site=1)
    return dict(w["system"], H=w["system"]["H"][:3, :3], trap_per_ps=np.array([0, 0, 1.0]),
                rec_per_ps=np.full(3, 1e-3)), w["rho0"][:3, :3]


CASES = {
    "fmo7_d4": lambda: (workloads.fmo_like(seed=0, site=1)["system"], 4,
                        workloads.site_state(7, 1), 300),
    "sweep7_k1_d3": lambda: (workloads.sweep_instance(5)["system"], 3,
                             workloads.site_state(7, 1), 300),
    "three_d10": lambda: (*_three_sites()[:1], 10, _three_sites()[1], 500),
}


@pytest.mark.parametrize("name", list(CASES))
def test_scaled_against_oracle(name):
    sys_, depth, rho0, steps = CASES[name]()
    _say(f"case: scaled {name}, {steps} steps, FP64 vs the oracle's scaled equations")
    h = heom.Hierarchy(sys_, depth, scaled=True)
    rho, sinks, ws = heom.propagate(h, rho0, 1.0, steps, record_every=10)
    ref = oracle.propagate(sys_, depth, rho0, 1.0, steps, record_every=10, scaled=True,
                           want_state=True)
    assert np.max(np.abs(rho - ref["rho"])) <= FP64_TOL * np.max(np.abs(ref["rho"]))
    assert np.max(np.abs(sinks - ref["scalars"])) <= FP64_TOL * np.max(np.abs(ref["scalars"]))
    sig, _ = heom.read_state(h, ws)
    multi, _, _ = h.tables()
    perm = match_oracle_order(multi, oracle.enumerate_ados(sys_, depth))
    assert_tiers(multi, sig, ref["state"][0][perm], FP64_TOL, min_nonzero_tier=depth)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_scaled_tile_equals_wide(name, precision):
    """Scaled hierarchies of N <= 12 run on the tile kernel by default; the
    wide kernel (launch shape 5, forced) gives the same records, sinks and
    state bitwise, with and without the filter."""
    sys_, depth, rho0, steps = CASES[name]()
    for tol in (0.0, 1e-7):
        _say(f"case: scaled {name}, filter {tol:g}, tile vs wide kernel, {precision}")
        h = heom.Hierarchy(sys_, depth, scaled=True, filter_tol=tol)
        a = heom.propagate(h, rho0, 1.0, steps, record_every=10, precision=precision)
        b = heom.propagate(h, rho0, 1.0, steps, record_every=10, precision=precision,
                           tile_shape=5)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        sa, _ = heom.read_state(h, a[2], precision=precision)
        sb, _ = heom.read_state(h, b[2], precision=precision)
        assert np.array_equal(sa, sb)
        h.close()


def test_scaled_equals_unscaled_on_sigma0():
    """Same equations in other variables: the scaled and unscaled GPU runs
    give the same reduced density matrix to rounding over 2 ps."""
    w = workloads.fmo_like(seed=3, site=6, depth=5)
    _say("case: FMO-like depth 5, scaled vs unscaled GPU, 2000 steps")
    a = heom.propagate(heom.Hierarchy(w["system"], 5), w["rho0"], 1.0, 2000, record_every=20)
    b = heom.propagate(heom.Hierarchy(w["system"], 5, scaled=True), w["rho0"], 1.0, 2000,
                       record_every=20)
    assert np.max(np.abs(a[0] - b[0])) <= 1e-12 * np.max(np.abs(a[0]))
    assert np.max(np.abs(a[1] - b[1])) <= 1e-12


@pytest.mark.parametrize("tol", [1e-5, 1e-7])
def test_filtered_against_oracle(tol):
    sys_, rho0 = _three_sites()
    D, steps = 10, 2000
    _say(f"case: scaled + filter {tol:g}, three sites depth 10, {steps} steps, FP64")
    h = heom.Hierarchy(sys_, D, scaled=True, filter_tol=tol)
    rho, sinks, ws = heom.propagate(h, rho0, 1.0, steps, record_every=20)
    ref = oracle.propagate(sys_, D, rho0, 1.0, steps, record_every=20, scaled=True,
                           filter_tol=tol, want_state=True)
    assert np.max(np.abs(rho - ref["rho"])) <= FP64_TOL * np.max(np.abs(ref["rho"])) + tol
    assert abs(sinks[0] - ref["scalars"][0]) <= FP64_TOL * ref["scalars"][0] + tol
    sig, _ = heom.read_state(h, ws)
    kept = int(np.sum(np.max(np.abs(sig), axis=(1, 2)) > 0))
    kept_ref = int(np.sum(np.max(np.abs(ref["state"][0]), axis=(1, 2)) > 0))
    assert abs(kept - kept_ref) <= max(1, kept_ref // 100)
    assert kept < h.n_ados  # the filter dropped ADOs
    # Every surviving ADO (sigma_0 aside) has an entry at or above the threshold.
    big = np.maximum(np.abs(sig.real), np.abs(sig.imag)).max(axis=(1, 2))
    assert np.all(big[1:][big[1:] > 0] >= tol)


def test_filtered_fp32_mixed_and_batch():
    """FP32-mixed storage with the filter against the FP64 oracle (1e-5), and
    scaled, filtered and plain instances in one batch equal to each alone."""
    sys_, rho0 = _three_sites(seed=1)
    D, steps, tol = 8, 1000, 1e-6
    _say("case: scaled + filter 1e-6 FP32-mixed vs oracle; mixed batch vs alone")
    h = heom.Hierarchy(sys_, D, scaled=True, filter_tol=tol)
    rho, sinks, _ = heom.propagate(h, rho0, 1.0, steps, record_every=10, precision="fp32")
    ref = oracle.propagate(sys_, D, rho0, 1.0, steps, record_every=10, scaled=True,
                           filter_tol=tol)
    pops = np.real(np.diagonal(rho - ref["rho"], axis1=1, axis2=2))
    assert np.max(np.abs(pops)) <= FP32_TOL and abs(sinks[0] - ref["scalars"][0]) <= FP32_TOL
    fmo = workloads.fmo_like(seed=0, site=1, depth=3)
    hs = [h, heom.Hierarchy(fmo["system"], 3), heom.Hierarchy(fmo["system"], 3, scaled=True)]
    r0 = [rho0, fmo["rho0"], fmo["rho0"]]
    for prec in ("fp64", "fp32"):
        rhos, sk, _ = heom.propagate_batch(hs, r0, 1.0, 96, record_every=8, precision=prec)
        for k, hk in enumerate(hs):
            alone, s_alone, _ = heom.propagate(hk, r0[k], 1.0, 96, record_every=8,
                                               precision=prec)
            assert np.array_equal(rhos[k], alone), (prec, k)
            assert np.array_equal(sk[k], s_alone), (prec, k)


def test_scaled_rejects_the_other_kernels():
    w = workloads.fmo_like(seed=0, site=1, depth=2)
    h = heom.Hierarchy(w["system"], 2, scaled=True)
    for kernel in ("generic", "lane"):
        with pytest.raises(heom.HeomError) as e:
            heom.propagate(h, w["rho0"], 1.0, 4, kernel=kernel)
        assert e.value.status == heom.HEOM_E_UNSUPPORTED
