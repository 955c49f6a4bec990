"""GPU parity of the wide stage kernel (13 <= N <= 32, real H) with the FP64 oracle.

The wide kernel runs the systems too large for the 64-ADO tile kernel: the
N = 24 chains and rings of the serving workload, and any real-H system with up
to 32 sites.  Each case has a ragged last tile (ADO counts are not multiples
of 16).  FP64 bar 1e-10 relative over the trajectory; FP32-mixed bar 1e-5 on
populations and P_trap.
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


def _chain(N, seed, ring=False, K=0):
    """Nearest-neighbour chain (or ring) as in the serving workload."""
    rng = np.random.default_rng(seed)
    H = np.diag(rng.normal(12400.0, 100.0, N))
    for i in range(N - 1):
        H[i, i + 1] = H[i + 1, i] = rng.normal(-80.0, 20.0)
    if ring:
        H[0, N - 1] = H[N - 1, 0] = rng.normal(-80.0, 20.0)
    trap = np.zeros(N)
    trap[-1] = 1.0
    return workloads.system(H, K=K, trap=trap, rec=np.full(N, 1e-3))


def _dense(N, seed, K=0):
    """Dense couplings (every H entry nonzero)."""
    H = workloads.fmo_like_hamiltonian(np.random.default_rng(seed), N)
    trap = np.zeros(N)
    trap[2] = 1.0
    return workloads.system(H, K=K, trap=trap, rec=np.full(N, 1e-3))


CASES = {
    # name: (system, depth, steps)
    "ring16_d2": (lambda: _chain(16, 16, ring=True), 2, 200),     # 153 ADOs
    "chain24_d2": (lambda: _chain(24, 24), 2, 100),                # 325 ADOs
    "chain32_d1": (lambda: _chain(32, 32), 1, 200),                # 33 ADOs, 32-bit row masks
    "dense13_k1_d2": (lambda: _dense(13, 13, K=1), 2, 100),        # 378 ADOs, 26 modes
}
_REF = {}


def _ref(name):
    if name not in _REF:
        mk, depth, steps = CASES[name]
        sys_ = mk()
        N = sys_["H"].shape[0]
        _REF[name] = (sys_, oracle.propagate(sys_, depth, workloads.site_state(N, 1), 1.0, steps,
                                             record_every=10, want_state=True))
    return _REF[name]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_wide_kernel_against_oracle(name, precision):
    mk, depth, steps = CASES[name]
    sys_, ref = _ref(name)
    N = sys_["H"].shape[0]
    _say(f"case: wide {name} N={N} depth={depth} {steps} steps {precision}")
    h = heom.Hierarchy(sys_, depth)
    rho, sinks, ws = heom.propagate(h, workloads.site_state(N, 1), 1.0, steps, record_every=10,
                                    precision=precision)
    if precision == "fp64":
        assert float(np.max(np.abs(rho - ref["rho"])) / np.max(np.abs(ref["rho"]))) <= FP64_TOL
        assert abs(sinks[0] - ref["scalars"][0]) <= FP64_TOL * max(abs(ref["scalars"][0]), 1e-3)
        # Every ADO of the final state, matched by multi-index, each tier
        # against its own largest entry.
        sig, _ = heom.read_state(h, ws)
        multi, _, _ = h.tables()
        perm = match_oracle_order(multi, oracle.enumerate_ados(sys_, depth))
        assert_tiers(multi, sig, ref["state"][0][perm], FP64_TOL, min_nonzero_tier=depth)
    else:
        p = np.real(np.diagonal(rho, axis1=1, axis2=2))
        pr = np.real(np.diagonal(ref["rho"], axis1=1, axis2=2))
        assert np.max(np.abs(p - pr)) <= FP32_TOL
        assert abs(sinks[0] - ref["scalars"][0]) <= FP32_TOL


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_wide_and_tile_instances_in_one_batch(precision):
    """A batch of tile-kernel (N = 7) and wide-kernel (N = 16, 24) instances
    equals the instances run alone, bitwise, with and without graphs."""
    fmo = workloads.fmo_like(seed=3, site=1, depth=3)
    items = [(fmo["system"], 3), (_chain(24, 24), 2), (_chain(16, 16, ring=True), 2)]
    hs = [heom.Hierarchy(s, d) for s, d in items]
    r0 = [workloads.site_state(h.N, 1) for h in hs]
    _say(f"case: mixed batch N=7/24/16 {precision}")
    rhos, sinks, _ = heom.propagate_batch(hs, r0, 1.0, 96, record_every=8, precision=precision)
    rhos_ng, sinks_ng, _ = heom.propagate_batch(hs, r0, 1.0, 96, record_every=8,
                                                precision=precision, graphs=False)
    for k, h in enumerate(hs):
        alone, s_alone, _ = heom.propagate(h, r0[k], 1.0, 96, record_every=8, precision=precision)
        assert np.array_equal(rhos[k], alone), k
        assert np.array_equal(sinks[k], s_alone), k
        assert np.array_equal(rhos_ng[k], alone), k
    assert np.array_equal(sinks, sinks_ng)


def test_beyond_wide_limit_uses_generic_kernel():
    """N = 33 exceeds the wide kernel's 32-site row masks: the generic kernel
    runs it, still within the FP64 bar."""
    sys_ = _chain(33, 33)
    _say("case: chain N=33 depth 1 (generic kernel)")
    h = heom.Hierarchy(sys_, 1)
    rho0 = workloads.site_state(33, 1)
    rho, sinks, _ = heom.propagate(h, rho0, 1.0, 100, record_every=10)
    ref = oracle.propagate(sys_, 1, rho0, 1.0, 100, record_every=10)
    assert float(np.max(np.abs(rho - ref["rho"])) / np.max(np.abs(ref["rho"]))) <= FP64_TOL
