"""GPU: the resident kernels (whole RK4 steps of small hierarchies in one
workgroup) against the stage-per-launch path and the FP64 oracle.

The resident kernels repeat the tile kernel's operations in its order, so the
paths must agree bitwise: records, sinks and the full final state.  The
default ("auto") takes a resident kernel where a run fits one: the
compile-time kernel where every instance of the call has the same N <= 8 and
K+1 <= 2 (one to four packed elements x ADOs per thread, full matrices in
LDS, each element's threads padded to a multiple of 16 where the workgroup
holds them), else the run-time-N kernel for batches that mix hierarchies
(N <= 4, at most 1024 elements x ADOs each); "tiled" forces the stage
kernels.  Cases: the dimer (15 ADOs), a 3-site hierarchy with sinks and a
Matsubara term (84 ADOs), a 4-site depth-3 hierarchy (35 ADOs), the 7-site
FMO model at depth 2 (36 ADOs, unpadded), an 8-site depth-1 hierarchy, two
items per thread (the dimer at depth 25, 351 ADOs, an odd count that leaves
the last thread of each element one item), three items per thread on 768
threads (a 6-site depth-3 hierarchy, 84 ADOs; 8 sites at depth 2, 45 ADOs),
four items per thread on 512 threads where two and three would spill (3
sites with a Matsubara term at depth 4, 210 ADOs, the last group ragged),
mixed and same-N batches (one of 8-site instances of depths 2, 1 and 2 on three
items per thread), ring drains over 512 records, runs longer than one resident
launch, resume, and the efficiency entry point.
"""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import heom, workloads
from tiers import assert_tiers, match_oracle_order

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


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _four_site(seed=0, depth=3):
    rng = np.random.default_rng(100 + seed)
    H = workloads.fmo_like_hamiltonian(rng, N=4)
    tr, rc = workloads.fmo_sinks(N=4, trap_site=3)
    sys_ = workloads.system(H, trap=tr, rec=rc)
    return sys_, depth, workloads.site_state(4, 1)


def _three_site_matsubara():
    rng = np.random.default_rng(5)
    H = workloads.fmo_like_hamiltonian(rng, N=3)
    tr, rc = workloads.fmo_sinks(N=3, trap_site=2)
    sys_ = workloads.system(H, lam=60.0, gamma_inv_fs=80.0, T=150.0, K=1, trap=tr, rec=rc)
    return sys_, 3, workloads.site_state(3, 1)


def _n_site(N, depth, seed=0, K=0):
    rng = np.random.default_rng(200 + seed)
    H = workloads.fmo_like_hamiltonian(rng, N=N)
    tr, rc = workloads.fmo_sinks(N=N, trap_site=N)
    return workloads.system(H, K=K, trap=tr, rec=rc), depth, workloads.site_state(N, 1)


CASES = {
    "dimer": lambda: (workloads.dimer()["system"], 4, workloads.dimer()["rho0"]),
    "4site_depth3": _four_site,
    "3site_K1_depth3": _three_site_matsubara,
    "fmo_table1_depth2": lambda: (workloads.fmo_table1(), 2, workloads.site_state(7, 1)),
    "8site_depth1": lambda: _n_site(8, 1),
    "6site_depth3_three_items": lambda: _n_site(6, 3, seed=1),
    "dimer_depth25_ragged": lambda: (workloads.dimer()["system"], 25, workloads.dimer()["rho0"]),
    "8site_depth2_three_items": lambda: _n_site(8, 2, seed=2),
    "3site_K1_depth4_four_items": lambda: _n_site(3, 4, seed=3, K=1),
}


def _run(sys_, depth, rho0, steps, record_every, kernel, **kw):
    h = heom.Hierarchy(sys_, depth)
    rho, sinks, ws = heom.propagate(h, rho0, 1.0, steps, record_every=record_every, kernel=kernel,
                                    **kw)
    sig, sc = heom.read_state(h, ws)
    return h, rho, sinks, sig, sc


@pytest.mark.parametrize("name", list(CASES))
def test_resident_equals_tiled_and_oracle(name):
    sys_, depth, rho0 = CASES[name]()
    _say(f"case: resident vs tiled vs oracle, {name}, 600 steps, records every 3")
    h, rho, sinks, sig, sc = _run(sys_, depth, rho0, 600, 3, "auto")
    _, rho_t, sinks_t, sig_t, sc_t = _run(sys_, depth, rho0, 600, 3, "tiled")
    assert np.array_equal(rho, rho_t)
    assert np.array_equal(sinks, sinks_t)
    assert np.array_equal(sig, sig_t) and np.array_equal(sc, sc_t)
    ref = oracle.propagate(sys_, depth, rho0, 1.0, 600, record_every=3, want_state=True)
    assert _rel(rho, ref["rho"]) <= FP64_TOL
    multi, _, _ = h.tables()
    perm = match_oracle_order(multi, oracle.enumerate_ados(sys_, depth))
    assert_tiers(multi, sig, ref["state"][0][perm], FP64_TOL)
    for q in range(3):
        if ref["scalars"][q] != 0.0:
            assert abs(sinks[q] - ref["scalars"][q]) <= FP64_TOL * abs(ref["scalars"][q])


def test_resident_batch_ring_drains_and_chunks():
    """A batch that mixes hierarchies (the run-time-N kernel, one workgroup
    per instance), 1100 records (two ring drains), and a run without records
    longer than one resident launch."""
    batch = [CASES["dimer"](), _four_site(1), _four_site(2), _three_site_matsubara()]
    hs = [heom.Hierarchy(s, d) for s, d, _ in batch]
    r0 = [r for _, _, r in batch]
    _say("case: resident batch of 4 small instances, 1100 steps, records every step")
    rho, sinks, ws = heom.propagate_batch(hs, r0, 1.0, 1100, record_every=1)
    rho_t, sinks_t, ws_t = heom.propagate_batch(hs, r0, 1.0, 1100, record_every=1,
                                                kernel="tiled")
    for k in range(len(hs)):
        assert np.array_equal(rho[k], rho_t[k]), k
    assert np.array_equal(np.asarray(sinks), np.asarray(sinks_t))
    _say("case: resident batch, 9000 steps without records (three resident launches)")
    _, s1, _ = heom.propagate_batch(hs, r0, 1.0, 9000, want_rho=False)
    _, s2, _ = heom.propagate_batch(hs, r0, 1.0, 9000, want_rho=False, kernel="tiled")
    assert np.array_equal(np.asarray(s1), np.asarray(s2))
    for h in hs:
        h.close()


def test_resident_fixed_batch_ring_drains_and_chunks():
    """A batch of 4-site instances of depths 3 and 5 (the compile-time kernel
    with two items per thread, which the smaller instance takes too), 1100
    records and a run longer than one resident launch."""
    batch = [_four_site(4, depth=3), _four_site(5, depth=5), _four_site(6, depth=3)]
    hs = [heom.Hierarchy(s, d) for s, d, _ in batch]
    r0 = [r for _, _, r in batch]
    _say("case: compile-time resident batch, 4 sites depths 3/5/3, 1100 steps, every step")
    rho, sinks, _ = heom.propagate_batch(hs, r0, 1.0, 1100, record_every=1)
    rho_t, sinks_t, _ = heom.propagate_batch(hs, r0, 1.0, 1100, record_every=1, kernel="tiled")
    for k in range(len(hs)):
        assert np.array_equal(rho[k], rho_t[k]), k
    assert np.array_equal(np.asarray(sinks), np.asarray(sinks_t))
    ref = oracle.propagate(batch[1][0], 5, r0[1], 1.0, 1100, record_every=100)
    assert _rel(rho[1][::100], ref["rho"]) <= FP64_TOL
    _say("case: compile-time resident batch, 9000 steps without records")
    _, s1, ws1 = heom.propagate_batch(hs, r0, 1.0, 9000, want_rho=False)
    _, s2, ws2 = heom.propagate_batch(hs, r0, 1.0, 9000, want_rho=False, kernel="tiled")
    assert np.array_equal(np.asarray(s1), np.asarray(s2))
    for h in hs:
        h.close()


def test_resident_fixed_three_items_ragged_batch():
    """A batch of 8-site instances of depths 2, 1 and 2 (the compile-time
    kernel with three items per thread on 768 threads, chosen for the costlier
    depth-2 instances; each element's threads padded to 16, so the depth-1
    instance, 9 ADOs, leaves 13 of every 16 threads without items), 600
    records, against the stage launches bitwise and the oracle."""
    batch = [_n_site(8, 2, seed=4), _n_site(8, 1, seed=5), _n_site(8, 2, seed=6)]
    hs = [heom.Hierarchy(s, d) for s, d, _ in batch]
    r0 = [r for _, _, r in batch]
    _say("case: compile-time resident batch, 8 sites depths 2/1/2, 600 steps, every step")
    rho, sinks, _ = heom.propagate_batch(hs, r0, 1.0, 600, record_every=1)
    rho_t, sinks_t, _ = heom.propagate_batch(hs, r0, 1.0, 600, record_every=1, kernel="tiled")
    for k in range(len(hs)):
        assert np.array_equal(rho[k], rho_t[k]), k
    assert np.array_equal(np.asarray(sinks), np.asarray(sinks_t))
    for k in (0, 1):
        sys_, depth, _ = batch[k]
        ref = oracle.propagate(sys_, depth, r0[k], 1.0, 600, record_every=100)
        assert _rel(rho[k][::100], ref["rho"]) <= FP64_TOL, k
    for h in hs:
        h.close()


def test_resident_resume_and_efficiency():
    sys_, depth, rho0 = _four_site(3)
    h = heom.Hierarchy(sys_, depth)
    _say("case: resident resume, 4 sites depth 3, 250 + 350 steps vs 600 straight")
    rho_a, _, ws = heom.propagate(h, rho0, 1.0, 250, record_every=50)
    rho_b, s_b, ws = heom.propagate(h, rho0, 1.0, 350, record_every=50, workspace=ws,
                                    resume=True)
    rho_c, s_c, _ = heom.propagate(h, rho0, 1.0, 600, record_every=50)
    assert np.array_equal(np.concatenate([rho_a, rho_b[1:]]), rho_c)
    assert np.array_equal(s_b, s_c)
    _say("case: efficiency on the resident path, 2 ps horizon, vs oracle")
    eff = heom.efficiency(h, rho0, 1.0, 2000.0)
    ref = oracle.propagate(sys_, depth, rho0, 1.0, 2000, record_every=2000)
    assert abs(eff["eta"] - ref["scalars"][0]) <= FP64_TOL * abs(ref["scalars"][0])
    h.close()


def test_resident_is_faster_for_the_dimer():
    """The point of the resident kernel: the dimer's steps in a few launches
    instead of four stage launches each (the compile-time form measured 9.6x
    on 1000 steps with every step recorded, the run-time form 2.0x over 5000
    steps with records every 10; here 10000 steps, workspace and stream
    reused, the best of three calls, bar 1.5x)."""
    import torch

    w = workloads.dimer()
    h = heom.Hierarchy(w["system"], w["depth"])
    ws = heom.allocate_workspace(h.workspace_bytes[heom.HEOM_FP64])
    stream = torch.cuda.Stream()
    times = {}
    for kernel in ("tiled", "auto"):
        best = float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            heom.propagate(h, w["rho0"], 1.0, 10000, record_every=10000, kernel=kernel,
                           workspace=ws, stream=stream)
            best = min(best, time.perf_counter() - t0)
        times[kernel] = best
    _say(f"  dimer 10000 steps: tiled {times['tiled'] * 1e3:.1f} ms, resident "
         f"{times['auto'] * 1e3:.1f} ms")
    assert times["auto"] * 1.5 < times["tiled"]
    h.close()
