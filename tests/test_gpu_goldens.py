"""The benchmarked launches over their full length against the oracle.

The references are the FP64 oracle's trajectories stored in tests/golden/ by
make_oracle_goldens.py, which calls only the oracle and the seeded input
generators.  Each test runs the launch configuration the benchmark times (the
batched, autotuned LDS-tiled kernels, the benchmark's record interval) and
compares it with the oracle over the whole run:

* the FMO-shaped 8-solve batch at depth 7: populations every 10 steps and
  sigma_0 every 100 steps over 5 ps, and eta = P_trap(5 ps) (eq:eta), FP64;
* the precision workload at depth 8, T = 77 and 300 K, 5 ps: FP32-mixed
  within 1e-5 absolute on populations (every 10 steps) and eta, FP64 within
  1e-10;
* the 64-instance parameter sweep (one Matsubara term per bath, depth 3-5)
  in one batched launch, 1000 steps, every instance against the oracle, FP64
  and FP32-mixed;
* served requests of the serving trace against the same request run alone
  (bitwise) and against the oracle (at full length where it covers it; the
  24-site requests at depth 3 and 4 over the oracle's first steps).

FP64 bar: 1e-10 relative to the largest entry of the compared quantity over
the trajectory; FP32-mixed bar: 1e-5 absolute on populations and eta.
"""
import os
import sys

import numpy as np
import pytest

from paper_1012_4382_amd import heom, workloads

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} has not been written (tests/golden/make_oracle_goldens.py)")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _pops(rho):
    return np.real(np.diagonal(rho, axis1=1, axis2=2))


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_fmo_batch_benchmarked_launch_over_5ps():
    g = _golden("oracle_fmo_like_depth7.npz")
    batch = [workloads.fmo_like(seed=int(s), site=int(site), depth=7, steps=5000)
             for s, site in zip(g["seeds"], g["sites"])]
    _say("case: FMO-shaped 8-solve batch, depth 7, 5000 steps, records every 10, FP64, autotuned")
    hs = [heom.Hierarchy(w["system"], 7) for w in batch]
    rhos, sinks, _ = heom.propagate_batch(hs, [w["rho0"] for w in batch], 1.0, 5000,
                                          record_every=10)
    for k in range(len(hs)):
        assert _rel(_pops(rhos[k]), g["pops"][k]) <= FP64_TOL, k
        assert _rel(rhos[k][::10], g["rho"][k]) <= FP64_TOL, k
        for q in range(3):  # P_trap (eta at 5 ps), P_rec, Q
            ref = g["scalars"][k][q]
            assert abs(sinks[k][q] - ref) <= FP64_TOL * abs(ref), (k, q)
    assert np.all(g["scalars"][:, 0] > 0.05)  # eta is not small


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_precision_workload_over_5ps(precision):
    g = _golden("oracle_precision_depth8.npz")
    cases = [workloads.fmo_like(seed=int(s), site=1, depth=8, T=float(T))
             for s, T in zip(g["seeds"], g["temperatures"])]
    _say(f"case: precision workload depth 8 (6435 ADOs), T 77/300 K, 5000 steps, {precision}")
    hs = [heom.Hierarchy(w["system"], 8) for w in cases]
    rhos, sinks, _ = heom.propagate_batch(hs, [w["rho0"] for w in cases], 1.0, 5000,
                                          record_every=10, precision=precision)
    for k in range(len(hs)):
        dp = float(np.max(np.abs(_pops(rhos[k]) - g["pops"][k])))
        de = abs(sinks[k][0] - g["scalars"][k][0])
        _say(f"  seed {g['seeds'][k]} T {g['temperatures'][k]}: max |dp| {dp:.2e}, "
             f"|d eta| {de:.2e}")
        if precision == "fp32":
            assert dp <= FP32_TOL and de <= FP32_TOL, k
        else:
            assert _rel(_pops(rhos[k]), g["pops"][k]) <= FP64_TOL, k
            assert _rel(rhos[k][::10], g["rho"][k]) <= FP64_TOL, k
            assert de <= FP64_TOL * g["scalars"][k][0], k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sweep_batched_launch_64_instances(precision):
    g = _golden("oracle_sweep_k1.npz")
    cases = [workloads.sweep_instance(i) for i in range(64)]
    _say(f"case: sweep, 64 instances in one batched launch, 1000 steps, records every 100, "
         f"{precision}")
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in cases]
    rhos, sinks, _ = heom.propagate_batch(hs, [w["rho0"] for w in cases], 1.0, 1000,
                                          record_every=100, precision=precision)
    assert sorted({int(d) for d in g["depth"]}) == [3, 4, 5]
    assert sorted(int(i) for i in g["instances"]) == list(range(64))
    for k, i in enumerate(g["instances"]):
        i = int(i)
        assert hs[i].depth == int(g["depth"][k])
        if precision == "fp64":
            assert _rel(rhos[i], g["rho"][k]) <= FP64_TOL, i
            for q in range(3):
                assert abs(sinks[i][q] - g["scalars"][k][q]) <= FP64_TOL * abs(g["scalars"][k][q])
        else:
            assert np.max(np.abs(_pops(rhos[i]) - _pops(g["rho"][k]))) <= FP32_TOL, i
            assert abs(sinks[i][0] - g["scalars"][k][0]) <= FP32_TOL, i
    # Every instance conserves population exactly: Tr sigma_0 + P_trap +
    # P_rec = 1.
    for r, s in zip(rhos, sinks):
        assert abs(np.trace(r[-1]).real + s[0] + s[1] - 1.0) < (1e-12 if precision == "fp64"
                                                                else 1e-6)


def _serve(reqs_w, precision):
    from paper_1012_4382_amd.serve import Engine, GpuBackend, Request

    reqs = [Request(id=w["id"], system=w["system"], depth=w["depth"], rho0=w["rho0"],
                    steps=w["steps"], arrival_s=w["arrival_s"], precision=precision)
            for w in reqs_w]
    eng = Engine(GpuBackend(), hbm_budget_bytes=64 << 30, chunk_steps=200)
    m = eng.run(reqs)
    assert m["completed"] == len(reqs)
    return reqs, m


@pytest.mark.parametrize("precision,n_requests", [("fp64", 40), ("fp32", 20)])
def test_served_requests_against_alone_and_oracle(precision, n_requests):
    g = _golden("oracle_serving.npz")
    trace = workloads.serving_trace(200)[:n_requests]
    n24 = sum(w["system"]["H"].shape[0] == 24 for w in trace)
    _say(f"case: serving, first {n_requests} requests of the trace ({n24} with 24 sites), "
         f"{precision}")
    served, m = _serve(trace, precision)
    assert m["mean_occupancy"] > 1.5  # requests really shared launches
    checked_full = checked_head = 0
    for r in served:
        j, N = r.id, r.system["H"].shape[0]
        h = heom.Hierarchy(r.system, r.depth)
        # Alone: the same request by itself, straight through (bitwise equal).
        rho, sinks, _ = heom.propagate(h, r.rho0, 1.0, r.steps, record_every=r.steps,
                                       precision=precision)
        assert np.array_equal(r.rho_final, rho[-1]), j
        assert np.array_equal(r.sinks, sinks), j
        if not g["done"][j]:
            continue
        ref = g["rho_flat"][g["rho_off"][j]:g["rho_off"][j + 1]].reshape(N, N)
        n = int(g["steps"][j])
        if n != r.steps:
            # The oracle covers the first n steps of this request: compare a
            # run of the request alone over those steps.
            rho, sinks, _ = heom.propagate(h, r.rho0, 1.0, n, record_every=n,
                                           precision=precision)
            got, got_sinks = rho[-1], sinks
            checked_head += 1
        else:
            got, got_sinks = r.rho_final, r.sinks
            checked_full += 1
        if precision == "fp64":
            assert _rel(got, ref) <= FP64_TOL, j
            assert abs(got_sinks[0] - g["scalars"][j][0]) <= FP64_TOL * abs(g["scalars"][j][0]), j
        else:
            assert np.max(np.abs(np.real(np.diag(got)) - np.real(np.diag(ref)))) <= FP32_TOL, j
            assert abs(got_sinks[0] - g["scalars"][j][0]) <= FP32_TOL, j
        h.close()
    _say(f"  oracle: {checked_full} requests over their whole run, {checked_head} over their "
         f"first steps")
    assert checked_full + checked_head > 0
