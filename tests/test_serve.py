"""Serving engine logic on the CPU: admission by memory budget, continuous
batching, cancellation, rejection, failure isolation and latency bookkeeping,
with a virtual clock.  The device is replaced by a backend that advances each
request with the FP64 oracle (so results can be checked) and charges virtual
time for the work."""
import math

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import workloads
from paper_1012_4382_amd.serve import Engine, Request


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class OracleBackend:
    """Engine backend on the oracle; 1 ns of virtual time per ADO-step."""

    def __init__(self, clock, fail_ids=(), bytes_per_ado=1000, raise_after=False):
        self.clock = clock
        self.fail_ids = set(fail_ids)
        self.bytes_per_ado = bytes_per_ado
        # raise_after: a call that holds a failing request advances every
        # state, then raises (the caller cannot tell which states moved).
        self.raise_after = raise_after
        self.calls = []  # ids advanced together, per call
        self.steps = {}  # id -> RK4 steps actually applied to its state

    def footprint(self, req):
        n, _ = oracle.count(req.system, req.depth)
        return n * self.bytes_per_ado, n

    def admit(self, req, n):
        req.n_ados = n
        return {"state": None, "n": n}

    def advance(self, reqs, slots, k):
        """Every state advances by k steps; a request in fail_ids reports a
        failure of its own (or, with raise_after, the whole call raises after
        the states have moved)."""
        self.calls.append([r.id for r in reqs])
        rhos, sinks, errors = [], np.zeros((len(reqs), 3)), []
        for i, (r, s) in enumerate(zip(reqs, slots)):
            out = oracle.propagate(r.system, r.depth, r.rho0, r.dt, k, record_every=max(k, 1),
                                   want_state=True, state_in=s["state"], n_threads=1)
            s["state"] = out["state"]
            self.steps[r.id] = self.steps.get(r.id, 0) + k
            rhos.append(out["rho"][-1])
            sinks[i] = out["scalars"]
            errors.append("device fault in a request" if r.id in self.fail_ids else None)
        self.clock.t += k * sum(s["n"] for s in slots) * 1e-9
        if self.raise_after and any(e is not None for e in errors):
            raise RuntimeError("launch failed after the states were advanced")
        return rhos, sinks, errors

    def release(self, slot):
        slot["state"] = None


def _req(i, arrival, steps=120, depth=2, N=2):
    rng = np.random.default_rng(i)
    H = np.diag(rng.normal(12400, 100, N))
    for a in range(N - 1):
        H[a, a + 1] = H[a + 1, a] = rng.normal(-80, 20)
    trap = np.zeros(N)
    trap[-1] = 1.0
    return Request(id=i, system=workloads.system(H, trap=trap, rec=np.full(N, 1e-3)),
                   depth=depth, rho0=workloads.site_state(N, 1), steps=steps, arrival_s=arrival)


def test_results_match_the_request_run_alone():
    """Chunked, batched service gives bitwise the oracle's straight run."""
    clock = VClock()
    eng = Engine(OracleBackend(clock), hbm_budget_bytes=10**9, chunk_steps=50, clock=clock,
                 sleep=clock.sleep)
    reqs = [_req(i, arrival=i * 1e-7, steps=60 + 37 * i, depth=2 + i % 2, N=2 + i % 3)
            for i in range(5)]
    m = eng.run(reqs)
    assert m["completed"] == 5
    for r in reqs:
        ref = oracle.propagate(r.system, r.depth, r.rho0, r.dt, r.steps, record_every=r.steps,
                               n_threads=1)
        assert np.array_equal(r.rho_final, ref["rho"][-1]), r.id
        assert np.array_equal(r.sinks, ref["scalars"]), r.id


def test_admission_respects_budget_and_fifo():
    clock = VClock()
    be = OracleBackend(clock, bytes_per_ado=1000)
    # Depth 2 dimer: 6 ADOs -> 6000 bytes each; budget fits two at a time.
    eng = Engine(be, hbm_budget_bytes=13000, chunk_steps=40, clock=clock, sleep=clock.sleep)
    reqs = [_req(i, arrival=0.0, steps=80) for i in range(5)]
    m = eng.run(reqs)
    assert m["completed"] == 5
    assert max(len(c) for c in be.calls) == 2
    admits = [r.admit_s for r in sorted(reqs, key=lambda r: r.id)]
    assert admits == sorted(admits)  # first come, first served
    assert eng.in_use == 0


def test_continuous_batching_admits_while_others_run():
    clock = VClock()
    be = OracleBackend(clock)
    eng = Engine(be, hbm_budget_bytes=10**9, chunk_steps=10, clock=clock, sleep=clock.sleep)
    long = _req(0, arrival=0.0, steps=400)
    late = _req(1, arrival=0.5e-6, steps=40)   # arrives while `long` is running
    m = eng.run([long, late])
    assert m["completed"] == 2
    assert any(set(c) == {0, 1} for c in be.calls)  # they shared launches
    assert late.finish_s < long.finish_s
    assert late.admit_s < long.finish_s


def test_rejection_cancellation_and_failure_isolation():
    clock = VClock()
    be = OracleBackend(clock, fail_ids={2})
    eng = Engine(be, hbm_budget_bytes=20000, chunk_steps=20, clock=clock, sleep=clock.sleep)
    big = _req(9, arrival=0.0, depth=6, N=3)      # 84 ADOs -> 84000 bytes > budget
    reqs = [_req(i, arrival=0.0, steps=60) for i in range(4)] + [big]
    for r in reqs:
        eng.submit(r)
    assert big.status == "rejected" and "budget" in big.error
    assert eng.cancel(3) and reqs[3].status == "cancelled"
    while eng.step():
        pass
    assert reqs[2].status == "failed" and "device fault" in reqs[2].error
    assert reqs[0].status == reqs[1].status == "done"
    ref = oracle.propagate(reqs[0].system, 2, reqs[0].rho0, 1.0, 60, record_every=60, n_threads=1)
    assert np.array_equal(reqs[0].sinks, ref["scalars"])
    assert eng.in_use == 0
    m = eng.metrics()
    assert (m["completed"], m["failed"], m["rejected"], m["cancelled"]) == (2, 1, 1, 1)


def test_latency_bookkeeping_with_virtual_clock():
    clock = VClock()
    eng = Engine(OracleBackend(clock), hbm_budget_bytes=10**9, chunk_steps=100, clock=clock,
                 sleep=clock.sleep)
    reqs = [_req(i, arrival=1.0 + i, steps=100) for i in range(3)]  # well separated
    m = eng.run(reqs)
    for r in reqs:
        # Alone on the device: latency = its own work, 6 ADOs x 100 steps x 1 ns.
        assert r.latency_s == pytest.approx(600e-9, rel=1e-6)
    assert m["p50_latency_s"] == pytest.approx(600e-9, rel=1e-6)
    assert math.isclose(m["mean_occupancy"], 1.0)


def test_engine_argument_validation():
    with pytest.raises(ValueError):
        Engine(OracleBackend(VClock()), hbm_budget_bytes=0)
    with pytest.raises(ValueError):
        Engine(OracleBackend(VClock()), hbm_budget_bytes=10, chunk_steps=0)
    with pytest.raises(ValueError):
        Engine(OracleBackend(VClock()), hbm_budget_bytes=10, max_active=0)


def test_one_at_a_time_baseline_and_finish_callback():
    """max_active=1 serves strictly one request at a time (the FIFO baseline);
    on_finish sees every request once, in completion order."""
    clock = VClock()
    be = OracleBackend(clock)
    eng = Engine(be, hbm_budget_bytes=10**9, chunk_steps=30, clock=clock, sleep=clock.sleep,
                 max_active=1)
    reqs = [_req(i, arrival=0.0, steps=60) for i in range(3)]
    seen = []
    m = eng.run(reqs, on_finish=lambda r: seen.append(r.id))
    assert m["completed"] == 3 and seen == [0, 1, 2]
    assert all(len(c) == 1 for c in be.calls)
    assert [r.admit_s for r in reqs] == sorted(r.admit_s for r in reqs)
    assert reqs[1].admit_s >= reqs[0].finish_s


def test_failed_slot_does_not_rerun_the_others():
    """A request that fails inside a batched advance leaves alone; the requests
    advanced with it are not advanced again, so their results are those of
    the request run alone and their step counts match the steps applied."""
    clock = VClock()
    be = OracleBackend(clock, fail_ids={1})
    eng = Engine(be, hbm_budget_bytes=10**9, chunk_steps=30, clock=clock, sleep=clock.sleep)
    reqs = [_req(i, arrival=0.0, steps=90) for i in range(3)]
    m = eng.run(reqs)
    assert reqs[1].status == "failed" and "device fault" in reqs[1].error
    assert m["completed"] == 2 and m["failed"] == 1
    for r in (reqs[0], reqs[2]):
        assert be.steps[r.id] == r.steps_done == r.steps
        ref = oracle.propagate(r.system, r.depth, r.rho0, r.dt, r.steps, record_every=r.steps,
                               n_threads=1)
        assert np.array_equal(r.rho_final, ref["rho"][-1]), r.id
        assert np.array_equal(r.sinks, ref["scalars"]), r.id
    assert eng.in_use == 0


def test_backend_exception_fails_the_call_without_rerun():
    """When the backend raises after moving the states, the engine cannot tell
    which requests advanced: every request of that call fails, none is run
    again, and no result is reported for them."""
    clock = VClock()
    be = OracleBackend(clock, fail_ids={1}, raise_after=True)
    eng = Engine(be, hbm_budget_bytes=10**9, chunk_steps=30, clock=clock, sleep=clock.sleep)
    reqs = [_req(i, arrival=0.0, steps=90) for i in range(3)]
    late = _req(5, arrival=1.0, steps=60)  # arrives after the failure, runs normally
    m = eng.run(reqs + [late])
    assert all(r.status == "failed" for r in reqs)
    assert len(be.calls) == 3 and be.calls[0] == [0, 1, 2]  # one call, then `late` alone
    assert all(be.steps[r.id] == 30 for r in reqs)  # advanced once, never re-run
    assert late.status == "done" and m["completed"] == 1 and m["failed"] == 3
    ref = oracle.propagate(late.system, late.depth, late.rho0, 1.0, 60, record_every=60,
                           n_threads=1)
    assert np.array_equal(late.sinks, ref["scalars"])
    assert eng.in_use == 0
