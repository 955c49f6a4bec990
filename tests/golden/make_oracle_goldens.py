"""Writes the oracle's reference trajectories of the benchmarked workloads.

This script calls only the oracle (``oracle/``) and the seeded input
generators (``paper_1012_4382_amd/workloads.py``, which hold no arithmetic of
the method).  Nothing it stores comes from the GPU path.  The files it writes
are compared with the GPU runs in ``tests/test_gpu_goldens.py``:

* ``oracle_fmo_like_depth7.npz`` -- the FMO-shaped 7-site workload at depth 7
  (3432 ADOs): all 8 solves (Hamiltonian seeds 0-3, start at site 1 or 6),
  5000 RK4 steps of 1 fs (5 ps, eq:eta at t = 5 ps), FP64;
* ``oracle_precision_depth8.npz`` -- the same generator at depth 8 (6435 ADOs),
  seeds 0 and 1, T = 77 K and 300 K, start at site 1, 5000 steps;
* ``oracle_sweep_k1.npz`` -- all 64 parameter-sweep instances
  (one Matsubara term per bath; depths 3, 4 and 5), 1000 steps;
* ``oracle_serving.npz`` -- every request of the 200-request serving trace:
  at its full length where N <= 12 or depth 2; the 24-site requests at depth 3
  over their first 100 steps and at depth 4 over their first 50 steps (the
  oracle's full N x N matrices make a 24-site ADO-step about 20x the cost of a
  7-site one, so their full runs would take days of CPU time here; those
  requests are checked over their whole length on the GPU by the
  served-versus-alone comparison).

Arrays (all float64 or complex128, no object arrays; load with
``numpy.load(..., allow_pickle=False)``):
  pops   [solves, steps/10 + 1, N]   site populations every 10 steps
  rho    [solves, steps/100 + 1, N, N] reduced density matrix every 100 steps
  scalars [solves, 3]                P_trap, P_rec, Q after the last step
For the serving file, per request j: ``steps[j]`` (steps checked),
``scalars[j]`` and the final reduced density matrix in ``rho_flat`` at
``rho_off[j]`` (N*N complex, row-major); ``done[j]`` marks requests written.

Usage: python tests/golden/make_oracle_goldens.py {fmo,precision,sweep,serving,all}
       [--threads T]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1012_4382_amd import workloads  # noqa: E402

FILES = {
    "fmo": os.path.join(HERE, "oracle_fmo_like_depth7.npz"),
    "precision": os.path.join(HERE, "oracle_precision_depth8.npz"),
    "sweep": os.path.join(HERE, "oracle_sweep_k1.npz"),
    "serving": os.path.join(HERE, "oracle_serving.npz"),
}


def serving_check_steps(N: int, depth: int, steps: int) -> int:
    """Steps of a serving request that the oracle covers."""
    if N < 24 or depth <= 2:
        return steps
    return 100 if depth == 3 else 50


def fmo_cases():
    return [dict(seed=s, site=site) for s in (0, 1, 2, 3) for site in (1, 6)]


def precision_cases():
    return [dict(seed=s, T=T) for s in (0, 1) for T in (77.0, 300.0)]


def _save(path, **arrays):
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, **arrays)
    os.replace(tmp, path)


def _trajectory(w, threads):
    res = oracle.propagate(w["system"], w["depth"], w["rho0"], w["dt"], w["steps"],
                           record_every=10, n_threads=threads)
    rho = res["rho"]
    pops = np.real(np.diagonal(rho, axis1=1, axis2=2)).copy()
    return pops, rho[::10].copy(), res["scalars"].copy()


def make_fmo(threads):
    cases = fmo_cases()
    pops, rho, sc = [], [], []
    for c in cases:
        t0 = time.perf_counter()
        w = workloads.fmo_like(seed=c["seed"], site=c["site"], depth=7, steps=5000)
        p, r, s = _trajectory(w, threads)
        pops.append(p), rho.append(r), sc.append(s)
        print(f"fmo seed {c['seed']} site {c['site']}: eta {s[0]:.12f} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    _save(FILES["fmo"], seeds=np.array([c["seed"] for c in cases]),
          sites=np.array([c["site"] for c in cases]), depth=np.array(7), steps=np.array(5000),
          pops=np.array(pops), rho=np.array(rho), scalars=np.array(sc))


def make_precision(threads):
    cases = precision_cases()
    pops, rho, sc = [], [], []
    for c in cases:
        t0 = time.perf_counter()
        w = workloads.fmo_like(seed=c["seed"], site=1, depth=8, T=c["T"], steps=5000)
        p, r, s = _trajectory(w, threads)
        pops.append(p), rho.append(r), sc.append(s)
        print(f"precision seed {c['seed']} T {c['T']}: eta {s[0]:.12f} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    _save(FILES["precision"], seeds=np.array([c["seed"] for c in cases]),
          temperatures=np.array([c["T"] for c in cases]), depth=np.array(8),
          steps=np.array(5000), pops=np.array(pops), rho=np.array(rho), scalars=np.array(sc))


SWEEP_INSTANCES = 64


def make_sweep(threads):
    """Every instance of the sweep over 1000 steps, sigma_0 every 100 steps;
    continues a partly written file (instances are written as they finish)."""
    path = FILES["sweep"]
    rho, sc, depth, done = [], [], [], []
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            done = [int(i) for i in z["instances"]]
            rho = list(z["rho"])
            sc = list(z["scalars"])
            depth = [int(d) for d in z["depth"]]
    for i in range(SWEEP_INSTANCES):
        if i in done:
            continue
        t0 = time.perf_counter()
        w = workloads.sweep_instance(i)
        res = oracle.propagate(w["system"], w["depth"], w["rho0"], w["dt"], w["steps"],
                               record_every=100, n_threads=threads)
        rho.append(res["rho"].copy())
        sc.append(res["scalars"].copy())
        depth.append(w["depth"])
        done.append(i)
        _save(path, instances=np.array(done), depth=np.array(depth), steps=np.array(1000),
              rho=np.array(rho), scalars=np.array(sc))
        print(f"sweep {i} depth {w['depth']}: P_trap {res['scalars'][0]:.12f} "
              f"({time.perf_counter() - t0:.0f} s, {len(done)} done)", flush=True)


def make_serving(threads, n_requests=200):
    trace = workloads.serving_trace(n_requests)
    sizes = [r["system"]["H"].shape[0] for r in trace]
    off = np.concatenate([[0], np.cumsum([n * n for n in sizes])]).astype(np.int64)
    path = FILES["serving"]
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            done = z["done"].copy()
            steps = z["steps"].copy()
            scalars = z["scalars"].copy()
            rho_flat = z["rho_flat"].copy()
    else:
        done = np.zeros(n_requests, bool)
        steps = np.zeros(n_requests, np.int64)
        scalars = np.zeros((n_requests, 3))
        rho_flat = np.zeros(int(off[-1]), np.complex128)
    # Cheapest first, so that most requests are covered early.
    from math import comb

    def cost(r):
        N = r["system"]["H"].shape[0]
        n = serving_check_steps(N, r["depth"], r["steps"])
        return comb(N + r["depth"], r["depth"]) * n * N ** 3

    for r in sorted(trace, key=cost):
        j = r["id"]
        if done[j]:
            continue
        N = sizes[j]
        n = serving_check_steps(N, r["depth"], r["steps"])
        t0 = time.perf_counter()
        res = oracle.propagate(r["system"], r["depth"], r["rho0"], r["dt"], n, record_every=n,
                               n_threads=threads)
        rho_flat[off[j]:off[j + 1]] = res["rho"][-1].ravel()
        scalars[j] = res["scalars"]
        steps[j] = n
        done[j] = True
        _save(path, n_requests=np.array(n_requests), done=done, steps=steps, scalars=scalars,
              rho_off=off, rho_flat=rho_flat, n_sites=np.array(sizes),
              depth=np.array([q["depth"] for q in trace]),
              full_steps=np.array([q["steps"] for q in trace]))
        print(f"serving {j}: N {N} depth {r['depth']} steps {n}/{r['steps']} "
              f"({time.perf_counter() - t0:.0f} s, {int(done.sum())} done)", flush=True)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("what", choices=["fmo", "precision", "sweep", "serving", "all"])
    p.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = p.parse_args()
    todo = ["fmo", "precision", "sweep", "serving"] if a.what == "all" else [a.what]
    todo = [t for t in todo if a.what != "all" or t == "serving" or not os.path.exists(FILES[t])]
    for t in todo:
        {"fmo": make_fmo, "precision": make_precision, "sweep": make_sweep,
         "serving": make_serving}[t](a.threads)


if __name__ == "__main__":
    main()
