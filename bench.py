"""Throughput benchmark of the HEOM propagation on one MI355X.

One benchmark step is one pass of the whole hot path over one batch of
synthetic input: the batched parameter sweep, 64 instances of the 7-site
FMO-shaped system, each with its own Hamiltonian, bath (lambda, 1/gamma, T),
one Matsubara term per bath (14 bath modes) and hierarchy depth 3-5 (680 to
11628 ADOs, 381956 in all, 449 MB of FP64 state, beyond the 256 MB Infinity
Cache), propagated 1000 RK4 steps of 1 fs in FP64 with trapping and
recombination sinks, sigma_0 recorded every 100 steps, as one batched launch
sequence.  Inputs, tables and parameters are on the device before the timed
region starts.

Printed: one JSON line with ADO-steps/s (whole job), the roofline of the
dominant kernel from HIP events around the timed launches themselves (on the
classic RK4 algorithmic bytes, on the bytes the nested form moves, and on the
counted traffic of the committed rocprofv3 profile), the check of the timed
runs against the oracle's stored trajectories, and the oracle timed on this
host (1 thread and all threads) on a bounded sample.  Further legs, each
skippable: the FMO-shaped 8-solve batch at depth 7 (5 ps, eta) with its own
roofline, single-solve and FP32-mixed rates, the depth-16 and 24-site sizing
launches, the depth-16 hierarchy split over 8 ranks, the scaled hierarchy and
its filter at depths 12 and 16, batch scaling (2-128 solves and a plain device
copy for scale), the precision comparison against
the oracle, and the 200-request serving trace in FP64 and FP32-mixed.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import subprocess
import sys
import time
from math import comb

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# Algorithmic bytes per ADO per stage launch, in packed ADOs (N*N reals).
# RK4 in its classic k1..k4 form moves 16 packed ADOs per ADO-step (4 per
# stage): that is the algorithmic figure.  The nested form this library runs
# moves 11 per step (11/4 per stage); both rates are reported.
ALG_ADOS_PER_LAUNCH = 4.0
MOVED_ADOS_PER_LAUNCH = 11.0 / 4.0
ROOT = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(ROOT, "tests", "golden")
# rocprofv3 summaries of the stage kernels (FETCH_SIZE / WRITE_SIZE traffic
# per launch, by kernel and workload) and the sources whose digest they record.
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_1012_4382_amd/csrc/stage_kernels.h",
                  "paper_1012_4382_amd/csrc/heom_internal.h",
                  "paper_1012_4382_amd/csrc/kernels_tile_7.hip", "paper_1012_4382_amd/build.py"]


def _rates(n_ados, N, s, k_ms):
    """Bandwidth figures of a stage launch over n_ados ADOs of N sites (s bytes
    per real) that took k_ms milliseconds."""
    alg = n_ados * ALG_ADOS_PER_LAUNCH * N * N * s / (k_ms * 1e-3) / 1e9
    moved = n_ados * MOVED_ADOS_PER_LAUNCH * N * N * s / (k_ms * 1e-3) / 1e9
    return {"achieved_GBps": alg, "frac_of_hbm_peak": alg / HBM_PEAK_GBS,
            "moved_GBps": moved, "moved_frac_of_hbm_peak": moved / HBM_PEAK_GBS}


def _kernel_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profiled_traffic(workload: str, kernel: str):
    """Counted HBM bytes per launch of `kernel` on `workload` from the committed
    profiles (a block of "- kernel:", "- workload:", "- source digest:" and
    "- traffic per launch (bytes):" lines), or None when no profile covers it
    or its sources have changed since."""
    digest = _kernel_digest()
    try:
        names = sorted(f for f in os.listdir(PROFILE_DIR) if f.endswith(".md"))
    except OSError:
        return None
    for name in names:
        text = open(os.path.join(PROFILE_DIR, name)).read()
        for block in re.split(r"(?m)^(?=- kernel: )", text)[1:]:
            k = re.search(r"^- kernel: `([^`]+)`", block, re.M)
            w = re.search(r"^- workload: `([^`]+)`", block, re.M)
            d = re.search(r"^- source digest: `([0-9a-f]+)`", block, re.M)
            t = re.search(r"^- traffic per launch \(bytes\): (\d+)", block, re.M)
            if (k and w and d and t and k.group(1) == kernel and w.group(1) == workload and
                    d.group(1) == digest):
                return float(t.group(1))
    return None


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--rk4-steps", type=int, default=1000,
                   help="RK4 steps of one pass of the sweep (the benchmark step)")
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                   help="storage precision of the timed sweep")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fmo", action="store_true",
                   help="skip the FMO-shaped 8-solve batch (depth 7, 5 ps)")
    p.add_argument("--fmo-steps", type=int, default=5000,
                   help="RK4 steps of the FMO-shaped batch (5000: 5 ps, checked against the "
                        "oracle; fewer for profiler runs, then unchecked)")
    p.add_argument("--no-variants", action="store_true",
                   help="skip single-solve, FP32-mixed and one-at-a-time rates and precision")
    p.add_argument("--kernel", default="auto", choices=["auto", "lane", "generic"],
                   help="stage kernel (lane and generic are diagnostic)")
    p.add_argument("--no-small", action="store_true",
                   help="skip the small-hierarchy runs (resident kernel against stage launches)")
    p.add_argument("--no-sizing", action="store_true",
                   help="skip the depth-16 and 24-site sizing launches")
    p.add_argument("--no-shard", action="store_true",
                   help="skip the depth-16 hierarchy split over 8 ranks")
    p.add_argument("--no-scaled", action="store_true",
                   help="skip the scaled hierarchy and its filter at depths 12 and 16")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 256 MiB device copy (reference for traffic counters)")
    p.add_argument("--no-batch-scaling", action="store_true",
                   help="skip the 2-128 solve batches of the FMO-shaped workload")
    p.add_argument("--serve", type=int, default=200, metavar="R",
                   help="serve the first R requests of the serving trace (0: skip)")
    p.add_argument("--serve-precision", default="both", choices=["fp64", "fp32", "both"],
                   help="storage precision of the served solves")
    return p.parse_args()


def _load_golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def _timed(run, stream, torch, reps, warmup, launches_per_rep):
    """Times `reps` calls of run() after `warmup` untimed ones: wall clock
    between two device synchronisations, and HIP events recorded on the
    library's stream around the same calls.  Returns (seconds, device ms per
    stage launch, last result)."""
    out = None
    for _ in range(warmup):
        out = run()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(reps):
        out = run()
    ev1.record(stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return el, ev0.elapsed_time(ev1) / (reps * launches_per_rep), out


def _roofline(workload, kernel, n_ados, N, s, k_ms):
    """Roofline object of a stage launch over n_ados ADOs that took k_ms."""
    alg = n_ados * ALG_ADOS_PER_LAUNCH * N * N * s
    moved = n_ados * MOVED_ADOS_PER_LAUNCH * N * N * s
    traffic = _profiled_traffic(workload, kernel)
    r = {"bound": "hbm", "achieved": alg / (k_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": alg / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": traffic,
         "kernel": kernel, "kernel_avg_us": k_ms * 1e3, "bytes_per_launch": alg,
         "moved": moved / (k_ms * 1e-3) / 1e9,
         "moved_frac": moved / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
         "bytes_moved_per_launch": moved}
    if traffic is not None:
        r["counted"] = traffic / (k_ms * 1e-3) / 1e9
        r["counted_frac"] = r["counted"] / HBM_PEAK_GBS
    return r


def _kernel_name(heom, N, KP, n_tiles, precision, kernel):
    shape, shape_us, streaming, streaming_us = heom.autotune_lookup(N, KP, n_tiles, precision)
    T = "double" if precision == "fp64" else "float"
    # The 64-ADO tile kernel is built up to 12 sites; above that the wide
    # kernel is the only LDS-tiled choice and is not tuned.
    wide = shape == 5 or N > 12
    name = {"auto": (f"stage_tile<{N},{KP},{T},{max(shape, 0)}>" if not wide
                     else f"stage_wide<{T},{KP}>")
                    + (" with streaming stores" if streaming == 1 else ""),
            "lane": f"stage_fixed<{N},{KP},{T}>",
            "generic": f"stage_generic<{T}>"}[kernel]
    tune = {"tiles": n_tiles, "shape": shape, "streaming_stores": streaming,
            "stage_us_per_shape": [round(float(u), 3) for u in shape_us],
            "stage_us_streaming": round(float(streaming_us), 3),
            "shapes": [heom.tile_shape_info(N, KP, precision, k)
                       for k in range(heom.tile_shape_count())]}
    return name, tune


def _check_sweep(rhos, sinks, golden, prec):
    """The timed sweep's instances against the oracle's stored trajectories:
    max relative deviation of sigma_0 (every 100 steps) and of P_trap."""
    if golden is None or len(rhos[0]) != len(golden["rho"][0]):
        return None  # no stored trajectory, or a run of another length
    idx = [int(i) for i in golden["instances"]]
    drho = max(float(np.max(np.abs(rhos[i] - golden["rho"][k])) / np.max(np.abs(golden["rho"][k])))
               for k, i in enumerate(idx))
    dtrap = max(abs(float(sinks[i][0]) - float(golden["scalars"][k][0])) /
                abs(float(golden["scalars"][k][0])) for k, i in enumerate(idx))
    return {"instances_checked": len(idx), "max_rel_rho_error": drho,
            "max_rel_p_trap_error": dtrap, "bar": 1e-10 if prec == "fp64" else 1e-5}


def _fmo_batch(heom, torch, workloads, stream, args):
    """The FMO-shaped 7-site workload at depth 7 (3432 ADOs per solve), all 8
    solves (seeds 0-3, start at site 1 or 6), 5000 RK4 steps (5 ps), sigma_0
    every 10 steps, FP64: timed like the headline, its roofline, and its
    timed runs against the oracle's trajectories (populations every 10 steps,
    sigma_0 every 100, eta at 5 ps)."""
    steps = args.fmo_steps
    batch = workloads.fmo_like_batch(steps=steps)
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in batch]
    r0 = [w["rho0"] for w in batch]
    N = hs[0].N
    total = sum(h.n_ados for h in hs)
    ws = heom.allocate_workspace(heom.batch_workspace_bytes(hs, "fp64"))

    def run():
        return heom.propagate_batch(hs, r0, 1.0, steps, record_every=10, workspace=ws,
                                    stream=stream, kernel=args.kernel)

    reps = max(2, args.steps // 4)
    el, k_ms, (rhos, sinks, _) = _timed(run, stream, torch, reps, 1, 4 * steps)
    name, tune = _kernel_name(heom, N, 1, sum((h.n_ados + 63) // 64 for h in hs), "fp64",
                              args.kernel)
    out = {"workload": f"fmo_like_7site_depth7_fp64_8solves_{steps}steps", "n_ados": total,
           "passes": reps, "ado_steps_per_s": total * steps * reps / el,
           "ms_per_pass": 1e3 * el / reps,
           "roofline": _roofline("fmo_like_7site_depth7_fp64_8solves", name, total, N, 8, k_ms),
           "autotune": tune}
    g = _load_golden("oracle_fmo_like_depth7.npz")
    if g is not None and steps == int(g["steps"]):
        pops = [np.real(np.diagonal(r, axis1=1, axis2=2)) for r in rhos]
        out["check_vs_oracle"] = {
            "solves": len(hs),
            "max_rel_pop_error": max(float(np.max(np.abs(p - g["pops"][k])) /
                                           np.max(np.abs(g["pops"][k])))
                                     for k, p in enumerate(pops)),
            "max_rel_rho_error": max(float(np.max(np.abs(r[::10] - g["rho"][k])) /
                                           np.max(np.abs(g["rho"][k])))
                                     for k, r in enumerate(rhos)),
            "max_rel_eta_error": max(abs(float(sinks[k][0]) - float(g["scalars"][k][0])) /
                                     float(g["scalars"][k][0]) for k in range(len(hs))),
            "eta_5ps": [float(s[0]) for s in sinks], "bar": 1e-10}
    if not args.no_variants:
        # Plain single solve (FP64 and FP32-mixed) and the FP32-mixed batch.
        def single(prec):
            w1 = heom.allocate_workspace(hs[0].workspace_bytes[heom.PRECISIONS[prec]])
            heom.propagate(hs[0], r0[0], 1.0, 64, record_every=64, workspace=w1, stream=stream,
                           precision=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            heom.propagate(hs[0], r0[0], 1.0, 5000, record_every=10, workspace=w1,
                           stream=stream, precision=prec)
            torch.cuda.synchronize()
            return hs[0].n_ados * 5000 / (time.perf_counter() - t0)

        ws32 = heom.allocate_workspace(heom.batch_workspace_bytes(hs, "fp32"))
        el32, _, _ = _timed(lambda: heom.propagate_batch(hs, r0, 1.0, 5000, record_every=10,
                                                         precision="fp32", workspace=ws32,
                                                         stream=stream), stream, torch, 1, 1, 1)
        p64, p32 = single("fp64"), single("fp32")
        out["variants"] = {"fp64_single_solve_ado_steps_per_s": p64,
                           "fp32_single_solve_ado_steps_per_s": p32,
                           "fp32_mixed_batched_ado_steps_per_s": total * 5000 / el32,
                           "fp64_batched_over_single": out["ado_steps_per_s"] / p64,
                           "fp32_batched_over_single": total * 5000 / el32 / p32}
    for h in hs:
        h.close()
    return out


def _precision(heom, workloads, stream):
    """Precision workload: depth 8 (6435 ADOs), seeds 0-1, T = 77 and 300 K,
    excitation at site 1, 5 ps, FP32-mixed and FP64, against the FP64
    oracle's trajectories: max |dp| over all populations every 10 steps, and
    |d eta| at 5 ps."""
    g = _load_golden("oracle_precision_depth8.npz")
    if g is None:
        return None
    cases = [workloads.fmo_like(seed=int(s), site=1, depth=8, T=float(T))
             for s, T in zip(g["seeds"], g["temperatures"])]
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in cases]
    r0 = [w["rho0"] for w in cases]
    out = {"workload": "fmo_like_7site_depth8_T77_300_seeds01_5ps", "n_ados": hs[0].n_ados,
           "reference": "FP64 oracle (tests/golden/oracle_precision_depth8.npz)"}
    for prec in ("fp32", "fp64"):
        rhos, sinks, _ = heom.propagate_batch(hs, r0, 1.0, 5000, record_every=10, precision=prec,
                                              stream=stream)
        dp = max(float(np.max(np.abs(np.real(np.diagonal(r, axis1=1, axis2=2)) - g["pops"][k])))
                 for k, r in enumerate(rhos))
        de = max(abs(float(sinks[k][0]) - float(g["scalars"][k][0])) for k in range(len(hs)))
        out[prec] = {"max_abs_pop_error": dp, "max_abs_eta_error": de,
                     "max_rel_eta_error": max(abs(float(sinks[k][0]) - float(g["scalars"][k][0])) /
                                              float(g["scalars"][k][0]) for k in range(len(hs))),
                     "bar": 1e-5 if prec == "fp32" else 1e-10}
    for h in hs:
        h.close()
    return out


def _alg_bytes(r):
    N = r.system["H"].shape[0]
    return comb(N + r.depth, r.depth) * r.steps * 128.0 * N * N


def _serve(heom, workloads, stream, n_requests, precision):
    """The first n_requests of the serving trace (Poisson arrivals, mean 50 ms;
    N in {2,7,8,12,24}, depth 2-4, 2-10 ps), served by the continuous-batching
    engine in real time, then the same requests one at a time (FIFO).  Every
    served result is compared with the same request served alone (bitwise)
    and with the FP64 oracle's stored result where that covers the whole run
    (FP64 1e-10 relative, FP32-mixed 1e-5 absolute on populations and eta).
    Utilisation: the offered load (algorithmic bytes of the trace per second
    of its arrival span) over the engine's measured capacity (bytes per
    second of makespan while saturated); the highest sustainable arrival
    rate is the capacity over the mean bytes of a request."""
    from paper_1012_4382_amd.serve import Engine, GpuBackend, Request

    def reqs():
        return [Request(id=w["id"], system=w["system"], depth=w["depth"], rho0=w["rho0"],
                        steps=w["steps"], arrival_s=w["arrival_s"], precision=precision)
                for w in workloads.serving_trace(n_requests)]

    def progress(tag):
        count = [0]

        def on_finish(r):
            count[0] += 1
            if count[0] % 20 == 0 or count[0] == n_requests:
                print(f"serve {tag} {precision}: {count[0]}/{n_requests} finished",
                      file=sys.stderr, flush=True)
        return on_finish

    import torch
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.9)
    eng = Engine(GpuBackend(stream=stream), hbm_budget_bytes=budget, chunk_steps=200)
    served = reqs()
    m = eng.run(served, on_finish=progress("batched"))
    fifo = Engine(GpuBackend(stream=stream), hbm_budget_bytes=budget, chunk_steps=200,
                  max_active=1)
    alone = reqs()
    mf = fifo.run(alone, on_finish=progress("fifo"))
    total_bytes = sum(_alg_bytes(r) for r in served)
    span = max(r.arrival_s for r in served)
    capacity = total_bytes / m["makespan_s"]
    offered = total_bytes / span
    # Served against alone (bitwise: the same arithmetic), every request.
    by_id = {r.id: r for r in alone}
    bitwise = all(r.status == "done" and np.array_equal(r.rho_final, by_id[r.id].rho_final) and
                  np.array_equal(r.sinks, by_id[r.id].sinks) for r in served)
    out = {"requests": n_requests, "precision": precision, "budget_bytes": budget,
           "continuous_batching": m, "fifo_one_at_a_time": mf,
           "batched_over_fifo_ado_steps_per_s": m["ado_steps_per_s"] / mf["ado_steps_per_s"],
           "offered_alg_bytes_per_s": offered, "capacity_alg_bytes_per_s": capacity,
           "utilisation": offered / capacity,
           "arrival_rate_per_s": n_requests / span,
           "highest_sustainable_arrival_rate_per_s": capacity / (total_bytes / n_requests),
           "served_equal_alone_bitwise": {"requests": len(served), "all_equal": bool(bitwise),
                                          "n_sites_24": sum(r.system["H"].shape[0] == 24
                                                            for r in served)}}
    g = _load_golden("oracle_serving.npz")
    if g is not None:
        full, dp, dt_, rel = 0, 0.0, 0.0, 0.0
        for r in served:
            j = r.id
            if j >= len(g["done"]) or not g["done"][j] or int(g["steps"][j]) != r.steps:
                continue
            N = r.system["H"].shape[0]
            ref = g["rho_flat"][g["rho_off"][j]:g["rho_off"][j + 1]].reshape(N, N)
            full += 1
            dp = max(dp, float(np.max(np.abs(np.real(np.diag(r.rho_final)) -
                                             np.real(np.diag(ref))))))
            dt_ = max(dt_, abs(float(r.sinks[0]) - float(g["scalars"][j][0])))
            rel = max(rel, float(np.max(np.abs(r.rho_final - ref)) / np.max(np.abs(ref))))
        partial = int(np.sum(g["done"][:n_requests])) - full
        out["check_vs_oracle"] = {
            "requests_full_length": full, "max_abs_pop_error": dp, "max_abs_eta_error": dt_,
            "max_rel_rho_error": rel,
            "requests_checked_over_first_steps_in_tests": partial,
            "bar": 1e-10 if precision == "fp64" else 1e-5}
    return out


def _stage_kernel_timing(heom, torch, hs, rho0s, stream, kernel, precision="fp64", steps=500):
    """Average stage-kernel duration (ms) from HIP events on the library's
    stream over a run without history records (the faster of two runs), and
    the run's ADO-steps/s."""
    ws = heom.allocate_workspace(heom.batch_workspace_bytes(hs, precision))
    heom.propagate_batch(hs, rho0s, 1.0, 20, record_every=20, workspace=ws, stream=stream,
                         want_rho=False, kernel=kernel, precision=precision)
    total_ms = float("inf")
    for _ in range(2):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        heom.propagate_batch(hs, rho0s, 1.0, steps, record_every=steps, workspace=ws,
                             stream=stream, want_rho=False, kernel=kernel, precision=precision)
        ev1.record(stream)
        ev1.synchronize()
        total_ms = min(total_ms, ev0.elapsed_time(ev1))
    ados = sum(h.n_ados for h in hs)
    return total_ms / (4 * steps), ados * steps / (total_ms * 1e-3)


def _small(heom, torch, workloads, stream, reps=5):
    """Small hierarchies, where a stage launch lasts about its launch floor:
    the dimer (15 ADOs, 1000 steps, every step recorded), a 3-site solve with a
    Matsubara term (84 ADOs), a 7-site depth-2 solve (36 ADOs), a 6-site
    depth-3 solve (84 ADOs) and an 8-site depth-2 solve (45 ADOs), both three
    packed elements x ADOs per thread on 768 threads, 5000 steps
    with records every 10, each on the default path (the resident kernel:
    every step of a chunk in one launch) and on the stage-per-launch path,
    wall clock per solve (the faster of `reps`), results compared bitwise."""
    rng = np.random.default_rng(5)
    tr, rc = workloads.fmo_sinks(N=3, trap_site=2)
    three = {"system": workloads.system(workloads.fmo_like_hamiltonian(rng, N=3), lam=60.0,
                                        gamma_inv_fs=80.0, T=150.0, K=1, trap=tr, rec=rc),
             "depth": 3, "rho0": workloads.site_state(3, 1)}
    tr6, rc6 = workloads.fmo_sinks(N=6, trap_site=6)
    six = {"system": workloads.system(workloads.fmo_like_hamiltonian(rng, N=6), trap=tr6,
                                      rec=rc6),
           "depth": 3, "rho0": workloads.site_state(6, 1)}
    tr8, rc8 = workloads.fmo_sinks(N=8, trap_site=8)
    eight = {"system": workloads.system(workloads.fmo_like_hamiltonian(rng, N=8), trap=tr8,
                                        rec=rc8),
             "depth": 2, "rho0": workloads.site_state(8, 1)}
    cases = [("dimer_depth4_1000steps_every_step", workloads.dimer(), 1000, 1),
             ("3site_k1_depth3_5000steps", three, 5000, 10),
             ("fmo_like_7site_depth2_5000steps", workloads.fmo_like(seed=0, site=1, depth=2),
              5000, 10),
             ("6site_depth3_5000steps", six, 5000, 10),
             ("8site_depth2_5000steps", eight, 5000, 10)]
    out = {}
    for name, w, steps, rec in cases:
        h = heom.Hierarchy(w["system"], w["depth"])
        ws = heom.allocate_workspace(h.workspace_bytes[heom.HEOM_FP64])
        row, res = {"n_ados": h.n_ados, "rk4_steps": steps}, {}
        for kernel in ("auto", "tiled"):
            best = float("inf")
            for _ in range(reps + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res[kernel] = heom.propagate(h, w["rho0"], 1.0, steps, record_every=rec,
                                             workspace=ws, stream=stream, kernel=kernel)[:2]
                best = min(best, time.perf_counter() - t0)
            key = "resident" if kernel == "auto" else "stage_launches"
            row[key] = {"ms_per_solve": best * 1e3, "ado_steps_per_s": h.n_ados * steps / best,
                        "us_per_step": best * 1e6 / steps}
        row["resident_over_stage_launches"] = (row["stage_launches"]["ms_per_solve"] /
                                               row["resident"]["ms_per_solve"])
        row["bitwise_equal"] = bool(np.array_equal(res["auto"][0], res["tiled"][0]) and
                                    np.array_equal(res["auto"][1], res["tiled"][1]))
        out[name] = row
        h.close()
    return out


def _sizing(heom, torch, workloads, stream, kernel):
    """The paper's largest hierarchy shape: 7 sites, depth 16 (245157 ADOs), one
    solve, FP64 and FP32-mixed; state well beyond the 256 MB Infinity Cache."""
    w = workloads.fmo_like(seed=0, site=1, depth=16, steps=200)
    h = heom.Hierarchy(w["system"], w["depth"])
    out = {"workload": "fmo_like_7site_depth16_single_solve", "n_ados": h.n_ados}
    return _sizing_rows(heom, torch, h, w, stream, kernel, out)


def _sizing_rows(heom, torch, h, w, stream, kernel, out):
    """FP64 and FP32-mixed rows of a one-solve sizing leg: ADO-steps/s and the
    stage kernel's roofline (counted traffic from the committed profiles)."""
    for prec, s in (("fp64", 8), ("fp32", 4)):
        k_ms, rate = _stage_kernel_timing(heom, torch, [h], [w["rho0"]], stream, kernel, prec,
                                          steps=100)
        name, _ = _kernel_name(heom, h.N, h.n_modes // h.N, (h.n_ados + 63) // 64, prec, kernel)
        out[prec] = {"ado_steps_per_s": rate,
                     "roofline": _roofline(f"{out['workload']}_{prec}", name, h.n_ados, h.N, s,
                                           k_ms)}
    return out


def _wide_sizing(heom, torch, workloads, stream, kernel):
    """The serving workload's largest shape: a 24-site chain or ring at depth 4
    (20475 ADOs), one solve, FP64 and FP32-mixed, on the LDS-tiled kernels
    (the autotuner's pick; for N = 24 only the 16-ADO wide kernel exists)."""
    w = next(r for r in workloads.serving_trace(200)
             if r["system"]["H"].shape[0] == 24 and r["depth"] == 4)
    h = heom.Hierarchy(w["system"], w["depth"])
    out = {"workload": f"serving_24site_{w['topology']}_depth4_single_solve",
           "n_ados": h.n_ados}
    return _sizing_rows(heom, torch, h, w, stream, kernel, out)


def _shard_sizing(heom, torch, workloads, stream, ranks=8, steps=100):
    """The paper's largest shape (7 sites, depth 16, 245157 ADOs) split over
    `ranks` contiguous ranges of its ADO order, as a multi-GPU run would place
    it, and run on this one GPU: per rank its share, its halo (ADOs of other
    ranks it links to) and the bytes an exchange of it moves per RK4 stage,
    against the bytes its own share moves; and the stage time of the split
    launch (halo copies included) against the unsplit one."""
    w = workloads.fmo_like(seed=0, site=1, depth=16, steps=steps)
    h = heom.Hierarchy(w["system"], w["depth"])
    N = h.N
    sh = heom.Shard(h, ranks)
    rows = []
    for r in range(ranks):
        inf = sh.info(r)
        local_moved = inf["n_local"] * MOVED_ADOS_PER_LAUNCH * N * N * 8
        rows.append({**inf, "halo_bytes_per_stage": inf["halo_reals"] * 8,
                     "halo_bytes_min_per_stage": inf["halo_reals_min"] * 8,
                     "halo_min_over_local_moved": inf["halo_reals_min"] * 8 / local_moved})
    ws = heom.allocate_workspace(sh.workspace_bytes)
    heom.propagate_sharded(sh, w["rho0"], 1.0, 20, record_every=20, workspace=ws, stream=stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    heom.propagate_sharded(sh, w["rho0"], 1.0, steps, record_every=steps, workspace=ws,
                           stream=stream)
    ev1.record(stream)
    ev1.synchronize()
    split_us = ev0.elapsed_time(ev1) * 1e3 / (4 * steps)
    unsplit_ms, _ = _stage_kernel_timing(heom, torch, [h], [w["rho0"]], stream, "auto", "fp64",
                                         steps=steps)
    sh.close()
    return {"workload": "fmo_like_7site_depth16_split", "n_ados": h.n_ados, "ranks": ranks,
            "rows": rows, "split_stage_us": split_us, "unsplit_stage_us": unsplit_ms * 1e3,
            "halo_copy_bytes_per_stage": sum(r["halo_bytes_min_per_stage"] for r in rows) * 2}


def _scaled_filtered(heom, torch, workloads, stream, depths=(12, 16), tols=(1e-6, 1e-8, 1e-10),
                     steps=5000):
    """The scaled hierarchy and its filter on the FMO-shaped 7-site solve
    (seed 0, site 1, 300 K) at depths 12 and 16 over 5 ps: eta and the share
    of ADOs the filter keeps (nonzero at the end of the run) per threshold,
    against the unfiltered scaled run and the plain (unscaled) run."""
    out = {"workload": "fmo_like_7site_seed0_site1_5ps", "rk4_steps": steps, "rows": []}
    for D in depths:
        w = workloads.fmo_like(seed=0, site=1, depth=D, steps=steps)
        h0 = heom.Hierarchy(w["system"], D)
        t0 = time.perf_counter()
        _, s0, _ = heom.propagate(h0, w["rho0"], 1.0, steps, record_every=steps, stream=stream)
        plain_s = time.perf_counter() - t0
        h0.close()
        row = {"depth": D, "n_ados": None, "eta_plain": float(s0[0]), "plain_seconds": plain_s,
               "filtered": []}
        for tol in (0.0,) + tuple(tols):
            h = heom.Hierarchy(w["system"], D, scaled=True, filter_tol=tol)
            row["n_ados"] = h.n_ados
            t0 = time.perf_counter()
            _, sk, ws = heom.propagate(h, w["rho0"], 1.0, steps, record_every=steps,
                                       stream=stream)
            el = time.perf_counter() - t0
            sig, _ = heom.read_state(h, ws, stream=stream)
            nz = np.max(np.abs(sig), axis=(1, 2)) > 0
            kept = int(np.sum(nz))
            multi, up, down = h.tables()
            tiers = np.sum(multi, axis=1)
            by_tier = [int(np.sum(nz[tiers == t])) for t in range(D + 1)]
            # 64-ADO tiles (in the library's order) that hold a nonzero ADO, and
            # those within 4 links of one: one RK4 step reaches 4 links, so only
            # those tiles can change in the next step.
            reach = nz.copy()
            for _ in range(4):
                nxt = reach.copy()
                for tab in (up, down):
                    src = np.nonzero(reach[:, None] & (tab >= 0))
                    nxt[tab[src]] = True
                reach = nxt
            tiles_nz = int(np.unique(np.nonzero(nz)[0] // 64).size)
            tiles_reach = int(np.unique(np.nonzero(reach)[0] // 64).size)
            # The same for the wide kernel's 16-ADO tiles.
            t16_nz = int(np.unique(np.nonzero(nz)[0] // 16).size)
            t16_reach = int(np.unique(np.nonzero(reach)[0] // 16).size)
            del sig, ws
            entry = {"filter_tol": tol, "eta": float(sk[0]),
                     "abs_eta_error_vs_plain": abs(float(sk[0]) - float(s0[0])),
                     "ados_nonzero_at_end": kept, "kept_fraction": kept / h.n_ados,
                     "nonzero_by_tier": by_tier, "tiles": (h.n_ados + 63) // 64,
                     "tiles_nonzero": tiles_nz, "tiles_within_4_links": tiles_reach,
                     "tiles16": (h.n_ados + 15) // 16, "tiles16_nonzero": t16_nz,
                     "tiles16_within_4_links": t16_reach, "seconds": el}

            row["filtered"].append(entry)
            h.close()
        out["rows"].append(row)
    return out


def _batch_scaling(heom, torch, workloads, stream, kernel, sizes=(2, 4, 8, 16, 32, 64, 128)):
    """The FMO-shaped workload with more solves per launch sequence (seeds
    0..n/2-1, sites 1 and 6): where the stage kernel leaves the latency-bound
    regime of a few hundred tiles.  Beside it, a plain 1 GiB device copy, the
    bandwidth a kernel that only streams can reach on this GPU."""
    rows = []
    for n in sizes:
        batch = workloads.fmo_like_batch(seeds=tuple(range(n // 2)), steps=200)
        hs = [heom.Hierarchy(w["system"], w["depth"]) for w in batch]
        r0 = [w["rho0"] for w in batch]
        row = {"solves": n, "n_ados": sum(h.n_ados for h in hs)}
        for prec, s in (("fp64", 8), ("fp32", 4)):
            # 500 steps, so that the capture of the run's graphs (once per call)
            # weighs little on the small launches.
            k_ms, rate = _stage_kernel_timing(heom, torch, hs, r0, stream, kernel, prec,
                                              steps=500)
            row[prec] = {"ado_steps_per_s": rate, "kernel_avg_us": k_ms * 1e3,
                         **_rates(row["n_ados"], hs[0].N, s, k_ms)}
        rows.append(row)
        for h in hs:
            h.close()
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    with torch.cuda.stream(stream):
        for _ in range(3):
            dst.copy_(src)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(20):
            dst.copy_(src)
        ev1.record(stream)
    ev1.synchronize()
    copy_gbs = 2 * src.numel() * 8 * 20 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    return {"workload": "fmo_like_7site_depth7_n_solves", "rows": rows,
            "device_copy_1GiB_GBps": copy_gbs,
            "device_copy_frac_of_hbm_peak": copy_gbs / HBM_PEAK_GBS}


def _cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        m = re.search(r"^Model name:\s*(.+)$", out, re.M)
        if m:
            return m.group(1).strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(target_s=12.0):
    """The oracle (as it stands) on this host, on a bounded sample of the
    benchmark's workload: sweep instance 2 (depth 5, 11628 ADOs, the largest
    shape of the sweep) for as many of its 1000 RK4 steps as fit in about
    target_s seconds, on every host thread and then on one thread."""
    import oracle
    from paper_1012_4382_amd import workloads

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    w = workloads.sweep_instance(2)
    n_ado = oracle.count(w["system"], w["depth"])[0]
    out = {"unit": "ADO-steps/s", "kind": "oracle", "cpu_model": _cpu_model()}
    for threads in (cores, 1):
        t0 = time.perf_counter()
        oracle.propagate(w["system"], w["depth"], w["rho0"], w["dt"], 2, record_every=2,
                         n_threads=threads)
        per_step = (time.perf_counter() - t0) / 2
        steps = int(max(2, min(w["steps"], target_s / per_step)))
        t0 = time.perf_counter()
        oracle.propagate(w["system"], w["depth"], w["rho0"], w["dt"], steps, record_every=steps,
                         n_threads=threads)
        el = time.perf_counter() - t0
        rate = n_ado * steps / el
        if threads == cores:
            out.update(value=rate, cores=cores,
                       sample=f"sweep instance 2 of the benchmark (N=7, one Matsubara term per "
                              f"bath, depth {w['depth']}, {n_ado} ADOs), first {steps} of its "
                              f"{w['steps']} RK4 steps, {el:.1f} s on {cores} OpenMP threads")
        else:
            out["one_thread"] = {"value": rate, "cores": 1,
                                 "sample": f"the same instance, first {steps} steps, {el:.1f} s "
                                           f"on 1 thread"}
    return out


def main():
    args = _parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(the propagation of one hierarchy is not sharded here)"}))
        sys.exit(2)
    import torch

    from paper_1012_4382_amd import heom, workloads

    torch.cuda.init()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)
    prec = args.precision
    steps_rk = args.rk4_steps
    record_every = 100
    cases = [workloads.sweep_instance(i) for i in range(64)]
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in cases]
    rho0s = [w["rho0"] for w in cases]
    N, KP = hs[0].N, hs[0].n_modes // hs[0].N
    total_ados = sum(h.n_ados for h in hs)
    ws = heom.allocate_workspace(heom.batch_workspace_bytes(hs, prec))

    def one_pass():
        return heom.propagate_batch(hs, rho0s, 1.0, steps_rk, record_every=record_every,
                                    precision=prec, workspace=ws, stream=stream,
                                    kernel=args.kernel)

    print(f"bench: sweep of 64 instances ({total_ados} ADOs), {steps_rk} RK4 steps, {prec}: "
          f"{args.warmup} warm-up and {args.steps} timed passes", file=sys.stderr, flush=True)
    el, kernel_ms, (rhos, sinks, _) = _timed(one_pass, stream, torch, args.steps, args.warmup,
                                             4 * steps_rk)
    value = total_ados * steps_rk * args.steps / el
    ms_per_step = 1e3 * el / args.steps
    # Population conservation of the timed runs (exact for RK4): Tr rho + P_trap + P_rec = 1.
    defect = max(abs(np.trace(r[-1]).real + s[0] + s[1] - 1.0) for r, s in zip(rhos, sinks))
    n_tiles = sum((h.n_ados + 63) // 64 for h in hs)
    kernel_name, autotune = _kernel_name(heom, N, KP, n_tiles, prec, args.kernel)
    s_bytes = 8 if prec == "fp64" else 4
    roof = _roofline(f"sweep_64x_fmo_like_7site_k1_depth3to5_{prec}", kernel_name, total_ados, N,
                     s_bytes, kernel_ms)
    roof["kernel_avg_us_note"] = ("device time of the timed passes per stage launch (HIP events "
                                  "on the library's stream), an upper bound of the kernel's "
                                  "average duration: it includes the gaps between launches "
                                  "and the sigma_0 snapshot kernels")
    result = {
        "metric": "HEOM ADO-steps/s (FP64, FP32) vs plain; serving p50/p99 latency at ≤1e-5 error",
        "value": value,
        "unit": "ADO-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"sweep_64x_fmo_like_7site_k1_depth3to5_{prec}_1000steps",
                   "instances": len(hs), "n_sites": N, "matsubara_per_bath": KP - 1,
                   "depths": [h.depth for h in hs], "n_ados_total": total_ados,
                   "rk4_steps": steps_rk, "dt_fs": 1.0, "record_every": record_every,
                   "parallelism": "single_gpu"},
        "roofline": roof,
        "population_defect": defect,
        "timed_run_check": _check_sweep(rhos, sinks, _load_golden("oracle_sweep_k1.npz"), prec),
        "autotune": autotune,
    }
    if not args.no_variants:
        # The same sweep in the other precision and one instance at a time.
        other = "fp32" if prec == "fp64" else "fp64"
        ws_o = heom.allocate_workspace(heom.batch_workspace_bytes(hs, other))
        el_o, k_o, (rh_o, sk_o, _) = _timed(
            lambda: heom.propagate_batch(hs, rho0s, 1.0, steps_rk, record_every=record_every,
                                         precision=other, workspace=ws_o, stream=stream),
            stream, torch, 2, 1, 4 * steps_rk)
        wsb = heom.allocate_workspace(max(h.workspace_bytes[heom.PRECISIONS[prec]] for h in hs))

        def one_at_a_time():
            for h, r in zip(hs, rho0s):
                heom.propagate(h, r, 1.0, steps_rk, record_every=steps_rk, workspace=wsb,
                               stream=stream, precision=prec)

        el_1, _, _ = _timed(one_at_a_time, stream, torch, 1, 0, 1)
        result["sweep_variants"] = {
            f"{other}_batched_ado_steps_per_s": total_ados * steps_rk * 2 / el_o,
            f"{other}_kernel_avg_us": k_o * 1e3,
            f"{other}_timed_run_check": _check_sweep(rh_o, sk_o,
                                                     _load_golden("oracle_sweep_k1.npz"), other),
            f"{prec}_one_at_a_time_ado_steps_per_s": total_ados * steps_rk / el_1,
            f"{prec}_batched_over_one_at_a_time": value / (total_ados * steps_rk / el_1)}
    if not args.no_fmo:
        result["fmo_batch"] = _fmo_batch(heom, torch, workloads, stream, args)
    if not args.no_small:
        result["small_hierarchies"] = _small(heom, torch, workloads, stream)
    if not args.no_sizing:
        result["hbm_sizing"] = _sizing(heom, torch, workloads, stream, args.kernel)
        result["wide_sizing"] = _wide_sizing(heom, torch, workloads, stream, args.kernel)
    if not args.no_shard:
        result["shard_sizing"] = _shard_sizing(heom, torch, workloads, stream)
    if not args.no_scaled:
        result["scaled_filtered"] = _scaled_filtered(heom, torch, workloads, stream)
    if not args.no_batch_scaling:
        result["batch_scaling"] = _batch_scaling(heom, torch, workloads, stream, args.kernel)
    if not args.no_variants:
        result["precision"] = _precision(heom, workloads, stream)
    if args.serve > 0:
        precs = ("fp64", "fp32") if args.serve_precision == "both" else (args.serve_precision,)
        result["serving"] = {p: _serve(heom, workloads, stream, args.serve, p) for p in precs}
    if args.copy_calibration:
        # A plain device copy of known size: FETCH_SIZE / WRITE_SIZE of this
        # kernel calibrate the traffic counters of the stage kernel.
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = _cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
