"""Throughput benchmark of the HEOM propagation on one MI355X.

One benchmark step is one pass of the whole hot path over one batch of
synthetic input: the FMO-shaped 7-site workload at hierarchy depth 7 (3432
ADOs per solve), all 8 solves (Hamiltonian seeds 0-3, excitation starting at
site 1 or site 6), each propagated 5000 RK4 steps of 1 fs (5 ps) in FP64 with
trapping and recombination sinks, as one batched launch sequence.  Inputs,
tables and parameters are on the device before the timed region starts.

Printed: one JSON line with ADO-steps/s (whole job), the roofline of the
dominant kernel (on the classic RK4 algorithmic bytes and on the bytes the
nested form moves, with the counted traffic of the committed profile), and the
oracle timed on this host on a bounded sample.  Further legs, each skippable:
single-solve and FP32-mixed rates, the depth-16 and 24-site sizing launches,
batch scaling (2-128 solves, and a plain device copy for scale), the
64-instance parameter sweep, the precision comparison, and serving.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
# Algorithmic bytes per ADO per stage launch, in packed ADOs (N*N reals).
# RK4 in its classic k1..k4 form moves 16 packed ADOs per ADO-step (4 per
# stage): that is the algorithmic figure.  The nested form this library runs
# moves 11 per step (11/4 per stage); both rates are reported.
ALG_ADOS_PER_LAUNCH = 4.0
MOVED_ADOS_PER_LAUNCH = 11.0 / 4.0


def _rates(n_ados, N, s, k_ms):
    """Bandwidth figures of a stage launch over n_ados ADOs of N sites (s bytes
    per real) that took k_ms milliseconds."""
    alg = n_ados * ALG_ADOS_PER_LAUNCH * N * N * s / (k_ms * 1e-3) / 1e9
    moved = n_ados * MOVED_ADOS_PER_LAUNCH * N * N * s / (k_ms * 1e-3) / 1e9
    return {"achieved_GBps": alg, "frac_of_hbm_peak": alg / HBM_PEAK_GBS,
            "moved_GBps": moved, "moved_frac_of_hbm_peak": moved / HBM_PEAK_GBS}
ROOT = os.path.dirname(os.path.abspath(__file__))
# rocprofv3 summary of the dominant kernel (FETCH_SIZE / WRITE_SIZE traffic),
# and the sources whose digest it records.
PROFILE = os.path.join(ROOT, "profiles", "stage_tile_7_fp64_fmo_batch.md")
KERNEL_SOURCES = ["paper_1012_4382_amd/csrc/stage_kernels.h",
                  "paper_1012_4382_amd/csrc/heom_internal.h",
                  "paper_1012_4382_amd/csrc/kernels_tile_7.hip", "paper_1012_4382_amd/build.py"]


def _kernel_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profiled_traffic(kernel: str):
    """Counted HBM bytes per launch from the committed profile, or None when
    the profile is of another kernel or of sources that have changed since."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    import re

    k = re.search(r"^- kernel: `([^`]+)`", text, re.M)
    d = re.search(r"^- source digest: `([0-9a-f]+)`", text, re.M)
    t = re.search(r"^- traffic per launch \(bytes\): (\d+)", text, re.M)
    if not (k and d and t) or k.group(1) != kernel or d.group(1) != _kernel_digest():
        return None
    return float(t.group(1))


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--rk4-steps", type=int, default=5000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-variants", action="store_true")
    p.add_argument("--kernel", default="auto", choices=["auto", "lane", "generic"],
                   help="stage kernel (lane and generic are diagnostic)")
    p.add_argument("--no-sizing", action="store_true",
                   help="skip the HBM-resident N=7, depth-16 measurement")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run a plain 256 MiB device copy (reference for traffic counters)")
    p.add_argument("--no-batch-scaling", action="store_true",
                   help="skip the 2-128 solve batches of the benchmarked workload")
    p.add_argument("--no-sweep", action="store_true",
                   help="skip the 64-instance parameter-sweep measurement")
    p.add_argument("--serve", type=int, default=40, metavar="R",
                   help="serve the first R requests of the serving trace (0: skip)")
    p.add_argument("--serve-precision", default="fp64", choices=["fp64", "fp32"],
                   help="storage precision of the served solves")
    return p.parse_args()


def _sweep(heom, torch, workloads, stream):
    """64 uneven parameter-sweep instances (one Matsubara term per bath, depth
    3-5), 1000 RK4 steps: one batched launch sequence vs one instance at a time."""
    ws_ = [workloads.sweep_instance(i) for i in range(64)]
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in ws_]
    r0 = [w["rho0"] for w in ws_]
    steps = ws_[0]["steps"]
    total = sum(h.n_ados for h in hs) * steps
    out = {"instances": len(hs), "ados_min": min(h.n_ados for h in hs),
           "ados_max": max(h.n_ados for h in hs), "rk4_steps": steps}
    for prec in ("fp64", "fp32"):
        ws = heom.allocate_workspace(heom.batch_workspace_bytes(hs, prec))
        heom.propagate_batch(hs, r0, 1.0, 50, record_every=50, precision=prec, workspace=ws,
                             stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        heom.propagate_batch(hs, r0, 1.0, steps, record_every=steps, precision=prec, workspace=ws,
                             stream=stream)
        torch.cuda.synchronize()
        out[f"{prec}_batched_ado_steps_per_s"] = total / (time.perf_counter() - t0)
    wsb = heom.allocate_workspace(max(h.workspace_bytes[heom.HEOM_FP64] for h in hs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h, r in zip(hs, r0):
        heom.propagate(h, r, 1.0, steps, record_every=steps, workspace=wsb, stream=stream)
    torch.cuda.synchronize()
    out["fp64_one_at_a_time_ado_steps_per_s"] = total / (time.perf_counter() - t0)
    out["fp64_batched_over_one_at_a_time"] = (out["fp64_batched_ado_steps_per_s"] /
                                             out["fp64_one_at_a_time_ado_steps_per_s"])
    return out


def _precision(heom, workloads, stream):
    """Precision workload: depth 8 (6435 ADOs), seeds 0-1, T = 77 and 300 K,
    excitation at site 1, 5 ps.  Reports the FP32-mixed path's deviation from
    the FP64 path (itself checked against the FP64 oracle to 1e-10 by the
    tests): max |dp| over all populations and steps, and |d eta|."""
    cases = [workloads.fmo_like(seed=s, site=1, depth=8, T=T) for s in (0, 1) for T in (77.0, 300.0)]
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in cases]
    r0 = [w["rho0"] for w in cases]
    steps = cases[0]["steps"]
    res = {}
    for prec in ("fp64", "fp32"):
        rhos, sinks, _ = heom.propagate_batch(hs, r0, 1.0, steps, record_every=10, precision=prec,
                                              stream=stream)
        res[prec] = (rhos, sinks)
    dp = max(float(np.max(np.abs(np.real(np.diagonal(a, axis1=1, axis2=2)) -
                                 np.real(np.diagonal(b, axis1=1, axis2=2)))))
             for a, b in zip(res["fp32"][0], res["fp64"][0]))
    ptrap = res["fp64"][1][:, 0]
    dtrap = np.abs(res["fp32"][1][:, 0] - ptrap)
    return {"workload": "fmo_like_7site_depth8_T77_300_seeds01_5ps", "n_ados": hs[0].n_ados,
            "max_abs_pop_error": dp, "max_abs_p_trap_error": float(np.max(dtrap)),
            "max_rel_p_trap_error": float(np.max(dtrap / ptrap)), "bar": 1e-5}


def _serve(heom, workloads, stream, n_requests, precision="fp64"):
    """The first n_requests of the serving trace (Poisson arrivals, mean 50 ms;
    N in {2,7,8,12,24}, depth 2-4, 2-10 ps), served by the continuous-batching
    engine in real time, then the same requests one at a time (FIFO).  A sample
    of the served results is checked against the same solves run alone in
    FP64 (bitwise for FP64 serving, within 1e-5 for FP32-mixed)."""
    from paper_1012_4382_amd.serve import Engine, GpuBackend, Request

    def reqs():
        return [Request(id=w["id"], system=w["system"], depth=w["depth"], rho0=w["rho0"],
                        steps=w["steps"], arrival_s=w["arrival_s"], precision=precision)
                for w in workloads.serving_trace(n_requests)]

    def progress(tag):
        count = [0]

        def on_finish(r):
            count[0] += 1
            if count[0] % 10 == 0 or count[0] == n_requests:
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
    mf = fifo.run(reqs(), on_finish=progress("fifo"))
    # Check: up to 8 served solves (of at most 2e7 ADO-steps each) against the
    # same solve alone in FP64.
    sample = [r for r in served if r.status == "done" and r.n_ados * r.steps <= 2e7][:8]
    dp, dtrap, bitwise = 0.0, 0.0, True
    for r in sample:
        h = heom.Hierarchy(r.system, r.depth)
        rho, sinks, _ = heom.propagate(h, r.rho0, r.dt, r.steps, record_every=r.steps,
                                       stream=stream)
        ref = rho[-1]
        dp = max(dp, float(np.max(np.abs(np.real(np.diag(r.rho_final)) - np.real(np.diag(ref))))))
        dtrap = max(dtrap, abs(float(r.sinks[0]) - float(sinks[0])))
        bitwise = bitwise and np.array_equal(r.rho_final, ref) and np.array_equal(r.sinks, sinks)
    return {"requests": n_requests, "precision": precision, "budget_bytes": budget,
            "continuous_batching": m, "fifo_one_at_a_time": mf,
            "check_vs_fp64_alone": {"sample": [r.id for r in sample],
                                    "max_abs_pop_error": dp, "max_abs_p_trap_error": dtrap,
                                    "bitwise_equal": bool(bitwise), "bar": 1e-5}}


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


def _sizing(heom, torch, workloads, stream, kernel):
    """The paper's largest hierarchy shape: 7 sites, depth 16 (245157 ADOs), one
    solve, FP64 and FP32-mixed; state well beyond the 256 MB Infinity Cache."""
    w = workloads.fmo_like(seed=0, site=1, depth=16, steps=200)
    h = heom.Hierarchy(w["system"], w["depth"])
    out = {"workload": "fmo_like_7site_depth16_single_solve", "n_ados": h.n_ados}
    for prec, s in (("fp64", 8), ("fp32", 4)):
        k_ms, rate = _stage_kernel_timing(heom, torch, [h], [w["rho0"]], stream, kernel, prec,
                                          steps=100)
        out[prec] = {"ado_steps_per_s": rate, "kernel_avg_us": k_ms * 1e3,
                     **_rates(h.n_ados, h.N, s, k_ms)}
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
    for prec, s in (("fp64", 8), ("fp32", 4)):
        k_ms, rate = _stage_kernel_timing(heom, torch, [h], [w["rho0"]], stream, kernel, prec,
                                          steps=100)
        out[prec] = {"ado_steps_per_s": rate, "kernel_avg_us": k_ms * 1e3,
                     **_rates(h.n_ados, h.N, s, k_ms)}
    return out


def _batch_scaling(heom, torch, workloads, stream, kernel, sizes=(2, 4, 16, 32, 64, 128)):
    """The benchmarked workload with more solves per launch sequence (seeds
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
            k_ms, rate = _stage_kernel_timing(heom, torch, hs, r0, stream, kernel, prec,
                                              steps=100)
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


def _cpu_baseline(w, target_s=12.0):
    """The oracle (as it stands) on this host, on a bounded sample of one solve."""
    import oracle

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    n_ado = oracle.count(w["system"], w["depth"])[0]
    t0 = time.perf_counter()
    oracle.propagate(w["system"], w["depth"], w["rho0"], w["dt"], 10, record_every=10,
                     n_threads=cores)
    per_step = (time.perf_counter() - t0) / 10
    steps = max(10, int(target_s / per_step))
    t0 = time.perf_counter()
    oracle.propagate(w["system"], w["depth"], w["rho0"], w["dt"], steps, record_every=steps,
                     n_threads=cores)
    el = time.perf_counter() - t0
    return {"value": n_ado * steps / el, "unit": "ADO-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"one solve of the benchmarked workload (seed 0, site 1, {n_ado} ADOs), "
                      f"first {steps} of its 5000 RK4 steps, {el:.1f} s, {cores} OpenMP threads"}


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
    steps_rk = args.rk4_steps
    batch = workloads.fmo_like_batch(steps=steps_rk)
    hs = [heom.Hierarchy(w["system"], w["depth"]) for w in batch]
    rho0s = [w["rho0"] for w in batch]
    n_ados = hs[0].n_ados
    N = hs[0].N
    total_ados = sum(h.n_ados for h in hs)
    ws = heom.allocate_workspace(heom.batch_workspace_bytes(hs, "fp64"))
    record_every = 10

    def one_pass(precision="fp64", workspace=ws, hh=hs, r0=rho0s):
        return heom.propagate_batch(hh, r0, 1.0, steps_rk, record_every=record_every,
                                    precision=precision, workspace=workspace, stream=stream,
                                    kernel=args.kernel)

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rhos, sinks, _ = one_pass()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ado_steps = total_ados * steps_rk * args.steps
    value = ado_steps / el
    ms_per_step = 1e3 * el / args.steps
    # Population conservation of the timed runs (exact for RK4): Tr rho + P_trap + P_rec = 1.
    defect = max(abs(np.trace(r[-1]).real + s[0] + s[1] - 1.0) for r, s in zip(rhos, sinks))

    # Dominant kernel: the fused RK4 stage.  Average duration per launch from
    # HIP events on the library's stream over a run without history records.
    kernel_ms, _ = _stage_kernel_timing(heom, torch, hs, rho0s, stream, args.kernel)
    # Algorithmic bytes per launch (4 packed ADOs per ADO, the classic RK4
    # figure) and the bytes the nested form moves (11/4 per ADO).
    bytes_per_launch = total_ados * ALG_ADOS_PER_LAUNCH * N * N * 8
    bytes_moved = total_ados * MOVED_ADOS_PER_LAUNCH * N * N * 8
    achieved = bytes_per_launch / (kernel_ms * 1e-3) / 1e9
    moved = bytes_moved / (kernel_ms * 1e-3) / 1e9
    # Launch shape the autotuner chose for this workload (during the warm-up).
    n_tiles = sum((h.n_ados + 63) // 64 for h in hs)
    shape, shape_us, streaming, streaming_us = heom.autotune_lookup(N, 1, n_tiles, "fp64")
    kernel_name = {"auto": f"stage_tile<{N},1,double,{max(shape, 0)}>"
                           + (" with streaming stores" if streaming == 1 else ""),
                   "lane": f"stage_fixed<{N},1,double>",
                   "generic": "stage_generic<double>"}[args.kernel]
    autotune = {"tiles": n_tiles, "shape": shape, "streaming_stores": streaming,
                "stage_us_per_shape": [round(float(u), 3) for u in shape_us],
                "stage_us_streaming": round(float(streaming_us), 3),
                "shapes": [heom.tile_shape_info(N, 1, "fp64", k)
                           for k in range(heom.tile_shape_count())]}

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fmo_like_7site_depth7_fp64_8solves_5ps", "n_sites": 7,
                   "depth": 7, "n_ados_per_solve": n_ados, "solves": len(hs),
                   "rk4_steps": steps_rk, "dt_fs": 1.0, "record_every": record_every,
                   "parallelism": "single_gpu"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": _profiled_traffic(kernel_name),
                     "kernel": kernel_name,
                     "kernel_avg_us": kernel_ms * 1e3, "bytes_per_launch": bytes_per_launch,
                     "moved": moved, "moved_frac": moved / HBM_PEAK_GBS,
                     "bytes_moved_per_launch": bytes_moved},
        "population_defect": defect,
        "autotune": autotune,
    }
    if not args.no_variants:
        # Plain single solve (one instance at a time, FP64 and FP32-mixed, each
        # after a short warm-up call) and the FP32-mixed batch.
        ws1 = heom.allocate_workspace(hs[0].workspace_bytes[heom.HEOM_FP64])
        heom.propagate(hs[0], rho0s[0], 1.0, 64, record_every=64, workspace=ws1, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        heom.propagate(hs[0], rho0s[0], 1.0, steps_rk, record_every=record_every, workspace=ws1,
                       stream=stream)
        torch.cuda.synchronize()
        plain = n_ados * steps_rk / (time.perf_counter() - t0)
        ws32 = heom.allocate_workspace(heom.batch_workspace_bytes(hs, "fp32"))
        one_pass("fp32", ws32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_pass("fp32", ws32)
        torch.cuda.synchronize()
        fp32 = total_ados * steps_rk / (time.perf_counter() - t0)
        ws1f = heom.allocate_workspace(hs[0].workspace_bytes[heom.HEOM_FP32_MIXED])
        heom.propagate(hs[0], rho0s[0], 1.0, 64, record_every=64, workspace=ws1f, stream=stream,
                       precision="fp32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        heom.propagate(hs[0], rho0s[0], 1.0, steps_rk, record_every=record_every, workspace=ws1f,
                       stream=stream, precision="fp32")
        torch.cuda.synchronize()
        plain32 = n_ados * steps_rk / (time.perf_counter() - t0)
        result["variants"] = {"fp64_single_solve_ado_steps_per_s": plain,
                              "fp32_single_solve_ado_steps_per_s": plain32,
                              "fp32_batched_over_single": fp32 / plain32,
                              "fp32_mixed_batched_ado_steps_per_s": fp32,
                              "fp64_batched_over_single": value / plain}
    if not args.no_sizing:
        result["hbm_sizing"] = _sizing(heom, torch, workloads, stream, args.kernel)
        result["wide_sizing"] = _wide_sizing(heom, torch, workloads, stream, args.kernel)
    if not args.no_batch_scaling:
        result["batch_scaling"] = _batch_scaling(heom, torch, workloads, stream, args.kernel)
    if not args.no_sweep:
        result["sweep"] = _sweep(heom, torch, workloads, stream)
    if not args.no_variants:
        result["precision"] = _precision(heom, workloads, stream)
    if args.serve > 0:
        result["serving"] = _serve(heom, workloads, stream, args.serve, args.serve_precision)
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
        result["cpu_baseline"] = _cpu_baseline(batch[0])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
