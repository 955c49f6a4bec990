"""The paper's FMO study on the HIP path: trapping time and efficiency against
the reorganization energy, and the thermal limit of the isolated complex.

Section "Trapping time for different reorganization energies" of the paper
scans lambda at 300 K for the Table 1 Hamiltonian, with trapping from BChl 3
and 4 (1/Gamma_RC = 2.5 ps) and radiative decay (1/Gamma_phot = 250 ps),
propagating until the population left on the sites drops below 1e-5 (t_max)
and raising the hierarchy depth until the trapping time changes by at most
0.02 ps between consecutive depths (here: for two increments in a row).  This module runs that protocol with
``heom.efficiency`` (eq:eta, eq:trappingtime); every propagation runs in the
library's kernels.  ``thermal_check`` compares the long-time populations of
the isolated complex with the Gibbs state (section on temperature).

    python -m paper_1012_4382_amd.fmo_study --lambdas 20,35,55,85,130 --sites 1,6
"""
from __future__ import annotations

import argparse
import json
import sys
from typing import Callable, Optional

import numpy as np

from . import heom, workloads

# k_B / (h c) in cm^-1 per K, from the exact SI values of k_B, h and c.
KB_CM_PER_K = 1.380649e-23 / (6.62607015e-34 * 2.99792458e10)


def converge_depth(run: Callable[[int], dict], depth0: int, tol_fs: float, max_depth: int) -> dict:
    """Raises the depth from depth0 until the trapping times of consecutive
    depths differ by at most tol_fs (the paper's criterion, 0.02 ps) for two
    increments in a row, so that a chance agreement of two shallow depths does
    not end the search.  `run` maps a depth to an efficiency result.  Returns
    the deepest result with 'depth', 'converged' and 'delta_fs' (its last
    change) added."""
    prev = run(depth0)
    depth, small = depth0, 0
    while True:
        if depth >= max_depth:
            return dict(prev, depth=depth, converged=False, delta_fs=float("nan"))
        cur = run(depth + 1)
        delta = abs(cur["mean_trap_time_fs"] - prev["mean_trap_time_fs"])
        depth += 1
        small = small + 1 if delta <= tol_fs else 0
        if small == 2:
            return dict(cur, depth=depth, converged=True, delta_fs=delta)
        prev = cur


def trapping_scan(lambdas, sites=(1, 6), gamma_inv_fs: float = 166.0, T: float = 300.0,
                  dt_fs: float = 2.5, depth0: int = 3, tol_ps: float = 0.02, max_depth: int = 14,
                  precision: str = "fp64", theta_form: int = 0, stream=None,
                  log: Optional[Callable[[dict], None]] = None) -> list:
    """Efficiency and trapping time of the Table 1 model for each (site, lambda)
    at its converged depth."""
    out = []
    for site in sites:
        for lam in lambdas:
            sys_ = workloads.fmo_table1(lam=lam, gamma_inv_fs=gamma_inv_fs, T=T,
                                        theta_form=theta_form)
            rho0 = workloads.site_state(7, site)

            def run(depth):
                h = heom.Hierarchy(sys_, depth)
                try:
                    return heom.efficiency(h, rho0, dt_fs, 0.0, 1e-5, precision=precision,
                                           stream=stream)
                finally:
                    h.close()

            r = converge_depth(run, depth0, tol_ps * 1e3, max_depth)
            row = {"site": site, "lambda_cm": lam, "gamma_inv_fs": gamma_inv_fs, "T_K": T,
                   "depth": r["depth"], "converged": r["converged"], "eta": r["eta"],
                   "trap_time_ps": r["mean_trap_time_fs"] / 1e3,
                   "delta_ps": r["delta_fs"] / 1e3, "t_max_ps": r["t_end_fs"] / 1e3,
                   "p_recomb": r["p_recomb"], "p_remaining": r["p_remaining"]}
            out.append(row)
            if log:
                log(row)
    return out


def optimum(rows, site):
    """The scanned lambda with the shortest trapping time for a start site."""
    r = min((r for r in rows if r["site"] == site), key=lambda r: r["trap_time_ps"])
    return {"site": site, "lambda_cm": r["lambda_cm"], "trap_time_ps": r["trap_time_ps"]}


def gibbs_populations(H_cm: np.ndarray, T: float) -> np.ndarray:
    """Site populations of exp(-H / k_B T) / Z."""
    E, V = np.linalg.eigh(H_cm)
    w = np.exp(-(E - E.min()) / (KB_CM_PER_K * T))
    rho = (V * (w / w.sum())) @ V.T
    return np.real(np.diag(rho))


def thermal_check(lam: float = 35.0, gamma_inv_fs: float = 166.0, T: float = 300.0,
                  depth: int = 6, t_end_fs: float = 20000.0, dt_fs: float = 2.5, site: int = 1,
                  precision: str = "fp64", stream=None) -> dict:
    """Isolated complex (no sinks) from |site><site| to t_end: final site
    populations against the Gibbs populations of the bare Hamiltonian (the
    paper's validation criterion; finite lambda shifts the true steady state,
    so this is a plausibility check, not a pin)."""
    sys_ = workloads.fmo_table1(lam=lam, gamma_inv_fs=gamma_inv_fs, T=T, sinks=False)
    h = heom.Hierarchy(sys_, depth)
    steps = int(round(t_end_fs / dt_fs))
    rho, _, _ = heom.propagate(h, workloads.site_state(7, site), dt_fs, steps,
                               record_every=steps, precision=precision, stream=stream)
    h.close()
    p = np.real(np.diag(rho[-1]))
    g = gibbs_populations(workloads.FMO_TABLE1_H, T)
    return {"lambda_cm": lam, "gamma_inv_fs": gamma_inv_fs, "T_K": T, "depth": depth,
            "t_end_ps": t_end_fs / 1e3, "populations": p.tolist(), "gibbs": g.tolist(),
            "max_abs_diff": float(np.max(np.abs(p - g))), "trace": float(np.sum(p))}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--lambdas", default="20,35,45,55,65,75,85,100,130")
    ap.add_argument("--sites", default="1,6")
    ap.add_argument("--gamma-inv", type=float, default=166.0)
    ap.add_argument("--T", type=float, default=300.0)
    ap.add_argument("--dt", type=float, default=2.5)
    ap.add_argument("--depth0", type=int, default=3)
    ap.add_argument("--max-depth", type=int, default=14)
    ap.add_argument("--tol-ps", type=float, default=0.02)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--theta-form", type=int, default=0, choices=[0, 1])
    ap.add_argument("--thermal", action="store_true", help="also run the thermal check")
    a = ap.parse_args(argv)
    lams = [float(x) for x in a.lambdas.split(",")]
    sites = [int(x) for x in a.sites.split(",")]
    rows = trapping_scan(lams, sites, a.gamma_inv, a.T, a.dt, a.depth0, a.tol_ps, a.max_depth,
                         a.precision, a.theta_form,
                         log=lambda r: print(json.dumps(r), flush=True))
    print(json.dumps({"optimum": [optimum(rows, s) for s in sites]}), flush=True)
    if a.thermal:
        print(json.dumps({"thermal": thermal_check(T=a.T, gamma_inv_fs=a.gamma_inv,
                                                   dt_fs=a.dt)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
