"""Exact results the HEOM must reproduce in special cases.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Pure dephasing (all inter-site couplings zero).  For a bath correlation
  C(t) = sum_k c_k exp(-nu_k t) + 2 Delta delta(t), the untruncated hierarchy
  is solved exactly by sigma_n = prod_m (i F_m)^{n_m} sigma_0 on a coherence,
  with F_m = (c_m / nu_m)(1 - exp(-nu_m t)), which gives

      rho_ab(t) = rho_ab(0) exp(-i (e_a - e_b) t - g_a(t) - conj(g_b(t))),
      g(t) = sum_k c_k / nu_k^2 (exp(-nu_k t) + nu_k t - 1) + Delta t,

  the second-order cumulant (lineshape) result; populations stay constant.
* No bath (lambda = 0): rho(t) = exp(-i H t) rho(0) exp(+i H t).
* Sinks only (no coupling, no bath): rho_aa(t) = rho_aa(0) exp(-G_a t) and
  P_trap(t) = sum_a (trap_a / G_a) rho_aa(0) (1 - exp(-G_a t)), G = trap + rec.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .dense import CM_TO_RAD_FS, bath_modes


def lineshape(sys: dict, site: int, t: np.ndarray) -> np.ndarray:
    modes, delta = bath_modes(sys)
    t = np.asarray(t, float)
    g = np.zeros_like(t, dtype=np.complex128)
    for s, c, nu in modes:
        if s != site:
            continue
        g += c / nu**2 * (np.exp(-nu * t) + nu * t - 1.0)
    return g + delta[site] * t


def pure_dephasing_coherence(sys: dict, a: int, b: int, rho_ab0: complex, t: np.ndarray):
    H = np.asarray(sys["H"], np.complex128) * CM_TO_RAD_FS
    w = (H[a, a] - H[b, b]).real
    return rho_ab0 * np.exp(-1j * w * t - lineshape(sys, a, t) - np.conj(lineshape(sys, b, t)))


def unitary(sys: dict, rho0: np.ndarray, t: float) -> np.ndarray:
    H = np.asarray(sys["H"], np.complex128) * CM_TO_RAD_FS
    U = scipy.linalg.expm(-1j * H * t)
    return U @ rho0 @ U.conj().T


def pure_decay(sys: dict, rho0: np.ndarray, t: float):
    N = rho0.shape[0]
    trap = np.zeros(N) if sys.get("trap_per_ps") is None else np.asarray(sys["trap_per_ps"]) * 1e-3
    rec = np.zeros(N) if sys.get("rec_per_ps") is None else np.asarray(sys["rec_per_ps"]) * 1e-3
    G = trap + rec
    pops = np.real(np.diag(rho0)) * np.exp(-G * t)
    with np.errstate(divide="ignore", invalid="ignore"):
        frac = np.where(G > 0, trap / np.where(G > 0, G, 1.0), 0.0)
    p_trap = float(np.sum(frac * np.real(np.diag(rho0)) * (1.0 - np.exp(-G * t))))
    return pops, p_trap
