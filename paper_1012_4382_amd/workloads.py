"""Seeded synthetic inputs for the HEOM workloads (inputs only, no method arithmetic).

Both the GPU path and the oracle consume these dictionaries; the draws use
numpy's PCG64 generator (``numpy.random.default_rng``) in the fixed order
documented on each function.  Units are those of the inputs: cm^-1, fs, K and
1/ps.  The shapes follow the paper's own workload, the Frenkel exciton model of
the FMO complex (section "Model": 7 sites, site energies around 12200-12600
cm^-1, couplings of tens of cm^-1, identical Drude-Lorentz baths; trapping at
the reaction-centre site and radiative recombination on every site).
"""
from __future__ import annotations

import numpy as np

DIMER_H = np.array([[12410.0, -87.7], [-87.7, 12530.0]])  # BChl 1-2 block of Table 1


def system(H, lam=35.0, gamma_inv_fs=50.0, T=300.0, K=0, ltc=1, theta_form=0, trap=None,
           rec=None) -> dict:
    return dict(H=np.asarray(H), lam=lam, gamma_inv_fs=gamma_inv_fs, T=T, K=K, ltc=ltc,
                theta_form=theta_form, trap_per_ps=trap, rec_per_ps=rec)


def site_state(N: int, site: int) -> np.ndarray:
    """|site><site| with 1-based site label."""
    r = np.zeros((N, N), np.complex128)
    r[site - 1, site - 1] = 1.0
    return r


def dimer() -> dict:
    """Dimer, FP64: N=2, Table 1 block, lambda 35 cm^-1, 1/gamma 50 fs, 300 K,
    no Matsubara term, correction on, depth 4 (15 ADOs), rho0 = |1><1|, dt 1 fs,
    1000 steps, no sinks."""
    return dict(system=system(DIMER_H), depth=4, rho0=site_state(2, 1), dt=1.0, steps=1000)


# Table 1 of the paper (label tab:tab1): the FMO exciton Hamiltonian in the
# site basis, BChl 1..7, cm^-1.
FMO_TABLE1_H = np.array([
    [12410.0, -87.7, 5.5, -5.9, 6.7, -13.7, -9.9],
    [-87.7, 12530.0, 30.8, 8.2, 0.7, 11.8, 4.3],
    [5.5, 30.8, 12210.0, -53.5, -2.2, -9.6, 6.0],
    [-5.9, 8.2, -53.5, 12320.0, -70.7, -17.0, -63.3],
    [6.7, 0.7, -2.2, -70.7, 12480.0, 81.1, -1.3],
    [-13.7, 11.8, -9.6, -17.0, 81.1, 12630.0, 39.7],
    [-9.9, 4.3, 6.0, -63.3, -1.3, 39.7, 12440.0],
])


def fmo_table1(lam: float = 35.0, gamma_inv_fs: float = 166.0, T: float = 300.0,
               trap_sites=(3, 4), trap_inv_ps: float = 2.5, rec_inv_ps: float = 250.0,
               theta_form: int = 0, sinks: bool = True) -> dict:
    """The paper's FMO model (section on trapping times): Table 1 Hamiltonian,
    identical Drude-Lorentz baths (lambda, 1/gamma) at T, K = 0 with the
    correction on; trapping from BChl 3 and 4 with 1/Gamma_RC = 2.5 ps and
    radiative decay from every site with 1/Gamma_phot = 250 ps (sinks=False:
    the isolated complex)."""
    trap = rec = None
    if sinks:
        trap = np.zeros(7)
        for s in trap_sites:
            trap[s - 1] = 1.0 / trap_inv_ps
        rec = np.full(7, 1.0 / rec_inv_ps)
    return system(FMO_TABLE1_H, lam=lam, gamma_inv_fs=gamma_inv_fs, T=T, trap=trap, rec=rec,
                  theta_form=theta_form)


def fmo_like_hamiltonian(rng, N: int = 7) -> np.ndarray:
    """Draw order: site energies uniform(12200, 12600, N); then for i < j in
    row-major order J_ij = normal(0, 60) * exp(-|i - j| / 2); real symmetric."""
    eps = rng.uniform(12200.0, 12600.0, N)
    H = np.diag(eps)
    for i in range(N):
        for j in range(i + 1, N):
            H[i, j] = H[j, i] = rng.normal(0.0, 60.0) * np.exp(-abs(i - j) / 2.0)
    return H


def fmo_sinks(N: int = 7, trap_site: int = 3, trap_rate: float = 1.0, rec_rate: float = 1e-3):
    trap = np.zeros(N)
    trap[trap_site - 1] = trap_rate
    return trap, np.full(N, rec_rate)


def fmo_like(seed: int, site: int = 1, depth: int = 7, T: float = 300.0, steps: int = 5000) -> dict:
    """FMO-shaped 7-site transfer: Hamiltonian from rng(seed) as in
    fmo_like_hamiltonian; lambda 35 cm^-1, 1/gamma 50 fs, K = 0, correction on;
    trap at site 3 with 1/ps, recombination 1/ns on all sites; rho0 = |site><site|;
    dt 1 fs, `steps` steps (5 ps by default)."""
    rng = np.random.default_rng(seed)
    H = fmo_like_hamiltonian(rng)
    trap, rec = fmo_sinks()
    return dict(system=system(H, T=T, trap=trap, rec=rec), depth=depth,
                rho0=site_state(7, site), dt=1.0, steps=steps)


def fmo_like_batch(seeds=(0, 1, 2, 3), sites=(1, 6), depth: int = 7, steps: int = 5000):
    """All solves of the FMO-shaped workload: every seed with every start site."""
    return [fmo_like(s, site, depth=depth, steps=steps) for s in seeds for site in sites]


def sweep_instance(i: int) -> dict:
    """Parameter-sweep instance i: rng(1000 + i) draws, in order, the FMO-like
    Hamiltonian (7 energies, 21 couplings), lambda uniform(10, 100) cm^-1,
    1/gamma uniform(25, 200) fs, T uniform(77, 300) K, depth integers(3, 6).
    One Matsubara term per bath, correction on, sinks as fmo_like, rho0 = |1><1|,
    dt 1 fs, 1000 steps."""
    rng = np.random.default_rng(1000 + i)
    H = fmo_like_hamiltonian(rng)
    lam = rng.uniform(10.0, 100.0)
    gi = rng.uniform(25.0, 200.0)
    T = rng.uniform(77.0, 300.0)
    depth = int(rng.integers(3, 6))
    trap, rec = fmo_sinks()
    return dict(system=system(H, lam=lam, gamma_inv_fs=gi, T=T, K=1, trap=trap, rec=rec),
                depth=depth, rho0=site_state(7, 1), dt=1.0, steps=1000)


def serving_trace(n_requests: int = 200, mean_interarrival_s: float = 0.05):
    """Poisson arrivals (exponential gaps from rng(7)) and request j from
    rng(10000 + j): N from {2, 7, 8, 12, 24}; chain or ring; site energies
    normal(12400, 100); bond couplings normal(-80, 20); depth from {2, 3, 4};
    duration uniform(2, 10) ps rounded to whole fs.  lambda 35 cm^-1, 1/gamma
    50 fs, 300 K, K = 0, correction on; trap at site N (1/ps), recombination
    1/ns; rho0 = |1><1|; dt 1 fs."""
    arr_rng = np.random.default_rng(7)
    gaps = arr_rng.exponential(mean_interarrival_s, n_requests)
    arrivals = np.cumsum(gaps)
    reqs = []
    for j in range(n_requests):
        rng = np.random.default_rng(10000 + j)
        N = int(rng.choice([2, 7, 8, 12, 24]))
        topo = str(rng.choice(["chain", "ring"]))
        eps = rng.normal(12400.0, 100.0, N)
        bonds = [(i, i + 1) for i in range(N - 1)]
        if topo == "ring" and N > 2:
            bonds.append((N - 1, 0))
        J = rng.normal(-80.0, 20.0, len(bonds))
        H = np.diag(eps)
        for (a, b), v in zip(bonds, J):
            H[a, b] = H[b, a] = v
        depth = int(rng.choice([2, 3, 4]))
        duration = float(np.round(rng.uniform(2000.0, 10000.0)))
        trap, rec = fmo_sinks(N, trap_site=N)
        reqs.append(dict(id=j, arrival_s=float(arrivals[j]), topology=topo,
                         system=system(H, trap=trap, rec=rec), depth=depth,
                         rho0=site_state(N, 1), dt=1.0, steps=int(duration)))
    return reqs
