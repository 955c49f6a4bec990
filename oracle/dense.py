"""Dense-matrix form of the HEOM generator, for pinning the C++ oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The generator of eq:lab8 (paper, Appendix A) is linear and time independent, so
on a tiny hierarchy it can be written as one matrix L acting on the stacked,
row-major vectorised ADOs plus the three scalars (P_trap, P_rec, Q).  Here it is
assembled from superoperators with Kronecker products, which is an independent
formulation of the same equation:

    vec(A X B) = (A kron B^T) vec(X)      (row-major vec)
    V^x  -> V kron I - I kron V^T,        V^o -> V kron I + I kron V^T.

Bath coefficients are recomputed here from the inputs (Drude-Lorentz spectral
density, eq:gamma; Matsubara expansion; low-temperature residual), and the
hierarchy neighbours are looked up in a dictionary keyed by multi-index.
"""
from __future__ import annotations

import math

import numpy as np

CM_TO_RAD_FS = 2.0 * math.pi * 2.99792458e10 * 1e-15
KB_CM_PER_K = 1.380649e-23 / (6.62607015e-34 * 2.99792458e10)


def bath_modes(sys: dict):
    """Modes (site, c, nu) and residual Delta per site, recomputed in Python."""
    N = np.asarray(sys["H"]).shape[0]
    K = int(sys.get("K", 0))
    lam = np.broadcast_to(np.asarray(sys["lam"], float), (N,)) * CM_TO_RAD_FS
    gam = 1.0 / np.broadcast_to(np.asarray(sys["gamma_inv_fs"], float), (N,))
    kT = KB_CM_PER_K * float(sys["T"]) * CM_TO_RAD_FS
    form = int(sys.get("theta_form", 0))
    modes = []
    delta = np.zeros(N)
    for s in range(N):
        cot = math.cos(gam[s] / (2 * kT)) / math.sin(gam[s] / (2 * kT))
        if form == 0:
            c0 = lam[s] * gam[s] * complex(cot, -1.0)
        else:
            c0 = complex(2 * lam[s] * kT, -lam[s] * gam[s])
        modes.append((s, c0, gam[s]))
        tail = 0.0
        for k in range(1, K + 1):
            nu = 2 * math.pi * k * kT
            ck = 4 * lam[s] * gam[s] * kT * nu / (nu * nu - gam[s] ** 2)
            modes.append((s, complex(ck, 0.0), nu))
            tail += ck / nu
        if int(sys.get("ltc", 1)):
            delta[s] = 2 * lam[s] * kT / gam[s] - lam[s] * cot - tail
    return modes, delta


def generator(sys: dict, multi: np.ndarray) -> np.ndarray:
    """Dense L for the hierarchy listed in ``multi`` (rows = multi-indices).

    Vector layout: ADO blocks of N*N (row-major) in the order of ``multi``, then
    P_trap, P_rec, Q.
    """
    H = np.asarray(sys["H"], np.complex128) * CM_TO_RAD_FS
    N = H.shape[0]
    trap = np.zeros(N) if sys.get("trap_per_ps") is None else np.asarray(sys["trap_per_ps"]) * 1e-3
    rec = np.zeros(N) if sys.get("rec_per_ps") is None else np.asarray(sys["rec_per_ps"]) * 1e-3
    modes, delta = bath_modes(sys)
    n_ado = multi.shape[0]
    N2 = N * N
    dim = n_ado * N2 + 3
    L = np.zeros((dim, dim), np.complex128)
    I = np.eye(N)
    Heff = H - 0.5j * np.diag(trap + rec)

    def left(A):  # X -> A X
        return np.kron(A, I)

    def right(B):  # X -> X B
        return np.kron(I, B.T)

    def proj(s):
        V = np.zeros((N, N))
        V[s, s] = 1.0
        return V

    comm = [left(proj(s)) - right(proj(s)) for s in range(N)]
    coherent = -1j * (left(Heff) - right(Heff.conj().T))
    index = {tuple(int(v) for v in row): i for i, row in enumerate(multi)}
    for i, row in enumerate(multi):
        n = tuple(int(v) for v in row)
        blk = slice(i * N2, (i + 1) * N2)
        damp = sum(n[m] * modes[m][2] for m in range(len(modes)))
        diag = coherent - damp * np.eye(N2)
        for s in range(N):
            diag = diag - delta[s] * (comm[s] @ comm[s])
        L[blk, blk] += diag
        for m, (s, c, _nu) in enumerate(modes):
            up = list(n)
            up[m] += 1
            j = index.get(tuple(up))
            if j is not None:
                L[blk, j * N2:(j + 1) * N2] += 1j * comm[s]
            if n[m] > 0:
                dn = list(n)
                dn[m] -= 1
                j = index[tuple(dn)]
                V = proj(s)
                L[blk, j * N2:(j + 1) * N2] += n[m] * 1j * (c * left(V) - np.conj(c) * right(V))
    # Scalars: dP_trap/dt = sum_s trap_s Re(rho_ss); dP_rec similarly; dQ/dt = P_trap.
    # Re(rho_ss) of a Hermitian rho equals rho_ss; the operator is applied to the
    # complex vector, so the real part is taken by the caller's check of
    # Hermitian states (the test states used with the scalars are Hermitian).
    i0 = index[tuple([0] * multi.shape[1])]
    for s in range(N):
        L[n_ado * N2 + 0, i0 * N2 + s * N + s] = trap[s]
        L[n_ado * N2 + 1, i0 * N2 + s * N + s] = rec[s]
    L[n_ado * N2 + 2, n_ado * N2 + 0] = 1.0
    return L


def rk4_polynomial(L: np.ndarray, dt: float) -> np.ndarray:
    """For a constant generator one classic RK4 step is exactly sum_k (dt L)^k / k!, k <= 4."""
    A = dt * L
    P = np.eye(L.shape[0], dtype=np.complex128)
    term = np.eye(L.shape[0], dtype=np.complex128)
    for k in range(1, 5):
        term = term @ A / k
        P = P + term
    return P
