"""Oracle for the HEOM propagation: plain, slow, FP64, CPU only.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1012_4382_amd``) and never imports it.

Contents
  * ``heom_oracle.cpp`` -- the reference propagator (full N x N complex ADOs,
    classic RK4), built into ``libheom_oracle.so`` and wrapped here;
  * ``dense.py`` -- the same generator assembled as one dense matrix with
    Kronecker products, used to pin the C++ right-hand side;
  * ``closed_forms.py`` -- exact results the method must reproduce in special
    cases (pure dephasing, unitary limit, pure decay).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heom_oracle.cpp")
_LIB_PATH = os.environ.get("HEOM_ORACLE_LIB") or os.path.join(_HERE, "libheom_oracle.so")

# -fcx-limited-range only removes the NaN/Inf recovery branch of complex
# multiplication (results for finite operands are unchanged); no fast-math.
_CXXFLAGS = ["-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-fcx-limited-range"]


def build(force: bool = True, src: str = _SRC, out: str | None = None) -> str:
    """Compile the oracle library with g++ (in place, next to its source)."""
    out = out or _LIB_PATH
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["g++", *_CXXFLAGS, src, "-o", tmp])
        os.replace(tmp, out)
    return out


class _System(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32),
        ("hamiltonian_cm", ctypes.POINTER(ctypes.c_double)),
        ("lambda_cm", ctypes.POINTER(ctypes.c_double)),
        ("gamma_inv_fs", ctypes.POINTER(ctypes.c_double)),
        ("temperature_K", ctypes.c_double),
        ("n_matsubara", ctypes.c_int32),
        ("low_temp_correction", ctypes.c_int32),
        ("theta_form", ctypes.c_int32),
        ("trap_rate_per_ps", ctypes.POINTER(ctypes.c_double)),
        ("recomb_rate_per_ps", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        lib.oracle_count.argtypes = [P(_System), i32, P(i64), P(i32)]
        lib.oracle_modes.argtypes = [P(_System), P(i32), P(d), P(d), P(d), P(d)]
        lib.oracle_enumerate.argtypes = [P(_System), i32, P(i32)]
        lib.oracle_rhs.argtypes = [P(_System), i32, P(d), P(d), i32]
        lib.oracle_propagate.argtypes = [P(_System), i32, P(d), d, i64, i64, P(d), P(d), P(d),
                                         P(d), i32]
        lib.oracle_rhs_scaled.argtypes = [P(_System), i32, i32, P(d), P(d), i32]
        lib.oracle_propagate_scaled.argtypes = [P(_System), i32, i32, d, P(d), d, i64, i64, P(d),
                                                P(d), P(d), P(d), i32]
        for f in (lib.oracle_count, lib.oracle_modes, lib.oracle_enumerate, lib.oracle_rhs,
                  lib.oracle_propagate, lib.oracle_rhs_scaled, lib.oracle_propagate_scaled):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class System:
    """A system description in the inputs' own units (cm^-1, fs, K, 1/ps).

    ``sys`` is a mapping with keys: H (N x N complex or real, cm^-1), lam (N,),
    gamma_inv_fs (N,), T, K, ltc, theta_form, trap_per_ps (N,) or None,
    rec_per_ps (N,) or None.
    """

    def __init__(self, sys: dict):
        H = np.asarray(sys["H"], dtype=np.complex128)
        self.N = H.shape[0]
        self._H = np.ascontiguousarray(H).view(np.float64).copy()
        self._lam = np.ascontiguousarray(np.broadcast_to(np.asarray(sys["lam"], float), (self.N,)))
        self._gi = np.ascontiguousarray(
            np.broadcast_to(np.asarray(sys["gamma_inv_fs"], float), (self.N,)))
        tr = sys.get("trap_per_ps")
        rc = sys.get("rec_per_ps")
        self._trap = None if tr is None else np.ascontiguousarray(np.asarray(tr, float))
        self._rec = None if rc is None else np.ascontiguousarray(np.asarray(rc, float))
        self.K = int(sys.get("K", 0))
        self._c = _System(self.N, _dptr(self._H), _dptr(self._lam), _dptr(self._gi),
                          float(sys["T"]), self.K, int(sys.get("ltc", 1)),
                          int(sys.get("theta_form", 0)), _dptr(self._trap), _dptr(self._rec))

    @property
    def ref(self):
        return ctypes.byref(self._c)


def count(sys: dict, depth: int) -> tuple[int, int]:
    s = System(sys)
    n = ctypes.c_int64()
    m = ctypes.c_int32()
    if _load().oracle_count(s.ref, depth, ctypes.byref(n), ctypes.byref(m)) != 0:
        raise ValueError("oracle_count failed")
    return n.value, m.value


def modes(sys: dict):
    """(site, c complex, nu, delta) of the bath modes."""
    s = System(sys)
    M = s.N * (s.K + 1)
    site = np.zeros(M, np.int32)
    cr, ci, nu = np.zeros(M), np.zeros(M), np.zeros(M)
    delta = np.zeros(s.N)
    rc = _load().oracle_modes(s.ref, site.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              _dptr(cr), _dptr(ci), _dptr(nu), _dptr(delta))
    if rc != 0:
        raise ValueError("oracle_modes failed")
    return site, cr + 1j * ci, nu, delta


def enumerate_ados(sys: dict, depth: int) -> np.ndarray:
    n, M = count(sys, depth)
    out = np.zeros((n, M), np.int32)
    s = System(sys)
    if _load().oracle_enumerate(s.ref, depth, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))):
        raise ValueError("oracle_enumerate failed")
    return out


def rhs(sys: dict, depth: int, sigma: np.ndarray, scalars=(0.0, 0.0, 0.0), n_threads: int = 1,
        scaled: bool = False):
    """Right-hand side for sigma[n_ado, N, N] (oracle order) and (P_trap, P_rec, Q);
    scaled=True: sigma holds the scaled ADOs and the scaled equations apply."""
    s = System(sys)
    n_ado = sigma.shape[0]
    buf = np.concatenate([np.ascontiguousarray(sigma, np.complex128).view(np.float64).ravel(),
                          np.asarray(scalars, float)])
    out = np.zeros_like(buf)
    if _load().oracle_rhs_scaled(s.ref, depth, int(scaled), _dptr(buf), _dptr(out),
                                 n_threads) != 0:
        raise ValueError("oracle_rhs failed")
    N = s.N
    f = out[: 2 * n_ado * N * N].view(np.complex128).reshape(n_ado, N, N)
    return f, out[2 * n_ado * N * N:].copy()


def propagate(sys: dict, depth: int, rho0: np.ndarray, dt_fs: float, n_steps: int,
              record_every: int = 1, want_state: bool = False, state_in=None,
              n_threads: int | None = None, scaled: bool = False, filter_tol: float = 0.0):
    """Classic RK4 propagation.

    scaled=True propagates the scaled ADOs (the state holds them); filter_tol > 0
    zeroes, after every step, each ADO n != 0 whose entries are all below it.
    Returns dict(rho=[records, N, N], scalars=[P_trap, P_rec, Q], state=(sigma, scalars)|None).
    """
    s = System(sys)
    N = s.N
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    rho0 = np.ascontiguousarray(np.asarray(rho0, np.complex128))
    n_rec = n_steps // record_every + 1
    rho_out = np.zeros((n_rec, N, N), np.complex128)
    scal = np.zeros(3)
    state = None
    sin = None
    n_ado, _ = count(sys, depth)
    if state_in is not None:
        sig, sc = state_in
        sin = np.concatenate([np.ascontiguousarray(sig, np.complex128).view(np.float64).ravel(),
                              np.asarray(sc, float)])
    if want_state:
        state = np.zeros(2 * n_ado * N * N + 3)
    rc = _load().oracle_propagate_scaled(s.ref, depth, int(scaled), float(filter_tol),
                                         _dptr(rho0.view(np.float64)), float(dt_fs),
                                         int(n_steps), int(record_every),
                                         _dptr(rho_out.view(np.float64)), _dptr(scal),
                                         _dptr(state), _dptr(sin), int(n_threads))
    if rc != 0:
        raise ValueError("oracle_propagate failed")
    res = {"rho": rho_out, "scalars": scal, "state": None}
    if want_state:
        sig = state[: 2 * n_ado * N * N].view(np.complex128).reshape(n_ado, N, N)
        res["state"] = (sig, state[2 * n_ado * N * N:].copy())
    return res
