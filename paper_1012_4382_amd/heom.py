"""Python binding of libheom.so (argument marshalling only).

Every function here forwards to the C-ABI declared in include/heom.h; all of
the propagation runs in the library's HIP kernels.  PyTorch provides device
memory (workspaces) and streams.  There is no CPU fallback: if the library is
missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# HEOM_LIB selects another build of the same library (for A/B measurements).
LIB_PATH = os.environ.get("HEOM_LIB") or os.path.join(_HERE, "libheom.so")

HEOM_OK = 0
HEOM_E_INVALID = -1
HEOM_E_NOMEM = -2
HEOM_E_DEVICE = -3
HEOM_E_NUMERIC = -4
HEOM_E_WORKSPACE = -5
HEOM_E_UNSUPPORTED = -6

HEOM_FP64 = 0
HEOM_FP32_MIXED = 1
HEOM_RESUME = 1
HEOM_GENERIC_KERNEL = 2
HEOM_LANE_KERNEL = 4
HEOM_NO_GRAPH = 8
HEOM_NO_AUTOTUNE = 16
HEOM_STREAMING_STORES = 32
HEOM_PLAIN_STORES = 64
HEOM_NO_RESIDENT = 128
# "auto": the resident kernel where a run fits it, else the LDS-tiled stage
# kernels; "tiled": the stage kernels even there; "lane" / "generic": the
# diagnostic kernels.
KERNELS = {"auto": 0, "tiled": HEOM_NO_RESIDENT, "generic": HEOM_GENERIC_KERNEL,
           "lane": HEOM_LANE_KERNEL}
STORES = {None: 0, "streaming": HEOM_STREAMING_STORES, "plain": HEOM_PLAIN_STORES}


def _warn_dt(hs, dt_fs: float):
    """Warns when dt exceeds a hierarchy's RK4 stability guide
    (heom_max_stable_dt); the library does not refuse such a step."""
    for h in hs:
        if dt_fs > h.max_stable_dt_fs:
            warnings.warn(f"dt = {dt_fs} fs exceeds the RK4 stability guide "
                          f"{h.max_stable_dt_fs:.4g} fs of a depth-{h.depth} hierarchy "
                          "(dt * max sum_m n_m nu_m > 2.5)", RuntimeWarning, stacklevel=3)
            return


def tile_shape_flag(shape: int) -> int:
    """HEOM_TILE_SHAPE(shape): forces tile launch shape `shape`."""
    return ((int(shape) + 1) & 0xF) << 8


def _flags(resume: bool, kernel: str, graphs: bool, tile_shape, autotune: bool,
           stores=None) -> int:
    f = (HEOM_RESUME if resume else 0) | KERNELS[kernel] | (0 if graphs else HEOM_NO_GRAPH)
    f |= STORES[stores]
    if tile_shape is not None:
        f |= tile_shape_flag(tile_shape)
    elif not autotune:
        f |= HEOM_NO_AUTOTUNE
    return f

PRECISIONS = {"fp64": HEOM_FP64, "fp32": HEOM_FP32_MIXED, HEOM_FP64: HEOM_FP64,
              HEOM_FP32_MIXED: HEOM_FP32_MIXED}


class HeomError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class SlotsNumericError(HeomError):
    """heom_advance_slots advanced every slot, and some results are non-finite:
    ``failed`` lists those slots; ``rhos`` and ``sinks`` hold every slot's
    outputs (the other slots are valid and may be continued)."""

    def __init__(self, where: str, message: str, rhos, sinks, failed):
        super().__init__(HEOM_E_NUMERIC, where, message)
        self.rhos, self.sinks, self.failed = rhos, sinks, failed


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


class ShardRankInfo(ctypes.Structure):
    _fields_ = [("first_ado", ctypes.c_int64), ("n_local", ctypes.c_int64),
                ("n_halo", ctypes.c_int64), ("cut_links", ctypes.c_int64),
                ("halo_reals", ctypes.c_int64), ("halo_reals_min", ctypes.c_int64)]


class EffResult(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("mean_trap_time_fs", ctypes.c_double),
                ("p_recomb", ctypes.c_double), ("p_remaining", ctypes.c_double),
                ("t_end_fs", ctypes.c_double)]


_lib = None

# (name, restype, argtypes) of every exported function.
_P = ctypes.POINTER
_d, _i32, _i64, _sz, _vp = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, \
    ctypes.c_void_p
_SIGNATURES = [
    ("heom_build_hierarchy", ctypes.c_int, [_P(_System), _i32, _P(ctypes.c_void_p)]),
    ("heom_build_hierarchy_scaled", ctypes.c_int, [_P(_System), _i32, _d, _P(ctypes.c_void_p)]),
    ("heom_hierarchy_info", ctypes.c_int, [_vp, _P(_i64), _P(_i32), _P(_sz), _P(_sz)]),
    ("heom_hierarchy_tables", ctypes.c_int, [_vp, _P(_i32), _P(_i32), _P(_i32)]),
    ("heom_hierarchy_modes", ctypes.c_int, [_vp, _P(_i32), _P(_d), _P(_d), _P(_d), _P(_d)]),
    ("heom_max_stable_dt", ctypes.c_int, [_vp, _P(_d)]),
    ("heom_propagate", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _P(_d), _d, _i64, _i64, _vp,
                                      _sz, _vp, _P(_d), _P(_d)]),
    ("heom_batch_workspace_bytes", ctypes.c_int, [_P(_vp), _i32, ctypes.c_int, _P(_sz)]),
    ("heom_propagate_batch", ctypes.c_int, [_P(_vp), _i32, ctypes.c_int, ctypes.c_int, _P(_P(_d)),
                                            _d, _i64, _i64, _vp, _sz, _vp, _P(_P(_d)),
                                            _P(_P(_d))]),
    ("heom_efficiency", ctypes.c_int, [_vp, ctypes.c_int, _P(_d), _d, _d, _d, _vp, _sz, _vp,
                                       _P(EffResult)]),
    ("heom_read_state", ctypes.c_int, [_vp, ctypes.c_int, _vp, _sz, _vp, _P(_d)]),
    ("heom_slots_scratch_bytes", ctypes.c_int, [_P(_vp), _i32, _P(_sz)]),
    ("heom_advance_slots", ctypes.c_int, [_P(_vp), _i32, ctypes.c_int, ctypes.c_int, _P(_vp),
                                          _P(_sz), _P(_i32), _P(_P(_d)), _d, _i64, _vp, _sz, _vp,
                                          _P(_P(_d)), _P(_P(_d))]),
    ("heom_advance_slots_noalloc", ctypes.c_int, [_P(_vp), _i32, ctypes.c_int, ctypes.c_int,
                                                  _P(_vp), _P(_sz), _P(_i32), _P(_P(_d)), _d,
                                                  _i64, _vp, _P(_P(_d)), _P(_P(_d))]),
    ("heom_shard_build", ctypes.c_int, [_vp, _i32, _P(ctypes.c_void_p)]),
    ("heom_shard_info", ctypes.c_int, [_vp, _i32, _P(ShardRankInfo)]),
    ("heom_shard_workspace_bytes", ctypes.c_int, [_vp, ctypes.c_int, _P(_sz)]),
    ("heom_propagate_sharded", ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _P(_d), _d, _i64,
                                              _i64, _vp, _sz, _vp, _P(_d), _P(_d)]),
    ("heom_read_state_sharded", ctypes.c_int, [_vp, ctypes.c_int, _vp, _sz, _vp, _P(_d)]),
    ("heom_shard_destroy", None, [_vp]),
    ("heom_tile_shape_count", ctypes.c_int, []),
    ("heom_tile_shape_info", ctypes.c_int, [_i32, _i32, ctypes.c_int, _i32, _P(_i32), _P(_i32),
                                            _P(_i32), _P(_i32), _P(_i32)]),
    ("heom_autotune_lookup", ctypes.c_int,
     [_i32, _i32, ctypes.c_int, _i64, _P(_i32), _P(_d), _P(_i32), _P(_d)]),
    ("heom_autotune_clear", None, []),
    ("heom_destroy", None, [_vp]),
    ("heom_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("heom_last_error", ctypes.c_char_p, []),
]


def library():
    """Loads libheom.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch's HIP runtime is loaded first, so that the library binds to
        # the same runtime instance that allocates the workspaces and streams.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1012_4382_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status: int, where: str):
    if status != HEOM_OK:
        msg = library().heom_last_error().decode()
        raise HeomError(status, where, msg)


def _dp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


class Hierarchy:
    """A built hierarchy (owns the C handle).

    ``sys`` keys: H (N x N, cm^-1, real or complex Hermitian), lam (cm^-1, scalar
    or (N,)), gamma_inv_fs (fs, scalar or (N,)), T (K), K (Matsubara terms),
    ltc (0/1), theta_form (0/1), trap_per_ps and rec_per_ps ((N,) or None).
    scaled=True builds the scaled hierarchy (heom_build_hierarchy_scaled), with
    the filter threshold filter_tol (0: no filter).
    """

    def __init__(self, sys: dict, depth: int, scaled: bool = False, filter_tol: float = 0.0):
        H = np.ascontiguousarray(np.asarray(sys["H"], np.complex128))
        N = H.shape[0]
        self.N = N
        self.depth = int(depth)
        keep = {
            "H": H.view(np.float64).copy(),
            "lam": np.ascontiguousarray(np.broadcast_to(np.asarray(sys["lam"], float), (N,))),
            "gi": np.ascontiguousarray(np.broadcast_to(np.asarray(sys["gamma_inv_fs"], float),
                                                       (N,))),
            "tr": None if sys.get("trap_per_ps") is None else
            np.ascontiguousarray(np.asarray(sys["trap_per_ps"], float)),
            "rc": None if sys.get("rec_per_ps") is None else
            np.ascontiguousarray(np.asarray(sys["rec_per_ps"], float)),
        }
        cs = _System(N, _dp(keep["H"]), _dp(keep["lam"]), _dp(keep["gi"]), float(sys["T"]),
                     int(sys.get("K", 0)), int(sys.get("ltc", 1)), int(sys.get("theta_form", 0)),
                     _dp(keep["tr"]), _dp(keep["rc"]))
        h = ctypes.c_void_p()
        self.scaled, self.filter_tol = bool(scaled), float(filter_tol)
        if self.scaled:
            _check(library().heom_build_hierarchy_scaled(ctypes.byref(cs), self.depth,
                                                         self.filter_tol, ctypes.byref(h)),
                   "heom_build_hierarchy_scaled")
        else:
            _check(library().heom_build_hierarchy(ctypes.byref(cs), self.depth, ctypes.byref(h)),
                   "heom_build_hierarchy")
        self._h = h
        n, m, b64, b32 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(library().heom_hierarchy_info(h, ctypes.byref(n), ctypes.byref(m),
                                             ctypes.byref(b64), ctypes.byref(b32)),
               "heom_hierarchy_info")
        self.n_ados = n.value
        self.n_modes = m.value
        self.workspace_bytes = {HEOM_FP64: b64.value, HEOM_FP32_MIXED: b32.value}
        dt = ctypes.c_double()
        _check(library().heom_max_stable_dt(h, ctypes.byref(dt)), "heom_max_stable_dt")
        self.max_stable_dt_fs = dt.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            library().heom_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tables(self):
        """(multi [n_ados, M], up [n_ados, M], down [n_ados, M]) in library order."""
        shape = (self.n_ados, self.n_modes)
        multi, up, down = (np.zeros(shape, np.int32) for _ in range(3))
        ip = ctypes.POINTER(ctypes.c_int32)
        _check(library().heom_hierarchy_tables(self._h, multi.ctypes.data_as(ip),
                                               up.ctypes.data_as(ip), down.ctypes.data_as(ip)),
               "heom_hierarchy_tables")
        return multi, up, down

    def modes(self):
        """(site, c complex, nu, delta)."""
        M = self.n_modes
        site = np.zeros(M, np.int32)
        cr, ci, nu = np.zeros(M), np.zeros(M), np.zeros(M)
        delta = np.zeros(self.N)
        _check(library().heom_hierarchy_modes(
            self._h, site.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(cr), _dp(ci),
            _dp(nu), _dp(delta)), "heom_hierarchy_modes")
        return site, cr + 1j * ci, nu, delta


def allocate_workspace(nbytes: int, device=None):
    """A torch uint8 tensor on the GPU of at least nbytes (256-byte aligned)."""
    import torch

    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-t.data_ptr()) % 256
    return t[off:off + int(nbytes)]


def _ws_args(ws):
    if ws is None:
        return None, 0
    return ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


def propagate(h: Hierarchy, rho0, dt_fs: float, n_steps: int, record_every: int = 1,
              precision="fp64", workspace=None, stream=None, resume: bool = False,
              kernel: str = "auto", want_rho: bool = True, graphs: bool = True,
              tile_shape=None, autotune: bool = True, stores=None):
    """Runs heom_propagate (kernel: "auto", or the diagnostic "lane" / "generic";
    tile_shape forces a tile launch shape, autotune=False uses shape 0; stores
    "streaming" / "plain" forces the tile kernels' store policy).
    Returns (rho [records, N, N] complex | None, sinks [3], workspace)."""
    _warn_dt([h], dt_fs)
    prec = PRECISIONS[precision]
    if workspace is None:
        workspace = allocate_workspace(h.workspace_bytes[prec])
    ptr, nbytes = _ws_args(workspace)
    flags = _flags(resume, kernel, graphs, tile_shape, autotune, stores)
    r0 = None
    if rho0 is not None:
        r0 = np.ascontiguousarray(np.asarray(rho0, np.complex128)).view(np.float64)
    n_rec = n_steps // record_every + 1
    rho = np.zeros((n_rec, h.N, h.N), np.complex128) if want_rho else None
    sinks = np.zeros(3)
    _check(library().heom_propagate(h.handle, prec, flags, _dp(r0), float(dt_fs), int(n_steps),
                                    int(record_every), ptr, nbytes, _stream_handle(stream),
                                    _dp(None if rho is None else rho.view(np.float64)),
                                    _dp(sinks)), "heom_propagate")
    return rho, sinks, workspace


def batch_workspace_bytes(hs, precision="fp64") -> int:
    arr = (ctypes.c_void_p * len(hs))(*[h.handle.value for h in hs])
    out = ctypes.c_size_t()
    _check(library().heom_batch_workspace_bytes(arr, len(hs), PRECISIONS[precision],
                                                ctypes.byref(out)), "heom_batch_workspace_bytes")
    return out.value


def propagate_batch(hs, rho0s, dt_fs: float, n_steps: int, record_every: int = 1,
                    precision="fp64", workspace=None, stream=None, resume: bool = False,
                    kernel: str = "auto", want_rho: bool = True, graphs: bool = True,
                    tile_shape=None, autotune: bool = True, stores=None):
    """Runs heom_propagate_batch.  Returns (list of rho | None, sinks [n, 3], workspace)."""
    _warn_dt(hs, dt_fs)
    n = len(hs)
    prec = PRECISIONS[precision]
    if workspace is None:
        workspace = allocate_workspace(batch_workspace_bytes(hs, precision))
    ptr, nbytes = _ws_args(workspace)
    flags = _flags(resume, kernel, graphs, tile_shape, autotune, stores)
    DP = ctypes.POINTER(ctypes.c_double)
    keep = []
    r0 = (DP * n)()
    for k in range(n):
        if rho0s is not None and rho0s[k] is not None:
            a = np.ascontiguousarray(np.asarray(rho0s[k], np.complex128)).view(np.float64)
            keep.append(a)
            r0[k] = _dp(a)
    n_rec = n_steps // record_every + 1
    rhos = [np.zeros((n_rec, h.N, h.N), np.complex128) for h in hs] if want_rho else None
    sinks = np.zeros((n, 3))
    ro = (DP * n)()
    so = (DP * n)()
    for k in range(n):
        if rhos is not None:
            ro[k] = _dp(rhos[k].view(np.float64))
        so[k] = sinks[k].ctypes.data_as(DP)
    arr = (ctypes.c_void_p * n)(*[h.handle.value for h in hs])
    _check(library().heom_propagate_batch(arr, n, prec, flags, r0, float(dt_fs), int(n_steps),
                                          int(record_every), ptr, nbytes, _stream_handle(stream),
                                          ro, so), "heom_propagate_batch")
    return rhos, sinks, workspace


def efficiency(h: Hierarchy, rho0, dt_fs: float, t_end_fs: float, pop_tol: float = 1e-5,
               precision="fp64", workspace=None, stream=None) -> dict:
    _warn_dt([h], dt_fs)
    prec = PRECISIONS[precision]
    if workspace is None:
        workspace = allocate_workspace(h.workspace_bytes[prec])
    ptr, nbytes = _ws_args(workspace)
    r0 = np.ascontiguousarray(np.asarray(rho0, np.complex128)).view(np.float64)
    out = EffResult()
    _check(library().heom_efficiency(h.handle, prec, _dp(r0), float(dt_fs), float(t_end_fs),
                                     float(pop_tol), ptr, nbytes, _stream_handle(stream),
                                     ctypes.byref(out)), "heom_efficiency")
    return {f: getattr(out, f) for f, _ in EffResult._fields_}


def read_state(h: Hierarchy, workspace, precision="fp64", stream=None):
    """(sigma [n_ados, N, N] complex in library order, scalars [3])."""
    ptr, nbytes = _ws_args(workspace)
    buf = np.zeros(2 * h.n_ados * h.N * h.N + 3)
    _check(library().heom_read_state(h.handle, PRECISIONS[precision], ptr, nbytes,
                                     _stream_handle(stream), _dp(buf)), "heom_read_state")
    sig = buf[: 2 * h.n_ados * h.N * h.N].view(np.complex128).reshape(h.n_ados, h.N, h.N)
    return sig, buf[2 * h.n_ados * h.N * h.N:].copy()


def slots_scratch_bytes(hs) -> int:
    arr = (ctypes.c_void_p * len(hs))(*[h.handle.value for h in hs])
    out = ctypes.c_size_t()
    _check(library().heom_slots_scratch_bytes(arr, len(hs), ctypes.byref(out)),
           "heom_slots_scratch_bytes")
    return out.value


def _slots_call(hs, workspaces, start, rho0s, want_rho):
    """Marshalled arguments of heom_advance_slots(_noalloc) and its output arrays."""
    n = len(hs)
    DP = ctypes.POINTER(ctypes.c_double)
    a = {"arr": (ctypes.c_void_p * n)(*[h.handle.value for h in hs]),
         "wsp": (ctypes.c_void_p * n)(*[w.data_ptr() for w in workspaces]),
         "wsb": (ctypes.c_size_t * n)(*[w.numel() * w.element_size() for w in workspaces]),
         "st": (ctypes.c_int32 * n)(*[1 if s else 0 for s in start]),
         "r0": (DP * n)(), "ro": (DP * n)(), "so": (DP * n)(), "keep": []}
    for k in range(n):
        if rho0s is not None and rho0s[k] is not None:
            r = np.ascontiguousarray(np.asarray(rho0s[k], np.complex128)).view(np.float64)
            a["keep"].append(r)
            a["r0"][k] = _dp(r)
    rhos = [np.zeros((h.N, h.N), np.complex128) for h in hs] if want_rho else None
    sinks = np.zeros((n, 3))
    for k in range(n):
        if rhos is not None:
            a["ro"][k] = _dp(rhos[k].view(np.float64))
        a["so"][k] = sinks[k].ctypes.data_as(DP)
    return a, rhos, sinks


def _slots_status(status, where, rhos, sinks):
    if status == HEOM_E_NUMERIC:
        failed = [k for k in range(len(sinks)) if not np.all(np.isfinite(sinks[k])) or
                  (rhos is not None and not np.all(np.isfinite(rhos[k])))]
        raise SlotsNumericError(where, library().heom_last_error().decode(), rhos, sinks, failed)
    _check(status, where)


def advance_slots(hs, workspaces, start, rho0s, dt_fs: float, n_steps: int, scratch,
                  precision="fp64", stream=None, kernel: str = "auto", graphs: bool = True,
                  want_rho: bool = True, tile_shape=None, autotune: bool = True,
                  stores=None):
    """Runs heom_advance_slots.  Returns (list of final rho [N, N] | None, sinks [n, 3]).
    Raises SlotsNumericError when some slots' results are non-finite (every
    slot was advanced), HeomError on any other failure."""
    _warn_dt(hs, dt_fs)
    a, rhos, sinks = _slots_call(hs, workspaces, start, rho0s, want_rho)
    sptr, sbytes = _ws_args(scratch)
    flags = _flags(False, kernel, graphs, tile_shape, autotune, stores)
    status = library().heom_advance_slots(a["arr"], len(hs), PRECISIONS[precision], flags,
                                          a["wsp"], a["wsb"], a["st"], a["r0"], float(dt_fs),
                                          int(n_steps), sptr, sbytes, _stream_handle(stream),
                                          a["ro"], a["so"])
    _slots_status(status, "heom_advance_slots", rhos, sinks)
    return rhos, sinks


def advance_slots_noalloc(hs, workspaces, start, rho0s, dt_fs: float, n_steps: int,
                          precision="fp64", stream=None, kernel: str = "auto",
                          want_rho: bool = True, tile_shape=None, autotune: bool = True,
                          stores=None):
    """Runs heom_advance_slots_noalloc (no scratch argument; nothing is
    allocated on the device).  Returns and raises as advance_slots."""
    _warn_dt(hs, dt_fs)
    a, rhos, sinks = _slots_call(hs, workspaces, start, rho0s, want_rho)
    flags = _flags(False, kernel, True, tile_shape, autotune, stores)
    status = library().heom_advance_slots_noalloc(a["arr"], len(hs), PRECISIONS[precision],
                                                  flags, a["wsp"], a["wsb"], a["st"], a["r0"],
                                                  float(dt_fs), int(n_steps),
                                                  _stream_handle(stream), a["ro"], a["so"])
    _slots_status(status, "heom_advance_slots_noalloc", rhos, sinks)
    return rhos, sinks


class Shard:
    """A hierarchy split over n_ranks ranks (heom_shard_build); owns the handle."""

    def __init__(self, h: Hierarchy, n_ranks: int):
        s = ctypes.c_void_p()
        _check(library().heom_shard_build(h.handle, int(n_ranks), ctypes.byref(s)),
               "heom_shard_build")
        self._s = s
        self.h = h
        self.n_ranks = int(n_ranks)
        b = ctypes.c_size_t()
        _check(library().heom_shard_workspace_bytes(s, HEOM_FP64, ctypes.byref(b)),
               "heom_shard_workspace_bytes")
        self.workspace_bytes = b.value

    @property
    def handle(self):
        return self._s

    def info(self, rank: int) -> dict:
        out = ShardRankInfo()
        _check(library().heom_shard_info(self._s, int(rank), ctypes.byref(out)),
               "heom_shard_info")
        return {f: getattr(out, f) for f, _ in ShardRankInfo._fields_}

    def close(self):
        if getattr(self, "_s", None):
            library().heom_shard_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def propagate_sharded(s: Shard, rho0, dt_fs: float, n_steps: int, record_every: int = 1,
                      workspace=None, stream=None, resume: bool = False, kernel: str = "auto",
                      graphs: bool = True, tile_shape=None, autotune: bool = True, stores=None):
    """Runs heom_propagate_sharded (FP64).  Returns (rho [records, N, N], sinks [3], workspace)."""
    _warn_dt([s.h], dt_fs)
    if workspace is None:
        workspace = allocate_workspace(s.workspace_bytes)
    ptr, nbytes = _ws_args(workspace)
    flags = _flags(resume, kernel, graphs, tile_shape, autotune, stores)
    r0 = None
    if rho0 is not None:
        r0 = np.ascontiguousarray(np.asarray(rho0, np.complex128)).view(np.float64)
    N = s.h.N
    rho = np.zeros((n_steps // record_every + 1, N, N), np.complex128)
    sinks = np.zeros(3)
    _check(library().heom_propagate_sharded(s.handle, HEOM_FP64, flags, _dp(r0), float(dt_fs),
                                            int(n_steps), int(record_every), ptr, nbytes,
                                            _stream_handle(stream), _dp(rho.view(np.float64)),
                                            _dp(sinks)), "heom_propagate_sharded")
    return rho, sinks, workspace


def read_state_sharded(s: Shard, workspace, stream=None):
    """(sigma [n_ados, N, N] complex in the hierarchy's order, scalars [3])."""
    ptr, nbytes = _ws_args(workspace)
    h = s.h
    buf = np.zeros(2 * h.n_ados * h.N * h.N + 3)
    _check(library().heom_read_state_sharded(s.handle, HEOM_FP64, ptr, nbytes,
                                             _stream_handle(stream), _dp(buf)),
           "heom_read_state_sharded")
    sig = buf[: 2 * h.n_ados * h.N * h.N].view(np.complex128).reshape(h.n_ados, h.N, h.N)
    return sig, buf[2 * h.n_ados * h.N * h.N:].copy()


def tile_shape_count() -> int:
    return int(library().heom_tile_shape_count())


def tile_shape_info(n_sites: int, modes_per_site: int, precision="fp64", shape: int = 0):
    """(ADOs per workgroup, threads per workgroup, elements per wave, load
    chunk, minimum waves per SIMD) of a launch shape, or None if that shape is
    not built for n_sites."""
    a, t, e, c, w = (ctypes.c_int32() for _ in range(5))
    st = library().heom_tile_shape_info(int(n_sites), int(modes_per_site), PRECISIONS[precision],
                                        int(shape), ctypes.byref(a), ctypes.byref(t),
                                        ctypes.byref(e), ctypes.byref(c), ctypes.byref(w))
    if st == HEOM_E_UNSUPPORTED:
        return None
    _check(st, "heom_tile_shape_info")
    return a.value, t.value, e.value, c.value, w.value


def autotune_lookup(n_sites: int, modes_per_site: int, n_tiles: int, precision="fp64"):
    """(tuned shape or -1, microseconds per stage launch of each shape with
    plain stores, -1 where not timed, streaming stores chosen (1 / 0, -1 if
    not tuned), microseconds of the tuned shape with streaming stores) for
    the current device."""
    shape, streaming = ctypes.c_int32(), ctypes.c_int32()
    us, us_streaming = np.full(tile_shape_count(), -1.0), ctypes.c_double()
    _check(library().heom_autotune_lookup(int(n_sites), int(modes_per_site),
                                          PRECISIONS[precision], int(n_tiles),
                                          ctypes.byref(shape), _dp(us), ctypes.byref(streaming),
                                          ctypes.byref(us_streaming)), "heom_autotune_lookup")
    return shape.value, us, streaming.value, us_streaming.value


def autotune_clear():
    library().heom_autotune_clear()
