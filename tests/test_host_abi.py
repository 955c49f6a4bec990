"""Host-side checks of libheom.so through its C-ABI (no GPU needed).

The library loads without a GPU; everything here runs on the host: the
exported symbols, hierarchy enumeration and neighbour tables, bath
coefficients, and the argument validation of every entry point.  Expected
values come from the oracle (independent enumeration and coefficients) or from
the definitions.
"""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_1012_4382_amd import heom, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "heom.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(heom_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = heom.library()
    names = _declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    # The binding wraps each of them under the same name.
    wrapped = {n for n, _, _ in heom._SIGNATURES}
    assert set(names) == wrapped


def test_status_strings():
    lib = heom.library()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.heom_status_string(code).decode() not in ("", "unknown status")
    assert lib.heom_status_string(-99).decode() == "unknown status"


@pytest.mark.parametrize("N,K,D", [(2, 0, 4), (7, 0, 3), (3, 1, 4), (2, 2, 6), (4, 0, 0)])
def test_tables_match_oracle_enumeration(N, K, D):
    rng = np.random.default_rng(N + 10 * K + D)
    H = np.diag(rng.uniform(12200, 12600, N))
    sys = workloads.system(H, K=K)
    h = heom.Hierarchy(sys, D)
    multi, up, down = h.tables()
    M = N * (K + 1)
    assert (h.n_ados, h.n_modes) == (math.comb(M + D, D), M)
    ref = oracle.enumerate_ados(sys, D)
    assert {tuple(r) for r in multi} == {tuple(r) for r in ref}
    index = {tuple(r): i for i, r in enumerate(multi)}
    # Lexicographic order, last mode fastest.
    assert [tuple(r) for r in multi] == sorted(tuple(r) for r in multi)
    for i, n in enumerate(multi):
        for m in range(M):
            e = np.zeros(M, np.int32)
            e[m] = 1
            want_up = index.get(tuple(n + e), -1)
            want_dn = index.get(tuple(n - e), -1) if n[m] > 0 else -1
            assert up[i, m] == want_up and down[i, m] == want_dn
            if up[i, m] >= 0:
                assert down[up[i, m], m] == i


def test_paper_ado_counts_through_library():
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "paper_ado_counts.txt"), dtype=np.int64)
    for M, D, n in rows:
        h = heom.Hierarchy(workloads.system(np.eye(int(M)) * 12400.0), int(D))
        assert h.n_ados == n


@pytest.mark.parametrize("T,K,form", [(300.0, 0, 0), (77.0, 1, 0), (150.0, 3, 1), (300.0, 1, 1)])
def test_modes_match_oracle(T, K, form):
    rng = np.random.default_rng(3)
    N = 3
    sys = workloads.system(np.diag([12400.0, 12300.0, 12200.0]),
                           lam=rng.uniform(10, 100, N), gamma_inv_fs=rng.uniform(25, 200, N), T=T,
                           K=K, theta_form=form)
    h = heom.Hierarchy(sys, 1)
    s1, c1, nu1, d1 = h.modes()
    s2, c2, nu2, d2 = oracle.modes(sys)
    assert np.array_equal(s1, s2)
    assert np.allclose(c1, c2, rtol=1e-13, atol=0)
    assert np.allclose(nu1, nu2, rtol=1e-14, atol=0)
    assert np.allclose(d1, d2, rtol=1e-12, atol=1e-20)


def _expect(status, fn, *args, **kw):
    with pytest.raises(heom.HeomError) as ei:
        fn(*args, **kw)
    assert ei.value.status == status, str(ei.value)


def test_build_validation_errors():
    H = workloads.DIMER_H
    ok = workloads.system(H)
    heom.Hierarchy(ok, 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, H=np.array([[1.0, 2.0], [3.0, 1.0]])), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, H=np.array([[np.nan, 0], [0, 1.0]])), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, lam=-1.0), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, lam=np.nan), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, gamma_inv_fs=0.0), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, T=0.0), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, K=-1), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, theta_form=2), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, dict(ok, trap_per_ps=np.array([-1.0, 0.0])), 2)
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, ok, -1)
    # Too many ADOs for int32 indices: 64 modes at depth 12 -> C(76, 12) > 2^31.
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy, workloads.system(np.eye(64) * 12400.0), 12)
    # A Matsubara frequency equal to gamma: nu_1 = 2 pi kT = gamma.
    kT = 0.6950348004861274 * 300.0 * 2 * math.pi * 2.99792458e-5
    _expect(heom.HEOM_E_INVALID, heom.Hierarchy,
            dict(ok, K=1, gamma_inv_fs=1.0 / (2 * math.pi * kT)), 1)
    assert "Matsubara" in heom.library().heom_last_error().decode()


def test_propagate_validation_errors_need_no_device():
    h = heom.Hierarchy(workloads.system(workloads.DIMER_H), 2)
    rho0 = workloads.site_state(2, 1)
    lib = heom.library()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    r0 = np.ascontiguousarray(rho0).view(np.float64)
    P = heom._dp

    def call(prec=0, flags=0, dt=1.0, steps=10, rec=1, ws=fake, nbytes=1 << 30, rho=r0):
        return lib.heom_propagate(h.handle, prec, flags, P(rho), dt, steps, rec, ws, nbytes, None,
                                  None, None)

    assert call(prec=7) == heom.HEOM_E_UNSUPPORTED
    assert call(flags=1 << 13) == heom.HEOM_E_INVALID  # unknown flag
    assert call(flags=heom.HEOM_STREAMING_STORES | heom.HEOM_PLAIN_STORES) == heom.HEOM_E_INVALID
    assert call(dt=0.0) == heom.HEOM_E_INVALID
    assert call(dt=float("nan")) == heom.HEOM_E_INVALID
    assert call(steps=-1) == heom.HEOM_E_INVALID
    assert call(rec=0) == heom.HEOM_E_INVALID
    assert call(ws=None) == heom.HEOM_E_WORKSPACE
    assert call(ws=ctypes.c_void_p((1 << 20) + 8)) == heom.HEOM_E_WORKSPACE
    assert call(nbytes=16) == heom.HEOM_E_WORKSPACE
    bad = np.ascontiguousarray(np.array([[1, 1j], [1j, 0]], np.complex128)).view(np.float64)
    assert call(rho=bad) == heom.HEOM_E_INVALID
    assert "Hermitian" in lib.heom_last_error().decode()
    res = heom.EffResult()
    assert lib.heom_efficiency(h.handle, 0, P(r0), 1.0, 0.0, 2.0, fake, 1 << 30, None,
                               ctypes.byref(res)) == heom.HEOM_E_INVALID
    out = ctypes.c_size_t()
    assert lib.heom_batch_workspace_bytes(None, 0, 0, ctypes.byref(out)) == heom.HEOM_E_INVALID


def test_workspace_sizes_scale_with_precision():
    h = heom.Hierarchy(workloads.fmo_like(0)["system"], 7)
    b64, b32 = h.workspace_bytes[heom.HEOM_FP64], h.workspace_bytes[heom.HEOM_FP32_MIXED]
    planes = 3 * 49 * ((3432 + 63) // 64 * 64)
    assert b64 > 8 * planes and b32 > 4 * planes and b32 < b64
    two = heom.batch_workspace_bytes([h, h])
    assert two > 2 * 8 * planes


def test_product_path_does_not_use_the_oracle():
    """The package never imports or loads anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_1012_4382_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "heom_oracle" not in text, f


def test_tile_shapes_and_forced_shape_validation():
    """Launch shapes: the 64-ADO tile kernel in shapes 0-4 (every N <= 12 has
    shape 0, N <= 8 all five, with one Matsubara term N <= 8), its waves
    dividing the N(N+1)/2 packed elements; the 16-ADO wide kernel as shape 5 for N <= 32; a forced shape
    that is out of range or not built is rejected before device work."""
    lib = heom.library()
    count = heom.tile_shape_count()
    wide = count - 1
    assert count == 6
    for N in range(1, 34):
        P = N * (N + 1) // 2
        for prec in ("fp64", "fp32"):
            for s in range(wide):
                # K + 1 = 1: N <= 8 in every shape, N <= 12 in shape 0;
                # K + 1 = 2: N <= 8 in every shape.  Both storage types.
                for kp, built in ((1, N <= 8 or (s == 0 and N <= 12)), (2, N <= 8)):
                    info = heom.tile_shape_info(N, kp, prec, s)
                    assert (info is not None) == built, (N, kp, prec, s)
                    if info is not None:
                        ados, threads, epw, chunk, waves = info
                        assert ados == 64 and threads % 64 == 0 and 64 <= threads <= 1024
                        assert P % (threads // 64) == 0 and epw >= 1 and chunk >= 1
                        assert 1 <= waves <= 8
            for kp in (1, 2, 4):
                info = heom.tile_shape_info(N, kp, prec, wide)
                # LDS bound: with 4 modes per site, FP64 tiles of 32 sites do not fit.
                fits = N <= 32 and not (N == 32 and kp == 4 and prec == "fp64")
                assert (info is not None) == fits, (N, kp, prec)
                if info is not None:
                    assert info[:2] == (16, 1024)
    assert lib.heom_tile_shape_info(7, 1, 0, count, None, None, None, None, None) == \
        heom.HEOM_E_INVALID
    assert lib.heom_tile_shape_info(7, 1, 5, 0, None, None, None, None, None) == \
        heom.HEOM_E_UNSUPPORTED

    H = np.diag(np.linspace(12300.0, 12500.0, 12)) + np.diag(np.full(11, -80.0), 1) \
        + np.diag(np.full(11, -80.0), -1)
    h = heom.Hierarchy(workloads.system(H), 1)
    r0 = np.ascontiguousarray(workloads.site_state(12, 1)).view(np.float64)
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first

    def call(flags):
        return lib.heom_propagate(h.handle, 0, flags, heom._dp(r0), 1.0, 10, 1, fake, 1 << 30,
                                  None, None, None)

    assert call(heom.tile_shape_flag(1)) == heom.HEOM_E_UNSUPPORTED
    assert "not built" in lib.heom_last_error().decode()
    assert call(heom.tile_shape_flag(count)) == heom.HEOM_E_INVALID
    assert call(1 << 13) == heom.HEOM_E_INVALID


@pytest.mark.parametrize("N,K,D,G", [(7, 0, 8, 8), (7, 1, 4, 3), (3, 0, 12, 5), (7, 0, 16, 8)])
def test_shard_plan_matches_the_tables(N, K, D, G):
    """The split of a hierarchy over G ranks: contiguous tile-aligned ranges,
    and per rank the halo (ADOs of other ranks its ADOs link to), the links
    that leave the range and the reals a rank needs (rows and columns of the
    linking sites), recomputed here from the library's global tables."""
    rng = np.random.default_rng(N + 10 * K + D)
    H = np.diag(rng.uniform(12200, 12600, N))
    h = heom.Hierarchy(workloads.system(H, K=K), D)
    s = heom.Shard(h, G)
    multi, up, down = h.tables()
    site = np.repeat(np.arange(N), K + 1)
    firsts = [s.info(r)["first_ado"] for r in range(G)] + [h.n_ados]
    assert firsts[0] == 0 and all(f % 64 == 0 for f in firsts[:-1])
    assert all(a < b for a, b in zip(firsts, firsts[1:]))
    for r in range(G):
        lo, hi = firsts[r], firsts[r + 1]
        inf = s.info(r)
        links = {}
        for tab in (up, down):
            sub = tab[lo:hi]
            out = (sub >= 0) & ((sub < lo) | (sub >= hi))
            for i, m in zip(*np.nonzero(out)):
                links.setdefault(int(sub[i, m]), set()).add(int(site[m]))
        n_links = sum(int(np.sum((t[lo:hi] >= 0) & ((t[lo:hi] < lo) | (t[lo:hi] >= hi))))
                      for t in (up, down))

        def reals(k):
            return k + 2 * (N * (N - 1) // 2 - (N - k) * (N - k - 1) // 2)
        assert inf["n_local"] == hi - lo
        assert inf["n_halo"] == len(links)
        assert inf["cut_links"] == n_links
        assert inf["halo_reals"] == len(links) * N * N
        assert inf["halo_reals_min"] == sum(reals(len(v)) for v in links.values())
    s.close()


def test_shard_rejects_bad_requests():
    h = heom.Hierarchy(workloads.fmo_like(seed=0, depth=2)["system"], 2)  # 36 ADOs
    with pytest.raises(heom.HeomError) as e:
        heom.Shard(h, 2)  # fewer than 64 ADOs per rank
    assert e.value.status == heom.HEOM_E_INVALID
    h3 = heom.Hierarchy(workloads.fmo_like(seed=0, depth=3)["system"], 3)  # 120 ADOs
    with pytest.raises(heom.HeomError):
        heom.Shard(h3, 0)
    s = heom.Shard(h3, 1)
    assert s.info(0)["n_halo"] == 0 and s.info(0)["n_local"] == 120
    lib = heom.library()
    b = ctypes.c_size_t()
    assert lib.heom_shard_workspace_bytes(s.handle, heom.HEOM_FP32_MIXED,
                                          ctypes.byref(b)) == heom.HEOM_E_UNSUPPORTED


def test_scaled_hierarchy_build_and_validation():
    w = workloads.fmo_like(seed=0, depth=3)
    h = heom.Hierarchy(w["system"], 3, scaled=True, filter_tol=1e-9)
    plain = heom.Hierarchy(w["system"], 3)
    assert (h.n_ados, h.n_modes) == (plain.n_ados, plain.n_modes)
    # The weight tables (2 x M x (depth + 1) doubles) enlarge the parameter block.
    assert h.workspace_bytes[heom.HEOM_FP64] >= plain.workspace_bytes[heom.HEOM_FP64]
    for bad in (-1e-9, float("nan"), float("inf")):
        with pytest.raises(heom.HeomError) as e:
            heom.Hierarchy(w["system"], 3, scaled=True, filter_tol=bad)
        assert e.value.status == heom.HEOM_E_INVALID
    with pytest.raises(heom.HeomError) as e:  # lambda = 0: no scale for the modes
        heom.Hierarchy(dict(w["system"], lam=0.0), 3, scaled=True)
    assert e.value.status == heom.HEOM_E_INVALID
    with pytest.raises(heom.HeomError) as e:
        heom.Shard(heom.Hierarchy(workloads.fmo_like(seed=0, depth=5)["system"], 5,
                                  scaled=True), 2)
    assert e.value.status == heom.HEOM_E_UNSUPPORTED


def test_max_stable_dt_guide_and_warning():
    """heom_max_stable_dt: dt * depth * max nu_m = 2.5 for the deepest ADO on
    the fastest mode (classic RK4's stability interval, Appendix B's fixed-step
    RK4); +inf at depth 0; the binding warns above it and stays silent below."""
    w = workloads.sweep_instance(2)  # one Matsubara term per bath: nu_1 >> gamma
    h = heom.Hierarchy(w["system"], w["depth"])
    _, _, nu, _ = h.modes()
    assert h.max_stable_dt_fs == pytest.approx(2.5 / (w["depth"] * nu.max()), rel=1e-15)
    assert heom.Hierarchy(w["system"], 0).max_stable_dt_fs == float("inf")
    lib = heom.library()
    assert lib.heom_max_stable_dt(None, None) == heom.HEOM_E_INVALID
    with pytest.warns(RuntimeWarning, match="stability"):
        heom._warn_dt([h], 1.01 * h.max_stable_dt_fs)
    import warnings as _w
    with _w.catch_warnings():
        _w.simplefilter("error")
        heom._warn_dt([h], 0.99 * h.max_stable_dt_fs)
