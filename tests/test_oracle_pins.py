"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle (oracle/heom_oracle.cpp) against something other
than itself: printed values of the paper, closed forms, an independent dense
(Kronecker) assembly of the generator, the exact Taylor polynomial that RK4 is
for a linear system, matrix exponentials, numeric quadrature of the bath
correlation function, and exact invariants.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.linalg
import scipy.special

import oracle
from paper_1012_4382_amd import workloads
from oracle import closed_forms as cf
from oracle import dense

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dimer(**kw):
    s = dict(H=np.array([[12410.0, -87.7], [-87.7, 12530.0]]), lam=35.0, gamma_inv_fs=50.0,
             T=300.0, K=0, ltc=1, theta_form=0, trap_per_ps=None, rec_per_ps=None)
    s.update(kw)
    return s


def _random_system(N, K, seed, sinks=True, T=150.0, complex_h=False):
    rng = np.random.default_rng(seed)
    H = rng.normal(0, 50, (N, N))
    H = H + H.T
    if complex_h:
        A = rng.normal(0, 20, (N, N))
        H = H + 1j * (A - A.T)
    H = H + np.diag(rng.uniform(12200, 12600, N))
    return dict(H=H, lam=rng.uniform(10, 100, N), gamma_inv_fs=rng.uniform(25, 200, N), T=T,
                K=K, ltc=1, theta_form=0,
                trap_per_ps=rng.uniform(0, 2, N) if sinks else None,
                rec_per_ps=rng.uniform(0, 0.01, N) if sinks else None)


def _fmo_table1():
    return np.loadtxt(os.path.join(GOLDEN, "fmo_table1_cm.txt"))


# --- units -------------------------------------------------------------------

def test_unit_constants():
    # 1/(2 pi c) in cm^-1 fs: the period-frequency conversion of spectroscopy.
    assert abs(1.0 / dense.CM_TO_RAD_FS - 5308.837458876) < 1e-6
    # k_B/(h c) = 0.695034800... cm^-1/K (exact SI constants).
    assert abs(dense.KB_CM_PER_K - 0.6950348004861274) < 1e-15
    # The oracle's Drude amplitude at one known point reproduces the same units:
    # Im c_0 = -lambda * gamma with lambda = 35 cm^-1, gamma = 1/50 fs^-1.
    _, c, nu, _ = oracle.modes(_dimer())
    assert abs(c[0].imag - (-35.0 * 2 * math.pi * 2.99792458e-5 / 50.0)) < 1e-18
    assert nu[0] == pytest.approx(1 / 50.0, rel=1e-15)


# --- bath coefficients ---------------------------------------------------------

def _correlation_quadrature(lam_cm, gamma_inv, T, t):
    """C(t) = (1/pi) int_0^inf J(w) [coth(w/2kT) cos wt - i sin wt] dw, by quadrature."""
    lam = lam_cm * dense.CM_TO_RAD_FS
    gam = 1.0 / gamma_inv
    kT = dense.KB_CM_PER_K * T * dense.CM_TO_RAD_FS

    def f_re(w):
        x = w / (2 * kT)
        xcoth = 1.0 if x < 1e-8 else x / math.tanh(x)
        return 2 * lam * gam / (w * w + gam * gam) * 2 * kT * xcoth / math.pi

    def f_im(w):
        return -2 * lam * w * gam / (w * w + gam * gam) / math.pi

    re = scipy.integrate.quad(f_re, 0, np.inf, weight="cos", wvar=t, limlst=500, limit=500,
                              epsabs=1e-17)[0]
    im = scipy.integrate.quad(f_im, 0, np.inf, weight="sin", wvar=t, limlst=500, limit=500,
                              epsabs=1e-17)[0]
    return complex(re, im)


@pytest.mark.parametrize("T,gi,lam", [(300.0, 50.0, 35.0), (77.0, 166.0, 35.0), (150.0, 25.0, 90.0)])
def test_mode_expansion_matches_quadrature(T, gi, lam):
    """Drude + Matsubara amplitudes reproduce the correlation function of eq:gamma."""
    sys = dict(H=np.diag([0.0]), lam=lam, gamma_inv_fs=gi, T=T, K=200, ltc=0)
    _, c, nu, _ = oracle.modes(sys)
    for t in (5.0, 20.0, 60.0, 150.0, 400.0):
        series = np.sum(c * np.exp(-nu * t))
        ref = _correlation_quadrature(lam, gi, T, t)
        assert abs(series - ref) <= 1e-7 * abs(ref), (t, series, ref)


def test_high_temperature_form():
    """theta_form 1 is the paper's high-temperature amplitude 2 lambda kT - i lambda gamma."""
    s = _dimer(theta_form=1)
    _, c, _, _ = oracle.modes(s)
    lam = 35.0 * dense.CM_TO_RAD_FS
    kT = dense.KB_CM_PER_K * 300.0 * dense.CM_TO_RAD_FS
    assert c[0] == pytest.approx(complex(2 * lam * kT, -lam / 50.0), rel=1e-14)
    # The exact amplitude tends to it when gamma/kT -> 0.
    hot = _dimer(T=1e7)  # gamma/2kT ~ 8e-6: relative gap ~ (gamma/2kT)^2/3
    _, ce, _, _ = oracle.modes(hot)
    _, ch, _, _ = oracle.modes(dict(hot, theta_form=1))
    assert abs(ce[0] - ch[0]) < 1e-9 * abs(ch[0])


@pytest.mark.parametrize("K", [0, 1, 3])
def test_ltc_residual_is_matsubara_tail(K):
    """Delta equals the sum over the Matsubara terms beyond K of c_k/nu_k (brute force)."""
    T, gi, lam = 300.0, 50.0, 35.0
    s = dict(H=np.diag([0.0]), lam=lam, gamma_inv_fs=gi, T=T, K=K, ltc=1)
    _, _, _, delta = oracle.modes(s)
    lam_r = lam * dense.CM_TO_RAD_FS
    gam = 1 / gi
    kT = dense.KB_CM_PER_K * T * dense.CM_TO_RAD_FS
    k = np.arange(K + 1, 2_000_001, dtype=float)
    nu = 2 * math.pi * k * kT
    tail = np.sum(4 * lam_r * gam * kT / (nu * nu - gam * gam))
    # Remainder beyond the partial sum: sum_{k>k_max} 4 lam gam kT / nu_k^2 ~ lam gam / (pi^2 kT k_max).
    tail += lam_r * gam / (math.pi**2 * kT * k[-1])
    assert abs(delta[0] - tail) <= 1e-9 * abs(tail)
    assert delta[0] > 0


# --- hierarchy enumeration -----------------------------------------------------

def test_ado_counts_printed_in_paper():
    rows = np.loadtxt(os.path.join(GOLDEN, "paper_ado_counts.txt"), dtype=np.int64)
    for M, D, n in rows:
        if n > 60000:
            # Too large to enumerate quickly with the plain oracle; check the closed form.
            assert math.comb(int(M + D), int(D)) == n
            continue
        sys = dict(H=np.eye(int(M)), lam=35.0, gamma_inv_fs=50.0, T=300.0, K=0, ltc=1)
        assert oracle.count(sys, int(D)) == (n, M)


@pytest.mark.parametrize("N,K,D", [(2, 0, 4), (2, 1, 5), (3, 1, 3), (7, 0, 3), (4, 2, 2)])
def test_enumeration_is_the_full_simplex(N, K, D):
    sys = dict(H=np.eye(N), lam=35.0, gamma_inv_fs=50.0, T=300.0, K=K, ltc=1)
    multi = oracle.enumerate_ados(sys, D)
    M = N * (K + 1)
    assert multi.shape == (math.comb(M + D, D), M)
    assert np.all(multi >= 0) and np.all(multi.sum(1) <= D)
    assert len({tuple(r) for r in multi}) == multi.shape[0]
    assert np.all(multi[0] == 0)


# --- right-hand side -------------------------------------------------------------

@pytest.mark.parametrize("N,D,K,complex_h", [(2, 4, 0, False), (2, 3, 1, False), (3, 3, 0, True),
                                             (3, 2, 1, False)])
def test_rhs_matches_dense_kronecker_generator(N, D, K, complex_h):
    sys = _random_system(N, K, seed=N * 10 + D + K, sinks=True, complex_h=complex_h)
    multi = oracle.enumerate_ados(sys, D)
    L = dense.generator(sys, multi)
    rng = np.random.default_rng(7)
    n = multi.shape[0]
    # Arbitrary (non-Hermitian) state: the ADO part of the generator.
    x = rng.normal(size=(n, N, N)) + 1j * rng.normal(size=(n, N, N))
    sc = rng.normal(size=3)
    f, fs = oracle.rhs(sys, D, x, sc)
    ref = L @ np.concatenate([x.reshape(-1), sc])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(f.reshape(-1) - ref[: n * N * N])) <= 1e-13 * scale
    # Hermitian state: the scalar part (populations are real there).
    xh = x + np.conj(np.transpose(x, (0, 2, 1)))
    f, fs = oracle.rhs(sys, D, xh, sc)
    ref = L @ np.concatenate([xh.reshape(-1), sc])
    assert np.max(np.abs(fs - ref[n * N * N:].real)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_rk4_step_is_the_taylor_polynomial():
    """For a constant generator classic RK4 is exactly sum_{k<=4} (dt L)^k/k! per step."""
    sys = _random_system(3, 1, seed=3, sinks=True)
    D = 2
    multi = oracle.enumerate_ados(sys, D)
    L = dense.generator(sys, multi)
    dt, steps = 2.0, 40
    P = dense.rk4_polynomial(L, dt)
    n, N = multi.shape[0], 3
    rng = np.random.default_rng(11)
    sig = rng.normal(size=(n, N, N)) + 1j * rng.normal(size=(n, N, N))
    sig = sig + np.conj(np.transpose(sig, (0, 2, 1)))
    sc = np.array([0.1, 0.2, 0.3])
    x = np.concatenate([sig.reshape(-1), sc]).astype(np.complex128)
    ref = np.linalg.matrix_power(P, steps) @ x
    out = oracle.propagate(sys, D, None if False else sig[0], dt, steps, record_every=steps,
                           want_state=True, state_in=(sig, sc))
    got = np.concatenate([out["state"][0].reshape(-1), out["state"][1]])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_fourth_order_convergence_to_exponential():
    sys = _random_system(2, 1, seed=5, sinks=True)
    D = 3
    multi = oracle.enumerate_ados(sys, D)
    L = dense.generator(sys, multi)
    rho0 = np.array([[1, 0], [0, 0]], complex)
    n = multi.shape[0]
    x0 = np.zeros(n * 4 + 3, complex)
    x0[:4] = rho0.reshape(-1)
    t_end = 200.0
    exact = scipy.linalg.expm(t_end * L) @ x0
    errs = []
    for dt in (4.0, 2.0, 1.0):
        r = oracle.propagate(sys, D, rho0, dt, int(t_end / dt), record_every=int(t_end / dt))
        errs.append(np.max(np.abs(r["rho"][-1].reshape(-1) - exact[:4])))
    for a, b in zip(errs, errs[1:]):
        assert 16 * 0.85 < a / b < 16 * 1.15, errs


# --- closed forms -----------------------------------------------------------------

def test_pure_dephasing_closed_form():
    """J = 0: the coherence follows exp(-i w t - g_1(t) - conj(g_2(t))) (2nd cumulant, exact)."""
    sys = _dimer(H=np.diag([12410.0, 12530.0]))
    rho0 = np.full((2, 2), 0.5, complex)
    errs = {}
    for D in (4, 8, 12, 20):
        r = oracle.propagate(sys, D, rho0, 0.125, 2400, record_every=200)
        t = np.arange(r["rho"].shape[0]) * 25.0
        ex = cf.pure_dephasing_coherence(sys, 0, 1, 0.5, t)
        errs[D] = np.max(np.abs(r["rho"][:, 0, 1] - ex)) / 0.5
        # Populations are constant in pure dephasing.
        assert np.max(np.abs(r["rho"][:, 0, 0] - 0.5)) < 1e-14
    assert errs[4] > errs[8] > errs[12] > errs[20]
    # RK4 at dt = 0.125 fs leaves ~1e-11 (it falls by 16 per halving of dt).
    assert errs[20] < 3e-11, errs
    # Different baths on the two sites, with a Matsubara term: checks the
    # site-a / site-b (conj) assignment.
    sys2 = dict(H=np.diag([12400.0, 12300.0]), lam=np.array([60.0, 20.0]),
                gamma_inv_fs=np.array([40.0, 120.0]), T=150.0, K=1, ltc=1)
    r = oracle.propagate(sys2, 14, rho0, 0.25, 800, record_every=80)
    t = np.arange(r["rho"].shape[0]) * 20.0
    ex = cf.pure_dephasing_coherence(sys2, 0, 1, 0.5, t)
    assert np.max(np.abs(r["rho"][:, 0, 1] - ex)) / 0.5 < 1e-8


def test_unitary_limit():
    """lambda = 0: every deeper ADO stays zero and rho evolves unitarily."""
    N = 3
    H = _fmo_table1()[:N, :N]
    sys = dict(H=H, lam=0.0, gamma_inv_fs=50.0, T=300.0, K=0, ltc=1)
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    r = oracle.propagate(sys, 3, rho0, 0.05, 2000, record_every=2000, want_state=True)
    assert np.all(r["state"][0][1:] == 0)
    ex = cf.unitary(sys, rho0, 100.0)
    assert np.max(np.abs(r["rho"][-1] - ex)) < 1e-10
    # At dt = 1 fs compare with the RK4 polynomial of the system generator itself.
    Hr = H * dense.CM_TO_RAD_FS
    Ls = -1j * (np.kron(Hr, np.eye(N)) - np.kron(np.eye(N), Hr.T))
    P = dense.rk4_polynomial(Ls, 1.0)
    r = oracle.propagate(sys, 2, rho0, 1.0, 1000, record_every=1000)
    ref = (np.linalg.matrix_power(P, 1000) @ rho0.reshape(-1)).reshape(N, N)
    assert np.max(np.abs(r["rho"][-1] - ref)) < 1e-12


def test_pure_decay_sinks_and_trapping_time():
    """No coupling, no bath: exponential decay; P_trap and Q in closed form."""
    N = 3
    sys = dict(H=np.diag([12400.0, 12300.0, 12200.0]), lam=0.0, gamma_inv_fs=50.0, T=300.0, K=0,
               ltc=1, trap_per_ps=np.array([0.0, 0.0, 0.4]), rec_per_ps=np.array([4e-3, 4e-3, 4e-3]))
    rho0 = np.diag([0.2, 0.3, 0.5]).astype(complex)
    T = 3000.0
    r = oracle.propagate(sys, 1, rho0, 0.5, int(T / 0.5), record_every=int(T / 0.5))
    pops, p_trap = cf.pure_decay(sys, rho0, T)
    assert np.max(np.abs(np.real(np.diag(r["rho"][-1])) - pops)) < 1e-12
    assert abs(r["scalars"][0] - p_trap) < 1e-12
    # Q = int_0^T P_trap dt and <t> = T P_trap(T) - Q = int_0^T t dP_trap (eq:trappingtime).
    G = 0.4e-3 + 4e-3 * 1e-3
    tr = 0.4e-3
    mean_t = 0.5 * tr * (1 / G**2 - math.exp(-G * T) * (T / G + 1 / G**2))
    assert abs((T * r["scalars"][0] - r["scalars"][2]) - mean_t) < 1e-9 * mean_t


# --- invariants ------------------------------------------------------------------

def test_hermiticity_and_population_invariants():
    N = 3
    H = _fmo_table1()[:N, :N]
    sys = dict(H=H, lam=35.0, gamma_inv_fs=50.0, T=150.0, K=1, ltc=1,
               trap_per_ps=np.array([0.0, 0.0, 1.0]), rec_per_ps=np.full(N, 1e-3))
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    r = oracle.propagate(sys, 3, rho0, 1.0, 2000, record_every=100, want_state=True)
    sig, sc = r["state"]
    anti = np.max(np.abs(sig - np.conj(np.transpose(sig, (0, 2, 1)))), axis=(1, 2))
    norm = np.max(np.abs(sig), axis=(1, 2))
    assert np.all(anti <= 1e-13 * np.maximum(norm, 1e-300))
    tr = np.trace(r["rho"], axis1=1, axis2=2).real
    assert abs(tr[-1] + sc[0] + sc[1] - 1.0) < 1e-12
    assert sc[0] > 0.05  # something was trapped
    # Without sinks the trace itself is conserved.
    sys0 = dict(sys, trap_per_ps=None, rec_per_ps=None)
    r0 = oracle.propagate(sys0, 3, rho0, 1.0, 1000, record_every=100)
    assert np.max(np.abs(np.trace(r0["rho"], axis1=1, axis2=2) - 1.0)) < 1e-12


def test_depth_convergence_of_efficiency():
    N = 3
    H = _fmo_table1()[:N, :N]
    sys = dict(H=H, lam=35.0, gamma_inv_fs=50.0, T=300.0, K=0, ltc=1,
               trap_per_ps=np.array([0.0, 0.0, 1.0]), rec_per_ps=np.full(N, 1e-3))
    rho0 = np.zeros((N, N), complex)
    rho0[0, 0] = 1
    eta = [oracle.propagate(sys, D, rho0, 1.0, 1500, record_every=1500)["scalars"][0]
           for D in range(1, 7)]
    diffs = np.abs(np.diff(eta))
    assert np.all(diffs[1:] < diffs[:-1]), eta
    assert diffs[-1] < 1e-4


# --- scaled hierarchy and filter -------------------------------------------------


def _scale_weights(sys_, multi):
    """w_n = sqrt(prod_m n_m! |c_m|^n_m) from the modes recomputed in oracle.dense."""
    modes, _ = dense.bath_modes(sys_)
    absc = np.array([abs(c) for _, c, _ in modes])
    out = np.empty(len(multi))
    for i, row in enumerate(multi):
        out[i] = math.sqrt(math.prod(math.factorial(int(v)) * absc[m] ** int(v)
                                     for m, v in enumerate(row)))
    return out


@pytest.mark.parametrize("N,D,K", [(2, 4, 0), (2, 3, 1), (3, 2, 1)])
def test_scaled_rhs_is_the_similarity_transform(N, D, K):
    """Holding sigma_n / w_n turns the generator L into W^-1 L W with
    W = diag(w_n): the oracle's scaled right-hand side must equal that
    product, assembled from the independent Kronecker generator."""
    rng = np.random.default_rng(40 + N + D + K)
    H = np.diag(rng.uniform(12200, 12600, N)) + 0j
    for a in range(N):
        for b in range(a + 1, N):
            H[a, b] = rng.normal(0, 50)
            H[b, a] = H[a, b]
    trap = np.zeros(N)
    trap[-1] = 1.0
    sys_ = workloads.system(H, lam=60.0, T=150.0, K=K, trap=trap, rec=np.full(N, 1e-3))
    multi = oracle.enumerate_ados(sys_, D)
    L = dense.generator(sys_, multi)
    w = _scale_weights(sys_, multi)
    Wd = np.concatenate([np.repeat(w, N * N), np.ones(3)])
    Ls = L * Wd[None, :] / Wd[:, None]
    n_ado = len(multi)
    x = rng.normal(size=(n_ado, N, N)) + 1j * rng.normal(size=(n_ado, N, N))
    x = x + np.conj(np.transpose(x, (0, 2, 1)))
    sc = rng.normal(size=3)
    f, fs = oracle.rhs(sys_, D, x, sc, scaled=True)
    want = Ls @ np.concatenate([x.reshape(-1), sc])
    got = np.concatenate([f.reshape(-1), fs])
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))
    # The scaling is not the identity here (it would hide a dropped weight).
    assert np.max(np.abs(w - 1.0)) > 0.5


def test_scaled_propagation_equals_unscaled():
    """The scaled hierarchy is the same equations in other variables: sigma_0
    agrees to rounding over the whole run, and every ADO equals w_n times its
    scaled counterpart."""
    w = workloads.sweep_instance(6)  # 7 sites, one Matsubara term per bath
    sys_ = dict(w["system"], H=w["system"]["H"][:3, :3], trap_per_ps=np.array([0, 0, 1.0]),
                rec_per_ps=np.full(3, 1e-3))
    D = 4
    a = oracle.propagate(sys_, D, w["rho0"][:3, :3], 1.0, 400, record_every=10, want_state=True)
    b = oracle.propagate(sys_, D, w["rho0"][:3, :3], 1.0, 400, record_every=10, want_state=True,
                         scaled=True)
    assert np.max(np.abs(a["rho"] - b["rho"])) <= 1e-12 * np.max(np.abs(a["rho"]))
    assert np.max(np.abs(a["scalars"] - b["scalars"])) <= 1e-12
    multi = oracle.enumerate_ados(sys_, D)
    wts = _scale_weights(sys_, multi)
    tiers = multi.sum(axis=1)
    sa, sb = a["state"][0], b["state"][0] * wts[:, None, None]
    for t in range(D + 1):
        sel = tiers == t
        assert np.max(np.abs(sa[sel] - sb[sel])) <= 1e-11 * np.max(np.abs(sa[sel])), t


def test_filter_zero_threshold_changes_nothing():
    w = workloads.fmo_like(seed=0, site=1, depth=3, steps=200)
    a = oracle.propagate(w["system"], 3, w["rho0"], 1.0, 200, record_every=20, scaled=True)
    b = oracle.propagate(w["system"], 3, w["rho0"], 1.0, 200, record_every=20, scaled=True,
                         filter_tol=0.0)
    assert np.array_equal(a["rho"], b["rho"]) and np.array_equal(a["scalars"], b["scalars"])


def test_filter_drops_small_ados_and_its_error_shrinks_with_the_threshold():
    """Three FMO-like sites at depth 10 (286 ADOs), 2 ps.  The stated error of
    the filter: populations and P_trap within twice the threshold of the
    unfiltered scaled run (measured 1.5x at 1e-4 and 1e-5, 0.13x at 1e-6),
    falling with the threshold, while the filter keeps under half of the
    ADOs at 1e-5 (110 of 286)."""
    w = workloads.fmo_like(seed=2, site=1)
    sys_ = dict(w["system"], H=w["system"]["H"][:3, :3], trap_per_ps=np.array([0, 0, 1.0]),
                rec_per_ps=np.full(3, 1e-3))
    rho0 = w["rho0"][:3, :3]
    D, steps = 10, 2000
    ref = oracle.propagate(sys_, D, rho0, 1.0, steps, record_every=20, scaled=True,
                           want_state=True)
    n_ado = len(ref["state"][0])
    errs, kept = [], []
    for tol in (1e-4, 1e-5, 1e-6):
        r = oracle.propagate(sys_, D, rho0, 1.0, steps, record_every=20, scaled=True,
                             filter_tol=tol, want_state=True)
        dp = np.max(np.abs(np.real(np.diagonal(r["rho"] - ref["rho"], axis1=1, axis2=2))))
        errs.append(max(dp, abs(r["scalars"][0] - ref["scalars"][0])))
        assert errs[-1] <= 2 * tol, (tol, errs[-1])
        nz = np.max(np.abs(r["state"][0]), axis=(1, 2)) > 0
        kept.append(int(nz.sum()))
        # Zeroed ADOs are exactly those below the threshold: every survivor
        # (sigma_0 aside) has an entry at or above it.
        big = np.maximum(np.abs(r["state"][0].real), np.abs(r["state"][0].imag)).max(axis=(1, 2))
        assert np.all(big[1:][nz[1:]] >= tol)
    assert errs[0] > errs[1] > errs[2]
    assert kept[0] <= kept[1] <= kept[2] < n_ado and kept[1] < 0.5 * n_ado
