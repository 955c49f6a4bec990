"""Planted mistakes in the oracle must be caught by its pins.

Each case applies one textual change to a temporary copy of
oracle/heom_oracle.cpp (a dropped term, a flipped sign, a wrong index, a
transposed operand, a wrong coefficient), builds it, and runs the pin suite
against it in a subprocess; the suite must fail.  Nothing here touches a GPU.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = {
    "up_coupling_sign": ("out[k] += wu * (I * (L[k] - R[k]));",
                         "out[k] -= wu * (I * (L[k] - R[k]));"),
    "scaled_up_weight": ("std::sqrt((m.ados[n][mode] + 1.0) * std::abs(c))",
                         "std::sqrt((m.ados[n][mode] + 0.0) * std::abs(c))"),
    "scaled_down_weight": ("std::sqrt(m.ados[n][mode] / std::abs(c))",
                           "std::sqrt(m.ados[n][mode] * std::abs(c))"),
    "filter_inverted": ("if (mx < tol)", "if (mx > tol)"),
    "dropped_damping": ("axpy(&out, cplx(-damp, 0.0), X);", "(void)damp;"),
    "down_missing_conj": ("std::conj(c) * R[k]", "c * R[k]"),
    "down_missing_occupation": ("out[k] += nm * I *", "out[k] += I *"),
    "projector_transposed": ("for (int j = 0; j < N; ++j) R[s * N + j] = X[s * N + j];",
                             "for (int j = 0; j < N; ++j) R[j * N + s] = X[j * N + s];"),
    "ltc_sign": ("out[k] -= m.delta[s] * (L2[k] - R2[k]);", "out[k] += m.delta[s] * (L2[k] - R2[k]);"),
    "sink_factor": ("cplx(0.0, 0.5 * (m.trap[a] + m.rec[a]))", "cplx(0.0, (m.trap[a] + m.rec[a]))"),
    "heff_not_daggered": ("Mat XH = matmul(X, HeffDag, N);", "Mat XH = matmul(X, Heff, N);"),
    "rk4_weight": ("2.0 * k3.sigma[n][e]", "1.0 * k3.sigma[n][e]"),
    "matsubara_amplitude": ("4.0 * lam * gam * kT", "2.0 * lam * gam * kT"),
    "drude_cot_vs_tan": ("const double cot = 1.0 / std::tan(gam / (2.0 * kT));",
                         "const double cot = std::tan(gam / (2.0 * kT));"),
    "truncation_depth": ("for (int t = 0; t < D; ++t)", "for (int t = 0; t < D - 1; ++t)"),
    "trap_flux_index": ("const double pop = x.sigma[0][a * m.N + a].real();",
                        "const double pop = x.sigma[0][a].real();"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique or missing: {old}"
    mut_src = tmp_path / "mutant.cpp"
    mut_src.write_text(src.replace(old, new))
    lib = oracle.build(force=True, src=str(mut_src), out=str(tmp_path / "libmutant.so"))
    env = dict(os.environ, HEOM_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:warnings",
                        "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived the pins:\n{r.stdout[-2000:]}"
