// params.cpp -- parameter normalisation for the HEOM propagation (host).
//
// Converts the caller's system (cm^-1, fs, K, 1/ps) to hbar = 1 units
// (rad/fs and 1/fs) and derives the bath modes:
//   * Drude-Lorentz spectral density J(w) = 2 lambda w gamma / (w^2 + gamma^2)
//     (paper, eq:gamma); its correlation function is expanded as
//     sum_m c_m exp(-nu_m t) with the Drude pole nu = gamma and the Matsubara
//     poles nu_k = 2 pi k kT of coth;
//   * Drude amplitude lambda*gamma*(cot(gamma/2kT) - i), or the paper's
//     high-temperature form 2*lambda*kT - i*lambda*gamma (theta after eq:M,
//     with k_B T moved to the numerator so that the units agree);
//   * Matsubara amplitudes 4 lambda gamma kT nu_k / (nu_k^2 - gamma^2);
//   * low-temperature correction (the first quantum correction the paper applies
//     to the high-temperature bath statistics, section
//     "Trapping time for different temperatures"): the Matsubara terms beyond
//     K act as a white-noise residual -Delta [V,[V, .]] with
//     Delta = 2 lambda kT / gamma - lambda cot(gamma/2kT) - sum_{k<=K} c_k/nu_k;
//   * sinks (eq:lab2, eq:lab3): the exciton block of each Lindblad term is the
//     anti-Hermitian part -(i/2) Gamma_a on site a.
// The mean site energy is removed from the diagonal of H: only energy
// differences enter [H, sigma], and removing the ~2.3 rad/fs offset keeps the
// FP32 path from cancelling large numbers.
#include <cmath>
#include <cstring>

#include "heom_internal.h"

namespace heom {
namespace {

constexpr double kPi = 3.14159265358979323846;
// Speed of light (cm/s), Planck and Boltzmann constants: exact SI values.
constexpr double kLightCmPerS = 2.99792458e10;
constexpr double kPlanckJs = 6.62607015e-34;
constexpr double kBoltzmannJPerK = 1.380649e-23;

inline double wavenumber_to_rad_per_fs(double cm) { return cm * 2.0 * kPi * kLightCmPerS * 1e-15; }
inline double kelvin_to_wavenumber(double T) { return T * kBoltzmannJPerK / (kPlanckJs * kLightCmPerS); }

bool finite(double x) { return std::isfinite(x); }

}  // namespace

int build_params(const heom_system *sys, heom_hierarchy *h) {
  if (!sys) return fail(HEOM_E_INVALID, "system is NULL");
  const int N = sys->n_sites;
  if (N < 1 || N > kMaxSites) return fail(HEOM_E_INVALID, "n_sites must be in [1, 64]");
  if (!sys->hamiltonian_cm || !sys->lambda_cm || !sys->gamma_inv_fs)
    return fail(HEOM_E_INVALID, "hamiltonian_cm, lambda_cm and gamma_inv_fs are required");
  if (!(sys->temperature_K > 0.0) || !finite(sys->temperature_K))
    return fail(HEOM_E_INVALID, "temperature_K must be > 0 and finite");
  if (sys->n_matsubara < 0 || sys->n_matsubara > 64)
    return fail(HEOM_E_INVALID, "n_matsubara must be in [0, 64]");
  if (sys->theta_form != 0 && sys->theta_form != 1)
    return fail(HEOM_E_INVALID, "theta_form must be 0 or 1");
  if (sys->low_temp_correction != 0 && sys->low_temp_correction != 1)
    return fail(HEOM_E_INVALID, "low_temp_correction must be 0 or 1");

  // Hamiltonian: finite and Hermitian within 1e-12 of its largest entry.
  const double *Hc = sys->hamiltonian_cm;
  double hmax = 0.0;
  for (int k = 0; k < 2 * N * N; ++k) {
    if (!finite(Hc[k])) return fail(HEOM_E_INVALID, "hamiltonian has a non-finite entry");
    hmax = std::fmax(hmax, std::fabs(Hc[k]));
  }
  bool real = true;
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      const double re_ab = Hc[2 * (a * N + b)], im_ab = Hc[2 * (a * N + b) + 1];
      const double re_ba = Hc[2 * (b * N + a)], im_ba = Hc[2 * (b * N + a) + 1];
      if (std::fabs(re_ab - re_ba) > 1e-12 * hmax || std::fabs(im_ab + im_ba) > 1e-12 * hmax)
        return fail(HEOM_E_INVALID, "hamiltonian is not Hermitian");
      if (im_ab != 0.0) real = false;
    }
  for (int a = 0; a < N; ++a) {
    if (!(sys->lambda_cm[a] >= 0.0) || !finite(sys->lambda_cm[a]))
      return fail(HEOM_E_INVALID, "lambda_cm must be >= 0 and finite");
    if (!(sys->gamma_inv_fs[a] > 0.0) || !finite(sys->gamma_inv_fs[a]))
      return fail(HEOM_E_INVALID, "gamma_inv_fs must be > 0 and finite");
    if (sys->trap_rate_per_ps &&
        (!(sys->trap_rate_per_ps[a] >= 0.0) || !finite(sys->trap_rate_per_ps[a])))
      return fail(HEOM_E_INVALID, "trap rates must be >= 0 and finite");
    if (sys->recomb_rate_per_ps &&
        (!(sys->recomb_rate_per_ps[a] >= 0.0) || !finite(sys->recomb_rate_per_ps[a])))
      return fail(HEOM_E_INVALID, "recombination rates must be >= 0 and finite");
  }

  const int K = sys->n_matsubara;
  const int KP = K + 1;
  const int M = N * KP;
  h->N = N;
  h->K = K;
  h->KP = KP;
  h->M = M;
  h->h_real = real;

  const double kT = wavenumber_to_rad_per_fs(kelvin_to_wavenumber(sys->temperature_K));
  h->site.assign(M, 0);
  h->c_re.assign(M, 0.0);
  h->c_im.assign(M, 0.0);
  h->nu.assign(M, 0.0);
  h->delta.assign(N, 0.0);
  for (int s = 0; s < N; ++s) {
    const double lam = wavenumber_to_rad_per_fs(sys->lambda_cm[s]);
    const double gam = 1.0 / sys->gamma_inv_fs[s];
    const double x = gam / (2.0 * kT);
    const double cotx = std::cos(x) / std::sin(x);
    const int m0 = s * KP;
    h->site[m0] = s;
    h->nu[m0] = gam;
    h->c_im[m0] = -lam * gam;
    h->c_re[m0] = (sys->theta_form == 0) ? lam * gam * cotx : 2.0 * lam * kT;
    double tail_head = 0.0;  // sum_{k<=K} c_k / nu_k
    for (int k = 1; k <= K; ++k) {
      const double nuk = 2.0 * kPi * k * kT;
      if (std::fabs(nuk - gam) <= 1e-9 * gam)
        return fail(HEOM_E_INVALID, "a Matsubara frequency coincides with gamma");
      const double ck = 4.0 * lam * gam * kT * nuk / (nuk * nuk - gam * gam);
      h->site[m0 + k] = s;
      h->nu[m0 + k] = nuk;
      h->c_re[m0 + k] = ck;
      h->c_im[m0 + k] = 0.0;
      tail_head += ck / nuk;
    }
    if (sys->low_temp_correction) h->delta[s] = 2.0 * lam * kT / gam - lam * cotx - tail_head;
    if (!finite(h->c_re[m0]) || !finite(h->delta[s]))
      return fail(HEOM_E_INVALID, "bath parameters give a non-finite amplitude");
  }

  // Parameter block (rho0 slot left zero; filled per run).
  const ParamOffsets o = param_offsets(N, M);
  h->params.assign(o.total, 0.0);
  double mean_diag = 0.0;
  for (int a = 0; a < N; ++a) mean_diag += Hc[2 * (a * N + a)];
  mean_diag /= N;
  h->energy_offset = wavenumber_to_rad_per_fs(mean_diag);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) {
      double re = Hc[2 * (a * N + b)];
      if (a == b) re -= mean_diag;
      h->params[o.h_re + a * N + b] = wavenumber_to_rad_per_fs(re);
      h->params[o.h_im + a * N + b] = wavenumber_to_rad_per_fs(Hc[2 * (a * N + b) + 1]);
    }
  for (int a = 0; a < N; ++a) {
    const double tr = sys->trap_rate_per_ps ? sys->trap_rate_per_ps[a] * 1e-3 : 0.0;
    const double rc = sys->recomb_rate_per_ps ? sys->recomb_rate_per_ps[a] * 1e-3 : 0.0;
    h->params[o.half_gamma + a] = 0.5 * (tr + rc);
    h->params[o.delta + a] = h->delta[a];
    h->params[o.trap + a] = tr;
    h->params[o.rec + a] = rc;
  }
  for (int m = 0; m < M; ++m) {
    h->params[o.c_re + m] = h->c_re[m];
    h->params[o.c_im + m] = h->c_im[m];
    h->params[o.nu + m] = h->nu[m];
  }
  // FP32 copy: each value rounded once here, as the FP32 kernels would round
  // it on use.
  unsigned char *f32 = reinterpret_cast<unsigned char *>(h->params.data() + o.f32);
  for (int q = 0; q < o.rho0; ++q) {
    const float v = static_cast<float>(h->params[q]);
    std::memcpy(f32 + sizeof(float) * q, &v, sizeof(float));
  }
  return HEOM_OK;
}

}  // namespace heom
