// heom_oracle.cpp -- plain, slow FP64 reference for the hierarchical equations
// of motion (HEOM) of Kreisbeck, Kramer, Rodriguez and Hein (arXiv:1012.4382).
//
// TEST INFRASTRUCTURE ONLY.  This library is the oracle against which the GPU
// path is checked.  Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark may load it.  It shares no code, header, table or
// constant generator with the GPU library, and it never reads anything the GPU
// path produced.
//
// What it computes (paper, Appendix A "ME-HEOM", eqs. eq:labsevena / eq:lab8,
// and Appendix B for the RK4 propagation):
//   * every auxiliary density operator (ADO) sigma_n, n a multi-index over the
//     bath modes with |n| <= D (truncation, Appendix A after eq:lab8), is held as
//     a full N x N complex matrix; Hermiticity is never assumed;
//   * the right-hand side of eq:lab8 is evaluated with textbook operator
//     formulas: commutators V^x X = VX - XV and anticommutators; V_s = |s><s| is
//     applied by its definition (V_s X keeps row s of X, X V_s keeps column s);
//   * the trapping and recombination Lindblad terms (eq:lab2, eq:lab3) restricted
//     to the exciton block become the anti-Hermitian part -(i/2) diag(Gamma) of
//     an effective Hamiltonian (paper, text after eq:lab3); the populations that
//     leave are accumulated in P_trap and P_rec;
//   * classic fourth-order Runge-Kutta (Appendix B) on the augmented vector
//     (all sigma_n, P_trap, P_rec, Q) with dQ/dt = P_trap, which gives the mean
//     trapping time of eq:trappingtime by integration by parts.
//   * optionally the scaled hierarchy that the introduction names as the way
//     to fewer auxiliary matrices: every ADO is held divided by
//     w_n = sqrt(prod_m n_m! |c_m|^n_m) (so sigma_0 is unchanged), which turns
//     the coupling to n + e_m into sqrt((n_m + 1)|c_m|) i[V, .] and the
//     coupling to n - e_m into sqrt(n_m / |c_m|) i(c V . - c* . V); and a
//     filter that, after every RK4 step, sets to zero every ADO n != 0 whose
//     stored entries are all below a threshold in absolute value (real and
//     imaginary parts).
//
// Readings of points the paper leaves open (each is also listed in the design
// notes of the repository):
//   * damping: -sum_m n_m nu_m (the printed "+" in eq:lab8 would make the
//     hierarchy grow without bound);
//   * the high-temperature correlation printed after eq:gamma has k_B T in the
//     denominator; the dimensionally consistent coefficient is 2 lambda k_B T;
//   * Drude coefficient: theta_form 0 uses the exact lambda*gamma*(cot(gamma/2kT)-i),
//     theta_form 1 the paper's high-temperature 2*lambda*kT - i*lambda*gamma;
//   * Matsubara terms (not written in the paper) follow from the Drude-Lorentz
//     spectral density eq:gamma: nu_k = 2 pi k kT,
//     c_k = 4 lambda gamma kT nu_k / (nu_k^2 - gamma^2);
//   * the low-temperature correction (the first quantum correction to the
//     high-temperature bath statistics that the paper applies,
//     section "Trapping time for different temperatures") is the Markovian
//     residual -Delta_s [V_s,[V_s, .]] on every ADO, with
//     Delta_s = 2 lambda kT/gamma - lambda cot(gamma/2kT) - sum_{k<=K} c_k/nu_k;
//   * zero truncation: sigma_n = 0 for |n| > D;
//   * the Hamiltonian is used exactly as given (no energy offset removed).
//
// Units: hbar = 1; energies in cm^-1 become angular frequencies in rad/fs,
// rates given per ps become per fs.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef std::complex<double> cplx;
typedef std::vector<cplx> Mat;  // N*N, row-major

const double kPi = 3.14159265358979323846;
// 1 cm^-1 expressed as an angular frequency in rad/fs: 2*pi*c*1e-15 s/fs with
// c = 2.99792458e10 cm/s (exact SI value).
const double kCmToRadFs = 2.0 * kPi * 2.99792458e10 * 1e-15;
// Boltzmann constant in cm^-1/K: k_B / (h c) from the exact SI values of
// k_B = 1.380649e-23 J/K, h = 6.62607015e-34 J s, c = 2.99792458e10 cm/s.
const double kBoltzmannCmPerK = 1.380649e-23 / (6.62607015e-34 * 2.99792458e10);

struct Mode {
  int site;
  cplx c;     // amplitude of c * exp(-nu t) in the bath correlation function
  double nu;  // decay rate, 1/fs
};

struct Model {
  int N = 0;
  int depth = 0;
  bool scaled = false;      // ADOs held divided by w_n (see the header)
  double filter_tol = 0.0;  // > 0: filter after every step
  Mat H;                          // rad/fs, as given
  std::vector<double> trap, rec;  // 1/fs, per site
  std::vector<double> delta;      // low-temperature-correction residual per site
  std::vector<Mode> modes;
  std::vector<std::vector<int> > ados;  // multi-indices
  std::map<std::vector<int>, int> index;
  std::vector<std::vector<int> > up, down;  // per ADO, per mode, -1 if absent
};

}  // namespace

extern "C" {

// The oracle's own description of a system (not shared with the GPU library).
typedef struct {
  int32_t n_sites;
  const double* hamiltonian_cm;   // N*N complex, interleaved (re, im), row-major
  const double* lambda_cm;        // [N]
  const double* gamma_inv_fs;     // [N]
  double temperature_K;
  int32_t n_matsubara;            // K
  int32_t low_temp_correction;    // 0 or 1
  int32_t theta_form;             // 0 exact cot, 1 paper high-temperature form
  const double* trap_rate_per_ps; // [N] or NULL
  const double* recomb_rate_per_ps;  // [N] or NULL
} oracle_system;

}  // extern "C"

namespace {

// Bath modes and the correction residual, from the Drude-Lorentz spectral
// density J(w) = 2 lambda w gamma / (w^2 + gamma^2) (eq:gamma) and the
// expansion of coth into its Matsubara poles.
bool make_modes(const oracle_system* s, Model* m) {
  const int N = s->n_sites;
  const int K = s->n_matsubara;
  const double kT = kBoltzmannCmPerK * s->temperature_K * kCmToRadFs;
  m->modes.clear();
  m->delta.assign(N, 0.0);
  for (int site = 0; site < N; ++site) {
    const double lam = s->lambda_cm[site] * kCmToRadFs;
    const double gam = 1.0 / s->gamma_inv_fs[site];
    const double cot = 1.0 / std::tan(gam / (2.0 * kT));
    Mode d;
    d.site = site;
    d.nu = gam;
    if (s->theta_form == 0) {
      d.c = cplx(lam * gam * cot, -lam * gam);
    } else {
      d.c = cplx(2.0 * lam * kT, -lam * gam);
    }
    m->modes.push_back(d);
    double matsubara_sum = 0.0;  // sum_{k<=K} c_k / nu_k
    for (int k = 1; k <= K; ++k) {
      Mode mk;
      mk.site = site;
      mk.nu = 2.0 * kPi * k * kT;
      const double ck = 4.0 * lam * gam * kT * mk.nu / (mk.nu * mk.nu - gam * gam);
      mk.c = cplx(ck, 0.0);
      matsubara_sum += ck / mk.nu;
      m->modes.push_back(mk);
    }
    if (s->low_temp_correction) {
      m->delta[site] = 2.0 * lam * kT / gam - lam * cot - matsubara_sum;
    }
  }
  return true;
}

// Hierarchy enumeration, breadth first from the zero multi-index: tier t+1 is
// every n + e_m with n in tier t, in order of discovery.  (The GPU library
// uses a different order; comparisons go through the multi-indices.)
void enumerate(int M, int D, Model* m) {
  m->ados.clear();
  m->index.clear();
  std::vector<int> zero(M, 0);
  m->index[zero] = 0;
  m->ados.push_back(zero);
  size_t tier_begin = 0, tier_end = 1;
  for (int t = 0; t < D; ++t) {
    for (size_t i = tier_begin; i < tier_end; ++i) {
      for (int mode = 0; mode < M; ++mode) {
        std::vector<int> n = m->ados[i];
        n[mode] += 1;
        if (m->index.find(n) == m->index.end()) {
          m->index[n] = static_cast<int>(m->ados.size());
          m->ados.push_back(n);
        }
      }
    }
    tier_begin = tier_end;
    tier_end = m->ados.size();
  }
  const int n_ado = static_cast<int>(m->ados.size());
  m->up.assign(n_ado, std::vector<int>(M, -1));
  m->down.assign(n_ado, std::vector<int>(M, -1));
  for (int i = 0; i < n_ado; ++i) {
    for (int mode = 0; mode < M; ++mode) {
      std::vector<int> n = m->ados[i];
      n[mode] += 1;
      std::map<std::vector<int>, int>::const_iterator it = m->index.find(n);
      if (it != m->index.end()) m->up[i][mode] = it->second;
      if (m->ados[i][mode] > 0) {
        n[mode] -= 2;
        m->down[i][mode] = m->index.find(n)->second;
      }
    }
  }
}

bool build_model(const oracle_system* s, int depth, Model* m) {
  if (!s || s->n_sites < 1 || depth < 0 || s->n_matsubara < 0) return false;
  const int N = s->n_sites;
  m->N = N;
  m->depth = depth;
  m->H.assign(N * N, cplx(0, 0));
  for (int i = 0; i < N * N; ++i)
    m->H[i] = cplx(s->hamiltonian_cm[2 * i], s->hamiltonian_cm[2 * i + 1]) * kCmToRadFs;
  m->trap.assign(N, 0.0);
  m->rec.assign(N, 0.0);
  for (int a = 0; a < N; ++a) {
    if (s->trap_rate_per_ps) m->trap[a] = s->trap_rate_per_ps[a] * 1e-3;
    if (s->recomb_rate_per_ps) m->rec[a] = s->recomb_rate_per_ps[a] * 1e-3;
  }
  make_modes(s, m);
  enumerate(static_cast<int>(m->modes.size()), depth, m);
  return true;
}

// --- plain matrix helpers -------------------------------------------------

Mat matmul(const Mat& A, const Mat& B, int N) {
  Mat C(N * N, cplx(0, 0));
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j) C[i * N + j] += A[i * N + k] * B[k * N + j];
  return C;
}

Mat dagger(const Mat& A, int N) {
  Mat B(N * N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) B[i * N + j] = std::conj(A[j * N + i]);
  return B;
}

// V_s X: only row s of X survives.
Mat proj_left(int s, const Mat& X, int N) {
  Mat R(N * N, cplx(0, 0));
  for (int j = 0; j < N; ++j) R[s * N + j] = X[s * N + j];
  return R;
}

// X V_s: only column s of X survives.
Mat proj_right(int s, const Mat& X, int N) {
  Mat R(N * N, cplx(0, 0));
  for (int i = 0; i < N; ++i) R[i * N + s] = X[i * N + s];
  return R;
}

void axpy(Mat* y, cplx a, const Mat& x) {
  for (size_t i = 0; i < y->size(); ++i) (*y)[i] += a * x[i];
}

// --- right-hand side -------------------------------------------------------

struct State {
  std::vector<Mat> sigma;  // per ADO
  double p_trap = 0.0, p_rec = 0.0, q = 0.0;
};

// Effective Hamiltonian H - (i/2) diag(Gamma_trap + Gamma_rec).
Mat effective_hamiltonian(const Model& m) {
  Mat Heff = m.H;
  for (int a = 0; a < m.N; ++a)
    Heff[a * m.N + a] -= cplx(0.0, 0.5 * (m.trap[a] + m.rec[a]));
  return Heff;
}

// d sigma_n / dt of eq:lab8 (with the readings listed at the top of the file).
Mat rhs_one(const Model& m, const Mat& Heff, const Mat& HeffDag, const State& x, int n) {
  const int N = m.N;
  const int M = static_cast<int>(m.modes.size());
  const Mat& X = x.sigma[n];
  const cplx I(0.0, 1.0);
  // Coherent part with the sinks: -i (Heff X - X Heff^dagger).
  Mat out = matmul(Heff, X, N);
  Mat XH = matmul(X, HeffDag, N);
  for (int k = 0; k < N * N; ++k) out[k] = -I * (out[k] - XH[k]);
  // Damping -sum_m n_m nu_m.
  double damp = 0.0;
  for (int mode = 0; mode < M; ++mode) damp += m.ados[n][mode] * m.modes[mode].nu;
  axpy(&out, cplx(-damp, 0.0), X);
  // Low-temperature correction: -Delta_s [V_s, [V_s, X]].
  for (int s = 0; s < N; ++s) {
    if (m.delta[s] == 0.0) continue;
    Mat C(N * N);  // [V_s, X]
    Mat L = proj_left(s, X, N), R = proj_right(s, X, N);
    for (int k = 0; k < N * N; ++k) C[k] = L[k] - R[k];
    Mat L2 = proj_left(s, C, N), R2 = proj_right(s, C, N);
    for (int k = 0; k < N * N; ++k) out[k] -= m.delta[s] * (L2[k] - R2[k]);
  }
  for (int mode = 0; mode < M; ++mode) {
    const int s = m.modes[mode].site;
    // Coupling to the deeper ADO: + i [V_s, sigma_{n+e_m}] (scaled form:
    // w_{n+e_m} / w_n = sqrt((n_m + 1)|c_m|) times it).
    const cplx c = m.modes[mode].c;
    const int u = m.up[n][mode];
    if (u >= 0) {
      const Mat& Y = x.sigma[u];
      Mat L = proj_left(s, Y, N), R = proj_right(s, Y, N);
      const double wu = m.scaled ? std::sqrt((m.ados[n][mode] + 1.0) * std::abs(c)) : 1.0;
      for (int k = 0; k < N * N; ++k) out[k] += wu * (I * (L[k] - R[k]));
    }
    // Coupling to the shallower ADO: + n_m i (c V_s Z - c* Z V_s) (scaled
    // form: n_m w_{n-e_m} / w_n = sqrt(n_m / |c_m|) in place of n_m).
    const int d = m.down[n][mode];
    if (d >= 0) {
      const Mat& Z = x.sigma[d];
      const double nm = m.scaled ? std::sqrt(m.ados[n][mode] / std::abs(c)) : m.ados[n][mode];
      Mat L = proj_left(s, Z, N), R = proj_right(s, Z, N);
      for (int k = 0; k < N * N; ++k) out[k] += nm * I * (c * L[k] - std::conj(c) * R[k]);
    }
  }
  return out;
}

void rhs(const Model& m, const State& x, State* f, int n_threads) {
  const int n_ado = static_cast<int>(m.ados.size());
  const Mat Heff = effective_hamiltonian(m);
  const Mat HeffDag = dagger(Heff, m.N);
  f->sigma.resize(n_ado);
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(n_threads > 0 ? n_threads : 1)
#endif
  for (int n = 0; n < n_ado; ++n) f->sigma[n] = rhs_one(m, Heff, HeffDag, x, n);
  (void)n_threads;
  // Populations that leave through the sinks (eq:lab2, eq:lab3).
  double ft = 0.0, fr = 0.0;
  for (int a = 0; a < m.N; ++a) {
    const double pop = x.sigma[0][a * m.N + a].real();
    ft += m.trap[a] * pop;
    fr += m.rec[a] * pop;
  }
  f->p_trap = ft;
  f->p_rec = fr;
  f->q = x.p_trap;
}

// y + a * k
State combine(const State& y, double a, const State& k) {
  State r = y;
  for (size_t n = 0; n < r.sigma.size(); ++n) axpy(&r.sigma[n], cplx(a, 0.0), k.sigma[n]);
  r.p_trap += a * k.p_trap;
  r.p_rec += a * k.p_rec;
  r.q += a * k.q;
  return r;
}

// One classic RK4 step.
void rk4_step(const Model& m, State* y, double dt, int n_threads) {
  State k1, k2, k3, k4;
  rhs(m, *y, &k1, n_threads);
  rhs(m, combine(*y, 0.5 * dt, k1), &k2, n_threads);
  rhs(m, combine(*y, 0.5 * dt, k2), &k3, n_threads);
  rhs(m, combine(*y, dt, k3), &k4, n_threads);
  for (size_t n = 0; n < y->sigma.size(); ++n) {
    Mat& s = y->sigma[n];
    for (size_t e = 0; e < s.size(); ++e)
      s[e] += (dt / 6.0) * (k1.sigma[n][e] + 2.0 * k2.sigma[n][e] + 2.0 * k3.sigma[n][e] +
                            k4.sigma[n][e]);
  }
  y->p_trap += (dt / 6.0) * (k1.p_trap + 2.0 * k2.p_trap + 2.0 * k3.p_trap + k4.p_trap);
  y->p_rec += (dt / 6.0) * (k1.p_rec + 2.0 * k2.p_rec + 2.0 * k3.p_rec + k4.p_rec);
  y->q += (dt / 6.0) * (k1.q + 2.0 * k2.q + 2.0 * k3.q + k4.q);
}

// The filter: every ADO n != 0 whose entries (real and imaginary parts) are
// all below tol in absolute value becomes zero.
void filter_state(State* y, double tol) {
  for (size_t n = 1; n < y->sigma.size(); ++n) {
    double mx = 0.0;
    for (const cplx& v : y->sigma[n]) mx = std::fmax(mx, std::fmax(std::fabs(v.real()), std::fabs(v.imag())));
    if (mx < tol)
      for (cplx& v : y->sigma[n]) v = cplx(0.0, 0.0);
  }
}

void load_state(const Model& m, const double* in, State* x) {
  const int N2 = m.N * m.N;
  const size_t n_ado = m.ados.size();
  x->sigma.assign(n_ado, Mat(N2));
  for (size_t n = 0; n < n_ado; ++n)
    for (int k = 0; k < N2; ++k) x->sigma[n][k] = cplx(in[2 * (n * N2 + k)], in[2 * (n * N2 + k) + 1]);
  const double* sc = in + 2 * n_ado * N2;
  x->p_trap = sc[0];
  x->p_rec = sc[1];
  x->q = sc[2];
}

void store_state(const Model& m, const State& x, double* out) {
  const int N2 = m.N * m.N;
  const size_t n_ado = m.ados.size();
  for (size_t n = 0; n < n_ado; ++n)
    for (int k = 0; k < N2; ++k) {
      out[2 * (n * N2 + k)] = x.sigma[n][k].real();
      out[2 * (n * N2 + k) + 1] = x.sigma[n][k].imag();
    }
  double* sc = out + 2 * n_ado * N2;
  sc[0] = x.p_trap;
  sc[1] = x.p_rec;
  sc[2] = x.q;
}

}  // namespace

extern "C" {

// Number of ADOs for n_modes modes and depth D, by enumeration.
int oracle_count(const oracle_system* s, int32_t depth, int64_t* n_ados, int32_t* n_modes) {
  Model m;
  if (!build_model(s, depth, &m)) return -1;
  if (n_ados) *n_ados = static_cast<int64_t>(m.ados.size());
  if (n_modes) *n_modes = static_cast<int32_t>(m.modes.size());
  return 0;
}

// Bath modes (site, c, nu) in mode order and the correction residual per site.
int oracle_modes(const oracle_system* s, int32_t* site, double* c_re, double* c_im, double* nu,
                 double* delta) {
  Model m;
  if (!s || s->n_sites < 1) return -1;
  m.N = s->n_sites;
  make_modes(s, &m);
  for (size_t k = 0; k < m.modes.size(); ++k) {
    if (site) site[k] = m.modes[k].site;
    if (c_re) c_re[k] = m.modes[k].c.real();
    if (c_im) c_im[k] = m.modes[k].c.imag();
    if (nu) nu[k] = m.modes[k].nu;
  }
  if (delta)
    for (int a = 0; a < m.N; ++a) delta[a] = m.delta[a];
  return 0;
}

// Multi-indices in the oracle's own order: out[i * M + mode].
int oracle_enumerate(const oracle_system* s, int32_t depth, int32_t* out) {
  Model m;
  if (!build_model(s, depth, &m)) return -1;
  const size_t M = m.modes.size();
  for (size_t i = 0; i < m.ados.size(); ++i)
    for (size_t k = 0; k < M; ++k) out[i * M + k] = m.ados[i][k];
  return 0;
}

// Right-hand side for an arbitrary state (not necessarily Hermitian).
// State layout: n_ado blocks of N*N complex (interleaved re, im), row-major,
// in the oracle's order, followed by 3 doubles (P_trap, P_rec, Q).
// scaled = 1: the state holds the scaled ADOs and the scaled equations apply.
int oracle_rhs_scaled(const oracle_system* s, int32_t depth, int32_t scaled,
                      const double* state_in, double* state_out, int32_t n_threads) {
  Model m;
  if (!build_model(s, depth, &m)) return -1;
  m.scaled = scaled != 0;
  State x, f;
  load_state(m, state_in, &x);
  rhs(m, x, &f, n_threads);
  store_state(m, f, state_out);
  return 0;
}

int oracle_rhs(const oracle_system* s, int32_t depth, const double* state_in, double* state_out,
               int32_t n_threads) {
  Model m;
  if (!build_model(s, depth, &m)) return -1;
  State x, f;
  load_state(m, state_in, &x);
  rhs(m, x, &f, n_threads);
  store_state(m, f, state_out);
  return 0;
}

// Propagates rho0 (N*N complex) with classic RK4 for n_steps steps of dt_fs.
//   rho_out      [(n_steps / record_every) + 1][N][N] complex, or NULL
//   scalars_out  [3] = P_trap, P_rec, Q at the end, or NULL
//   state_out    full final state as in oracle_rhs, or NULL
//   state_in     full initial state as in oracle_rhs (overrides rho0), or NULL
//   scaled       1: propagate the scaled ADOs (state_in / state_out hold them)
//   filter_tol   > 0: filter the state after every step
int oracle_propagate_scaled(const oracle_system* s, int32_t depth, int32_t scaled,
                            double filter_tol, const double* rho0, double dt_fs, int64_t n_steps,
                            int64_t record_every, double* rho_out, double* scalars_out,
                            double* state_out, const double* state_in, int32_t n_threads) {
  Model m;
  if (!build_model(s, depth, &m)) return -1;
  if (dt_fs <= 0.0 || n_steps < 0 || record_every < 1 || !(filter_tol >= 0.0)) return -1;
  m.scaled = scaled != 0;
  m.filter_tol = filter_tol;
  const int N2 = m.N * m.N;
  State y;
  if (state_in) {
    load_state(m, state_in, &y);
  } else {
    y.sigma.assign(m.ados.size(), Mat(N2, cplx(0, 0)));
    for (int k = 0; k < N2; ++k) y.sigma[0][k] = cplx(rho0[2 * k], rho0[2 * k + 1]);
  }
  int64_t rec = 0;
  if (rho_out) {
    for (int k = 0; k < N2; ++k) {
      rho_out[2 * k] = y.sigma[0][k].real();
      rho_out[2 * k + 1] = y.sigma[0][k].imag();
    }
    rec = 1;
  }
  for (int64_t step = 1; step <= n_steps; ++step) {
    rk4_step(m, &y, dt_fs, n_threads);
    if (m.filter_tol > 0.0) filter_state(&y, m.filter_tol);
    if (rho_out && step % record_every == 0) {
      double* o = rho_out + 2 * rec * N2;
      for (int k = 0; k < N2; ++k) {
        o[2 * k] = y.sigma[0][k].real();
        o[2 * k + 1] = y.sigma[0][k].imag();
      }
      ++rec;
    }
  }
  if (scalars_out) {
    scalars_out[0] = y.p_trap;
    scalars_out[1] = y.p_rec;
    scalars_out[2] = y.q;
  }
  if (state_out) store_state(m, y, state_out);
  return 0;
}

int oracle_propagate(const oracle_system* s, int32_t depth, const double* rho0, double dt_fs,
                     int64_t n_steps, int64_t record_every, double* rho_out, double* scalars_out,
                     double* state_out, const double* state_in, int32_t n_threads) {
  return oracle_propagate_scaled(s, depth, 0, 0.0, rho0, dt_fs, n_steps, record_every, rho_out,
                                 scalars_out, state_out, state_in, n_threads);
}

}  // extern "C"
