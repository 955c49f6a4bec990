// stage_kernels.hip -- fused RK4-stage kernels of the HEOM propagation (gfx950).
//
// One launch evaluates the right-hand side of eq:lab8 (paper, Appendix A) for
// every ADO of a set of instances and applies one RK4 stage to it.
//
// RK4 (Appendix B) on the linear, time-independent generator L of the
// hierarchy is the degree-4 Taylor polynomial of exp(dt L).  It is evaluated
// in nested form,
//     u1 = y + dt/4 L y,  u2 = y + dt/3 L u1,  u3 = y + dt/2 L u2,
//     y <- y + dt L u3,
// which equals the classic k1..k4 combination in exact arithmetic but needs
// only the state y and one stage input per stage: 11 ADO transfers per step
// instead of 16.  Stage s reads its input from buffer in(s) = {y, A, B, A} and
// writes out(s) = {A, B, A, y}; no stage reads what it writes except the last,
// whose in-place update of y touches only each lane's own ADO.
//
// Right-hand side of ADO n, element (a, b), with X the stage input, V_s the
// projector on site s, modes m = (site s(m), k) with amplitude c_m and rate
// nu_m, and Y^m = X_{n+e_m}, Z^m = X_{n-e_m}:
//   -i sum_c (H_ac X_cb - X_ac H_cb)                      coherent part
//   - (sum_m n_m nu_m) X_ab                               damping
//   - (Gamma_a + Gamma_b)/2 X_ab                           sinks (eq:lab2, eq:lab3)
//   - (1 - delta_ab)(Delta_a + Delta_b) X_ab               low-temperature correction
//   + i sum_{m in a} Y^m_ab - i sum_{m in b} Y^m_ab         i [V, X_{n+e_m}]
//   + i sum_{m in a} n_m c_m Z^m_ab - i sum_{m in b} n_m conj(c_m) Z^m_ab
// Every V_s is a site projector, so the bath couplings are element-wise: each
// output element needs the same element of at most 2(K+1) deeper and 2(K+1)
// shallower neighbours.  Every ADO is Hermitian, so only the upper triangle is
// stored (N*N reals per ADO, see heom_internal.h).
//
// Lane mapping: one lane per ADO, consecutive lanes on consecutive ADOs.  Each
// element of the stored state is a plane over ADOs, so every self access of a
// wave is one contiguous 512-byte (FP64) segment, and neighbour gathers (whose
// indices are nearly consecutive in the lexicographic order of the hierarchy)
// touch few cache lines.  The ADO of sigma_0 (lane 0 of its instance) also
// integrates the sink populations and writes the history record.
//
// Two kernels:
//  * stage_fixed<N, KP>: N <= 8 sites, K+1 = KP modes per site, real H.  The
//    ADO's N*N reals live in registers, every loop is unrolled at compile time
//    and H, c, nu are wave-uniform scalar loads.
//  * stage_generic: any N <= 64, any K, complex H; reads the stage input
//    straight from the planes (all such reads are coalesced across lanes).
#include <hip/hip_runtime.h>

#include "heom_internal.h"

namespace heom {
namespace {

template <typename C>
struct Cx {
  C re, im;
};

// Buffers used by stage s.
struct StageBufs {
  const void *x;   // stage input planes
  const void *y;   // state planes (may alias x at stage 0)
  void *out;       // output planes
  const double *x0, *y0;  // FP64 sigma_0 (mixed precision)
  double *out0;
  const double *xs, *ys;  // scalars
  double *outs;
};

__device__ __forceinline__ StageBufs stage_bufs(const InstDesc &d, int stage) {
  StageBufs b;
  switch (stage) {
    case 0:
      b.x = d.y; b.y = d.y; b.out = d.a;
      b.x0 = d.y0; b.y0 = d.y0; b.out0 = d.a0;
      b.xs = d.sc_y; b.ys = d.sc_y; b.outs = d.sc_a;
      break;
    case 1:
      b.x = d.a; b.y = d.y; b.out = d.b;
      b.x0 = d.a0; b.y0 = d.y0; b.out0 = d.b0;
      b.xs = d.sc_a; b.ys = d.sc_y; b.outs = d.sc_b;
      break;
    case 2:
      b.x = d.b; b.y = d.y; b.out = d.a;
      b.x0 = d.b0; b.y0 = d.y0; b.out0 = d.a0;
      b.xs = d.sc_b; b.ys = d.sc_y; b.outs = d.sc_a;
      break;
    default:
      b.x = d.a; b.y = d.y; b.out = d.y;
      b.x0 = d.a0; b.y0 = d.y0; b.out0 = d.y0;
      b.xs = d.sc_a; b.ys = d.sc_y; b.outs = d.sc_y;
      break;
  }
  return b;
}

__host__ __device__ constexpr int re_plane(int N, int a, int b) {
  // a < b
  return N + 2 * (a * N - a * (a + 1) / 2 + (b - a - 1));
}

// Sink flux of sigma_0 and the scalar part of one stage, then (last stage) the
// history record.  `x0e(e)` returns packed element e of the stage input of
// sigma_0, `newy(e)` the packed element e just written to the state.
template <typename LoadX>
__device__ __forceinline__ void scalar_update(const InstDesc &d, const StageBufs &b, int N,
                                              double coef, LoadX x0e) {
  const ParamOffsets o = param_offsets(N, d.M);
  double ft = 0.0, fr = 0.0;
  for (int s = 0; s < N; ++s) {
    const double pop = x0e(s);
    ft += d.params[o.trap + s] * pop;
    fr += d.params[o.rec + s] * pop;
  }
  const double xq = b.xs[0];
  const double y_t = b.ys[0], y_r = b.ys[1], y_q = b.ys[2];
  b.outs[0] = y_t + coef * ft;
  b.outs[1] = y_r + coef * fr;
  b.outs[2] = y_q + coef * xq;
}

// ---------------------------------------------------------------------------
// Specialised kernel: compile-time N and modes per site, real Hamiltonian.
// ---------------------------------------------------------------------------

template <int N, int KP, typename C, typename T, bool MIXED, bool IS0>
__device__ __forceinline__ void update_fixed(const InstDesc &d, int64_t i, int stage, double coef_d,
                                             int hist_slot) {
  constexpr int N2 = N * N;
  constexpr int M = N * KP;
  constexpr ParamOffsets o = {0,
                              N * N,
                              2 * N * N,
                              2 * N * N + N,
                              2 * N * N + 2 * N,
                              2 * N * N + 3 * N,
                              2 * N * N + 4 * N,
                              2 * N * N + 4 * N + M,
                              2 * N * N + 4 * N + 2 * M,
                              2 * N * N + 4 * N + 3 * M,
                              2 * N * N + 4 * N + 3 * M + N * N};
  const StageBufs bufs = stage_bufs(d, stage);
  const int64_t S = d.stride;
  const T *__restrict__ X = static_cast<const T *>(bufs.x);
  const T *__restrict__ Yp = static_cast<const T *>(bufs.y);
  T *__restrict__ Out = static_cast<T *>(bufs.out);
  const double *__restrict__ P = d.params;
  const C coef = static_cast<C>(coef_d);

  // Own stage input, packed.
  C x[N2];
#pragma unroll
  for (int e = 0; e < N2; ++e) {
    if constexpr (MIXED && IS0)
      x[e] = bufs.x0[e];
    else
      x[e] = static_cast<C>(X[e * S + i]);
  }
  // Neighbour indices and occupations.
  int32_t up[M], dn[M];
  C occ[M];
  C damp = C(0);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    up[m] = d.up[m * S + i];
    dn[m] = d.down[m * S + i];
    occ[m] = static_cast<C>(d.occ[m * S + i]);
    damp += occ[m] * static_cast<C>(P[o.nu + m]);
  }

  auto elem = [&](int c, int b) -> Cx<C> {
    if (c == b) return {x[c], C(0)};
    if (c < b) {
      const int e = re_plane(N, c, b);
      return {x[e], x[e + 1]};
    }
    const int e = re_plane(N, b, c);
    return {x[e], -x[e + 1]};
  };

#pragma unroll
  for (int a = 0; a < N; ++a) {
#pragma unroll
    for (int b = a; b < N; ++b) {
      const int e = (a == b) ? a : re_plane(N, a, b);
      // Coherent part: s = sum_c H_ac X_cb - X_ac H_cb; contribution -i s.
      C sr = C(0), si = C(0);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const C hac = static_cast<C>(P[o.h_re + a * N + c]);
        const C hcb = static_cast<C>(P[o.h_re + c * N + b]);
        const Cx<C> xcb = elem(c, b);
        const Cx<C> xac = elem(a, c);
        sr += hac * xcb.re - xac.re * hcb;
        si += hac * xcb.im - xac.im * hcb;
      }
      C ar = si, ai = -sr;
      const Cx<C> xab = elem(a, b);
      C dec = damp + static_cast<C>(P[o.half_gamma + a]) + static_cast<C>(P[o.half_gamma + b]);
      if (a != b) dec += static_cast<C>(P[o.delta + a]) + static_cast<C>(P[o.delta + b]);
      ar -= dec * xab.re;
      ai -= dec * xab.im;
      // Deeper neighbours: + i Y (mode of site a) - i Y (mode of site b).
      if (a != b) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          const int ja = up[a * KP + k];
          if (ja >= 0) {
            const C vr = static_cast<C>(X[e * S + ja]);
            const C vi = static_cast<C>(X[(e + 1) * S + ja]);
            ar -= vi;
            ai += vr;
          }
          const int jb = up[b * KP + k];
          if (jb >= 0) {
            const C vr = static_cast<C>(X[e * S + jb]);
            const C vi = static_cast<C>(X[(e + 1) * S + jb]);
            ar += vi;
            ai -= vr;
          }
        }
      }
      // Shallower neighbours: + i n c Z (site a) - i n conj(c) Z (site b).
#pragma unroll
      for (int k = 0; k < KP; ++k) {
        const int ma = a * KP + k;
        const int mb = b * KP + k;
        const int ja = dn[ma];
        if (ja >= 0) {
          const C vr = static_cast<C>(X[e * S + ja]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[(e + 1) * S + ja]);
          const C cr = occ[ma] * static_cast<C>(P[o.c_re + ma]);
          const C ci = occ[ma] * static_cast<C>(P[o.c_im + ma]);
          // i (cr + i ci)(vr + i vi) = -(ci vr + cr vi) + i (cr vr - ci vi)
          ar -= ci * vr + cr * vi;
          ai += cr * vr - ci * vi;
        }
        const int jb = dn[mb];
        if (jb >= 0) {
          const C vr = static_cast<C>(X[e * S + jb]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[(e + 1) * S + jb]);
          const C cr = occ[mb] * static_cast<C>(P[o.c_re + mb]);
          const C ci = occ[mb] * static_cast<C>(P[o.c_im + mb]);
          // -i (cr - i ci)(vr + i vi) = -(ci vr - cr vi) ... expanded:
          // (cr - i ci)(vr + i vi) = (cr vr + ci vi) + i (cr vi - ci vr)
          // -i * that = (cr vi - ci vr) - i (cr vr + ci vi)
          ar += cr * vi - ci * vr;
          ai -= cr * vr + ci * vi;
        }
      }
      // RK4 stage: out = y + coef * rhs.
      C yr, yi;
      if (stage == 0) {
        yr = xab.re;
        yi = xab.im;
      } else if constexpr (MIXED && IS0) {
        yr = bufs.y0[e];
        yi = (a == b) ? C(0) : bufs.y0[e + 1];
      } else {
        yr = static_cast<C>(Yp[e * S + i]);
        yi = (a == b) ? C(0) : static_cast<C>(Yp[(e + 1) * S + i]);
      }
      const C nr = yr + coef * ar;
      const C ni = yi + coef * ai;
      if constexpr (MIXED && IS0) {
        bufs.out0[e] = nr;
        Out[e * S + i] = static_cast<T>(nr);
        if (a != b) {
          bufs.out0[e + 1] = ni;
          Out[(e + 1) * S + i] = static_cast<T>(ni);
        }
      } else {
        Out[e * S + i] = static_cast<T>(nr);
        if (a != b) Out[(e + 1) * S + i] = static_cast<T>(ni);
      }
      if constexpr (IS0) {
        if (stage == 3 && hist_slot >= 0) {
          double *h = d.hist + static_cast<int64_t>(hist_slot) * (N2 + kScalars);
          h[e] = static_cast<double>(nr);
          if (a != b) h[e + 1] = static_cast<double>(ni);
        }
      }
    }
  }
  if constexpr (IS0) {
    scalar_update(d, bufs, N, coef_d, [&](int s) { return static_cast<double>(x[s]); });
    if (stage == 3 && hist_slot >= 0) {
      double *h = d.hist + static_cast<int64_t>(hist_slot) * (N2 + kScalars);
      h[N2 + 0] = bufs.outs[0];
      h[N2 + 1] = bufs.outs[1];
      h[N2 + 2] = bufs.outs[2];
    }
  }
}

template <int N, int KP, typename T>
__global__ void __launch_bounds__(256) stage_fixed(const InstDesc *__restrict__ descs,
                                                   const WorkItem *__restrict__ work, int stage,
                                                   double coef, int hist_slot) {
  const WorkItem w = work[blockIdx.x];
  const InstDesc &d = descs[w.inst];
  const int64_t i = static_cast<int64_t>(w.first) + threadIdx.x;
  if (i >= d.n_ados) return;
  constexpr bool MIXED = sizeof(T) == 4;
  if (i == 0)
    update_fixed<N, KP, double, T, MIXED, true>(d, i, stage, coef, hist_slot);
  else
    update_fixed<N, KP, T, T, MIXED, false>(d, i, stage, coef, hist_slot);
}

// ---------------------------------------------------------------------------
// Generic kernel: runtime N and modes per site, complex Hermitian H.
// ---------------------------------------------------------------------------

template <typename C, typename T, bool MIXED, bool IS0>
__device__ __forceinline__ void update_generic(const InstDesc &d, int64_t i, int stage,
                                               double coef_d, int hist_slot) {
  const int N = d.N;
  const int M = d.M;
  const int KP = d.KP;
  const int N2 = N * N;
  const ParamOffsets o = param_offsets(N, M);
  const StageBufs bufs = stage_bufs(d, stage);
  const int64_t S = d.stride;
  const T *__restrict__ X = static_cast<const T *>(bufs.x);
  const T *__restrict__ Yp = static_cast<const T *>(bufs.y);
  T *__restrict__ Out = static_cast<T *>(bufs.out);
  const double *__restrict__ P = d.params;
  const C coef = static_cast<C>(coef_d);

  auto ld = [&](int e) -> C {  // own stage input, packed element e
    if constexpr (MIXED && IS0) return bufs.x0[e];
    return static_cast<C>(X[e * S + i]);
  };
  auto elem = [&](int c, int b) -> Cx<C> {
    if (c == b) return {ld(c), C(0)};
    if (c < b) {
      const int e = re_plane(N, c, b);
      return {ld(e), ld(e + 1)};
    }
    const int e = re_plane(N, b, c);
    return {ld(e), -ld(e + 1)};
  };
  C damp = C(0);
  for (int m = 0; m < M; ++m)
    damp += static_cast<C>(d.occ[m * S + i]) * static_cast<C>(P[o.nu + m]);

  for (int a = 0; a < N; ++a) {
    for (int b = a; b < N; ++b) {
      const int e = (a == b) ? a : re_plane(N, a, b);
      C sr = C(0), si = C(0);
      for (int c = 0; c < N; ++c) {
        const C hr_ac = static_cast<C>(P[o.h_re + a * N + c]);
        const C hi_ac = static_cast<C>(P[o.h_im + a * N + c]);
        const C hr_cb = static_cast<C>(P[o.h_re + c * N + b]);
        const C hi_cb = static_cast<C>(P[o.h_im + c * N + b]);
        const Cx<C> xcb = elem(c, b);
        const Cx<C> xac = elem(a, c);
        // H_ac X_cb - X_ac H_cb
        sr += hr_ac * xcb.re - hi_ac * xcb.im - (xac.re * hr_cb - xac.im * hi_cb);
        si += hr_ac * xcb.im + hi_ac * xcb.re - (xac.re * hi_cb + xac.im * hr_cb);
      }
      C ar = si, ai = -sr;
      const Cx<C> xab = elem(a, b);
      C dec = damp + static_cast<C>(P[o.half_gamma + a]) + static_cast<C>(P[o.half_gamma + b]);
      if (a != b) dec += static_cast<C>(P[o.delta + a]) + static_cast<C>(P[o.delta + b]);
      ar -= dec * xab.re;
      ai -= dec * xab.im;
      for (int k = 0; k < KP; ++k) {
        const int ma = a * KP + k;
        const int mb = b * KP + k;
        if (a != b) {
          const int ja = d.up[ma * S + i];
          if (ja >= 0) {
            ar -= static_cast<C>(X[(e + 1) * S + ja]);
            ai += static_cast<C>(X[e * S + ja]);
          }
          const int jb = d.up[mb * S + i];
          if (jb >= 0) {
            ar += static_cast<C>(X[(e + 1) * S + jb]);
            ai -= static_cast<C>(X[e * S + jb]);
          }
        }
        const int ja = d.down[ma * S + i];
        if (ja >= 0) {
          const C n = static_cast<C>(d.occ[ma * S + i]);
          const C vr = static_cast<C>(X[e * S + ja]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[(e + 1) * S + ja]);
          const C cr = n * static_cast<C>(P[o.c_re + ma]);
          const C ci = n * static_cast<C>(P[o.c_im + ma]);
          ar -= ci * vr + cr * vi;
          ai += cr * vr - ci * vi;
        }
        const int jb = d.down[mb * S + i];
        if (jb >= 0) {
          const C n = static_cast<C>(d.occ[mb * S + i]);
          const C vr = static_cast<C>(X[e * S + jb]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[(e + 1) * S + jb]);
          const C cr = n * static_cast<C>(P[o.c_re + mb]);
          const C ci = n * static_cast<C>(P[o.c_im + mb]);
          ar += cr * vi - ci * vr;
          ai -= cr * vr + ci * vi;
        }
      }
      C yr, yi;
      if (stage == 0) {
        yr = xab.re;
        yi = xab.im;
      } else if constexpr (MIXED && IS0) {
        yr = bufs.y0[e];
        yi = (a == b) ? C(0) : bufs.y0[e + 1];
      } else {
        yr = static_cast<C>(Yp[e * S + i]);
        yi = (a == b) ? C(0) : static_cast<C>(Yp[(e + 1) * S + i]);
      }
      const C nr = yr + coef * ar;
      const C ni = yi + coef * ai;
      // The stage input is still read below (elem) by this lane only after all
      // of its own writes: the last stage writes y in place, but y is never the
      // stage input of the last stage, so the reads above stay valid.
      if constexpr (MIXED && IS0) {
        bufs.out0[e] = nr;
        if (a != b) bufs.out0[e + 1] = ni;
      }
      Out[e * S + i] = static_cast<T>(nr);
      if (a != b) Out[(e + 1) * S + i] = static_cast<T>(ni);
      if constexpr (IS0) {
        if (stage == 3 && hist_slot >= 0) {
          double *h = d.hist + static_cast<int64_t>(hist_slot) * (N2 + kScalars);
          h[e] = static_cast<double>(nr);
          if (a != b) h[e + 1] = static_cast<double>(ni);
        }
      }
    }
  }
  if constexpr (IS0) {
    scalar_update(d, bufs, N, coef_d, [&](int s) { return static_cast<double>(ld(s)); });
    if (stage == 3 && hist_slot >= 0) {
      double *h = d.hist + static_cast<int64_t>(hist_slot) * (N2 + kScalars);
      h[N2 + 0] = bufs.outs[0];
      h[N2 + 1] = bufs.outs[1];
      h[N2 + 2] = bufs.outs[2];
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) stage_generic(const InstDesc *__restrict__ descs,
                                                     const WorkItem *__restrict__ work, int stage,
                                                     double coef, int hist_slot) {
  const WorkItem w = work[blockIdx.x];
  const InstDesc &d = descs[w.inst];
  const int64_t i = static_cast<int64_t>(w.first) + threadIdx.x;
  if (i >= d.n_ados) return;
  constexpr bool MIXED = sizeof(T) == 4;
  if (i == 0)
    update_generic<double, T, MIXED, true>(d, i, stage, coef, hist_slot);
  else
    update_generic<T, T, MIXED, false>(d, i, stage, coef, hist_slot);
}

// ---------------------------------------------------------------------------
// Initialisation and snapshot kernels.
// ---------------------------------------------------------------------------

// sigma_0 <- rho0 (packed, from the parameter block), every other ADO <- 0,
// scalars <- 0.
template <typename T>
__global__ void __launch_bounds__(256) init_state(const InstDesc *__restrict__ descs,
                                                  const WorkItem *__restrict__ work) {
  const WorkItem w = work[blockIdx.x];
  const InstDesc &d = descs[w.inst];
  const int64_t i = static_cast<int64_t>(w.first) + threadIdx.x;
  if (i >= d.n_ados) return;
  const int N2 = d.N * d.N;
  const ParamOffsets o = param_offsets(d.N, d.M);
  T *y = static_cast<T *>(d.y);
  for (int e = 0; e < N2; ++e) y[e * d.stride + i] = (i == 0) ? static_cast<T>(d.params[o.rho0 + e]) : T(0);
  if (i == 0) {
    if (sizeof(T) == 4)
      for (int e = 0; e < N2; ++e) d.y0[e] = d.params[o.rho0 + e];
    for (int k = 0; k < kScalars; ++k) d.sc_y[k] = 0.0;
  }
}

// Writes the current sigma_0 and scalars of each instance to history slot.
template <typename T>
__global__ void snapshot(const InstDesc *__restrict__ descs, int n_inst, int slot) {
  const int inst = blockIdx.x;
  if (inst >= n_inst) return;
  const InstDesc &d = descs[inst];
  const int N2 = d.N * d.N;
  double *h = d.hist + static_cast<int64_t>(slot) * (N2 + kScalars);
  const T *y = static_cast<const T *>(d.y);
  for (int e = threadIdx.x; e < N2; e += blockDim.x)
    h[e] = (sizeof(T) == 4) ? d.y0[e] : static_cast<double>(y[e * d.stride]);
  if (threadIdx.x < 3) h[N2 + threadIdx.x] = d.sc_y[threadIdx.x];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launch entry points used by the host runtime.
// ---------------------------------------------------------------------------

typedef void (*StageKernel)(const InstDesc *, const WorkItem *, int, double, int);

template <typename T>
static StageKernel fixed_kernel(int N, int KP) {
#define HEOM_CASE(n, kp) \
  if (N == n && KP == kp) return &stage_fixed<n, kp, T>;
  HEOM_CASE(1, 1) HEOM_CASE(2, 1) HEOM_CASE(3, 1) HEOM_CASE(4, 1)
  HEOM_CASE(5, 1) HEOM_CASE(6, 1) HEOM_CASE(7, 1) HEOM_CASE(8, 1)
  HEOM_CASE(1, 2) HEOM_CASE(2, 2) HEOM_CASE(3, 2) HEOM_CASE(4, 2)
  HEOM_CASE(5, 2) HEOM_CASE(6, 2) HEOM_CASE(7, 2) HEOM_CASE(8, 2)
#undef HEOM_CASE
  return nullptr;
}

bool has_fixed_kernel(int N, int KP) { return fixed_kernel<double>(N, KP) != nullptr; }

hipError_t launch_stage(bool fixed, bool mixed, int N, int KP, const InstDesc *descs,
                        const WorkItem *work, int n_items, int block, int stage, double coef,
                        int hist_slot, hipStream_t stream) {
  StageKernel k;
  if (fixed)
    k = mixed ? fixed_kernel<float>(N, KP) : fixed_kernel<double>(N, KP);
  else
    k = mixed ? &stage_generic<float> : &stage_generic<double>;
  if (!k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(n_items), dim3(block), 0, stream, descs, work, stage, coef, hist_slot);
  return hipGetLastError();
}

hipError_t launch_init(bool mixed, const InstDesc *descs, const WorkItem *work, int n_items,
                       int block, hipStream_t stream) {
  if (mixed)
    hipLaunchKernelGGL(init_state<float>, dim3(n_items), dim3(block), 0, stream, descs, work);
  else
    hipLaunchKernelGGL(init_state<double>, dim3(n_items), dim3(block), 0, stream, descs, work);
  return hipGetLastError();
}

hipError_t launch_snapshot(bool mixed, const InstDesc *descs, int n_inst, int slot,
                           hipStream_t stream) {
  if (mixed)
    hipLaunchKernelGGL(snapshot<float>, dim3(n_inst), dim3(64), 0, stream, descs, n_inst, slot);
  else
    hipLaunchKernelGGL(snapshot<double>, dim3(n_inst), dim3(64), 0, stream, descs, n_inst, slot);
  return hipGetLastError();
}

}  // namespace heom
