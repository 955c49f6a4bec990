// stage_kernels.h -- device code of the fused RK4-stage kernels (gfx950),
// included by the kernels_*.hip translation units, which instantiate and
// launch them (split so that the build compiles them in parallel).
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
// Lane mapping: consecutive lanes on consecutive ADOs.  Each element of the
// stored state is a plane over ADOs, so a wave's access to one element of its
// ADOs is a contiguous segment, and neighbour gathers (whose indices are
// nearly consecutive in the lexicographic order of the hierarchy) touch few
// cache lines.  The sigma_0 part of each stage (sink fluxes, P_trap, P_rec, Q)
// is done where ADO 0 is (in FP32-mixed tile launches, by a work item of its
// own that also updates sigma_0 in FP64); history records are written by the
// snapshot kernel.
//
// Kernels:
//  * stage_tile<N, KP, T, shape> (N <= 12, real H): 64-ADO tiles in LDS,
//    compile-time element groups per wave; the default.
//  * stage_wide<T, KP> (N <= 32, real H): 16-ADO tiles in LDS, runtime N;
//    launch shape 5 of the same family (the autotuner chooses).
//  * stage_fixed<N, KP> (N <= 8, real H): one lane per ADO with the ADO's N*N
//    reals in registers; a diagnostic alternative.
//  * stage_generic: any N <= 64, any K, complex H; reads the stage input
//    straight from the planes (all such reads are coalesced across lanes).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "heom_internal.h"

namespace heom {
namespace {

template <typename C>
struct Cx {
  C re, im;
};

// Address-space views of workspace pointers.  Pointers read from the
// descriptor are generic; without these casts every access would be a FLAT
// instruction (counted against both the vector-memory and the LDS counters, so
// each LDS wait would also wait for every outstanding global load) and the
// wave-uniform parameter reads could not become scalar loads.
#define HEOM_GLOBAL __attribute__((address_space(1)))
#define HEOM_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const HEOM_GLOBAL T *gmem(const T *p) {
  return (const HEOM_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ HEOM_GLOBAL T *gmem(T *p) {
  return (HEOM_GLOBAL T *)p;
}
__device__ __forceinline__ const HEOM_CONST double *cmem(const double *p) {
  return (const HEOM_CONST double *)p;
}
__device__ __forceinline__ const HEOM_CONST float *cmem(const float *p) {
  return (const HEOM_CONST float *)p;
}
// Load / store at a 32-bit per-lane byte offset from a wave-uniform base, so
// that the address is one VGPR added to a scalar base (no 64-bit arithmetic
// per lane).  Every plane, table and state buffer is far below 4 GiB.
template <typename T>
__device__ __forceinline__ T ld_off(const HEOM_GLOBAL T *base, uint32_t off) {
  return *(const HEOM_GLOBAL T *)((const HEOM_GLOBAL char *)base + off);
}
// STREAM marks the store non-temporal.  On gfx950 that shortens small,
// latency-bound FP64 stage launches (by about 8 % at 432 tiles) and lengthens
// large, bandwidth-bound ones (by 6-11 % at 3500 tiles and more), so the FP64
// tile kernels are built both ways and the autotuner picks per launch size.
// (A run-time choice between the two stores does not work: the compiler
// merges them into one plain store.)
template <bool STREAM, typename T>
__device__ __forceinline__ void st_off(HEOM_GLOBAL T *base, uint32_t off, T v) {
  HEOM_GLOBAL T *p = (HEOM_GLOBAL T *)((HEOM_GLOBAL char *)base + off);
  if constexpr (STREAM)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
// (Re, Im) of a pair element of one ADO: one access of two values (16 bytes
// in FP64 storage, 8 in FP32) at byte offset `off` of the pair's block.
template <typename T>
using Pair2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ Pair2<T> ld_pair(const HEOM_GLOBAL T *block, uint32_t off) {
  return *(const HEOM_GLOBAL Pair2<T> *)((const HEOM_GLOBAL char *)block + off);
}
// Neighbour index of ADO i along one mode from a table row that is either
// int32 indices (t16 false) or int16 offsets from i (0: no neighbour), read
// with one aligned 32-bit load in both cases (the 16-bit form as the word that
// holds ADOs 2k and 2k + 1, so adjacent lanes share it), no branch: the
// element size and the decoding are wave-uniform selects.  -1: no neighbour.
__device__ __forceinline__ int table_load(const HEOM_GLOBAL char *row, bool t16, uint32_t i) {
  const uint32_t off = t16 ? (i & ~1u) * 2u : i * 4u;
  return *(const HEOM_GLOBAL int32_t *)(row + off);
}
__device__ __forceinline__ int table_decode(int32_t w, bool t16, uint32_t i) {
  if (!t16) return w;
  const int32_t delta = (i & 1u) ? (w >> 16) : ((w << 16) >> 16);
  return delta != 0 ? static_cast<int>(i) + delta : -1;
}

template <bool STREAM, typename T>
__device__ __forceinline__ void st_pair(HEOM_GLOBAL T *block, uint32_t off, T re, T im) {
  HEOM_GLOBAL Pair2<T> *p = (HEOM_GLOBAL Pair2<T> *)((HEOM_GLOBAL char *)block + off);
  Pair2<T> v;
  v.x = re;
  v.y = im;
  if constexpr (STREAM)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

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

// Fused multiply-add, a * b + c with one rounding.  The tile kernel writes
// every multiply-add through this and turns off the compiler's own
// contraction, so its rounding is fixed by the source and does not depend on
// how a launch shape schedules the elements of a wave.
__device__ __forceinline__ double fmad(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Sink flux of sigma_0 and the scalar part of one stage, then (last stage) the
// history record.  `x0e(e)` returns packed element e of the stage input of
// sigma_0, `newy(e)` the packed element e just written to the state.
template <typename LoadX>
__device__ __forceinline__ void scalar_update(const InstDesc &d, const StageBufs &b, int N,
                                              double coef, LoadX x0e) {
#pragma clang fp contract(off)
  const ParamOffsets o = param_offsets(N, d.M);
  double ft = 0.0, fr = 0.0;
  for (int s = 0; s < N; ++s) {
    const double pop = x0e(s);
    ft = fmad(d.params[o.trap + s], pop, ft);
    fr = fmad(d.params[o.rec + s], pop, fr);
  }
  const double xq = b.xs[0];
  const double y_t = b.ys[0], y_r = b.ys[1], y_q = b.ys[2];
  b.outs[0] = fmad(coef, ft, y_t);
  b.outs[1] = fmad(coef, fr, y_r);
  b.outs[2] = fmad(coef, xq, y_q);
}

// Sum over the 64 lanes of a wave, by a butterfly of lane shuffles (every
// lane ends with the same value; the order of additions is fixed).
__device__ __forceinline__ double wave_sum(double v) {
#pragma clang fp contract(off)
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// scalar_update for the LDS-tiled kernels, run by a whole wave with every
// lane active: lane s forms site s's terms of the trap and recombination
// fluxes, and the wave reduces them with shuffles.
template <typename LoadX>
__device__ __forceinline__ void scalar_update_wave(const InstDesc &d, const StageBufs &b, int N,
                                                   double coef, int lane, LoadX x0e) {
#pragma clang fp contract(off)
  const ParamOffsets o = param_offsets(N, d.M);
  double ft = 0.0, fr = 0.0;
  for (int s = lane; s < N; s += 64) {
    const double pop = x0e(s);
    ft = fmad(d.params[o.trap + s], pop, ft);
    fr = fmad(d.params[o.rec + s], pop, fr);
  }
  ft = wave_sum(ft);
  fr = wave_sum(fr);
  if (lane == 0) {
    const double xq = b.xs[0];
    const double y_t = b.ys[0], y_r = b.ys[1], y_q = b.ys[2];
    b.outs[0] = fmad(coef, ft, y_t);
    b.outs[1] = fmad(coef, fr, y_r);
    b.outs[2] = fmad(coef, xq, y_q);
  }
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
      x[e] = static_cast<C>(X[elem_index(N, e, S, i)]);
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
            const C vr = static_cast<C>(X[elem_index(N, e, S, ja)]);
            const C vi = static_cast<C>(X[elem_index(N, e + 1, S, ja)]);
            ar -= vi;
            ai += vr;
          }
          const int jb = up[b * KP + k];
          if (jb >= 0) {
            const C vr = static_cast<C>(X[elem_index(N, e, S, jb)]);
            const C vi = static_cast<C>(X[elem_index(N, e + 1, S, jb)]);
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
          const C vr = static_cast<C>(X[elem_index(N, e, S, ja)]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[elem_index(N, e + 1, S, ja)]);
          const C cr = occ[ma] * static_cast<C>(P[o.c_re + ma]);
          const C ci = occ[ma] * static_cast<C>(P[o.c_im + ma]);
          // i (cr + i ci)(vr + i vi) = -(ci vr + cr vi) + i (cr vr - ci vi)
          ar -= ci * vr + cr * vi;
          ai += cr * vr - ci * vi;
        }
        const int jb = dn[mb];
        if (jb >= 0) {
          const C vr = static_cast<C>(X[elem_index(N, e, S, jb)]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[elem_index(N, e + 1, S, jb)]);
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
        yr = static_cast<C>(Yp[elem_index(N, e, S, i)]);
        yi = (a == b) ? C(0) : static_cast<C>(Yp[elem_index(N, e + 1, S, i)]);
      }
      const C nr = yr + coef * ar;
      const C ni = yi + coef * ai;
      if constexpr (MIXED && IS0) {
        bufs.out0[e] = nr;
        Out[elem_index(N, e, S, i)] = static_cast<T>(nr);
        if (a != b) {
          bufs.out0[e + 1] = ni;
          Out[elem_index(N, e + 1, S, i)] = static_cast<T>(ni);
        }
      } else {
        Out[elem_index(N, e, S, i)] = static_cast<T>(nr);
        if (a != b) Out[elem_index(N, e + 1, S, i)] = static_cast<T>(ni);
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
  if (i == 0 && !(d.flags & kInstNoSigma0))
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
  const HEOM_GLOBAL T *X = gmem(static_cast<const T *>(bufs.x));
  const HEOM_GLOBAL T *Yp = gmem(static_cast<const T *>(bufs.y));
  HEOM_GLOBAL T *Out = gmem(static_cast<T *>(bufs.out));
  const HEOM_CONST double *P = cmem(d.params);
  const HEOM_GLOBAL int32_t *up = gmem(d.up);
  const HEOM_GLOBAL int32_t *down = gmem(d.down);
  const HEOM_GLOBAL uint8_t *occ = gmem(d.occ);
  const HEOM_GLOBAL double *x0 = gmem(bufs.x0);
  const HEOM_GLOBAL double *y0 = gmem(bufs.y0);
  HEOM_GLOBAL double *out0 = gmem(bufs.out0);
  const C coef = static_cast<C>(coef_d);

  auto ld = [&](int e) -> C {  // own stage input, packed element e
    if constexpr (MIXED && IS0) return x0[e];
    return static_cast<C>(X[elem_index(N, e, S, i)]);
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
    damp += static_cast<C>(occ[m * S + i]) * static_cast<C>(P[o.nu + m]);

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
          const int ja = up[ma * S + i];
          if (ja >= 0) {
            ar -= static_cast<C>(X[elem_index(N, e + 1, S, ja)]);
            ai += static_cast<C>(X[elem_index(N, e, S, ja)]);
          }
          const int jb = up[mb * S + i];
          if (jb >= 0) {
            ar += static_cast<C>(X[elem_index(N, e + 1, S, jb)]);
            ai -= static_cast<C>(X[elem_index(N, e, S, jb)]);
          }
        }
        const int ja = down[ma * S + i];
        if (ja >= 0) {
          const C n = static_cast<C>(occ[ma * S + i]);
          const C vr = static_cast<C>(X[elem_index(N, e, S, ja)]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[elem_index(N, e + 1, S, ja)]);
          const C cr = n * static_cast<C>(P[o.c_re + ma]);
          const C ci = n * static_cast<C>(P[o.c_im + ma]);
          ar -= ci * vr + cr * vi;
          ai += cr * vr - ci * vi;
        }
        const int jb = down[mb * S + i];
        if (jb >= 0) {
          const C n = static_cast<C>(occ[mb * S + i]);
          const C vr = static_cast<C>(X[elem_index(N, e, S, jb)]);
          const C vi = (a == b) ? C(0) : static_cast<C>(X[elem_index(N, e + 1, S, jb)]);
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
        yr = static_cast<C>(Yp[elem_index(N, e, S, i)]);
        yi = (a == b) ? C(0) : static_cast<C>(Yp[elem_index(N, e + 1, S, i)]);
      }
      const C nr = yr + coef * ar;
      const C ni = yi + coef * ai;
      // The last stage writes y in place; y is never the stage input of the
      // last stage, so the stage-input reads of later elements stay valid.
      if constexpr (MIXED && IS0) {
        out0[e] = nr;
        if (a != b) out0[e + 1] = ni;
      }
      Out[elem_index(N, e, S, i)] = static_cast<T>(nr);
      if (a != b) Out[elem_index(N, e + 1, S, i)] = static_cast<T>(ni);
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
  if (i == 0 && !(d.flags & kInstNoSigma0))
    update_generic<double, T, MIXED, true>(d, i, stage, coef, hist_slot);
  else
    update_generic<T, T, MIXED, false>(d, i, stage, coef, hist_slot);
}

// ---------------------------------------------------------------------------
// Tile kernel: compile-time N <= 12 and modes per site, real Hamiltonian.
// A workgroup stages the stage input of 64 consecutive ADOs (one "tile") and
// their neighbour tables in LDS; wave w then produces the packed elements
// p = w, w + W, w + 2W, ... for all 64 ADOs.  Each wave's element group is
// known at compile time (the kernel dispatches on the wave index), so every
// LDS offset, Hamiltonian entry and plane index is a constant: a wave issues
// all LDS reads and neighbour gathers of its elements back to back and pays
// the memory latency about once.  The ADOs of a tile are consecutive, so each
// gather of a wave reads one element plane at nearly consecutive indices.
// ---------------------------------------------------------------------------

constexpr int kTile = 64;

// Packed element p -> (a, b), a <= b: p < N are the diagonal entries, then
// the pairs a < b in row-major order.
__host__ __device__ constexpr int elem_a(int N, int p) {
  if (p < N) return p;
  int q = p - N, a = 0;
  while (q >= N - 1 - a) {
    q -= N - 1 - a;
    ++a;
  }
  return a;
}
__host__ __device__ constexpr int elem_b(int N, int p) {
  if (p < N) return p;
  int q = p - N, a = 0;
  while (q >= N - 1 - a) {
    q -= N - 1 - a;
    ++a;
  }
  return a + 1 + q;
}
// Plane of the real part of entry (r, c) and of its imaginary part (N*N, a
// plane of zeros, on the diagonal), and the sign of the imaginary part.
__host__ __device__ constexpr int ent_re(int N, int r, int c) {
  return r == c ? r : (r < c ? re_plane(N, r, c) : re_plane(N, c, r));
}
__host__ __device__ constexpr int ent_im(int N, int r, int c) {
  return r == c ? N * N : ent_re(N, r, c) + 1;
}
__host__ __device__ constexpr int ent_sg(int r, int c) { return r > c ? -1 : 1; }

// Launch shapes of the tile kernel, the candidates of the autotuner: the
// target number of packed elements per wave (which sets the waves per
// workgroup, see tile_waves_for), how many of a wave's elements have their
// global loads in flight together (one chunk), and the minimum waves per SIMD
// asked of the register allocator (7 caps a wave at 72 VGPRs, so that two
// 14-wave workgroups fit on a CU).  Small launches are latency-bound and
// prefer few load round trips with every workgroup resident; large ones are
// bandwidth-bound.  Shape 0 is the default (HEOM_NO_AUTOTUNE).  Every shape
// computes each element with the same instructions in the same order, so the
// results do not depend on the shape.
struct TileShape {
  int elems_per_wave, chunk, min_waves;
};
constexpr int kTileShapes = kWideShape;
constexpr TileShape kShapesF64[kTileShapes] = {{7, 2, 1}, {7, 7, 1}, {2, 2, 1}, {4, 2, 1}, {2, 1, 7}};
constexpr TileShape kShapesF32[kTileShapes] = {{4, 4, 1}, {4, 2, 1}, {2, 2, 1}, {7, 2, 1}, {2, 1, 7}};
__host__ __device__ constexpr TileShape tile_shape(bool fp64, int s) {
  return fp64 ? kShapesF64[s] : kShapesF32[s];
}
#ifndef HEOM_TILE_CHUNK_BARRIER
#define HEOM_TILE_CHUNK_BARRIER 1
#endif

// Waves per tile workgroup: the divisor of the N(N+1)/2 packed elements
// (at most 16) that gives closest to `target` elements per wave.
__host__ __device__ constexpr int tile_waves_for(int N, int target) {
  const int P = N * (N + 1) / 2;
  int best = 1;
  for (int w = 1; w <= 16 && w <= P; ++w) {
    if (P % w) continue;
    const int d_best = (target * best - P) < 0 ? P - target * best : target * best - P;
    const int d_w = (target * w - P) < 0 ? P - target * w : target * w - P;
    if (d_w < d_best) best = w;
  }
  return best;
}
__host__ __device__ constexpr int tile_waves(int N, bool fp64, int s) {
  return tile_waves_for(N, tile_shape(fp64, s).elems_per_wave);
}

// The tile units are compiled once per shape (HEOM_SHAPE) and storage
// precision (HEOM_TILE_F64: 1 for the FP64 instances, 0 for the FP32-mixed
// ones, so that each precision can be built with its own code-generation
// options); their instance tables carry both in their names.
#ifndef HEOM_SHAPE
#define HEOM_SHAPE 0
#endif
#ifndef HEOM_TILE_F64
#define HEOM_TILE_F64 1
#endif
#define HEOM_SHAPED_CAT(name, s, f) name##_s##s##_f##f
#define HEOM_SHAPED_EXPAND(name, s, f) HEOM_SHAPED_CAT(name, s, f)
#define HEOM_SHAPED(name) HEOM_SHAPED_EXPAND(name, HEOM_SHAPE, HEOM_TILE_F64)

template <typename T>
struct TileCtx {
  const HEOM_CONST double *P;         // parameter block
  const HEOM_CONST float *P32;        // its FP32 copy (same offsets)
  const T *sx;                        // LDS tile of the stage input, [N*N + 1][64]
  const int32_t *sup, *sdn;
  const uint8_t *socc;                // LDS neighbour tables, [M][64]
  const HEOM_GLOBAL T *X;             // stage input planes (neighbour gathers)
  const HEOM_GLOBAL T *Yp;            // state planes
  HEOM_GLOBAL T *Out;                 // output planes
  const double *sx0;                  // LDS copy of the FP64 sigma_0 stage input (mixed)
  const double *sf0;                  // the same, unpacked: Re [N*N], Im [N*N], and H_re
                                      // [N*N] (mixed, sigma_0 item only)
  const HEOM_GLOBAL double *y0;       // FP64 sigma_0 state (mixed precision)
  HEOM_GLOBAL double *out0;           // FP64 sigma_0 output (mixed precision)
  int64_t S, i;
  int lane;
  double damp, coef;
  // Scaled hierarchies: the coupling weights by mode and occupation, up then
  // down ([M][levels] each, after the parameter block).
  const double *wu, *wd;
  int levels;
};

// Parameter q in the arithmetic type C: FP32 arithmetic reads the FP32 copy
// (the value a conversion on use would give, without the conversion and with
// half the scalar registers).
template <typename C, typename T>
__device__ __forceinline__ C par(const TileCtx<T> &c, int q) {
  if constexpr (sizeof(C) == 4)
    return c.P32[q];
  else
    return c.P[q];
}

// Values of one element (A, B) read from global memory: the same element of
// the deeper (y*) and shallower (z*) neighbours along the modes of sites A
// and B, and of the state.
template <typename C, int KP>
struct ElemLoads {
  C yar[KP], yai[KP], ybr[KP], ybi[KP];  // deeper neighbours
  C zar[KP], zai[KP], zbr[KP], zbi[KP];  // shallower neighbours
  C str, sti;                            // state
  C wua[KP], wub[KP], wda[KP], wdb[KP];  // scaled: coupling weights of the modes
};

// Phase 1 of element (A, B): issue every global load.  Neighbour gathers are
// branch-free: a missing neighbour (index -1) reads the lane's own entry and
// is weighted by zero (the occupation is zero exactly where the shallower
// neighbour is missing), so the loads of all elements of a wave are in
// flight together.
template <int N, int KP, int A, int B, typename C, typename T, bool SCALED>
__device__ __forceinline__ void tile_load(const TileCtx<T> &c, ElemLoads<C, KP> &L) {
  constexpr int E = ent_re(N, A, B);
  const int lane = c.lane;
  // Wave-uniform base: the diagonal element's plane, or the pair's block of
  // (Re, Im) pairs (each neighbour one access of both parts).
  const HEOM_GLOBAL T *pre = c.X + E * c.S;
  constexpr uint32_t W = (A != B ? 2 : 1) * sizeof(T);  // bytes per ADO in that plane
  const uint32_t self = static_cast<uint32_t>(c.i);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int ma = A * KP + k;
    const int mb = B * KP + k;
    if constexpr (A != B) {
      const int ja = c.sup[ma * kTile + lane];
      const int jb = c.sup[mb * kTile + lane];
      const uint32_t oa = (ja >= 0 ? static_cast<uint32_t>(ja) : self) * W;
      const uint32_t ob = (jb >= 0 ? static_cast<uint32_t>(jb) : self) * W;
      const Pair2<T> ya = ld_pair(pre, oa), yb = ld_pair(pre, ob);
      L.yar[k] = static_cast<C>(ya.x);
      L.yai[k] = static_cast<C>(ya.y);
      L.ybr[k] = static_cast<C>(yb.x);
      L.ybi[k] = static_cast<C>(yb.y);
    }
    const int ja = c.sdn[ma * kTile + lane];
    const int jb = c.sdn[mb * kTile + lane];
    const uint32_t oa = (ja >= 0 ? static_cast<uint32_t>(ja) : self) * W;
    const uint32_t ob = (jb >= 0 ? static_cast<uint32_t>(jb) : self) * W;
    if constexpr (A != B) {
      const Pair2<T> za = ld_pair(pre, oa), zb = ld_pair(pre, ob);
      L.zar[k] = static_cast<C>(za.x);
      L.zai[k] = static_cast<C>(za.y);
      L.zbr[k] = static_cast<C>(zb.x);
      L.zbi[k] = static_cast<C>(zb.y);
    } else {
      L.zar[k] = static_cast<C>(ld_off(pre, oa));
      L.zbr[k] = static_cast<C>(ld_off(pre, ob));
    }
  }
  if constexpr (A != B) {
    const Pair2<T> st = ld_pair(c.Yp + E * c.S, self * W);
    L.str = static_cast<C>(st.x);
    L.sti = static_cast<C>(st.y);
  } else {
    L.str = static_cast<C>(ld_off(c.Yp + E * c.S, self * W));
  }
  if constexpr (SCALED) {
    // Weights of the couplings along the modes of sites A and B, by the
    // ADO's occupation of each mode (loaded with the gathers).
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int ma = A * KP + k, mb = B * KP + k;
      const int oa = c.socc[ma * kTile + lane], ob = c.socc[mb * kTile + lane];
      L.wua[k] = static_cast<C>(c.wu[ma * c.levels + oa]);
      L.wub[k] = static_cast<C>(c.wu[mb * c.levels + ob]);
      L.wda[k] = static_cast<C>(c.wd[ma * c.levels + oa]);
      L.wdb[k] = static_cast<C>(c.wd[mb * c.levels + ob]);
    }
  }
}

// Phase 2 of element (A, B): right-hand side from the LDS tile and the loaded
// values, RK4 stage update, store.  C is the arithmetic type.
template <int N, int KP, int A, int B, typename C, typename T, bool STREAM, bool SCALED>
__device__ __forceinline__ void tile_finish(const TileCtx<T> &c, const ElemLoads<C, KP> &L) {
#pragma clang fp contract(off)
  constexpr int M = N * KP;
  constexpr int o_hg = 2 * N * N, o_dl = 2 * N * N + N, o_cr = 2 * N * N + 4 * N,
                o_ci = 2 * N * N + 4 * N + M;
  constexpr int E = ent_re(N, A, B);
  const int lane = c.lane;
  auto xe = [&](int e) -> C { return static_cast<C>(c.sx[e * kTile + lane]); };
  // Coherent part: s = sum_k H_Ak X_kB - X_Ak H_kB; contribution -i s.
  C sr = C(0), si = C(0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const C hak = par<C>(c, A * N + k);
    const C hkb = par<C>(c, k * N + B);
    const C xkb_r = xe(ent_re(N, k, B));
    const C xkb_i = static_cast<C>(ent_sg(k, B)) * xe(ent_im(N, k, B));
    const C xak_r = xe(ent_re(N, A, k));
    const C xak_i = static_cast<C>(ent_sg(A, k)) * xe(ent_im(N, A, k));
    sr = fmad(-xak_r, hkb, fmad(hak, xkb_r, sr));
    si = fmad(-xak_i, hkb, fmad(hak, xkb_i, si));
  }
  C ar = si, ai = -sr;
  const C xr = xe(E), xi = xe(ent_im(N, A, B));
  C dec = static_cast<C>(c.damp) + par<C>(c, o_hg + A) + par<C>(c, o_hg + B);
  if constexpr (A != B) dec += par<C>(c, o_dl + A) + par<C>(c, o_dl + B);
  ar = fmad(-dec, xr, ar);
  ai = fmad(-dec, xi, ai);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int ma = A * KP + k;
    const int mb = B * KP + k;
    if constexpr (A != B) {
      // Deeper neighbours: + i Y (mode of site A) - i Y (mode of site B),
      // weighted by zero where the neighbour is missing (scaled: by the
      // coupling weight where it exists).
      C fa = c.sup[ma * kTile + lane] >= 0 ? C(1) : C(0);
      C fb = c.sup[mb * kTile + lane] >= 0 ? C(1) : C(0);
      if constexpr (SCALED) {
        fa = c.sup[ma * kTile + lane] >= 0 ? L.wua[k] : C(0);
        fb = c.sup[mb * kTile + lane] >= 0 ? L.wub[k] : C(0);
      }
      ar = fmad(-fa, L.yai[k], fmad(fb, L.ybi[k], ar));
      ai = fmad(-fb, L.ybr[k], fmad(fa, L.yar[k], ai));
    }
    // Shallower neighbours: + i n c Z (site A) - i n conj(c) Z (site B)
    // (scaled: the down weight in place of n).
    C na = static_cast<C>(c.socc[ma * kTile + lane]);
    C nb = static_cast<C>(c.socc[mb * kTile + lane]);
    if constexpr (SCALED) {
      na = L.wda[k];
      nb = L.wdb[k];
    }
    const C car = na * par<C>(c, o_cr + ma), cai = na * par<C>(c, o_ci + ma);
    const C cbr = nb * par<C>(c, o_cr + mb), cbi = nb * par<C>(c, o_ci + mb);
    const C zai = (A == B) ? C(0) : L.zai[k];
    const C zbi = (A == B) ? C(0) : L.zbi[k];
    // i (car + i cai) z_a = -(cai zar + car zai) + i (car zar - cai zai)
    ar = fmad(-car, zai, fmad(-cai, L.zar[k], ar));
    ai = fmad(-cai, zai, fmad(car, L.zar[k], ai));
    // -i (cbr - i cbi) z_b = (cbr zbi - cbi zbr) - i (cbr zbr + cbi zbi)
    ar = fmad(-cbi, L.zbr[k], fmad(cbr, zbi, ar));
    ai = fmad(-cbi, zbi, fmad(-cbr, L.zbr[k], ai));
  }
  // RK4 stage: out = y + coef * rhs (at stage 0 the state planes are the
  // stage input, so the loaded state equals the tile).
  const C coef = static_cast<C>(c.coef);
  const C nr = fmad(coef, ar, L.str);
  const C ni = fmad(coef, ai, (A == B) ? C(0) : L.sti);
  // In FP32-mixed runs sigma_0 is written by tile_sigma0 alone.
  if (sizeof(T) == 4 && c.i == 0) return;
  const uint32_t oi = static_cast<uint32_t>(c.i) * sizeof(T);
  if constexpr (A != B)
    st_pair<STREAM>(c.Out + E * c.S, 2 * oi, static_cast<T>(nr), static_cast<T>(ni));
  else
    st_off<STREAM>(c.Out + E * c.S, oi, static_cast<T>(nr));
}

// One chunk of wave G's elements (element indices OFF + K): all global loads
// first, then arithmetic and stores.
template <int N, int KP, int G, int W, int OFF, typename C, typename T, bool STREAM, bool SCALED,
          int... K>
__device__ __forceinline__ void tile_chunk(const TileCtx<T> &c, std::integer_sequence<int, K...>) {
  ElemLoads<C, KP> L[sizeof...(K)];
  (tile_load<N, KP, elem_a(N, G + (OFF + K) * W), elem_b(N, G + (OFF + K) * W), C, T, SCALED>(
       c, L[K]),
   ...);
  (tile_finish<N, KP, elem_a(N, G + (OFF + K) * W), elem_b(N, G + (OFF + K) * W), C, T, STREAM,
               SCALED>(c, L[K]),
   ...);
}

template <int N, int KP, int G, int W, int CH0, int OFF, typename C, typename T, bool STREAM,
          bool SCALED>
__device__ __forceinline__ void tile_chunks(const TileCtx<T> &c) {
  constexpr int P = N * (N + 1) / 2;
  constexpr int count = (P - G + W - 1) / W;
  // An element gathers 4 neighbours per mode of its sites: with more modes
  // per site, fewer elements per chunk keep the loaded values in registers.
  constexpr int CH = CH0 / KP > 0 ? CH0 / KP : 1;
  if constexpr (OFF < count) {
    constexpr int len = (count - OFF < CH) ? count - OFF : CH;
    tile_chunk<N, KP, G, W, OFF, C, T, STREAM, SCALED>(c, std::make_integer_sequence<int, len>{});
    // Keep the next chunk's LDS reads from being hoisted above this chunk
    // (they cannot alias its global stores), which would hold every operand
    // of the wave's elements in registers at once.
#if HEOM_TILE_CHUNK_BARRIER
    __builtin_amdgcn_sched_barrier(0);
#endif
    tile_chunks<N, KP, G, W, CH0, OFF + CH, C, T, STREAM, SCALED>(c);
  }
}

// Elements G, G + W, ... of every ADO of the tile (wave G of W).
template <int N, int KP, int W, int CH0, typename C, typename T, bool STREAM, bool SCALED,
          int G = 0>
__device__ __forceinline__ void tile_dispatch(int wave, const TileCtx<T> &c) {
  if constexpr (G < W) {
    if (wave == G)
      tile_chunks<N, KP, G, W, CH0, 0, C, T, STREAM, SCALED>(c);
    else
      tile_dispatch<N, KP, W, CH0, C, T, STREAM, SCALED, G + 1>(wave, c);
  }
}

// sigma_0 of an FP32-mixed run, in FP64 (packed element p, chosen at run
// time, so that one lane per element of the sigma_0 work item covers
// sigma_0): the right-hand side
// from the FP64 copy of the stage input (LDS), the FP32 neighbour planes and
// the FP64 state, with the operations of tile_finish in the same order, so
// the result does not depend on the launch shape.  It is the only writer of
// sigma_0, in both the FP64 copy and the FP32 planes.  Keeping this pass out
// of the unrolled element code keeps FP64 operands out of the register
// allocation of the FP32 kernel.
template <int N, int KP, typename T, bool SCALED>
__device__ __forceinline__ void tile_sigma0(const TileCtx<T> &c, int p) {
#pragma clang fp contract(off)
  constexpr int M = N * KP;
  constexpr int o_hg = 2 * N * N, o_dl = 2 * N * N + N, o_cr = 2 * N * N + 4 * N,
                o_ci = 2 * N * N + 4 * N + M, o_nu = 2 * N * N + 4 * N + 2 * M;
  const int A = elem_a(N, p), B = elem_b(N, p);
  const bool off = A != B;
  const int E = ent_re(N, A, B);
  // The element's plane (diagonal) or the pair's block, (Re, Im) of ADO j at
  // 2j and 2j + 1.
  const HEOM_GLOBAL T *pre = c.X + E * c.S;
  const uint32_t W = off ? 2u : 1u;
  // Loads, as tile_load issues them for ADO 0 (entry 0 of the LDS tables; a
  // missing neighbour reads ADO 0 itself and is weighted by zero).
  double yar[KP], yai[KP], ybr[KP], ybi[KP], zar[KP], zai[KP], zbr[KP], zbi[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int ma = A * KP + k, mb = B * KP + k;
    yar[k] = yai[k] = ybr[k] = ybi[k] = zai[k] = zbi[k] = 0.0;
    if (off) {
      const int ja = c.sup[ma * kTile], jb = c.sup[mb * kTile];
      const uint32_t oa = static_cast<uint32_t>(ja >= 0 ? ja : 0) * W;
      const uint32_t ob = static_cast<uint32_t>(jb >= 0 ? jb : 0) * W;
      yar[k] = pre[oa];
      yai[k] = pre[oa + 1];
      ybr[k] = pre[ob];
      ybi[k] = pre[ob + 1];
    }
    const int ja = c.sdn[ma * kTile], jb = c.sdn[mb * kTile];
    const uint32_t oa = static_cast<uint32_t>(ja >= 0 ? ja : 0) * W;
    const uint32_t ob = static_cast<uint32_t>(jb >= 0 ? jb : 0) * W;
    zar[k] = pre[oa];
    zbr[k] = pre[ob];
    if (off) {
      zai[k] = pre[oa + 1];
      zbi[k] = pre[ob + 1];
    }
  }
  const double str = c.y0[E];
  const double sti = off ? c.y0[E + 1] : 0.0;
  // Entries of the unpacked copy are the packed values with the sign of the
  // imaginary part applied (+0 for the diagonal), as tile_finish forms them.
  const double *Xr = c.sf0, *Xi = c.sf0 + N * N, *Hr = c.sf0 + 2 * N * N;
  double sr = 0.0, si = 0.0;
  // Not unrolled: this pass must not raise the kernel's register count
  // above that of the element code.
#pragma nounroll
  for (int k = 0; k < N; ++k) {
    const double hak = Hr[A * N + k];
    const double hkb = Hr[k * N + B];
    sr = fmad(-Xr[A * N + k], hkb, fmad(hak, Xr[k * N + B], sr));
    si = fmad(-Xi[A * N + k], hkb, fmad(hak, Xi[k * N + B], si));
  }
  double ar = si, ai = -sr;
  const double xr = Xr[A * N + B], xi = Xi[A * N + B];
  double damp = 0.0;
#pragma unroll
  for (int m = 0; m < M; ++m)
    damp = fmad(static_cast<double>(c.socc[m * kTile]), c.P[o_nu + m], damp);
  double dec = damp + c.P[o_hg + A] + c.P[o_hg + B];
  if (off) dec += c.P[o_dl + A] + c.P[o_dl + B];
  ar = fmad(-dec, xr, ar);
  ai = fmad(-dec, xi, ai);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int ma = A * KP + k, mb = B * KP + k;
    if (off) {
      double fa = c.sup[ma * kTile] >= 0 ? 1.0 : 0.0;
      double fb = c.sup[mb * kTile] >= 0 ? 1.0 : 0.0;
      if constexpr (SCALED) {
        fa = c.sup[ma * kTile] >= 0 ? c.wu[ma * c.levels + c.socc[ma * kTile]] : 0.0;
        fb = c.sup[mb * kTile] >= 0 ? c.wu[mb * c.levels + c.socc[mb * kTile]] : 0.0;
      }
      ar = fmad(-fa, yai[k], fmad(fb, ybi[k], ar));
      ai = fmad(-fb, ybr[k], fmad(fa, yar[k], ai));
    }
    double na = static_cast<double>(c.socc[ma * kTile]);
    double nb = static_cast<double>(c.socc[mb * kTile]);
    if constexpr (SCALED) {
      na = c.wd[ma * c.levels + c.socc[ma * kTile]];
      nb = c.wd[mb * c.levels + c.socc[mb * kTile]];
    }
    const double car = na * c.P[o_cr + ma], cai = na * c.P[o_ci + ma];
    const double cbr = nb * c.P[o_cr + mb], cbi = nb * c.P[o_ci + mb];
    ar = fmad(-car, zai[k], fmad(-cai, zar[k], ar));
    ai = fmad(-cai, zai[k], fmad(car, zar[k], ai));
    ar = fmad(-cbi, zbr[k], fmad(cbr, zbi[k], ar));
    ai = fmad(-cbi, zbi[k], fmad(-cbr, zbr[k], ai));
  }
  const double nr = fmad(c.coef, ar, str);
  const double ni = fmad(c.coef, ai, sti);
  c.out0[E] = nr;
  c.Out[E * c.S] = static_cast<T>(nr);
  if (off) {
    c.out0[E + 1] = ni;
    c.Out[E * c.S + 1] = static_cast<T>(ni);  // ADO 0 of the pair's block
  }
}

template <int N, int KP, typename T, int SHAPE, bool STREAM, bool SCALED>
__global__ void __launch_bounds__(64 * tile_waves(N, sizeof(T) == 8, SHAPE),
                                  tile_shape(sizeof(T) == 8, SHAPE).min_waves)
    stage_tile(const InstDesc *__restrict__ descs, const WorkItem *__restrict__ work, int stage,
               double coef, int /*hist_slot: recorded by the snapshot kernel*/) {
  constexpr int N2 = N * N;
  constexpr int M = N * KP;
  constexpr int W = tile_waves(N, sizeof(T) == 8, SHAPE);
  constexpr int CH0 = tile_shape(sizeof(T) == 8, SHAPE).chunk;
  constexpr bool MIXED = sizeof(T) == 4;
  __shared__ T sx[(N2 + 1) * kTile];
  __shared__ double sx0[MIXED ? N2 : 1];      // FP64 sigma_0 stage input (sigma_0 item)
  __shared__ double sf0[MIXED ? 3 * N2 : 1];  // its unpacked form and H_re (sigma_0 item)
  __shared__ int32_t sup[M * kTile];
  __shared__ int32_t sdn[M * kTile];
  __shared__ uint8_t socc[M * kTile];

  const WorkItem w = work[blockIdx.x];
  const InstDesc &d = descs[w.inst];
  const StageBufs bufs = stage_bufs(d, stage);
  const int64_t S = d.stride;
  const int lane = threadIdx.x & (kTile - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const HEOM_GLOBAL T *X = gmem(static_cast<const T *>(bufs.x));
  const HEOM_GLOBAL int32_t *up = gmem(d.up);
  const HEOM_GLOBAL int32_t *dn = gmem(d.down);
  const HEOM_GLOBAL uint8_t *oc = gmem(d.occ);
  if constexpr (MIXED) {
    // The FP32-mixed work list carries one extra item per instance (first =
    // -1): the FP64 update of sigma_0 and of the sink scalars, in a
    // workgroup of its own, beside the tiles rather than after the tile of
    // ADO 0.  The tile of ADO 0 leaves sigma_0 to it.
    if (w.first < 0) {
      for (int e = threadIdx.x; e < N2; e += blockDim.x) {
        const int r = e / N, q = e % N;
        const double re = bufs.x0[ent_re(N, r, q)];
        const double im = r == q ? 0.0 : bufs.x0[ent_im(N, r, q)];
        sx0[e] = bufs.x0[e];
        sf0[e] = re;
        sf0[N2 + e] = static_cast<double>(ent_sg(r, q)) * im;
        sf0[2 * N2 + e] = d.params[e];
      }
      for (int m = threadIdx.x; m < M; m += blockDim.x) {  // ADO 0's table entries
        sup[m * kTile] = up[m * S];
        sdn[m * kTile] = dn[m * S];
        socc[m * kTile] = oc[m * S];
      }
      __syncthreads();
      if (wave == 0) scalar_update_wave(d, bufs, N, coef, lane, [&](int q) { return sx0[q]; });
      const TileCtx<T> c0{cmem(d.params),
                          cmem(reinterpret_cast<const float *>(d.params + param_offsets(N, M).f32)),
                          sx,
                          sup,
                          sdn,
                          socc,
                          X,
                          gmem(static_cast<const T *>(bufs.y)),
                          gmem(static_cast<T *>(bufs.out)),
                          sx0,
                          sf0,
                          gmem(bufs.y0),
                          gmem(bufs.out0),
                          S,
                          0,
                          lane,
                          0.0,
                          coef,
                          d.params + param_offsets(N, M).total,
                          d.params + param_offsets(N, M).total + M * d.levels,
                          d.levels};
      for (int p = threadIdx.x; p < N * (N + 1) / 2; p += blockDim.x)
        tile_sigma0<N, KP, T, SCALED>(c0, p);
      return;
    }
  }
  const int64_t i = static_cast<int64_t>(w.first) + lane;
  const bool valid = i < d.n_ados;
  // Stage the tile: wave w loads element slots w, w + W, ... (a compile-time
  // count, clamped in bounds, so that every load is issued before the first
  // wait): slot s < N is diagonal plane s, slot N + p pair p's block, both
  // parts in one access.
  const int64_t ic = valid ? i : 0;  // invalid lanes load ADO 0 and store defaults
  constexpr int NS = N * (N + 1) / 2;
  constexpr int RX = (NS + W - 1) / W;
  constexpr int RM = (M + W - 1) / W;
  T vx[RX], vy[RX];
  int32_t vu[RM], vd[RM];
  uint8_t vo[RM];
  const uint32_t ic4 = static_cast<uint32_t>(ic) * 4u;
  const uint32_t icb = static_cast<uint32_t>(ic) * static_cast<uint32_t>(sizeof(T));
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    const int sl = min(wave + r * W, NS - 1);
    if (sl < N) {
      vx[r] = ld_off(X + sl * S, icb);
      vy[r] = T(0);
    } else {
      const Pair2<T> v = ld_pair(X + (N + 2 * (sl - N)) * S, 2 * icb);
      vx[r] = v.x;
      vy[r] = v.y;
    }
  }
  // Neighbour tables: the 16-bit offsets where the instance has them (half
  // the bytes), else the 32-bit indices, through the same loads.
  const bool t16 = d.up16 != nullptr;
  const HEOM_GLOBAL char *upb = (const HEOM_GLOBAL char *)(
      t16 ? reinterpret_cast<const char *>(d.up16) : reinterpret_cast<const char *>(d.up));
  const HEOM_GLOBAL char *dnb = (const HEOM_GLOBAL char *)(
      t16 ? reinterpret_cast<const char *>(d.down16) : reinterpret_cast<const char *>(d.down));
  const uint32_t row_bytes = static_cast<uint32_t>(S) * (t16 ? 2u : 4u);
  const uint32_t ic32 = static_cast<uint32_t>(ic);
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int m = min(wave + r * W, M - 1);
    vu[r] = table_load(upb + m * row_bytes, t16, ic32);
    vd[r] = table_load(dnb + m * row_bytes, t16, ic32);
    vo[r] = ld_off(oc + m * S, ic32);
  }
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    const int sl = wave + r * W;
    if (sl < N) {
      sx[sl * kTile + lane] = valid ? vx[r] : T(0);
    } else if (sl < NS) {
      const int e = N + 2 * (sl - N);
      sx[e * kTile + lane] = valid ? vx[r] : T(0);
      sx[(e + 1) * kTile + lane] = valid ? vy[r] : T(0);
    }
  }
  if (wave == 0) sx[N2 * kTile + lane] = T(0);
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int m = wave + r * W;
    if (m < M) {
      // Valid lanes decode at their own index (invalid ones store -1).
      const uint32_t iself = static_cast<uint32_t>(w.first) + static_cast<uint32_t>(lane);
      const int ju = table_decode(vu[r], t16, iself);
      const int jd = table_decode(vd[r], t16, iself);
      sup[m * kTile + lane] = valid ? ju : -1;
      sdn[m * kTile + lane] = valid ? jd : -1;
      socc[m * kTile + lane] = valid ? vo[r] : 0;
    }
  }
  __syncthreads();
  // Sink fluxes and scalars of sigma_0 (FP64 storage; FP32-mixed runs do
  // this in the sigma_0 item): wave 0 of the first tile, every lane still
  // active.
  if constexpr (!MIXED) {
    if (w.first == 0 && wave == 0 && !(d.flags & kInstNoSigma0))
      scalar_update_wave(d, bufs, N, coef, lane, [&](int q) { return sx[q * kTile]; });
  }
  const HEOM_CONST double *P = cmem(d.params);
  TileCtx<T> ctx{P,
                 cmem(reinterpret_cast<const float *>(d.params + param_offsets(N, M).f32)),
                 sx,
                 sup,
                 sdn,
                 socc,
                 X,
                 gmem(static_cast<const T *>(bufs.y)),
                 gmem(static_cast<T *>(bufs.out)),
                 sx0,
                 sf0,
                 gmem(bufs.y0),
                 gmem(bufs.out0),
                 S,
                 i,
                 lane,
                 0.0,
                 coef,
                 d.params + param_offsets(N, M).total,
                 d.params + param_offsets(N, M).total + M * d.levels,
                 d.levels};
  if (!valid) return;  // no barrier below
#pragma unroll
  for (int m = 0; m < M; ++m)
    ctx.damp = fmad(static_cast<double>(socc[m * kTile + lane]), P[2 * N * N + 4 * N + 2 * M + m],
                    ctx.damp);
  tile_dispatch<N, KP, W, CH0, T, T, STREAM, SCALED>(wave, ctx);
}

// The instance of a tile unit for storage `mixed`, the store policy and
// scaled hierarchies: null for the precision the unit is not compiled for
// (the other unit of the same shape provides it), for streaming stores in
// FP32-mixed storage (not built: at most 1 % faster there, on small launches
// only), and for scaled hierarchies outside shape 0 with plain stores (their
// only instance).
template <int N, int KP, int S>
StageKernel tile_instance(bool mixed, bool streaming, bool scaled) {
#if HEOM_TILE_F64
  if (mixed) return nullptr;
  if (scaled) {
    if constexpr (S == 0)
      return streaming ? nullptr : &stage_tile<N, KP, double, S, false, true>;
    return nullptr;
  }
  return streaming ? &stage_tile<N, KP, double, S, true, false>
                   : &stage_tile<N, KP, double, S, false, false>;
#else
  if (!mixed || streaming) return nullptr;
  if (scaled) {
    if constexpr (S == 0) return &stage_tile<N, KP, float, S, false, true>;
    return nullptr;
  }
  return &stage_tile<N, KP, float, S, false, false>;
#endif
}

// ---------------------------------------------------------------------------
// Wide kernel: runtime N up to kWideMaxN, real H.
//
// A 64-ADO tile of a large system does not fit in LDS (N = 24 in FP64 would
// need 295 KB), so this kernel stages kWideAdos = 16 consecutive ADOs, with
// the Hamiltonian and the neighbour tables, and spreads a wave over 4 packed
// elements x 16 ADOs: lane l handles ADO l % 16 of the tile and element slot
// l / 16.  Each element plane is then read in 16-ADO (128-byte in FP64)
// segments.  The commutator visits only the k where H_ak or H_kb is nonzero
// (row masks built in LDS), in increasing k: for the chains and rings of the
// serving workload that is at most 6 of the N terms, which keeps the LDS
// traffic of the product small.  Each element is computed with the same
// sequence of operations as in the tile kernel (terms with H = 0 are exact
// no-ops there), so the two kernels agree bitwise where both exist.
// ---------------------------------------------------------------------------

constexpr int kWideAdos = 16;
constexpr int kWideWaves = 16;
constexpr int kWideSlots = kWideWaves * (64 / kWideAdos);  // element slots per workgroup
constexpr int kWideMaxN = 32;
constexpr int kWideMaxKP = 4;  // modes per site (K + 1) the wide kernel is built for

// Entry (r, c) of a packed ADO in the wide kernel's LDS tile: byte offsets
// of its real and imaginary planes (the zero plane N*N for the imaginary part
// of a diagonal entry; bit 31 of `im` set when the imaginary part is
// negated, r > c), and H_rc in the storage precision: FP64, or with FP32
// storage the FP32 value (rounded once, as a conversion at each use would
// round it) in the low word of `h`.  One 16-byte read gives the commutator
// both.
struct WideEntry {
  uint32_t re, im;
  double h;
};
template <typename T>
__device__ __forceinline__ double wide_h_slot(double h) {
  if constexpr (sizeof(T) == 4)
    return __longlong_as_double(static_cast<long long>(__float_as_uint(static_cast<float>(h))));
  else
    return h;
}
template <typename T>
__device__ __forceinline__ T wide_h_value(double slot) {
  if constexpr (sizeof(T) == 4)
    return __uint_as_float(static_cast<uint32_t>(__double_as_longlong(slot)));
  else
    return slot;
}

// LDS layout of the wide kernel (byte offsets; every region 16-byte aligned).
// `levels` > 0 (scaled hierarchies) adds the coupling-weight tables.
struct WideLds {
  int x, ent, nz, dec, dl, cr, ci, nu, up, dn, occ, pa, pb, x0, wu, wd, total;
};
__host__ __device__ inline int wide_align(int v) { return (v + 15) & ~15; }
__host__ __device__ inline WideLds wide_lds(int N, int M, int s, int levels = 0) {
  const int P = N * (N + 1) / 2;
  WideLds L;
  L.x = 0;                                                    // T [N*N + 1][kWideAdos]
  L.ent = wide_align(L.x + (N * N + 1) * kWideAdos * s);      // WideEntry [N*N]
  L.nz = wide_align(L.ent + N * N * 16);                      // uint32 [N] row masks
  L.dec = wide_align(L.nz + N * 4);                           // double [N] (trap + rec) / 2
  L.dl = wide_align(L.dec + N * 8);                           // double [N] delta
  L.cr = wide_align(L.dl + N * 8);                            // double [M]
  L.ci = wide_align(L.cr + M * 8);                            // double [M]
  L.nu = wide_align(L.ci + M * 8);                            // double [M]
  L.up = wide_align(L.nu + M * 8);                            // int32 [M][kWideAdos]
  L.dn = wide_align(L.up + M * kWideAdos * 4);                // int32 [M][kWideAdos]
  L.occ = wide_align(L.dn + M * kWideAdos * 4);               // uint8 [M][kWideAdos]
  L.pa = wide_align(L.occ + M * kWideAdos);                   // uint8 [P] element -> a
  L.pb = wide_align(L.pa + P);                                // uint8 [P] element -> b
  L.x0 = wide_align(L.pb + P);                                // double [N*N] (FP32 storage)
  L.wu = wide_align(L.x0 + (s == 4 ? N * N * 8 : 0));         // double [M][levels] (scaled)
  L.wd = wide_align(L.wu + M * levels * 8);                   // double [M][levels] (scaled)
  L.total = wide_align(L.wd + M * levels * 8);
  return L;
}

template <typename T>
struct WideCtx {
  int N, t;
  const T *sx;
  const WideEntry *sent;
  const double *sdec, *sdl, *scr, *sci;
  const uint32_t *snz;
  const int32_t *sup, *sdn;
  const uint8_t *socc;
  const HEOM_GLOBAL T *X, *Yp;
  HEOM_GLOBAL T *Out;
  const double *sx0;  // LDS copy of the FP64 sigma_0 stage input (FP32 storage)
  const HEOM_GLOBAL double *hg;  // H_re (FP64, parameter block): the FP64 sigma_0 pass
  const HEOM_GLOBAL double *y0;
  HEOM_GLOBAL double *out0;
  uint32_t S;  // plane stride in ADOs; every buffer of a wide launch is below 4 GiB
  int64_t i;
  double damp, coef;
  const double *swu, *swd;  // scaled hierarchies: coupling weights [M][levels] (LDS)
  int levels;
};

// Global values one element needs: neighbour gathers along the modes of its
// sites, and its state entry.
template <typename C, int KP>
struct WideLoads {
  C yar[KP], yai[KP], ybr[KP], ybi[KP], zar[KP], zai[KP], zbr[KP], zbi[KP];
  int jua[KP], jub[KP];
  C str, sti;
};

// Plane of a tile byte offset (entry fields) and the tile's bytes per plane.
template <typename T>
__device__ __forceinline__ int wide_plane(uint32_t off) {
  return static_cast<int>((off & 0x7fffffffu) / (kWideAdos * sizeof(T)));
}

// Phase 1 of element (a, b) of the lane's ADO (tile_load with runtime a, b):
// every global load, at 32-bit byte offsets from the buffers' bases.  An
// off-diagonal element reads each neighbour's (Re, Im) with one access from
// the pair's block; a diagonal one reads the real plane and skips the loads
// the tile kernel skips (their values are not used).  The element list puts
// the N diagonal elements first and a wave takes kWideSlots consecutive ones
// per pass, so for N a multiple of kWideSlots the branch is wave-uniform.
// X0SRC reads sigma_0's state from its FP64 copy.
template <typename C, typename T, bool X0SRC, int KP>
__device__ __forceinline__ void wide_load(const WideCtx<T> &c, int a, int b,
                                          WideLoads<C, KP> &L) {
  const int N = c.N, t = c.t;
  const int E = wide_plane<T>(c.sent[a * N + b].re);
  const bool offd = a != b;
  const uint32_t sz = static_cast<uint32_t>(sizeof(T));
  const uint32_t pre = static_cast<uint32_t>(E) * c.S * sz;
  const uint32_t self = static_cast<uint32_t>(c.i);
  if (offd) {
    const HEOM_GLOBAL T *blk = c.X + static_cast<uint32_t>(E) * c.S;
    auto off = [&](int j) -> uint32_t {
      return (j >= 0 ? static_cast<uint32_t>(j) : self) * (2 * sz);
    };
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int ma = a * KP + k, mb = b * KP + k;
      L.jua[k] = c.sup[ma * kWideAdos + t];
      L.jub[k] = c.sup[mb * kWideAdos + t];
      const int jda = c.sdn[ma * kWideAdos + t], jdb = c.sdn[mb * kWideAdos + t];
      const Pair2<T> ya = ld_pair(blk, off(L.jua[k])), yb = ld_pair(blk, off(L.jub[k]));
      const Pair2<T> za = ld_pair(blk, off(jda)), zb = ld_pair(blk, off(jdb));
      L.yar[k] = static_cast<C>(ya.x);
      L.yai[k] = static_cast<C>(ya.y);
      L.ybr[k] = static_cast<C>(yb.x);
      L.ybi[k] = static_cast<C>(yb.y);
      L.zar[k] = static_cast<C>(za.x);
      L.zai[k] = static_cast<C>(za.y);
      L.zbr[k] = static_cast<C>(zb.x);
      L.zbi[k] = static_cast<C>(zb.y);
    }
    if constexpr (X0SRC) {
      L.str = static_cast<C>(c.y0[E]);
      L.sti = static_cast<C>(c.y0[E + 1]);
    } else {
      const Pair2<T> st = ld_pair(c.Yp + static_cast<uint32_t>(E) * c.S, self * (2 * sz));
      L.str = static_cast<C>(st.x);
      L.sti = static_cast<C>(st.y);
    }
  } else {
    auto off = [&](int j) -> uint32_t { return (j >= 0 ? static_cast<uint32_t>(j) : self) * sz; };
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int ma = a * KP + k, mb = b * KP + k;
      L.jua[k] = c.sup[ma * kWideAdos + t];
      L.jub[k] = c.sup[mb * kWideAdos + t];
      const int jda = c.sdn[ma * kWideAdos + t], jdb = c.sdn[mb * kWideAdos + t];
      L.yar[k] = L.yai[k] = L.ybr[k] = L.ybi[k] = C(0);
      L.zar[k] = static_cast<C>(ld_off(c.X, pre + off(jda)));
      L.zbr[k] = static_cast<C>(ld_off(c.X, pre + off(jdb)));
      L.zai[k] = L.zbi[k] = C(0);
    }
    L.sti = C(0);
    if constexpr (X0SRC)
      L.str = static_cast<C>(c.y0[E]);
    else
      L.str = static_cast<C>(ld_off(c.Yp, pre + self * sz));
  }
}

// Phase 2 of element (a, b) (tile_finish with runtime a, b): the commutator
// from LDS over the nonzero couplings in increasing k (negating an imaginary
// part equals the tile kernel's multiplication by -1), then decay, bath
// couplings, RK4 stage and store, in the tile kernel's order.  SCALED: the
// hierarchy holds sigma_n / w_n, so the coupling to n + e_m is weighted by
// sqrt((n_m + 1)|c_m|) instead of 1 and the one to n - e_m by sqrt(n_m / |c_m|)
// instead of n_m (weights from the host, by mode and occupation).
template <typename C, typename T, bool X0SRC, int KP, bool SCALED>
__device__ __forceinline__ void wide_finish(const WideCtx<T> &c, int a, int b,
                                            const WideLoads<C, KP> &L) {
#pragma clang fp contract(off)
  const int N = c.N, t = c.t;
  const char *sxt = reinterpret_cast<const char *>(c.sx) + t * sizeof(T);
  auto xre = [&](uint32_t off) -> C {
    if constexpr (X0SRC) {
      const int e = wide_plane<T>(off);
      return e < N * N ? static_cast<C>(c.sx0[e]) : C(0);
    } else {
      return static_cast<C>(*reinterpret_cast<const T *>(sxt + off));
    }
  };
  // The entry's sign bit moved onto the value (negation, exact).
  auto xim = [&](uint32_t im) -> C {
    const C v = xre(im & 0x7fffffffu);
    if constexpr (sizeof(C) == 8) {
      const uint64_t u = static_cast<uint64_t>(__double_as_longlong(static_cast<double>(v))) ^
                         (static_cast<uint64_t>(im & 0x80000000u) << 32);
      return static_cast<C>(__longlong_as_double(static_cast<long long>(u)));
    } else {
      return static_cast<C>(
          __uint_as_float(__float_as_uint(static_cast<float>(v)) ^ (im & 0x80000000u)));
    }
  };
  // H_rc of an entry: the FP64 pass of sigma_0 reads FP64 H.
  auto hval = [&](const WideEntry &e, int rc) -> C {
    if constexpr (X0SRC)
      return static_cast<C>(c.hg[rc]);
    else
      return static_cast<C>(wide_h_value<T>(e.h));
  };
  const WideEntry eab = c.sent[a * N + b];
  const bool offd = a != b;
  const WideEntry *rowA = c.sent + a * N;
  const WideEntry *colB = c.sent + b;
  C sr = C(0), si = C(0);
  uint32_t mask = c.snz[a] | c.snz[b];
  while (mask) {
    const int k = __builtin_ctz(mask);
    mask &= mask - 1;
    const WideEntry eak = rowA[k];
    const WideEntry ekb = colB[k * N];
    const C hak = hval(eak, a * N + k);
    const C hkb = hval(ekb, k * N + b);
    const C xkb_r = xre(ekb.re);
    const C xkb_i = xim(ekb.im);
    const C xak_r = xre(eak.re);
    const C xak_i = xim(eak.im);
    sr = fmad(-xak_r, hkb, fmad(hak, xkb_r, sr));
    si = fmad(-xak_i, hkb, fmad(hak, xkb_i, si));
  }
  C ar = si, ai = -sr;
  const C xr = xre(eab.re), xi = xim(eab.im);
  C dec = static_cast<C>(c.damp) + static_cast<C>(c.sdec[a]) + static_cast<C>(c.sdec[b]);
  if (offd) dec += static_cast<C>(c.sdl[a]) + static_cast<C>(c.sdl[b]);
  ar = fmad(-dec, xr, ar);
  ai = fmad(-dec, xi, ai);
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int ma = a * KP + k, mb = b * KP + k;
    const int oa = c.socc[ma * kWideAdos + t], ob = c.socc[mb * kWideAdos + t];
    if (offd) {
      C fa = L.jua[k] >= 0 ? C(1) : C(0);
      C fb = L.jub[k] >= 0 ? C(1) : C(0);
      if constexpr (SCALED) {
        fa = L.jua[k] >= 0 ? static_cast<C>(c.swu[ma * c.levels + oa]) : C(0);
        fb = L.jub[k] >= 0 ? static_cast<C>(c.swu[mb * c.levels + ob]) : C(0);
      }
      ar = fmad(-fa, L.yai[k], fmad(fb, L.ybi[k], ar));
      ai = fmad(-fb, L.ybr[k], fmad(fa, L.yar[k], ai));
    }
    const C za_i = offd ? L.zai[k] : C(0);
    const C zb_i = offd ? L.zbi[k] : C(0);
    C na = static_cast<C>(oa), nb = static_cast<C>(ob);
    if constexpr (SCALED) {
      na = static_cast<C>(c.swd[ma * c.levels + oa]);
      nb = static_cast<C>(c.swd[mb * c.levels + ob]);
    }
    const C car = na * static_cast<C>(c.scr[ma]), cai = na * static_cast<C>(c.sci[ma]);
    const C cbr = nb * static_cast<C>(c.scr[mb]), cbi = nb * static_cast<C>(c.sci[mb]);
    ar = fmad(-car, za_i, fmad(-cai, L.zar[k], ar));
    ai = fmad(-cai, za_i, fmad(car, L.zar[k], ai));
    ar = fmad(-cbi, L.zbr[k], fmad(cbr, zb_i, ar));
    ai = fmad(-cbi, zb_i, fmad(-cbr, L.zbr[k], ai));
  }
  const C coef = static_cast<C>(c.coef);
  const C nr = fmad(coef, ar, L.str);
  const C ni = fmad(coef, ai, L.sti);
  const int E = wide_plane<T>(eab.re);
  if constexpr (X0SRC) {
    c.out0[E] = nr;
    if (offd) c.out0[E + 1] = ni;
  }
  const uint32_t sz = static_cast<uint32_t>(sizeof(T));
  const uint32_t base = static_cast<uint32_t>(E) * c.S * sz;
  if (offd)
    st_pair<false>(c.Out + static_cast<uint32_t>(E) * c.S, static_cast<uint32_t>(c.i) * (2 * sz),
                   static_cast<T>(nr), static_cast<T>(ni));
  else
    st_off<false>(c.Out, base + static_cast<uint32_t>(c.i) * sz, static_cast<T>(nr));
}

template <typename T, int KP, bool SCALED>
__global__ void __launch_bounds__(64 * kWideWaves)
    stage_wide(const InstDesc *__restrict__ descs, const WorkItem *__restrict__ work, int stage,
               double coef, int /*hist_slot: recorded by the snapshot kernel*/) {
  extern __shared__ __align__(16) char wide_smem[];
  constexpr bool MIXED = sizeof(T) == 4;
  const WorkItem w = work[blockIdx.x];
  const InstDesc &d = descs[w.inst];
  const int N = d.N, M = d.M, N2 = N * N, P = N * (N + 1) / 2;
  const int levels = SCALED ? d.levels : 0;
  const WideLds L = wide_lds(N, M, static_cast<int>(sizeof(T)), levels);
  T *sx = reinterpret_cast<T *>(wide_smem + L.x);
  WideEntry *sent = reinterpret_cast<WideEntry *>(wide_smem + L.ent);
  uint32_t *snz = reinterpret_cast<uint32_t *>(wide_smem + L.nz);
  double *sdec = reinterpret_cast<double *>(wide_smem + L.dec);
  double *sdl = reinterpret_cast<double *>(wide_smem + L.dl);
  double *scr = reinterpret_cast<double *>(wide_smem + L.cr);
  double *sci = reinterpret_cast<double *>(wide_smem + L.ci);
  double *snu = reinterpret_cast<double *>(wide_smem + L.nu);
  int32_t *sup = reinterpret_cast<int32_t *>(wide_smem + L.up);
  int32_t *sdn = reinterpret_cast<int32_t *>(wide_smem + L.dn);
  uint8_t *socc = reinterpret_cast<uint8_t *>(wide_smem + L.occ);
  uint8_t *spa = reinterpret_cast<uint8_t *>(wide_smem + L.pa);
  uint8_t *spb = reinterpret_cast<uint8_t *>(wide_smem + L.pb);
  double *sx0 = reinterpret_cast<double *>(wide_smem + L.x0);
  double *swu = reinterpret_cast<double *>(wide_smem + L.wu);
  double *swd = reinterpret_cast<double *>(wide_smem + L.wd);

  const StageBufs bufs = stage_bufs(d, stage);
  const int64_t S = d.stride;
  const int tid = threadIdx.x;
  const HEOM_GLOBAL T *X = gmem(static_cast<const T *>(bufs.x));
  const HEOM_GLOBAL double *Pg = gmem(d.params);
  const ParamOffsets o = param_offsets(N, M);
  // Stage the tile (invalid ADOs of the last tile read ADO 0 and store 0),
  // the entry table with H, the parameters, the neighbour tables and the
  // element map.
  // Element slots: slot s < N is diagonal plane s, slot N + p pair p's block
  // (both parts in one access).
  const int NS = N * (N + 1) / 2;
  for (int idx = tid; idx < NS * kWideAdos; idx += blockDim.x) {
    const int sl = idx / kWideAdos, t = idx % kWideAdos;
    const int64_t i = static_cast<int64_t>(w.first) + t;
    const bool ok = i < d.n_ados;
    const int64_t ic = ok ? i : 0;
    if (sl < N) {
      const T v = X[sl * S + ic];
      sx[sl * kWideAdos + t] = ok ? v : T(0);
    } else {
      const int e = N + 2 * (sl - N);
      const Pair2<T> v = ld_pair(X + e * S, static_cast<uint32_t>(ic) * 2u * sizeof(T));
      sx[e * kWideAdos + t] = ok ? v.x : T(0);
      sx[(e + 1) * kWideAdos + t] = ok ? v.y : T(0);
    }
  }
  if (tid < kWideAdos) sx[N2 * kWideAdos + tid] = T(0);
  constexpr uint32_t kPlaneBytes = kWideAdos * sizeof(T);
  for (int idx = tid; idx < N2; idx += blockDim.x) {
    const int r = idx / N, c = idx % N;
    sent[idx] = WideEntry{static_cast<uint32_t>(ent_re(N, r, c)) * kPlaneBytes,
                          static_cast<uint32_t>(ent_im(N, r, c)) * kPlaneBytes |
                              (r > c ? 0x80000000u : 0u),
                          wide_h_slot<T>(Pg[o.h_re + idx])};
  }
  for (int idx = tid; idx < N; idx += blockDim.x) {
    uint32_t m = 0;
    for (int k = 0; k < N; ++k)
      if (Pg[o.h_re + idx * N + k] != 0.0) m |= 1u << k;
    snz[idx] = m;
    sdec[idx] = Pg[o.half_gamma + idx];
    sdl[idx] = Pg[o.delta + idx];
  }
  for (int idx = tid; idx < M; idx += blockDim.x) {
    scr[idx] = Pg[o.c_re + idx];
    sci[idx] = Pg[o.c_im + idx];
    snu[idx] = Pg[o.nu + idx];
  }
  const bool t16 = d.up16 != nullptr;
  const HEOM_GLOBAL char *upb = (const HEOM_GLOBAL char *)(
      t16 ? reinterpret_cast<const char *>(d.up16) : reinterpret_cast<const char *>(d.up));
  const HEOM_GLOBAL char *dnb = (const HEOM_GLOBAL char *)(
      t16 ? reinterpret_cast<const char *>(d.down16) : reinterpret_cast<const char *>(d.down));
  const uint32_t row_bytes = static_cast<uint32_t>(S) * (t16 ? 2u : 4u);
  for (int idx = tid; idx < M * kWideAdos; idx += blockDim.x) {
    const int m = idx / kWideAdos, t = idx % kWideAdos;
    const int64_t i = static_cast<int64_t>(w.first) + t;
    const bool ok = i < d.n_ados;
    const uint32_t ic = static_cast<uint32_t>(ok ? i : 0);
    const int ju = table_decode(table_load(upb + m * row_bytes, t16, ic), t16, ic);
    const int jd = table_decode(table_load(dnb + m * row_bytes, t16, ic), t16, ic);
    sup[idx] = ok ? ju : -1;
    sdn[idx] = ok ? jd : -1;
    socc[idx] = ok ? gmem(d.occ)[m * S + i] : 0;
  }
  for (int p = tid; p < P; p += blockDim.x) {
    spa[p] = static_cast<uint8_t>(elem_a(N, p));
    spb[p] = static_cast<uint8_t>(elem_b(N, p));
  }
  for (int idx = tid; idx < M * levels; idx += blockDim.x) {  // scaled only
    swu[idx] = Pg[o.total + idx];
    swd[idx] = Pg[o.total + M * levels + idx];
  }
  if constexpr (MIXED) {
    if (w.first == 0)
      for (int e = tid; e < N2; e += blockDim.x) sx0[e] = bufs.x0[e];
  }
  __syncthreads();
  // Sink fluxes and scalars of sigma_0: wave 0 of the first tile.
  if (w.first == 0 && tid < 64 && !(d.flags & kInstNoSigma0)) {
    scalar_update_wave(d, bufs, N, coef, tid, [&](int e) {
      if constexpr (MIXED)
        return sx0[e];
      else
        return static_cast<double>(sx[e * kWideAdos]);
    });
  }

  const int lane = tid & 63;
  const int t = lane % kWideAdos;
  const int slot = (tid >> 6) * (64 / kWideAdos) + lane / kWideAdos;
  const int64_t i = static_cast<int64_t>(w.first) + t;
  auto make_ctx = [&](int tt, int64_t ii) {
    double damp = 0.0;
    for (int m = 0; m < M; ++m)
      damp = fmad(static_cast<double>(socc[m * kWideAdos + tt]), snu[m], damp);
    return WideCtx<T>{N,
                      tt,
                      sx,
                      sent,
                      sdec,
                      sdl,
                      scr,
                      sci,
                      snz,
                      sup,
                      sdn,
                      socc,
                      X,
                      gmem(static_cast<const T *>(bufs.y)),
                      gmem(static_cast<T *>(bufs.out)),
                      sx0,
                      Pg + o.h_re,
                      gmem(bufs.y0),
                      gmem(bufs.out0),
                      static_cast<uint32_t>(S),
                      ii,
                      damp,
                      coef,
                      swu,
                      swd,
                      levels};
  };
  // With FP32 storage, sigma_0 is computed separately below, in FP64.
  if (i < d.n_ados && !(MIXED && i == 0)) {
    const WideCtx<T> ctx = make_ctx(t, i);
    for (int p = slot; p < P; p += kWideSlots) {
      WideLoads<T, KP> Ld;
      wide_load<T, T, false, KP>(ctx, spa[p], spb[p], Ld);
      wide_finish<T, T, false, KP, SCALED>(ctx, spa[p], spb[p], Ld);
    }
  }
  if constexpr (MIXED) {
    // sigma_0 in FP64 from its FP64 copies, its elements spread over the
    // whole workgroup of the first tile.
    if (w.first == 0) {
      const WideCtx<T> ctx0 = make_ctx(0, 0);
      for (int p = tid; p < P; p += blockDim.x) {
        WideLoads<double, KP> L0;
        wide_load<double, T, true, KP>(ctx0, spa[p], spb[p], L0);
        wide_finish<double, T, true, KP, SCALED>(ctx0, spa[p], spb[p], L0);
      }
    }
  }
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
  const bool s0 = i == 0 && !(d.flags & kInstNoSigma0);
  for (int e = 0; e < N2; ++e)
    y[elem_index(d.N, e, d.stride, i)] = s0 ? static_cast<T>(d.params[o.rho0 + e]) : T(0);
  if (s0) {
    if (sizeof(T) == 4)
      for (int e = 0; e < N2; ++e) d.y0[e] = d.params[o.rho0 + e];
    for (int k = 0; k < kScalars; ++k) d.sc_y[k] = 0.0;
  }
}

// Copies the halo ADOs of split hierarchies into the input buffer of `stage`
// (one lane per halo ADO, a loop over the rows and columns of its linking
// sites): on one GPU this stands in for the point-to-point exchange between
// the ranks that hold the shares.
template <typename T>
__global__ void __launch_bounds__(256) halo_fill(const InstDesc *__restrict__ descs,
                                                 const HaloEntry *__restrict__ list, int n,
                                                 int stage) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const HaloEntry h = list[q];
  const InstDesc &dd = descs[h.dst];
  const InstDesc &ds = descs[h.src];
  const T *src = static_cast<const T *>(stage_bufs(ds, stage).x);
  T *dst = static_cast<T *>(const_cast<void *>(stage_bufs(dd, stage).x));
  const int N = dd.N;
  auto copy = [&](int e) {
    dst[elem_index(dd.N, e, dd.stride, h.dst_index)] = src[elem_index(ds.N, e, ds.stride, h.src_index)];
  };
  for (int a = 0; a < N; ++a) {
    const bool in_a = (h.sites >> a) & 1;
    if (in_a) copy(a);
    for (int b = a + 1; b < N; ++b)
      if (in_a || ((h.sites >> b) & 1)) {
        copy(re_plane(N, a, b));
        copy(re_plane(N, a, b) + 1);
      }
  }
}

// The filter of a scaled hierarchy, after the last stage of a step: every ADO
// n != 0 (one lane each, one workgroup per 64-ADO work item) whose stored
// reals are all below the instance's threshold in absolute value is set to
// zero in the state.
template <typename T>
__global__ void __launch_bounds__(64) filter_ados(const InstDesc *__restrict__ descs,
                                                   const WorkItem *__restrict__ work) {
  const WorkItem w = work[blockIdx.x];
  const InstDesc &d = descs[w.inst];
  const int64_t i = static_cast<int64_t>(w.first) + threadIdx.x;
  if (i >= d.n_ados || (i == 0 && !(d.flags & kInstNoSigma0))) return;
  T *y = static_cast<T *>(d.y);
  const int N2 = d.N * d.N;
  double mx = 0.0;
  for (int e = 0; e < N2; ++e)
    mx = fmax(mx, fabs(static_cast<double>(y[elem_index(d.N, e, d.stride, i)])));
  if (mx < d.filter_tol)
    for (int e = 0; e < N2; ++e) y[elem_index(d.N, e, d.stride, i)] = T(0);
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
    h[e] = (sizeof(T) == 4) ? d.y0[e] : static_cast<double>(y[elem_index(d.N, e, d.stride, 0)]);
  if (threadIdx.x < 3) h[N2 + threadIdx.x] = d.sc_y[threadIdx.x];
}

}  // namespace

}  // namespace heom
