// resident_kernel.h -- whole RK4 steps of small hierarchies in one workgroup.
//
// A hierarchy whose state, two stage buffers and neighbour tables fit in one
// CU's LDS needs no kernel boundary between its RK4 stages: every coupling
// (eq:lab8, the n +- e_m links) stays inside the workgroup, so a workgroup
// barrier orders the stages.  One workgroup per instance loads the state from
// its workspace, runs a chunk of steps (all four stages of the nested RK4 form
// per step, the sink scalars by one wave, the sigma_0 records straight into the
// history ring) and writes the state back.  This removes the launch floor of
// about 5 us per stage that bounds a plain solve of a small hierarchy.
//
// Each packed element is computed with the operations of the tile kernel's
// tile_finish, in its order (the same explicit fused multiply-adds, the same
// zero weights for missing neighbours), so the two paths agree bitwise.
//
// Included after stage_kernels.h (fmad, ent_re, scalar_update_wave, ...).

#pragma once

namespace heom {
namespace {

constexpr int kResidentThreads = 1024;

// Workgroup barrier that orders LDS only.  Every value shared between the
// waves lives in LDS; the global stores of the records need no ordering
// inside the kernel, so the barrier does not wait for them.
__device__ __forceinline__ void res_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS layout of the resident kernel (byte offsets, 16-byte aligned regions)
// for an instance of n ADOs: the state Y and the stage buffers A and B as
// [N*N + 1][n] planes (plane N*N is zero: the imaginary part of a diagonal
// entry), the neighbour tables [M][n], H_re, the decay, delta, sink and mode
// parameters, the per-ADO damping sum, the scalar blocks of Y, A and B, and
// the packed element map.
struct ResidentLds {
  int y, a, b, up, dn, occ, h, hg, dl, tr, rc, cr, ci, damp, sc, pa, pb, total;
};
__host__ __device__ inline int res_align(int v) { return (v + 15) & ~15; }
__host__ __device__ inline ResidentLds resident_lds(int N, int M, int n) {
  const int P = N * (N + 1) / 2;
  const int plane_bytes = (N * N + 1) * n * 8;
  ResidentLds L;
  L.y = 0;
  L.a = res_align(L.y + plane_bytes);
  L.b = res_align(L.a + plane_bytes);
  L.up = res_align(L.b + plane_bytes);
  L.dn = res_align(L.up + M * n * 4);
  L.occ = res_align(L.dn + M * n * 4);
  L.h = res_align(L.occ + M * n);
  L.hg = res_align(L.h + N * N * 8);
  L.dl = res_align(L.hg + N * 8);
  L.tr = res_align(L.dl + N * 8);
  L.rc = res_align(L.tr + N * 8);
  L.cr = res_align(L.rc + N * 8);
  L.ci = res_align(L.cr + M * 8);
  L.damp = res_align(L.ci + M * 8);
  L.sc = res_align(L.damp + n * 8);
  L.pa = res_align(L.sc + 3 * kScalars * 8);
  L.pb = res_align(L.pa + P);
  L.total = res_align(L.pb + P);
  return L;
}

struct ResidentCtx {
  int N, KP, n;
  const double *x;   // stage input planes
  const double *y;   // state planes
  double *out;       // output planes
  const double *h, *hg, *dl, *cr, *ci, *damp;
  const int32_t *up, *dn;
  const uint8_t *occ;
};

// Packed element (A, B) of ADO i: tile_finish's right-hand side and stage
// update with runtime A and B, every operand read from LDS.
__device__ __forceinline__ void resident_element(const ResidentCtx &c, int A, int B, int i,
                                                 double coef) {
#pragma clang fp contract(off)
  const int N = c.N, n = c.n;
  auto xe = [&](int e) -> double { return c.x[e * n + i]; };
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < N; ++k) {
    const double hak = c.h[A * N + k];
    const double hkb = c.h[k * N + B];
    const double xkb_r = xe(ent_re(N, k, B));
    const double xkb_i = static_cast<double>(ent_sg(k, B)) * xe(ent_im(N, k, B));
    const double xak_r = xe(ent_re(N, A, k));
    const double xak_i = static_cast<double>(ent_sg(A, k)) * xe(ent_im(N, A, k));
    sr = fmad(-xak_r, hkb, fmad(hak, xkb_r, sr));
    si = fmad(-xak_i, hkb, fmad(hak, xkb_i, si));
  }
  double ar = si, ai = -sr;
  const int E = ent_re(N, A, B);
  const bool offd = A != B;
  const double xr = xe(E), xi = xe(ent_im(N, A, B));
  double dec = c.damp[i] + c.hg[A] + c.hg[B];
  if (offd) dec += c.dl[A] + c.dl[B];
  ar = fmad(-dec, xr, ar);
  ai = fmad(-dec, xi, ai);
  const double *pre = c.x + E * n;
  const double *pim = c.x + (offd ? E + 1 : E) * n;
  for (int k = 0; k < c.KP; ++k) {
    const int ma = A * c.KP + k, mb = B * c.KP + k;
    if (offd) {
      // Deeper neighbours; a missing one reads the ADO's own entry, weighted
      // by zero.
      const int ja = c.up[ma * n + i], jb = c.up[mb * n + i];
      const int oa = ja >= 0 ? ja : i, ob = jb >= 0 ? jb : i;
      const double yar = pre[oa], yai = pim[oa], ybr = pre[ob], ybi = pim[ob];
      const double fa = ja >= 0 ? 1.0 : 0.0;
      const double fb = jb >= 0 ? 1.0 : 0.0;
      ar = fmad(-fa, yai, fmad(fb, ybi, ar));
      ai = fmad(-fb, ybr, fmad(fa, yar, ai));
    }
    // Shallower neighbours (occupation zero exactly where one is missing).
    const int da = c.dn[ma * n + i], db = c.dn[mb * n + i];
    const int oa = da >= 0 ? da : i, ob = db >= 0 ? db : i;
    const double zar = pre[oa], zbr = pre[ob];
    const double zai = offd ? pim[oa] : 0.0;
    const double zbi = offd ? pim[ob] : 0.0;
    const double na = static_cast<double>(c.occ[ma * n + i]);
    const double nb = static_cast<double>(c.occ[mb * n + i]);
    const double car = na * c.cr[ma], cai = na * c.ci[ma];
    const double cbr = nb * c.cr[mb], cbi = nb * c.ci[mb];
    ar = fmad(-car, zai, fmad(-cai, zar, ar));
    ai = fmad(-cai, zai, fmad(car, zar, ai));
    ar = fmad(-cbi, zbr, fmad(cbr, zbi, ar));
    ai = fmad(-cbi, zbi, fmad(-cbr, zbr, ai));
  }
  const double str = c.y[E * n + i];
  const double sti = offd ? c.y[(E + 1) * n + i] : 0.0;
  c.out[E * n + i] = fmad(coef, ar, str);
  if (offd) c.out[(E + 1) * n + i] = fmad(coef, ai, sti);
}

// Runs steps step0 + 1 ... step0 + n_steps of instance blockIdx.x (FP64
// storage, real H, ADO 0 = sigma_0).  With record_every > 0, the state after
// every step whose index is a multiple of record_every is recorded in history
// slots slot0, slot0 + 1, ... (the host sizes the chunk so that they exist).
__global__ void __launch_bounds__(kResidentThreads)
    stage_resident(const InstDesc *__restrict__ descs, int64_t step0, int64_t n_steps,
                   int64_t record_every, int slot0, double dt) {
  extern __shared__ __align__(16) char res_smem[];
  const InstDesc &d = descs[blockIdx.x];
  const int N = d.N, M = d.M, N2 = N * N, P = N * (N + 1) / 2;
  const int n = static_cast<int>(d.n_ados);
  const int64_t S = d.stride;
  const ResidentLds L = resident_lds(N, M, n);
  double *Y = reinterpret_cast<double *>(res_smem + L.y);
  double *A = reinterpret_cast<double *>(res_smem + L.a);
  double *B = reinterpret_cast<double *>(res_smem + L.b);
  int32_t *up = reinterpret_cast<int32_t *>(res_smem + L.up);
  int32_t *dn = reinterpret_cast<int32_t *>(res_smem + L.dn);
  uint8_t *occ = reinterpret_cast<uint8_t *>(res_smem + L.occ);
  double *H = reinterpret_cast<double *>(res_smem + L.h);
  double *hg = reinterpret_cast<double *>(res_smem + L.hg);
  double *dl = reinterpret_cast<double *>(res_smem + L.dl);
  double *tr = reinterpret_cast<double *>(res_smem + L.tr);
  double *rc = reinterpret_cast<double *>(res_smem + L.rc);
  double *cr = reinterpret_cast<double *>(res_smem + L.cr);
  double *ci = reinterpret_cast<double *>(res_smem + L.ci);
  double *damp = reinterpret_cast<double *>(res_smem + L.damp);
  double *sc = reinterpret_cast<double *>(res_smem + L.sc);  // [Y, A, B][kScalars]
  uint8_t *pa = reinterpret_cast<uint8_t *>(res_smem + L.pa);
  uint8_t *pb = reinterpret_cast<uint8_t *>(res_smem + L.pb);
  const int tid = threadIdx.x;
  const int KP = d.KP;
  double *const hist = d.hist;
  const double *yg = static_cast<const double *>(d.y);
  const ParamOffsets o = param_offsets(N, M);

  for (int q = tid; q < (N2 + 1) * n; q += kResidentThreads) {
    const int e = q / n, i = q % n;
    Y[q] = e < N2 ? yg[e * S + i] : 0.0;
    A[q] = 0.0;
    B[q] = 0.0;
  }
  for (int q = tid; q < M * n; q += kResidentThreads) {
    const int m = q / n, i = q % n;
    up[q] = d.up[m * S + i];
    dn[q] = d.down[m * S + i];
    occ[q] = d.occ[m * S + i];
  }
  for (int q = tid; q < N2; q += kResidentThreads) H[q] = d.params[o.h_re + q];
  for (int q = tid; q < N; q += kResidentThreads) {
    hg[q] = d.params[o.half_gamma + q];
    dl[q] = d.params[o.delta + q];
    tr[q] = d.params[o.trap + q];
    rc[q] = d.params[o.rec + q];
  }
  for (int q = tid; q < M; q += kResidentThreads) {
    cr[q] = d.params[o.c_re + q];
    ci[q] = d.params[o.c_im + q];
  }
  for (int p = tid; p < P; p += kResidentThreads) {
    pa[p] = static_cast<uint8_t>(elem_a(N, p));
    pb[p] = static_cast<uint8_t>(elem_b(N, p));
  }
  for (int q = tid; q < 3 * kScalars; q += kResidentThreads) sc[q] = q < kScalars ? d.sc_y[q] : 0.0;
  __syncthreads();
  // The damping sum of each ADO, in the tile kernel's order of modes.
  for (int i = tid; i < n; i += kResidentThreads) {
    double s = 0.0;
    for (int m = 0; m < M; ++m)
      s = fmad(static_cast<double>(occ[m * n + i]), d.params[o.nu + m], s);
    damp[i] = s;
  }
  res_barrier();

  const double coef[4] = {dt / 4.0, dt / 3.0, dt / 2.0, dt};
  // Stage buffers as in stage_bufs: Y -> A -> B -> A -> Y.
  double *const xin[4] = {Y, A, B, A};
  double *const xout[4] = {A, B, A, Y};
  const int sin_[4] = {0, 1, 2, 1};
  const int sout[4] = {1, 2, 1, 0};
  const int wave = tid >> 6, lane = tid & 63;
  int slot = slot0;
  for (int64_t s = 0; s < n_steps; ++s) {
    for (int st = 0; st < 4; ++st) {
      if (wave == kResidentThreads / 64 - 1) {
        // scalar_update_wave's operations, with the sink rates from LDS, on
        // the last wave (the element items fill the first waves first).
        const double *x = xin[st];
        double ft = 0.0, fr = 0.0;
        for (int q = lane; q < N; q += 64) {
          const double pop = x[q * n];
          ft = fmad(tr[q], pop, ft);
          fr = fmad(rc[q], pop, fr);
        }
        ft = wave_sum(ft);
        fr = wave_sum(fr);
        if (lane == 0) {
          const double *xs = sc + sin_[st] * kScalars;
          double *outs = sc + sout[st] * kScalars;
          const double xq = xs[0];
          const double y_t = sc[0], y_r = sc[1], y_q = sc[2];
          outs[0] = fmad(coef[st], ft, y_t);
          outs[1] = fmad(coef[st], fr, y_r);
          outs[2] = fmad(coef[st], xq, y_q);
        }
      }
      const ResidentCtx c{N, KP, n, xin[st], Y, xout[st], H, hg, dl, cr, ci, damp, up, dn, occ};
      for (int q = tid; q < P * n; q += kResidentThreads) {
        const int p = q / n, i = q % n;
        resident_element(c, pa[p], pb[p], i, coef[st]);
      }
      res_barrier();
    }
    if (record_every > 0 && (step0 + s + 1) % record_every == 0) {
      double *h = hist + static_cast<int64_t>(slot) * (N2 + kScalars);
      for (int e = tid; e < N2; e += kResidentThreads) h[e] = Y[e * n];
      if (tid < 3) h[N2 + tid] = sc[tid];
      ++slot;
    }
  }
  double *yo = static_cast<double *>(d.y);
  for (int q = tid; q < N2 * n; q += kResidentThreads) yo[(q / n) * S + q % n] = Y[q];
  if (tid < 3) d.sc_y[tid] = sc[tid];
}

}  // namespace
}  // namespace heom
