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
// Two forms: stage_resident reads N and K+1 of each instance at run time (a
// batch may mix hierarchies) and keeps the planes of the stage launches in
// LDS; stage_resident_fixed is compiled per (N, K+1) and keeps full matrices,
// so each thread's operands sit at fixed offsets (below).  Each packed
// element is computed with the operations of the tile kernel's tile_finish,
// in its order (the same explicit fused multiply-adds, the same zero weights
// for missing neighbours), so every path agrees bitwise.
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

// wave_sum's lane-0 result where lanes 0 .. N-1 (N <= 8) hold term(0 .. N-1)
// and the other lanes zero, as one lane's additions in the butterfly's
// order: offsets 32, 16 and 8 add zeros (which only turn -0 into +0), then
// 4, 2 and 1 pair the sites.  Bitwise equal to wave_sum, without its chain
// of dependent shuffles (the scalar wave's longest chain in a stage of the
// compile-time kernel).
template <typename Term>
__device__ __forceinline__ double site_sum(int N, Term term) {
#pragma clang fp contract(off)
  double w[8];
#pragma unroll
  for (int l = 0; l < 8; ++l) w[l] = l < N ? term(l) + 0.0 : 0.0;
  return ((w[0] + w[4]) + (w[2] + w[6])) + ((w[1] + w[5]) + (w[3] + w[7]));
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

// Pointers into the LDS layout of one instance.
struct ResidentView {
  double *Y, *A, *B, *H, *hg, *dl, *tr, *rc, *cr, *ci, *damp, *sc;  // sc: [Y, A, B][kScalars]
  int32_t *up, *dn;
  uint8_t *occ, *pa, *pb;
};
__device__ __forceinline__ ResidentView resident_view(char *smem, const ResidentLds &L) {
  ResidentView v;
  v.Y = reinterpret_cast<double *>(smem + L.y);
  v.A = reinterpret_cast<double *>(smem + L.a);
  v.B = reinterpret_cast<double *>(smem + L.b);
  v.H = reinterpret_cast<double *>(smem + L.h);
  v.hg = reinterpret_cast<double *>(smem + L.hg);
  v.dl = reinterpret_cast<double *>(smem + L.dl);
  v.tr = reinterpret_cast<double *>(smem + L.tr);
  v.rc = reinterpret_cast<double *>(smem + L.rc);
  v.cr = reinterpret_cast<double *>(smem + L.cr);
  v.ci = reinterpret_cast<double *>(smem + L.ci);
  v.damp = reinterpret_cast<double *>(smem + L.damp);
  v.sc = reinterpret_cast<double *>(smem + L.sc);
  v.up = reinterpret_cast<int32_t *>(smem + L.up);
  v.dn = reinterpret_cast<int32_t *>(smem + L.dn);
  v.occ = reinterpret_cast<uint8_t *>(smem + L.occ);
  v.pa = reinterpret_cast<uint8_t *>(smem + L.pa);
  v.pb = reinterpret_cast<uint8_t *>(smem + L.pb);
  return v;
}

// Copies instance d (n ADOs) into LDS: the state, zeroed stage buffers, the
// neighbour tables, the parameters, the packed element map and the scalars,
// then the damping sum of each ADO (in the tile kernel's order of modes).
// Ends with a barrier.
__device__ __forceinline__ void resident_load(const InstDesc &d, const ResidentView &v, int N,
                                              int M, int n, int tid) {
#pragma clang fp contract(off)
  const int N2 = N * N, P = N * (N + 1) / 2;
  const int64_t S = d.stride;
  const double *yg = static_cast<const double *>(d.y);
  const ParamOffsets o = param_offsets(N, M);
  for (int q = tid; q < (N2 + 1) * n; q += kResidentThreads) {
    const int e = q / n, i = q % n;
    v.Y[q] = e < N2 ? yg[elem_index(N, e, S, i)] : 0.0;
    v.A[q] = 0.0;
    v.B[q] = 0.0;
  }
  for (int q = tid; q < M * n; q += kResidentThreads) {
    const int m = q / n, i = q % n;
    v.up[q] = d.up[m * S + i];
    v.dn[q] = d.down[m * S + i];
    v.occ[q] = d.occ[m * S + i];
  }
  for (int q = tid; q < N2; q += kResidentThreads) v.H[q] = d.params[o.h_re + q];
  for (int q = tid; q < N; q += kResidentThreads) {
    v.hg[q] = d.params[o.half_gamma + q];
    v.dl[q] = d.params[o.delta + q];
    v.tr[q] = d.params[o.trap + q];
    v.rc[q] = d.params[o.rec + q];
  }
  for (int q = tid; q < M; q += kResidentThreads) {
    v.cr[q] = d.params[o.c_re + q];
    v.ci[q] = d.params[o.c_im + q];
  }
  for (int p = tid; p < P; p += kResidentThreads) {
    v.pa[p] = static_cast<uint8_t>(elem_a(N, p));
    v.pb[p] = static_cast<uint8_t>(elem_b(N, p));
  }
  for (int q = tid; q < 3 * kScalars; q += kResidentThreads)
    v.sc[q] = q < kScalars ? d.sc_y[q] : 0.0;
  __syncthreads();
  for (int i = tid; i < n; i += kResidentThreads) {
    double s = 0.0;
    for (int m = 0; m < M; ++m)
      s = fmad(static_cast<double>(v.occ[m * n + i]), d.params[o.nu + m], s);
    v.damp[i] = s;
  }
  res_barrier();
}

// Stage buffers as in the stage launches: Y -> A -> B -> A -> Y, with the
// scalar blocks alongside.
struct ResidentStages {
  double *xin[4], *xout[4];
  int sin_[4], sout[4];
  double coef[4];
};
__device__ __forceinline__ ResidentStages resident_stages(const ResidentView &v, double dt) {
  return ResidentStages{{v.Y, v.A, v.B, v.A}, {v.A, v.B, v.A, v.Y}, {0, 1, 2, 1}, {1, 2, 1, 0},
                        {dt / 4.0, dt / 3.0, dt / 2.0, dt}};
}

// The scalar part of stage st, on one whole wave: scalar_update_wave's
// operations with the sink rates from LDS.  (Each lane forming every site's
// term and summing them as site_sum does measured slower here than the
// shuffles: with N known at run time that is 3N guarded LDS reads a lane.)
__device__ __forceinline__ void resident_scalars(const ResidentView &v, const ResidentStages &g,
                                                 int st, int N, int n, int lane) {
#pragma clang fp contract(off)
  const double *x = g.xin[st];
  double ft = 0.0, fr = 0.0;
  for (int q = lane; q < N; q += 64) {
    const double pop = x[q * n];
    ft = fmad(v.tr[q], pop, ft);
    fr = fmad(v.rc[q], pop, fr);
  }
  ft = wave_sum(ft);
  fr = wave_sum(fr);
  if (lane == 0) {
    const double *xs = v.sc + g.sin_[st] * kScalars;
    double *outs = v.sc + g.sout[st] * kScalars;
    const double xq = xs[0];
    const double y_t = v.sc[0], y_r = v.sc[1], y_q = v.sc[2];
    outs[0] = fmad(g.coef[st], ft, y_t);
    outs[1] = fmad(g.coef[st], fr, y_r);
    outs[2] = fmad(g.coef[st], xq, y_q);
  }
}

// sigma_0 and the sink scalars of the state into history slot `slot`.
__device__ __forceinline__ void resident_record(const InstDesc &d, const ResidentView &v, int N,
                                                int n, int slot, int tid) {
  const int N2 = N * N;
  double *h = d.hist + static_cast<int64_t>(slot) * (N2 + kScalars);
  for (int e = tid; e < N2; e += kResidentThreads) h[e] = v.Y[e * n];
  if (tid < 3) h[N2 + tid] = v.sc[tid];
}

// The state and its scalars back to the workspace.
__device__ __forceinline__ void resident_store(const InstDesc &d, const ResidentView &v, int N,
                                               int n, int tid) {
  const int64_t S = d.stride;
  double *yo = static_cast<double *>(d.y);
  for (int q = tid; q < N * N * n; q += kResidentThreads) yo[elem_index(N, q / n, S, q % n)] = v.Y[q];
  if (tid < 3) d.sc_y[tid] = v.sc[tid];
}

// Runs steps step0 + 1 ... step0 + n_steps of instance blockIdx.x (FP64
// storage, real H, ADO 0 = sigma_0), N and K+1 of each instance read at run
// time (a batch may mix them).  With record_every > 0, the state after every
// step whose index is a multiple of record_every is recorded in history slots
// slot0, slot0 + 1, ... (the host sizes the chunk so that they exist).
__global__ void __launch_bounds__(kResidentThreads)
    stage_resident(const InstDesc *__restrict__ descs, int64_t step0, int64_t n_steps,
                   int64_t record_every, int slot0, double dt) {
  extern __shared__ __align__(16) char res_smem[];
  const InstDesc &d = descs[blockIdx.x];
  const int N = d.N, M = d.M, P = N * (N + 1) / 2;
  const int n = static_cast<int>(d.n_ados);
  const ResidentView v = resident_view(res_smem, resident_lds(N, M, n));
  const int tid = threadIdx.x;
  resident_load(d, v, N, M, n, tid);
  const ResidentStages g = resident_stages(v, dt);
  const int wave = tid >> 6, lane = tid & 63;
  // This thread's item (at most one: the host keeps P * n <= the threads).
  const bool has_item = tid < P * n;
  const int ip = has_item ? tid / n : 0, ii = has_item ? tid % n : 0;
  int slot = slot0;
  int64_t to_rec = record_every > 0 ? record_every - step0 % record_every : -1;
  for (int64_t s = 0; s < n_steps; ++s) {
    for (int st = 0; st < 4; ++st) {
      // The scalars on the last wave (the element items fill the first
      // waves first).
      if (wave == kResidentThreads / 64 - 1) resident_scalars(v, g, st, N, n, lane);
      const ResidentCtx c{N,    d.KP, n,    g.xin[st], v.Y,  g.xout[st], v.H, v.hg,
                          v.dl, v.cr, v.ci, v.damp,    v.up, v.dn,       v.occ};
      if (has_item) resident_element(c, v.pa[ip], v.pb[ip], ii, g.coef[st]);
      res_barrier();
    }
    // Steps until the next recorded one, counted down (no 64-bit remainder
    // per step).
    if (--to_rec == 0) {
      to_rec = record_every;
      resident_record(d, v, N, n, slot++, tid);
    }
  }
  resident_store(d, v, N, n, tid);
}

// ---------------------------------------------------------------------------
// Compile-time N and K+1.  LDS holds the state Y and the stage buffers A and
// B as [n][N][N] complex entries, (re, im) double pairs, with the lower
// triangle stored as the conjugate of the upper one and the imaginary part
// of the diagonal zero, each ADO's matrix padded to an odd number of 16-byte
// entries (consecutive ADOs start in different banks).  Then the scalar
// blocks of Y, A and B.
//
// Thread t of THREADS takes packed element (a, b), p = t / W, of the ADOs j,
// j + W, ..., j + (R - 1) W (j = t mod W, W = ceil(n / R)); four items per
// thread run on 512 threads, so that each has the registers for them.  Row a and column b of a
// matrix sit at compile-time offsets from one base address each, so the
// commutator's operands are 16-byte loads with immediate offsets; the row of
// H, the column of H and each item's neighbour offsets, coupling factors and
// damping are read once per launch into registers.  A stage is then only
// LDS loads and the element's fused multiply-adds, in tile_finish's order;
// the stored conjugate is the exact negation that tile_finish applies to an
// imaginary part below the diagonal, so the results equal the stage
// launches' bitwise.
// ---------------------------------------------------------------------------

// Bytes of one ADO's matrix in the compile-time kernel's LDS.
__host__ __device__ constexpr int fixed_ado_bytes(int N) {
  return (N * N + (N % 2 == 0 ? 1 : 0)) * 16;
}
// The three buffers of n ADOs, the scalars of each, and the (trap,
// recombination) rate pair of each site.
__host__ __device__ inline int fixed_lds_bytes(int N, int n) {
  return 3 * n * fixed_ado_bytes(N) + 3 * kScalars * 8 + N * 16;
}

// Threads of one element in the compile-time kernel, whose P elements each
// take W items per pass on `threads` threads: W rounded up to a multiple of
// 16 where that leaves the last wave without items, else W.  An LDS access
// of 16 bytes per lane serves 16 lanes at a time; lanes of one element read
// one entry of consecutive ADOs, whose 16-byte offsets (an odd count apart)
// fall in distinct banks, so a group of 16 lanes that holds one element only
// has no bank conflict there, where a group that spans two elements mostly
// has.  The last wave also sums the sink populations of every stage; items
// there would add that chain to the stage's longest wave.
__host__ __device__ constexpr int fixed_lanes(int P, int W, int threads) {
  return P * ((W + 15) / 16 * 16) <= threads - 64 ? (W + 15) / 16 * 16 : W;
}

struct Cplx {
  double re, im;
};
__device__ __forceinline__ Cplx lds_c(const char *base, uint32_t off) {
  return *reinterpret_cast<const Cplx *>(base + off);
}
__device__ __forceinline__ void lds_put(char *base, uint32_t off, double re, double im) {
  *reinterpret_cast<Cplx *>(base + off) = Cplx{re, im};
}

// One item's launch-invariant operands (LDS byte offsets within a buffer).
// A missing neighbour points at the item's own entry, weighted by zero.
template <int KP>
struct FixedItem {
  uint32_t own;                 // entry (a, b) of the item's ADO
  uint32_t row, col;            // entry (a, 0) and entry (0, b) of the ADO
  double dec;                   // damping of the element
  uint32_t ua[KP], ub[KP];      // entry (a, b) of the deeper neighbours
  uint32_t da[KP], db[KP];      // entry (a, b) of the shallower neighbours
  double fa[KP], fb[KP];        // 1 where the deeper neighbour exists, else 0
  double car[KP], cai[KP], cbr[KP], cbi[KP];  // n_m c_m of the modes of sites a and b
};

template <int N, int KP, int R, int THREADS>
__global__ void __launch_bounds__(THREADS)
    stage_resident_fixed(const InstDesc *__restrict__ descs, int64_t step0, int64_t n_steps,
                         int64_t record_every, int slot0, double dt) {
#pragma clang fp contract(off)
  static_assert(N >= 1 && N <= 8, "site_sum covers up to 8 sites");
  constexpr int N2 = N * N, P = N * (N + 1) / 2, M = N * KP;
  constexpr uint32_t SD = fixed_ado_bytes(N);
  extern __shared__ __align__(16) char res_smem[];
  const InstDesc &d = descs[blockIdx.x];
  const int n = static_cast<int>(d.n_ados);
  const int64_t S = d.stride;
  const ParamOffsets o = param_offsets(N, M);
  const double *const prm = d.params;
  char *const buf0 = res_smem;
  char *const buf1 = res_smem + n * SD;
  char *const buf2 = res_smem + 2 * n * SD;
  double *const sc = reinterpret_cast<double *>(res_smem + 3 * n * SD);  // [Y, A, B][kScalars]
  // (trap, recombination) rates of each site, read by the scalar wave every
  // stage (from LDS, so that no register holds them across the steps).
  char *const rates = res_smem + 3 * n * SD + 3 * kScalars * 8;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;

  // The state into buffer 0, as full matrices; the stage buffers zeroed.
  const double *yg = static_cast<const double *>(d.y);
  for (int q = tid; q < P * n; q += THREADS) {
    const int pp = q / n, i = q % n;
    const int a = elem_a(N, pp), b = elem_b(N, pp);
    char *X = buf0 + i * SD;
    if (a == b) {
      lds_put(X, (a * N + a) * 16, yg[a * S + i], 0.0);
    } else {
      const int e = N + 2 * (pp - N);
      const double re = yg[e * S + 2 * i], im = yg[e * S + 2 * i + 1];
      lds_put(X, (a * N + b) * 16, re, im);
      lds_put(X, (b * N + a) * 16, re, -im);
    }
  }
  for (int q = tid; q < 2 * n * static_cast<int>(SD / 8); q += THREADS)
    reinterpret_cast<double *>(buf1)[q] = 0.0;
  for (int q = tid; q < 3 * kScalars; q += THREADS)
    sc[q] = q < kScalars ? d.sc_y[q] : 0.0;
  if (tid < N) lds_put(rates, tid * 16, prm[o.trap + tid], prm[o.rec + tid]);

  // This thread's element and items: items j, j + W, ... of element p.
  const int W = (n + R - 1) / R;
  const int L = fixed_lanes(P, W, THREADS);
  const bool active = tid < P * L && tid % L < W;
  const int p = active ? tid / L : 0;
  const int j = active ? tid - p * L : 0;
  const int a = elem_a(N, p), b = elem_b(N, p);
  const bool offd = a != b;
  double hak[N], hkb[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    hak[k] = prm[o.h_re + a * N + k];
    hkb[k] = prm[o.h_re + k * N + b];
  }
  const uint32_t e_own = static_cast<uint32_t>(a * N + b) * 16u;
  const uint32_t e_conj = static_cast<uint32_t>(b * N + a) * 16u;
  FixedItem<KP> it[R];
  bool valid[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = j + r * W;
    valid[r] = active && i < n;
    const int ii = valid[r] ? i : 0;
    FixedItem<KP> &u = it[r];
    const uint32_t base = static_cast<uint32_t>(ii) * SD;
    u.own = base + e_own;
    u.row = base + static_cast<uint32_t>(a * N) * 16u;
    u.col = base + static_cast<uint32_t>(b) * 16u;
    double damp = 0.0;
    for (int m = 0; m < M; ++m)
      damp = fmad(static_cast<double>(d.occ[m * S + ii]), prm[o.nu + m], damp);
    double dec = damp + prm[o.half_gamma + a] + prm[o.half_gamma + b];
    if (offd) dec += prm[o.delta + a] + prm[o.delta + b];
    u.dec = dec;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int ma = a * KP + k, mb = b * KP + k;
      const int ja = d.up[ma * S + ii], jb = d.up[mb * S + ii];
      u.ua[k] = static_cast<uint32_t>(ja >= 0 ? ja : ii) * SD + e_own;
      u.ub[k] = static_cast<uint32_t>(jb >= 0 ? jb : ii) * SD + e_own;
      u.fa[k] = ja >= 0 ? 1.0 : 0.0;
      u.fb[k] = jb >= 0 ? 1.0 : 0.0;
      const int za = d.down[ma * S + ii], zb = d.down[mb * S + ii];
      u.da[k] = static_cast<uint32_t>(za >= 0 ? za : ii) * SD + e_own;
      u.db[k] = static_cast<uint32_t>(zb >= 0 ? zb : ii) * SD + e_own;
      const double na = static_cast<double>(d.occ[ma * S + ii]);
      const double nb = static_cast<double>(d.occ[mb * S + ii]);
      u.car[k] = na * prm[o.c_re + ma];
      u.cai[k] = na * prm[o.c_im + ma];
      u.cbr[k] = nb * prm[o.c_re + mb];
      u.cbi[k] = nb * prm[o.c_im + mb];
    }
  }
  res_barrier();

  // Stage buffers as in the stage launches: Y -> A -> B -> A -> Y.
  const double coefs[4] = {dt / 4.0, dt / 3.0, dt / 2.0, dt};
  int slot = slot0;
  int64_t to_rec = record_every > 0 ? record_every - step0 % record_every : -1;
  for (int64_t s = 0; s < n_steps; ++s) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const char *const xb = st == 0 ? buf0 : (st == 2 ? buf2 : buf1);
      char *const ob = st == 3 ? buf0 : (st == 1 ? buf2 : buf1);
      const int sin_ = st == 0 ? 0 : (st == 2 ? 2 : 1);
      const int sout = st == 3 ? 0 : (st == 1 ? 2 : 1);
      const double coef = coefs[st];
      if (wave == THREADS / 64 - 1) {
        // The scalar part: scalar_update_wave's operations, every site's
        // flux term in each lane (broadcast LDS reads) and lane 0's sum.
        double vt[N], vr[N];
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const double pop = lds_c(xb, static_cast<uint32_t>(a * N + a) * 16u).re;
          const Cplx rate = lds_c(rates, a * 16);
          vt[a] = fmad(rate.re, pop, 0.0);
          vr[a] = fmad(rate.im, pop, 0.0);
        }
        const double ft = site_sum(N, [&](int a) { return vt[a]; });
        const double fr = site_sum(N, [&](int a) { return vr[a]; });
        if (lane == 0) {
          const double xq = sc[sin_ * kScalars];
          const double y_t = sc[0], y_r = sc[1], y_q = sc[2];
          sc[sout * kScalars + 0] = fmad(coef, ft, y_t);
          sc[sout * kScalars + 1] = fmad(coef, fr, y_r);
          sc[sout * kScalars + 2] = fmad(coef, xq, y_q);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!valid[r]) continue;
        const FixedItem<KP> &u = it[r];
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const Cplx xkb = lds_c(xb, u.col + k * N * 16);  // X_kb
          const Cplx xak = lds_c(xb, u.row + k * 16);      // X_ak
          sr = fmad(-xak.re, hkb[k], fmad(hak[k], xkb.re, sr));
          si = fmad(-xak.im, hkb[k], fmad(hak[k], xkb.im, si));
        }
        double ar = si, ai = -sr;
        const Cplx x = lds_c(xb, u.own);
        ar = fmad(-u.dec, x.re, ar);
        ai = fmad(-u.dec, x.im, ai);
#pragma unroll
        for (int k = 0; k < KP; ++k) {
          if (offd) {
            const Cplx ya = lds_c(xb, u.ua[k]), yb = lds_c(xb, u.ub[k]);
            ar = fmad(-u.fa[k], ya.im, fmad(u.fb[k], yb.im, ar));
            ai = fmad(-u.fb[k], yb.re, fmad(u.fa[k], ya.re, ai));
          }
          const Cplx za = lds_c(xb, u.da[k]), zb = lds_c(xb, u.db[k]);
          // On the diagonal the stored imaginary parts are zero.
          ar = fmad(-u.car[k], za.im, fmad(-u.cai[k], za.re, ar));
          ai = fmad(-u.cai[k], za.im, fmad(u.car[k], za.re, ai));
          ar = fmad(-u.cbi[k], zb.re, fmad(u.cbr[k], zb.im, ar));
          ai = fmad(-u.cbi[k], zb.im, fmad(-u.cbr[k], zb.re, ai));
        }
        const Cplx y = lds_c(buf0, u.own);
        const double nr = fmad(coef, ar, y.re);
        if (offd) {
          const double ni = fmad(coef, ai, y.im);
          lds_put(ob, u.own, nr, ni);
          lds_put(ob, u.own - e_own + e_conj, nr, -ni);
        } else {
          lds_put(ob, u.own, nr, 0.0);
        }
      }
      res_barrier();
    }
    // Steps until the next recorded one, counted down (no 64-bit remainder
    // per step).
    if (--to_rec == 0) {
      to_rec = record_every;
      // sigma_0 (packed) and the sink scalars into the history ring.
      double *h = d.hist + static_cast<int64_t>(slot) * (N2 + kScalars);
      for (int e = tid; e < N2; e += THREADS) {
        double v;
        if (e < N) {
          v = lds_c(buf0, static_cast<uint32_t>(e * N + e) * 16u).re;
        } else {
          const int pp = N + (e - N) / 2;
          const Cplx c = lds_c(buf0, static_cast<uint32_t>(elem_a(N, pp) * N + elem_b(N, pp)) * 16u);
          v = (e - N) % 2 == 0 ? c.re : c.im;
        }
        h[e] = v;
      }
      if (tid < 3) h[N2 + tid] = sc[tid];
      ++slot;
    }
  }
  // The state and its scalars back to the workspace.
  double *yo = static_cast<double *>(d.y);
  for (int q = tid; q < N2 * n; q += THREADS) {
    const int e = q / n, i = q % n;
    const char *X = buf0 + i * SD;
    double v;
    if (e < N) {
      v = lds_c(X, static_cast<uint32_t>(e * N + e) * 16u).re;
    } else {
      const int pp = N + (e - N) / 2;
      const Cplx c = lds_c(X, static_cast<uint32_t>(elem_a(N, pp) * N + elem_b(N, pp)) * 16u);
      v = (e - N) % 2 == 0 ? c.re : c.im;
    }
    yo[elem_index(N, e, S, i)] = v;
  }
  if (tid < 3) d.sc_y[tid] = sc[tid];
}

}  // namespace
}  // namespace heom
