/* heom.h -- C-ABI of the MI355X (gfx950) HEOM propagation library, libheom.so.
 *
 * The library propagates the hierarchical equations of motion of
 * Kreisbeck, Kramer, Rodriguez and Hein (arXiv:1012.4382) for an N-site
 * Frenkel exciton system (section "Model", eq. H_ex) whose sites couple
 * linearly to independent Drude-Lorentz phonon baths (eq:gamma), with
 * trapping and recombination sinks treated in the Born-Markov limit
 * (eq:lab2, eq:lab3; hybrid "ME-HEOM" of Appendix A), by classic fourth-order
 * Runge-Kutta (Appendix B).  The hierarchy is eq:labsevena / eq:lab8,
 * truncated at depth N_max = sum_m n_m (text after eq:lab8); its size is
 * C(M + D, D) for M bath modes (Appendix B).
 *
 * Conventions for every entry point:
 *   - All functions except heom_destroy return a status (HEOM_OK or one of the
 *     negative codes below).  On HEOM_E_INVALID nothing has been written.
 *     heom_last_error() returns a thread-local message for the last failure.
 *   - No C++ exception crosses this interface.
 *   - Host arrays are owned by the caller and only read (or, for outputs,
 *     written) during the call; the library keeps copies of what it needs.
 *   - Complex numbers are interleaved (re, im) doubles; matrices are row-major.
 *   - Device workspaces are owned by the caller (any device allocation of at
 *     least the stated size, 256-byte aligned); the library never frees them.
 *     The state of a run lives entirely in its workspace, so a run can be
 *     continued with HEOM_RESUME.  Calls that use one workspace must not
 *     overlap; distinct workspaces and streams may be used concurrently with
 *     one hierarchy handle, which is immutable after it is built.
 *   - Calls that return host data synchronise their stream before returning.
 *   - Units: energies in cm^-1, times in fs, temperatures in K, rates in 1/ps.
 *     Internally hbar = 1 and energies become angular frequencies in rad/fs.
 */
#ifndef HEOM_H
#define HEOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  HEOM_OK = 0,
  HEOM_E_INVALID = -1,     /* an argument failed validation                     */
  HEOM_E_NOMEM = -2,       /* host or device allocation failed                  */
  HEOM_E_DEVICE = -3,      /* a HIP runtime call failed (text in last error)    */
  HEOM_E_NUMERIC = -4,     /* NaN/Inf in the reduced density matrix, or a drift
                              of Tr rho + P_trap + P_rec (conserved exactly)
                              beyond 1e-7 relative (HEOM_DRIFT_TOL overrides) */
  HEOM_E_WORKSPACE = -5,   /* workspace missing, too small or misaligned        */
  HEOM_E_UNSUPPORTED = -6  /* valid request this build cannot serve             */
};

/* Precision of the bulk ADO update.  HEOM_FP32_MIXED stores and updates every
 * sigma_n with n != 0 in FP32; sigma_0 (the reduced density matrix), its
 * update, the sink integrals and the recorded history stay FP64. */
enum { HEOM_FP64 = 0, HEOM_FP32_MIXED = 1 };

/* Flags for heom_propagate / heom_propagate_batch. */
enum {
  HEOM_RESUME = 1,          /* continue from the state held in the workspace   */
  HEOM_GENERIC_KERNEL = 2,  /* diagnostic: use the generic stage kernel even
                               where a specialised one exists                   */
  HEOM_LANE_KERNEL = 4,     /* diagnostic: use the one-lane-per-ADO specialised
                               kernel instead of the LDS-tiled one (N <= 8)     */
  HEOM_NO_GRAPH = 8,        /* diagnostic: launch every stage kernel directly
                               instead of replaying captured graphs of steps    */
  HEOM_NO_AUTOTUNE = 16,    /* use the default launch shape of the LDS-tiled
                               kernels instead of the autotuned one             */
  HEOM_STREAMING_STORES = 32, /* FP64 tile kernels write their output with
                               non-temporal (streaming) stores (other kernels
                               always store plainly)                            */
  HEOM_PLAIN_STORES = 64,   /* tile kernels write their output with plain
                               stores (exclusive with HEOM_STREAMING_STORES;
                               without either, the autotuner's policy, or
                               plain stores where no tuning is done)            */
  HEOM_NO_RESIDENT = 128    /* diagnostic: launch every RK4 stage even where
                               the run fits a resident kernel (all steps of a
                               chunk in one launch, one workgroup per instance,
                               the hierarchy in LDS): FP64, real H, unscaled,
                               and either every instance with the same N <= 8
                               and K+1 <= 2 and at most 2048 packed elements x
                               ADOs (P * ceil(n / 4) <= 512 for P packed
                               elements and n ADOs; with K+1 = 1 also
                               P * ceil(n / 3) <= 768, up to 2304), or N <= 4
                               and at most 1024 of them; results are bitwise
                               the same                                       */
};
/* Flag bits that force tile launch shape s (0 <= s < heom_tile_shape_count())
 * for every tile-kernel group of a call. */
#define HEOM_TILE_SHAPE(s) (((((int)(s)) + 1) & 0xf) << 8)

typedef struct heom_hierarchy heom_hierarchy; /* opaque, library-owned */

/* Physical system (section "Model" and Appendix A of the paper). */
typedef struct {
  int32_t n_sites;                 /* N, 1 <= N <= 64                               */
  const double *hamiltonian_cm;    /* N*N complex, Hermitian (to 1e-12 max|H|), cm^-1;
                                      site energies on the diagonal (eq. H_ex)      */
  const double *lambda_cm;         /* [N] reorganisation energies, >= 0, cm^-1      */
  const double *gamma_inv_fs;      /* [N] bath correlation times 1/gamma, > 0, fs   */
  double temperature_K;            /* > 0                                           */
  int32_t n_matsubara;             /* K >= 0 Matsubara terms per bath               */
  int32_t low_temp_correction;     /* 1: Markovian residual of the Matsubara tail
                                      beyond K on every ADO; 0: none               */
  int32_t theta_form;              /* 0: Drude amplitude lambda*gamma*(cot(gamma/2kT) - i);
                                      1: the paper's high-temperature
                                      2*lambda*kT - i*lambda*gamma                 */
  const double *trap_rate_per_ps;  /* [N] trapping rate to the reaction centre
                                      per site (eq:lab3), or NULL for none         */
  const double *recomb_rate_per_ps;/* [N] recombination rate to the ground state
                                      per site (eq:lab2), or NULL for none         */
} heom_system;

/* Result of heom_efficiency (eq:eta, eq:trappingtime). */
typedef struct {
  double eta;               /* P_trap(t_end): population trapped in the reaction centre */
  double mean_trap_time_fs; /* int_0^t_end t dP_trap(t), eq:trappingtime               */
  double p_recomb;          /* population lost to the ground state by t_end           */
  double p_remaining;       /* Tr sigma_0(t_end): population still on the sites       */
  double t_end_fs;          /* time actually reached                                  */
} heom_eff_result;

/* Builds the hierarchy for `sys` truncated at depth `depth` (>= 0): bath modes
 * and amplitudes from eq:gamma and its Matsubara expansion, the multi-index
 * map of every ADO with |n| <= depth, and the neighbour tables n +- e_m
 * (Appendix B: each matrix is linked to its neighbours).  Host-only work; the
 * tables are copied to a device on first use there: 9 bytes per mode and ADO
 * (ADOs padded to a multiple of 64), plus 4 more where every neighbour lies
 * within 32767 ADOs (a 16-bit copy the stage kernels read instead).
 * Errors: HEOM_E_INVALID (see the field comments; also a Matsubara frequency
 * within 1e-9 relative of gamma, or more than 2^31 - 1 ADOs), HEOM_E_NOMEM.
 * On success *out owns the handle; release it with heom_destroy. */
int heom_build_hierarchy(const heom_system *sys, int32_t depth, heom_hierarchy **out);

/* heom_build_hierarchy for the scaled hierarchy, the form the introduction
 * names as the way to fewer auxiliary matrices (its reference [Zhu 2011]).
 * Every ADO n is held divided by w_n = sqrt(prod_m n_m! |c_m|^n_m), which
 * leaves sigma_0 unchanged and makes the ADOs of one size, so that a single
 * threshold can drop the negligible ones: in eq:lab8 the coupling to n + e_m
 * gains the factor sqrt((n_m + 1)|c_m|) and the coupling to n - e_m has
 * sqrt(n_m / |c_m|) in the place of n_m.  The weights are tabulated per mode
 * and occupation on the host.
 *   filter_tol  0: no filter; > 0: after every RK4 step each ADO n != 0 whose
 *               stored entries (real and imaginary parts) are all below
 *               filter_tol in absolute value is set to zero
 * The propagation entry points accept the handle like any other; its stages
 * run on the LDS-tiled wide kernel (real H, N <= 32, K + 1 <= 4), otherwise
 * HEOM_E_UNSUPPORTED.  rho (sigma_0) and the sinks are those of the unscaled
 * equations; heom_read_state returns the scaled ADOs.  Errors as
 * heom_build_hierarchy; HEOM_E_INVALID also for a negative or non-finite
 * filter_tol or a zero bath amplitude (lambda = 0). */
int heom_build_hierarchy_scaled(const heom_system *sys, int32_t depth, double filter_tol,
                                heom_hierarchy **out);

/* Sizes of a built hierarchy.  Any output pointer may be NULL.
 *   n_ados      number of ADOs, C(M + depth, depth)
 *   n_modes     M = N * (K + 1)
 *   workspace_bytes_fp64 / _fp32   workspace needed by heom_propagate */
int heom_hierarchy_info(const heom_hierarchy *h, int64_t *n_ados, int32_t *n_modes,
                        size_t *workspace_bytes_fp64, size_t *workspace_bytes_fp32);

/* Copies the hierarchy description to host arrays (any may be NULL):
 *   multi [n_ados][M]  multi-index of each ADO in the library's order
 *   up    [n_ados][M]  index of n + e_m, or -1 beyond the truncation
 *   down  [n_ados][M]  index of n - e_m, or -1 where n_m = 0 */
int heom_hierarchy_tables(const heom_hierarchy *h, int32_t *multi, int32_t *up, int32_t *down);

/* Bath modes in mode order m = site * (K + 1) + k (k = 0 is the Drude term):
 * site[m], amplitude c_m = c_re + i c_im (rad/fs^2) and rate nu_m (1/fs) of the
 * correlation function sum_m c_m exp(-nu_m t), and the correction residual
 * delta[N] (rad/fs).  Any pointer may be NULL. */
int heom_hierarchy_modes(const heom_hierarchy *h, int32_t *site, double *c_re, double *c_im,
                         double *nu, double *delta);

/* The largest time step (fs) at which every ADO's damping rate stays inside
 * classic RK4's stability interval on the negative real axis, by the rule
 * dt * max_n (sum_m n_m nu_m) <= 2.5: 2.5 / (depth * max_m nu_m), or +inf
 * at depth 0.  A step above it is not refused (the Hamiltonian and the
 * couplings also bound it, so it is a guide, not a guarantee); the Python
 * binding warns when a call's dt exceeds it.  Appendix B: fixed-step RK4. */
int heom_max_stable_dt(const heom_hierarchy *h, double *dt_fs);

/* Propagates rho0 by n_steps RK4 steps of dt_fs on the current device.
 *   precision      HEOM_FP64 or HEOM_FP32_MIXED
 *   flags          HEOM_RESUME: continue the run held in d_workspace (rho0 is
 *                  then ignored and may be NULL); HEOM_GENERIC_KERNEL,
 *                  HEOM_LANE_KERNEL, HEOM_NO_GRAPH, HEOM_NO_AUTOTUNE,
 *                  HEOM_STREAMING_STORES, HEOM_PLAIN_STORES, HEOM_TILE_SHAPE(s)
 *                  (see the autotuner below)
 *   rho0           [N][N] complex Hermitian initial reduced density matrix;
 *                  every deeper ADO starts at zero (text after eq:lab8)
 *   record_every   >= 1; rho is recorded at step 0 and every record_every steps
 *   d_workspace    device memory of at least workspace_bytes_* for `precision`
 *   hip_stream     hipStream_t to run on, NULL for the default stream
 *   rho_out        host [(n_steps / record_every) + 1][N][N] complex, or NULL
 *   sinks_out      host [3] = {P_trap, P_recomb, Q = int_0^t P_trap dt'} after
 *                  the last step, or NULL
 * Errors: HEOM_E_INVALID, HEOM_E_WORKSPACE, HEOM_E_DEVICE, HEOM_E_NUMERIC
 * (NaN/Inf in a recorded rho, or Tr rho + P_trap + P_rec moved from its value
 * at the call's first record by more than 1e-7 relative, or the value of the
 * environment variable HEOM_DRIFT_TOL; the run stops there). */
int heom_propagate(heom_hierarchy *h, int precision, int flags, const double *rho0, double dt_fs,
                   int64_t n_steps, int64_t record_every, void *d_workspace,
                   size_t workspace_bytes, void *hip_stream, double *rho_out, double *sinks_out);

/* Workspace needed to propagate the n hierarchies hs[] together. */
int heom_batch_workspace_bytes(heom_hierarchy *const *hs, int32_t n, int precision,
                               size_t *bytes);

/* Propagates n independent instances with one kernel launch per RK4 stage
 * (per distinct kernel variant), all with the same dt_fs, n_steps and
 * record_every.  rho0s[i], rho_outs[i] and sinks_outs[i] are as in
 * heom_propagate for instance i (rho_outs / sinks_outs may be NULL, or hold
 * NULL entries).  Each instance's arithmetic does not depend on the others:
 * results equal those of heom_propagate on the instance alone. */
int heom_propagate_batch(heom_hierarchy *const *hs, int32_t n, int precision, int flags,
                         const double *const *rho0s, double dt_fs, int64_t n_steps,
                         int64_t record_every, void *d_workspace, size_t workspace_bytes,
                         void *hip_stream, double *const *rho_outs, double *const *sinks_outs);

/* Device scratch needed by heom_advance_slots for the n hierarchies hs[]
 * (the launch's descriptors and work list). */
int heom_slots_scratch_bytes(heom_hierarchy *const *hs, int32_t n, size_t *bytes);

/* Advances n independent runs by n_steps RK4 steps of dt_fs, each run held in
 * its own workspace, with one kernel launch per RK4 stage (per distinct kernel
 * variant) for all of them.  This lets a caller batch runs that start and
 * finish at different times without moving their state (continuous batching).
 *   d_workspaces[i]     device memory laid out as for heom_propagate on hs[i]
 *                       (at least workspace_bytes_* of heom_hierarchy_info for
 *                       `precision`), workspace_bytes[i] its size; distinct
 *   start[i]            1: initialise run i from rho0s[i] (N*N complex
 *                       Hermitian); 0: continue the run held in its workspace
 *                       (as HEOM_RESUME; rho0s[i] may be NULL)
 *   flags               HEOM_GENERIC_KERNEL, HEOM_LANE_KERNEL, HEOM_NO_GRAPH,
 *                       HEOM_NO_AUTOTUNE, HEOM_STREAMING_STORES,
 *                       HEOM_PLAIN_STORES, HEOM_TILE_SHAPE(s)
 *   d_scratch           at least heom_slots_scratch_bytes(hs, n) bytes, 256-byte
 *                       aligned; its contents are not needed after the call
 *   rho_out[i]          host N*N complex: sigma_0 after the last step, or NULL
 *   sinks_out[i]        host [3] = {P_trap, P_recomb, Q}, or NULL
 * Each run's arithmetic does not depend on the others: its results equal
 * those of heom_propagate on that run alone.  A workspace advanced here can be
 * continued by heom_propagate with HEOM_RESUME and vice versa.
 * Errors as heom_propagate, except HEOM_E_NUMERIC: it means that every slot
 * was advanced by n_steps and rho_out / sinks_out were written for all of
 * them, and that the slots whose outputs hold a NaN or Inf (listed in
 * heom_last_error) are the failed ones; the other slots are valid and may be
 * continued.  After any other error the state of every slot is undefined. */
int heom_advance_slots(heom_hierarchy *const *hs, int32_t n, int precision, int flags,
                       void *const *d_workspaces, const size_t *workspace_bytes,
                       const int32_t *start, const double *const *rho0s, double dt_fs,
                       int64_t n_steps, void *d_scratch, size_t scratch_bytes, void *hip_stream,
                       double *const *rho_out, double *const *sinks_out);

/* heom_advance_slots for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and results without d_scratch.  The
 * launch's descriptors and work list go to a static device array of the
 * library (2 MiB per GPU, held until the process ends); slots that need more
 * (heom_slots_scratch_bytes > 2 MiB, about 2.9 million ADOs in all) are
 * rejected with HEOM_E_WORKSPACE.  The call allocates no device memory and
 * creates no stream, event or graph:
 *   - every hierarchy must already have its neighbour tables on this device,
 *     i.e. have been used here by an allocating call (heom_propagate,
 *     heom_propagate_batch or heom_advance_slots); otherwise
 *     HEOM_E_UNSUPPORTED and nothing runs;
 *   - launch shapes come from the autotuner's entries of this process (or
 *     its cache file), else the defaults; no timing runs are made (results
 *     do not depend on the shape);
 *   - every stage kernel is launched directly on hip_stream.
 * All calls on one GPU share that GPU's static array, whose contents the
 * next call overwrites in full: calls that overlap on one GPU (from several
 * host threads or on several streams) race and must be serialised by the
 * caller. */
int heom_advance_slots_noalloc(heom_hierarchy *const *hs, int32_t n, int precision, int flags,
                               void *const *d_workspaces, const size_t *workspace_bytes,
                               const int32_t *start, const double *const *rho0s, double dt_fs,
                               int64_t n_steps, void *hip_stream, double *const *rho_out,
                               double *const *sinks_out);

/* Energy-transfer efficiency (eq:eta) and mean trapping time (eq:trappingtime)
 * for an excitation starting in rho0.
 *   t_end_fs > 0   propagate to this fixed time (rounded to whole steps)
 *   t_end_fs <= 0  propagate until the population left on the sites drops
 *                  below pop_tol (the paper's t_max criterion, 1e-5 there)
 * Errors as heom_propagate; HEOM_E_NUMERIC also when the criterion is not met
 * within 10^8 steps. */
int heom_efficiency(heom_hierarchy *h, int precision, const double *rho0, double dt_fs,
                    double t_end_fs, double pop_tol, void *d_workspace, size_t workspace_bytes,
                    void *hip_stream, heom_eff_result *out);

/* Copies the full state held in a workspace to the host:
 * state_out [n_ados][N][N] complex (library order, full Hermitian matrices)
 * followed by 3 doubles {P_trap, P_recomb, Q}.  Synchronises hip_stream. */
int heom_read_state(const heom_hierarchy *h, int precision, const void *d_workspace,
                    size_t workspace_bytes, void *hip_stream, double *state_out);

/* A hierarchy split over ranks: the one-GPU part of propagating a hierarchy
 * too large for one GPU on several.  Every ADO is linked to its neighbours
 * n +- e_m (eq:lab8; Appendix B: each matrix is connected to 2N neighbours),
 * and all of them are accessed in every step (Appendix B), so a split
 * hierarchy must exchange, before every RK4 stage, the stage input of the
 * ADOs each rank links to but does not hold: its halo (the communication that
 * the introduction names as what limits CPU clusters).
 *
 * heom_shard_build splits h into n_ranks contiguous ranges of its ADO order
 * (equal sizes rounded to 64-ADO tiles; rank 0 holds sigma_0; at least 64 ADOs
 * per rank).  Each rank becomes an instance of its own whose neighbour tables
 * point at its own ADOs and at halo slots after them.  Host-only work; h is
 * only read and may be destroyed afterwards.  Errors: HEOM_E_INVALID,
 * HEOM_E_NOMEM.  Release the result with heom_shard_destroy (NULL-safe). */
typedef struct heom_shard heom_shard; /* opaque, library-owned */
typedef struct {
  int64_t first_ado;      /* first ADO of the rank's range in h's order          */
  int64_t n_local;        /* ADOs the rank holds                                 */
  int64_t n_halo;         /* ADOs of other ranks it links to (halo ADOs)         */
  int64_t cut_links;      /* links n -> n +- e_m from its ADOs to halo ADOs      */
  int64_t halo_reals;     /* reals of its halo ADOs in full: n_halo * N * N      */
  int64_t halo_reals_min; /* reals it needs and receives per RK4 stage: of each
                             halo ADO only the rows and columns of the sites whose
                             modes link to it (the entries the stage reads)      */
} heom_shard_rank_info;
int heom_shard_build(const heom_hierarchy *h, int32_t n_ranks, heom_shard **out);
int heom_shard_info(const heom_shard *s, int32_t rank, heom_shard_rank_info *out);
/* Workspace for heom_propagate_sharded (every rank's state and halo slots,
 * the halo list).  FP64 only: HEOM_E_UNSUPPORTED for other precisions. */
int heom_shard_workspace_bytes(const heom_shard *s, int precision, size_t *bytes);
/* heom_propagate for a split hierarchy on the current device: before each RK4
 * stage a copy kernel fills every rank's halo slots (halo_reals_min reals per
 * rank) from the owning ranks' stage inputs, standing in for the exchange
 * between GPUs; then one stage launch runs every rank's share.  Arguments, outputs and errors as
 * heom_propagate (precision HEOM_FP64 only); the results equal those of
 * heom_propagate on h bitwise. */
int heom_propagate_sharded(heom_shard *s, int precision, int flags, const double *rho0,
                           double dt_fs, int64_t n_steps, int64_t record_every, void *d_workspace,
                           size_t workspace_bytes, void *hip_stream, double *rho_out,
                           double *sinks_out);
/* heom_read_state for a split hierarchy: the full state in h's order. */
int heom_read_state_sharded(const heom_shard *s, int precision, const void *d_workspace,
                            size_t workspace_bytes, void *hip_stream, double *state_out);
void heom_shard_destroy(heom_shard *s);

/* Launch shapes of the LDS-tiled stage kernels and their autotuner.
 *
 * For real H the stage runs in an LDS-tiled kernel: a workgroup stages a block
 * of consecutive ADOs with the Hamiltonian and their neighbour tables in LDS
 * (the paper's blocking of ADOs per thread block, Appendix B, redone for
 * wave64 and LDS).  Shapes 0-4 are the 64-ADO tile kernel (N <= 12), which
 * differ in the waves per workgroup, the packed elements each wave computes,
 * how many elements have their neighbour gathers in flight together and the
 * register budget.  Shape 5 is the 16-ADO wide kernel (N <= 32 and K + 1 <= 4
 * while its LDS fits 160 KB: all of them except FP64 with N = 32 and
 * K + 1 >= 3; state buffers below 4 GiB).  Every shape computes each element with
 * the same operations, so results do not depend on the shape.  Unless a call
 * passes HEOM_NO_AUTOTUNE (then shape 0, or 5 where 0 is not built) or
 * HEOM_TILE_SHAPE(s), the first call that meets a new key (GPU architecture,
 * precision, N, K + 1, floor(log2(tiles))) - tiles being the 64-ADO blocks of
 * all of the call's instances with that N and K + 1 - times each distinct
 * available shape on its own launch (repeated sequences of RK4 stages 1, 2,
 * 3, 2, which never write the state, so the run is unchanged), then the
 * fastest one again with non-temporal (streaming) output stores where that
 * instance is built (FP64 tile shapes 0-4), and uses and remembers the faster
 * configuration; later calls with that key reuse it.
 * Results do not depend on the store policy either.  If the
 * environment variable HEOM_AUTOTUNE_CACHE names a file, entries are read
 * from it on first use and new ones are appended (one JSON object per line).
 *
 * heom_tile_shape_count: number of shape slots (shapes are 0 .. count-1).
 * heom_tile_shape_info: for N sites and K + 1 modes per site, the ADOs per
 *   workgroup, threads per workgroup, packed elements per wave, load chunk
 *   and minimum waves per SIMD (register budget) of `shape`; any output may
 *   be NULL.  HEOM_E_UNSUPPORTED if the shape is not built for this N.
 * heom_autotune_lookup: the tuned shape for that key on the current device,
 *   or -1 if not tuned yet; us_per_shape [count] (or NULL) receives the
 *   measured microseconds per stage launch of each shape with plain stores,
 *   -1 where a shape was not timed; streaming (or NULL) whether the tuned
 *   configuration uses streaming stores (1, 0, or -1 if not tuned), and
 *   us_streaming (or NULL) the tuned shape's time with them (-1 where that
 *   instance is not built).
 * heom_autotune_clear: forgets every tuned entry of the process (entries in
 *   the cache file are read again on next use). */
int heom_tile_shape_count(void);
int heom_tile_shape_info(int32_t n_sites, int32_t modes_per_site, int precision, int32_t shape,
                         int32_t *ados_per_workgroup, int32_t *threads, int32_t *elems_per_wave,
                         int32_t *chunk, int32_t *min_waves_per_simd);
int heom_autotune_lookup(int32_t n_sites, int32_t modes_per_site, int precision, int64_t n_tiles,
                         int32_t *shape, double *us_per_shape, int32_t *streaming,
                         double *us_streaming);
void heom_autotune_clear(void);

/* Releases a handle and its device tables.  NULL is accepted. */
void heom_destroy(heom_hierarchy *h);

/* Static text for a status code. */
const char *heom_status_string(int status);

/* Thread-local text of the last failure on this thread ("" if none). */
const char *heom_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HEOM_H */
