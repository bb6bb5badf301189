/*
 * flb.h — C ABI of libflb: the fluctuating D2Q9 lattice-Boltzmann step in the
 * velocity-dependent f-norm moment basis on AMD MI355X (gfx950).
 *
 * Method: Kaehler & Wagner, "A fluctuating lattice-Boltzmann method with
 * improved Galilean invariance".
 *   - update: Sec. II, eq. (1) (stream) and eq. (6) (collision in moment
 *     space, Lambda^{ab} = -delta^{ab}/tau^a, unit Gaussian N per mode);
 *   - noise amplitude: eq. (20), xi^a = sqrt(mu rho (2 tau^a - 1)) / tau^a,
 *     with the noise strength mu = kT / theta = 3 kT (the paper's unit-mass
 *     Poisson gas is mu = 1);
 *   - moment basis: Sec. IV, Gram-Schmidt of the Hermite rows of eq. (A3)
 *     under sum_i a_i f_i^0(1,u) b_i at the local velocity (eqs. (27)-(32)),
 *     or the fixed Hermite basis of App. A, or the basis at the nearest point
 *     of the 51 x 51 velocity grid of Sec. IV (table variant);
 *   - observables: correlators <df_i df_j> (eq. (16)) and moment correlators
 *     (eq. (23)) in the f-norm at (rho0, u0) (Sec. IV, after eq. (34)) and in
 *     the Hermite norm; structure factors, eqs. (24)-(26).
 *
 * Conventions (all entry points):
 *   - Return 0 (FLB_OK) or a negative FLB_E_* code; flb_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - Lattices are periodic nx x ny, velocities ordered as the columns of
 *     eq. (A3): (0,0),(1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1).
 *   - Host arrays of populations or moments are FP64, structure of arrays
 *     [9][ny][nx] (index a*nx*ny + y*nx + x), unshifted f, whatever the
 *     storage precision.  Per-site fields are [ny][nx].  Callers own every
 *     host buffer; the library owns handles and, except with *_create_on,
 *     the device memory behind them.
 *   - Work is enqueued on the stream given at creation (a hipStream_t; NULL
 *     means a library-created non-blocking stream).  step() only enqueues;
 *     read_*, sync and checkpoint synchronise the stream and report device
 *     errors found so far.  Handles are not thread-safe; the server is.
 */
#ifndef FLB_H
#define FLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FLB_OK = 0,
  FLB_E_ARG = -1,              /* invalid argument (sizes, tau <= 1/2, kT < 0, ...) */
  FLB_E_OOM = -2,              /* device or host allocation failed                 */
  FLB_E_HIP = -3,              /* HIP runtime error                                */
  FLB_E_INVALID_VELOCITY = -4, /* some f_i^0(1,u) <= 0: no f-norm basis (Fig. 11)  */
  FLB_E_NONFINITE = -5,        /* density <= 0 or a non-finite population          */
  FLB_E_ADMISSION = -6,        /* server: request can never fit / queue closed     */
  FLB_E_STATE = -7             /* call not valid in the handle's current state     */
};

typedef enum { FLB_FP64 = 0, FLB_FP32_SHIFTED = 1 } flb_precision;
typedef enum {
  FLB_BASIS_FNORM_LOCAL = 0, /* Sec. IV, exact local f-norm basis          */
  FLB_BASIS_HERMITE = 1,     /* App. A, Hermite norm (velocity independent) */
  FLB_BASIS_FNORM_LUT = 2    /* Sec. IV, basis at the nearest grid velocity */
} flb_basis;
typedef enum { FLB_INIT_EQUILIBRIUM = 0, FLB_INIT_THERMAL = 1, FLB_INIT_FIELDS = 2 } flb_init;
typedef enum { FLB_AT_LOCAL = 0, FLB_AT_U0 = 1, FLB_AT_HERMITE = 2 } flb_moment_basis;
typedef enum {
  FLB_SK_RHO = 0, FLB_SK_JX = 1, FLB_SK_JY = 2, FLB_SK_JXJY_RE = 3, FLB_SK_JXJY_IM = 4
} flb_sk_field;

/* Parameters of one lattice. */
typedef struct {
  int32_t nx, ny;       /* periodic sides, each >= 3                              */
  double rho0;          /* reference density (> 0); storage keeps f - f^0(rho0,u0) */
  double ux0, uy0;      /* background velocity (inside the validity region)       */
  double kT;            /* noise temperature (>= 0); mu = 3 kT                    */
  double tau[6];        /* relaxation times of modes 3..8 (Pi_xx-yy, Pi_xy,
                           Pi_xx+yy, q_x, q_y, eps), each > 1/2.  When all six
                           are equal the f-norm collision takes a shorter form
                           (L M~ / tau = d / tau: no triangular solve), equal to
                           the general one up to rounding                       */
  uint64_t seed;        /* Philox key: noise is keyed by (seed, step, site)       */
  int32_t precision;    /* flb_precision.  FP32_SHIFTED stores f - f^0(rho0, u0) in
                           FP32 and collides in FP32 up to |u0| = 0.25, above it in
                           FP64 (with FP32 Gaussians); FP64 does everything in FP64 */
  int32_t basis;        /* flb_basis                                              */
  int32_t init;         /* flb_init: EQUILIBRIUM f^0(rho0,u0); THERMAL adds ideal-
                           gas fluctuations sqrt(mu f^0) N; FIELDS waits for
                           flb_lattice_set_fields                                 */
  int32_t sample_every; /* correlator sample every n steps (0: off)               */
  int32_t sk_every;     /* structure-factor sample every n steps (0: off)         */
  int32_t block_steps;  /* samples per time block for standard errors (0: none)   */
} flb_params;

/* Correlators of df = f - f^0(rho0, u0) over all (site, sample) pairs. */
typedef struct {
  uint64_t nsamples;          /* site-samples                                     */
  uint64_t nblocks;           /* closed time blocks behind the standard errors    */
  double mean_df[9];          /* <f_i> - f_i^0(rho0, u0)                          */
  double cov_f[81];           /* <df_i df_j>, centred on the sample mean          */
  double cov_m_fnorm_u0[81];  /* m~(u0) C m~(u0)^T, f-norm at (rho0,u0), eq. (23) */
  double cov_m_hermite[81];   /* m C m^T, Hermite rows of eq. (A3)                */
  double se_cov_f[81];        /* standard errors from the time blocks (NaN if < 2)*/
  double se_cov_m[81];        /* same for cov_m_fnorm_u0                          */
  double se_cov_m_hermite[81];  /* same for cov_m_hermite                         */
} flb_cov;

typedef struct flb_lattice flb_lattice;

/* Creates a periodic lattice (Sec. III set-up) and initialises the
 * populations per p->init: f^0(rho0, u0) of eq. (A1), optionally plus
 * ideal-gas fluctuations with the covariance of eq. (16) scaled by mu.
 * hip_stream: a hipStream_t or NULL.  *out receives a library-owned handle.
 * Errors: FLB_E_ARG (sizes, tau, kT), FLB_E_INVALID_VELOCITY (u0 outside the
 * region of Fig. 11), FLB_E_OOM, FLB_E_HIP; *out is NULL then. */
int flb_lattice_create(const flb_params* p, void* hip_stream, flb_lattice** out);

/* Device bytes a lattice with these parameters needs (for create_on). */
size_t flb_lattice_bytes(const flb_params* p);

/* As create, but all device arrays are carved from the caller's buffer
 * dev_buf of `bytes` >= flb_lattice_bytes(p) (e.g. a torch tensor); the
 * caller keeps ownership and must outlive the handle. */
int flb_lattice_create_on(const flb_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                          flb_lattice** out);

/* f = f^0(rho(x), u(x)) per site (eq. (A1)); three host arrays [ny][nx]
 * (read only, caller-owned).  Synchronous.  FLB_E_ARG on NULL. */
int flb_lattice_set_fields(flb_lattice* L, const double* rho, const double* ux, const double* uy);

/* Replace the populations (host [9][ny][nx], unshifted FP64, caller-owned)
 * and set the lattice time t (the noise of step t is keyed by t). */
int flb_lattice_set_populations(flb_lattice* L, const double* f, uint64_t t);

/* Enqueue nsteps updates of eq. (1): collision in the basis p->basis (eq.
 * (6) with the f-norm of eqs. (27)-(32), the Hermite norm of App. A or the
 * grid-velocity basis of Sec. IV), FDT noise of eq. (20), streaming; and,
 * when due, correlator samples (eqs. (16), (23)) and structure-factor
 * samples (eqs. (24)-(26)) of the pre-collision state.  Asynchronous on the
 * handle's stream; device errors surface at the next sync/read. */
int flb_lattice_step(flb_lattice* L, uint64_t nsteps);

/* Graph chunk length: with steps > 0 (rounded up to an even number K),
 * flb_lattice_step replays a captured hipGraph of K steps, with their
 * correlator and structure-factor samples, at every time that is a multiple
 * of K, and launches the rest eagerly; replays are used only when the
 * sampling and structure-factor intervals divide K and never straddle the
 * close of a time block.  Results are bit-identical to eager launches.  0
 * (the default) launches every step eagerly.  FLB_E_ARG for steps outside
 * 0..65536.  For small lattices, whose steps are bound by the launch rate. */
int flb_lattice_set_graph_chunk(flb_lattice* L, int32_t steps);

/* Wait for the stream; returns the first device error (FLB_E_INVALID_VELOCITY
 * or FLB_E_NONFINITE) raised since creation, with flb_lattice_error_step()
 * naming the step. */
int flb_lattice_sync(flb_lattice* L);

/* Current populations, unshifted FP64, into caller-owned host [9][ny][nx].
 * Synchronises; returns a pending device error instead of data. */
int flb_lattice_read_populations(flb_lattice* L, double* f);
/* Rows [y0, y0 + nrows) only, into host [9][nrows][nx] (same conventions);
 * for lattices too large to copy out whole.  FLB_E_ARG for rows outside
 * 0..ny. */
int flb_lattice_read_rows(flb_lattice* L, int32_t y0, int32_t nrows, double* f);
/* Moments per site into host [9][ny][nx]: FLB_AT_LOCAL = f-norm at the local
 * velocity (eq. (31): rho, 0, 0, then the non-equilibrium M~^{3..8}),
 * FLB_AT_U0 = f-norm at (rho0, u0) (the measurement basis of Sec. IV, after
 * eq. (34)), FLB_AT_HERMITE = rows of eq. (A3).  Synchronises. */
int flb_lattice_read_moments(flb_lattice* L, int32_t at, double* m);
/* Correlators of all samples since creation / reset_stats (eqs. (16), (23));
 * standard errors from time blocks of p->block_steps samples (pairs of
 * blocks merge when 1024 are full).  Synchronises. */
int flb_lattice_read_covariance(flb_lattice* L, flb_cov* out);
/* <|dA(k)|^2> / (nx ny) (which = RHO, JX, JY) or <dj~_x(k) dj~_y(-k)> / (nx ny)
 * (real, imaginary part), k = 2 pi (kx/nx, ky/ny), host [ky][kx]. */
int flb_lattice_read_structure_factor(flb_lattice* L, int32_t which, double* out);
/* sum_x dA(x) exp(-i k.x) of the current state, which = 0 rho, 1 j~_x, 2 j~_y. */
int flb_lattice_read_fourier_mode(flb_lattice* L, int32_t which, int32_t kx, int32_t ky,
                                  double out[2]);
/* Clears correlator and structure-factor accumulators (e.g. after
 * thermalisation).  Synchronises. */
int flb_lattice_reset_stats(flb_lattice* L);

/* Checkpoint: exact storage bits plus time and parameters; restoring into a
 * lattice with the same parameters continues bit-identically (the noise is
 * keyed by the step).  Statistics are not part of the checkpoint.  restore
 * needs the same nx, ny, precision, rho0 and u0 (the stored values are
 * offsets from f^0(rho0, u0)), else FLB_E_ARG; kT, tau, seed, basis and
 * sampling may differ and take effect from the restored step on. */
size_t flb_lattice_checkpoint_bytes(flb_lattice* L);
int flb_lattice_checkpoint(flb_lattice* L, void* host, size_t bytes);
int flb_lattice_restore(flb_lattice* L, const void* host, size_t bytes);

/* Lattice time (steps taken; the streaming phase is its parity). */
uint64_t flb_lattice_time(flb_lattice* L);
/* Step at which the first device error was raised, -1 when none. */
int64_t flb_lattice_error_step(flb_lattice* L);

/* Device time of the step kernels enqueued since the last reset, measured
 * with HIP events around each launch (enable first; adds two events per
 * launch). */
int flb_lattice_profile(flb_lattice* L, int32_t on);
int flb_lattice_kernel_time(flb_lattice* L, double* ms, uint64_t* launches);

/* Releases the handle and the device memory it owns (NULL is ignored). */
void flb_lattice_destroy(flb_lattice* L);
/* Message of the last failed call on this thread (never NULL). */
const char* flb_last_error(void);

/* Measurement utilities, not part of the method.
 *
 * flb_copy_probe: the device time of one pass of the step kernel's memory
 * traffic with none of its arithmetic, over an nx x ny lattice of the given
 * precision (flb_precision): the same storage layout, tiles, workgroup
 * order and addressing, every site loading its nine values at a streaming
 * phase and storing them back in place.  Averaged over reps (1..1000) pairs
 * of an even and an odd pass after three unmeasured pairs.  18 values per
 * site over that time is the practical bandwidth ceiling of the step's
 * access pattern.  FLB_E_ARG for sizes flb_lattice_create rejects.
 *
 * flb_stream_copy_probe: the device time of one copy of `bytes` (a multiple
 * of 16, below 2^40) between two contiguous buffers, 16 bytes per thread,
 * averaged over reps (1..1000) copies after three unmeasured ones: the
 * device's streaming ceiling, independent of any layout.
 *
 * Both allocate and free their buffers on the current device (FLB_E_OOM if
 * that fails) and synchronise the device's null stream. */
int flb_copy_probe(int32_t nx, int32_t ny, int32_t precision, int32_t reps, double* ms_per_pass);
int flb_stream_copy_probe(uint64_t bytes, int32_t reps, double* ms_per_copy);

/* ------------------------------------------------- no device allocation
 * For callers that cannot allocate device memory: code under HIP stream
 * capture, serving loops that own all their memory, harnesses that forbid
 * allocation.  flb_step_noalloc is flb_lattice_step on populations the
 * caller holds: nsteps updates of the lattice p describes, starting at
 * lattice time t0 (the noise of step t is keyed by t, the streaming phase is
 * t's parity), with the correlator sums of every sampled step.
 *   p        sizes, reference state, kT, tau, seed, precision, basis and
 *            sample_every as for flb_lattice_create; p->init and
 *            p->block_steps are ignored; p->sk_every must be 0 (FLB_E_ARG).
 *   pop      device buffer of flb_population_bytes(p) bytes holding the
 *            populations in the library's storage layout at time t0 (e.g.
 *            copied from flb_lattice_population_buffer of a lattice at that
 *            time); updated in place.  Caller-owned.
 *   sums     device array of 54 doubles (caller-owned; may be NULL when
 *            p->sample_every == 0): overwritten with the sums over the
 *            call's sampled (site, step) pairs of df_i (9 values) and of
 *            df_i df_j for i <= j (45, row-major), df = f - f^0(rho0, u0).
 *   status   device int32 (caller-owned, may be NULL): set to FLB_OK,
 *            FLB_E_INVALID_VELOCITY or FLB_E_NONFINITE when the work ends.
 *   hip_stream  the stream the work is enqueued on (NULL: the null stream).
 * Asynchronous: returns once the work is enqueued (FLB_E_ARG / FLB_E_HIP on
 * bad arguments or launch failures).  Allocates nothing: the descriptor,
 * clock, error flags and per-tile partials live in a file-scope device
 * array of the library (about 14 MiB per device, held until the process
 * ends), which limits sampled lattices to FLB_NOALLOC_MAX_TILES tiles of
 * 256 sites (8.4 million sites); unsampled lattices have no such limit.
 * Every call on a device uses that device's one array, so calls that
 * overlap on one GPU (other streams, other threads) race; each call clears
 * what it uses first. */
#define FLB_NOALLOC_MAX_TILES 32768
int flb_step_noalloc(const flb_params* p, void* pop, uint64_t t0, uint64_t nsteps, double* sums,
                     int32_t* status, void* hip_stream);
/* Bytes of a lattice's population storage (0 for invalid parameters). */
size_t flb_population_bytes(const flb_params* p);
/* The device address and size of a lattice's population storage and its
 * time (the storage's phase): read-only access for copying a state into a
 * caller's buffer.  Synchronises the lattice's stream. */
int flb_lattice_population_buffer(flb_lattice* L, void** dev, size_t* bytes, uint64_t* t);

/* ------------------------------------------------------------- ensembles
 * n replicas of one lattice shape (same nx, ny, precision, basis), each with
 * its own rho0, u0, kT, tau, seed and sampling, advanced by one batched
 * kernel launch per step (two when some FP32 replicas have |u0| > 0.25 and
 * need the FP64 collision: those form their own launch); chunks of steps are
 * replayed from a captured hipGraph.  Replica results are bit-identical to
 * running each alone. */
typedef struct flb_ensemble flb_ensemble;
int flb_ensemble_create(const flb_params* per_replica, int32_t n, void* hip_stream,
                        flb_ensemble** out);
/* Graph chunk length (steps per captured graph), 0 = launch eagerly. */
int flb_ensemble_set_graph_chunk(flb_ensemble* E, int32_t steps);
int flb_ensemble_step(flb_ensemble* E, uint64_t nsteps);
int flb_ensemble_sync(flb_ensemble* E);
int flb_ensemble_read_populations(flb_ensemble* E, int32_t i, double* f);
int flb_ensemble_read_covariance(flb_ensemble* E, int32_t i, flb_cov* out);
/* Restart the correlator sums of every replica (as flb_lattice_reset_stats). */
int flb_ensemble_reset_stats(flb_ensemble* E);
uint64_t flb_ensemble_time(flb_ensemble* E);
/* Device time of the step launches (graph replays count one launch per step). */
int flb_ensemble_profile(flb_ensemble* E, int32_t on);
int flb_ensemble_kernel_time(flb_ensemble* E, double* ms, uint64_t* launches);
void flb_ensemble_destroy(flb_ensemble* E);

/* ------------------------------------------------------------ launch shape
 * The batched step works on tiles of 256 sites, four 64-lane wavefronts:
 * 256 x 1 (the four along one lattice row) on lattices at least 256 sites
 * wide, 64 x 4 (one per tile row) on narrower ones.  Its launch shape is a
 * tuning choice that never changes a
 * result: every shape computes bit-identical populations and correlator
 * sums (each tile forms its partial sums in the same order).
 *   tiles_per_block  tiles per workgroup: 1, 2 or 4 (256, 512, 1024 threads)
 *   grid_blocks      0: one workgroup per group of tiles; > 0 (a multiple
 *                    of 8, the XCD count): a persistent grid of that many
 *                    workgroups, each striding over the tile groups
 *   ms_per_step      output of the autotuner: measured device time per step
 *                    (one even and one odd step averaged); ignored on input
 * Steps that sample correlators or structure-factor fields always give each
 * tile group its own workgroup, and they and every step computed in FP64
 * take at most 2 tiles per workgroup (a larger value is lowered to 2).
 * A new lattice or ensemble starts with {1, 0}, or with the shape an earlier
 * autotune in this process chose for the same device, precision, basis and
 * tile count. */
typedef struct {
  int32_t tiles_per_block;
  int32_t grid_blocks;
  double ms_per_step;
} flb_launch_config;

/* Time every candidate shape for `reps` (1..1000) pairs of steps, keep the
 * fastest for all later steps (and for new lattices of the same kind in this
 * process) and write up to `max_results` measurements, fastest first, to
 * `results` (may be NULL when max_results is 0); *n_results (nullable)
 * receives the number of candidates measured.  Timing follows a device
 * warm-up of at least 50 ms and takes each shape's faster of two interleaved
 * rounds.  The trial steps run on a device copy of the populations, which is
 * put back afterwards: the lattice's state, time, statistics and error flags
 * are as before the call.  Synchronises the stream; allocates a temporary
 * device buffer the size of the populations (FLB_E_OOM if that fails).  A
 * captured step graph is dropped and recaptured with the new shape. */
int flb_lattice_autotune(flb_lattice* L, int32_t reps, flb_launch_config* results,
                         int32_t max_results, int32_t* n_results);
int flb_ensemble_autotune(flb_ensemble* E, int32_t reps, flb_launch_config* results,
                          int32_t max_results, int32_t* n_results);
/* Force a shape (FLB_E_ARG for tiles_per_block not in {1, 2, 4} or a
 * negative grid_blocks or one that is not a multiple of 8). */
int flb_lattice_set_launch(flb_lattice* L, const flb_launch_config* c);
int flb_ensemble_set_launch(flb_ensemble* E, const flb_launch_config* c);
int flb_lattice_get_launch(flb_lattice* L, flb_launch_config* c);
int flb_ensemble_get_launch(flb_ensemble* E, flb_launch_config* c);

/* ---------------------------------------------------------- D3Q19 lattices
 * The same step on the D3Q19 velocity set (the paper's construction carried
 * over to three dimensions, Sec. V): rest, six face and twelve edge
 * velocities (opposite pairs adjacent: index 2k-1 <-> 2k), weights 1/3,
 * 1/18, 1/36, equilibrium of the form of eq. (A1); basis rows = Gram-Schmidt
 * under the weights of the polynomials 1; v_x, v_y, v_z; v_x v_y, v_x v_z,
 * v_y v_z, v_x^2 - v_y^2, v_x^2 + v_y^2 - 2 v_z^2, v^2; v_x (v_y^2 + v_z^2),
 * v_y (v_x^2 + v_z^2), v_z (v_x^2 + v_y^2), v_x (v_y^2 - v_z^2),
 * v_y (v_z^2 - v_x^2), v_z (v_x^2 - v_y^2); v^4, (2 v_x^2 - v_y^2 - v_z^2) v^2,
 * (v_y^2 - v_z^2) v^2; f-norm rows = their Gram-Schmidt under f^0(1, u)
 * (eqs. (27)-(30)); fifteen non-conserved modes a = 4..18 with their own
 * tau and the amplitude of eq. (20).  Noise: four Philox4x32-10 blocks per
 * site and step, counter (site, block 0..3, step lo, step hi), key = seed;
 * the top 24 bits of the sixteen words as uniforms (U + 1/2) 2^-24,
 * Box-Muller on consecutive pairs, the first fifteen Gaussians.  Sites are
 * (z ny + y) nx + x; populations cross the boundary unshifted in FP64,
 * [19][nz][ny][nx].  FP32-shifted lattices compute in FP32 at every u0.
 * Lattices only (no ensembles, server or structure factors). */
typedef struct {
  int32_t nx, ny, nz;      /* periodic, >= 3 each, 19 nx ny nz < 2^32             */
  int32_t precision;       /* FLB_FP64 or FLB_FP32_SHIFTED                         */
  int32_t basis;           /* FLB_BASIS_FNORM_LOCAL or FLB_BASIS_HERMITE           */
  int32_t sample_every;    /* correlator sampling interval (0: none)              */
  int32_t block_steps;     /* time-block length for standard errors               */
  int32_t pad_;
  double rho0, ux0, uy0, uz0;
  double kT;               /* mu = 3 kT                                            */
  double tau[15];          /* modes a = 4..18, each > 1/2; all equal: the shorter
                              f-norm form without the triangular solve          */
  uint64_t seed;
} flb3_params;

typedef struct {
  uint64_t nsamples, nblocks;
  double mean_df[19];      /* <f_i> - f_i^0(rho0, u0)                              */
  double cov_f[361];       /* <df_i df_j>, empirical-mean centred                  */
  double se_cov_f[361];    /* time-block standard errors (NaN below two blocks)    */
} flb3_cov;

typedef struct flb3_lattice flb3_lattice;
/* Equilibrium start f = f^0(rho0, u0); FLB_E_ARG / FLB_E_INVALID_VELOCITY /
 * FLB_E_OOM / FLB_E_HIP as for flb_lattice_create. */
int flb3_lattice_create(const flb3_params* p, void* hip_stream, flb3_lattice** out);
int flb3_lattice_set_populations(flb3_lattice* L, const double* f, uint64_t t);
/* Asynchronous; errors of the kernels surface at the next sync or read. */
int flb3_lattice_step(flb3_lattice* L, uint64_t nsteps);
int flb3_lattice_sync(flb3_lattice* L);
int flb3_lattice_read_populations(flb3_lattice* L, double* f);
int flb3_lattice_read_covariance(flb3_lattice* L, flb3_cov* out);
int flb3_lattice_reset_stats(flb3_lattice* L);
uint64_t flb3_lattice_time(flb3_lattice* L);
int64_t flb3_lattice_error_step(flb3_lattice* L);
int flb3_lattice_profile(flb3_lattice* L, int32_t on);
int flb3_lattice_kernel_time(flb3_lattice* L, double* ms, uint64_t* launches);
void flb3_lattice_destroy(flb3_lattice* L);

/* ---------------------------------------------------------------- serving
 * Continuous batching of simulation requests of mixed size, temperature and
 * background velocity.  Requests wait in FIFO order; one is admitted as soon
 * as a slot is free and its device footprint fits the memory budget; all
 * admitted requests advance together, one batched launch per step, in
 * chunks of `chunk_steps`; finished requests leave at chunk boundaries and
 * free their slot and memory for the next.  A request's result equals the
 * result of running it alone (noise keyed by its own seed, step and site;
 * per-request reduction order). */
typedef struct {
  size_t mem_budget_bytes; /* device bytes for admitted lattices                   */
  int32_t max_slots;       /* concurrent requests                                  */
  int32_t chunk_steps;     /* steps between admission points                       */
  int32_t precision;       /* storage of every request (flb_precision)             */
  int32_t basis;           /* basis of every request (flb_basis)                   */
  int32_t threaded;        /* 1: a worker thread drives the GPU; 0: flb_server_pump */
} flb_server_config;

typedef struct {
  flb_params p;            /* p.precision / p.basis are ignored: the config's apply */
  uint64_t nsteps;         /* 1 .. 2^62 - 1 (FLB_E_ARG otherwise)                  */
  uint64_t tag;            /* caller's id, returned with the result                */
} flb_request;

typedef struct {
  uint64_t id, tag;
  int32_t status;          /* FLB_OK or an error code                              */
  int32_t pad_;
  uint64_t nsteps;
  double t_submit, t_admit, t_done;  /* seconds on the server clock              */
  flb_cov cov;
} flb_result;

typedef struct flb_server flb_server;
int flb_server_create(const flb_server_config* cfg, void* hip_stream, flb_server** out);
/* Device bytes a request occupies while admitted to a server with this
 * configuration (the server stores every request in cfg->precision, whatever
 * r->p.precision says, and admission charges exactly this); 0 for invalid
 * parameters or a NULL argument. */
size_t flb_server_request_bytes(const flb_server_config* cfg, const flb_request* r);
int flb_server_submit(flb_server* S, const flb_request* r, uint64_t* id);
/* Non-threaded servers: run up to max_chunks chunks (admit, step, retire). */
int flb_server_pump(flb_server* S, int32_t max_chunks, int32_t* did_work);
/* Completed results, oldest first; *n = number written (<= max). */
int flb_server_poll(flb_server* S, flb_result* out, int32_t max, int32_t* n);
/* Block until every submitted request has completed. */
int flb_server_drain(flb_server* S);
/* Queue lengths and device-busy statistics. */
int flb_server_stats(flb_server* S, int32_t* queued, int32_t* active, uint64_t* completed,
                     double* busy_seconds, double* wall_seconds);
void flb_server_destroy(flb_server* S);

#ifdef __cplusplus
}
#endif
#endif
