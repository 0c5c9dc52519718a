/*
 * mlfilm.h -- C ABI of libmlfilm, an MI355X (gfx950) implementation of the
 * N-layer thin-film shallow-water lattice Boltzmann time step of
 * Richter, Malgaretti & Harting, "Modeling of thin liquid films with
 * arbitrary many layers" (arXiv 2409.16659).
 *
 * One step (Sec. III with the pressures and friction of Sec. II), for every
 * lattice node x and layer i = 1..N:
 *   h_i = sum_k f_ki, q_i = h_i U_i = sum_k c_k f_ki         (moments)
 *   z_i = z_{i-1} + h_i, z_0 = 0                              (Sec. II, Fig. 1)
 *   Delta_i = p_i - p_{i+1} = Lambda_i + Pi_i  (Eqs. Laplace_pressure,
 *             disjoining_pressure, wetting_potential); p_i = sum_{j>=i} Delta_j
 *   F_i = -h_i grad p_i + 2 mu_i h_i a_i        (Eq. force; friction from the
 *             boundary conditions Eqs. no_slip, flux, viscous_boundary)
 *   f_ki(x + c_k, t+1) = f_ki - (f_ki - f^eq_ki)/tau + w_k c_k.F_i / c_s^2
 *                                              (Eqs. BGK, equilibrium_distribution)
 * on a periodic D2Q9 lattice (c_s^2 = 1/3, dx = dt = 1).  The gradient and
 * Laplacian, which the paper does not state, are the isotropic 9-point
 * lattice stencils.
 *
 * Conventions for every function:
 *  - Return MLF_OK or a negative mlf_status; no exception crosses the ABI.
 *    mlf_last_error() gives a text for the last failure on a handle.
 *  - Device memory belongs to the caller: the library never allocates or
 *    frees device memory.  The caller sizes the two population buffers and
 *    the scratch buffer with mlf_query_sizes() and keeps them alive until
 *    mlf_destroy().  Host arrays are caller-owned and only read or written
 *    during the call.
 *  - Work is issued on the stream given to mlf_create (a hipStream_t; NULL
 *    is the default stream).  mlf_step is asynchronous except for the guard
 *    polls; every call that returns host data synchronises the stream.
 *  - Fields are [N][ny][nx] row-major (x fastest).  Populations are stored
 *    per direction: the rest plane, then the eight moving planes, each of
 *    ny rows of `pitch` nodes, x fastest; a node holds the N layers'
 *    values of that plane's type next to each other.
 *  - A handle is not thread-safe.
 */
#ifndef MLFILM_H
#define MLFILM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLF_MAX_LAYERS 4
#define MLF_MAX_PAIRS (MLF_MAX_LAYERS * (MLF_MAX_LAYERS + 1) / 2)

typedef enum {
  MLF_OK = 0,
  MLF_EINVAL = -1,        /* bad argument (sizes, pointers, parameters)        */
  MLF_EUNSUPPORTED = -2,  /* valid but not implemented on this path            */
  MLF_EDEVICE = -3,       /* a HIP runtime call failed                          */
  MLF_ENONFINITE = -4,    /* a layer height or flux became NaN/Inf              */
  MLF_ENONPOSITIVE = -5,  /* a layer height became <= 0                         */
  MLF_EUNSTABLE = -6      /* explicit friction would be unstable (see below)    */
} mlf_status;

/* Storage of the populations.  Arithmetic is FP64 for MLF_F64 and FP32
 * otherwise.  All formats store the rest population as a deviation from the
 * rest-state equilibrium h_ref_i (f_0 - h_ref_i), the moving ones as they
 * are; h_ref_i is the per-layer mean of the initial heights.  IEEE half
 * values are scaled by a per-layer power of two near 2^12 / h_ref_i.
 * In the all-16-bit formats a height change per step below half an ulp of
 * the stored deviation is lost (slow dynamics stall); the MIX formats keep
 * the rest population, which carries the height, in FP32 (40 instead of 36
 * bytes per layer-node update), and mlf_set_rounding can round the rest
 * population stochastically instead. */
typedef enum {
  MLF_F64 = 0,
  MLF_F32 = 1,
  MLF_F16 = 2,      /* IEEE half storage of deviations, FP32 arithmetic          */
  MLF_BF16 = 3,     /* bfloat16 storage of deviations, FP32 arithmetic           */
  MLF_F16_MIX = 4,  /* FP32 rest population, IEEE half moving ones, FP32 arith.  */
  MLF_BF16_MIX = 5  /* FP32 rest population, bfloat16 moving ones, FP32 arith.   */
} mlf_precision;

/* Lattice.  D1Q3 (velocities 0, +1, -1; 3-point stencils) is the pseudo-1D
 * form of the scheme: it needs ny == 1 and F64 or F32 storage
 * (EUNSUPPORTED otherwise) and stores three planes (rest, +x, -x).  In
 * exact arithmetic it equals D2Q9 on a film one row high.  D1Q3 films run
 * many steps per kernel launch with the film held on chip: up to 128 nodes
 * in one workgroup; longer ones (any length) in tiles of 32 nodes, one
 * workgroup each, that also hold 48 nodes on either side and run 16 steps
 * per launch.  In a batch each D1Q3 film must fit one workgroup's LDS
 * (5 N nx values of the storage type within 64 KiB, nx <= 1024). */
typedef enum { MLF_D2Q9 = 0, MLF_D1Q3 = 1 } mlf_lattice;

typedef struct mlf_params {
  int32_t n_layers;   /* N, 1..MLF_MAX_LAYERS                                  */
  int32_t nx, ny;     /* periodic grid, >= 1 each (ny == 1: pseudo-1D film)     */
  int32_t precision;  /* mlf_precision                                          */
  double tau;         /* BGK relaxation time (> 0.5); 1 selects the fast path   */
  double hstar;       /* precursor thickness h* > 0, Eq. (wetting_potential)    */
  int32_t exp_a;      /* wetting exponents a > b >= 1 (the paper's n > m)       */
  int32_t exp_b;
  double gamma[MLF_MAX_LAYERS];  /* gamma_{i,i+1}, i = 1..N (gamma_N: layer N / gas) */
  double mu[MLF_MAX_LAYERS];     /* viscosities mu_1..mu_N > 0                   */
  double slip[MLF_MAX_LAYERS];   /* slip lengths beta_i >= 0 (0: no slip)        */
  /* spreading coefficients S_lk packed l-major: l = 0..N-1, k = 1..N-l, i.e.
   * S_01..S_0N, S_11..S_1(N-1), ..., S_(N-1)1 (Eq. spreading_parameters). */
  double spread[MLF_MAX_PAIRS];
  int32_t check_every;   /* guard poll interval in steps; 0: only at the end of mlf_step */
  int32_t allow_unstable;/* nonzero: skip the friction-stiffness check in mlf_init */
  int32_t lattice;       /* mlf_lattice; 0 (zero-initialised) is D2Q9          */
} mlf_params;

typedef struct mlf_handle mlf_handle;

/* Byte sizes of each of the two population buffers and of the scratch
 * buffer for these parameters.  Pure host function.  EINVAL on bad params. */
mlf_status mlf_query_sizes(const mlf_params* p, size_t* pop_bytes, size_t* scratch_bytes);

/* Row pitch (elements) used for the population planes. */
mlf_status mlf_query_pitch(const mlf_params* p, int32_t* pitch);

/* Bind parameters, caller-owned device buffers (pop_a, pop_b of pop_bytes,
 * scratch of scratch_bytes, all 256-byte aligned) and a stream.  Validates
 * the parameters (EINVAL / EUNSUPPORTED) and uploads nothing yet. */
mlf_status mlf_create(const mlf_params* p, void* pop_a, void* pop_b, void* scratch,
                      void* stream, mlf_handle** out);

/* Initial state f = f^eq(h, U) (populations at equilibrium; U = 0 when ux/uy
 * are NULL).  h, ux, uy: host FP64 [N][ny][nx].  The per-layer reference
 * heights h_ref_i become the means of h_i.  Checks h > 0 and finite
 * (ENONPOSITIVE / ENONFINITE) and, unless allow_unstable, that the explicit
 * friction is stable: with each layer at h* or at h_ref the spectral radius
 * of I + K (friction = K q; the per-step amplification of the fluxes) must
 * stay below 1 (without slip: every eigenvalue of -K below 2), else
 * EUNSTABLE.  Resets the step
 * counter.  Synchronises. */
mlf_status mlf_init(mlf_handle* h, const double* hgt, const double* ux, const double* uy);

/* As mlf_init with device FP64 arrays (ux/uy may be NULL). */
mlf_status mlf_init_device(mlf_handle* h, const double* hgt, const double* ux, const double* uy);

/* Advance nsteps >= 0 steps.  Asynchronous, except that every check_every
 * steps (and at the end) the device guard flag is read back: a height that
 * became non-positive or non-finite returns ENONPOSITIVE / ENONFINITE (the
 * state is then undefined; reload a checkpoint). */
mlf_status mlf_step(mlf_handle* h, int64_t nsteps);

/* Heights h_i and velocities U_i = q_i / h_i (moment definition, no
 * half-force shift) in FP64, host arrays [N][ny][nx]; any may be NULL. */
mlf_status mlf_read(mlf_handle* h, double* hgt, double* ux, double* uy);

/* As mlf_read into device FP64 arrays; asynchronous on the stream. */
mlf_status mlf_read_device(mlf_handle* h, double* hgt, double* ux, double* uy);

/* Per-layer mass sum_x h_i in FP64 (device reduction in a fixed order),
 * host array [N].  Synchronises. */
mlf_status mlf_layer_mass(mlf_handle* h, double* mass);

/* Allocation-free form of mlf_layer_mass, for callers that cannot allocate
 * device memory or synchronise (code under HIP graph capture, serving
 * loops).  The same per-layer FP64 sums in the same fixed order (results
 * bit-identical to mlf_layer_mass), but the reduction partials live in a
 * fixed 16 KiB device array inside the library (one per GPU, taken on the
 * first call on each device and held until the process ends; the partial
 * count does not depend on the film size, so every film fits) instead of
 * the handle's scratch buffer, and the result goes to the caller-owned
 * device array mass_dev[N] (FP64, written by a kernel; no memset, no copy).
 * Asynchronous on the handle's stream, no host synchronisation; call with
 * the handle's device current.  Calls that overlap on one GPU (any handle,
 * any stream) share that array and race: order them on one stream or
 * synchronise between them.  Allocates nothing.  EINVAL for NULL pointers
 * or before init; EDEVICE if the array's address cannot be taken or a
 * launch fails. */
mlf_status mlf_layer_mass_static(mlf_handle* h, double* mass_dev);

/* Per-layer minimum height min_x h_i in FP64, host array [N]; the heights
 * are bit-identical to those mlf_read returns (same summation order).
 * Synchronises.  A layer has ruptured once it shows its first hole, i.e.
 * its minimum drops to the precursor scale (Sec. IV.E). */
mlf_status mlf_layer_min(mlf_handle* h, double* hmin);

/* Rupture detection.  Steps in chunks of check_every (>= 1) steps, up to
 * max_steps (>= 0) in total, taking the per-layer minimum after each
 * chunk, and stops after the first chunk at whose end some layer i has
 * min_x h_i <= threshold[i] (host [N]).  *steps_taken: steps run by this
 * call; *layer: the first layer at or below its threshold, -1 if none
 * was.  The time of the event is resolved to check_every steps.  Guard
 * trips return as from mlf_step (with *steps_taken counting the failed
 * chunk).  Synchronises after every chunk.  EINVAL for null pointers,
 * max_steps < 0 or check_every < 1. */
mlf_status mlf_step_until(mlf_handle* h, int64_t max_steps, int32_t check_every, const double* threshold,
                          int64_t* steps_taken, int32_t* layer);

/* Absolute populations f_ki in FP64, host [N][Q][ny][nx] with Q = 9 (D2Q9)
 * or 3 (D1Q3, order rest, +x, -x) (read) or set from such an array (write;
 * keeps h_ref).  Synchronise. */
mlf_status mlf_read_populations(mlf_handle* h, double* f);
mlf_status mlf_write_populations(mlf_handle* h, const double* f);

/* Checkpoint.  mlf_save with blob == NULL stores the needed size in *bytes;
 * otherwise writes the state (parameters digest, step counter, h_ref and
 * the raw population buffer) into blob of *bytes.  mlf_load restores it on a
 * handle with identical parameters (else EINVAL).  Synchronise. */
mlf_status mlf_save(mlf_handle* h, void* blob, size_t* bytes);
mlf_status mlf_load(mlf_handle* h, const void* blob, size_t bytes);

/* D2Q9 films one row high (ny == 1) with F64 or F32 storage run many steps
 * per launch with the film held on chip, with results bit-identical to the
 * step kernel: up to 128 columns in one workgroup; wider rows in tiles of
 * 32 columns, one workgroup each, that also hold 48 columns on either side
 * (what 16 steps can carry across a tile edge) and run 16 steps per launch.
 * Once a graph is captured (mlf_capture) mlf_step replays it with the step
 * kernel instead.
 *
 * Launch shape of the step kernel: block_w threads (64, 128, 192, 256 or 512;
 * 512 is MLF_EINVAL for FP64 films of four layers, whose kernel is compiled
 * for at most 256), one per column of a strip of block_w - 4 columns plus two
 * halo columns on each side, and seg_h rows per workgroup (>= 1).  Results
 * do not depend on the shape.  0 = default.  D1Q3 films keep their fixed
 * kernel shapes (the values are stored and ignored; mlf_autotune returns
 * them unchanged). */
mlf_status mlf_set_launch(mlf_handle* h, int32_t block_w, int32_t seg_h);
mlf_status mlf_get_launch(const mlf_handle* h, int32_t* block_w, int32_t* seg_h);

/* Rows of populations the step kernel keeps in flight while it processes a
 * row: 1 (default; 0 selects it) or 2.  Two are available for D2Q9 films
 * with tau == 1 and storage other than MLF_F64 (FP32 arithmetic): they hide
 * more load latency on HBM-sized films at the cost of registers (fewer waves
 * per SIMD).  Results do not depend on it.  MLF_EINVAL for other values, or
 * for 2 on other films (mlf_last_error says why).  Drops a captured graph.
 * mlf_get_prefetch writes the current value (rows must not be NULL). */
mlf_status mlf_set_prefetch(mlf_handle* h, int32_t rows);
mlf_status mlf_get_prefetch(const mlf_handle* h, int32_t* rows);

/* Rounding of the stored rest population (the population that carries a
 * layer's height change).  MLF_ROUND_NEAREST (default): round to nearest.
 * MLF_ROUND_STOCHASTIC_REST (D2Q9 films with MLF_F16 or MLF_BF16 storage
 * only, else MLF_EINVAL): each node's rest population of each layer is
 * rounded to the representable value below or above it, the upper one with
 * probability equal to its distance from the lower one over their gap, so
 * that height changes below half an ulp accumulate on average instead of
 * being lost.  The draws are 16-bit uniforms, two per counter-based hash
 * of (node, pair of layers, step count): results are reproducible and
 * independent of the launch shape,
 * but differ from round-to-nearest ones.  A film with stochastic rounding
 * cannot be captured into a graph (MLF_EUNSUPPORTED from mlf_capture).
 * Drops a captured graph.  mlf_get_rounding writes the current mode (mode
 * must not be NULL). */
typedef enum { MLF_ROUND_NEAREST = 0, MLF_ROUND_STOCHASTIC_REST = 1 } mlf_rounding;
mlf_status mlf_set_rounding(mlf_handle* h, int32_t mode);
mlf_status mlf_get_rounding(const mlf_handle* h, int32_t* mode);

/* Autotuner: times candidate launch shapes on the current state and keeps
 * the fastest (written to block_w / seg_h if not NULL).  Each candidate is
 * launched `reps` times (>= 1) from the current population buffer into the
 * other one without swapping, so the state and step counter are unchanged;
 * the four fastest are then re-timed twice with 4 x reps launches each and
 * the smallest time wins.  Candidates: block_w in {64, 128, 192, 256, 512}
 * (not 512 for FP64 films of four layers), segment heights from a fixed
 * list plus those that fill whole dispatch rounds of the device, and 1 or 2
 * rows in flight where mlf_set_prefetch allows 2 (the choice is kept; read
 * it with mlf_get_prefetch).  Synchronises. */
mlf_status mlf_autotune(mlf_handle* h, int32_t reps, int32_t* block_w, int32_t* seg_h);

/* Capture `steps` (even, > 0) consecutive step launches into a HIP graph
 * that mlf_step replays whenever at least `steps` steps remain (guard polls
 * then fall on replay boundaries); 0 drops it.  The graph holds the step
 * constants: mlf_init, mlf_init_device, mlf_load, mlf_set_launch and
 * mlf_autotune drop it.  EUNSUPPORTED on the default stream and for D1Q3
 * films (which already run many steps per launch). */
mlf_status mlf_capture(mlf_handle* h, int32_t steps);

/* Steps taken since init; mlf_load restores the count saved with the
 * checkpoint (-1 for NULL). */
int64_t mlf_steps_done(const mlf_handle* h);
/* Text of the last failure on this handle ("" if none; a guard trip names
 * the failing step); valid until the next call on it. */
const char* mlf_last_error(const mlf_handle* h);
/* Free the host handle and its captured graph (not the device buffers,
 * which stay the caller's); EINVAL for NULL. */
mlf_status mlf_destroy(mlf_handle* h);

/* ---- batches of independent films ------------------------------------
 * Many films (the paper's parameter sweeps over wavenumber, tension,
 * contact angle and layer count, Sec. IV) advanced together: every step
 * is ONE kernel launch over a work list of (film, tile) items, largest
 * film first, with each film's constants in a device table; films may
 * differ in size, layer count and every physical parameter but share the
 * precision, tau and the wetting exponents.  Results of each film are
 * bit-identical to stepping it alone with the same launch shape.
 * Conventions as above; device memory is caller-owned. */
typedef struct mlf_batch mlf_batch;

/* Sizes of each of the two population buffers (the films' buffers back to
 * back, 256-byte aligned) and of the scratch buffer.  EINVAL / EUNSUPPORTED
 * as mlf_query_sizes, also for films that do not share precision, tau,
 * exponents and lattice, or n outside 1..4096.  A D1Q3 batch holds films
 * that each fit one workgroup's LDS (as for the resident single-film
 * kernel; else EUNSUPPORTED) and advances them one workgroup per film,
 * many steps per launch; its launch shape is fixed (set_launch values are
 * kept and ignored, autotune returns them). */
mlf_status mlf_batch_query_sizes(const mlf_params* films, int32_t n, size_t* pop_bytes, size_t* scratch_bytes);

/* Bind n films to caller-owned buffers (sizes from mlf_batch_query_sizes,
 * 256-byte aligned) and a stream.  A non-default stream is needed for
 * mlf_batch_capture. */
mlf_status mlf_batch_create(const mlf_params* films, int32_t n, void* pop_a, void* pop_b, void* scratch,
                            void* stream, mlf_batch** out);

/* Initialise film `film` exactly as mlf_init does for one film (same
 * checks and errors).  Every film must be initialised before stepping. */
mlf_status mlf_batch_init(mlf_batch* b, int32_t film, const double* hgt, const double* ux, const double* uy);
/* As mlf_batch_init from device FP64 arrays (as mlf_init_device). */
mlf_status mlf_batch_init_device(mlf_batch* b, int32_t film, const double* hgt, const double* ux, const double* uy);
/* Every film at once from device FP64 heights (U = 0): hgts is a host
 * array of n device pointers, hgts[f] of film f's shape [N][ny][nx].  Same
 * checks as mlf_init for each film, one synchronisation for all. */
mlf_status mlf_batch_init_device_all(mlf_batch* b, const double* const* hgts);
/* As mlf_batch_init_device_all with initial velocities: uxs, uys host
 * arrays of n device pointers to FP64 [N][ny][nx] (both NULL: U = 0, the
 * plain form), f = f^eq(h, U) for every film. */
mlf_status mlf_batch_init_device_all_u(mlf_batch* b, const double* const* hgts, const double* const* uxs,
                                       const double* const* uys);

/* Advance every film by nsteps >= 0 steps: one launch per step, or replays
 * of the captured graph where it fits.  The guard flags of all films are
 * read at the end; a tripped film gives ENONPOSITIVE / ENONFINITE and
 * mlf_batch_failed_film names it. */
mlf_status mlf_batch_step(mlf_batch* b, int64_t nsteps);

/* Capture `steps` (even, > 0) consecutive batch launches into a HIP graph
 * that mlf_batch_step replays; 0 drops the graph.  Changing the launch
 * shape drops it too.  EUNSUPPORTED on the default stream and for D1Q3
 * batches. */
mlf_status mlf_batch_capture(mlf_batch* b, int32_t steps);

/* Read-back and FP64 per-layer mass of one film, as mlf_read and
 * mlf_layer_mass (synchronise). */
mlf_status mlf_batch_read(mlf_batch* b, int32_t film, double* hgt, double* ux, double* uy);
/* As mlf_batch_read into device FP64 arrays; asynchronous on the stream. */
mlf_status mlf_batch_read_device(mlf_batch* b, int32_t film, double* hgt, double* ux, double* uy);
/* Heights of every film into device FP64 arrays outs[f] (host array of n
 * device pointers); asynchronous on the stream. */
mlf_status mlf_batch_read_device_all(mlf_batch* b, double* const* outs);
mlf_status mlf_batch_layer_mass(mlf_batch* b, int32_t film, double* mass);
/* Per-layer minimum height of one film, as mlf_layer_min (synchronises). */
mlf_status mlf_batch_layer_min(mlf_batch* b, int32_t film, double* hmin);
/* Minima of all films from one pass over the batch: host
 * [n][MLF_MAX_LAYERS], +inf past a film's layer count.  Synchronises. */
mlf_status mlf_batch_layer_min_all(mlf_batch* b, double* hmin);
/* Rupture times of all films: the batch steps in chunks of check_every
 * (>= 1) until every film has some layer i with min_x h_i <=
 * threshold[f][i] (host [n][MLF_MAX_LAYERS]) or max_steps have run.
 * t_hit[f] (host [n]): mlf_batch_steps_done at the end of the chunk in
 * which film f first did, -1 if it never did; layer_hit[f]: that layer
 * (-1); *steps_taken: steps run by this call.  Films that have got there
 * keep stepping with the rest.  Synchronises after every chunk. */
mlf_status mlf_batch_step_until(mlf_batch* b, int64_t max_steps, int32_t check_every, const double* threshold,
                                int64_t* t_hit, int32_t* layer_hit, int64_t* steps_taken);

/* Launch shape shared by all films: block_w in {64, 128, 192, 256}, seg_h
 * >= 1 rows (clamped to each film's ny), persistent != 0: as many
 * workgroups as fit the device at once, each taking work items in turn;
 * 0: one workgroup per item.  0 for block_w / seg_h selects 256 / 8.
 * EINVAL if the work list would exceed its scratch area. */
mlf_status mlf_batch_set_launch(mlf_batch* b, int32_t block_w, int32_t seg_h, int32_t persistent);
mlf_status mlf_batch_get_launch(const mlf_batch* b, int32_t* block_w, int32_t* seg_h, int32_t* persistent);

/* Rows of populations in flight in the batch kernel, as mlf_set_prefetch
 * for a single film (2 only for D2Q9 batches with tau == 1 and storage
 * other than MLF_F64; results do not depend on it).  Drops a captured
 * graph.  rows must not be NULL for the getter. */
mlf_status mlf_batch_set_prefetch(mlf_batch* b, int32_t rows);
mlf_status mlf_batch_get_prefetch(const mlf_batch* b, int32_t* rows);

/* Rounding of the stored rest population for every film of the batch, as
 * mlf_set_rounding for a single film (MLF_ROUND_STOCHASTIC_REST only for
 * D2Q9 batches with MLF_F16 or MLF_BF16 storage, else MLF_EINVAL).  The
 * draws use each film's node indices and the batch's step count, so a film
 * stepped in a batch equals the same film stepped alone from the same step
 * count, bit for bit.  A batch with stochastic rounding cannot be captured
 * (MLF_EUNSUPPORTED from mlf_batch_capture).  Drops a captured graph.
 * mode must not be NULL for the getter. */
mlf_status mlf_batch_set_rounding(mlf_batch* b, int32_t mode);
mlf_status mlf_batch_get_rounding(const mlf_batch* b, int32_t* mode);

/* Autotuner over block_w x seg_h x persistent x rows in flight (1, and 2
 * where mlf_batch_set_prefetch allows it), `reps` timed launches each from
 * the current buffer into the other (state unchanged); keeps the fastest
 * (read the depth with mlf_batch_get_prefetch).  Drops a captured graph.
 * Synchronises. */
mlf_status mlf_batch_autotune(mlf_batch* b, int32_t reps, int32_t* block_w, int32_t* seg_h, int32_t* persistent);

/* Steps the batch has taken since it was created (-1 for NULL). */
int64_t mlf_batch_steps_done(const mlf_batch* b);
/* Index of the film whose guard tripped in the last failing step (-1 if
 * none, or for NULL). */
int32_t mlf_batch_failed_film(const mlf_batch* b);
/* Text of the last failure on this batch ("" if none); valid until the
 * next call on it. */
const char* mlf_batch_last_error(const mlf_batch* b);
/* Free the batch's host state and graph (not the device buffers); EINVAL
 * for NULL. */
mlf_status mlf_batch_destroy(mlf_batch* b);

/* Stokes-limit velocities of a height field: U_i = q_i / h_i with the
 * flux q at which the pressure force -h_i grad p_i and the inter-layer
 * friction balance, q = K^-1 diag(h) grad p = -M grad Delta (M the
 * mobility of Eq. thin_film_equation_n, Delta the pressure jumps), the
 * flux of the thin-film equation's Stokes limit (Sec. II.B).  Pressures,
 * stencils and friction as in the step (isotropic 9-point gradient and
 * Laplacian, Eqs. Laplace_pressure and disjoining_pressure; friction from
 * the boundary conditions of Sec. II.A.2 without slip), in FP64.  For a
 * restart f = f^eq(h, U) (mlf_init_device) that starts the scheme on its
 * friction-dominated trajectory instead of from rest.
 *  p       film parameters (n_layers, nx, ny, hstar, exponents, gamma, mu,
 *          spread; precision, tau and lattice are ignored)
 *  hgt     device FP64 [N][ny][nx], h > 0; ux, uy device FP64 [N][ny][nx]
 *          (caller-owned, not aliased with hgt)
 *  stream  hipStream_t (NULL: default); asynchronous.
 * EINVAL for bad parameters or NULL pointers, EUNSUPPORTED for slip
 * lengths != 0, EDEVICE if the launch fails. */
mlf_status mlf_stokes_velocity(const mlf_params* p, const double* hgt, double* ux, double* uy, void* stream);

/* ---- measurement helper ----------------------------------------------
 * Streaming bandwidth probe.  Not a step of the method: one pass of a
 * read, write or copy kernel over `bytes` bytes with 16-byte buffer
 * accesses (the widest access the step kernel uses), to measure the rate a
 * single-pass kernel reaches on a buffer of that size (the practical
 * ceiling of the HBM-bound step) and to provide a kernel of exactly known
 * traffic for scaling memory counters (READ: bytes read; WRITE: bytes
 * written; COPY: both).
 *  mode         mlf_stream_mode
 *  schedule     0: chunked, every workgroup walks one contiguous range;
 *               1: grid-stride, all lanes sweep the buffer together
 *  nontemporal  nonzero: non-temporal cache policy on every access
 *  src, dst     caller-owned device buffers of at least `bytes` bytes; dst
 *               must be writable in every mode (READ may store 4 bytes at
 *               dst to keep its loads alive); src is not read by WRITE
 *  bytes        multiple of 16, 16 <= bytes <= 4 GiB - 16
 *  blocks       workgroups of 256 lanes, 0: 64 per compute unit
 *  stream       hipStream_t (NULL: default stream)
 * Asynchronous; time it with events on the same stream.  EINVAL for bad
 * sizes, modes or NULL pointers; EDEVICE if the launch fails. */
typedef enum { MLF_STREAM_READ = 0, MLF_STREAM_WRITE = 1, MLF_STREAM_COPY = 2 } mlf_stream_mode;
mlf_status mlf_stream_probe(int32_t mode, int32_t schedule, int32_t nontemporal, const void* src, void* dst,
                            uint64_t bytes, int32_t blocks, void* stream);

/* ---- host helpers (no device work) ---------------------------------- */

/* Spreading coefficients from a full symmetric tension table
 * g[(N+2)*(N+2)] (index 0 = substrate, N+1 = gas), Eq. (spreading_parameters):
 * S_l1 = g_{l,l+2} - g_{l,l+1} - g_{l+1,l+2},
 * S_lk = g_{l,l+k+1} + g_{l+1,l+k} - g_{l,l+k} - g_{l+1,l+k+1} (k >= 2);
 * written packed as in mlf_params.spread. */
mlf_status mlf_spreading_from_tensions(int32_t n_layers, const double* g, double* spread);

/* Friction matrix K (row-major N x N, friction = K q) of one node with
 * thicknesses h[N] and viscosities mu[N], from the boundary conditions of
 * Sec. II.A.2 (no slip), and the largest |eigenvalue| of -K. */
mlf_status mlf_friction_matrix(int32_t n_layers, const double* h, const double* mu,
                               double* K, double* max_rate);

/* As mlf_friction_matrix with slip lengths slip[N] >= 0: each layer's
 * profile extrapolated slip_i below its base meets the velocity of the layer
 * beneath (0 at the substrate), the boundary condition of Eq. (no_slip)
 * with a slip length. */
mlf_status mlf_friction_matrix_slip(int32_t n_layers, const double* h, const double* mu, const double* slip,
                                    double* K, double* max_rate);

/* Library version string. */
const char* mlf_version(void);

#ifdef __cplusplus
}
#endif
#endif
