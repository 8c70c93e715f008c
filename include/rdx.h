/*
 * rdx.h -- C ABI of the MI355X (gfx950) operator-splitting stochastic
 * reaction-diffusion library.
 *
 * The method is the one of "Parallel STEPS" (Chen & De Schutter,
 * arXiv:1610.02258): the run from t to t_end is cut into windows of constant
 * length tau (section 2.1); in each window every tetrahedron runs an exact SSA
 * over its own reactions, tracking species occupancy, and then every
 * diffusive species leaves each tet in a binomial number that is split among
 * the face neighbours in proportion to the face diffusion rates (section 2.2,
 * Algorithm 1).  On one GPU the paper's remote change buffers become direct
 * neighbour updates through the tet adjacency.
 *
 * Conventions shared by every entry point
 *   - Counts are int32, laid out species-major: counts[s * n_tets + tet].
 *   - Time is in seconds (FP64); lengths in metres; diffusion coefficients in
 *     m^2/s; rate constants in SI molar units: order 0 in M/s, order 1 in 1/s,
 *     order 2 in 1/(M s).  The mesoscopic constant of a reaction in a tet of
 *     volume V is k (N_A V[L])^(1 - order); a homodimer 2A uses N(N-1)/2 pairs.
 *   - Random numbers: Philox4x32-10 keyed by the 64-bit seed; counter =
 *     (draw call, stream, tet, window), stream 0 = the tet's SSA, stream 1+s =
 *     diffusion of species s.  Results depend only on (instance, seed, initial
 *     counts, window sequence), not on launch shapes or on other simulations
 *     sharing the GPU.
 *   - Every function returns an rdx_status; on failure rdx_last_error()
 *     returns a message for the calling thread.  Nothing is thrown across the
 *     ABI.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Host pointers
 *     are read or written before the call returns; device pointers
 *     (is_device_ptr != 0) are accessed in stream order and must stay valid
 *     until the stream reaches the call.
 *   - Input arrays are owned by the caller and copied; device state is owned
 *     by the library and released by rdx_destroy.
 */
#ifndef RDX_H
#define RDX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RDX_OK = 0,
  RDX_EINVAL = -1,      /* bad argument (null pointer, size out of range, bad table) */
  RDX_EMESH = -2,       /* non-positive tet volume, or a face shared by more than two tets */
  RDX_ENODIFF = -3,     /* no diffusive species and no tau override: tau undefined */
  RDX_ENOMEM = -4,      /* host or device allocation failed */
  RDX_EOVERFLOW = -5,   /* a molecule count passed 2^30 */
  RDX_EHIP = -6,        /* a HIP runtime call failed */
  RDX_EBUDGET = -7,     /* request larger than the server's device-memory budget */
  RDX_ECANCELLED = -8,  /* request cancelled */
  RDX_EEVENTS = -9,     /* more than 2^22 SSA events in one tet in one window */
  RDX_ESTATE = -10      /* call not valid in the object's current state */
} rdx_status;

/* Tetrahedral mesh.  verts [n_verts*3] (x, y, z per vertex, metres);
 * tets [n_tets*4] vertex indices; region [n_tets] region label per tet (< the
 * model's n_regions) or NULL for all zero.  Face k of a tet is the face
 * opposite its local vertex k. */
typedef struct rdx_mesh {
  int32_t n_verts;
  int32_t n_tets;
  const double* verts;
  const int32_t* tets;
  const uint8_t* region;
} rdx_mesh;

/* Reaction-diffusion model (section 2.1: the per-tet SSA system and the
 * diffusions it hosts).  diff_coef [n_species] (0 = immobile);
 * lhs, rhs [n_reactions*n_species] stoichiometry (reaction order = row sum of
 * lhs, at most 2); kcst [n_regions*n_reactions] rate constant of each reaction
 * in each mesh region.  Limits: 1 <= n_species <= 16, 0 <= n_reactions <= 32,
 * 1 <= n_regions <= 8; a reaction changes at most 8 species. */
typedef struct rdx_model {
  int32_t n_species;
  int32_t n_reactions;
  int32_t n_regions;
  const double* diff_coef;
  const int32_t* lhs;
  const int32_t* rhs;
  const double* kcst;
} rdx_model;

/* Cumulative tallies since the last rdx_set_counts: windows run, voxel-steps
 * (tets x windows), applied SSA events, molecules moved between tets, and
 * the nonzero (tet, species, face) moves -- each one an update of a
 * neighbour's count, the term that prices the diffusion update's writes. */
typedef struct rdx_stats {
  int64_t windows;
  int64_t voxel_steps;
  int64_t ssa_events;
  int64_t moves;
  double t;
  int64_t window_index;
  int64_t face_moves;
} rdx_stats;

typedef struct rdx_sim rdx_sim;

/* Set-up (section 2.1): builds the face adjacency, the face couplings
 * g_k = A_k / (V h_k) (A shared-face area, h barycentre distance), the window
 * tau = min over (species, tet) of 1/(D_S sum_k g_k) -- or tau_override when
 * > 0 -- and uploads the instance to the current HIP device.  seed keys all
 * random streams.  *out receives a handle with zero counts at t = 0.
 * Errors: RDX_EINVAL, RDX_EMESH, RDX_ENODIFF, RDX_ENOMEM, RDX_EHIP. */
rdx_status rdx_create(const rdx_mesh* mesh, const rdx_model* model, uint64_t seed,
                      double tau_override, rdx_sim** out);

/* Releases all host and device memory of the simulation (NULL is ignored),
 * after waiting for the work the simulation's calls enqueued on each stream
 * (it does not synchronise the whole device, so it may run while another
 * thread captures a graph). */
void rdx_destroy(rdx_sim* sim);

/* Initial populations (section 2.1, last step): counts [n_species*n_tets].
 * Resets t, the window index and the tallies to zero.
 * Errors: RDX_EINVAL (null, negative or > 2^30 entries), RDX_EHIP. */
rdx_status rdx_set_counts(rdx_sim* sim, const int32_t* counts, int is_device_ptr, void* stream);

/* Current counts into out [n_species*n_tets] (host or device pointer). */
rdx_status rdx_get_counts(rdx_sim* sim, int32_t* out, int is_device_ptr, void* stream);

/* Runtime main loop (Algorithm 1): windows of tau from the current t to t_end,
 * the last one truncated to t_end - t (after it t = t_end exactly).  Enqueued
 * on `stream`; does not synchronise.  t_end <= t is a no-op.
 * Errors: RDX_EINVAL, RDX_EHIP; device-side RDX_EOVERFLOW / RDX_EEVENTS are
 * reported by the next rdx_get_stats or rdx_sync. */
rdx_status rdx_run(rdx_sim* sim, double t_end, void* stream);

/* n_windows full windows of length tau (t advances by tau each). */
rdx_status rdx_step(rdx_sim* sim, int64_t n_windows, void* stream);

/* Waits for the simulation's work on `stream`, then reports any device-side
 * error flag (RDX_EOVERFLOW, RDX_EEVENTS). */
rdx_status rdx_sync(rdx_sim* sim, void* stream);

/* Synchronises `stream` and returns the tallies, t and window index. */
rdx_status rdx_get_stats(rdx_sim* sim, rdx_stats* stats, void* stream);

/* Time-varying forcing (section 3.2: the calcium influx, a zero-order
 * reaction, changes every 1 ms).  Replaces the rate constants kcst
 * [n_regions*n_reactions] (host pointer, region-major as in rdx_model,
 * n = n_regions*n_reactions) for every window enqueued on `stream` after
 * this call; windows enqueued before it keep the old constants.  To switch
 * at a time t_s, run to t_s first (the window that crosses t_s is cut there,
 * as at any t_end).  Synchronises `stream` before it returns, so kcst may be
 * freed at once; for the same reason it may not be called while `stream` is
 * being captured into a graph.  tau does not change (it depends on diffusion only).  The
 * table is not part of a checkpoint (rdx_save): set it again after rdx_load.
 * Errors: RDX_EINVAL (null handle, null kcst with n > 0, wrong n, a negative
 * or non-finite constant; the old table stays), RDX_EHIP. */
rdx_status rdx_set_rate_constants(rdx_sim* sim, const double* kcst, int64_t n, void* stream);

/* Recording (section 3.2 records per-region counts every 0.02 ms): out
 * [n_regions*n_species] int64, region-major, the molecules of each species
 * summed over the tets of each region, for the counts after all windows
 * enqueued so far on `stream`.  With is_device_ptr the sums are written by
 * kernels on `stream` and the call returns at once, so that a caller fills
 * a device ring buffer (one slot of n_regions*n_species per record) with no
 * host synchronisation between windows; the caller owns out and keeps it
 * alive until `stream` reaches the call.  With a host pointer the call waits.
 * The first call allocates a 257 KB device buffer for partial sums, kept
 * until rdx_destroy; calls on one handle share it, so order them on one
 * stream.
 * Errors: RDX_EINVAL (null), RDX_EHIP. */
rdx_status rdx_region_counts(rdx_sim* sim, int64_t* out, int is_device_ptr, void* stream);

/* rdx_region_counts for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same sums into the device pointer out
 * [n_regions*n_species] int64, enqueued on `stream` without waiting, with
 * no hipMalloc, hipFree or other allocation.  The partial sums live in one
 * static device array of 256 KiB per GPU, held until the process ends; its address is looked up at the first call on a device.
 * Every call on one GPU shares that array and fully rewrites the part it
 * reads, so nothing needs clearing, but calls that overlap in time on one
 * GPU (different streams, or different host threads without ordering) race
 * on it: order them on one stream.  The call records nothing on `stream`
 * for rdx_destroy to wait on: destroy the simulation only once `stream` has
 * reached the call.  Sizes: any n_tets; the slots needed for
 * (n_tets, n_species) are checked against the array.
 * Errors: RDX_EINVAL (null handle or out, or more scratch than the array
 * holds), RDX_EHIP. */
rdx_status rdx_region_counts_static(rdx_sim* sim, int64_t* out, void* stream);

/* Recording at a fixed window interval (section 3.2 records every 0.02 ms):
 * n_windows full windows of tau, and after each `every` of them the
 * per-region sums (as rdx_region_counts) into slot j mod ring_slots of the
 * device ring [ring_slots][n_regions*n_species] int64, for records j = 0, 1,
 * ... of this call (a trailing group shorter than `every` is not recorded).
 * The loop runs in the library, so the records cost no host round trip per
 * window; everything is enqueued on `stream` and the call does not wait.
 * *n_records (may be NULL) receives the number of records written.
 * Errors: RDX_EINVAL (n_windows < 0, every <= 0, ring_slots <= 0, null
 * ring), RDX_EHIP. */
rdx_status rdx_step_recorded(rdx_sim* sim, int64_t n_windows, int64_t every, int64_t* ring,
                             int64_t ring_slots, int64_t* n_records, void* stream);

rdx_status rdx_get_tau(const rdx_sim* sim, double* tau);
rdx_status rdx_get_sizes(const rdx_sim* sim, int32_t* n_tets, int32_t* n_species,
                         int32_t* n_reactions);

/* Derived set-up arrays, host pointers, each may be NULL: nbr [n_tets*4]
 * (-1 = boundary), g [n_tets*4], G [n_tets] (sum of g), cum [n_tets*4]
 * (cumulative split fractions (g_0 + ... + g_k) / G for k < 3, cum_3 = 1),
 * nav [n_tets] (N_A V[L]). */
rdx_status rdx_get_geometry(const rdx_sim* sim, int32_t* nbr, double* g, double* G,
                            double* cum, double* nav);

/* The same set-up arrays and tau computed on the host only, without creating
 * a simulation or touching a GPU (same layouts as rdx_get_geometry; *tau
 * receives the window).  Errors as rdx_create except RDX_ENOMEM/RDX_EHIP. */
rdx_status rdx_setup_geometry(const rdx_mesh* mesh, const rdx_model* model, double tau_override,
                              int32_t* nbr, double* g, double* G, double* cum, double* nav,
                              double* tau);

/* Per-kernel device time, measured with HIP events recorded on the launch
 * stream around every window's two kernels while timing is enabled: the
 * detect kernel (propensities and first SSA waiting time of every tet; lists
 * the tets with an event in the window) and the main kernel (diffusion of
 * every other tet, and the full SSA window and diffusion of the listed tets
 * in blocks of their own).  Timing adds three event records per window and
 * plain launches; it is off by default. */
typedef struct rdx_kernel_times {
  int64_t windows;        /* windows timed since the last reset */
  double detect_ms;       /* summed duration of the detect kernel */
  double main_ms;         /* summed duration of the main kernel */
} rdx_kernel_times;

rdx_status rdx_set_kernel_timing(rdx_sim* sim, int enable);

/* Synchronises the stream of the timed windows and returns the sums; with
 * reset != 0 the sums restart from zero. */
rdx_status rdx_get_kernel_times(rdx_sim* sim, rdx_kernel_times* out, int reset);

/* Checkpoint: counts, t, window index and tallies.  With buf == NULL, *len
 * receives the required size.  Resume is bit-identical because every draw is
 * addressed by the window index. */
rdx_status rdx_save(rdx_sim* sim, void* buf, size_t* len, void* stream);
rdx_status rdx_load(rdx_sim* sim, const void* buf, size_t len, void* stream);

/* Launch shape of the window kernels.  Results never depend on it (every
 * draw is addressed by (seed, stream, tet, window) and moves are integer
 * sums), only speed does.
 *   autotune       1: time the candidate shapes on the next windows run
 *                  (those windows are real work of the simulation) and keep
 *                  the fastest; get returns 1 while tuning is under way
 *   fast_grid_div  main kernel grid = resident grid / this (1, 2 or 4)
 *   graph_windows  windows per captured HIP graph, replayed as one launch;
 *                  1 = plain launches (1..256)
 *   event_group    most queued tiles (tiles with a tet whose first SSA event
 *                  falls in the window) one event block takes as a group,
 *                  their listed tets packed into chunks of up to 64 lanes
 *                  (1..64; 0 = the default, 4).  Where listed tets are sparse
 *                  (one per tile), larger groups leave fewer, fuller event
 *                  blocks and more blocks for the diffusion of every tet.
 *   event_bins     1: listed tets whose expected events in the window
 *                  (a0 tau) exceed 1 are queued apart from the others and
 *                  packed into event chunks of their own, so that a chunk's
 *                  lanes, which run their SSA chains in lock-step, have
 *                  chains of similar length (load balancing of skewed event
 *                  loads, section 3.2); 0: one queue.  Default 1.
 *   tile_claim     1: after its first tile, a diffusion block claims its
 *                  next tile at run time from a counter of its XCD's tile
 *                  range, so that blocks finish within about one tile of each
 *                  other where tiles differ in cost (molecules clustered in
 *                  part of the mesh); 0: static tile ranges.  Default 0. */
typedef struct rdx_exec_options {
  int32_t autotune;
  int32_t fast_grid_div;
  int32_t graph_windows;
  int32_t event_group;
  int32_t event_bins;
  int32_t tile_claim;
} rdx_exec_options;

rdx_status rdx_set_exec_options(rdx_sim* sim, const rdx_exec_options* opts);
rdx_status rdx_get_exec_options(const rdx_sim* sim, rdx_exec_options* opts);

/* ---- batch: many independent runs advanced by the same launches ----
 *
 * Run i is a complete simulation (its own mesh, model parameters, seed,
 * counts, t and window index), exactly as rdx_create would make it; every run
 * must share the species/reaction structure (n_species, n_reactions, lhs, rhs)
 * of run 0, while meshes, diffusion coefficients, rate constants and regions
 * may differ.  One window launch covers the tiles of every run with a window
 * to do, so small runs fill the GPU together.  Each run's counts equal those
 * of the same run alone (rdx_create + the same calls), bit for bit.  Device
 * memory for all runs is reserved at creation.  The launch shape starts in
 * autotune mode (see rdx_exec_options).  Calls on one batch must be ordered
 * by the caller (one stream, or synchronised streams).
 * Errors of create: as rdx_create, prefixed with the failing run's index;
 * RDX_EINVAL if a run's structure differs from run 0's. */
typedef struct rdx_batch rdx_batch;

rdx_status rdx_batch_create(int32_t n_runs, const rdx_mesh* meshes /* [n_runs] */,
                            const rdx_model* models /* [n_runs] */, const uint64_t* seeds /* [n_runs] */,
                            const double* tau_overrides /* [n_runs] or NULL */, rdx_batch** out);
void rdx_batch_destroy(rdx_batch* batch);
rdx_status rdx_batch_size(const rdx_batch* batch, int32_t* n_runs);
/* n_tets and tau of run i (either may be NULL). */
rdx_status rdx_batch_get_run_info(const rdx_batch* batch, int32_t i, int32_t* n_tets, double* tau);
/* As rdx_set_counts / rdx_get_counts for run i. */
rdx_status rdx_batch_set_counts(rdx_batch* batch, int32_t i, const int32_t* counts, int is_device_ptr,
                                void* stream);
rdx_status rdx_batch_get_counts(rdx_batch* batch, int32_t i, int32_t* out, int is_device_ptr,
                                void* stream);
/* As rdx_set_rate_constants / rdx_region_counts for run i (each run has its
 * own rate table). */
rdx_status rdx_batch_set_rate_constants(rdx_batch* batch, int32_t i, const double* kcst, int64_t n,
                                        void* stream);
rdx_status rdx_batch_region_counts(rdx_batch* batch, int32_t i, int64_t* out, int is_device_ptr,
                                   void* stream);
/* rdx_batch_set_counts for every run at once, from device memory, in one
 * launch: counts[i] is a device pointer to run i's [n_species*n_tets] int32
 * counts (caller-owned, alive until `stream` reaches the call); the host
 * array `counts` itself is read during the call.  Every run restarts at t = 0,
 * window 0, tallies cleared.  Errors: RDX_EINVAL (null pointer), RDX_EHIP. */
rdx_status rdx_batch_set_counts_all(rdx_batch* batch, const int32_t* const* counts /* [n_runs] */,
                                    void* stream);
/* Algorithm 1 for every run i from its t to t_end[i] (as rdx_run); the
 * windows of all runs are enqueued together on `stream`. */
rdx_status rdx_batch_run(rdx_batch* batch, const double* t_end /* [n_runs] */, void* stream);
/* n_windows full windows for every run (as rdx_step). */
rdx_status rdx_batch_step(rdx_batch* batch, int64_t n_windows, void* stream);
/* Waits for `stream`; reports the first device error flag of any run. */
rdx_status rdx_batch_sync(rdx_batch* batch, void* stream);
rdx_status rdx_batch_get_stats(rdx_batch* batch, int32_t i, rdx_stats* stats, void* stream);
rdx_status rdx_batch_set_exec_options(rdx_batch* batch, const rdx_exec_options* opts);
rdx_status rdx_batch_get_exec_options(const rdx_batch* batch, rdx_exec_options* opts);

/* ---- served form: a request loop with continuous batching ----
 *
 * A server owns a device-memory budget and one worker thread.  Each submitted
 * request (mesh, model parameters, seed, initial counts, t_end) is validated
 * and set up (section 2.1) on the submitting thread, then queued.  The
 * worker admits queued requests in arrival order while the budget has room
 * for their device state, enqueues one tick -- up to tick_windows windows of
 * every resident request, in the same launches -- and retires requests that
 * reached t_end, releasing their memory for the next admissions.  The ticks
 * are pipelined: uploads of new requests and reads of finished ones go on a
 * second stream while the tick before runs, and the worker waits for a
 * tick's end only to retire what it finished, after the next tick is already
 * enqueued.  A request's result is bit-identical to the same simulation run
 * alone (rdx_create, rdx_set_counts, rdx_run(t_end)).  Latency is measured
 * from submission to retirement.
 *
 * All requests share the species/reaction structure given at creation
 * (n_species, n_reactions, lhs, rhs); meshes, diffusion coefficients, rate
 * constants and regions may differ per request.  Functions may be called
 * from any thread; rdx_server_destroy cancels what is still queued or
 * running and must not race with other calls on the same server. */
typedef struct rdx_server rdx_server;

typedef enum {
  RDX_REQ_QUEUED = 0,
  RDX_REQ_RUNNING = 1,
  RDX_REQ_DONE = 2,
  RDX_REQ_FAILED = 3,
  RDX_REQ_CANCELLED = 4
} rdx_request_state;

typedef struct rdx_server_options {
  size_t hbm_budget_bytes;  /* device memory for the worklist and the requests' state (>= 1 MiB) */
  int32_t max_runs;         /* requests resident at once (0: up to 1024, as the budget allows) */
  int32_t tick_windows;     /* windows per scheduling tick (0 = 8) */
  int32_t graph_windows;    /* windows per captured graph (0 = tick_windows, 1 = plain launches) */
} rdx_server_options;

typedef struct rdx_request_info {
  int32_t state;            /* rdx_request_state */
  int32_t status;           /* rdx_status of a finished request */
  int32_t n_tets;
  int32_t n_species;
  double t_submit;          /* seconds since server creation */
  double t_admit;
  double t_done;
  rdx_stats stats;          /* tallies of a finished request */
} rdx_request_info;

typedef struct rdx_server_stats {
  int64_t submitted, completed, failed, cancelled, queued, running, ticks;
  int64_t voxel_steps, ssa_events, moves;  /* summed over completed requests */
  double busy_s;            /* device time of the ticks: from each tick's first to its last
                               launch on the device (HIP events), summed over retired ticks */
  double uptime_s;
  double latency_p50_s;     /* nearest-rank quantiles of completion - submission */
  double latency_p99_s;
  int64_t capacity_tets;    /* worklist capacity derived from the budget */
  double worker_s;          /* worker thread time spent on admissions' uploads and on planning
                               and enqueueing ticks (not on waiting for the device) */
} rdx_server_stats;

/* Errors: RDX_EINVAL (bad structure or options), RDX_ENOMEM, RDX_EHIP. */
rdx_status rdx_server_create(const rdx_model* structure, const rdx_server_options* opts,
                             rdx_server** out);
void rdx_server_destroy(rdx_server* server);
/* counts0 [n_species*n_tets] host pointer, copied.  *ticket identifies the
 * request.  Errors: as rdx_create; RDX_EINVAL if the structure differs;
 * RDX_EBUDGET if the request can never fit the budget; RDX_ESTATE while
 * shutting down. */
rdx_status rdx_server_submit(rdx_server* server, const rdx_mesh* mesh, const rdx_model* model,
                             uint64_t seed, const int32_t* counts0, double t_end,
                             double tau_override, int64_t* ticket);
rdx_status rdx_server_poll(rdx_server* server, int64_t ticket, rdx_request_info* info);
/* Blocks until the request is done, failed or cancelled (timeout_s < 0: no
 * limit; on timeout RDX_ESTATE and the request stays).  A done request's
 * counts go to counts_out (host, may be NULL).  Returns the request's status
 * and forgets the ticket. */
rdx_status rdx_server_wait(rdx_server* server, int64_t ticket, double timeout_s, int32_t* counts_out,
                           rdx_request_info* info);
/* Queued requests are dropped at once, running ones at the next tick boundary. */
rdx_status rdx_server_cancel(rdx_server* server, int64_t ticket);
rdx_status rdx_server_get_stats(rdx_server* server, rdx_server_stats* stats);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* rdx_last_error(void);

/* ABI version of this header (major * 100 + minor); the library returns
 * RDX_ABI_VERSION of the header it was built from. */
#define RDX_ABI_VERSION 209
int32_t rdx_version(void);

/* ---- device self-tests of the random layer (host pointers, synchronous) ---- */

/* Philox4x32-10 on the device: in [n*6] = (ctr0..3, key0, key1), out [n*4]. */
rdx_status rdx_selftest_philox(const uint32_t* in, uint32_t* out, int64_t n);

/* The library's basic-operation natural logarithm on the device, x > 0 normal. */
rdx_status rdx_selftest_ln(const double* x, double* y, int64_t n);

/* n binomial variates Bin(m, p); sample j is drawn from the species stream
 * (seed, stream_id, tet = j, window), exactly as the diffusion step draws. */
rdx_status rdx_selftest_binom(uint64_t seed, uint32_t stream_id, uint32_t window, int64_t m,
                              double p, int64_t n, int64_t* out);

/* A plain device-to-device copy of `bytes` bytes (16-byte vector loads and
 * stores, grid-stride), launched `reps` times after one warm-up; *gbps
 * receives (read + write bytes) / time.  Calibrates hardware byte counters
 * and measures the attainable copy bandwidth. */
rdx_status rdx_selftest_copy(int64_t bytes, int32_t reps, double* gbps);

#ifdef __cplusplus
}
#endif

#endif /* RDX_H */
