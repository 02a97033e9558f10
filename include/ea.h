/*
 * ea.h -- C ABI of the MI355X (gfx950) library for checkerboard Metropolis
 * ageing simulations of the three-dimensional +-J Edwards-Anderson model
 * (Manssen & Hartmann, "Ageing at the Spin-Glass/Ferromagnet Transition:
 * Monte Carlo Simulation using GPUs").
 *
 * Model (Sec. II, eq. 1): N = L^3 Ising spins on a periodic cubic lattice,
 * H = -sum_<ij> J_ij S_i S_j with i.i.d. couplings J = +-1.  In this library
 * p is the probability of an antiferromagnetic coupling, P(J = -1) = p (the
 * paper's p is the ferromagnetic fraction, 1 - p here).  A run is one
 * coupling realisation ("sample") with two replicas that start from
 * independent random spins (quench from infinite temperature) and evolve
 * with independent thermal noise.
 *
 * Dynamics (Sec. III, eq. 9): single-spin-flip Metropolis on the two
 * checkerboard sub-lattices.  Colour c(x,y,z) = (x+y+z) & 1.  A sweep is two
 * half-steps; replica r updates colour r in the first and colour 1-r in the
 * second (the interlaced order of Fig. 1).  A site whose flip changes the
 * energy by dE <= 0 flips; dE = 4k > 0 flips iff its random word u is below
 * thr_k = floor(exp(-4k/T) 2^32) (0 at T = 0).  The random word of a site is
 * word (h & 3) of the Philox4x32-10 block with key = seed and counter
 * (t, h >> 2, tag << 8 | colour << 1 | replica, sample), where
 * h = (x >> 1) + (L/2)(y + L z) is the site's index inside its colour, t the
 * 0-based sweep index and tag 0.  Couplings use tag 1 (counter word 0 = bond
 * direction d, replica 0; J = -1 iff u < floor(p 2^32) compared in 64 bits),
 * initial spins tag 2 (counter word 0 = 0; S = -1 iff the top bit of u is
 * set).  Results
 * therefore depend only on (L, p, T, seed, sample, schedule), never on the
 * launch configuration.
 *
 * Conventions of the ABI:
 *   - every call returns ea_status; EA_OK = 0, errors are negative and
 *     ea_last_error() returns a message for the calling thread;
 *   - handles are owned by the caller from *_create until *_destroy
 *     (destroy accepts NULL);
 *   - host arrays are owned by the caller and must have the documented size;
 *   - device memory is owned by the library unless ea_config.dev_buf is
 *     given, in which case the library carves its arrays from that buffer
 *     (at least ea_footprint() bytes, 256-byte aligned, outliving the handle);
 *   - work is enqueued on ea_config.stream (a hipStream_t; NULL means the
 *     library creates and owns one); ea_sweep and ea_snapshot return without
 *     waiting, every call that hands data to the host synchronises that
 *     stream;
 *   - a handle is used by one host thread at a time.
 * Spin and coupling arrays exchanged with the host are int8 +-1 in canonical
 * order s = x + L (y + L z); couplings are laid out [s][d], J[3 s + d]
 * coupling s to s + e_d (d = 0, 1, 2 for x, y, z), the "left/up" bonds of
 * Sec. III.
 */
#ifndef EA_H
#define EA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EA_OK = 0,
    EA_ERR_ARG = -1,     /* an argument is out of range or inconsistent */
    EA_ERR_NOMEM = -2,   /* device or host allocation failed */
    EA_ERR_DEVICE = -3,  /* a HIP call failed */
    EA_ERR_STATE = -4,   /* the call does not fit the handle's state */
    EA_ERR_BUSY = -5     /* a queue is full; retry later */
} ea_status;

/* Message of the last failed call on this thread ("" if none). */
const char *ea_last_error(void);

/* Library version string. */
const char *ea_version(void);

typedef struct ea_sim ea_sim;

typedef struct {
    int32_t L;            /* side length: multiple of 8, 8..256 */
    double p;             /* P(J = -1), in [0, 1] */
    double T;             /* temperature >= 0, finite (J = 1, k_B = 1) */
    uint64_t seed;        /* Philox key */
    uint32_t sample;      /* disorder sample index (counter word 3) */
    int32_t n_tw_slots;   /* number of reference configurations S(t_w), 0..64 */
    void *stream;         /* hipStream_t to enqueue on, or NULL */
    void *dev_buf;        /* optional caller-owned device buffer, or NULL */
    size_t dev_buf_bytes; /* its size in bytes */
    int32_t words_per_row; /* bit packing: 32-bit words per row of L/2 same-colour sites,
                              each holding a whole number of 4-site blocks and at most 32
                              sites; 0 = the library's choice (autotuned by ea_tune_plain
                              if it ran for L, else enough words that one half-step launch
                              has at least 65536 threads).  Results never depend on it. */
} ea_config;

/* Observables at the current time t, integer sums over the N sites (the
 * paper's normalised quantities are these divided by N):
 *   unsat[r]    unsatisfied bonds of replica r; energy E_r = 2 unsat[r] - 3N (eq. 1)
 *   mag[r]      sum_s S_r(s)
 *   overlap     sum_s S_0(s) S_1(s)  (N q, eq. 2)
 *   autocorr    [2][n_tw]: sum_s S_r(s,t) S_r(s,tw_k)  (N C(t - tw_k, tw_k), eq. 7)
 *   c4          [3][rmax+1]: sum_s q(s) q(s + rho e_d), q = S_0 S_1, rho = 0..rmax
 *               (N C4(rho e_d, t), eq. 3)
 *   tw          [n_tw]: time at which each slot was taken (0 if never);
 *               a slot that was never taken reports autocorr 0
 * The caller provides tw/autocorr (n_tw = the handle's slot count, or 0 and
 * NULL to skip) and c4 (rmax = L/2, or NULL to skip). */
typedef struct {
    uint64_t t;
    int64_t unsat[2];
    int64_t mag[2];
    int64_t overlap;
    int32_t n_tw;
    uint64_t *tw;
    int64_t *autocorr;
    int32_t rmax;
    int64_t *c4;
} ea_obs;

/* Device bytes a run of side L with n_tw snapshot slots needs, in the
 * packing the library would choose now (words_per_row = 0); ea_footprint_ex
 * takes L, n_tw_slots and words_per_row from a config. */
ea_status ea_footprint(int32_t L, int32_t n_tw, size_t *bytes);
ea_status ea_footprint_ex(const ea_config *cfg, size_t *bytes);

/* Acceptance thresholds of eq. (9): out[k-1] for dE = 4k, k = 1..3. */
ea_status ea_thresholds(double T, uint32_t out[3]);

/* Race and order debug mode.  Within a half-step of the checkerboard
 * schedule (Sec. III, Fig. 1) the sites of one colour depend only on the
 * other colour, so the result may not depend on which workgroup updates
 * which part of the lattice, in what order, or on what LDS held before a
 * kernel started; this mode changes all three so that a test can check that
 * the bits stay the same.  flags (any combination; 0 = off, the default):
 *   EA_DEBUG_REVERSE  workgroups take their tiles in reverse order: blocks
 *                     of the half-step launches (plain, grouped, multispin),
 *                     shares of the slab launches, units of the batched and
 *                     serving launches (split pairs stay in front, so that
 *                     they are still resident together);
 *   EA_DEBUG_ROTATE   the same orders rotated by `seed` positions;
 *   EA_DEBUG_POISON   the persistent kernels (slab, batched) fill their LDS
 *                     with a pattern derived from `seed` before loading.
 * Process-wide; it applies to launches made after the call, on any device
 * (a graph captured before keeps the mode it was captured with; the plain
 * form's own sweep graph is captured again).  Set it while no work of the
 * library is in flight.  Results are bit-identical in every mode; the
 * launches are as fast as the default ones up to the changed placement.
 * EA_ERR_ARG for unknown flag bits. */
enum { EA_DEBUG_REVERSE = 1, EA_DEBUG_ROTATE = 2, EA_DEBUG_POISON = 4 };
ea_status ea_set_debug(uint32_t flags, uint32_t seed);
ea_status ea_get_debug(uint32_t *flags, uint32_t *seed);

/* Create a run and generate its couplings and initial spins on the device
 * (t = 0).  EA_ERR_ARG for L not a multiple of 8 or outside 8..256, p outside
 * [0,1] or NaN, T negative or not finite, n_tw_slots outside 0..64, or a
 * dev_buf smaller than ea_footprint(). */
ea_status ea_create(int32_t L, double p, double T, uint64_t seed, ea_sim **out);
ea_status ea_create_ex(const ea_config *cfg, ea_sim **out);
void ea_destroy(ea_sim *sim);

/* The run's bit packing (words per row). */
ea_status ea_words_per_row(const ea_sim *sim, int32_t *rw);

/* Full-vector four-point correlation at the current time (eq. 3 over every
 * displacement r, not only the lattice axes), summed by distance shell:
 * out[k] = sum over all r in Z_L^3 with minimum-image squared length
 * sum_d min(r_d, L - r_d)^2 = k of sum_s q(s) q(s + r), q = S_0 S_1, for
 * k = 0 .. n_shells - 1.  n_shells = (L/2)^2 + 1 covers |r| <= L/2, the range
 * of the integral estimators (eqs. 5, 6); 3 (L/2)^2 + 1 covers every r.
 * Dividing a shell by N and by the number of lattice vectors in it gives the
 * shell average of C4.  Two routes give the same integers (ea_set_shell_route):
 * the direct one counts differing bits for every displacement (work ~ L^6 /
 * 64: about 20 ms at L = 128, over a second at L = 256); for L = 2^k or
 * 3 2^k the FFT route takes the fp64 3D DFT of q, its squared modulus and the
 * inverse DFT (the Wiener-Khinchin theorem), rounds each sum to the nearest
 * integer and bins it (work ~ L^3 log L).  Synchronises; allocates a device
 * scratch buffer of 8 (2 L^2 ceil(L/64) + 3 (L/2)^2 + 1) bytes on the first
 * call, and on the first FFT-route call one of 16 L^3 + 256 bytes (256 MiB
 * at L = 256), both kept until ea_destroy.  EA_ERR_ARG for n_shells outside
 * [1, 3 (L/2)^2 + 1]; EA_ERR_NOMEM if a scratch buffer cannot be allocated;
 * EA_ERR_DEVICE if a sum of the FFT route is not within 1/4 of an integer
 * (outside the fp64 error bound, which is below 1e-7 here). */
ea_status ea_c4_shells(ea_sim *sim, int32_t n_shells, int64_t *out);

/* Route of the full-vector C4 shells (ea_c4_shells, ea_batch_c4_shells,
 * ea_msc_c4_shells; ea_c4_shells_into always takes the direct route):
 *   EA_SHELLS_AUTO    the FFT route for L = 2^k or 3 2^k >= 64, else direct
 *                     (the default);
 *   EA_SHELLS_DIRECT  the direct route for every L;
 *   EA_SHELLS_FFT     the FFT route for every L = 2^k (8 .. 256) or 3 2^k (24 .. 192); other
 *                     L take the direct route.
 * Both routes give identical results.  Process-wide, read at each call.
 * EA_ERR_ARG for another value. */
enum { EA_SHELLS_AUTO = 0, EA_SHELLS_DIRECT = 1, EA_SHELLS_FFT = 2 };
ea_status ea_set_shell_route(int32_t route);
ea_status ea_get_shell_route(int32_t *route);

/* ea_c4_shells for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The same shell sums, written as int64 to the caller's device array
 * out_dev[n_shells] (device memory, caller-owned), enqueued on the run's
 * stream without synchronising: they are valid once the stream has reached
 * this call.  The scratch (the dense overlap rows) is a static device array
 * of 512 KiB on every device the library runs on, held until the process
 * ends; hence L <= 128 here (EA_ERR_ARG beyond, and for n_shells outside
 * [1, 3 (L/2)^2 + 1]).  All calls on one device share that array: calls
 * that overlap on a device (runs on different streams) race, so order them
 * on one stream or synchronise between them.  Allocates nothing. */
ea_status ea_c4_shells_into(ea_sim *sim, int32_t n_shells, int64_t *out_dev);

/* Restart the run in place for another disorder sample: regenerate the
 * couplings and both replicas' initial spins for (seed, sample), set t = 0
 * and forget every snapshot; asynchronous, allocates nothing. */
ea_status ea_reset(ea_sim *sim, uint64_t seed, uint32_t sample);

/* Advance both replicas by n sweeps (t += n); asynchronous.  EA_ERR_ARG if
 * t + n would reach 2^32 (the sweep index is one counter word). */
ea_status ea_sweep(ea_sim *sim, uint64_t n);

/* Advance n_sims runs of the same L and words_per_row by n sweeps each,
 * up to 16 runs per launch (slab launches as in ea_set_slab_plan, else one
 * launch per half-step), giving exactly the
 * spins that n_sims separate ea_sweep calls give (Sec. III's update; every
 * run keeps its own key, sample, T and sweep counter).  For several small
 * independent samples, such as Sec. IV's L = 128 averages, whose single
 * half-steps are too short to fill the device.  The work is enqueued on the
 * first run's stream after everything already queued on the others, and the
 * others' later work waits for it; asynchronous.  EA_ERR_ARG if sims is NULL
 * or n_sims < 1, a run is NULL or listed twice, L or words_per_row differ,
 * or t + n would reach 2^32 for any run; then no run advances.  A group runs
 * fastest when its members use the densest packing (fewest words per row),
 * since it needs no extra threads to fill the device. */
ea_status ea_sweep_group(ea_sim *const *sims, int32_t n_sims, uint64_t n);

/* Persistent slab path of the plain form.  ea_sweep and ea_sweep_group run
 * a lattice whose plane of one colour has at most 1024 packed words
 * (L x words_per_row <= 1024) in one persistent launch per call (up to 16384
 * sweeps each; longer calls are split): every replica is cut into `slabs`
 * z-slabs of consecutive planes, each held with `ghost` extra planes on
 * either side in one workgroup's LDS, and the slabs exchange their boundary
 * planes through device memory once every `ghost` half-steps.  The ghost
 * planes are updated redundantly with the same keyed random words as their
 * owners', so results are bit-identical to one launch per half-step
 * (Sec. III's schedule).  slabs: 0 = the library's choice (the default),
 * -1 = off (one launch per half-step), 1..L = that many slabs per replica;
 * ghost: 0 = the library's choice for that slab count, else 1..8.
 * EA_ERR_ARG if the plan does not fit the device with one workgroup per
 * compute unit (2 x slabs workgroups per run) or a slab with its ghost
 * planes does not fit one workgroup's LDS.  Every workgroup of a launch must
 * be resident at once: if work of other streams keeps compute units busy for
 * seconds, the launch gives up and the next synchronising call (ea_sync,
 * ea_measure, ea_get_spins) returns EA_ERR_DEVICE; the run's state is then
 * undefined until ea_reset.  ea_sweep_group follows the first run's setting.
 * Allocates nothing (the exchange area is part of ea_footprint). */
ea_status ea_set_slab_plan(ea_sim *sim, int32_t slabs, int32_t ghost);
/* The plan ea_sweep uses for this run alone: slabs per replica and ghost
 * planes, or slabs = -1 and ghost = 0 when it launches once per half-step. */
ea_status ea_get_slab_plan(const ea_sim *sim, int32_t *slabs, int32_t *ghost);

/* Store the current spins as reference S(t_w) in slot k, t_w = t. */
ea_status ea_snapshot(ea_sim *sim, int32_t slot);

/* Measure the observables at the current time (synchronises). */
ea_status ea_measure(ea_sim *sim, ea_obs *out);

ea_status ea_time(const ea_sim *sim, uint64_t *t);
/* Set the sweep counter (resume from a checkpoint taken at time t). */
ea_status ea_set_time(ea_sim *sim, uint64_t t);
ea_status ea_sync(ea_sim *sim);

/* Spins of replica r (0 or 1) as int8 +-1 [N], and couplings [3N]. */
ea_status ea_get_spins(ea_sim *sim, int32_t r, int8_t *pm1);
ea_status ea_set_spins(ea_sim *sim, int32_t r, const int8_t *pm1);
ea_status ea_get_bonds(ea_sim *sim, int8_t *pm1);
ea_status ea_set_bonds(ea_sim *sim, const int8_t *pm1);

/* ------------------------------------------------------------------------
 * Batched form: many independent runs of different L, p, T and schedule in
 * one persistent launch.  Each replica of each job is owned by one
 * workgroup that keeps the replica's spins and the job's couplings in LDS and
 * takes the scheduled snapshots and measurements itself, so L is limited by
 * the LDS of one compute unit (multiple of 8 in 8..64).  A job's results are
 * bit-identical to a plain run (ea_create) with the same parameters: the
 * random words depend only on (seed, sample, replica, sweep, site).
 */
typedef struct ea_batch ea_batch;

typedef struct {
    int32_t L;               /* multiple of 8 in 8..64 */
    double p;                /* P(J = -1) in [0, 1] */
    double T;                /* temperature >= 0, finite */
    uint64_t seed;
    uint32_t sample;
    uint64_t n_sweeps;       /* below 2^32 */
    const uint64_t *meas_t;  /* [n_meas] measurement times, strictly increasing, <= n_sweeps */
    int32_t n_meas;
    const uint64_t *tw;      /* [n_tw] snapshot times S(t_w), strictly increasing, <= n_sweeps */
    int32_t n_tw;            /* 0..64 */
} ea_job;

typedef struct {
    void *stream;            /* hipStream_t to enqueue on, or NULL for a library stream */
    int32_t autotune;        /* 1: run each lattice size with its autotuned configuration */
    int32_t split;           /* replicas split across two workgroups (see below): 0 automatic,
                                1 never, 2 every job that can be (L >= 48, default configuration),
                                as long as all slabs fit the device at once */
} ea_batch_opts;

/* Split replicas.  When one replica of the largest samples on one compute
 * unit would set the length of a run, ea_batch_create may cut the replicas of
 * samples with L >= 48 (default configuration only) into two z-slabs held by
 * two workgroups that exchange their boundary planes every half-step through
 * device memory.  The choice is made by simulating the dispatch of the unit
 * list; results are identical either way.  A pair that never meets (its
 * partner never became resident within seconds) ends its units and makes
 * ea_batch_run / ea_batch_replay return EA_ERR_DEVICE. */

/* Launch configuration of the batched kernel for one lattice size. */
typedef struct {
    int32_t words_per_row;   /* packed words per row of L/2 same-colour sites */
    int32_t threads;         /* working threads per workgroup */
    int32_t select;          /* threshold select: 0 = LDS table, 1 = register bit-field selects */
    double ms;               /* time of the probe run with this configuration */
    int32_t parity_ok;       /* 1 if its results equal the default configuration's bit for bit */
} ea_tune_choice;

/* Autotune the batched kernel for lattice size L: time every valid
 * configuration (row packing, threads, select variant) on a probe batch of 64
 * samples, reject any whose results differ from the default configuration's,
 * keep the fastest.  The choice is cached for the process and, if the
 * environment variable EA_TUNE_CACHE names a file, appended to it and read
 * back by later processes.  force = 1 re-tunes.  tried[0..max_tried) receives
 * the candidates (the first is the default); *n_tried their number (0 when
 * the choice came from the cache). */
ea_status ea_tune(int32_t L, int32_t force, ea_tune_choice *chosen, ea_tune_choice *tried, int32_t max_tried,
                  int32_t *n_tried);

/* Autotune the plain form's bit packing for side L: time a burst of sweeps
 * for every valid words-per-row, reject any whose final spins differ from the
 * coarsest packing's, keep the fastest for later ea_create calls with
 * words_per_row = 0 (and append it to EA_TUNE_CACHE if set).  tried[i]
 * reports words_per_row, threads per half-step launch, ms and parity_ok
 * (select = 1); *n_tried = 0 when the choice came from the cache. */
ea_status ea_tune_plain(int32_t L, int32_t force, int32_t *chosen_rw, ea_tune_choice *tried, int32_t max_tried,
                        int32_t *n_tried);

/* Copy the job list (the caller's schedule arrays may be freed afterwards),
 * allocate device memory for every job and generate the initial states.
 * EA_ERR_ARG names the first invalid job. */
ea_status ea_batch_create(const ea_job *jobs, int32_t n_jobs, const ea_batch_opts *opts, ea_batch **out);
void ea_batch_destroy(ea_batch *b);

/* Regenerate every job's couplings and initial spins, t = 0, clear results. */
ea_status ea_batch_reset(ea_batch *b);

/* Advance every job to min(t_stop, its n_sweeps), taking the snapshots and
 * measurements scheduled on the way; returns when the launch has finished. */
ea_status ea_batch_run(ea_batch *b, uint64_t t_stop);

/* Capture "reset every job, then run every job to its end" as a hipGraph;
 * ea_batch_replay launches it and waits.  Replays give identical results. */
ea_status ea_batch_capture(ea_batch *b);
ea_status ea_batch_replay(ea_batch *b);

/* Sweeps done by job j. */
ea_status ea_batch_time(ea_batch *b, int32_t job, uint64_t *t);

/* Observables of job j's k-th scheduled measurement (ea_obs as for a plain
 * run; n_tw = the job's snapshot count, slots whose t_w lies after the
 * measurement report autocorr 0).  EA_ERR_STATE if it was not reached. */
ea_status ea_batch_result(ea_batch *b, int32_t job, int32_t k, ea_obs *out);

/* Full-vector C4 shells (as ea_c4_shells, eq. 3 over every displacement) of
 * job `job` at its measurement k, from the configuration of both replicas
 * that the batched kernel publishes at each measurement: out[n_shells].
 * Synchronises; allocates a scratch buffer of 8 (2 L^2 ceil(L/64) +
 * n_shells) bytes (16 L^3 more on the FFT route) on the first call, grown
 * when a later call needs more, kept until ea_batch_destroy.  EA_ERR_ARG for a job or k out of
 * range or n_shells outside [1, 3 (L/2)^2 + 1]; EA_ERR_STATE if measurement
 * k has not been reached. */
ea_status ea_batch_c4_shells(ea_batch *b, int32_t job, int32_t k, int32_t n_shells, int64_t *out);

/* Current spins of replica r of job j, int8 +-1 in canonical order [L^3]. */
ea_status ea_batch_get_spins(ea_batch *b, int32_t job, int32_t r, int8_t *pm1);

/* Workgroups per replica of job j: 1, or 2 if its replicas run split. */
ea_status ea_batch_parts(ea_batch *b, int32_t job, int32_t *parts);

/* ------------------------------------------------------------------------
 * Serving form: continuous batching of a stream of jobs.  The dynamics
 * (Sec. III, eq. 9) and measurements (eqs. 1-3, 7) are those of a run
 * alone; only the scheduling is new.  Jobs are admitted first-come
 * first-served while their device footprint fits hbm_budget and fewer than
 * max_resident are resident.  Each epoch advances every resident job by a
 * span of sweeps, taking its scheduled snapshots and measurements:
 *   - L <= 64: one persistent launch of the batched kernel holds every such
 *     job in LDS; its span is about epoch_site_sweeps site updates per
 *     replica (at least one sweep);
 *   - 64 < L <= 256 (multiple of 8): the job is a plain-form simulation in
 *     its pool region, advanced by persistent slab launches (as ea_sweep)
 *     from one of a few worker threads, each with a library stream of its
 *     own (as many as the process's hardware queues, GPU_MAX_HW_QUEUES,
 *     allow beside the batched stream, at most four), on the compute units
 *     the batched launch leaves free; its span is sized so that the streamed
 *     work takes about as long as the last batched launch;
 *   - a job with 48 <= L <= 64 takes that slab path too when it is admitted
 *     while some worker has no job, and a batched one with much work left
 *     moves to it mid-run when a worker frees up (its state, snapshots and
 *     measurements so far carried over), so that a lone small job does not
 *     run on two compute units while the device idles.
 * Finished jobs hand their results to the host and free their memory;
 * waiting jobs join at the next epoch.  A job's results are identical to a
 * run alone (ea_create, or ea_batch_create for L <= 64) with the same
 * parameters.  The calls are thread-safe: jobs can be submitted while a
 * worker thread (ea_server_start) runs the epochs.
 */
typedef struct ea_server ea_server;

typedef struct {
    size_t hbm_budget;           /* bytes of device memory for resident jobs */
    int32_t max_resident;        /* resident jobs at most (1..4096) */
    int32_t max_pending;         /* waiting jobs at most; submit returns EA_ERR_BUSY beyond */
    uint64_t epoch_site_sweeps;  /* site updates per replica per epoch; 0 = 64^4 */
    void *stream;                /* hipStream_t of the batched launches, or NULL for a library stream */
} ea_server_opts;

typedef struct {
    uint64_t submitted, admitted, completed, epochs;
    int32_t resident, pending;
    double p50_latency_s, p99_latency_s, mean_latency_s, max_latency_s; /* submit -> results on host */
    double flips;         /* attempted flips done (both replicas) */
    double busy_s;        /* time inside epoch launches */
    double wall_s;        /* since the first submit */
    double ps_per_flip;   /* busy_s / flips */
    size_t hbm_in_use, hbm_peak;
    uint64_t streamed_small; /* jobs with L <= 64 admitted to the slab path (a worker was free) */
    uint64_t moved;          /* jobs moved from the batched launch to the slab path mid-run */
} ea_server_report;

enum { EA_JOB_PENDING = 0, EA_JOB_RUNNING = 1, EA_JOB_DONE = 2 };

ea_status ea_server_create(const ea_server_opts *opts, ea_server **out);
void ea_server_destroy(ea_server *s);

/* Device bytes a job occupies while resident. */
ea_status ea_server_footprint(const ea_job *job, size_t *bytes);

/* Queue a job (its schedule is copied); *id names it from now on.
 * EA_ERR_BUSY if max_pending jobs already wait; EA_ERR_ARG for an invalid job
 * or one larger than the whole budget. */
ea_status ea_server_submit(ea_server *s, const ea_job *job, uint64_t *id);

/* Run one epoch on the calling thread (*progressed = 0 if there was nothing
 * to run).  EA_ERR_STATE while a worker thread runs. */
ea_status ea_server_step(ea_server *s, int32_t *progressed);

/* Run epochs on a worker thread until ea_server_stop. */
ea_status ea_server_start(ea_server *s);
ea_status ea_server_stop(ea_server *s);

/* Wait until every submitted job is done (runs epochs itself when no worker
 * runs).  EA_ERR_BUSY on timeout. */
ea_status ea_server_drain(ea_server *s, double timeout_s);

/* EA_JOB_PENDING, EA_JOB_RUNNING or EA_JOB_DONE. */
ea_status ea_server_poll(ea_server *s, uint64_t id, int32_t *state);

/* Measurement k of a finished job (ea_obs as for ea_batch_result), and the
 * time from its submission to its results reaching the host. */
ea_status ea_server_result(ea_server *s, uint64_t id, int32_t k, ea_obs *out);
ea_status ea_server_latency(ea_server *s, uint64_t id, double *seconds);

/* Forget a finished job's results. */
ea_status ea_server_release(ea_server *s, uint64_t id);

ea_status ea_server_stats(ea_server *s, ea_server_report *out);

/* ------------------------------------------------------------------------
 * Multispin-coded batch: asynchronous multispin coding (Sec. III).  The same
 * site of n_samples samples shares one word, and one random word per (sweep,
 * colour, replica, site) decides the Metropolis move (eq. 9) of that site in
 * every sample: Philox key (seed lo, seed hi), counter (t, h >> 2,
 * 3 << 8 | colour << 1 | replica, shared), word h & 3, with h the site's half
 * index as in the one-sample form.  Sample b (0 <= b < n_samples) gets the
 * couplings and initial spins that ea_create gives sample sample0 + b, and
 * then follows its own Metropolis chain, correlated with the others only
 * through the shared words; two batches with the same seed and shared id use
 * the same words.  All samples share L, p and T.
 *
 * Packing.  A 32-bit word holds M = min(n_samples, 32) samples; with fewer
 * than 32 the lattice is cut along z into 32 / M slabs whose same-position
 * sites share a word, a neighbour across a slab face being the word rotated
 * by M bits (the slab split of Sec. III); n_samples = 32 G (G up to 8) uses
 * G words per site that share the random words, as the paper's 64-bit words
 * do for G = 2.  The packing changes no result, only the work per random
 * word.
 *
 * Device memory: (4 + 2 (1 + n_tw_slots)) n_samples L^3 / 8 bytes of words
 * (couplings, spins, snapshots and the overlap words of the C4 pass) plus
 * counters (ea_msc_footprint).  Calls follow the one-sample form:
 * ea_msc_sweep and ea_msc_snapshot enqueue and return, calls that hand data
 * to the host synchronise the stream, one host thread at a time. */
typedef struct ea_msc ea_msc;

typedef struct {
    int32_t L;            /* multiple of 8 in 8..256, and of 64 / n_samples when n_samples < 32 */
    int32_t n_samples;    /* 1, 2, 4, 8, 16, or a multiple of 32 up to 256 */
    double p;             /* P(J = -1), in [0, 1] */
    double T;             /* temperature >= 0, finite */
    uint64_t seed;        /* Philox key */
    uint32_t sample0;     /* sample b draws couplings and start as sample sample0 + b */
    uint32_t shared;      /* counter word 3 of the shared Metropolis words */
    int32_t n_tw_slots;   /* reference configurations S(t_w), 0..64 */
    void *stream;         /* hipStream_t to enqueue on, or NULL */
    void *dev_buf;        /* optional caller-owned device buffer (256-byte aligned), or NULL */
    size_t dev_buf_bytes; /* its size in bytes */
} ea_msc_config;

/* Device bytes of a batch; EA_ERR_ARG for an invalid L, n_samples or slot count. */
ea_status ea_msc_footprint(const ea_msc_config *cfg, size_t *bytes);

/* Create the batch and generate every sample's couplings and spins on the
 * device (t = 0).  EA_ERR_ARG for an invalid config (see the fields),
 * EA_ERR_NOMEM if the device allocation fails. */
ea_status ea_msc_create(const ea_msc_config *cfg, ea_msc **out);
void ea_msc_destroy(ea_msc *batch);

/* n sweeps of every sample (t += n); asynchronous.  EA_ERR_ARG if t + n
 * would reach 2^32. */
ea_status ea_msc_sweep(ea_msc *batch, uint64_t n);

/* Store every sample's spins as reference S(t_w) in slot k, t_w = t. */
ea_status ea_msc_snapshot(ea_msc *batch, int32_t slot);

/* Observables of every sample at the current time: out[b] for sample b,
 * b < n_samples, each filled as ea_measure fills its ea_obs (tw/autocorr
 * and c4 may be NULL per sample).  Synchronises. */
ea_status ea_msc_measure(ea_msc *batch, ea_obs *out);

/* Full-vector C4 shells (as ea_c4_shells) of sample `sample` (0 .. B-1) of
 * the batch at the current time: out[n_shells].  Synchronises; allocates a
 * scratch buffer of 8 (2 L^2 ceil(L/64) + n_shells) bytes (16 L^3 more on
 * the FFT route) on the first call, grown when a later call needs more, kept
 * until ea_msc_destroy.  EA_ERR_ARG for a sample out of range or n_shells outside
 * [1, 3 (L/2)^2 + 1]. */
ea_status ea_msc_c4_shells(ea_msc *m, int32_t sample, int32_t n_shells, int64_t *out);

/* Spins of sample b, replica r, as int8 +-1 [N] in canonical order; set
 * rejects values other than +-1.  Couplings of sample b, [3N] as in
 * ea_get_bonds.  Synchronise. */
ea_status ea_msc_get_spins(ea_msc *batch, int32_t b, int32_t r, int8_t *pm1);
ea_status ea_msc_set_spins(ea_msc *batch, int32_t b, int32_t r, const int8_t *pm1);
ea_status ea_msc_get_bonds(ea_msc *batch, int32_t b, int8_t *pm1);

ea_status ea_msc_time(const ea_msc *batch, uint64_t *t);
/* Set the sweep counter (resume from a checkpoint taken at time t < 2^32). */
ea_status ea_msc_set_time(ea_msc *batch, uint64_t t);
ea_status ea_msc_sync(ea_msc *batch);

#ifdef __cplusplus
}
#endif
#endif
