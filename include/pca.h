/*
 * pca.h - C ABI of the lazy Probabilistic Cellular Automaton (PCA) sampler for lattice
 * MRF posteriors, built for AMD Instinct MI355X (gfx950).
 *
 * Method: Costarelli, Piconi, Troiani, "Bayesian Inversion via Probabilistic Cellular
 * Automata: an application to image denoising" (arXiv 2507.14869).  Every sweep draws
 * the new grey level of every pixel of every chain independently from the lazy
 * posterior conditional of Sec. 5.2 (pair Hamiltonian eq.
 * (denoising_pair_posterior_Hamiltonian)): a nearest-neighbour pair prior with coupling
 * J, an inertia weight q tying each site to its own previous value, and a Gaussian data
 * term with standard deviation sigma that the inverse temperature beta does not scale
 * (Sec. 2 eq. (posterior_hamiltonian)).  The sweep also accumulates the running
 * posterior mean (Sec. 2 'Bayesian inference', law-of-large-numbers average) and a
 * per-pixel level histogram for the marginal posterior mode.
 *
 * Conventions shared by all entry points:
 *  - Every device pointer is caller-owned and must stay valid until the work enqueued
 *    on `stream` that uses it has finished.  Pointers are plain device addresses (for
 *    example a torch tensor's data_ptr()).
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.  All calls
 *    except pca_sync and pca_destroy only enqueue work and return immediately.
 *  - Argument errors are returned synchronously as negative codes and leave the context
 *    unchanged.  Errors raised by the device are returned by the next call on the
 *    context or by pca_sync.  pca_last_error() gives a message for the calling thread.
 *  - A context belongs to the device that was current at pca_init; call it with that
 *    device current.  A context is not thread-safe; distinct contexts are independent.
 *  - Randomness depends only on (seed, chain, sweep index, pixel): results do not depend
 *    on how sweeps are split across calls, on streams, or on other work on the device.
 *  - Layouts: images are row-major [height][width]; chain states are uint8 level
 *    indices, row-major [chains][height][width] at this boundary.
 *  - Failure handling can be exercised from the host: the environment variable
 *    PCA_FAULT_INJECT, read at every call, lists allocation sites that then fail as if
 *    memory were exhausted ("init": pca_init's device buffers; "admit:<id>" / "readout:<id>":
 *    a server request's device buffers at admission / host buffers for its results; a site
 *    without ":<id>" fails for every request).  Unset, it changes nothing.
 */
#ifndef PCA_MI355X_H
#define PCA_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pca_ctx pca_ctx; /* opaque, library-owned */

enum {
    PCA_OK = 0,
    PCA_EINVAL = -1,  /* invalid argument or parameter */
    PCA_ENOMEM = -2,  /* device (or host) allocation failed */
    PCA_EDEVICE = -3, /* HIP runtime or kernel error */
    PCA_ESTATE = -4,  /* operation not valid in the context's current state */
    PCA_EBUSY = -5    /* request refused by the server's load-shedding limit */
};

enum {
    PCA_PRIOR_POTTS = 0,       /* Potts pair potential V = -J if equal else +J, eq. (prior_pair_potential) */
    PCA_PRIOR_TRUNC_LINEAR = 1 /* J * min(|a - b|, trunc) in level units */
};

typedef struct {
    int32_t height, width; /* lattice size, >= 1 each, height*width < 2^31 */
    int32_t levels;        /* L grey levels, 2..256; level k has value vmin + k*(vmax-vmin)/(L-1) (Sec. 4) */
    int32_t chains;        /* independent chains, 1..1024 */
    int32_t neighbourhood; /* 4 or 8; the paper's neighbourhood eq. (neighborhood) is 8; free boundary */
    int32_t prior;         /* PCA_PRIOR_* */
    int32_t trunc;         /* truncation T >= 1 of the linear prior (ignored for Potts) */
    float J;               /* pair coupling >= 0 */
    float q;               /* inertia weight >= 0: a change of a site from x to k costs beta*q*|k-x|^p (Sec. 3) */
    float sigma;           /* noise standard deviation > 0, value units */
    float vmin, vmax;      /* values of levels 0 and L-1, vmax > vmin */
    const float *beta;     /* host array of per-sweep inverse temperatures (> 0), copied at init; NULL => 1 */
    int32_t beta_len;      /* sweeps past the end reuse the last value (schedule of Sec. 6) */
    uint64_t seed;         /* Philox4x32-10 key */
    int32_t init_mode;     /* 0: every chain starts at the level nearest the observation; 1: uniform random */
    int32_t burn_in;       /* sweeps with index < burn_in are not accumulated */
    int32_t tally_stride;  /* histogram every tally_stride-th sweep from burn_in on; 0 = no histogram */
    int32_t inertia;       /* exponent p of the inertia norm (Sec. 3, with 0^0 = 0): 0 = indicator, the
                              paper's experiments (Sec. 5.2); 1 = L1; 2 = L2 (both named in Sec. 5.2). */
} pca_params;

/* Creates a context: validates `params`, allocates the chain states, the mean
 * accumulator and (if tally_stride > 0) the histogram of height*width*levels uint16
 * counters, converts the observation to level units and initialises every chain.
 * obs_dev: device float32 [height][width] observation in value units, finite; it is read
 * during the enqueued initialisation only.  On success *out receives the context and the
 * sweep index is 0.  Errors: PCA_EINVAL (bad parameters, NULL pointers), PCA_ENOMEM,
 * PCA_EDEVICE. */
int pca_init(const pca_params *params, const float *obs_dev, void *stream, pca_ctx **out);

/* Enqueues n >= 0 sweeps of the lazy PCA (Sec. 5.2): sweep t reads state t of every chain
 * and writes state t+1, drawing each site from its conditional given the previous state
 * only; then adds every chain's new levels to the mean accumulator if t >= burn_in and to
 * the histogram on tally sweeps.  n = 0 is a no-op.  A sweep of more than 2^31 threads
 * (height*width*chains/4 for 3 or more chains) is enqueued as several kernel launches,
 * and on lattices with at most 16 levels too small to fill the GPU one kernel launch
 * advances several sweeps (pca_sweeps_per_launch), all with the same results.  Errors: PCA_EINVAL (n < 0),
 * PCA_ESTATE (the uint32 sum or a uint16 histogram counter could overflow, or the sweep
 * index, a 32-bit counter word of the random stream, would pass 2^32 - 1), PCA_EDEVICE. */
int pca_sweep(pca_ctx *ctx, int32_t n, void *stream);

/* Writes the posterior-mean estimate (Sec. 2, conditional mean; Monte Carlo average over
 * chains and accumulated sweeps) in value units: out = vmin + (sum/count)*(vmax-vmin)/(L-1),
 * computed in double and rounded once.  out_dev: device float32 [height][width].
 * Errors: PCA_ESTATE if no sweep has been accumulated yet, PCA_EINVAL. */
int pca_posterior_mean(pca_ctx *ctx, float *out_dev, void *stream);

/* Writes the marginal posterior mode: per pixel the level index with the largest tally,
 * ties to the lowest level.  out_dev: device uint8 [height][width].  Errors: PCA_ESTATE if
 * the histogram is disabled or empty, PCA_EINVAL. */
int pca_marginal_map(pca_ctx *ctx, uint8_t *out_dev, void *stream);

/* Copies the current states (the last sample of each chain, the paper's MAP output after
 * annealing, Sec. 6) to out_dev: device uint8 [chains][height][width]. */
int pca_get_state(pca_ctx *ctx, uint8_t *out_dev, void *stream);

/* Replaces the current states with in_dev (device uint8 [chains][height][width]) and sets
 * the sweep index to t (0 <= t <= 2^32 - 1).  Accumulators are kept.  Used to resume a run
 * or to re-synchronise with another implementation.  Every value must be a level index
 * (< levels): the values are checked on the device first, so this call waits for
 * `stream`.  Errors: PCA_EINVAL (NULL pointer, t out of range, or a value >= levels; the
 * context is then unchanged), PCA_EDEVICE. */
int pca_set_state(pca_ctx *ctx, const uint8_t *in_dev, int64_t t, void *stream);

/* Reports the sweep index, the number of samples in the mean accumulator (chains times
 * accumulated sweeps) and the number of tally sweeps.  Any pointer may be NULL. */
int pca_stats(const pca_ctx *ctx, int64_t *sweep, int64_t *count, int64_t *tallies);

/* Reports in *out how many sweeps one kernel launch of pca_sweep advances: 1, or up to 12
 * where each workgroup keeps a tile of the lattice with a halo as deep as that in LDS
 * (lattices with at most 16 levels, the indicator inertia and fewer than 65536 threads in
 * a single-sweep launch).  The results do not depend on it.  Errors: PCA_EINVAL (NULL
 * context or out). */
int pca_sweeps_per_launch(const pca_ctx *ctx, int32_t *out);

/* Checkpoint of the accumulators (with pca_get_state and pca_stats, everything a run needs
 * to resume bit-exactly, since every draw is keyed by the sweep index and not by a
 * generator state).  sum_dev: device uint32 [height][width], the sum of the levels of all
 * chains over the accumulated sweeps; hist_dev: device uint16 [height][width][levels], the
 * tally of each level over chains and tally sweeps, or NULL (required to be NULL when the
 * histogram is disabled).  Errors: PCA_EINVAL. */
int pca_get_accumulators(pca_ctx *ctx, uint32_t *sum_dev, uint16_t *hist_dev, void *stream);

/* Restores the accumulators from buffers laid out as in pca_get_accumulators, with the
 * sample and tally counts that go with them (as pca_stats reports them).  Errors:
 * PCA_EINVAL for NULL buffers, a histogram where the run has none, negative counts, or
 * counts whose totals could overflow the accumulators (count * (levels-1) >= 2^32,
 * tallies * chains > 65535). */
int pca_set_accumulators(pca_ctx *ctx, const uint32_t *sum_dev, const uint16_t *hist_dev, int64_t count,
                         int64_t tallies, void *stream);

/* Waits for all work the context enqueued and reports any device error. */
int pca_sync(pca_ctx *ctx);

/* Waits for the context's last stream, then frees it.  NULL is a no-op. */
int pca_destroy(pca_ctx *ctx);

/* Message of the last error on the calling thread ("" if none). */
const char *pca_last_error(void);

/* ------------------------------------------------------------------------------------
 * Batches.  Many independent lattices - each with its own size, level count, chains,
 * parameters, beta schedule and seed, all with the same neighbourhood - advanced
 * together: every sweep of the batch is ONE kernel launch covering all lattices, and
 * the launches are replayed from captured HIP graphs.  Each lattice's results are bit-identical to running it alone with
 * pca_init/pca_sweep (the draws are keyed by its own seed, chain, sweep and pixel).
 * All lattices share one sweep index.  Conventions as above; `i` selects a lattice.
 * ------------------------------------------------------------------------------------ */
typedef struct pca_batch pca_batch; /* opaque, library-owned */

/* Creates a batch of n >= 1 lattices from params[0..n-1] and the device observations
 * obs_dev[0..n-1] (float32 [height][width] each, read during initialisation only).
 * Errors: PCA_EINVAL (any invalid parameter set, NULL pointer, mixed neighbourhoods,
 * inertia 0 mixed with inertia 1 or 2), PCA_ENOMEM, PCA_EDEVICE. */
int pca_batch_init(const pca_params *params, const float *const *obs_dev, int32_t n, void *stream,
                   pca_batch **out);

/* Launch-configuration autotuner: times every valid configuration (chains per thread
 * 1/2/4, lanes sharing a pixel's data factor 1/2/4, and the traversal: `tiled` 0 untiled -
 * 2-D pixel patches for L > 16, row-major otherwise - 1 tiles 16 pixels wide, 2 as 0 but
 * the lattices with L <= 16 advance 7 sweeps per launch from LDS tiles with halos) over
 * trial_sweeps (1..64) burn-in sweeps and trial_sweeps accumulating
 * sweeps of this batch (each lattice from sweep 0 and from its burn-in length), in two
 * rounds, keeps the configuration with the smallest time of a round, then restores the
 * initial states (sweep index 0, accumulators cleared).  Synchronous.  *best_ms (may be
 * NULL) receives the winner's mean time per trial sweep.  The configuration never changes
 * results. */
int pca_batch_autotune(pca_batch *b, int32_t trial_sweeps, void *stream, float *best_ms);

/* The launch configuration in use, or set one explicitly (PCA_EINVAL if not valid for the
 * batch).  Setting a configuration does not change the state. */
int pca_batch_config(const pca_batch *b, int32_t *chains_per_thread, int32_t *share, int32_t *tiled);
int pca_batch_set_config(pca_batch *b, int32_t chains_per_thread, int32_t share, int32_t tiled, void *stream);

/* Enqueues n >= 0 sweeps of every lattice (as pca_sweep).  The sweeps are replayed from
 * cached HIP graphs of at most 64 launches each (n = 64q + r replays the 64-sweep graph q
 * times and an r-sweep graph once); a graph is captured and instantiated on first use (a
 * few ms).  Errors: PCA_EINVAL, PCA_ESTATE (accumulator overflow), PCA_EDEVICE. */
int pca_batch_sweep(pca_batch *b, int32_t n, void *stream);

/* Per-lattice readouts and statistics, as pca_posterior_mean, pca_marginal_map,
 * pca_get_state and pca_stats. */
int pca_batch_posterior_mean(pca_batch *b, int32_t i, float *out_dev, void *stream);
int pca_batch_marginal_map(pca_batch *b, int32_t i, uint8_t *out_dev, void *stream);
int pca_batch_get_state(pca_batch *b, int32_t i, uint8_t *out_dev, void *stream);
int pca_batch_stats(const pca_batch *b, int32_t i, int64_t *sweep, int64_t *count, int64_t *tallies);

/* Waits for the batch's last stream and reports device errors; frees the batch. */
int pca_batch_sync(pca_batch *b);
int pca_batch_destroy(pca_batch *b);

/* ------------------------------------------------------------------------------------
 * Request server: continuous batching of denoising requests.  Submitted requests wait in
 * a first-come-first-served queue until their device footprint fits the memory budget
 * and an active slot is free.  Each pca_server_step admits what fits, then gives every
 * admitted request at least one sweep and spends the rest of a GPU-time budget (step_ms,
 * from a cost model refined with every measured step) half on the requests with the least
 * remaining work and half on the oldest ones; the sweeps run as batched kernel launches,
 * launch i covering every
 * request still advancing at i, each at its own sweep index.  Finished requests are read
 * out to host memory and their device memory released at once, so queued requests can
 * join at the next step.  A request's results are bit-identical to running it alone with
 * pca_init/pca_sweep.  The server is not thread-safe.
 * ------------------------------------------------------------------------------------ */
typedef struct pca_server pca_server; /* opaque, library-owned */

/* hbm_budget_bytes: device memory the admitted requests may hold together; max_active:
 * 1..4096 concurrently admitted requests; sweeps_per_step >= 1: most sweeps one request
 * takes in one step; step_ms > 0: GPU time a step aims at.  Errors: PCA_EINVAL,
 * PCA_ENOMEM. */
int pca_server_create(uint64_t hbm_budget_bytes, int32_t max_active, int32_t sweeps_per_step, float step_ms,
                      pca_server **out);

/* Queues a request: parameters as for pca_init, the observation as a HOST float32
 * [height][width] array (copied), and the number of sweeps to run.  *request_id receives
 * a positive id.  Errors: PCA_EINVAL (invalid parameters, a footprint above the whole
 * budget, or accumulators that could overflow), PCA_EBUSY (refused by the shedding limit,
 * see pca_server_set_shedding), PCA_ENOMEM (the host copy could not be allocated; nothing
 * was queued). */
int pca_server_submit(pca_server *sv, const pca_params *params, const float *obs_host, int32_t sweeps,
                      int64_t *request_id);

/* Load shedding.  With max_backlog_s > 0, pca_server_submit refuses a request with
 * PCA_EBUSY when the remaining work of the requests already accepted (admitted or queued),
 * converted to seconds by the server's cost model (refined from every measured step), is
 * above max_backlog_s; an idle server accepts any request that fits the budget.  0 (the
 * default) disables shedding.  Errors: PCA_EINVAL (NULL server, negative limit). */
int pca_server_set_shedding(pca_server *sv, double max_backlog_s);

/* Number of submissions refused by the shedding limit so far. */
int pca_server_shed_count(const pca_server *sv, int64_t *shed);

/* One scheduling step on `stream` (synchronous: returns when the step's work is done,
 * also on an error).  *n_completed (may be NULL) receives the number of requests that
 * ended in this step, finished or failed.  The memory budget is the caller's estimate: if
 * a request's device allocation fails at admission while other requests hold device
 * memory, it waits at the head of the queue until they finish; if it fails with no other
 * request admitted, it ends as failed (PCA_ENOMEM).  A request whose results cannot be
 * copied to host memory also ends as failed.  The admitted requests advance either way.
 * Errors: PCA_EDEVICE, PCA_ENOMEM (host memory for the step's own bookkeeping). */
int pca_server_step(pca_server *sv, void *stream, int32_t *n_completed);

/* Ids of requests finished since the last call (at most `capacity`, oldest first). */
int pca_server_completed(pca_server *sv, int64_t *ids, int32_t capacity, int32_t *n);

/* status: 0 queued, 1 active, 2 finished, 3 failed (pca_server_result returns its error);
 * *sweep: sweeps done so far. */
int pca_server_status(const pca_server *sv, int64_t id, int32_t *status, int64_t *sweep);

/* Copies a finished request's posterior mean (float32 [H][W], value units), marginal mode
 * (uint8 [H][W]) and last states (uint8 [chains][H][W]) to host arrays; any may be NULL.
 * Errors: PCA_ESTATE if the request has not finished or the output does not exist; for a
 * failed request, the error that ended it (PCA_ENOMEM, PCA_EDEVICE). */
int pca_server_result(pca_server *sv, int64_t id, float *mean_host, uint8_t *mpm_host, uint8_t *state_host);

/* Forgets a finished or failed request and its host results. */
int pca_server_release(pca_server *sv, int64_t id);

/* Queue length, admitted requests, device bytes they hold, steps and sweeps launched. */
int pca_server_stats(const pca_server *sv, int32_t *queued, int32_t *active, uint64_t *used_bytes, int64_t *steps,
                     int64_t *sweeps_launched);

/* Waits for the last stream used and frees everything.  NULL is a no-op. */
int pca_server_destroy(pca_server *sv);

/* ------------------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  pca_run_static allocates nothing: it
 * runs a whole job - pca_init, pca_sweep(sweeps), then the read-outs - with the chain
 * states, the observation in level units and the accumulators in a fixed device array of
 * PCA_STATIC_SCRATCH_BYTES that the library holds on each device it runs on until the
 * process ends.  The results are bit-identical to that sequence of calls with the same
 * parameters.  Every call on a device shares that device's array (it keeps the last
 * call's contents; the accumulators are cleared by a kernel at the start of each call), so
 * calls that overlap on one device - on different streams or from different threads -
 * race and give undefined results.
 * ------------------------------------------------------------------------------------ */
#define PCA_STATIC_SCRATCH_BYTES ((uint64_t)256 << 20)

/* Enqueues the job on `stream` and returns (nothing is waited for).
 * params, obs_dev: as for pca_init (params->beta, if any, is read during this call only).
 * sweeps >= 0: sweeps to run from sweep index 0.
 * mean_out_dev: device float32 [height][width] for the posterior mean, or NULL.
 * mpm_out_dev: device uint8 [height][width] for the marginal mode, or NULL.
 * state_out_dev: device uint8 [chains][height][width] for the last states, or NULL.
 * Working memory, in bytes, each part rounded up to 256: 4*N (observation) + 2*N*Cp
 * (states; Cp = chains, or chains rounded up to a multiple of 4 when chains >= 3) + 4*N
 * (level sum) + 4*N*ceil(levels/2) when tally_stride > 0 (histogram), N = height*width.
 * Errors: PCA_EINVAL (bad parameters or pointers, no output requested, or working memory
 * above PCA_STATIC_SCRATCH_BYTES), PCA_ESTATE (a requested output that the run does not
 * produce: mean with no accumulated sweep, mode with the histogram disabled or never
 * tallied; or an accumulator that could overflow), PCA_EDEVICE. */
int pca_run_static(const pca_params *params, const float *obs_dev, int32_t sweeps, float *mean_out_dev,
                   uint8_t *mpm_out_dev, uint8_t *state_out_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif
