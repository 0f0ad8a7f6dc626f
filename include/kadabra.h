/*
 * kadabra.h -- C ABI of the MI355X (gfx950) KADABRA adaptive-sampling
 * betweenness-centrality library.
 *
 * Method (van der Grinten, Angriman, Meyerhenke, "Parallel Adaptive Sampling
 * with almost no Synchronization"):
 *   - Algorithm 1: draw samples, aggregate them with an associative operator,
 *     and check a stopping condition on a consistent state only;
 *   - Section 2.3: a KADABRA sample is a uniformly random vertex pair (s, t)
 *     and a uniformly random shortest s-t path; b~(v) = (1/tau) * number of
 *     sampled paths with v as an interior vertex; sampling stops once
 *     f, g <= eps for every vertex (Appendix B) or after omega samples;
 *   - Appendix C.1: same-component test; paths rebuilt from the graph and
 *     distance vectors; Appendix C.2: the check runs every N samples;
 *   - Appendix D (indexed frames): sample i draws its randomness from its
 *     index only, so the result does not depend on the parallel schedule.
 *
 * Determinism contract: the result (tau and every counter) is a pure function
 * of (graph, eps, delta, seed, check_interval).  No other parameter set with
 * kadabra_set_param changes it.
 *
 * Every int-returning call returns KADABRA_OK (0) or a negative status and
 * then sets a thread-local message readable with kadabra_last_error().
 * A handle must not be used by two threads at once; distinct handles may be.
 */
#ifndef KADABRA_H
#define KADABRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KADABRA_OK = 0,
    KADABRA_EINVAL = -1,    /* malformed argument or graph */
    KADABRA_ENOMEM = -2,    /* device or host allocation failed */
    KADABRA_EDEVICE = -3,   /* HIP runtime error or device-side invariant failure */
    KADABRA_ESTATE = -4,    /* no completed run to read */
    KADABRA_ERANGE = -5,    /* n, arc count, degree or omega beyond the supported limits */
    KADABRA_ECANCELED = -6  /* kadabra_cancel() stopped the run */
};

typedef struct kadabra_graph kadabra_graph; /* opaque: device CSR, run state, last result */

typedef struct {
    int64_t tau;           /* samples drawn (a check boundary, or omega) */
    int64_t omega;         /* maximal number of samples (Section 2.3) */
    int64_t vd_bound;      /* vertex-diameter bound used for omega */
    int64_t epochs;        /* check boundaries reached */
    int64_t decision;      /* 1: stopping rule met; 2: omega reached */
    /* algorithmic work, summed over the tau samples (independent of mapping) */
    int64_t v_exp;         /* frontier vertices expanded */
    int64_t e_scan;        /* sum of the expanded frontiers' degrees: traversed edges */
    int64_t e_bt;          /* sum of the degrees of the path vertices backtracked from */
    int64_t path_interior; /* counter increments */
    int64_t disconnected;  /* samples with s, t in different components */
    double log_inv_delta;  /* L = log(1/delta_L) = log(4 n / delta) */
    double ms_sampling;    /* device time from the first sampling launch to the last check */
    double ms_total;       /* host wall time of kadabra_run */
    double ms_sample_kernels; /* summed HIP-event durations of the sampling launches whose
                                 samples count (epochs 1 .. epochs) */
    int64_t sample_launches;  /* number of those launches (= epochs) */
    /* balanced runs ("balance" = 1); all zero otherwise */
    int64_t first_samples; /* first-phase samples drawn (not part of tau or the counters) */
    int64_t plan_tau;      /* planned sample count t* of the constants (0: no plan, uniform L) */
    int64_t first_v_exp;   /* work counters of the first phase, as above */
    int64_t first_e_scan;
    int64_t first_e_bt;
    int64_t first_path_interior;
    int64_t first_disconnected;
    /* new vertices the level expansions wrote (distance code, sigma, list
     * entry): every level in full, except that a meeting level expanded with
     * the meeting probe writes only the meeting set.  Unlike the counters
     * above it depends on the mapping ("probe_min"); it feeds the roofline's
     * byte model. */
    int64_t v_written;
} kadabra_stats;

/*
 * Copies an undirected graph, given as symmetric CSR in host memory, to
 * library-owned device memory and runs the preprocessing that depends on the
 * graph only: connected components and the vertex-diameter bound (Section
 * 2.3; Appendix C.1).
 *   n        number of vertices, 2 <= n < 2^23
 *   num_arcs number of arcs (twice the edge count), 0 <= num_arcs < 2^31
 *   row_ptr  host int32[n + 1]; row_ptr[0] = 0, non-decreasing, row_ptr[n] = num_arcs
 *   col_idx  host int32[num_arcs]; each row strictly ascending, entries in
 *            [0, n), no self-loops, and (u, v) present iff (v, u) present
 *   out      receives the handle (NULL on failure)
 * A graph whose vertex-diameter bound is 64 or more is stored on the device in
 * a cluster order (computed on the host: BFS-grown clusters of 128 vertices,
 * seeded in reverse Cuthill-McKee order, each split into BFS-grown clusters of
 * 32), which keeps the search balls of high-diameter graphs compact in memory;
 * every result and every output is still in, and tie-broken by, the given
 * vertex ids.
 * The caller keeps ownership of its arrays.  Errors: EINVAL (malformed CSR),
 * ERANGE (n or a degree >= 2^23), ENOMEM, EDEVICE.
 */
int kadabra_create_graph(int32_t n, int64_t num_arcs, const int32_t *row_ptr,
                         const int32_t *col_idx, kadabra_graph **out);

/* A consistent state of an adaptive run at a check boundary (Algorithm 1:
 * the counters of exactly samples [0, tau), every boundary so far decided
 * "continue"), from which kadabra_resume continues to the same result as an
 * uninterrupted run (sample i depends on i alone; Appendix D). */
typedef struct {
    int64_t n;              /* vertices: the length of the counters */
    int64_t tau;            /* samples in the counters: a check boundary below omega */
    int64_t epochs;         /* boundaries checked so far */
    int64_t omega;
    int64_t check_interval;
    double eps, delta;
    uint64_t seed;
    int64_t work[6];        /* v_exp, e_scan, e_bt, path_interior, disconnected, v_written so far */
} kadabra_checkpoint;

/*
 * Sets a run parameter; it applies to the next kadabra_run.
 *   "check_interval"  N >= 1: the stopping rule is checked after every N
 *                     samples (Appendix C.2).  Default 1024.  With
 *                     "balance" and "balance_samples", the only keys that
 *                     change results.
 *   "team"            0 (auto), 64 (one wavefront per sample), 128, 256 or
 *                     512 (two, four or eight wavefronts per sample).
 *                     Default 0.
 *   "slots"           samples in flight, 0 = auto (bounded by device memory).
 *   "frames"          counter frames F >= 1 the workgroups' increments are
 *                     spread over, merged at every boundary.  Default 1.
 *   "overlap"         1: launch the next epoch's samples before the host has
 *                     read the current check (discarded if it stops); 0: no.
 *   "epochs_per_launch" E in [1, 4]: one sampling launch carries E consecutive
 *                     check intervals; each boundary is still merged and
 *                     checked on exactly its own samples (the samples of later
 *                     intervals of a run that stops are discarded).  Default 2.
 *   "balance"         1: per-vertex delta_L(v), delta_U(v) (Section 2.3 bounds
 *                     only their sum) chosen from a first sampling phase, so
 *                     that vertices whose counters need more samples get a
 *                     larger share; 0 (default): uniform delta / (4 n).  The
 *                     first phase draws sample indices 2^63 + m, m < M1, none
 *                     of which the adaptive loop draws; its counts c1 give
 *                     planning values (c1 + 1) / M1, f and g of Appendix B
 *                     are inverted at a planned sample count t*, the smallest
 *                     (by bisection) at which the summed probabilities fit in
 *                     0.9 delta/2, and 0.1 delta/2 is spread evenly on top;
 *                     if none fits below omega the uniform constants stay.
 *                     t* and the constants are computed on the host from
 *                     the histogram of c1 (summed over its nonzero rows in
 *                     ascending count), with the C library's exp and log.
 *   "balance_samples" M1 >= 1 first-phase samples; 0 (default): ceil(omega/20).
 *   "probe_min"       k >= 0: expansions scanning at least k arcs first look
 *                     for the meeting set without materialising the new level;
 *                     -1 (default): when the product of the two frontiers'
 *                     degree sums reaches h times the arc count: h = 4 on
 *                     graphs whose vertex-diameter bound is 64 or more, else
 *                     h = E[d^2] / E[d]^2 inverted and kept in [1/8, 1].
 *   "probe_pull"      1: a meeting probe scans the rows of the other side's
 *                     frontier for neighbours on the expanding side's
 *                     frontier (pull form) instead of the expanding side's
 *                     rows (push form); the same meeting set and path counts
 *                     either way.  256-lane teams only (others push).
 *                     Default 0.
 *   "test_fail_alloc" k >= 1: the k-th device allocation of the next run's
 *                     buffers fails with ENOMEM (failure-path testing); 0: off.
 *   "stop_after_epochs" k >= 1: the run stops at the end of the first round
 *                     (one sampling launch and its checks) after k boundaries
 *                     of this run, if it has not stopped by itself, and
 *                     returns ECANCELED with a checkpoint readable by
 *                     kadabra_get_checkpoint; 0 (default): off.  Uniform
 *                     constants only ("balance" = 0).
 *   "test_level_cap"  k >= 3: the sampler is given room for only k BFS levels
 *                     per side, so samples needing more fail its level-bound
 *                     check and the run ends with EDEVICE (failure-path
 *                     testing of device-side checks); 0 (default): off.
 * Errors: EINVAL (unknown key or value out of range).
 */
int kadabra_set_param(kadabra_graph *g, const char *key, int64_t value);

/* Reads a parameter set by kadabra_set_param (auto values read as 0), or one
 * of the graph's read-only values: "vd_bound" (the vertex-diameter bound),
 * "components", "max_degree", "relabeled" (1: stored in the internal vertex
 * order described at kadabra_create_graph, 0: in the given order), and the
 * mapping of the last run, "last_team" and "last_slots". */
int kadabra_get_param(const kadabra_graph *g, const char *key, int64_t *value);

/*
 * Selects the HIP stream (a hipStream_t passed as void*) all work of this
 * handle is issued on; NULL selects the library's own stream.  The stream
 * must outlive its use by the handle.
 */
int kadabra_set_stream(kadabra_graph *g, void *hip_stream);

/*
 * Runs adaptive sampling to completion (blocking): 0 < eps < 1 additive
 * error, 0 < delta < 1 failure probability, seed of the counter-based
 * generator.  omega = ceil(0.5/eps^2 (floor(log2(VD - 2)) + 1 + ln(2/delta)))
 * and uniform delta_L = delta_U = delta/(4n), or balanced per-vertex
 * constants with "balance" (the paper defers both to the original KADABRA
 * analysis).  Samples are drawn in epochs [B_{k-1}, B_k),
 * B_k = min(k N, omega); the stopping rule runs on the counters of exactly
 * samples [0, B_k).  A failed or canceled run leaves the handle usable and no
 * result readable.  Errors: EINVAL (eps, delta), ERANGE (omega >= 2^31),
 * ENOMEM, EDEVICE, ECANCELED.
 */
int kadabra_run(kadabra_graph *g, double eps, double delta, uint64_t seed);

/*
 * kadabra_run for callers that cannot allocate memory: code being captured
 * into a HIP graph, tight serving loops, and harnesses that forbid
 * allocation.  It calls no hipMalloc, hipFree, hipHostMalloc or other
 * allocating routine.  All run-time device state (sample slots, counter
 * frames, control block, claim counter and launch descriptor) lives in one
 * static device array of 256 MiB that the library holds on every GPU it runs
 * on until the process ends; the array's device address is looked up once per
 * device, on the first call there.
 *   g          a graph from kadabra_create_graph, with its device current
 *              (EINVAL otherwise); its "check_interval", "team", "slots" and
 *              "probe_min" apply, "balance" must be 0 (EINVAL otherwise)
 *   eps, delta, seed  as kadabra_run
 *   counts_dev caller-allocated device int32[n]; receives the counters of the
 *              tau samples, exactly those kadabra_run computes for the same
 *              (graph, eps, delta, seed, check_interval)
 *   stats      host kadabra_stats or NULL: tau, omega, vd_bound, epochs,
 *              decision, the work counters, log_inv_delta and ms_total
 * The run is blocking, one check interval per launch, on the handle's stream;
 * samples in flight are as many as fit in the array (at most "slots" if set,
 * else 1024).  The handle's last kadabra_run result is left as it is.
 * The array is shared by every call on one GPU and keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap on
 * one GPU race and must be serialised by the caller.
 * Errors: EINVAL (null pointer, eps, delta, balance, device), ERANGE (omega
 * >= 2^31, or the run state of one sample in flight, about 60 n bytes, does
 * not fit in the array: use kadabra_run), EDEVICE, ECANCELED.
 */
int kadabra_run_static(kadabra_graph *g, double eps, double delta, uint64_t seed, int32_t *counts_dev,
                       kadabra_stats *stats);

/*
 * The state of the last run when it stopped at a boundary ("stop_after_epochs",
 * or kadabra_cancel: both stop at the end of a round, whose boundaries were
 * all decided "continue"): *ck, and counts (host int32[n], or NULL) the
 * counters of samples [0, ck->tau), in the given vertex order.  The state may
 * be stored and handed to kadabra_resume on any handle of the same graph, in
 * this process or another.  Errors: ESTATE (the last run completed, failed
 * otherwise, or was balanced), EINVAL, EDEVICE.
 */
int kadabra_get_checkpoint(const kadabra_graph *g, kadabra_checkpoint *ck, int32_t *counts);

/*
 * Continues a run from a checkpoint to completion (blocking): the result
 * (tau, every counter, the decisions of every boundary, the work counters)
 * equals the uninterrupted kadabra_run(ck->eps, ck->delta, ck->seed) with
 * check interval ck->check_interval.  counts: host int32[n] as returned by
 * kadabra_get_checkpoint (read during the call only).  Mapping parameters of
 * g apply; "stop_after_epochs" may stop it again.  Errors: EINVAL (a
 * checkpoint that does not fit this graph: n, omega, tau not a boundary
 * before omega, counters out of range or not summing to the increments;
 * "balance" set), ENOMEM, EDEVICE, ECANCELED.
 */
int kadabra_resume(kadabra_graph *g, const kadabra_checkpoint *ck, const int32_t *counts);

/*
 * Reads the last completed run into caller-allocated host memory; any
 * pointer may be NULL.  scores: double[n], scores[v] = counts[v] / tau
 * (computed on the device); counts: int32[n]; stats: one kadabra_stats.
 * Errors: ESTATE (no completed run), EDEVICE.
 */
int kadabra_get_scores(const kadabra_graph *g, double *scores, int32_t *counts,
                       kadabra_stats *stats);

/*
 * As kadabra_get_scores, but writes device memory on the handle's stream
 * (scores: device double[n], counts: device int32[n], either may be NULL)
 * and returns without waiting for the copies.  Errors: ESTATE, EDEVICE.
 */
int kadabra_get_scores_device(const kadabra_graph *g, double *scores_dev, int32_t *counts_dev);

/*
 * Copies the per-boundary decisions of the last run (0: continue, 1: stop
 * rule met, 2: omega reached) into out[0 .. min(cap, epochs)); *count
 * receives the number of boundaries.  Errors: ESTATE.
 */
int kadabra_get_decisions(const kadabra_graph *g, int8_t *out, int64_t cap, int64_t *count);

/*
 * The per-vertex constants of the last completed run, into caller-allocated
 * host memory (any pointer may be NULL): log_inv_delta_L[v] =
 * log(1/delta_L(v)) and log_inv_delta_U[v] = log(1/delta_U(v)) (double[n]),
 * first_counts[v] = c1(v), the first-phase counter (int32[n]).  A run without
 * "balance" reads L = log(4 n / delta) and zero counts.  Errors: ESTATE (no
 * completed run), EDEVICE.
 */
int kadabra_get_balance(const kadabra_graph *g, double *log_inv_delta_L, double *log_inv_delta_U,
                        int32_t *first_counts);

/*
 * Evaluates the stopping-rule functions of Appendix B on the device for
 * host arrays: f[v], g[v] for b = counts[v] / tau, omega, L = log(1/delta_L),
 * with the same expression tree and rounding as the stop check inside
 * kadabra_run (IEEE double, no contraction).  counts: host int32[n];
 * f, g: host double[n].  Uses the current HIP device; allocates and frees
 * temporary device memory.  Errors: EINVAL (n < 1, tau < 1, null pointer),
 * ENOMEM, EDEVICE.
 */
int kadabra_eval_stop_fg(int32_t n, const int32_t *counts, int64_t tau, int64_t omega, double L,
                         double *f, double *g);

/*
 * Autotuner.  Times a fixed set of mapping candidates (one, two or four
 * wavefronts per sample, the number of samples in flight, the meeting probe
 * on or off), then the epochs per launch (1, 2, 4) for the best of them, on
 * the first trial_samples samples of this graph's query (eps, delta; a fixed
 * calibration seed; no stop checks) and keeps the fastest in the handle's
 * parameters ("team", "slots", "probe_min", "epochs_per_launch").  Results
 * never depend on these parameters.  Errors: EINVAL, ERANGE, ENOMEM, EDEVICE.
 */
int kadabra_autotune(kadabra_graph *g, double eps, double delta, int64_t trial_samples);

/* ------------------------------------------------------------------------ */
/* Batches: many queries, on any number of graphs, run in shared launches:   */
/* every sampling launch carries the current epoch of every active query and */
/* one merge-and-check launch handles all their boundaries.  Each query's    */
/* result is exactly the one kadabra_run gives for it alone.                 */
/* ------------------------------------------------------------------------ */
typedef struct kadabra_batch kadabra_batch;

/* Creates an empty batch on the current device.  Errors: ENOMEM, EDEVICE. */
int kadabra_batch_create(kadabra_batch **out);

/* As kadabra_set_param for the batch ("team", "slots", "frames", "overlap",
 * "epochs_per_launch", "probe_min", "balance", "balance_samples" and the test
 * hooks); each applies to every query at the next kadabra_batch_run.
 * "check_interval" is per query. */
int kadabra_batch_set_param(kadabra_batch *b, const char *key, int64_t value);
int kadabra_batch_get_param(const kadabra_batch *b, const char *key, int64_t *value);
int kadabra_batch_set_stream(kadabra_batch *b, void *hip_stream);

/*
 * Adds a query (graph g, eps, delta, seed, check interval N) and returns its
 * index.  g must stay alive until the batch is cleared or destroyed.
 * Errors: EINVAL (parameters), ERANGE (omega >= 2^31).
 */
int kadabra_batch_add(kadabra_batch *b, const kadabra_graph *g, double eps, double delta,
                      uint64_t seed, int64_t check_interval, int32_t *index);

/* Runs every query of the batch to completion (blocking).  Errors: ESTATE
 * (empty batch), ENOMEM, EDEVICE. */
int kadabra_batch_run(kadabra_batch *b);

/* Autotuner for the batch's mapping, as kadabra_autotune. */
int kadabra_batch_autotune(kadabra_batch *b, int64_t trial_samples);

/* Reads query `index` of the last completed batch run (as kadabra_get_scores).
 * Errors: EINVAL (index), ESTATE. */
int kadabra_batch_get_scores(const kadabra_batch *b, int32_t index, double *scores,
                             int32_t *counts, kadabra_stats *stats);

/* Drops all queries (the device pool is kept for the next ones). */
int kadabra_batch_clear(kadabra_batch *b);
void kadabra_batch_destroy(kadabra_batch *b);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching.  A server owns a worker thread and one      */
/* device engine over a fixed set of resident graphs.  Queries are submitted */
/* at any time from any thread; at every round boundary (one sampling launch */
/* plus one merge-and-check launch) the worker admits waiting queries, in    */
/* submission order, while their device memory fits the server's budget,    */
/* and they join the next sampling launch beside the queries in flight; a    */
/* query leaves as soon as its own stopping rule fires.  Each query's result */
/* is exactly the one kadabra_run gives for it alone (Algorithm 1 with the   */
/* checks of Appendix C.2 depends on the query only, never on its company).  */
/* ------------------------------------------------------------------------ */
typedef struct kadabra_server kadabra_server;

typedef struct {
    int64_t submitted;     /* queries accepted by kadabra_server_submit */
    int64_t completed;     /* finished (stop rule, omega, or error) */
    int64_t failed;        /* of which ended with an error */
    int64_t active;        /* admitted and sampling */
    int64_t pending;       /* waiting for admission */
    int64_t bytes_in_use;  /* device bytes held by admitted or unreleased queries */
    int64_t budget_bytes;  /* admission budget */
    int64_t peak_active;   /* most queries in one launch so far */
    double p50_ms;         /* latency (submit to result final) percentiles over */
    double p99_ms;         /* completed queries since creation or the last reset */
    double max_ms;
    double mean_queue_ms;  /* mean time from submit to admission */
} kadabra_server_info;

/*
 * Creates a server over graphs[0 .. ngraphs) (handles from
 * kadabra_create_graph; they must outlive the server and not be destroyed
 * meanwhile; their own runs stay independent).  hbm_budget_bytes bounds the
 * device memory of admitted queries (per query: counters 4n, score buffer
 * 8n, and while sampling the frame sets 8n * frames * epochs_per_launch
 * bytes, plus with "balance" the first-phase counters 4n and the plan tables
 * 20 (M1 + 1) bytes); 0 takes half of the device memory free after the
 * sample pool is sized.  max_active bounds the queries in one launch (0: 256).
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
int kadabra_server_create(const kadabra_graph *const *graphs, int32_t ngraphs, int64_t hbm_budget_bytes,
                          int32_t max_active, kadabra_server **out);

/* Mapping parameters as kadabra_batch_set_param, and "round_us": the round
 * work cap in microseconds (default 16000; 0: none).  Waiting queries are
 * admitted, in submission order, only while the estimated device time of the
 * first sampling launches of the admitted, unfinished queries stays within
 * the cap; a query is always admitted when none runs.  A long query then
 * shares its launches only with queries submitted before it, and short ones
 * are batched in short rounds.  The estimates come from one calibration
 * launch per graph (2048 samples, timed) on the first submission; they never
 * change a result.  Only before the first submit (ESTATE after).  get_param
 * also reads "graphs", "max_active", "budget". */
int kadabra_server_set_param(kadabra_server *s, const char *key, int64_t value);
int kadabra_server_get_param(const kadabra_server *s, const char *key, int64_t *value);

/*
 * Enqueues a query on graph `graph_index` and returns its ticket (> 0) at
 * once.  Errors: EINVAL (index or parameters), ERANGE (omega >= 2^31, or the
 * query alone exceeds the budget), EDEVICE (the worker hit a device error).
 */
int kadabra_server_submit(kadabra_server *s, int32_t graph_index, double eps, double delta, uint64_t seed,
                          int64_t check_interval, int64_t *ticket);

/* Blocks until the ticket's query is final or timeout_s seconds pass
 * (timeout_s < 0: no limit); *done = 1 if final.  Errors: EINVAL (unknown
 * ticket, or released by another thread while waiting). */
int kadabra_server_wait(kadabra_server *s, int64_t ticket, double timeout_s, int32_t *done);

/*
 * Reads a final query's scores (float64[n], counts / tau, computed on the
 * device) and/or counters (int32[n]) into host buffers, its statistics (with
 * ms_total = its latency from submit to final), and its latency.  Any
 * pointer may be NULL.  Returns the query's own error if it failed.
 * Errors: EINVAL (ticket), ESTATE (not final yet), the query's error.
 */
int kadabra_server_result(kadabra_server *s, int64_t ticket, double *scores, int32_t *counts,
                          kadabra_stats *stats, double *latency_ms);

/* Returns a final query's device memory to the server (the ticket becomes
 * invalid).  Results of one ticket may be read from several threads at once;
 * a release while a read is in progress is refused.  Errors: EINVAL (ticket),
 * ESTATE (not final yet, or a result read in progress). */
int kadabra_server_release(kadabra_server *s, int64_t ticket);

/* Counters and latency percentiles; reset = 1 restarts the latency window. */
int kadabra_server_info_get(kadabra_server *s, kadabra_server_info *info, int32_t reset);

/* Cancels waiting and running queries (ECANCELED), stops the worker, frees
 * everything (NULL is a no-op). */
void kadabra_server_destroy(kadabra_server *s);

/* Asks a run in progress on another thread (its setup included) to stop at
 * its next boundary (kadabra_run then returns ECANCELED).  Each kadabra_run or
 * kadabra_autotune clears earlier requests when it starts.  Safe to call
 * concurrently. */
int kadabra_cancel(kadabra_graph *g);

/* Frees the handle and its device memory (NULL is a no-op). */
void kadabra_destroy_graph(kadabra_graph *g);

/* Text of the last error raised on the calling thread ("" if none). */
const char *kadabra_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int kadabra_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KADABRA_H */
