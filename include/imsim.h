/*
 * imsim: Monte Carlo simulation of the independent cascade (IC) and linear
 * threshold (LT) diffusion models on one gfx950 GPU, behind a C ABI.
 *
 * The operation (paper Section 2, "Diffusion Models" and "Influence
 * Maximization"): given a directed graph G = (V, E) in CSR form (Section 3,
 * "Data Structures"), a per-arc parameter (IC activation probability p_uv, or
 * LT influence weight w_uv with sum_u w_uv <= 1 for every v), a seed set S and
 * a number of trials T, run T independent diffusions from S and report, per
 * trial, the number of nodes active at the end (seeds included), and per node
 * the number of trials in which it ended active.  sigma(S) = total / T.
 *
 * Randomness is a pure function of (rng_seed, trial, arc or node):
 *   H(seed, dom, t, id) = 32-bit half (t & 1) of word ((t & 7) >> 1) of
 *   Philox4x64-10(counter = (id, t >> 3, 0, 0), key = (seed, dom))
 *   (Salmon et al., SC'11).  dom = 1: IC coin of out-CSR arc id;
 *   dom = 2: LT threshold hash of node id.
 *   IC: arc e is live in trial t  iff  thr_e == 0xFFFFFFFF or H(seed,1,t,e) < thr_e.
 *   LT: v joins in trial t        iff  (active in-weight, 2^-32 units) > H(seed,2,t,v).
 * Every trial's final active set is therefore fixed by the inputs; the
 * library computes it exactly, independent of schedule and launch shape.
 *
 * Conventions
 *   - Functions return 0 (IMS_OK) or a negative IMS_E_* code; the message of
 *     the last failure on the calling thread is ims_last_error().  No C++
 *     exception crosses this boundary.  On failure, outputs are unspecified.
 *   - "host" pointers are read during the call only.  "device" pointers are
 *     caller-owned HBM (e.g. torch tensors); the library never frees or keeps
 *     them past the call.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = the null stream)
 *     and returns before it finishes, unless stated otherwise.
 *   - A graph handle owns its device copy of the graph and a workspace that
 *     grows on demand; calls on one handle must not overlap in time.
 *   - Trial t lives in word t / 64, bit t % 64.  Bit-masks are word-major:
 *     mask[w * n + v].  Bits of trials >= T are zero in every output.
 */
#ifndef IMSIM_H
#define IMSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IMS_OK = 0,
    IMS_E_INVALID_ARG = -1,   /* null pointer, T == 0, bad model, bad p or w */
    IMS_E_INVALID_GRAPH = -2, /* offsets not monotone, offsets[0] != 0, index >= n, n or m too large */
    IMS_E_WEIGHT_SUM = -3,    /* LT: sum of in-weights of a node above 2^32 (i.e. above 1) */
    IMS_E_SEED_RANGE = -4,    /* a seed id >= n */
    IMS_E_OOM = -5,           /* device allocation failed */
    IMS_E_HIP = -6,           /* a HIP runtime call failed */
    IMS_E_LEVEL_CAP = -7,     /* a run needed more steps than the graph allows (internal bug guard) */
    IMS_E_UNSUPPORTED = -8    /* valid request outside the library's limits */
};

enum { IMS_MODEL_IC = 0, IMS_MODEL_LT = 1 };

typedef struct ims_graph ims_graph;

/* Thread-local text of the last failure ("" if none). */
const char* ims_last_error(void);
const char* ims_version(void);

/* Parameter encoding (host arrays of length m).
 * IC (Section 2: arc (u,v) succeeds with probability p_uv):
 *   thr = min(floor(p * 2^32), 2^32 - 1), and thr == 2^32 - 1 means "always";
 *   p must lie in [0, 1] (NaN rejected).
 * LT (Section 2: in-weights with sum at most 1):
 *   w = floor(w_real * 2^32) as uint64; w_real must lie in [0, 1]. */
int ims_encode_p(const double* p, int64_t m, uint32_t* thr);
int ims_encode_w(const double* w, int64_t m, uint64_t* w64);

/* Host-side CSR check (Section 3, "Data Structures": out-neighbours of u are
 * indices[offsets[u] .. offsets[u+1])): offsets[0] == 0, non-decreasing,
 * offsets[n] == m, every index < n.  Needs no GPU. */
int ims_validate_csr(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices);

/* Build a graph plan on the current device from host arrays.
 *   offsets  host int64[n+1], indices host uint32[m]   (out-CSR; self-loops and
 *            repeated arcs are allowed: a self-loop never fires, repeated IC arcs
 *            draw independent coins, repeated LT arcs add their weights)
 *   model    IMS_MODEL_IC: param = host uint32 thr[m] (see ims_encode_p)
 *            IMS_MODEL_LT: param = host uint64 w[m]   (see ims_encode_w);
 *            every node's in-weights must sum to at most 2^32.
 * Parameters are in out-CSR order: the arc id of indices[e] is e.  Limits:
 * n < 2^32, m < 2^32.  Synchronous; copies everything it needs. */
int ims_graph_create(int64_t n, int64_t m, const int64_t* offsets, const uint32_t* indices,
                     int model, const void* param, ims_graph** out);
int ims_graph_destroy(ims_graph* g);
int ims_graph_info(const ims_graph* g, int64_t* n, int64_t* m, int* model);

/* Simulation options; NULL = automatic.  Any setting gives the same bits. */
typedef struct ims_opts {
    int shape;             /* 0 = auto (IC: word-local when the run has at least a quarter as
                              many 64-trial words as compute units, else grid-wide; LT: grid-
                              wide), 1 = word-local (a workgroup runs the whole cascade of its
                              trials: of one 64-trial word when active_bits is requested, else of
                              16 trials on persistent slots that add their own counts), 2 = grid-
                              wide steps (one launch per level / sweep) */
    int32_t blocks_per_cu; /* workgroups per compute unit; 0 = auto */
    double alpha;          /* LT grid shape: a sweep marks out-neighbours of joining nodes (and the
                              next sweep evaluates marked nodes only) when the previous sweep
                              changed fewer than alpha * W * n (node, word) pairs; 0 = 1/64 */
    int32_t profile;       /* nonzero: time the simulation kernels with HIP events (see ims_graph_profile) */
    int32_t test_flags;    /* test hooks, 0 in normal use: bit 0 = LT grid shape without a
                              threshold table (hashes drawn in the kernel); bit 1 = unused;
                              bit 2 = LT without the equal-in-weights form; bit 3 = LT grid
                              shape with full threshold hashes instead of count thresholds */
    /* IC direction (Section 3, "Algorithms", expands the out-arcs of the last
       step's new nodes: the push side).  The pull side instead lets every
       (node, word) pair with an inactive trial scan its in-arcs for frontier
       sources, drawing each arc's coin by its out-CSR id, and stop when its
       pending trials have all joined.  Per level, by Beamer's rule over the
       pairs of all words (word-local tasks: over the task's own nodes):
       push -> pull when the frontier's out-arcs times ic_alpha * pbar exceed
       the in-arcs of pairs with an inactive trial, where pbar is the mean
       firing probability of the graph's arcs (a pulled node stops early only
       as often as its arcs fire); pull -> push when the frontier's pairs
       times ic_beta fall below W * n (word-local: below n). */
    double ic_alpha;       /* 0 = 14 on the grid shape, 2 on the word-local shape and for seed sets;
                              with 0 and ic_direction 0, word-local runs on graphs whose mean arc
                              probability is below 0.25 push only */
    double ic_beta;        /* 0 = 24 */
    int32_t ic_direction;  /* 0 = by the rule, 1 = push only, 2 = pull only */
} ims_opts;

/* Run trials 0 .. n_trials-1 from one seed set (Section 2).
 *   seeds         host uint32[n_seeds]; duplicates allowed (set semantics),
 *                 every id must be < n; n_seeds may be 0.
 *   n_trials      T >= 1, T <= 2^18.
 *   trial_counts  device uint32[T]: |A_t|, seeds included.          required
 *   node_counts   device uint32[n]: #{t : v in A_t}.                 optional (NULL)
 *   total         device uint64[1]: sum_t |A_t|; sigma = total / T.  required
 *   active_bits   device uint64[ceil(T/64) * n], word-major.         optional (NULL)
 * Asynchronous on `stream` in the word-local shape; the grid shape reads one
 * step counter back per batch of steps and so returns once its last step has
 * run (the final pass and the status words are still in flight then). */
int ims_simulate(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials,
                 uint64_t rng_seed, const ims_opts* opts, uint32_t* trial_counts,
                 uint32_t* node_counts, uint64_t* total, uint64_t* active_bits, void* stream);

/* The simulation of ims_simulate plus, per trial, the number of nodes first
 * activated at each level (paper Section 4, "Visualizations": the mean number
 * of active nodes over time).  Level 0 holds the seeds; level l the nodes the
 * synchronous step l of Section 2 activates: for IC the nodes whose shortest
 * live-arc path from the seed set has l arcs, for LT the nodes whose active
 * in-weight after step l - 1 first exceeds their threshold (LT runs
 * synchronous steps here, not the in-place sweeps of ims_simulate; the final
 * state is the same).
 *   max_levels    >= 1; levels >= max_levels are not counted.
 *   level_counts  device uint32[max_levels * n_trials]: level_counts[l * T + t].
 *   trial_counts, total as ims_simulate.
 * Runs the word-local shape.  ims_graph_last_status() then gives the number
 * of levels processed: the deepest nonempty level is at most that number, so
 * a caller that sees it >= max_levels can retry with a larger buffer. */
int ims_simulate_levels(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                        uint32_t max_levels, uint32_t* level_counts, uint32_t* trial_counts, uint64_t* total,
                        void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run of
 * ims_simulate in its count-only word-local form (each 64-trial word as four
 * 16-trial tasks on persistent workgroup slots), with every per-call device
 * buffer (slot state, seed list, task counter) taken from one fixed device
 * array of IMS_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its
 * first use on that GPU until the process ends.  It calls no allocator.
 *   Arguments as ims_simulate (host seeds, duplicates allowed, ids < n;
 *   device outputs trial_counts uint32[T] and total uint64[1] required,
 *   node_counts uint32[n] optional); results are identical to ims_simulate's.
 *   The graph must live on the current device.
 *   Limit: the array must hold about 1 KiB + 8 B per seed + 4 B per node plus
 *   one workgroup slot of 48 B per node (so about 1.39M nodes at most);
 *   larger requests fail with IMS_E_UNSUPPORTED.  Smaller graphs get more
 *   slots (up to two per compute unit), so throughput drops only for large n.
 *   Every call on one GPU shares that GPU's array and clears what it needs at
 *   its start: calls that overlap in time on one GPU (other streams, other
 *   threads) race and give wrong results.  Asynchronous on `stream`; the
 *   seeds travel as kernel arguments, so they are read during the call only.
 *   ims_graph_last_status reports the run's steps and step guard as usual. */
#define IMS_NOALLOC_SCRATCH_BYTES (64u << 20)
int ims_simulate_noalloc(ims_graph* g, const uint32_t* seeds, uint32_t n_seeds, uint32_t n_trials, uint64_t rng_seed,
                         uint32_t* trial_counts, uint32_t* node_counts, uint64_t* total, void* stream);

/* Many seed sets on one graph with common random numbers (every set sees the
 * same coins / thresholds: same rng_seed and trials 0 .. n_trials-1), as the
 * greedy and CELF influence maximisation of Section 2 evaluate sigma(S + v)
 * for many v.
 *   set_offsets  host uint32[n_sets+1]: set i is set_nodes[set_offsets[i] ..
 *                set_offsets[i+1]); set_offsets[0] == 0, non-decreasing.
 *   set_nodes    host uint32[set_offsets[n_sets]]; duplicates within a set are
 *                ignored; ids must be < n.  Empty sets are allowed.
 *   totals       device uint64[n_sets]: sum over trials of |A_t(set)|;
 *                sigma(set) = totals[i] / n_trials.              required
 *   node_counts  device uint32[n_sets * n]: per set, trials in which each
 *                node ended active.                               optional (NULL)
 * Every set's results equal those of ims_simulate on that set.  Asynchronous
 * on `stream`. */
int ims_simulate_sets(ims_graph* g, const uint32_t* set_offsets, const uint32_t* set_nodes, uint32_t n_sets,
                      uint32_t n_trials, uint64_t rng_seed, const ims_opts* opts, uint64_t* totals,
                      uint32_t* node_counts, void* stream);

/* Marginal spreads from a stored state (greedy's sigma(S + v) - sigma(S),
 * Section 2, "Influence Maximization").  base_bits (device uint64[W * n],
 * word-major) is the active_bits output of ims_simulate for a seed set S with
 * the same n_trials and rng_seed.  Each set X is simulated from A_t(S) with
 * X added: IC continues the cascade over the same live arcs, LT the same
 * thresholds, so the final set is exactly A_t(S + X) (IC: reachability over
 * live arcs; LT: least fixpoint above A_t(S) + X, which is A_t(S + X) since
 * A_t(S) lies below it).  Outputs count new activations only:
 *   totals       device uint64[n_sets]: sum over trials of |A_t(S + X) \ A_t(S)|,
 *                so sigma(S + X) = (total(S) + totals[i]) / n_trials.
 *   node_counts  device uint32[n_sets * n] (optional): trials in which each
 *                node is active for S + X but not for S.
 * Other arguments, errors and asynchrony as ims_simulate_sets; base_bits
 * must stay unchanged until the call's work is done.  Results are exact only
 * when base_bits comes from the same graph, n_trials and rng_seed. */
int ims_simulate_sets_from(ims_graph* g, const uint64_t* base_bits, const uint32_t* set_offsets,
                           const uint32_t* set_nodes, uint32_t n_sets, uint32_t n_trials, uint64_t rng_seed,
                           const ims_opts* opts, uint64_t* totals, uint32_t* node_counts, void* stream);

/* Batch: several (graph, seeds, trials, rng_seed) runs, IC and LT mixed,
 * executed by one persistent launch that takes (item, 64-trial word, trial
 * part) tasks in a scheduled order, captured once in a HIP graph and
 * replayed.  Each item's outputs equal those of ims_simulate on that item
 * alone. */
typedef struct ims_batch ims_batch;

typedef struct ims_batch_item {
    ims_graph* graph;        /* not owned; must outlive the batch */
    const uint32_t* seeds;   /* host; copied at creation */
    uint32_t n_seeds;
    uint32_t n_trials;       /* 1 .. 2^18 */
    uint64_t rng_seed;
    uint32_t* trial_counts;  /* device uint32[n_trials], required */
    uint32_t* node_counts;   /* device uint32[n] or NULL */
    uint64_t* total;         /* device uint64[1], required */
} ims_batch_item;

typedef struct ims_tuning {
    int32_t blocks_per_cu;  /* persistent workgroups per compute unit (1..16) */
    int32_t order;          /* 0 = items by estimated cost, largest first; 1 = item order */
    int32_t split;          /* tasks per 64-trial word, 1 .. 64 (rounded down to a power of two;
                               values below 1 mean 1); each task takes 64 / split of the word's
                               trials and runs their cascade alone, so a split shortens the
                               longest task at the cost of more, smaller tasks; results do not
                               change */
    double ic_alpha;        /* IC tasks' push -> pull switch point (ims_opts.ic_alpha), 0 = 14 */
    double ic_beta;         /* IC tasks' pull -> push switch point (ims_opts.ic_beta), 0 = 24 */
} ims_tuning;

/* tuning NULL = defaults (2 per CU, largest first, 8 tasks per word, default
 * switch points).  Synchronous. */
int ims_batch_create(const ims_batch_item* items, uint32_t n_items, const ims_tuning* tuning, ims_batch** out);
/* Time candidate schedules `repeats` times each on `stream`: first
 * (workgroups per compute unit, order, split) at the default switch points,
 * then the IC push / pull switch points (alpha; a tiny alpha keeps every task
 * on the push side) for the fastest of those.  Check that every candidate
 * gives identical outputs (every item's trial counts, node counts and total;
 * IMS_E_HIP otherwise), keep the fastest (reported in *chosen if not NULL)
 * and drop the captured graph.  Synchronous. */
int ims_batch_autotune(ims_batch* b, int repeats, void* stream, ims_tuning* chosen);
/* Run the batch on `stream`: the first call (and the first after a tuning
 * change) captures the launch sequence into a HIP graph, later calls replay
 * it.  Asynchronous. */
int ims_batch_launch(ims_batch* b, void* stream);
int ims_batch_destroy(ims_batch* b);

/* Per-task timeline of batch launches (inspection hook for profiles):
 * ims_batch_task_timing(b, 1) makes every later launch record, for each task,
 * the device wall clock (a constant-rate counter, 100 MHz on this device
 * family) at its start and end and the workgroup slot that ran it; 0 turns
 * it off.  Either call drops the captured HIP graph.  ims_batch_task_times
 * waits for `stream` and copies, for the tasks of the last launch in the
 * order they are listed, their codes (item << 32 | log2 trials-per-task
 * split << 24 | part << 16 | word) into tasks (host uint64[max_tasks]) and
 * (start, end, slot) into times (host uint64[3 * max_tasks]); *count =
 * tasks written.  IMS_E_INVALID_ARG while timing is off. */
int ims_batch_task_timing(ims_batch* b, int enable);
int ims_batch_task_times(ims_batch* b, uint32_t max_tasks, uint64_t* tasks, uint64_t* times, uint32_t* count,
                         void* stream);

/* Status of the last run on this handle: out[0] = steps (IC frontier levels
 * or LT sweeps) taken, out[1] = nonzero if the step guard fired.  Waits for
 * `stream`. */
int ims_graph_last_status(ims_graph* g, void* stream, uint32_t out[2]);

/* All four status words of the last run on this handle: out[0], out[1] as
 * ims_graph_last_status; out[2] = tasks taken (word-local forms); out[3] =
 * times a word-local step found its 64 workgroup-wide walks of nodes with
 * more than 512 out-arcs taken and had a wavefront walk one more alone.
 * Waits for `stream`.  Inspection hook for tests. */
int ims_graph_last_counters(ims_graph* g, void* stream, uint32_t out[4]);

/* Directions taken by the last IC run of the grid shape on this handle, one
 * per expanded level: dirs[l] = 1 (push) or 2 (pull), for at most max_levels
 * levels (host array); *count = levels written (0 after any other kind of
 * run).  Waits for `stream`.  Inspection hook for tests and profiles. */
int ims_graph_level_directions(ims_graph* g, uint32_t max_levels, uint32_t* dirs, uint32_t* count, void* stream);

/* Kernel timing of runs made with opts->profile set: waits for the last such
 * run, then returns the summed duration (ms) of the simulation kernel over the
 * runs recorded since the last reset (at most 256) and their count; reset != 0
 * clears the record afterwards. */
int ims_graph_profile(ims_graph* g, int reset, double* total_ms, uint32_t* count);

/* Test hook: out[i] = H(rng_seed, domain, trials[i], ids[i]) for i < count,
 * computed by the device hash.  Device arrays. */
int ims_debug_hash(uint64_t rng_seed, uint64_t domain, const uint64_t* trials, const uint64_t* ids,
                   uint32_t* out, int64_t count, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* IMSIM_H */
