/*
 * kadabra.h -- C ABI of the MI355X sampled-betweenness library.
 *
 * The library approximates the normalised betweenness centrality
 *     bc(v) = 1/(n(n-1)) * sum over ordered pairs s != t, v not in {s,t}, of sigma_st(v)/sigma_st
 * (paper section 2, "Algorithm Overview") with the adaptive sampling algorithm of
 * Borassi & Natale (Algorithm 1): random pairs (s,t), one uniformly random shortest
 * s-t path per pair found by a balanced bidirectional BFS (section 4), hits on the
 * path's interior nodes, and a stopping rule built on the bounds f and g of
 * Theorem azuma-borassi with per-node failure probabilities chosen by computeDelta
 * (Algorithm 2).  Two tasks are offered: every centrality within +-epsilon
 * (section 2) and the top-k ranking (section 5, Algorithm 3).
 *
 * Conventions for every call:
 *   - All calls return a kad_status (0 = success, negative = error); none aborts.
 *     kad_last_error() gives a thread-local description of the last failure.
 *   - Pointers marked "host" are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the context's GPU.  The caller owns every buffer it passes;
 *     the library never frees them.
 *   - Results depend only on the graph and the parameters (kernel_batch excluded):
 *     all randomness is a counter-based Philox4x64-10 stream keyed by (seed,
 *     phase, sample id), so the output is identical for any launch shape.
 *   - hip_stream may be NULL (the library's own stream) or a hipStream_t of the
 *     context's device; calls are synchronous with respect to the host.
 */
#ifndef KADABRA_H
#define KADABRA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KAD_OK = 0,
  KAD_EINVAL = -1,    /* bad argument or malformed graph */
  KAD_ENOMEM = -2,    /* host or device allocation failed, or over the HBM budget */
  KAD_EDEVICE = -3,   /* HIP runtime error, or no usable GPU */
  KAD_EBUSY = -4,     /* the context is in use, or a served query is still running */
  KAD_ETOOSMALL = -5, /* an output buffer is too small; the needed size is reported */
  KAD_EOVERFLOW = -6, /* a result does not fit the library's fixed-width arithmetic */
  KAD_ERNG = -7,      /* a bounded random draw was rejected 64 times (probability < 2^-64) */
  KAD_ECANCELED = -8, /* a served query was dropped before it started */
  KAD_EINTERNAL = -9  /* an unexpected host-side failure (the message says what) */
} kad_status;
/* No C++ exception leaves the library: every call that returns a kad_status turns one
 * into a status (host memory or threads exhausted: KAD_ENOMEM, anything else:
 * KAD_EINTERNAL) with a message from kad_last_error(). */

enum { KAD_MEM_HOST = 0, KAD_MEM_DEVICE = 1 };
enum { KAD_ALL_NODES = 0, KAD_TOPK = 1 };
/* what the betweenness is estimated for (kad_params.target): the nodes, or the edges
 * (section 1: the method adapts to the centrality of edges; a sampled path hits every edge
 * on it, and bc(e) = 1/(n(n-1)) sum over ordered pairs s != t of sigma_st(e)/sigma_st) */
enum { KAD_TARGET_NODES = 0, KAD_TARGET_EDGES = 1 };
enum { KAD_STOP_OMEGA = 0, KAD_STOP_RULE = 1, KAD_STOP_FIXED = 2 };
/* sample schedules (kad_params.schedule) */
enum {
  KAD_SCHEDULE_ADAPTIVE = 0,  /* Algorithm 1: pilot, computeDelta, stopping rule (KADABRA) */
  KAD_SCHEDULE_RK = 1,        /* fixed c/eps^2 (floor(log2(VD-2)) + 1 + ln(1/delta)) samples
                                 (the Riondato-Kornaropoulos bound of section 6) */
  KAD_SCHEDULE_HOEFFDING = 2  /* fixed ln(2n/delta) / (2 eps^2) samples (Hoeffding's inequality
                                 with a union bound over the nodes, section 2) */
};

/* how kad_run launches its work (kad_ctx_set_exec); every mode gives the same result */
enum {
  KAD_EXEC_GRAPH = 0,  /* main-phase batches replay recorded hipGraphs: the sampling chain
                          (sampler, wide-count fix, edge rewrite, host mirrors) and, in
                          all-nodes runs, the batched reduction of the check intervals; the
                          batch's sample range is read from a device descriptor, so one
                          recording serves every batch of up to kernel_batch samples */
  KAD_EXEC_STREAM = 1, /* the same chains launched call by call on the context's streams */
  KAD_EXEC_PLAIN = 2   /* the plain single-graph path, kept as the baseline: no batching of
                          check intervals, no persistent workgroups (one sample per
                          workgroup, one launch per resident grid of samples), no pilot
                          overlap and no recorded graphs; the host waits for every launch
                          and checks after every interval */
};

/* per-sample flag bits reported by kad_sample_paths */
enum {
  KAD_SAMPLE_OVERFLOW = 1u, /* a path count or the candidate-edge total reached 2^128 */
  KAD_SAMPLE_CAPACITY = 2u, /* the wide-count arena or level tables, or the path, outgrew
                               their buffers (samples that outgrow the 128-bit sampler's
                               candidate-edge buffer are sampled again and are not flagged) */
  KAD_SAMPLE_RNG = 4u       /* a bounded draw exhausted its attempts */
};

typedef struct kad_ctx kad_ctx;
typedef struct kad_graph kad_graph;

/* ---------------------------------------------------------------- context */

/* Open HIP device `hip_device`.  hbm_budget_bytes caps the library's device memory
 * (graphs + per-sample working state); 0 means 90% of the free memory at creation.
 * The working state is one slot per resident sampler workgroup, 36 bytes per node of the
 * largest graph run so far plus 512 KiB each, in at most 70% of the budget left after
 * the graphs (fewer slots than workgroups only lower throughput).
 * Fails with KAD_EDEVICE when the device does not exist. */
kad_status kad_ctx_create(int hip_device, uint64_t hbm_budget_bytes, kad_ctx **out);
kad_status kad_ctx_destroy(kad_ctx *ctx);

/* ---------------------------------------------------------------- graphs */

/* Register an unweighted graph in CSR form (paper section 2: G = (V,E), directed or
 * undirected; section 4 uses out-arcs forward from s and in-arcs backward from t).
 *   n        : number of nodes, 2 <= n < 2^32; nodes are 0..n-1.
 *   arcs     : number of CSR entries, < 2^32 (an undirected edge is two arcs).
 *   row_ptr  : uint32[n+1], row_ptr[0] = 0, row_ptr[n] = arcs, non-decreasing.
 *   col      : uint32[arcs]; row v lists the heads of v's out-arcs, strictly
 *              ascending (no duplicates), no self-loops.
 *   rrow_ptr, rcol : the in-rows (transpose) in the same form.  Ignored for an
 *              undirected graph (which must be symmetric).  For a directed graph
 *              NULL means "build the transpose"; if given it must be the exact
 *              transpose.
 *   mem      : KAD_MEM_HOST (the library copies the arrays to the device) or
 *              KAD_MEM_DEVICE (the arrays are device pointers that the library
 *              borrows; the caller keeps them alive and unchanged until
 *              kad_graph_destroy; the library also keeps a host copy for the
 *              host-side vertex-diameter pass).
 * Every property above is validated; violations return KAD_EINVAL. */
kad_status kad_graph_create(kad_ctx *ctx, uint32_t n, uint64_t arcs, int directed,
                            const uint32_t *row_ptr, const uint32_t *col,
                            const uint32_t *rrow_ptr, const uint32_t *rcol, int mem,
                            kad_graph **out);
kad_status kad_graph_destroy(kad_graph *g);

/* ---------------------------------------------------------------- the adaptive run */

typedef struct {
  double epsilon;          /* lambda of the paper, in (0,1) */
  double delta;            /* failure probability, in (0,1) */
  uint32_t mode;           /* KAD_ALL_NODES or KAD_TOPK */
  uint32_t k;              /* top-k: 1 <= k <= n */
  uint64_t seed;           /* Philox key word 0 */
  uint32_t check_interval; /* samples between stopping checks; 0 = 2^floor(log2(omega/16))
                              clamped to [1024, 65536].  Part of the result contract. */
  uint32_t kernel_batch;   /* samples per sampler launch (rounded up to a multiple of the
                              check interval); 0 = library choice.  Performance only. */
  uint32_t vd_override;    /* 0 = library vertex-diameter rule (exact when n*arcs <= 1e9,
                              else a strongly-connected-component bound) */
  uint32_t schedule;       /* KAD_SCHEDULE_*; the fixed schedules take no pilot and no
                              stopping check, and report [bc - eps, bc + eps] (kad_run only) */
  double c;                /* constant of the sample cap omega; 0 = 0.5 */
  double balance_eps;      /* epsilon of computeDelta (Algorithm 2); 0 = 0.001 */
  uint32_t target;         /* KAD_TARGET_NODES (0) or KAD_TARGET_EDGES: the items of the run.
                              With edges every per-item array has one entry per edge id
                              (kad_graph_edge_ids), k counts edges, the union bounds run over
                              the edges, and the cap omega uses floor(log2(max(VD-1,1))) + 1
                              in place of floor(log2(max(VD-2,1))) + 1 (a path has at most
                              VD - 1 edges).  kad_run only (the engine refuses it). */
} kad_params;

typedef struct {
  /* scalar outputs */
  uint64_t tau;            /* samples taken in the main phase */
  uint64_t omega;          /* cap: ceil(c/eps^2 (floor(log2(max(VD-2,1))) + 1 + ln(2/delta)));
                              fixed schedules: their sample count */
  uint64_t alpha;          /* pilot samples: max(1, floor(omega/100)); fixed schedules: 0 */
  uint64_t interval;       /* check interval used */
  uint64_t arcs_scanned;   /* arcs scanned by the main phase's level expansions */
  uint64_t pilot_arcs_scanned;
  uint64_t overflow_samples; /* samples sampled again by the wide-count kernel: their 128-bit
                                path counts overflowed, or they met through more candidate
                                edges than a sampler slot holds (kad_run: over every launch,
                                including samples past the stopping point; engine: 0) */
  uint32_t vd, vd_exact;   /* vertex diameter used, and whether it is exact */
  uint32_t stop_reason;    /* KAD_STOP_RULE, KAD_STOP_OMEGA, or KAD_STOP_FIXED (fixed schedule) */
  uint32_t n;
  double seconds;          /* wall time of the call */
  double C;                /* the constant found by computeDelta's bisection */
  double seconds_setup;    /* vertex diameter, omega, buffers */
  double seconds_pilot;    /* pilot samples and their counts */
  double seconds_delta;    /* computeDelta and the stopping-check setup */
  double seconds_main;     /* main phase until the stopping check */
  /* caller-owned host arrays of length n; any may be NULL */
  uint64_t *count;         /* main-phase hits per node */
  double *bc;              /* count / tau */
  double *lower, *upper;   /* [bc - f, bc + g] after a rule stop, [bc - eps, bc + eps] at omega */
  /* top-k output (caller-owned, capacity topk_cap): nodes with rank_lo <= k in order of
     decreasing estimate (ties by id), with rank_lo = 1 + #{w != v: lower(w) >= upper(v)}
     and rank_hi = #{w: upper(w) > lower(v)}.  If more than topk_cap nodes qualify the call
     returns KAD_ETOOSMALL with topk_len set to the number needed. */
  uint32_t topk_cap, topk_len;
  uint32_t *topk_node, *rank_lo, *rank_hi;
  uint64_t items;          /* entries of the per-item arrays: n, or the number of edges */
} kad_result;

/* Run the adaptive algorithm (Algorithm 1) on the GPU: vertex diameter (host), omega,
 * pilot of alpha samples (phase 0) and computeDelta (host, binary64), then the main
 * phase (phase 1) in batches of samples with the stopping rule checked every
 * check_interval samples (host, binary64).  Fills `r`. */
kad_status kad_run(kad_ctx *ctx, const kad_graph *g, const kad_params *p, kad_result *r,
                   void *hip_stream);

/* ---------------------------------------------------------------- many queries at once */

/* Multi-query engine.  Several adaptive runs -- on one graph or on many graphs, with
 * their own epsilon, delta, mode, k and seed -- share every sampler launch: one
 * launch carries the next pilot samples and check intervals of all of them (a table
 * of (graph, seed, phase, sample ids) segments read by a persistent kernel), their
 * hits go to one counter pool in HBM (one reduction per check point for all queries),
 * and the host evaluates every query's stopping checks while the next launch runs.
 * Each query follows the schedule of kad_run exactly (same sample ids, same check
 * points), so every result is identical to kad_run's for the same graph and
 * parameters; kernel_batch caps a query's samples per launch.  Limits: graphs of up
 * to 2^25 nodes; the node counts of the queries running at once add up to at most
 * 2^25 (the counter pool, each query rounded up to 8192 nodes) -- further queries wait
 * in arrival order until running ones finish ("admission").  Graphs must belong to
 * the context. */

/* Run count queries (graphs[i], params[i]) together and fill results[i] as kad_run
 * would (caller-owned arrays, as for kad_run; seconds = wall time of the whole call's
 * query from start to its completion).  status[i] (may be NULL) receives each query's
 * status; the call returns the first failing one (KAD_OK if none).  Synchronous;
 * claims the context for its duration (KAD_EBUSY if a server or another call holds it). */
kad_status kad_run_batch(kad_ctx *ctx, uint32_t count, const kad_graph *const *graphs,
                         const kad_params *params, kad_result *results, kad_status *status);

/* Serving: a background thread owns the context and runs the engine continuously;
 * queries submitted at any time join the next launch once admitted (continuous
 * batching).  Results are identical to kad_run's.  While a server exists the context
 * is claimed: other calls on it return KAD_EBUSY. */
typedef struct kad_server kad_server;
kad_status kad_server_create(kad_ctx *ctx, kad_server **out);
/* Queue a query; *ticket identifies it.  Parameters are validated here (KAD_EINVAL). */
kad_status kad_server_submit(kad_server *srv, const kad_graph *g, const kad_params *p,
                             uint64_t *ticket);
/* KAD_EBUSY while the query runs; once done, fills `r` like kad_run (caller-owned arrays;
 * r->seconds = latency from submit to completion, r->seconds_setup = time queued before
 * admission) and forgets the ticket.  Returns the query's own status. */
kad_status kad_server_poll(kad_server *srv, uint64_t ticket, kad_result *r);
/* As poll, blocking up to timeout_s seconds (negative: no limit); KAD_EBUSY on timeout. */
kad_status kad_server_wait(kad_server *srv, uint64_t ticket, kad_result *r, double timeout_s);
/* Completed queries, sampler launches and samples launched so far (any may be NULL). */
kad_status kad_server_stats(kad_server *srv, uint64_t *completed, uint64_t *launches,
                            uint64_t *samples);
/* Cancel every query submitted so far that has not completed: poll/wait then report
 * KAD_ECANCELED for it (samples already on the GPU drain first).  The server keeps
 * serving later submissions. */
kad_status kad_server_cancel(kad_server *srv);
/* Stop the server: queries not yet admitted are dropped (their waiters get
 * KAD_ECANCELED), admitted ones finish first (cancel them before to stop sooner);
 * unretrieved results are discarded. */
kad_status kad_server_destroy(kad_server *srv);

/* ---------------------------------------------------------------- sampling primitives */

/* Exact per-sample trace of sample ids [first, first+count) of `phase` (0 pilot, 1 main)
 * (section 4: pair, balanced bidirectional BFS, uniform shortest path).  Host outputs:
 *   s[count], t[count]          : the pair
 *   path_off[count+1]           : sample k's path is path_nodes[path_off[k] .. path_off[k+1]),
 *                                 from s to t inclusive; empty when s and t are disconnected
 *   path_nodes[path_cap]        : KAD_ETOOSMALL (path_off[count] = needed) when short
 *   arcs_scanned[count]         : arcs scanned by the level expansions
 *   flags[count]                : KAD_SAMPLE_* bits (0 for a valid sample)
 * Any output pointer may be NULL except path_off when path_nodes is given. */
kad_status kad_sample_paths(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                            uint64_t first, uint32_t count, uint32_t *s, uint32_t *t,
                            uint64_t *path_off, uint32_t *path_nodes, uint64_t path_cap,
                            uint64_t *arcs_scanned, uint32_t *flags, void *hip_stream);

/* Hit counts of sample ids [first, first+count) of `phase`: count_out[v] (host, length n)
 * is incremented by the number of sampled paths with v as an interior node (section 2:
 * X_i(v) = 1 iff v lies on path i and differs from its ends).  *arcs_scanned (may be
 * NULL) receives the total arcs scanned. */
kad_status kad_hit_counts(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                          uint64_t first, uint64_t count, uint64_t *count_out,
                          uint64_t *arcs_scanned, void *hip_stream);

/* The same hit counts for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  This call allocates and
 * frees nothing: its working memory (sampler slots, one launch's per-sample outputs, a
 * small wide-count arena for samples with many candidate edges) lies in a fixed device
 * array of KAD_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends.  It only enqueues work on hip_stream (NULL: the device's null stream, not
 * the context's) and returns without waiting; it does not claim the context.
 *   count_dev : device uint64[n]; count_dev[v] += hits of v (as kad_hit_counts adds)
 *   arcs_dev  : device uint64[1]; += arcs scanned by the level expansions
 *   flags_dev : device uint32[1]; |= the KAD_SAMPLE_* bits of every sample (0 when every
 *               sample is valid; a flagged sample adds no hits)
 * Errors: KAD_EINVAL for a graph whose path counts may pass 128 bits (its samples need the
 * context's large wide-count arena: use kad_hit_counts); KAD_ENOMEM when the graph's
 * working memory does not fit the scratch (the message gives the sizes); about 3.5M nodes
 * at most, with fewer concurrent samples as n grows.  Calls that overlap on one GPU (any
 * context, any stream) race on the shared scratch and must be ordered by the caller. */
#define KAD_NOALLOC_SCRATCH_BYTES (128ull << 20)
kad_status kad_hit_counts_noalloc(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                                  uint64_t first, uint64_t count, uint64_t *count_dev,
                                  uint64_t *arcs_dev, uint32_t *flags_dev, void *hip_stream);

/* Edge hit counts of sample ids [first, first+count) of `phase`: count_out[e] (host, one
 * entry per edge id) is incremented by the number of sampled paths that contain edge e. */
kad_status kad_edge_hit_counts(kad_ctx *ctx, const kad_graph *g, uint64_t seed, uint32_t phase,
                               uint64_t first, uint64_t count, uint64_t *count_out,
                               uint64_t *arcs_scanned, void *hip_stream);

/* Edges of g: *count = arcs (directed) or arcs / 2 (undirected). */
kad_status kad_graph_edge_count(const kad_graph *g, uint64_t *count);
/* Edge id of every arc position (host uint32[arcs]): a directed graph's edge is its arc's
 * position in the out-rows; an undirected edge {u, v} is the rank of its arc u -> v (u < v)
 * in CSR order, and both of its arcs carry that id. */
kad_status kad_graph_edge_ids(const kad_graph *g, uint32_t *eid);

/* ---------------------------------------------------------------- host statistics */
/* These run on the CPU only (no device needed); binary64, no FMA contraction. */

/* Sample cap of Algorithm 1: ceil(c/eps^2 * (floor(log2(max(vd-2,1))) + 1 + ln(2/delta))). */
uint64_t kad_omega(double epsilon, double delta, uint32_t vd, double c);
/* Pilot size of Algorithm 2: max(1, floor(omega/100)). */
uint64_t kad_alpha(uint64_t omega);
/* Sample count of a fixed schedule: KAD_SCHEDULE_RK gives
 * ceil(c/eps^2 (floor(log2(max(vd-2,1))) + 1 + ln(1/delta))), KAD_SCHEDULE_HOEFFDING gives
 * ceil(ln(2n/delta) / (2 eps^2)); 0 for any other schedule.  c <= 0 means 0.5. */
uint64_t kad_fixed_samples(uint32_t schedule, double epsilon, double delta, uint32_t vd,
                           uint32_t n, double c);
/* Default check interval: 2^floor(log2(omega/16)) clamped to [1024, 65536]. */
uint64_t kad_default_interval(uint64_t omega);

/* Vertex diameter (largest number of nodes on a shortest path) of a host CSR (same layout
 * rules as kad_graph_create; rrow/rcol required for directed graphs).  The rows (and
 * in-rows) are checked as kad_graph_create checks them, KAD_EINVAL if malformed; the
 * in-rows are not compared with the transpose, nor an undirected graph for symmetry.  Exact by a BFS from
 * every node when n*arcs <= exact_limit; otherwise the bound: heaviest path of the
 * strongly-connected-component DAG where component C weighs ecc_out_C(r) + ecc_in_C(r) + 1,
 * r = C's node of largest in+out degree (lowest id on ties). */
kad_status kad_vertex_diameter(uint32_t n, uint64_t arcs, int directed, const uint32_t *row_ptr,
                               const uint32_t *col, const uint32_t *rrow_ptr,
                               const uint32_t *rcol, double exact_limit, uint32_t *vd,
                               uint32_t *exact);

/* f and g of Theorem azuma-borassi, L = ln(1/delta_L) or ln(1/delta_U), btilde = count/tau. */
double kad_bound_f(double btilde, double L, double omega, double tau);
double kad_bound_g(double btilde, double L, double omega, double tau);

/* computeDelta (Algorithm 2): L_l[v] = -ln(delta_L(v)), L_u[v] = -ln(delta_U(v)) from the
 * pilot counts count0 (alpha samples) and the wanted half-widths lambda_l/lambda_u (host
 * arrays of length n); *C receives the bisection's constant (may be NULL). */
kad_status kad_compute_delta(uint32_t n, const uint64_t *count0, uint64_t alpha, uint64_t omega,
                             const double *lambda_l, const double *lambda_u, double delta,
                             double balance_eps, double *L_l, double *L_u, double *C);

/* computeDelta (Algorithm 2) when every node has the same half-widths lambda_l and
 * lambda_u (the all-nodes task), from the histogram of the pilot counts: hist[c] nodes
 * have pilot count c, for c = 0..cmax (host array of cmax + 1 entries; n = the sum).  The
 * nodes with one count share their L values: group_of_count[c] receives the group of
 * count c (entries of counts absent from the histogram are 0), L_l[g] and L_u[g] the
 * group's -ln(delta_L), -ln(delta_U) (room for cmax + 1 groups), *ngroups the number of
 * groups, *C the bisection's constant (may be NULL).  The same values, bit for bit, as
 * kad_compute_delta gives each node. */
kad_status kad_compute_delta_hist(uint32_t n, const uint64_t *hist, uint64_t cmax, uint64_t alpha,
                                  uint64_t omega, double lambda_l, double lambda_u, double delta,
                                  double balance_eps, uint32_t *group_of_count, double *L_l,
                                  double *L_u, uint32_t *ngroups, double *C);

/* Wanted half-widths for the top-k task (section 5) from the pilot counts. */
kad_status kad_topk_lambdas(uint32_t n, uint32_t k, const uint64_t *count0, uint64_t alpha,
                            double epsilon, double *lambda_l, double *lambda_u);

/* The top-k output (section 5): the nodes v whose rank interval reaches the top k --
 * rank_lo(v) = 1 + #{w != v: lower(w) >= upper(v)} <= k -- ordered by count descending, id
 * ascending, with rank_lo and rank_hi(v) = #{w: upper(w) > lower(v)}.  count, lower and upper
 * are host arrays of n entries; node, rank_lo and rank_hi have room for cap entries (any may
 * be NULL).  *len receives the selection's size; KAD_ETOOSMALL when it exceeds cap (nothing
 * written), KAD_EINVAL for k outside [1, n]. */
kad_status kad_topk_select(uint32_t n, uint32_t k, const uint64_t *count, const double *lower,
                           const double *upper, uint32_t cap, uint32_t *node, uint32_t *rank_lo,
                           uint32_t *rank_hi, uint32_t *len);

/* Stopping conditions: all-nodes (every f <= eps and g <= eps) and top-k (Algorithm 3).
 * Return 1 (stop), 0 (continue) or a negative kad_status. */
int kad_have_to_stop(uint32_t n, uint32_t mode, uint32_t k, const uint64_t *count, uint64_t tau,
                     uint64_t omega, double epsilon, const double *L_l, const double *L_u);

/* ---------------------------------------------------------------- search strategy */

/* How graph g's samples find their shortest paths (every sampling call on g follows it):
 *   KAD_SEARCH_BALANCED (default) -- section 4's balanced bidirectional BFS: the side whose
 *       frontier has the smaller degree sum is expanded, until the two searches touch;
 *   KAD_SEARCH_FORWARD -- a plain BFS from s, level by level until the level that reaches
 *       t is finished: the search of the samplers the paper compares against (section 6,
 *       where it costs m_avg arcs per sample), kept to measure what the balanced search
 *       saves (Theorem 2).
 * Both give a uniformly random shortest s-t path of the same pair; the paths drawn differ,
 * so results depend on the choice (the oracle takes the same flag).  Returns KAD_EINVAL for
 * any other value. */
enum { KAD_SEARCH_BALANCED = 0, KAD_SEARCH_FORWARD = 1 };
kad_status kad_graph_set_search(kad_graph *g, uint32_t search);
kad_status kad_graph_get_search(const kad_graph *g, uint32_t *search);

/* ---------------------------------------------------------------- launch shape */

/* Sampler launch shape used for graph g (by kad_run, kad_sample_paths, kad_hit_counts and
 * engine launches where g has the most samples): `block` threads per workgroup (64, 128
 * or 256; one sample per workgroup) and `small_expansion`, the largest level expansion
 * (in arcs) handled by one combined scan instead of a touch scan plus a discovery scan.
 * (0, 0) restores the library default (128, 128).  Performance only: results never
 * depend on the shape. */
kad_status kad_graph_set_launch(kad_graph *g, uint32_t block, uint32_t small_expansion);
kad_status kad_graph_get_launch(const kad_graph *g, uint32_t *block, uint32_t *small_expansion);

/* Autotuner: time one sampler launch of `samples` main-phase sample ids (0 = 65,536) of
 * g with every candidate shape (block 64/128/256 x small_expansion 0/32/128/512; the
 * faster of two launches each) and keep the fastest as g's shape.  Reports it and its
 * launch time in seconds (any pointer may be NULL). */
kad_status kad_autotune(kad_ctx *ctx, kad_graph *g, uint32_t samples, uint32_t *block,
                        uint32_t *small_expansion, double *seconds);

/* ---------------------------------------------------------------- measurement hooks */

/* Time every sampler launch of this context with HIP events recorded on the launch
 * stream (enable != 0; this also resets the totals).  Adds one event synchronisation
 * per launch. */
kad_status kad_ctx_set_timing(kad_ctx *ctx, int enable);
/* Totals over the timed sampler launches since timing was enabled: launches, samples,
 * seconds (the time the launches kept the GPU busy: the sum of the event-measured launch
 * durations, except that within one kad_run, whose first main batch may run beside the
 * pilot, the union of the launches' intervals), arcs scanned, nodes reached by the two
 * searches, and hits (interior path nodes).  Any pointer may be NULL. */
kad_status kad_ctx_get_timing(kad_ctx *ctx, uint64_t *launches, uint64_t *samples,
                              double *seconds, uint64_t *arcs, uint64_t *nodes, uint64_t *hits);

/* Wide-count working memory, used by graphs whose path counts can pass 128 bits: the
 * number of first-pass slots (workgroups sampling at once) and each one's arena in 64-bit
 * limbs (0 = the library's choice: at most the sampler slots, as many as can be resident, and
 * as many as 80% of the memory left after the sampler slots allows, each with room for any
 * sample of the graph when that bound is at most 2^25 limbs, else 2^25 limbs or more).
 * Samples that outgrow a first-pass arena are sampled again, after the pass, by a second
 * pass with fewer and larger arenas (the graph's bound, at most 2^27 limbs, or all of the
 * first pass's memory) carved from the same memory; a sample that outgrows that too fails
 * the call with KAD_EOVERFLOW.  Results never depend on this layout.  Frees the current
 * arenas (laid out again on next use); KAD_EINVAL for 0 < limbs < 4096. */
kad_status kad_ctx_set_wide(kad_ctx *ctx, uint32_t slots, uint64_t limbs);
/* The current layout: first-pass slots and limbs per slot, second-pass slots and limbs per
 * slot (0 when no arena is allocated, or when there is one pass).  Any pointer may be NULL. */
kad_status kad_ctx_get_wide(kad_ctx *ctx, uint32_t *slots, uint64_t *limbs, uint32_t *slots2,
                            uint64_t *limbs2);

/* Sampler slot layout (section 4's searches keep, per sample, a tag and a 128-bit path
 * count for every node they reach).  log2_records = 0: the library's choice -- one
 * record per node of the largest graph seen, unless the memory budget then holds fewer
 * than 4 slots per CU and the graph has more than 2^16 nodes (about 10^7 nodes and more
 * at full budget); then a hash table of 2^16 records per slot.  1: always one record per
 * node.  6 to 24: always tables of 2^log2_records records.  With tables, memory per slot
 * no longer grows with the graph (32 B, 8 B of lists per record), the wide-count kernel
 * gets slots of its own with one record per node, and a sample whose reached nodes do
 * not fit its table (a node that finds no free record within 32 probes) is sampled again
 * by the wide-count kernel; a sample takes about 0.75x as long to draw with tables where
 * one record per node also fits.  Results never depend on the layout.  Frees nothing at
 * once: the slots are laid out again on next use.  KAD_EINVAL for another value;
 * KAD_EBUSY while the context is in use. */
kad_status kad_ctx_set_table(kad_ctx *ctx, uint32_t log2_records);
/* The current layout: log2 of the records per sampler slot (0: one record per node, or no
 * slots yet), the sampler slots and the slots the wide-count kernel can use (0 before the
 * first call that samples).  Any pointer may be NULL. */
kad_status kad_ctx_get_table(kad_ctx *ctx, uint32_t *log2_records, uint32_t *slots,
                             uint32_t *wide_slots);

/* The launch mode (KAD_EXEC_*; default KAD_EXEC_GRAPH) of kad_run and of the engine
 * (kad_run_batch, the server: KAD_EXEC_GRAPH replays each tick's sampling chain; the other
 * two modes launch it call by call).  While timing is enabled
 * KAD_EXEC_GRAPH launches call by call (the per-launch events sit inside the chain).
 * The recorded chains are kept in the context and recorded again when the graph, the
 * buffers or kernel_batch change.  KAD_EINVAL for an unknown mode. */
kad_status kad_ctx_set_exec(kad_ctx *ctx, uint32_t mode);
/* The mode, and how many chains this context has recorded and replayed (kad_run's batches
 * and the engine's ticks, whose sampling chain -- segment table, sampler, wide-count passes,
 * host mirrors -- is replayed the same way; any pointer may be NULL). */
kad_status kad_ctx_get_exec(kad_ctx *ctx, uint32_t *mode, uint64_t *records, uint64_t *replays);

const char *kad_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KADABRA_H */
