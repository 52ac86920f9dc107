/*
 * grass.h -- C ABI of the MI355X (gfx950) GRASS spectral sparsification library.
 *
 * What it computes (Feng, "GRASS: Graph Spectral Sparsification Leveraging
 * Scalable Spectral Perturbation Analysis", arXiv:1911.04382):
 *   - a spanning-tree backbone P of a weighted undirected graph G (Sec. III-I
 *     step 1; here the maximum-weight tree, ties broken by the smaller edge id);
 *   - t-step generalized power iterations h_t = (L_P^+ L_G)^t h_0 on k random
 *     vectors orthogonal to the all-ones vector (eqs. 28, 29);
 *   - the Joule heat w_pq sum_j (h_j(p) - h_j(q))^2 of every off-subgraph edge
 *     (eqs. 31, 35, 55);
 *   - lambda_max by a Rayleigh quotient of the iterated vectors (Sec. IV-C.1),
 *     lambda_min by the degree ratio of eq. (61), kappa = lambda_max/lambda_min
 *     (eq. 3);
 *   - the normalized-heat threshold theta = (sigma2 lambda_min/lambda_max)^(2t+1)
 *     of eq. (58), a similarity check and a per-pass budget (Sec. IV-D steps 5, 6),
 *     repeated as iterative densification until kappa <= sigma2 (Sec. IV-D).
 *
 * Conventions shared by every call:
 *   - A graph is a canonical edge list: src[e] < dst[e], edges sorted by
 *     (src, dst), no duplicates, 0 <= ids < n, weights finite and > 0; the edge
 *     id is the position e. Arrays are DEVICE pointers owned by the caller.
 *   - Every output is indexed by edge id (or node id), whatever node order the
 *     kernels use internally.
 *   - All work is enqueued on the caller's stream. Calls that must decide on
 *     device results (densification passes, PCG convergence) synchronize that
 *     stream; the outputs are complete when the call returns.
 *   - Device memory comes from the caller's workspace (`workspace`, `ws_bytes`,
 *     at least grass_workspace_bytes()). Passing workspace == NULL makes the
 *     context allocate and keep its own (grown on demand, freed by
 *     grass_destroy).
 *   - Negative status = failure: outputs are undefined and grass_last_error()
 *     holds a message. No exception crosses the ABI. A context is not
 *     thread-safe; use one per host thread.
 *   - Results are deterministic: the same inputs give the same output bits
 *     (no floating-point atomics; every reduction has a fixed order).
 */
#ifndef GRASS_H
#define GRASS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GRASS_OK = 0,
    GRASS_NOT_CONVERGED = 1,    /* warning: outputs valid, kappa > sigma2 after max_iters passes */
    GRASS_ERR_INVALID = -1,     /* bad arguments or non-canonical graph */
    GRASS_ERR_DISCONNECTED = -2,/* G is not connected (Sec. II-A assumes it is) */
    GRASS_ERR_OOM = -3,         /* workspace too small / allocation failed */
    GRASS_ERR_DEVICE = -4,      /* HIP runtime error or a device-side guard tripped */
    GRASS_ERR_UNIMPLEMENTED = -5,
    GRASS_ERR_CANCELLED = -6,
    GRASS_ERR_SOLVE = -7,       /* an L_P solve (eq. 29) ended above pcg_rtol, checked in FP64: the
                                   pass's heats are not trusted, so nothing was selected from them;
                                   grass_sparsify then stops with edge_mask = the subgraph before
                                   that pass and a summary/trace of every pass run (the last one
                                   flagged GRASS_PASS_SOLVE_FAILED); scores are undefined */
    GRASS_ERR_NONFINITE = -8    /* a NaN or infinity appeared in the vectors, heats or residuals
                                   (e.g. weights that overflow FP32 arithmetic); outputs undefined */
} grass_status;

/* grass_pass_stats.flags */
enum { GRASS_PASS_SOLVE_FAILED = 1 };

typedef struct grass_ctx grass_ctx;

/* Create a context on HIP device `device`. */
grass_status grass_create(int device, grass_ctx **out);
/* Destroy a context (frees only memory the context allocated itself). */
void grass_destroy(grass_ctx *ctx);
/* Text of the last failure on this context ("" if none). Valid until the next call. */
const char *grass_last_error(const grass_ctx *ctx);

/* Graph of the conventions above. src, dst: int32 [m]; w: float64 [m]; device. */
typedef struct {
    int64_t n, m;
    const int32_t *src;
    const int32_t *dst;
    const double *w;
} grass_graph;

/* Options (grass_opts_default() gives the defaults in brackets). */
typedef struct {
    double sigma2;          /* target relative condition number, eq. (5) [100] */
    int32_t k;              /* random vectors, 1..64 [16] */
    int32_t t;              /* power steps per pass, eq. (29) [2] */
    uint64_t seed;          /* Philox key of the start vectors [0] */
    int32_t max_iters;      /* densification passes; 0 = estimate only [50] */
    double budget_frac;     /* per-pass budget floor(budget_frac n) (>= 1); 0 = unlimited [0.01] */
    int32_t sim_hops;       /* similarity marks: -1 off, 0 endpoints, 1 endpoints + neighbours [1] */
    int32_t lambda_steps;   /* power steps for lambda_max (>= t continues the vectors) [0 = t] */
    double pcg_rtol;        /* relative residual target of every L_P solve, checked in FP64 [1e-6] */
    int32_t pcg_max_iters;  /* working-precision block-PCG iterations per L_P solve, all inner solves
                               together [8000] */
    double pcg_inner_rtol;  /* residual reduction of each inner block-PCG solve between the FP64
                               flexible-CG steps around it [1e-2] */
    int32_t pcg_max_outer;  /* FP64 flexible-CG steps per L_P solve [50] */
    int32_t precision;      /* 32: FP32 vectors (FP64 sums); 64: FP64 throughout [32] */
    const uint8_t *init_mask; /* optional device [m]: 1 = edge of a caller-given spanning tree,
                                 2 = already-added edge, 0 = off; NULL = compute the tree */
} grass_opts;

grass_opts grass_opts_default(void);

/* Per-pass record. */
typedef struct {
    int32_t pass;
    double lambda_max, lambda_min, kappa, theta, heat_max;
    int64_t m_off;          /* off-subgraph edges scored in this pass */
    int64_t candidates;     /* edges passing eq. (58) */
    int64_t accepted;       /* edges added after the similarity check and budget */
    int64_t pcg_iters;      /* inner PCG iterations summed over the pass's solves (max over vectors) */
    double pcg_resid64;     /* largest FP64 relative residual of the pass's L_P solves */
    double ms;              /* wall time of the pass */
    int32_t flags;          /* GRASS_PASS_SOLVE_FAILED: pcg_resid64 > pcg_rtol (or not finite) */
} grass_pass_stats;

typedef struct {
    double lambda_max, lambda_min, kappa; /* estimates on the final subgraph */
    double pcg_resid64;     /* FP64 relative residual of the last L_P solve (0 if only tree solves) */
    double heat_max;
    int32_t passes;
    int64_t tree_edges, added_edges;
    int64_t scored_edges;   /* sum over passes of m_off */
    int64_t pcg_iters;
} grass_summary;

/* Outputs of grass_sparsify. edge_mask, scores: device [m]; summary, trace: host. */
typedef struct {
    uint8_t *edge_mask;     /* 1 tree, 2 added, 0 not in the sparsifier */
    void *scores;           /* float32 (precision 32) or float64 (precision 64): heat/heat_max of the
                               last pass that filtered (the final pass if none did); 0 for edges in P */
    grass_summary *summary; /* may be NULL */
    grass_pass_stats *trace;/* may be NULL */
    int32_t trace_cap;
} grass_result;

/* Workspace bytes that grass_sparsify / grass_embed / grass_spanning_tree need for
 * a graph of n nodes and m edges under opts (the admission footprint). */
size_t grass_workspace_bytes(int64_t n, int64_t m, const grass_opts *opts);

/* The whole method: tree, passes of embedding + scoring + estimates, filtering
 * and densification until kappa <= sigma2 (Sec. IV-D). Returns GRASS_OK,
 * GRASS_NOT_CONVERGED, GRASS_ERR_SOLVE (a pass's L_P solve missed pcg_rtol; see
 * the status) or another error. */
grass_status grass_sparsify(grass_ctx *ctx, const grass_graph *g, const grass_opts *opts, void *workspace,
                            size_t ws_bytes, grass_result *res, void *stream);

/* Bytes of the static device scratch of grass_sparsify_static (one per GPU). */
#define GRASS_STATIC_SCRATCH_BYTES ((size_t)256 << 20)

/* grass_sparsify for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and outputs, with the workspace taken from a static device array of
 * GRASS_STATIC_SCRATCH_BYTES (256 MiB) that the library holds on each GPU until the
 * process ends, instead of a caller's buffer. No hipMalloc, hipFree or other
 * allocating routine is called (nor per-kernel event timing). A graph whose
 * grass_workspace_bytes exceeds the scratch is rejected with GRASS_ERR_OOM before
 * any device work (a 3-D mesh of about 110,000 nodes at k = 16, FP32). Every call
 * on one GPU shares that GPU's scratch, which keeps the last call's contents (each
 * call initializes what it reads): calls that overlap on one GPU race, so serialize
 * them (one stream, or host ordering). The scratch is resolved for a device by
 * grass_create. Inputs and outputs as grass_sparsify. */
grass_status grass_sparsify_static(grass_ctx *ctx, const grass_graph *g, const grass_opts *opts, grass_result *res,
                                   void *stream);

/* Many independent graphs in one call (the same method as grass_sparsify, per
 * graph: Sec. IV-D). graphs, opts, results, statuses: host arrays of count entries
 * (the grass_graph entries hold device pointers as for grass_sparsify; opts may
 * hold one entry, used for every graph, when opts_count is 1). Up to `workers`
 * graphs run at once, each on a HIP stream of its own (ordered after the work
 * already on `stream`; `stream` waits for all of them) and in its own slice of
 * the workspace; larger graphs start first. Each graph's outputs are exactly
 * those grass_sparsify gives it alone. statuses[i] is graph i's status; the call
 * returns GRASS_OK when every graph converged, GRASS_NOT_CONVERGED when some did
 * not, or the first error (the other graphs' outputs are still valid when their
 * status says so). The workspace needs grass_batch_workspace_bytes bytes. */
size_t grass_batch_workspace_bytes(int32_t count, const grass_graph *graphs, const grass_opts *opts,
                                   int32_t opts_count, int32_t workers);
grass_status grass_sparsify_batch(grass_ctx *ctx, int32_t count, const grass_graph *graphs, const grass_opts *opts,
                                  int32_t opts_count, int32_t workers, void *workspace, size_t ws_bytes,
                                  grass_result *results, grass_status *statuses, void *stream);

/* Launch schedule of the L_P solves' inner block-PCG loop on the concurrent paths
 * (grass_sparsify_batch, and servers created afterwards); the single-graph entry
 * points always launch kernel by kernel. The loop's decisions (iteration count and
 * cap, the end of an inner phase, the stall rule of FP32 solves) are taken on the
 * device in every mode.
 *   GRASS_LAUNCH_KERNELS: kernel by kernel, the host reading the loop state every
 *     4th iteration (8 bytes).
 *   GRASS_LAUNCH_CAPTURED (default): with FP32 and k of 16 or 32, four iterations
 *     are captured once per solve as a hipGraph and replayed chunks_per_read times
 *     between host reads; kernels replayed after a phase has ended return at once,
 *     so every output is the same as kernel by kernel. chunks_per_read 0 (default)
 *     lets the context's autotuner choose per size class (node count in powers of
 *     two, k): it times inner phases with 1, 2, 4 or 8 chunks and with kernel-by-
 *     kernel launches, three phases each, and keeps the fastest.
 * Other k and FP64 run kernel by kernel. A batch reads the mode when it starts and
 * a server when it is created: call this while no batch call of the context is
 * running. Returns GRASS_ERR_INVALID for an unknown mode or chunks_per_read
 * outside 0..64. */
enum { GRASS_LAUNCH_KERNELS = 0, GRASS_LAUNCH_CAPTURED = 1 };
grass_status grass_set_launch_mode(grass_ctx *ctx, int32_t mode, int32_t chunks_per_read);
/* Counters of the block-PCG loops run through the launch schedule above since the
 * context was created or last reset (reset != 0 clears them after the copy):
 * iterations, host reads of the loop state, graph replays and captures. */
typedef struct {
    int64_t iterations;
    int64_t host_reads;
    int64_t graph_replays;
    int64_t captures;
} grass_launch_stats;
grass_status grass_launch_stats_read(grass_ctx *ctx, grass_launch_stats *out, int32_t reset);

/* Serving: a queue of sparsify requests on one device with continuous batching.
 * grass_server_create preallocates a device arena of arena_bytes (the admission
 * budget) and starts `workers` host workers, each with its own HIP stream.
 * grass_server_submit queues a request and returns at once; a queued request is
 * admitted as soon as a worker is free and the arena has room for its workspace
 * (grass_workspace_bytes), in arrival order, smaller requests may pass a head
 * request that does not fit yet (at most 2 x workers times, then admission waits
 * for it). Requests in flight overlap on the device. A request's outputs are
 * exactly those grass_sparsify gives it alone. Its graph and result buffers
 * (device) and summary/trace (host) must stay valid until it is done or
 * cancelled. Requests larger than the arena are rejected with GRASS_ERR_OOM at
 * submission. */
typedef struct grass_server grass_server;
typedef enum { GRASS_REQ_QUEUED = 0, GRASS_REQ_RUNNING = 1, GRASS_REQ_DONE = 2, GRASS_REQ_CANCELLED = 3 } grass_req_state;
typedef struct {
    int32_t state;        /* grass_req_state */
    grass_status status;  /* the request's status once done */
    double t_submit, t_start, t_end; /* seconds since the server was created (steady clock) */
    size_t footprint;     /* workspace bytes admitted */
} grass_req_info;
grass_status grass_server_create(grass_ctx *ctx, size_t arena_bytes, int32_t workers, grass_server **out);
grass_status grass_server_submit(grass_server *srv, const grass_graph *g, const grass_opts *opts,
                                 grass_result *res, int64_t *ticket);
/* State and timing of a request (non-blocking). */
grass_status grass_server_poll(grass_server *srv, int64_t ticket, grass_req_info *info);
/* Block until the request is done or cancelled (ticket < 0: until every request is). */
grass_status grass_server_wait(grass_server *srv, int64_t ticket);
/* Cancel a request that has not started (GRASS_ERR_INVALID if it has). */
grass_status grass_server_cancel(grass_server *srv, int64_t ticket);
/* Text of the last error of a request (empty when none). */
const char *grass_server_error(grass_server *srv, int64_t ticket);
/* Wait for the requests in flight, drop the queued ones, free the arena. */
void grass_server_destroy(grass_server *srv);

/* Maximum-weight spanning tree (Boruvka; ties by smaller edge id): tree_mask[e] = 1
 * for the n-1 tree edges, else 0. tree_mask: device uint8 [m]. */
grass_status grass_spanning_tree(grass_ctx *ctx, const grass_graph *g, uint8_t *tree_mask, void *workspace,
                                 size_t ws_bytes, void *stream);

/* Low-stretch spanning tree (Sec. III-A builds the sparsifier on a low-stretch
 * tree; the paper cites star and petal decompositions). This one is the AKPW
 * construction over binary weight classes (class of e = (max ilogb(w) - ilogb(w_e))
 * / class_bits, class 0 the heaviest) with exponential start-time clustering in
 * each round: cluster u starts at 85 - d_u, d_u a geometric shift (P(d >= k) =
 * (7/8)^k) read from Philox4x64-10 at counter (u, round, 0x4C535354, 0), key
 * (seed, 0); a cluster joins the center minimising hops + start (smaller id on
 * ties) through the heaviest FP32 edge from a cluster one hop nearer to it (smaller
 * edge id on ties). tree_mask: device uint8 [m], 1 for the n-1 tree edges, else 0;
 * pass it to grass_sparsify as opts->init_mask to build on it. class_bits >= 1.
 * The tree depends only on the graph, seed and class_bits. Errors:
 * GRASS_ERR_INVALID (bad graph or class_bits), GRASS_ERR_DISCONNECTED. workspace:
 * grass_low_stretch_tree_workspace_bytes(n, m) device bytes, or NULL for the
 * context's own memory. */
size_t grass_low_stretch_tree_workspace_bytes(int64_t n, int64_t m);
grass_status grass_low_stretch_tree(grass_ctx *ctx, const grass_graph *g, uint64_t seed, int32_t class_bits,
                                    uint8_t *tree_mask, void *workspace, size_t ws_bytes, void *stream);

/* One pass of embedding and scoring for a given subgraph P (Sec. III-F, eqs. 28-35,
 * 55, 61): p_mask device uint8 [m] (1 = spanning-tree edge, 2 = added edge, 0 = off;
 * the 1-edges must span G); pass = the Philox counter word of the start vectors.
 * heat: device [m], float32 or float64 per opts->precision, the unnormalized heat of
 * every edge (scaled by a power of two common to all edges: only ratios are
 * meaningful); stats: host, filled except candidates/accepted/theta. Returns
 * GRASS_ERR_SOLVE (heat written but not trusted; stats filled and flagged) when an
 * L_P solve ended above pcg_rtol. */
grass_status grass_embed(grass_ctx *ctx, const grass_graph *g, const uint8_t *p_mask, const grass_opts *opts,
                         int32_t pass, void *heat, grass_pass_stats *stats, void *workspace, size_t ws_bytes,
                         void *stream);

/* Filtering and similarity check of one pass (eq. 58, Sec. IV-D steps 5-6): given
 * the heat of grass_embed and the pass's lambda estimates, add the accepted edges to
 * p_mask (value 2, in place) and write stats->theta/candidates/accepted.
 * scores (optional device [m], same type as heat): heat/heat_max off P, 0 in P. */
grass_status grass_select(grass_ctx *ctx, const grass_graph *g, uint8_t *p_mask, const grass_opts *opts,
                          const void *heat, double lambda_max, double lambda_min, grass_pass_stats *stats,
                          void *scores, void *workspace, size_t ws_bytes, void *stream);

/* The sparsifier as a preconditioner (Sec. V-E): solve L_G x = b for k = opts->k
 * right-hand sides by preconditioned CG, the preconditioner being L_P^+ for the
 * subgraph P of p_mask (device uint8 [m], 1 = spanning-tree edge, 2 = added edge,
 * as grass_sparsify writes it; NULL = the maximum-weight spanning tree alone).
 * L_P^+ is applied exactly (tree solve) when P is a tree, else inexactly, with
 * flexible CG coefficients: each application is one working-precision phase of the
 * power iterations' block PCG from zero, which ends once every column's residual has
 * fallen by max(opts->pcg_inner_rtol, opts->pcg_rtol) or after opts->pcg_max_iters
 * iterations (8000 when 0), with no FP64 correction. The system
 * is grounded at node 0 (row and column removed, x[0] = 0); b should sum to zero
 * per column. b, x: device n x k row-major, float32 or float64 per
 * opts->precision, distinct (b is not modified). Stops when every column has
 * ||r|| <= rtol ||b|| for the residual recomputed from x (the recurrence restarts
 * from it, at most 5 times, when working-precision drift leaves it above rtol) or
 * after max_iters outer iterations. A reduction of 1e-2, or a few iterations, per
 * application is enough inside the flexible recurrence; tighter costs inner
 * iterations. info (host, optional):
 * outer iterations (the paper's N), inner block-PCG iterations, the largest
 * ||b - L_G x|| / ||b|| recomputed from x, wall time, edges of P beyond the tree.
 * Returns GRASS_NOT_CONVERGED (x valid) when rtol was not reached. Workspace:
 * grass_solve_workspace_bytes (or NULL: the context allocates). */
typedef struct {
    int32_t iters;
    int64_t inner_iters;
    double resid;
    double ms;
    int64_t added_edges;
} grass_solve_info;
size_t grass_solve_workspace_bytes(int64_t n, int64_t m, const grass_opts *opts);
grass_status grass_solve(grass_ctx *ctx, const grass_graph *g, const uint8_t *p_mask, const grass_opts *opts,
                         const void *b, void *x, double rtol, int32_t max_iters, grass_solve_info *info,
                         void *workspace, size_t ws_bytes, void *stream);

/* Spectral partitioning with the sparsifier (Sec. V-F): `steps` inverse power
 * iterations u <- (L_G^+ u - mean(.)) / ||.|| from the start vector of eq. (28)
 * (opts->seed, pass 0, one vector), each solve by grass_solve's method to rtol with
 * the subgraph of p_mask (NULL = the spanning tree) as the preconditioner; the two
 * parts are the sign cut of the approximate Fiedler vector u. fiedler: device [n],
 * float32 or float64 per opts->precision (unit norm, mean zero); side: device
 * uint8 [n], 1 where u >= 0. opts->k is ignored (one vector); outer solves stop
 * after opts->pcg_max_iters iterations (1000 when 0). info (host, optional): outer
 * and inner iterations summed over the steps, the largest solve residual, wall
 * time. GRASS_NOT_CONVERGED (outputs valid) when a solve missed rtol. Workspace:
 * grass_partition_workspace_bytes (or NULL: the context allocates). */
typedef struct {
    int32_t steps;
    int64_t outer_iters;
    int64_t inner_iters;
    double resid;
    double ms;
} grass_partition_info;
size_t grass_partition_workspace_bytes(int64_t n, int64_t m, const grass_opts *opts);
grass_status grass_partition(grass_ctx *ctx, const grass_graph *g, const uint8_t *p_mask, const grass_opts *opts,
                             int32_t steps, double rtol, void *fiedler, uint8_t *side, grass_partition_info *info,
                             void *workspace, size_t ws_bytes, void *stream);

/* Start vectors h_0 of eq. (28): n x k row-major, float32 or float64 per precision,
 * Philox4x64-10 Gaussians with each vector's mean removed. out: device. */
grass_status grass_start_vectors(grass_ctx *ctx, int64_t n, int32_t k, uint64_t seed, int32_t pass,
                                 int32_t precision, void *out, void *stream);

/* Diagnostics: out = A'B (k x k, FP64, row-major, device) for device n x k row-major
 * blocks A, B (float32 or float64 per precision), computed by the same Gram kernel
 * (MFMA for FP32 with k in 9..32) that the block PCG of the L_P solves uses. */
grass_status grass_gram(grass_ctx *ctx, int64_t n, int32_t k, int32_t precision, const void *a, const void *b,
                        double *out, void *stream);

/* Diagnostics: per-kernel timing with HIP events recorded on the call's stream
 * around each launch of the selected kernel kinds (a few microseconds per timed
 * launch). grass_profile_enable(ctx, kinds) resets the counters and times the
 * kinds whose bit is set (bit i = the i-th record of grass_profile_read; 0 turns
 * timing off, 0xffffffff times everything). grass_profile_read copies up to cap
 * records (name, launches, summed milliseconds, summed algorithmic bytes: the
 * bytes the operation must move, each vector row read once) and returns the
 * number written (the number available when out is NULL). */
typedef struct {
    const char *name;
    int64_t launches;
    double total_ms;
    double alg_bytes;
} grass_kernel_stats;
grass_status grass_profile_enable(grass_ctx *ctx, uint32_t kinds);
int32_t grass_profile_read(const grass_ctx *ctx, grass_kernel_stats *out, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* GRASS_H */
