/*
 * askit.h -- C ABI of the MI355X (gfx950) ASKIT kernel-summation library.
 *
 * ASKIT (March, Xiao, Biros, arXiv 1410.0260) approximates the kernel sum
 *
 *     u_i = sum_{j=1..N} K(x_i, x_j) w_j,   i = 1..N        (Eq. e:problem)
 *
 * with the Gaussian kernel K(x, y_j) = exp(-|x - y_j|^2 / (2 h_j^2)), h
 * fixed or per source point.  Near interactions are summed directly over the
 * leaves kept by neighbour-based pruning (Eq. e:prune, Alg. 4); far
 * interactions use the skeleton S_alpha of each pruned node and its skeleton
 * weights w~_alpha = w(S_alpha) + P_alpha w(R_alpha) (Sec. 2.1); P_alpha
 * comes from an interpolative decomposition of a row-sampled kernel block
 * (Sec. 2.1 "Approximate skeletonization", Eq. e:sk_targets, Alg. 3).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers, row-major, with an explicit
 *     leading dimension in elements (ldx >= d, ldw >= nrhs, ...).  The
 *     caller owns them; the library never frees or retains them.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it.  setup and query synchronise the stream before
 *     returning (they read back list sizes).  update_weights and evaluate
 *     only enqueue work and never synchronise (so they can be captured in a
 *     HIP graph): outputs are valid after the caller synchronises the
 *     stream, and inputs must stay valid until then.
 *   - Results are returned in the caller's original point order.
 *   - Errors are reported by status code; askit_last_error() returns a
 *     thread-local message for the last failing call on the calling thread.
 *     No C++ exception crosses this boundary.
 *   - A handle is not thread-safe: one thread at a time per handle.
 */
#ifndef ASKIT_H
#define ASKIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ASKIT_ABI_VERSION 2u

typedef enum {
    ASKIT_OK = 0,
    ASKIT_ERR_INVALID_ARG = 1,   /* bad shape, parameter or non-finite input */
    ASKIT_ERR_OUT_OF_MEMORY = 2, /* device allocation failed */
    ASKIT_ERR_DEVICE = 3,        /* no usable gfx950 device, or a HIP call failed */
    ASKIT_ERR_NOT_READY = 4,     /* evaluate before any update_weights */
    ASKIT_ERR_UNSUPPORTED = 5,   /* valid request outside the built limits */
    ASKIT_ERR_BUSY = 6           /* serving: the request queue is full; submit again later */
} askit_status;

typedef enum {
    ASKIT_PREC_FP32 = 0,   /* distances on MFMA in FP32, kernel and sums in FP32 */
    ASKIT_PREC_BF16X3 = 1  /* distance products as bf16 hi/lo split (hi*hi + hi*lo + lo*hi)
                              on MFMA with FP32 accumulation */
} askit_precision;

/* Method parameters (Sec. 3 "Complexity and error", parameter list). */
typedef struct {
    uint32_t struct_size;   /* sizeof(askit_params) */
    uint32_t abi_version;   /* ASKIT_ABI_VERSION */
    int32_t leaf_size;      /* m: points per leaf (a node with more than m points is split) */
    int32_t kappa;          /* kappa: nearest neighbours per point, 1 <= kappa < N */
    int32_t max_skeleton;   /* s_max: largest skeleton size, >= 1 */
    int32_t sample_rows;    /* l: sampled rows per node; 0 selects s_max + 20; must be >= s_max */
    double id_tol;          /* tau >= 0: rank = first t with |R_tt| <= max(tau, 64 eps)|R_00| */
    double bandwidth;       /* h > 0 for the fixed-bandwidth Gaussian */
    int32_t bw_neighbor;    /* > 0: variable bandwidth h_j = distance from x_j to its
                               bw_neighbor-th nearest neighbour (1-based, <= kappa) */
    int32_t precision;      /* askit_precision */
    uint64_t seed;          /* sampler stream (SplitMix64) seed */
    int32_t prune_levels;   /* level restriction (Sec. 3, the error discussion): > 0 lets only the
                               prune_levels deepest tree levels be pruned; a target's traversal
                               goes on below any node above them, and a leaf it reaches there is
                               summed directly.  0 (default): every level may be pruned */
    int32_t reserved;       /* 0 */
} askit_params;

typedef struct askit_handle askit_handle;

/* Fills *p with defaults: m = 128, kappa = 16, s_max = 64, l = 0, tau = 1e-6,
 * h = 1, fixed bandwidth, FP32, seed 0. */
askit_status askit_params_default(askit_params *p);

/*
 * Builds everything that does not depend on the weights (Alg. 5 lines 1-3):
 * exact kappa-nearest-neighbour lists, the median-split tree (Sec. 2.2), the
 * node neighbour lists (Alg. 2), sampled rows (Eq. e:sk_targets), the
 * skeletons and projections P_alpha (Alg. 3), and the interaction lists of
 * the downward pass (Eq. e:prune).
 *   X    device, N x d FP32, row stride ldx >= d; read only during the call.
 *   N    number of points, 2 <= N < 2^31; d >= 1.
 *   out  receives a new handle that owns device copies of all it keeps.
 * Returns ASKIT_ERR_INVALID_ARG for N < 2, d < 1, kappa >= N, m < 1,
 * s_max < 1, l < s_max, h <= 0 with a fixed bandwidth, non-finite X, or a
 * zero variable bandwidth (duplicate points).  Synchronises `stream`.
 * The pivoted QR of every tree level runs on gangs of co-resident
 * workgroups (a cooperative launch) for N >= 2^18 when l <= 288 and a node
 * has at most 512 columns, else one workgroup per node; the environment variable
 * ASKIT_QR_GANG=1 selects that form at any N and ASKIT_QR_GANG=0 never (the
 * two forms take the same decisions with different summation orders).
 * ASKIT_ERR_DEVICE if a gang's exchange does not complete within 10 s.
 * Working memory: a setup takes its temporary buffers (neighbour-search
 * outputs, tile lists, the ID's G blocks, ...) from a per-device arena that
 * the library keeps for the process.  It grows, after a setup that needed
 * more, to that setup's total, up to 16 GiB (11.3 GiB at 2^20 x 64),
 * and is never returned while the process runs.  One setup at a time uses
 * it; concurrent setups and what does not fit use stream-ordered
 * allocations as usual.
 */
askit_status askit_setup(const float *X, int64_t N, int32_t d, int64_t ldx,
                         const askit_params *p, void *stream, askit_handle **out);

/*
 * askit_setup with the neighbour lists N(X) given by the caller instead of
 * the exact search: the paper's driver takes N(X) as an input (Alg. 5), and
 * its neighbours come from an approximate search (Sec. 2.2, "computing
 * nearest neighbors").  Every later step (tree, node lists, sampling,
 * skeletons, pruning) is the one askit_setup runs, on these lists.
 *   knn  device, N x kappa int32 original point ids, row stride ldk >= kappa;
 *        row i holds kappa distinct ids other than i, in any order.  The
 *        library computes their canonical FP64 squared distances and keeps
 *        each row sorted by (distance, id); read only during the call.
 * ASKIT_ERR_INVALID_ARG as askit_setup, and for an id out of [0, N), the
 * row's own id, or a repeated id in a row.  Synchronises `stream`.
 */
askit_status askit_setup_with_knn(const float *X, int64_t N, int32_t d, int64_t ldx, const int32_t *knn,
                                  int64_t ldk, const askit_params *p, void *stream, askit_handle **out);

/*
 * Approximate kappa nearest neighbours by the paper's greedy search with
 * random projection trees (Sec. 2.2, "computing nearest neighbors"): each of
 * `iterations` rounds builds a tree that splits every node with more than
 * leaf_size points at the median of its points' projections on a random
 * direction (the ceil(n/2) smallest (projection, position) go left), gives
 * each point the other points of its leaf as candidates (exhaustive search,
 * canonical FP64 squared distances), keeps each point's kappa best
 * (distance, id) pairs seen in all rounds, and discards the tree.  Directions
 * have +-1 coordinates from a SplitMix64 stream keyed by (seed, round, node),
 * so the result is reproducible bit for bit.  The lists feed
 * askit_setup_with_knn.
 *   X     device, N x d FP32, row stride ldx >= d; read only during the call.
 *   idx   device, N x kappa int32 (row stride kappa): original ids, each row in
 *         increasing (distance, id) order; dist: device N x kappa FP64, the
 *         squared distances.  Both owned by the caller.
 * 1 <= kappa <= 64, kappa < N; 1 <= iterations <= 2046; every leaf of the
 * tree shape (split at ceil(n/2) until at most leaf_size points) must hold
 * more than kappa points (ASKIT_ERR_INVALID_ARG otherwise).  Synchronises
 * `stream`.
 */
askit_status askit_knn_rptree(const float *X, int64_t N, int32_t d, int64_t ldx, int32_t kappa,
                              int32_t leaf_size, int32_t iterations, uint64_t seed, int32_t *idx,
                              double *dist, void *stream);

/*
 * Upward pass (Sec. 2.1, Alg. 3): computes the skeleton weights of every
 * node from W (device, N x nrhs FP32, original point order, row stride
 * ldw >= nrhs), 1 <= nrhs <= 64.  Enqueued on `stream`; W must stay valid
 * until the stream reaches the end of the call's work.
 */
askit_status askit_update_weights(askit_handle *h, const float *W, int64_t ldw, int32_t nrhs,
                                  void *stream);

/*
 * Downward pass (Alg. 4) at every point: U (device, N x nrhs FP32, row
 * stride ldu >= nrhs) receives u in the original point order.
 * ASKIT_ERR_NOT_READY before the first askit_update_weights.
 */
askit_status askit_evaluate(askit_handle *h, float *U, int64_t ldu, void *stream);

/*
 * askit_evaluate that also returns the near-field part of u: Unear (device,
 * N x nrhs FP32, row stride ldun >= nrhs, original point order) receives the
 * direct sums over each point's near leaves alone (Alg. 4, the leaf branch),
 * whose error against the exact sum is the paper's eps_kappa (Sec. 4).  U is
 * bit-identical to askit_evaluate's (the near sums are a prefix of the same
 * summation).  Same conditions and errors as askit_evaluate.
 */
askit_status askit_evaluate_parts(askit_handle *h, float *U, int64_t ldu, float *Unear, int64_t ldun,
                                  void *stream);

/*
 * Evaluation at M new target points Y (device, M x d FP32, row stride ldy)
 * that are not sources (an extension of Alg. 4: a node is pruned for y when
 * it holds none of y's kappa nearest sources).  U (device, M x nrhs FP32,
 * row stride ldu).  1 <= M; synchronises `stream` (it reads back list sizes).
 */
askit_status askit_query(askit_handle *h, const float *Y, int64_t M, int64_t ldy, float *U,
                         int64_t ldu, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): u = K w for
 * the weights W in one call -- the work of askit_update_weights followed by
 * askit_evaluate, with the same kernels and the same results -- without any
 * allocation.  Its working buffers (W in tree order, the skeleton weights and
 * one partial sum per (target, source node) pair and column) live in a fixed
 * device array of ASKIT_NOALLOC_SCRATCH_BYTES, one per GPU, held by the
 * library until the process ends.
 *   W  device, N x nrhs FP32, original point order, row stride ldw >= nrhs;
 *   U  device, N x nrhs FP32, row stride ldu >= nrhs; both owned by the caller.
 * 1 <= nrhs <= 64.  ASKIT_ERR_UNSUPPORTED when the working buffers,
 * 4 (N + num_nodes s_max + eval_pairs) nrhs bytes (each part rounded up to
 * 256 bytes), exceed the array.  Only enqueues work on `stream` (no host
 * synchronisation).  The handle's own weights (askit_update_weights) are left
 * unchanged.  Every call on one GPU shares that GPU's array: calls that overlap
 * on one device (two streams, two host threads) race and must be serialized by
 * the caller.
 */
#define ASKIT_NOALLOC_SCRATCH_BYTES (256ull << 20)
askit_status askit_evaluate_weights_noalloc(askit_handle *h, const float *W, int64_t ldw, int32_t nrhs,
                                            float *U, int64_t ldu, void *stream);

/*
 * The kappa nearest sources of M new points Y (device, M x d FP32, row
 * stride ldy): the neighbour search that askit_query runs for its targets
 * (Sec. 2.2; Alg. 4 prunes with these lists).  idx (device, M x kappa int32,
 * row stride kappa) receives original point ids and dist (device, M x kappa
 * FP64, same layout) the squared Euclidean distances, each row in increasing
 * (distance, id) order; the result is exact.  Needs no weights.  1 <= M;
 * synchronises `stream`.  Outputs are owned by the caller.
 */
askit_status askit_query_neighbors(askit_handle *h, const float *Y, int64_t M, int64_t ldy, int32_t *idx,
                                   double *dist, void *stream);

void askit_destroy(askit_handle *h);

/* Thread-local description of the last error on the calling thread ("" if none). */
const char *askit_last_error(void);

/* ---------------------------------------------------------------------------
 * Diagnostics.  Sizes, counters and host copies of the internal structures,
 * for verification against a reference implementation and for reporting.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t N;
    int32_t d, kappa, leaf_size, max_skeleton, sample_rows, nrhs;
    int32_t num_nodes, num_leaves, depth, ncol_max, num_slabs;
    int64_t near_entries, far_entries;   /* interaction-list entries (slab, node) */
    int64_t near_pairs, far_pairs;       /* algorithmic (target, source) pairs of one evaluation */
    int64_t knn_uncertified_rows;        /* rows that needed the exact fallback */
    double t_knn_ms, t_tree_ms, t_lists_ms, t_skel_ms, t_inter_ms; /* last setup, per phase */
    double t_update_ms;                  /* last update_weights */
    double t_knn_sweep_ms;               /* last setup: approximate kNN candidates (window, filter, select) */
    double t_qr_ms;                      /* last setup: the QR kernels alone (all levels) */
    double t_knn_filter_ms;              /* last setup: the kNN filter sweep launches alone (sum) */
    int64_t knn_filter_launches;         /* ... and their number */
    int64_t eval_pairs;                  /* (target, source node) pairs of one evaluation */
    int64_t eval_chunks;                 /* evaluation work items (up to 64 targets of one source node) */
    int64_t knn_retry_rows;              /* rows whose filter output overflowed (filtered again at
                                            sampled thresholds, then list sweeps if that overflows) */
    int64_t near_lists;                  /* sum over points of |near(i)|: near leaves per point (Alg. 4) */
    int64_t far_lists;                   /* sum over points of |far(i)|: pruned nodes per point; with
                                            near_lists, the paper's near and far counters (Sec. 4) */
    int64_t knn_tiles_swept;             /* last setup: (32-row wave group, 64-point tile) products
                                            the symmetric kNN sweep computed after skipping the pairs
                                            whose bounding balls are farther apart than the thresholds
                                            (-1: no skipping) */
} askit_info;

askit_status askit_get_info(const askit_handle *h, askit_info *out);

/*
 * Pruning diagnostic (Table t:prune): for every point as a target, the number
 * of tree nodes the traversal of Alg. 4 visits (a visited node that is pruned
 * or is a leaf ends its branch; otherwise both children are visited) under
 * the neighbour rule of Eq. (e:prune), into visits_kappa, and under distance
 * pruning -- prune a node when the target lies outside the ball centred at the
 * centroid of the node's points that holds all of them, tested on squared
 * distances in FP64 -- into visits_dist.  Both device, N int32, original
 * point order, owned by the caller.  Synchronises `stream`.
 */
askit_status askit_pruning_visits(const askit_handle *h, int32_t *visits_kappa, int32_t *visits_dist,
                                  void *stream);

/* Node record, breadth-first numbering (root = 0, left before right). */
typedef struct {
    int32_t lo, hi;          /* tree positions [lo, hi) */
    int32_t level, parent, left, right;  /* -1 where absent */
    int64_t path;            /* Morton path bits: left = 0, right = 1 */
} askit_node;

typedef enum {
    ASKIT_X_PERM = 1,        /* int32[N]: original id at each tree position */
    ASKIT_X_KNN_IDX = 2,     /* int32[N*kappa]: neighbours (original ids), original row order */
    ASKIT_X_KNN_DIST = 3,    /* double[N*kappa]: squared distances, ascending per row */
    ASKIT_X_NODES = 4,       /* askit_node[num_nodes] */
    ASKIT_X_NLIST_POS = 5,   /* int32[num_nodes*l]: node neighbour lists (tree positions) */
    ASKIT_X_NLIST_KEY = 6,   /* double[num_nodes*l] */
    ASKIT_X_NLIST_CNT = 7,   /* int32[num_nodes] */
    ASKIT_X_ROWS = 8,        /* int32[num_nodes*l]: sampled rows T_alpha (tree positions) */
    ASKIT_X_ROWS_CNT = 9,    /* int32[num_nodes] */
    ASKIT_X_SKEL = 10,       /* int32[num_nodes*s_max]: skeleton (tree positions) */
    ASKIT_X_SKEL_K = 11,     /* int32[num_nodes]: skeleton sizes */
    ASKIT_X_COLPERM = 12,    /* int32[num_nodes*ncol_max]: ID column pivot order */
    ASKIT_X_NCOLS = 13,      /* int32[num_nodes]: ID column counts */
    ASKIT_X_PROJ = 14,       /* float[num_nodes*s_max*ncol_max]: P_alpha, row stride ncols-k */
    ASKIT_X_SKEL_W = 15,     /* float[num_nodes*s_max*nrhs]: skeleton weights */
    ASKIT_X_SLAB_PTR = 16,   /* int32[2*num_slabs+2]: near offsets then far offsets (CSR) */
    ASKIT_X_SLAB_NODE = 17,  /* int32[near_entries+far_entries]: node ids, near block first */
    ASKIT_X_SLAB_MASK = 18,  /* uint64[near_entries+far_entries]: row masks */
    ASKIT_X_SLAB_ROW0 = 19,  /* int32[num_slabs]: first tree position of each slab */
    ASKIT_X_BANDWIDTH = 20,  /* double[N]: per-source bandwidth, original order */
    ASKIT_X_KNN_RETRY = 21   /* int32[knn_retry_rows]: tree positions of the rows whose kNN
                                filter output overflowed (any order) */
} askit_export_item;

/* Copies item `what` into host buffer `dst` of `cap` bytes; *bytes receives
 * the size needed (call with dst = NULL to query it). */
askit_status askit_export(const askit_handle *h, int32_t what, void *dst, size_t cap,
                          size_t *bytes);

/* ---------------------------------------------------------------------------
 * Serving.  A server keeps one setup resident (tree, skeletons, P_alpha and
 * interaction lists stay in device memory) and answers two kinds of request
 * with continuous batching:
 *   - weights: u = K w at all N points for the request's own weights (the
 *     per-iteration cost that setup amortizes, Sec. 4);
 *   - query:   u at M new points for the resident weights W0.
 * Requests are admitted against a device-memory budget; pending requests of
 * one kind are batched (weight columns side by side, query points stacked)
 * and run by `workers` threads, each on its own stream, so batches overlap on
 * the device.  Results are independent of the batch a request rides in: a
 * query's values are bit-identical to running it alone (its points are
 * sorted, cut into slabs and chunked among themselves only), a weight
 * request's columns agree to FP32 rounding (the contraction runs as wide as
 * the batch's columns).
 *
 * Cyclic weights (weight_passes = K > 0): weight requests go to one column
 * engine with a resident pool of max_batch_rhs columns instead of the
 * workers.  The evaluation's source-node chunks are cut into K ranges of
 * about equal pair counts, evaluated round robin, one range per pass, for
 * every column in flight; waiting requests are admitted into free columns
 * between passes (their upward pass runs then) and a request finishes after
 * K passes, whichever range it started at.  The pool (weights_bytes for
 * max_batch_rhs columns) is charged to mem_budget for the server's lifetime.
 * ------------------------------------------------------------------------- */
typedef struct askit_server askit_server;

typedef struct {
    uint32_t struct_size;       /* sizeof(askit_server_config) */
    int32_t workers;            /* concurrent batches, 1..16 */
    int32_t max_batch_rhs;      /* weight columns per batch, 1..64 */
    int32_t max_batch_queries;  /* query points per batch, >= 1 */
    uint64_t mem_budget;        /* device bytes for in-flight requests (0: 8 GiB) */
    int32_t weight_passes;      /* 0: weight requests batched whole by the workers;
                                   K in 1..4096: cyclic weights, K passes per cycle */
    int32_t max_pending;        /* queued requests beyond which submit returns
                                   ASKIT_ERR_BUSY (0: no limit) */
} askit_server_config;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t deferred;           /* requests that reached the queue head and waited for memory */
    int64_t batches, batched_requests;   /* cyclic weights: passes that admitted
                                            requests, and the requests admitted */
    double p50_ms, p99_ms, mean_ms;                 /* submit -> result ready, all requests */
    double p50_weights_ms, p99_weights_ms, p50_query_ms, p99_query_ms;
    double targets_rhs;         /* sum over completed requests of targets x RHS */
    double busy_s;              /* wall time from first submit to last completion */
    uint64_t peak_mem;          /* largest admitted total */
    int64_t joined_mid_cycle;   /* cyclic weights: requests admitted while other
                                   columns were part way through their cycle */
} askit_serving_stats;

/* Fills *c with defaults: 2 workers, 64 columns, 65536 points, 8 GiB, whole
 * weight batches (weight_passes 0), no queue limit. */
askit_status askit_server_config_default(askit_server_config *c);

/* Creates a server over a set-up handle (the handle must outlive the server
 * and must not be used by the caller meanwhile).  W0 (device, N x nrhs0,
 * original point order, row stride ldw0) are the resident weights of query
 * requests; they are copied. */
askit_status askit_server_create(askit_handle *h, const float *W0, int64_t ldw0, int32_t nrhs0,
                                 const askit_server_config *cfg, askit_server **out);

/* Weight request: W (device, N x nrhs, stride ldw) in, U (device, N x nrhs,
 * stride ldu) out.  Both must stay valid until the request completes, and W
 * must already hold its values (work that writes it has finished): the
 * server reads it on its own streams, unordered with the caller's.
 * ASKIT_ERR_OUT_OF_MEMORY if the request alone exceeds the budget (batch
 * mode; in cyclic mode the pool is charged at creation), ASKIT_ERR_BUSY if
 * max_pending requests are already queued (both kinds count). */
askit_status askit_server_submit_weights(askit_server *s, const float *W, int64_t ldw, int32_t nrhs,
                                         float *U, int64_t ldu, uint64_t *ticket);

/* Query request: Y (device, M x d, stride ldy) in, U (device, M x nrhs0,
 * stride ldu) out; valid until completion, Y already written (as above). */
askit_status askit_server_submit_query(askit_server *s, const float *Y, int64_t M, int64_t ldy,
                                       float *U, int64_t ldu, uint64_t *ticket);

/* *state: 0 pending, 1 done, -1 failed (askit_last_error() then describes the failure). */
askit_status askit_server_poll(askit_server *s, uint64_t ticket, int32_t *state);
/* Waits up to timeout_s seconds (< 0: no limit). */
askit_status askit_server_wait(askit_server *s, uint64_t ticket, double timeout_s, int32_t *state);
askit_status askit_server_stats(askit_server *s, askit_serving_stats *out);
/* Finishes pending requests, then stops the workers and frees the server. */
void askit_server_destroy(askit_server *s);

/* ---------------------------------------------------------------------------
 * Batched form.  Many independent problems (each with its own N and d, the
 * same parameters) behind one handle, for workloads of many small instances
 * where one launch per instance would leave the device idle.  The work per
 * weight vector (permutation, upward pass, evaluation: the per-iteration cost
 * of Sec. 4 that setup amortizes) runs as a few launches over all instances;
 * every instance's result is the one askit_setup/askit_update_weights/
 * askit_evaluate give for it alone (same kernels, same arithmetic).
 *
 * Row layout: W and U hold the rows of instance 0, then instance 1, ... in
 * each instance's original point order (instance i starts at row
 * N_0 + ... + N_{i-1}); nrhs columns, row strides ldw / ldu.
 * ------------------------------------------------------------------------- */
typedef struct askit_batch askit_batch;

typedef struct {
    int32_t count, nrhs;
    int64_t total_points, total_chunks;   /* chunks: evaluation work items of up to 64 targets */
    int64_t near_entries, far_entries, near_pairs, far_pairs;
    double t_setup_ms;
    double t_skel_ms;           /* of which the fused skeletonization of all instances (the
                                   instances' own t_skel_ms read 0) */
    int32_t tuned;              /* 1 once a launch shape is chosen for nrhs */
    int32_t launch_blocks;      /* chosen shape: 0 = one workgroup per slab, else persistent grid size */
    int32_t launch_plan;        /* chosen column tiles: 0 wide (64 or 32 columns per MFMA pass, 4 or 1
                                   per vector pass), 1 narrow (32 per MFMA pass, 1 per vector pass) */
    int32_t reserved;
    double candidate_ms[8];     /* evaluation time of plan 0, then plan 1, each with: one workgroup
                                   per slab; persistent 2, 4, 8 per CU */
    int32_t graphs;             /* cached graphs of askit_batch_run */
} askit_batch_info;

/* Sets up `count` instances: X[i] (device, N[i] x d[i], row stride ldx[i])
 * with the parameters *p.  Synchronises `stream` (the point sets must be
 * written), then builds the instances up to their skeletons several at a
 * time on worker streams, and the skeletons of all instances in one fused
 * pass over the tree levels on `stream` (every kernel of Alg. 3 launched once
 * per level for the nodes of every instance); the point sets are copied.
 * Errors name the failing instance. */
askit_status askit_batch_setup(int32_t count, const float *const *X, const int64_t *N, const int32_t *d,
                               const int64_t *ldx, const askit_params *p, void *stream, askit_batch **out);

/* Skeleton weights of every instance from W (device, rows as above). */
askit_status askit_batch_update_weights(askit_batch *b, const float *W, int64_t ldw, int32_t nrhs,
                                        void *stream);

/* u of every instance into U (device, rows as above).  Uses the launch shape
 * the tuner chose for nrhs, else one workgroup per slab with wide tiles. */
askit_status askit_batch_evaluate(askit_batch *b, float *U, int64_t ldu, void *stream);

/* update_weights + evaluate as one HIP graph, replayed on `stream`.  The first
 * call for an nrhs in a problem class -- the bucket (largest padded d, leaf
 * size m, s_max, nrhs, precision) -- times the evaluation's 8 launch shapes
 * (2 column-tile plans x 4 grid forms, eagerly, on `stream`) and keeps the
 * fastest for every later batch of that bucket in the process; every shape
 * gives bit-identical results.  The graph is captured once per (W, ldw,
 * nrhs, U, ldu) and replayed afterwards, so later calls must pass buffers
 * that are still allocated (new values in the same buffers are fine). */
askit_status askit_batch_run(askit_batch *b, const float *W, int64_t ldw, int32_t nrhs, float *U, int64_t ldu,
                             void *stream);

/* Fixes the evaluation's launch shape for nrhs instead of timing them:
 * blocks = 0 for one workgroup per slab, else the persistent grid size
 * (1 .. 64 x compute units); plan 0 (wide) or 1 (narrow) column tiles.
 * Graphs captured before keep their shape. */
askit_status askit_batch_set_launch(askit_batch *b, int32_t nrhs, int32_t blocks, int32_t plan);

askit_status askit_batch_get_info(const askit_batch *b, askit_batch_info *out);

/* Instance i's handle (owned by the batch; for exports and queries), NULL if out of range. */
askit_handle *askit_batch_instance(askit_batch *b, int32_t i);

/* Waits for the device, then frees the batch and its instances. */
void askit_batch_destroy(askit_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* ASKIT_H */
