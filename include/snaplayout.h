/*
 * snaplayout.h -- C ABI of the MI355X (gfx950) SNAP-tFDP layout library.
 *
 * The library lays out an undirected graph in 2D with the edge-centric
 * negative-sampling method of SNAP-tFDP: per epoch, every directed edge
 * (i, j) applies a bounded t-distribution attraction to the pair, then draws k
 * negative nodes uniformly from V \ {i} and applies the bounded t-distribution
 * repulsion to each (i, s), with immediate lock-free updates and a step size
 * that decays linearly over the epochs.
 *   - method and pair updates: Algorithm 1 and Sec. 3.3 of the paper;
 *   - forces: Table 1, t-FDP row (alpha = 0.1, beta = 8, gamma = 2, Sec. 3.1);
 *   - the implicit weight k (d_i + d_j) / (|V| - 1) of the sampled repulsion:
 *     Sec. 3.3 (expected force), Eq. (5) (linear normalised degree weight);
 *   - lock-free bundles (all out-edges of a source in one worker): Sec. 3.4.
 *
 * Conventions shared by every entry point
 *   - Graph input is CSR with int32 indices: row_ptr[n+1], col_idx[nnz].  Each
 *     undirected edge must appear in both directions (Sec. 3.3), rows sorted
 *     strictly increasing, no self-loops, no duplicates; nnz = row_ptr[n] <
 *     2^31 (layout_create64 takes int64 row pointers for larger graphs).
 *     Isolated nodes are allowed (they are drawn as negatives only).
 *   - Positions are float32, row-major n x 2 (x0, y0, x1, y1, ...).
 *   - Unless stated otherwise, pointers are host pointers owned by the caller
 *     and only read during the call; the library copies what it keeps.
 *   - Every function returns LAYOUT_OK (0) or a negative LAYOUT_E_* code and,
 *     on error, sets a thread-local message readable with layout_last_error().
 *     No C++ exception crosses the ABI.
 *   - A layout handle is not thread-safe: one thread at a time per handle.
 *   - Device faults are sticky for the process (HIP context); the library
 *     reports them as LAYOUT_E_DEVICE and cannot recover them in-process.
 */
#ifndef SNAPLAYOUT_H
#define SNAPLAYOUT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LAYOUT_OK = 0,
    LAYOUT_E_INVALID_ARG = -1, /* a scalar argument or pointer is out of range */
    LAYOUT_E_BAD_GRAPH = -2,   /* the CSR violates the conventions above */
    LAYOUT_E_OOM = -3,         /* device memory allocation failed */
    LAYOUT_E_DEVICE = -4,      /* a HIP runtime call failed */
    LAYOUT_E_DONE = -5,        /* all epochs of the schedule have run */
    LAYOUT_E_UNSUPPORTED = -6  /* valid request the library does not implement */
};

/* How concurrent position updates are committed (Sec. 3.4 lock-free scheme). */
enum {
    LAYOUT_HOGWILD_STORE = 0, /* device-scope plain stores; racing updates may be lost */
    LAYOUT_ATOMIC = 1,        /* device-scope float atomic adds; no update lost */
    LAYOUT_JACOBI = 2,        /* test mode: all pair forces from epoch-start positions */
    LAYOUT_UPDATE_AUTO = 3    /* ATOMIC on the LDS engine, HOGWILD_STORE on the others */
};


/* Initial layout when no positions are given. */
enum {
    LAYOUT_INIT_UNIFORM = 0, /* seeded uniform in [-sqrt(n), sqrt(n)]^2 */
    LAYOUT_INIT_PMDS = 1     /* Pivot MDS (Sec. 4.1), see layout_pmds */
};

/* Kernel of the forces (layout_opts.force_kernel). */
enum {
    LAYOUT_FORCE_T = 0,       /* Table 1, t-FDP row (Student-t kernel): the paper's method */
    LAYOUT_FORCE_GAUSSIAN = 1 /* Gaussian kernel variant (future work in the conclusion) */
};

/* Distribution of the negatives. */
enum {
    LAYOUT_NEG_UNIFORM = 0, /* uniform over V \ {i}: the paper's method (Algorithm 1) */
    LAYOUT_NEG_DEGREE = 1,  /* proportional to degree via an alias table (control);
                               needs nnz < 2^32 (the table's capacity W = nnz), else
                               LAYOUT_E_UNSUPPORTED */
    LAYOUT_NEG_CUSTOM = 2   /* proportional to the caller's integer weights w (opts
                               neg_weight_values, 0 < sum w < 2^32), drawn like DEGREE: an
                               alias table over w, a draw equal to the source rejected;
                               the more flexible negative sampling the conclusion names
                               as future work; single-graph layouts only */
};

/* Which kernel family runs the epochs. */
enum {
    LAYOUT_ENGINE_AUTO = 0,   /* LDS for small graphs, XCD-local for graphs whose positions
                                 fit one XCD's L2, global otherwise */
    LAYOUT_ENGINE_GLOBAL = 1, /* positions in device memory, all CUs */
    LAYOUT_ENGINE_LDS = 2,    /* positions in one workgroup's LDS (n * 8 B must fit) */
    LAYOUT_ENGINE_XCD = 3     /* positions in device memory, each epoch on the CUs of one
                                 XCD (accelerator complex die) with plain loads/stores that
                                 hit its L2; HOGWILD_STORE only; n * 8 B <= 3 MiB */
};

typedef struct layout layout_t;

typedef struct layout_opts {
    float alpha, beta, gamma; /* t-force parameters, defaults 0.1, 8, 2 (Table 1); gamma > 1
                                 (> 0 with LAYOUT_FORCE_GAUSSIAN) */
    float eta0;               /* initial step; eta_t = eta0 * (1 - t / epochs); default 1 */
    int32_t update_mode;      /* LAYOUT_UPDATE_AUTO (default) / LAYOUT_HOGWILD_STORE /
                                 LAYOUT_ATOMIC / LAYOUT_JACOBI */
    int32_t neg_weights;      /* LAYOUT_NEG_UNIFORM (default) / LAYOUT_NEG_DEGREE */
    int32_t engine;           /* LAYOUT_ENGINE_* (default AUTO) */
    int32_t start_epoch;      /* resume point in [0, epochs]; default 0 */
    int32_t bundle_edges;     /* target directed edges per lane chunk (whole rows); 0 = default */
    int32_t block_threads;    /* threads per workgroup; 0 = automatic (see nodes_per_lane) */
    int32_t grid_blocks;      /* workgroups of the epoch kernel; 0 = automatic: at most one
                                 256-lane workgroup per CU and n / nodes_per_lane lanes */
    int32_t hub_split_edges;  /* rows with more edges are split into segments of this many
                                 edges, one lane each; 0 = default (4 * bundle_edges on the
                                 global and XCD-local engines, 64 on the LDS engine) */
    int32_t nodes_per_lane;   /* concurrency cap of the automatic launch shape: lanes in
                                 flight <= n / nodes_per_lane on the global and XCD-local
                                 engines (workgroups of that many lanes rounded up to 64, at
                                 most 256), working lanes = n / nodes_per_lane rounded up to 64
                                 on the LDS engine, so that few concurrent updates hit one node
                                 (Sec. 3.4); 0 = default 32 */
    int32_t init_mode;        /* LAYOUT_INIT_UNIFORM (default) / LAYOUT_INIT_PMDS; ignored
                                 when init_pos is given */
    int32_t pmds_pivots;      /* pivots of LAYOUT_INIT_PMDS, 1..64; 0 = default 50 */
    const float *init_pos;    /* n*dim initial positions (host, or device when the
                                 inputs are on the device); NULL = init_mode */
    void *stream;             /* hipStream_t for all work of the handle; NULL = a
                                 stream owned by the library */
    const uint32_t *neg_weight_values; /* LAYOUT_NEG_CUSTOM: n weights (host, or device when
                                 the inputs are on the device), copied at create */
    int32_t hot_degree;       /* HOGWILD_STORE on the global engine: the update a node
                                 receives as the far end of an edge is committed as an
                                 atomic add of its change, not a store, when the node's
                                 degree is at least this (concurrent stores to such nodes
                                 collide and lose updates; Sec. 3.4 assumes they are rare).
                                 0 = never (default: plain stores only); negative is
                                 LAYOUT_E_INVALID_ARG.  Ignored by the other engines and
                                 policies */
    int32_t force_kernel;     /* LAYOUT_FORCE_T (default): Table 1's t-FDP forces;
                                 LAYOUT_FORCE_GAUSSIAN: the same forces with the Gaussian
                                 kernel exp(-|d|^2/2) in place of 1/(1+|d|^2) (the conclusion's
                                 Gaussian-based forces): A(d) = alpha (1 + beta exp(-|d|^2/2))
                                 d, R(d) = exp(-gamma |d|^2 / 2) d, gamma > 0.  The energy
                                 monitors take the t-FDP forces only (E_UNSUPPORTED) */
} layout_opts;

/* Fills *opts with the defaults listed above. */
void layout_opts_init(layout_opts *opts);

/* Pivot MDS layout of one graph (the initial layout of Sec. 4.1; Brandes and
 * Pich, GD 2006), also used by layout_create_ex when init_mode is
 * LAYOUT_INIT_PMDS.  Definition: the first pivot is the node of largest degree
 * (smallest index on ties); each further pivot is the node of the first
 * pivot's connected component farthest (in hops) from the pivots chosen so far
 * (smallest index on ties); min(pivots, component size) pivots.  With d_ij the
 * hop distance from pivot j to node i and C the double-centred matrix
 * -1/2 (d_ij^2 - column mean - row mean + grand mean) over the component,
 * v1, v2 the eigenvectors of the two largest eigenvalues mu1, mu2 of C^T C,
 * the component's coordinates are s (C v1 / mu1^(1/4), C v2 / mu2^(1/4)),
 * with s the least-squares fit of |y_i - y_pivot| to d_ij (an axis with
 * mu <= 1e-6 mu1 is 0).  Nodes outside the
 * component take the seeded uniform draws of the plain init (seed) in
 * [-R, R]^2, R = the largest |coordinate| of the component layout.
 * row_ptr/col_idx: host arrays, or device arrays if inputs_on_device = 1 (a
 * valid CSR as for layout_create; validated on the device).  pivots: 1..64,
 * 0 = 50.  Y_out: host n*2 FP32 (x, y interleaved).  pivots_out (nullable):
 * host [pivots], the pivots in order of choice.  dist_out (nullable): host
 * [pivots * n] int32, row j = hop distances from pivot j (-1 = unreachable).
 * *pivots_used (nullable) = pivots taken.  Blocking; device memory is
 * allocated for the call (pivots x n int32 distances) and freed before return.
 * Errors: E_INVALID_ARG, E_BAD_GRAPH, E_OOM, E_DEVICE. */
int layout_pmds(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t pivots,
                uint64_t seed, int32_t inputs_on_device, float *Y_out, int32_t *pivots_out,
                int32_t *dist_out, int32_t *pivots_used);

/* Creates a layout job with default options.  Validates the CSR on the device,
 * builds the chunk table, initialises positions.  Returns when the job is
 * ready.  row_ptr/col_idx: host arrays (copied).  dim: 2 (the paper's
 * layouts), or 3 (the same force law with q = |y_i - y_j|^2 over three
 * coordinates; positions are held as 16-byte (x, y, z, unused) entries on the
 * device and exchanged as n*3 floats); other values E_UNSUPPORTED.  A 3D job
 * has no Pivot MDS start and no 2D monitors (energies, silhouette, NP, gather
 * roofline: E_UNSUPPORTED).  k in [0, 8].  epochs >= 1.  seed keys every
 * random draw (init and negatives); the 3D init draws the third coordinate
 * from the third word of the node's init block. */
int layout_create(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t dim,
                  int32_t k, int32_t epochs, uint64_t seed, layout_t **out);

/* As layout_create, with options.  inputs_on_device = 1: row_ptr, col_idx and
 * opts->init_pos are device pointers (the caller keeps them alive until this
 * call returns; they are copied). */
int layout_create_ex(const int32_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t dim,
                     int32_t k, int32_t epochs, uint64_t seed, const layout_opts *opts,
                     int32_t inputs_on_device, layout_t **out);

/* As layout_create_ex with 64-bit row pointers (row_ptr: n+1 int64), for
 * graphs of 2^31 or more directed edges (the com-friendster shape of the
 * paper's case study: 1.8 billion undirected edges).  Internally every graph
 * uses 64-bit row pointers and chunk starts; the int32 entry points widen
 * theirs on the device.  Chunk indices stay 32-bit: a graph whose chunk
 * table (about nnz / bundle_edges + 2 nnz / hub_split_edges entries) would
 * exceed 2^31 - 2^24 entries is refused with LAYOUT_E_UNSUPPORTED before any
 * allocation (the defaults, 16 and 64, allow about 2.3 x 10^10 edges); the
 * degree-weighted alias table needs nnz < 2^32. */
int layout_create64(const int64_t *row_ptr, const int32_t *col_idx, int32_t n, int32_t dim,
                    int32_t k, int32_t epochs, uint64_t seed, const layout_opts *opts,
                    int32_t inputs_on_device, layout_t **out);

/* Enqueues min(count, remaining) epochs on the handle's stream and returns
 * without waiting.  Returns LAYOUT_E_DONE when no epoch remains. */
int layout_epoch(layout_t *L, int32_t count);

/* As layout_epoch, then waits and reports the device time of the enqueued
 * epoch kernels (HIP events on the handle's stream) in *ms. */
int layout_epoch_timed(layout_t *L, int32_t count, float *ms);

/* Copies the n*dim positions (row-major FP32) to host memory; waits for the
 * handle's stream. */
int layout_get_positions(const layout_t *L, float *host_out);

/* Copies the n*dim positions to a device buffer, ordered after the handle's
 * work; stream = NULL uses the handle's stream.  Does not wait. */
int layout_get_positions_device(const layout_t *L, float *dev_out, void *stream);

/* Overwrites the positions from host memory (n*dim floats); waits. */
int layout_set_positions(layout_t *L, const float *host_in);

/* Epochs run so far and device bytes held by the handle (either may be NULL). */
int layout_status(const layout_t *L, int32_t *epochs_done, int64_t *device_bytes);

/* Waits for all work enqueued on the handle. */
int layout_sync(layout_t *L);

/* Frees the handle and its device memory (waits first).  NULL is ignored. */
void layout_destroy(layout_t *L);

/* Message of the last error on the calling thread ("" if none). */
const char *layout_last_error(void);

/* ---- test and measurement support ------------------------------------- */

typedef struct layout_info {
    int32_t engine;        /* engine chosen for the epochs */
    int32_t bundle_edges;  /* B */
    int32_t block_threads;
    int32_t grid_blocks;
    int64_t n_chunks;      /* chunks of the row-aligned chunk table */
    int64_t nnz;
    int32_t n, k;
    int32_t epochs, update_mode; /* the resolved policy (never AUTO) */
    int32_t hub_split_edges;
    int32_t hot_degree;    /* resolved hot-node threshold; 0 = no hot nodes */
} layout_info;

int layout_get_info(const layout_t *L, layout_info *info);

/* ---------------------------------------------------------- energy monitors
 * The t-forces of Table 1 are the negative gradients (Eq. (2)) of the pair
 * potentials U_a(q) = alpha (q/2 + (beta/2) ln(1+q)) and
 * U_r(q) = (1+q)^(1-gamma) / (2 (gamma-1)) of the squared distance q.  Both
 * calls read the handle's current positions after the epochs already
 * launched, accumulate in FP64 (terms in FP32), and return when the values
 * are on the host.  The first call allocates 16 bytes of device memory that
 * the handle keeps. */

/* Energy that the samples of one epoch see (Sec. 3.3): *attr_out = sum over
 * the directed edges (i, j) of U_a(|y_i - y_j|^2); *rep_out = sum over the
 * directed edges e = (i, .) and the k negatives s drawn for e in epoch
 * `epoch` (the same draws as the epoch kernel) of U_r(|y_i - y_s|^2).
 * O(nnz (1 + k)).  Errors: NULL outputs or epoch < 0 -> E_INVALID_ARG. */
int layout_sampled_energy(layout_t *L, int32_t epoch, double *attr_out, double *rep_out);

/* The degree-weighted objective that the sampling realises in expectation
 * (Eq. (4) with the weight of Sec. 3.3): *attr_out as above (each undirected
 * edge counted in both directions), *rep_out = k/(n-1) * sum over unordered
 * pairs {i, j} of (d_i + d_j) U_r(|y_i - y_j|^2).  O(n^2): meant for graphs of
 * up to a few hundred thousand nodes.  The mean of layout_sampled_energy over
 * epochs at fixed positions tends to this value.  Errors as above. */
int layout_effective_energy(layout_t *L, double *attr_out, double *rep_out);

/* Silhouette index of the current positions for the clusters given by
 * labels (host int32[n], any values; at least 2 distinct, else
 * E_INVALID_ARG): the mean over all nodes of (b_i - a_i) / max(a_i, b_i),
 * a_i the mean distance to the other members of i's cluster, b_i the
 * smallest mean distance to another cluster, 0 for a node alone in its
 * cluster (the SI metric of Sec. 4.1, exact over all pairs rather than on a
 * node sample).  O(n^2) on the device: about 15 ms for 259k nodes.
 * Allocates and frees temporary device memory. */
int layout_silhouette(layout_t *L, const int32_t *labels, double *si_out);

/* Largest node count layout_silhouette_noalloc takes. */
#define LAYOUT_NOALLOC_MAX_NODES (1 << 18)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * silhouette of layout_silhouette, the same kernels and result, with its
 * working memory (5 MiB) in a fixed device array that each GPU holds for the
 * life of the process instead of temporary allocations; it allocates no
 * device memory.  n <= LAYOUT_NOALLOC_MAX_NODES, else LAYOUT_E_UNSUPPORTED.
 * Calls that overlap on one GPU (other threads or streams) share the array
 * and race; each call clears what must start at zero.  Synchronises the
 * handle's stream.  Other errors as layout_silhouette. */
int layout_silhouette_noalloc(layout_t *L, const int32_t *labels, double *si_out);

/* Neighbourhood preservation of the current positions at the listed query
 * nodes (the NP metric of Sec. 4.1, exact for each query rather than through
 * a spatial index).  For query i: R_i = the nodes at hop distance 1..radius
 * from i (i excluded; radius 1 or 2, else E_INVALID_ARG), k_i = |R_i|, and
 * K_i = the k_i nodes nearest to y_i (i excluded), ranked by the FP32
 * squared distance fl(fl(dx*dx) + fl(dy*dy)), dx = fl(y_l.x - y_i.x), ties
 * by node index.  nodes: host int32[count], each in [0, n), else
 * E_INVALID_ARG (repeats allowed).  k_out, inter_out: host int32[count],
 * receive k_i and |R_i ∩ K_i|.  np_out (nullable): the mean over the queries
 * with k_i > 0 of |R_i ∩ K_i| / |R_i ∪ K_i| (0 if there are none).  count = 0
 * is a no-op.  Cost per query: O(n) for the selection (about four passes over
 * the positions) plus O(sum of the ring's degrees); queries run in batches
 * whose bitmaps take at most 256 MiB of temporary device memory, allocated
 * and freed by the call.  Synchronises the handle's stream. */
int layout_neighbourhood(layout_t *L, const int32_t *nodes, int32_t count, int32_t radius,
                         int32_t *k_out, int32_t *inter_out, double *np_out);

/* Clustering quality of the current positions (the CQ metric of Sec. 4.1):
 * k-means of the layout, then the adjusted Rand index (Hubert and Arabie)
 * between the clusters and labels (host int32[n], any values).
 *   clusters: K, 0 = the number of distinct labels; 1 <= K <= min(n, 4096),
 *     and labels x K <= 2^27, else E_INVALID_ARG.
 *   init_centers (nullable): host K x 2 FP32 starting centers.  NULL = a
 *     k-means++ start (Arthur and Vassilvitskii) drawn from seed.  The first
 *     center is point floor(x_0 n / 2^64).  Center c is the first point
 *     whose running sum of D^2 (FP64, in node order) exceeds
 *     u_c * sum(D^2), with u_c = (x_c >> 11) 2^-53 and x_c word x0 of
 *     Philox block (c, 0, 0, 4).
 *   Lloyd's iterations: nearest center by FP64 squared distance (lowest
 *     index on ties); centers move to their clusters' means (an empty
 *     cluster keeps its center).  They stop when an assignment after the
 *     first changes nothing, or after max_iter (>= 1) passes.
 *   cq_out: the ARI (1 when both partitions are trivial in the same way).
 *   Optional outputs (host): assign_out int32[n], the final clusters;
 *     iters_out, the assignment passes; centers_out int32[K], the k-means++
 *     points (-1 when init_centers is given).
 * 2D handles only (E_UNSUPPORTED for 3D).  Allocates and frees temporary
 * device memory; synchronises the handle's stream. */
int layout_cluster_quality(layout_t *L, const int32_t *labels, int32_t clusters, uint64_t seed,
                           int32_t max_iter, const float *init_centers, double *cq_out,
                           int32_t *assign_out, int32_t *iters_out, int32_t *centers_out);

/* Writes the k negatives the epoch kernels draw for every directed edge in
 * epoch t (host array nnz*k, int32, edge-major).  Does not change positions. */
int layout_debug_draws(layout_t *L, int32_t epoch, int32_t *host_out);

/* The negatives of the listed directed edges only (host edges[count], each
 * in [0, nnz), else E_INVALID_ARG; host_out count*k int32, edge-major), for
 * graphs too large to dump every edge.  Does not change positions. */
int layout_debug_draws_at(layout_t *L, int32_t epoch, const int64_t *edges, int64_t count,
                          int32_t *host_out);

/* Conflict counter: runs min(count, remaining) epochs like layout_epoch,
 * through an instrumented copy of the epoch (slower; same chunks, draws and
 * launch shape) that keeps a version word per node.  *stores = position
 * writes; *conflicts = writes that followed another lane's write of the same
 * node since this lane loaded it (a lost update under HOGWILD_STORE, a
 * change computed from a stale read under ATOMIC: the conflicts of the
 * lock-free scheme, Sec. 3.4); *untracked = writes whose load the counter no
 * longer held (source commits of long runs without a reload).  2D layouts on
 * the global engine, lock-free policies (else E_UNSUPPORTED).  Synchronises;
 * allocates a version word per node for the call. */
int layout_debug_conflicts(layout_t *L, int32_t count, int64_t *stores, int64_t *conflicts,
                           int64_t *untracked);

/* Atomic probe: every lane of a launch of 8 workgroups (256 lanes) per CU
 * adds 1, reps times, at device scope to one FP64 and one u64 counter
 * (spread = 0), or each lane to its own pair of counters (spread = 1).
 * *fsum_out and *isum_out receive the totals, *adds_out the number of adds
 * per counter kind (exact totals show atomic visibility across the XCDs),
 * *ms the launch time.  Allocates and frees its counters. */
int layout_bench_atomics(int32_t reps, int32_t spread, double *fsum_out, int64_t *isum_out,
                         int64_t *adds_out, float *ms);

/* Copies the chunk table: begin[n_chunks + 1] (int64, first directed edge of
 * each lane chunk, begin[n_chunks] = nnz) and src[n_chunks] (row holding
 * that edge).  n_chunks comes from layout_get_info. */
int layout_debug_chunks(const layout_t *L, int64_t *begin_out, int32_t *src_out);

/* Copies the alias table (n entries each) used by LAYOUT_NEG_DEGREE. */
int layout_debug_alias(const layout_t *L, uint32_t *thr_out, uint32_t *alias_out);

/* Modes of layout_bench_gather beyond LAYOUT_HOGWILD_STORE / LAYOUT_ATOMIC
 * (read-modify-writes): the reads alone, and (OR-ed in) the cache bits of
 * every position access instead of the epoch's device-scope ones. */
enum {
    LAYOUT_GATHER_READ = 4,          /* the 1 + k random reads, no write */
    LAYOUT_GATHER_PLAIN = 0x10,      /* plain (L2-cached, not device-coherent) */
    LAYOUT_GATHER_NONTEMPORAL = 0x20 /* non-temporal */
};

/* Random-gather roofline of the handle's graph: the memory pattern of one
 * epoch (stream col; per directed edge one position access at col[e] and k
 * at hashed uniform nodes; the source per chunk) without force arithmetic or
 * generator, at the epoch's launch shape.  mode: LAYOUT_HOGWILD_STORE or
 * LAYOUT_ATOMIC (read-modify-writes, every touched position written), or
 * LAYOUT_GATHER_READ (the same reads, nothing written: a lower bound on the
 * epoch's time), optionally OR LAYOUT_GATHER_PLAIN / _NONTEMPORAL (not with
 * ATOMIC).  Runs reps launches, reports the mean launch time in *ms.  The
 * read-modify-write modes perturb the positions slightly (use on a scratch
 * job).  Global-engine layouts only (E_UNSUPPORTED otherwise). */
int layout_bench_gather(layout_t *L, int32_t mode, int32_t reps, float *ms);

/* Streaming copy of bytes bytes between two device buffers allocated by the
 * library; mean time of reps launches in *ms (HBM roofline and counter
 * calibration). */
int layout_bench_copy(int64_t bytes, int32_t reps, float *ms);

/* ---- batched layout: many graphs in one launch --------------------------
 *
 * Lays out many independent graphs together (the same method per graph, each
 * with its own seed, so each graph draws exactly the samples it would draw
 * alone).  The CSRs are packed into one allocation.  Graphs whose positions fit
 * one workgroup's LDS run whole, all epochs, one workgroup each (the LDS
 * engine, ATOMIC under LAYOUT_UPDATE_AUTO).  The others share one launch per
 * epoch of the global engine (HOGWILD_STORE under LAYOUT_UPDATE_AUTO).  All
 * epochs of both groups are captured in one HIP graph and replayed by
 * layout_batch_run.  k and the epoch count are common to the batch. */

typedef struct layout_graph {
    const int32_t *row_ptr; /* n+1, host (or device when inputs_on_device) */
    const int32_t *col_idx; /* row_ptr[n] entries */
    int32_t n;
    int32_t reserved;
    uint64_t seed;          /* keys this graph's draws */
    const float *init_pos;  /* n*2 or NULL (opts->init_mode: seeded uniform or
                               Pivot MDS) */
    const uint32_t *neg_weight_values; /* n negative weights (host, or device when
                               inputs_on_device) when opts->neg_weights is
                               LAYOUT_NEG_CUSTOM (each graph: 0 < sum < 2^32),
                               else NULL */
} layout_graph;

typedef struct layout_batch layout_batch_t;

typedef struct layout_batch_info {
    int32_t graphs, lds_graphs, global_graphs, epochs;
    int64_t nodes, nnz, global_chunks, device_bytes;
    int32_t bundle_edges, hub_split_edges; /* of the global group */
    int32_t grid_blocks, block_threads;    /* of the global group */
    int32_t lds_block_threads, update_mode_global, update_mode_lds, epochs_done;
    int32_t xcd_engine;       /* 1: the global group runs on the XCD-local engine */
    int32_t xcd_grid_blocks;  /* its launch size (kXcds x the largest bin's workgroups) */
} layout_batch_info;

/* Creates a batch of count graphs (validated like layout_create).  opts as for
 * layout_create_ex; init_pos and start_epoch are ignored (per-graph init_pos
 * and caller weights live in layout_graph).  init_mode LAYOUT_INIT_PMDS runs
 * the Pivot MDS start of every graph without init_pos at create, one graph
 * after another.  Graphs that fit LDS run whole in one workgroup
 * each; with engine AUTO the others run on XCD-local bins when all of them
 * fit one XCD's L2 (HOGWILD_STORE, automatic launch shape),
 * else in one all-CU launch per epoch; engine GLOBAL forces that launch for
 * every graph, engine XCD requires the bins.  Returns when the batch is ready
 * to run. */
int layout_batch_create(const layout_graph *graphs, int32_t count, int32_t k, int32_t epochs,
                        const layout_opts *opts, int32_t inputs_on_device,
                        layout_batch_t **out);

/* Replays the captured epochs (all of them) on the batch's stream; returns
 * without waiting.  LAYOUT_E_DONE if the batch already ran. */
int layout_batch_run(layout_batch_t *B);

/* As layout_batch_run, then waits; *ms = device time of the replay. */
int layout_batch_run_timed(layout_batch_t *B, float *ms);

/* Copies graph g's n_g*2 positions to host memory (waits). */
int layout_batch_get_positions(const layout_batch_t *B, int32_t g, float *host_out);

/* Copies every graph's positions, packed in graph order (sum of n_g * 2
 * floats), to a device buffer, ordered after the batch's work; does not wait. */
int layout_batch_get_positions_device(const layout_batch_t *B, float *dev_out);

/* Waits for all work enqueued on the batch. */
int layout_batch_sync(const layout_batch_t *B);

/* Negatives graph g draws in epoch t (host int32[nnz_g * k]). */
int layout_batch_debug_draws(const layout_batch_t *B, int32_t g, int32_t epoch, int32_t *host_out);

int layout_batch_get_info(const layout_batch_t *B, layout_batch_info *info);

/* Launch-shape autotuner of the global group.  Times trial_epochs epochs for
 * every candidate (directed edges per chunk in {8, 16, 32} x workgroups per CU
 * in {2, 4, 8, occupancy limit}) on a scratch copy of the positions, keeps the
 * fastest, rebuilds the chunk tables and re-captures the epochs.  With
 * cache_path (a text file, created if absent) a result for the same device
 * architecture, k, policy and size class is reused without timing.  Results
 * in *bundle_out, *blocks_per_cu_out, *ms_out (any may be NULL).  Call before
 * layout_batch_run. */
int layout_batch_autotune(layout_batch_t *B, int32_t trial_epochs, const char *cache_path,
                          int32_t *bundle_out, int32_t *blocks_per_cu_out, float *ms_out);

/* Frees the batch (waits first).  NULL is ignored. */
void layout_batch_destroy(layout_batch_t *B);

/* ---- served layout: continuous batching of submitted jobs -----------------
 *
 * A server owns a scheduler thread and one device stream per class of job.
 * Jobs (a graph, k, epochs, seed) are submitted from any host thread and
 * copied at submission.  The scheduler admits queued jobs in arrival order
 * while a slot is free and the job's device footprint fits the HBM budget,
 * and keeps every admitted job's CSR, positions and chunk table resident on
 * the device.  Each class runs launches of its own, the next one as soon as
 * its last one has ended, independently of the other classes:
 *   - jobs whose positions fit one workgroup's LDS: up to ten of their
 *     remaining epochs per launch, one workgroup each (LDS engine);
 *   - jobs whose positions fit one XCD's L2 (engine AUTO or XCD,
 *     HOGWILD_STORE, automatic launch shape): a slice of each one's current
 *     epoch on XCD-local bins;
 *   - every other job: a slice of the current epoch of the oldest jobs whose
 *     lane caps (n / 32 each) fit the device's lanes together, plus later ones
 *     that still fit, in one multi-graph launch on all CUs; the others wait.
 * A launch's slices share at most round_edges directed edges, in proportion
 * to the jobs' sizes; an epoch may span launches.  When a job's last epoch
 * ends its positions are copied to host memory, its device memory is freed
 * and the next queued job can be admitted.  Latency is measured from
 * submission to positions-on-host.  The method per job is the same as
 * layout_create + layout_epoch (same draws for the same seed). */

typedef struct layout_server layout_server_t;

enum {
    LAYOUT_JOB_QUEUED = 0,
    LAYOUT_JOB_RUNNING = 1,
    LAYOUT_JOB_DONE = 2,
    LAYOUT_JOB_FAILED = 3,
    LAYOUT_JOB_CANCELLED = 4
};

typedef struct layout_server_stats {
    int64_t submitted, completed, failed, rejected;
    int64_t queued, running;
    int64_t hbm_in_use, hbm_budget; /* bytes */
    int64_t rounds;        /* launches that have ended, over all classes */
    double edge_updates;   /* sum over completed jobs of |E| (1 + k) epochs */
    double busy_seconds;   /* wall time with at least one job admitted */
    double p50_latency_s, p99_latency_s, mean_latency_s; /* over completed jobs */
    int64_t cancelled;
} layout_server_stats;

/* Starts a server.  hbm_budget_bytes: cap on the summed device footprint of
 * admitted jobs (0 = 90% of the free device memory at start).  max_slots:
 * cap on concurrently admitted jobs (>= 1).  round_edges: directed edges of
 * a launch's epoch slices (0 = default, 32M).  opts: as for
 * layout_create_ex (init_pos, start_epoch, stream are ignored).
 * opts->update_mode = LAYOUT_JACOBI (engine AUTO or GLOBAL) serves the
 * synchronous test mode of layout_create_ex: every job runs on the global
 * engine, its pair forces of one epoch summed (over the epoch's slices) into
 * a per-job accumulator before the positions move, so that a served job's
 * result is the plain path's Jacobi result up to FP32 summation order. */
int layout_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int64_t round_edges,
                         const layout_opts *opts, layout_server_t **out);

/* Queues a job; host arrays are copied before returning.  *job_id identifies
 * it.  Malformed arguments are rejected here (LAYOUT_E_INVALID_ARG); a CSR that
 * fails device validation ends as LAYOUT_JOB_FAILED with a message.  A job
 * larger than the whole budget is refused with LAYOUT_E_OOM.  Thread-safe. */
int layout_server_submit(layout_server_t *S, const int32_t *row_ptr, const int32_t *col_idx,
                         int32_t n, int32_t k, int32_t epochs, uint64_t seed, int64_t *job_id);

/* As layout_server_submit, with per-job inputs (host arrays, copied before
 * returning).  neg_weight_values: n weights, required exactly when the
 * server's opts->neg_weights is LAYOUT_NEG_CUSTOM (0 < sum < 2^32), else
 * NULL; otherwise LAYOUT_E_INVALID_ARG.  init_pos: n*2 initial positions or
 * NULL (the server's init_mode: seeded uniform, or Pivot MDS computed at
 * admission, which holds the scheduler for that job's PMDS time). */
int layout_server_submit_ex(layout_server_t *S, const int32_t *row_ptr, const int32_t *col_idx,
                            int32_t n, int32_t k, int32_t epochs, uint64_t seed,
                            const uint32_t *neg_weight_values, const float *init_pos,
                            int64_t *job_id);

/* Cancels a job.  A queued job ends at once; a running one is retired after
 * its launch in flight, its device memory freed.  Its state becomes
 * LAYOUT_JOB_CANCELLED; layout_server_wait then returns LAYOUT_E_INVALID_ARG
 * and layout_server_take forgets it.  A job that has already ended (or an
 * unknown id): LAYOUT_E_INVALID_ARG.  Thread-safe. */
int layout_server_cancel(layout_server_t *S, int64_t job_id);

/* Current state (LAYOUT_JOB_*) of a job.  Thread-safe. */
int layout_server_poll(layout_server_t *S, int64_t job_id, int32_t *state);

/* Waits until the job is DONE, FAILED or CANCELLED, or timeout_s passes (< 0: no limit);
 * returns LAYOUT_OK when it is DONE, LAYOUT_E_DEVICE/BAD_GRAPH for a failed
 * job (message in layout_last_error), LAYOUT_E_INVALID_ARG on timeout. */
int layout_server_wait(layout_server_t *S, int64_t job_id, double timeout_s);

/* Copies a DONE job's n*2 positions, reports its latency (seconds from
 * submission to positions on host) and forgets the job.  Thread-safe. */
int layout_server_take(layout_server_t *S, int64_t job_id, float *host_out, double *latency_s);

int layout_server_get_stats(layout_server_t *S, layout_server_stats *stats);

/* hold != 0: the scheduler keeps admitting queued jobs and setting up their
 * device state (copy, validation, chunk and alias tables, initial positions)
 * but starts no launch until hold = 0; running jobs pause once their
 * current launches end.
 * Thread-safe. */
int layout_server_hold(layout_server_t *S, int32_t hold);

/* Test support: the k negatives that a queued or running job draws in epoch
 * `epoch` for each of its nnz directed edges, host_out[e*k + m] (caller-owned,
 * nnz*k int32), computed on the device from the job's own device state (its
 * seed, size and alias table) by the scheduler between launches.  Blocks until
 * the job has been admitted and the request answered; with the server held
 * (layout_server_hold) the answer precedes the job's first epoch.  A job
 * that has already ended: LAYOUT_E_DONE.  Thread-safe (Algorithm 1; the draw
 * definition of layout_debug_draws). */
int layout_server_debug_draws(layout_server_t *S, int64_t job_id, int32_t epoch,
                              int32_t *host_out);

/* Stops the scheduler once the launches in flight have ended, frees every
 * job.  NULL is ignored. */
int layout_server_destroy(layout_server_t *S);

#ifdef __cplusplus
}
#endif

#endif /* SNAPLAYOUT_H */
