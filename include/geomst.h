/*
 * geomst — exact Euclidean minimum spanning trees and HDBSCAN* mutual
 * reachability MSTs on one AMD Instinct MI355X (gfx950).
 *
 * Method: Wang, Yu, Gu, Shun, "Fast Parallel Algorithms for Euclidean Minimum
 * Spanning Tree and Hierarchical Spatial Clustering" (SIGMOD 2021):
 * a well-separated pair decomposition over a k-d tree (Sec. 3.1.1, Alg. 1),
 * bichromatic closest pairs of the separated node pairs (Sec. 2.3), and a
 * filtered Kruskal that takes the pairs in rounds of growing weight
 * thresholds and materialises only the pairs a round needs (Sec. 3.1.2-3.1.3,
 * Alg. 2-3).  HDBSCAN* uses core distances from k-NN queries and the
 * "geometrically separated or mutually unreachable" separation of Sec. 3.2.2.
 *
 * Result definition (Sec. 2.1, "Problem Definitions"):
 *   EMST      the minimum spanning tree of the complete graph on the points
 *             with Euclidean edge weights.
 *   HDBSCAN*  cd(p) = distance from p to its minPts-nearest neighbour
 *             counting p itself; the MST of the complete graph weighted by
 *             d_m(p,q) = max{cd(p), cd(q), d(p,q)}.
 * Arithmetic: d(p,q)^2 is summed over the dimensions in order in IEEE
 * binary64 without fused multiply-add.  Edges are totally ordered by
 * K = (w^2, d^2, min id, max id) (w = d for EMST, w = d_m for HDBSCAN*), which
 * makes the tree unique; the library returns exactly that tree.
 *
 * Conventions for every call:
 *   - points are row-major float64 [n][d], 1 <= d <= 7, 1 <= n <= 2^26;
 *   - edges[k] = {min id, max id} (0-based row indices), int64 [n-1][2],
 *     sorted ascending by K; weights[k] = correctly rounded sqrt(w^2);
 *   - the caller owns every buffer; the library keeps no pointer after a
 *     call returns and allocates its own device scratch (kept per device and
 *     reused across calls);
 *   - calls on one device are serialised internally (thread-safe);
 *   - return 0 on success or a negative GEOMST_E* code; on error the outputs
 *     are unspecified and geomst_last_error() describes the failure.
 */
#ifndef GEOMST_H
#define GEOMST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEOMST_OK 0
#define GEOMST_EINVAL (-1)   /* bad size, dimension, minPts or NULL pointer */
#define GEOMST_EDOM (-2)     /* a coordinate is not finite or |x| > 2^500 */
#define GEOMST_ENOMEM (-3)   /* device or host allocation failed */
#define GEOMST_EDEVICE (-4)  /* a HIP runtime call failed */
#define GEOMST_EBUSY (-5)    /* reserved for a bounded request queue; not returned by this version */
#define GEOMST_ETIMEDOUT (-6)/* geomst_wait: the request is not done yet */
#define GEOMST_ECANCELED (-7)/* geomst_wait: the request was withdrawn by geomst_cancel */
#define GEOMST_EINTERNAL (-8)/* an internal consistency check failed */
#define GEOMST_ENOENT (-9)   /* unknown or already released ticket; missing tuning file */

/*
 * Euclidean MST of host-resident points (Sec. 2.1, EMST).
 *   points   [n][d] float64, host memory, read only
 *   edges    [n-1][2] int64 out (host), sorted by K
 *   weights  [n-1] float64 out (host), may be NULL
 * n = 1 succeeds with no edges.  Uses device 0's default scratch and an
 * internal stream; the copies to and from the device are included.
 */
int geomst_emst(const double* points, int64_t n, int32_t d, int64_t* edges, double* weights);

/*
 * HDBSCAN* core distances and mutual reachability MST of host-resident points
 * (Sec. 2.1, HDBSCAN*; Sec. 3.2.2).
 *   min_pts    1 <= min_pts <= min(n, 64): the k-NN keeps each query's k
 *              smallest distances in registers, and 64 covers the paper's
 *              range (minPts 10 in its tables, up to 50 in its sweep); a
 *              larger value returns EINVAL
 *   core_dist  [n] float64 out (host), cd of each input row; may be NULL
 *   edges      [n-1][2] int64 out (host), sorted by K = (w^2, d^2, min, max)
 *   weights    [n-1] float64 out (host), mutual reachability distances; may be NULL
 */
int geomst_hdbscan(const double* points, int64_t n, int32_t d, int32_t min_pts, double* core_dist,
                   int64_t* edges, double* weights);

/*
 * Device-pointer variants: every pointer is device memory on the current
 * HIP device (all may come from torch tensors); work is queued on `stream`
 * (a hipStream_t, NULL = the legacy default stream) and the call returns
 * after the results are complete on that stream.  Optional outputs may be
 * NULL:
 *   d_weights_sq     [n-1] w^2 exactly as ordered;
 *   d_core_dist_sq   [n]   cd^2.
 */
int geomst_emst_dev(const double* d_points, int64_t n, int32_t d, int64_t* d_edges, double* d_weights,
                    double* d_weights_sq, void* stream);
int geomst_hdbscan_dev(const double* d_points, int64_t n, int32_t d, int32_t min_pts, double* d_core_dist,
                       double* d_core_dist_sq, int64_t* d_edges, double* d_weights, double* d_weights_sq,
                       void* stream);

/*
 * Approximate OPTICS (Appendix, "Parallel Approximate OPTICS", after Gan and
 * Tao): the MST of the approximate base graph on a well-separated pair
 * decomposition with separation s = sqrt(8 / rho).  Each pair (A, B)
 * contributes the lightest of its base-graph edges, chosen by the Appendix's
 * four cases (a node is large when it holds at least min_pts points: small
 * with small joins every point pair, large with small joins the large node's
 * representative to every point of the other, large with large joins the two
 * representatives), weighted max{cd(u), cd(v), d(u, v) / (1 + rho)}; the
 * result is the MST of these candidates under K = (w^2, d^2, min, max).  A
 * node's representative is its first point in the spatial tree's order (the
 * paper draws it at random), so results are deterministic and repeatable.
 * Feeding the tree to geomst_dendrogram gives the approximate OPTICS
 * reachability plot.
 *   min_pts    1 <= min_pts <= min(n, 64)
 *   rho        approximation parameter, rho > 0 and finite (rho = 0.125 gives
 *              s = 8); the decomposition grows about as s^d pairs per
 *              point, so small rho in high d is costly
 *   core_dist  [n] float64 out, cd of each input row (cd^2 in the _sq output)
 *   edges      [n-1][2] int64 out, sorted by K
 *   weights    [n-1] float64 out, w = sqrt(w^2) correctly rounded (w^2 in
 *              the _sq output)
 * Errors as for geomst_hdbscan, plus EINVAL for rho outside (0, 1e300) and
 * ENOMEM when the decomposition exceeds 2^31 pairs.  The _dev variant takes
 * device pointers and queues on `stream`; the plain one host pointers.
 */
int geomst_optics_approx_dev(const double* d_points, int64_t n, int32_t d, int32_t min_pts, double rho,
                             double* d_core_dist, double* d_core_dist_sq, int64_t* d_edges, double* d_weights,
                             double* d_weights_sq, void* stream);
int geomst_optics_approx(const double* points, int64_t n, int32_t d, int32_t min_pts, double rho,
                         double* core_dist, int64_t* edges, double* weights);

/*
 * Ordered dendrogram and reachability plot of a weighted spanning tree
 * (Sec. 2.1, "dendrogram" and "reachability plot"; Sec. 4.1, the ordered
 * dendrogram of a start vertex; Sec. 4.2, the top-down heavy/light
 * construction).  Single-linkage clustering with the EMST as input, the
 * HDBSCAN* hierarchy with the mutual-reachability MST (a point is noise for
 * eps below its core distance).
 *   edges     [n-1][2] int64, the tree's edges in their total order (as the
 *             MST calls return them: edge k is the k-th lightest); the
 *             library takes this order as given
 *   weights   [n-1] float64, edge k's height (the MST calls' weights)
 *   start     the plot's first point s, 0 <= start < n
 *   children  [n-1][2] int64 out (may be NULL): internal node n + k merges,
 *             at height weights[k], the clusters {children[k][0],
 *             children[k][1]} (ids < n are points, ids >= n internal nodes);
 *             the left child [0] holds the endpoint of edge k nearer to s in
 *             the tree, so an in-order traversal lists the points in plot
 *             order
 *   size      [n-1] int64 out (may be NULL): points below node n + k
 *   order     [n] int64 out: Prim's visiting order from s on the tree
 *             (lightest edge leaving the visited set first)
 *   reach     [n] float64 out: reach[i] = the weight of the edge that reached
 *             order[i] (the smallest weight from it to any earlier point);
 *             reach[0] = +inf
 * EINVAL for a bad n or start, an endpoint outside [0, n), a self-loop, or
 * edges that do not form a spanning tree.  n = 1: order = {0}, reach = {inf}.
 * The _dev variant takes device pointers and queues on `stream` (returns
 * after the results are complete); the plain variant host pointers.
 */
int geomst_dendrogram_dev(const int64_t* d_edges, const double* d_weights, int64_t n, int64_t start,
                          int64_t* d_children, int64_t* d_size, int64_t* d_order, double* d_reach, void* stream);
int geomst_dendrogram(const int64_t* edges, const double* weights, int64_t n, int64_t start, int64_t* children,
                      int64_t* size, int64_t* order, double* reach);

/*
 * No-allocation variant of geomst_emst_dev, for callers that cannot allocate
 * device memory (code that must not call hipMalloc, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, result and stream
 * semantics as geomst_emst_dev; the caller still passes the inputs and
 * outputs.  Every internal buffer is carved from one fixed device array of
 * GEOMST_NOALLOC_SCRATCH_MIB MiB that the library holds on each device it
 * runs on until the process ends; counter read-backs go to static host
 * memory.  The call allocates nothing (no hipMalloc, hipFree, hipHostMalloc,
 * event or stream creation) and keeps no state between calls: the array keeps
 * the last call's contents and every call clears what it needs.
 *   - n > GEOMST_NOALLOC_MAX_POINTS: GEOMST_EINVAL before any device work.
 *   - a solve whose internal pair or edge lists outgrow the array (possible
 *     for large, high-dimensional or tightly clustered inputs):
 *     GEOMST_ENOMEM, with the array size in geomst_last_error().
 *   - calls on one device share its array: they are serialised by a lock and
 *     each returns only after its stream has finished, so two calls never use
 *     the array at once; a caller must not run two such calls' kernels
 *     concurrently by other means.  Kernel timing ("kernel_timing") is not
 *     recorded for this call.
 */
#define GEOMST_NOALLOC_MAX_POINTS 65536
#define GEOMST_NOALLOC_SCRATCH_MIB 512
int geomst_emst_dev_noalloc(const double* d_points, int64_t n, int32_t d, int64_t* d_edges, double* d_weights,
                            double* d_weights_sq, void* stream);

/*
 * Batched solve: `count` independent instances in one device arena, solved
 * together as a forest (one tree build and one set of round launches for all
 * of them; pairs never cross instances).  Results are exactly those of solving
 * each instance alone.
 *
 *   d_points   device f64 [N][stride], N = sum of n_i; instance i occupies rows
 *              [offset_i, offset_i + n_i) with offset_0 = 0 and
 *              offset_{i+1} = offset_i + n_i (packed in order).  Columns at and
 *              beyond the instance's d must be 0.0 (a zero coordinate leaves
 *              every squared distance bit-identical).
 *   items      host array of `count` descriptors (offset, n, d <= stride, min_pts:
 *              0 = EMST, else HDBSCAN* with 1 <= min_pts <= min(n, 64)).
 *   d_edges    device int64 [N - count][2]; instance i's n_i - 1 edges start at
 *              row offset_i - i, with ids local to the instance (0..n_i-1),
 *              sorted by K as in the single-instance calls.
 *   d_weights, d_weights_sq   device f64 [N - count] (either may be NULL).
 *   d_core_dist, d_core_dist_sq   device f64 [N] (may be NULL; 0 for EMST rows).
 *   stream     hipStream_t (NULL = legacy default stream).
 * Errors as for the single calls (EINVAL names the first bad item).
 */
typedef struct {
    int64_t offset;
    int64_t n;
    int32_t d;
    int32_t min_pts;
} geomst_batch_item_t;

int geomst_batch_dev(const double* d_points, int32_t stride, const geomst_batch_item_t* items, int64_t count,
                     int64_t* d_edges, double* d_weights, double* d_weights_sq, double* d_core_dist,
                     double* d_core_dist_sq, void* stream);

/* Host-pointer batch: per-instance host arrays, packed by the library. */
typedef struct {
    const double* points; /* [n][d] host, row-major */
    int64_t n;
    int32_t d;
    int32_t min_pts;      /* 0 = EMST */
    double* core_dist;    /* [n] out or NULL */
    int64_t* edges;       /* [n-1][2] out */
    double* weights;      /* [n-1] out or NULL */
    int32_t status;       /* out: GEOMST_OK or the error of this item */
} geomst_instance_t;

int geomst_batch(geomst_instance_t* inst, int64_t count);

/*
 * Serving: a request loop with continuous batching over independent EMST and
 * HDBSCAN* solves (each request is the problem of Sec. 2.1 on its own points).
 * Worker threads each own a device workspace and a stream.  Requests go to
 * one of two lanes by size: small ones (n <= small_max_points) are taken from
 * the lane's front, in arrival order, up to the worker's share of the
 * device-memory budget (hbm_budget_bytes / workers, by the estimate below)
 * and the batch limits, and solved like geomst_batch, one forest per group of
 * equal d; large ones, and every HDBSCAN* request (forests that mix minPts
 * values and densities ran slower than their members alone), are solved one
 * per worker at a time.  With several workers, worker 0 serves the small lane first and
 * the others the large lane, each taking from the other lane when its own is
 * empty; a single worker takes requests in arrival order.  Requests that
 * arrive while batches run are admitted as workers free up; the batches of
 * different workers overlap on the device.  Each result is the unique tree of
 * its own points, identical to solving it alone.
 *
 * Admission estimate per request (device bytes):
 *   n * (720 + 2 * node + 16 * d + (min_pts > 0 ? 640 : 0) + 16 * pairs[d]),
 *   node = 64 for d <= 3, else 128; pairs[d] = 24, 24, 64, 100, 200, 600,
 *   1600 for d = 1..7 (waiting and queued pairs per point at their peak).
 * A worker's workspace may hold at most hbm_budget_bytes / workers device
 * bytes (counted as its buffers grow, before they are allocated).  A batch
 * that would outgrow that share (the estimate can undercount the pair lists
 * of clustered or high-dimensional inputs), or that meets a device
 * allocation failure, makes the worker release its workspace and solve the
 * batch's requests one at a time (counted in enomem_batches).  Workspaces
 * only grow, up to their share, so the device memory a server's workspaces
 * hold never exceeds hbm_budget_bytes.
 */
typedef struct geomst_server geomst_server_t;

typedef struct {
    uint64_t hbm_budget_bytes;  /* 0 = 200 GB */
    int32_t workers;            /* concurrent batches, 1..16; 0 = 2 */
    int32_t device;             /* HIP device index; -1 = the caller's current */
    int32_t max_batch_requests; /* small-lane batches; 0 = 4096 */
    int32_t small_max_points;   /* requests with n <= this are "small"; 0 = 32768 */
    int64_t max_batch_points;   /* small-lane batch points; 0 = 2^20; at most 2^26 */
    const char* tuning_cache;   /* tuning cache to load (geomst_load_tuning), or NULL */
} geomst_server_cfg_t;

/* Timings of one request, filled by geomst_wait (milliseconds). */
typedef struct {
    int32_t status;         /* the request's result code */
    int32_t batch_requests; /* requests in the batch it ran in */
    int64_t batch_points;   /* points in that batch */
    double queue_ms;        /* submit -> its batch started */
    double service_ms;      /* batch start -> batch done (copies included) */
    double latency_ms;      /* submit -> done */
} geomst_request_info_t;

/* Server counters (a snapshot). */
typedef struct {
    int64_t submitted, queued, running, completed, batches;
    int64_t reserved_bytes;      /* estimate held by the running batches */
    int64_t peak_reserved_bytes;
    int64_t max_batch_requests, max_batch_points;
    int64_t enomem_batches;      /* batches that outgrew a worker's share and were re-solved one request at a time */
    int64_t workspace_bytes;     /* device bytes the workers' workspaces hold now */
} geomst_server_stats_t;

/* Creates a server; cfg may be NULL for the defaults.  EINVAL on bad fields,
 * EDEVICE if the device cannot be selected. */
int geomst_server_create(const geomst_server_cfg_t* cfg, geomst_server_t** out);

/* Queues one request.  req->points is copied, so the caller may reuse it at
 * once; req->edges, req->weights and req->core_dist (as in geomst_batch) must
 * stay valid until geomst_wait returns the request's result or geomst_cancel
 * returns.  req->status is set to the admission result.  EINVAL / EDOM as for
 * geomst_batch; ENOMEM if the request alone exceeds a worker's share of the
 * budget or the batch point limit. */
int geomst_submit(geomst_server_t* srv, geomst_instance_t* req, uint64_t* ticket);

/* Waits up to timeout_us microseconds (< 0: forever; 0: poll).  When the
 * request is done: fills info (may be NULL), releases the ticket and returns
 * the request's result code.  Otherwise returns ETIMEDOUT and keeps the
 * ticket.  ECANCELED (once) for a ticket withdrawn by geomst_cancel, also
 * when the withdrawal happens during the wait; ENOENT for an unknown or
 * already released ticket. */
int geomst_wait(geomst_server_t* srv, uint64_t ticket, int64_t timeout_us, geomst_request_info_t* info);

/* Withdraws a request and releases its ticket.  A queued request is removed
 * without running; one already in a batch is waited for (its outputs may have
 * been written).  A later (or concurrent) geomst_wait on the ticket returns
 * ECANCELED.  Returns OK, or ENOENT for an unknown ticket. */
int geomst_cancel(geomst_server_t* srv, uint64_t ticket);

int geomst_server_stats(geomst_server_t* srv, geomst_server_stats_t* out);

/* Finishes the running batches, drops the queued requests unsolved, joins the
 * workers and frees the workspaces.  Tickets become invalid. */
void geomst_server_destroy(geomst_server_t* srv);

/* Kernel families timed by the "kernel_timing" option (index into
 * geomst_stats_t.kernel_ms / kernel_launches). */
enum {
    GEOMST_K_TREE = 0,     /* bounding box, Morton codes, permute, radix tree, node bounds */
    GEOMST_K_SORT = 1,     /* radix-sort passes (Morton keys and edge keys) */
    GEOMST_K_CORE = 2,     /* k-NN core distances */
    GEOMST_K_SPLIT = 3,    /* frontier and pool splits */
    GEOMST_K_EXPAND = 4,   /* pair expansion (FindPair) with inline small BCCPs */
    GEOMST_K_BCCP = 5,     /* small-pair BCCP (up to 16 point pairs, one pair per thread) */
    GEOMST_K_KRUSKAL = 6,  /* Boruvka pick / hook / reset */
    GEOMST_K_REFRESH = 7,  /* union-find compression and node components */
    GEOMST_K_OUTPUT = 8,   /* output writes */
    GEOMST_K_DENDRO = 9,   /* dendrogram and reachability plot */
    GEOMST_K_BCCP_LARGE = 10, /* medium and large pairs: block boxes, tasks, tiles and their combine */
    GEOMST_K_COUNT = 11
};

/* Counters and timings of the last solve made by the calling thread. */
typedef struct {
    int64_t n;
    int32_t d;
    int32_t min_pts;          /* 0 for EMST */
    int64_t rounds;           /* filtered-Kruskal rounds (weight thresholds) */
    int64_t pair_visits;      /* node pairs examined by the decomposition */
    int64_t bccp_pairs;       /* separated pairs whose BCCP was computed */
    int64_t bccp_evals;       /* point-pair distance evaluations inside BCCPs */
    int64_t big_pairs;        /* of which solved by the large-pair kernel */
    int64_t committed_edges;  /* edges handed to the Kruskal steps */
    int64_t max_frontier;     /* most node pairs waiting between rounds */
    double ms_total;          /* wall time of the call */
    double ms_tree;           /* bounding box, Morton sort, tree, bounds */
    double ms_core;           /* core distances (HDBSCAN*) */
    double ms_rounds;         /* all rounds */
    double ms_final;          /* output sort and write */
    int64_t big_evals;        /* distances the large-pair kernel evaluated (pruned blocks excluded) */
    int64_t sort_elems;       /* elements x 8-bit passes moved by the radix sorts */
    double kernel_ms[16];     /* device time per kernel family (kernel_timing on) */
    int64_t kernel_launches[16];
    int64_t bccp_evals_done;  /* distances the BCCP kernels evaluated (bccp_evals minus pruned blocks) */
    int64_t tuning_applied;   /* 1 if a loaded tuning-cache entry set this solve's knobs */
    int64_t level_launches[3];  /* expansion launches: whole grid, eight workgroups, 256 workgroups */
} geomst_stats_t;

int geomst_get_stats(geomst_stats_t* out);

/*
 * Tuning knobs (they never change the result):
 *   "beta_growth"    factor applied to the weight threshold between rounds,
 *                    > 1; 0 restores the default (2 for EMST: the threshold
 *                    doubles each round; sqrt(2) for HDBSCAN*).
 *   "beta_start_quantile"  [0, 1]: the first threshold is the low edge of the
 *                    binary64 binade in which this fraction of the initial
 *                    pairs' positive lower bounds is reached (default 0:
 *                    the smallest positive bound).
 *   "beta_schedule"  0 = default: the threshold grows by g per round, by g^2
 *                    while the tree holds fewer than n/16 edges (EMST) or
 *                    n/64 (HDBSCAN*), and (EMST) by g^4 after a round that
 *                    found no edge before the first one; 1 = plain: beta <- max(g * beta, smallest
 *                    waiting bound) every round, starting at the smallest
 *                    positive pair bound (doubling for EMST).
 *   "server_share_scale"  (0,1]: a server worker's batch may grow its
 *                    workspace to this fraction of its budget share (default 1;
 *                    small values force the one-request-at-a-time fallback, a
 *                    testing aid).
 *   "list_capacity_scale"  (0,1]: scale of the initial capacities of the
 *                    internal pair and edge lists (default 1); small values make
 *                    the lists overflow, grow and restart rounds (a testing aid).
 *   "kernel_timing"  1 = bracket every kernel family launch with HIP events on
 *                    the solve's stream and report device times in
 *                    geomst_stats_t.kernel_ms; 0 = off (default).
 *   "kernel_timing_families"  bit mask of GEOMST_K_* families to time while
 *                    "kernel_timing" is on (fewer events, less overhead);
 *                    0 = all (default).
 *   "schedule"       round schedule of the filtered Kruskal: 0 = weight
 *                    thresholds (default, see "beta_schedule"); 1 = Naive:
 *                    one round that materialises every well-separated pair
 *                    and its BCCP (Sec. 5, EMST-Naive); 2 = GFK (Alg. 2):
 *                    cardinality beta = 2, 4, 8, ..., each round computes
 *                    the BCCP of every unconnected pair with |A| + |B| <= beta
 *                    and commits the edges up to rho_hi, the smallest bound of
 *                    the larger unconnected pairs (heavier edges wait in the
 *                    BCCP cache); 3 = MemoGFK (Alg. 3): the same thresholds
 *                    (GetRho by a pruned traversal each round), retrieving
 *                    only the pairs with bounds up to rho_hi.  Single-
 *                    instance calls only (batches use 0).  Same tree.
 *   "separation_mode"  HDBSCAN* well-separation: 0 = geometrically separated
 *                    or mutually unreachable (Sec. 3.2.2, default); 1 =
 *                    geometrically separated only (the HDBSCAN*-GanTao
 *                    variant, Sec. 3.2.1: more pairs, same tree).
 *   "separation"     the constant s of the sphere separation test (Sec. 2.3),
 *                    in [0, 16]; default 2.
 *   "bccp_chunk"     B points per large-pair BCCP task, a multiple of 64 in
 *                    [64, 65536]; 0 restores the default 2048.
 *   "refresh_divisor"  node components are refreshed after a round that
 *                    merged at least n / this many components (and at least
 *                    every fourth round); default 1048576, about every round
 *                    that merged anything.
 *   "small_level_switch", "small_level_max"  expansion levels with at most
 *                    eight times the first many pairs run in eight
 *                    workgroups, one eighth each, and each workgroup keeps
 *                    expanding its share while its levels stay at most the
 *                    second size (defaults 2048 and 4096).
 *   "wide_level_switch", "wide_level_max"  larger levels with at most 256
 *                    times the first many pairs run in 256 workgroups, one
 *                    256th each, kept going in the same way while each
 *                    workgroup's levels stay at most the second size
 *                    (defaults 2048 and 4096; for HDBSCAN* with d >= 4 the
 *                    defaults mean off, as 0 does; used when each
 *                    workgroup's part of the level queues holds twice the
 *                    second size, which needs n of about 200,000 or more;
 *                    not used by geomst_emst_dev_noalloc).  Values up to
 *                    65536.
 * Options are process-wide; every solve reads them once when it starts
 * (under a lock), so a change never reaches a solve already running.
 * Returns GEOMST_EINVAL for an unknown name or a bad value.
 */
int geomst_set_option(const char* name, double value);

/*
 * Tuning cache (written by the project's tuner, paper_2104_01126_amd/tune.py):
 * a text file of flat JSON objects, one per line, e.g.
 *   {"kind": "emst", "d": 3, "nlog2": 25, "bccp_chunk": 1024,
 *    "small_level_switch": 2048, "small_level_max": 4096, "beta_growth": 2.0}
 * ("kind" emst or hdbscan, "d" the dimension or batch stride, "nlog2" =
 * floor(log2 of the solve's total points); knobs as for geomst_set_option:
 * bccp_chunk, small_level_switch, small_level_max, refresh_divisor,
 * beta_growth, beta_start_quantile; other keys are ignored).  A solve takes
 * the entry of its kind and d with the nearest nlog2 (within 2) for every
 * knob still at its built-in default.  The knobs never change the result.
 * path NULL clears the table.  ENOENT if the file cannot be opened, EINVAL
 * (table unchanged) for a malformed line.
 */
int geomst_load_tuning(const char* path);

/* Thread-local description of the last error (empty string if none). */
const char* geomst_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int geomst_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GEOMST_H */
