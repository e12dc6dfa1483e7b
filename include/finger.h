/*
 * finger.h - C ABI of libfinger, an MI355X (gfx950) implementation of FINGER
 * search: greedy beam search over a proximity graph in which the exact L2
 * distance to each neighbour is first screened by FINGER's low-rank +
 * distribution-matching estimate (Chen et al., "FINGER: Fast Inference for
 * Graph-based Approximate Nearest Neighbor Search").
 *
 * Conventions for every entry point below:
 *   - Pointers are DEVICE pointers unless marked (host).  Arrays are dense,
 *     row-major, with the stated element type.
 *   - Every call returns an int status: FINGER_OK (0) or a negative
 *     finger_status.  Nothing aborts or throws across the ABI.  On error the
 *     outputs are undefined, any handle stays valid, and finger_last_error()
 *     returns a message for the calling thread.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls marked "async" only enqueue work on it; the caller synchronizes.
 *   - The library never allocates device memory inside finger_search or
 *     finger_exact_knn: scratch space comes from the caller's workspace.
 *
 * Problem statement (Section 1): a dataset D of n points with m features, a
 * query q, the K closest points of D under squared L2 distance; recall@K =
 * |T intersect A| / K.
 */
#ifndef FINGER_H
#define FINGER_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define FINGER_API __attribute__((visibility("default")))
#else
#define FINGER_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FINGER_OK = 0,
  FINGER_EINVAL = -1,     /* invalid argument; message names it */
  FINGER_ENOMEM = -2,     /* device or host allocation failed */
  FINGER_EDEVICE = -3,    /* a HIP call failed; message has the HIP error */
  FINGER_ENODEV = -4,     /* no usable gfx950 device */
  FINGER_EOVERFLOW = -5,  /* a fixed capacity (LDS, table) cannot hold the request */
  FINGER_EINTERNAL = -6,
  FINGER_ECORRUPT = -7    /* a tables image fails its checksum or format checks */
} finger_status;

typedef enum {
  FINGER_L2 = 0,          /* squared Euclidean distance */
  FINGER_ANGULAR = 1,     /* squared L2 between unit-normalized vectors
                             (Supplementary A: normalize, then the same
                             decomposition); 1 - cos = d2 / 2 */
  FINGER_IP = 2           /* maximum inner product: the "distance" is -q.x,
                             so results are the K largest inner products and
                             reported values are their negatives.  The
                             estimate is Supplementary A's q_proj.d_proj +
                             |q_res| |d_res| t, negated.  The learned gate
                             (and its feature log) is for L2 only. */
} finger_metric;

typedef enum {
  FINGER_CODE_F32 = 0,    /* u_d stored as float: (r+2)*|E|*4 bytes (Suppl. F) */
  FINGER_CODE_BF16 = 1,   /* u_d rounded to bfloat16 (nearest-even) */
  FINGER_CODE_FP8E4M3 = 2 /* u_d / s_c rounded to OCP FP8 E4M3, s_c = per-node scale */
} finger_code_t;

typedef enum {
  FINGER_MODE_PLAIN = 0,  /* greedy graph search, Algorithm 1 */
  FINGER_MODE_FINGER = 1, /* approximate greedy search, Algorithm 4 */
  FINGER_MODE_GATED = 2   /* Algorithm 4 with the learned gate replacing the
                             distribution-matching map (needs finger_gate_attach) */
} finger_mode;

typedef enum {
  FINGER_SIGMA_STD = 0,      /* sigma = population standard deviation */
  FINGER_SIGMA_VARIANCE = 1  /* sigma = the mean squared deviation, as Algorithm 2 prints it */
} finger_sigma_mode;

/* Counters written per query by finger_search (int32 [nq][FINGER_NCOUNTERS]). */
enum {
  FINGER_CTR_EXPANSIONS = 0, /* nodes expanded (Algorithm 1's outer loop) */
  FINGER_CTR_EXACT = 1,      /* exact distances computed, the entry included */
  FINGER_CTR_SCREENED = 2,   /* neighbours screened by the estimate */
  FINGER_CTR_SKIPPED = 3,    /* screened neighbours whose estimate exceeded ub */
  FINGER_CTR_VISITED = 4,    /* |V| at the end */
  FINGER_CTR_PREPS = 5,      /* expansions that screened (each reads c.c and P c) */
  FINGER_CTR_STATUS = 6,     /* 0 = ok; bit 0: the visited set overflowed (its
                                LDS table and its spill table were both full):
                                the query's results are NOT valid, which is the
                                asynchronous form of FINGER_EOVERFLOW (raise
                                visited_capacity or spill_capacity and search
                                again); bit 1: ef_eff clipped to ef_max */
  FINGER_NCOUNTERS = 7
};

/* Start-point selectors for finger_search_params.entry (values >= 0 name a
 * node). */
#define FINGER_ENTRY_PIVOT (-1)
#define FINGER_ENTRY_DESCENT (-2)

/* ---------------------------------------------------------------- build */

typedef struct finger_build_params {
  int32_t rank;          /* r (Section 3.3), 0 <= r <= m and r <= 256;
                            0 builds a plain-search-only handle */
  int32_t code_type;     /* finger_code_t */
  int32_t metric;        /* finger_metric */
  int32_t sigma_mode;    /* finger_sigma_mode */
  int64_t n_samples;     /* sampled nodes N_s; <= 0 means min(n, 100000) */
  uint64_t seed;         /* SplitMix64 seed for the samples (see below) */
  const int32_t* pivots; /* device int32 [n_pivots] node ids, or NULL.  With
                            pivots a search may start each query at its
                            nearest pivot (entry = -1). */
  int32_t n_pivots;      /* 0..65536 */
  int32_t dm_override;   /* 1: use dm[] instead of the measured statistics */
  double dm[5];          /* mu, sigma, mu_hat, sigma_hat, eps (override) */
  const double* basis;   /* host [rank][m] row-major, or NULL.  Given, it is
                            used as P instead of the top-r eigenvectors of
                            D_res D_res^T (which are then not computed, and
                            FINGER_T_EIGENVALUES reads as NaN): e.g. a basis
                            computed elsewhere, or the random projections of
                            the paper's RPLSH comparison (Section 4.2).  Rows
                            need not be orthonormal; values must be finite.
                            Copied during the call. */
} finger_build_params;

/* Fill *p with the defaults (rank 0, F32 codes, L2, sigma = std, N_s = min(n,
 * 100000), seed 0, no pivots, no override). */
FINGER_API void finger_build_params_init(finger_build_params* p /* host */);

typedef struct finger_tables finger_tables; /* opaque handle */

/*
 * finger_build_tables - FINGER construction, Algorithm 2 with the
 * precomputation of Supplementary G.  Synchronous on return.
 *
 *   data  [n][m] float: the dataset D.  Borrowed: must stay valid and
 *         unchanged until finger_free_tables (for FINGER_ANGULAR the handle
 *         keeps its own normalized copy instead).
 *   graph [n][max_degree] int32: out-neighbours of each node, valid ids
 *         first, then -1 padding; no self loops, no repeated ids in a row.
 *         Borrowed like data.  1 <= max_degree <= 64.
 *   m     1..2048, a multiple of 4, data 16-byte aligned.
 *
 * Sampling: N_s samples; sample i uses node c = i when N_s == n, else
 * c = h(3i) mod n, where h(j) is the j-th output of SplitMix64 seeded with
 * `seed`; nodes with fewer than 2 neighbours are dropped; the neighbour pair
 * is slots a = h(3i+1) mod deg and (a + 1 + h(3i+2) mod (deg-1)) mod deg.
 * Residuals d_res = d - (c.d / c.c) c (Eq. 1) of the first neighbour form
 * D_res; P holds the top-r eigenvectors of D_res D_res^T (the left singular
 * vectors of Proposition 3.1, computed in float64).  X and Y are the cosines
 * of (d_res, d'_res) and of their projections; mu, sigma, mu_hat, sigma_hat
 * and eps follow Algorithm 2, accumulated in float64.
 * Per node: c.c and P c.  Per edge slot (c -> d): alpha_d = c.d / c.c,
 * rho_d = ||d_res||, u_d = P d_res / ||P d_res|| (0 if that norm is 0), i.e.
 * (r+2) values per edge (Supplementary F); -1 slots hold zeros.
 *
 * Errors: EINVAL (n <= 0, m out of range, max_degree out of range, rank out
 * of range, bad code_type/metric/sigma_mode, a graph id out of range, a self
 * loop or repeated id, a pivot out of range, NULL pointers), ENOMEM,
 * EDEVICE, ENODEV.
 */
FINGER_API int finger_build_tables(const float* data, int64_t n, int32_t m,
                        const int32_t* graph, int32_t max_degree,
                        const finger_build_params* p /* host */,
                        finger_tables** out /* host */, void* stream);

/* Release a handle and everything it owns (NULL is a no-op). */
FINGER_API void finger_free_tables(finger_tables* t);

typedef struct finger_tables_info {
  int64_t n;
  int32_t m, rank, max_degree, code_type, metric, n_pivots;
  int64_t n_samples_used;   /* samples kept after dropping degree < 2 nodes */
  double mu, sigma, mu_hat, sigma_hat, eps; /* the constants the search uses */
  double eps_gate;          /* learned-gate correction (0 if no gate) */
  int32_t gate_attached;
  int64_t edge_table_bytes; /* bytes of alpha, rho and u over all slots */
  double corr_xy;           /* Pearson correlation of the sampled X (true residual
                               cosines) and Y (low-rank ones): Supplementary E's
                               rank rule grows r until it reaches 0.7 */
  int32_t hierarchy_top_level; /* highest upper layer attached (0: none) */
  int32_t hierarchy_top;       /* node the descent starts at (-1: none) */
  int64_t hierarchy_rows;      /* upper-layer rows attached */
} finger_tables_info;

FINGER_API int finger_tables_info_get(const finger_tables* t, finger_tables_info* info /* host */);

/* Selectors for finger_tables_read (sizes in elements):
 *   P_F64      double [r][m]     basis (rows = eigenvectors, descending eigenvalue)
 *   EIGVALS    double [m]        eigenvalues of D_res D_res^T, descending
 *   P_F32      float  [r][m]     basis used by the kernels
 *   NODE_CC    float  [n]        c.c
 *   NODE_PC    float  [n][r]     P c
 *   EDGE_ALPHA float  [n][deg]   alpha_d
 *   EDGE_RHO   float  [n][deg]   rho_d
 *   EDGE_CODES raw    [n][deg][r] u_d as stored (float, bf16 bits or fp8 bytes)
 *   EDGE_SCALE float  [n]        FP8 per-node scale (1 for other code types)
 *   SAMPLES    int32  [N][3]     kept samples (c, d, d')
 *   XY         double [N][2]     (X_i, Y_i) per kept sample
 */
enum {
  FINGER_T_P_F64 = 0, FINGER_T_EIGVALS = 1, FINGER_T_P_F32 = 2, FINGER_T_NODE_CC = 3,
  FINGER_T_NODE_PC = 4, FINGER_T_EDGE_ALPHA = 5, FINGER_T_EDGE_RHO = 6,
  FINGER_T_EDGE_CODES = 7, FINGER_T_EDGE_SCALE = 8, FINGER_T_SAMPLES = 9, FINGER_T_XY = 10
};

/* Copy one table to host memory.  *bytes (host) in: capacity of dst; out:
 * the table's size.  dst == NULL only queries the size.  EINVAL for an
 * unknown selector, EOVERFLOW if the capacity is too small.  Synchronous. */
FINGER_API int finger_tables_read(const finger_tables* t, int32_t which, void* dst /* host */,
                       size_t* bytes /* host */);

/* --------------------------------------------------------------- search */

typedef struct finger_search_params {
  int32_t mode;          /* finger_mode */
  int32_t k;             /* K for every query (ignored with k_per_query) */
  int32_t ef;            /* efs for every query (ignored with ef_per_query);
                            the search keeps ef_eff = max(ef, K) entries */
  int32_t entry;         /* >= 0: start point p of every query (Algorithm 1);
                            FINGER_ENTRY_PIVOT (-1): each query starts at its
                            nearest pivot; FINGER_ENTRY_DESCENT (-2): where the
                            descent through the attached upper layers ends
                            (finger_hierarchy_attach, finger_descend) */
  int32_t warmup;        /* W: screening starts once more than W nodes have
                            been expanded (Algorithm 4's warm-up); < 0 = 5 */
  int32_t k_max;         /* row stride of out_ids/out_dist; >= every K */
  const int32_t* k_per_query;  /* device int32 [nq] or NULL */
  const int32_t* ef_per_query; /* device int32 [nq] or NULL */
  int32_t ef_max;        /* >= ef_eff of every query; 0 = derive from k/ef
                            (required when ef_per_query or k_per_query is set) */
  int32_t persistent;    /* 1: one launch drains an atomic queue of queries
                            (uneven K/ef); 0: static assignment */
  int32_t waves_per_cu;  /* resident query waves per CU; 0 = library default */
  int32_t visited_capacity; /* visited-set slots per query in LDS (power of
                               two, >= 256); ids beyond it go to the spill
                               table; 0 = default 2048 */
  int32_t spill_capacity; /* visited-set spill slots per resident query wave
                             in the workspace (power of two, >= 64); 0 =
                             default next_pow2(ef_max * max_degree) clamped
                             to [1024, 65536].  Together with the LDS table
                             it bounds |V| per query (status bit 0). */
  int32_t visited_probe;  /* LDS slots a visited test examines before it
                             continues in the spill table: a multiple of 4 in
                             [4, 64]; 0 = default 24.  Fewer spill sooner but
                             walk less of a nearly full table.  Results do not
                             depend on it. */
  int32_t code_prefetch; /* FINGER mode: 1 = request every slot's edge code
                            together with the adjacency row (one round trip
                            fewer; also reads the codes of visited and
                            padding slots); -1 or 0 (default) = request the
                            codes of unvisited neighbours only, after the
                            visited test */
  int32_t ef_classes;    /* with k_per_query or ef_per_query, how the queries
                            are grouped by ef class (ef_eff = max(ef, K) in
                            (16, 32], (32, 64], ... up to ef_max):
                            0 (default) or 3 = one persistent launch, every
                            wave reserving LDS, a visited table and resident
                            waves for ef_max, its queue serving the largest
                            class first so that the short queries fill the
                            launch's end; 1 = one persistent launch per
                            class, each reserving for its own bound; 2 = one
                            launch reserving for ef_max with the queue in
                            query order.  Results do not depend on it. */
  float gate_band;        /* GATED mode: 0 (default) = the gate decides every
                            screened neighbour; > 0 = a cascade: the gate
                            decides only neighbours whose distribution-
                            matched estimate (Algorithm 3) lies within
                            gate_band * ub^2 of the bound ub^2, the others
                            keep Algorithm 3's decision */
  int32_t screen_layout; /* FINGER mode: how lanes read the edge codes.
                            0 = library default (coalesced where it applies);
                            1 = coalesced: each load instruction reads 1 KB of
                            the centre's contiguous code block, a lane holds
                            one 16-byte piece of a slot's code (code rows of
                            32..256 bytes and max_degree <= 32; other shapes
                            fall back to 2); 2 = per-lane chunks: a lane holds
                            32 consecutive elements of one slot's code.
                            Results do not depend on it. */
  /* Gate-training log (mode FINGER only; NULL = off).  For every screened
   * neighbour the kernel appends one row of FINGER_GATE_FEATURES(r) floats
   * (see finger_gate_attach) to log_features, its exact squared distance
   * and the screening bound to log_targets ([row][2]: d2, ub2) and counts rows in
   * *log_count (int64); rows past log_capacity are counted, not written. */
  float* log_features;
  float* log_targets;
  int64_t log_capacity;
  int64_t* log_count;
  /* Optional hipEvent_t pair recorded on `stream` immediately before and
   * after the search kernel (not the query preparation), for timing the
   * kernel alone; NULL = none. */
  void* kernel_events[2];
} finger_search_params;

FINGER_API void finger_search_params_init(finger_search_params* p /* host */);

/* Bytes of device workspace finger_search needs for nq queries.  EINVAL as
 * for finger_search. */
FINGER_API int finger_search_workspace_size(const finger_tables* t, int64_t nq,
                                 const finger_search_params* p /* host */,
                                 size_t* bytes /* host */);

/*
 * finger_search - batched greedy search (Algorithm 1) or FINGER search
 * (Algorithm 4 with Algorithm 3's estimate), one wavefront per query.  Async.
 *
 *   queries      [nq][m] float.
 *   out_ids      [nq][k_max] int32: the K best (d2, id) of T in ascending
 *                order; slots past K or past |T| hold -1.
 *   out_dist     [nq][k_max] float: their squared distances (+inf padding).
 *   out_counters [nq][FINGER_NCOUNTERS] int32, or NULL.
 *   workspace    >= finger_search_workspace_size bytes, 256-byte aligned.
 *
 * Semantics (each a reading of the pseudo-code): keys are (d2, id); a
 * neighbour is admitted iff |T| < ef_eff or its key is below the worst key
 * of T; the search ends when T has no unexpanded entry.  FINGER screens the
 * unvisited neighbours of an expansion only when T is full and more than W
 * nodes have been expanded, against ub = worst d2 of T at the start of that
 * expansion; a neighbour is skipped iff its estimate exceeds ub (it stays
 * visited); survivors get exact distances and the admission rule above.
 * Returned distances are always exact (Supplementary G).
 *
 * Errors: EINVAL (nq < 0, k < 1 or k > n, ef < 1, entry out of range,
 * entry = -1 without pivots, entry = -2 without upper layers, FINGER/GATED mode on a rank-0 handle, GATED
 * without a gate, workspace too small or misaligned, ef_max > 1024, NULL
 * pointers), EOVERFLOW (ef_max or visited_capacity beyond the LDS budget),
 * EDEVICE.
 */
FINGER_API int finger_search(const finger_tables* t, const float* queries, int64_t nq,
                  const finger_search_params* p /* host */,
                  int32_t* out_ids, float* out_dist, int32_t* out_counters,
                  void* workspace, size_t workspace_bytes, void* stream);

/*
 * finger_search_noalloc - finger_search for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same search, with its scratch (query norms and
 * projections, entries, queue counter, pivot candidates, visited-set spill
 * tables, normalized queries) in a fixed device array of
 * finger_search_noalloc_capacity() bytes (64 MiB) that the library holds on
 * each GPU it runs on until the process ends, instead of a caller workspace.
 * The call allocates nothing; the scratch parts that must start cleared are
 * cleared at every call on `stream` (the queue counter by a fill kernel, each
 * visited-set spill table by its search wave before first use).  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialized by the caller.  Arguments,
 * results and errors as finger_search, plus EOVERFLOW when the search needs
 * more scratch than the array holds (fewer queries per call then fit).
 * Async.
 */
FINGER_API size_t finger_search_noalloc_capacity(void);
FINGER_API int finger_search_noalloc(const finger_tables* t, const float* queries, int64_t nq,
                                     const finger_search_params* p /* host */, int32_t* out_ids,
                                     float* out_dist, int32_t* out_counters, void* stream);

/* ---------------------------------------------------------------- graph */

typedef struct finger_graph_stats {
  int64_t sym_edges;              /* directed edges after symmetrization */
  int32_t sym_degree_max;         /* longest row before pruning */
  int32_t components_before_repair; /* 1 + number of repair steps */
  int64_t edges_added;            /* edges the repair appended */
  double ms_knn, ms_symmetrize, ms_prune, ms_repair; /* wall time per phase */
} finger_graph_stats;

/*
 * finger_build_graph - the flat proximity graph the search runs over, built
 * on the GPU.  The paper takes the graph as given (Section 3.3 and
 * Algorithm 2 start from G = (D, E); its experiments use HNSW graphs); this
 * is the stand-in for HNSW's layer 0, in four steps:
 *   1. the knn_k nearest other points of every point, by (d2, id);
 *   2. symmetrization: every edge and its reverse, rows sorted by (d2, id),
 *      no duplicates;
 *   3. rows longer than max_degree: HNSW's neighbour-selection heuristic
 *      (scan the row in order; keep a candidate iff fewer than max_degree
 *      are kept and it is strictly closer to the base than to every kept
 *      neighbour);
 *   4. reachability repair from `entry`: while a node is unreached, the
 *      smallest-id unreached node u gets an edge from the reached node with a
 *      free slot of smallest (d2 to u, id), appended to that node's row; u
 *      gets the reverse edge if it has a free slot and does not list the node
 *      yet; everything reachable from u is then reached.
 * Distances are float32 sums of squared differences (exact for integer data
 * whose squared norms stay below 2^24); FINGER_ANGULAR builds the graph of
 * the unit-normalized points.
 *   data      [n][m] float (device, 16-byte aligned), m % 4 == 0.
 *   out_graph [n][max_degree] int32 (device): rows of neighbour ids, -1
 *             padded; repair edges follow the row's own entries.
 *   stats     host, or NULL.
 * The kNN runs in query batches of at most 2^20 points.  Synchronous;
 * allocates its scratch (about 2nk * 40 bytes plus one batch's kNN candidate
 * lists) and frees it before returning.
 * Errors: EINVAL (NULL pointers, n < 2, m, knn_k outside 1..min(n - 1, 127),
 * max_degree outside 1..64, metric not L2/ANGULAR, entry out of range),
 * EOVERFLOW (2 n knn_k >= 2^31, or no reached node has a free slot for a
 * repair), ENOMEM, EDEVICE.
 */
/* Progress report: called on the host after each finished step (phase
 * "knn" per query batch with done/total queries, then "symmetrize", "prune"
 * and "repair"); may be NULL. */
typedef void (*finger_progress_fn)(const char* phase, int64_t done, int64_t total, void* user);

FINGER_API int finger_build_graph(const float* data, int64_t n, int32_t m, int32_t knn_k,
                                  int32_t max_degree, int32_t metric, int32_t entry,
                                  int32_t* out_graph, finger_graph_stats* stats /* host */,
                                  finger_progress_fn progress, void* progress_user,
                                  void* stream);

/*
 * finger_build_graph_grouped - finger_build_graph with step 1 restricted to
 * groups: the points are ordered so that each group is a contiguous range
 * [group_offsets[g], group_offsets[g + 1]) (host int64, group_offsets[0] = 0,
 * group_offsets[n_groups] = n, every group at least knn_k + 1 points), and a
 * point's knn_k nearest are taken among the points of its own group; steps
 * 2-4 are unchanged.  This is the exact kNN graph whenever every point's
 * knn_k nearest lie in its own group, e.g. for well separated clusters whose
 * labels are known (a workload generator's), at a cost of sum of group
 * sizes squared instead of n squared.  Errors as finger_build_graph, plus
 * EINVAL for offsets that do not run from 0 to n or a group that is too
 * small.  Synchronous.
 */
FINGER_API int finger_build_graph_grouped(const float* data, int64_t n, int32_t m, int32_t knn_k,
                                          int32_t max_degree, int32_t metric, int32_t entry,
                                          const int64_t* group_offsets /* host */, int64_t n_groups,
                                          int32_t* out_graph, finger_graph_stats* stats /* host */,
                                          finger_progress_fn progress, void* progress_user,
                                          void* stream);

/* ------------------------------------------------------------ hierarchy */

/*
 * finger_hierarchy_attach - give the handle the upper layers of an HNSW-style
 * hierarchical graph; the handle's graph is its layer 0.  The paper runs
 * FINGER on HNSW graphs (Sections 1 and 4), where the start point p of
 * Algorithm 1 is where a greedy descent through these layers ends
 * (finger_descend; search with entry = FINGER_ENTRY_DESCENT).
 *
 *   levels [n] int32 (device): the highest layer of each node, 0..64.
 *   upper  [rows][width] int32 (device): one row per (node, layer) with
 *          1 <= layer <= levels[node], ordered by node id and then layer
 *          (a node's rows start at the sum of the levels of the nodes before
 *          it); a row lists the node's neighbours in that layer (ids of nodes
 *          whose level is at least that layer, never the node itself), padded
 *          with -1.  rows = sum of levels; 1 <= width <= 64.
 *
 * The descent starts at the smallest id among the nodes of the highest
 * level.  Both arrays are copied (checked on the host); a later attach
 * replaces the earlier one.  Synchronous.
 * Errors: EINVAL (NULL handle or levels, upper NULL with rows > 0, width out
 * of range, a level out of range, rows not the sum of the levels, a
 * neighbour out of range, equal to its node or below the row's layer),
 * EOVERFLOW (rows >= 2^31), ENOMEM, EDEVICE.
 */
FINGER_API int finger_hierarchy_attach(finger_tables* t, const int32_t* levels,
                                       const int32_t* upper, int64_t rows, int32_t width);

/*
 * finger_descend - start points from the attached upper layers.  For each
 * query, from the top node, in each layer from the highest down to 1: move
 * to the listed neighbour of smallest (d, id) key while that key is below
 * the current node's key, then keep the node for the layer below (HNSW's
 * layer search with a result list of one).  d is the handle's distance
 * (squared L2, or -q.x for FINGER_IP; queries are unit-normalized first for
 * FINGER_ANGULAR).  Async.
 *   queries     [nq][m] float (device, 16-byte aligned).
 *   out_entries [nq] int32: the layer-0 start point of each query.
 *   out_calls   [nq] int32 or NULL: distance evaluations, the top node's
 *               included; a neighbour met again at a later hop is counted
 *               again.
 * Errors: EINVAL (NULL handle, no upper layers attached, nq < 0, NULL or
 * misaligned pointers with nq > 0), ENOMEM, EDEVICE.
 */
FINGER_API int finger_descend(const finger_tables* t, const float* queries, int64_t nq,
                              int32_t* out_entries, int32_t* out_calls, void* stream);

/*
 * finger_estimate_edges - evaluate the search kernel's estimate for given
 * (query, centre, edge slot) triples, for testing the factorized arithmetic
 * against a direct evaluation.  Async.
 *   q_index, centers, slots [n_items] int32 (device); slot indexes the centre's
 *   graph row and must hold a valid neighbour.
 *   out_est   [n_items] float: the estimated squared distance (Algorithm 3
 *             plugged into Eq. 2), computed exactly as finger_search does.
 *   out_t_hat [n_items] float: the low-rank cosine cos(P q_res, P d_res).
 * Errors: EINVAL (rank-0 handle, NULL pointers, n_items < 0), EDEVICE.
 * Indices are not range-checked on the device: the caller guarantees them.
 */
FINGER_API int finger_estimate_edges(const finger_tables* t, const float* queries, int64_t nq,
                          const int32_t* q_index, const int32_t* centers,
                          const int32_t* slots, int64_t n_items,
                          float* out_est, float* out_t_hat, void* stream);

/* ----------------------------------------------------------- exact kNN */

/* Workspace for finger_exact_knn. */
FINGER_API int finger_exact_knn_workspace_size(int64_t n, int32_t m, int64_t nq, int32_t k,
                                    size_t* bytes /* host */);

/*
 * finger_exact_knn - brute-force K nearest neighbours (the ground truth A of
 * recall@K, Section 1).  Candidates are selected with an MFMA GEMM
 * (|q|^2 + |x|^2 - 2 q.x), the best K+16 per query are re-ranked by direct
 * differences in float32 and returned sorted by (d2, id).  Async.
 *   data [n][m], queries [nq][m] float; out_ids int32 / out_dist float
 *   [nq][k].  k <= n, k <= 256.  FINGER_ANGULAR normalizes both sides.
 * Errors: EINVAL, EDEVICE.
 */
FINGER_API int finger_exact_knn(const float* data, int64_t n, int32_t m,
                     const float* queries, int64_t nq, int32_t k, int32_t metric,
                     int32_t* out_ids, float* out_dist,
                     void* workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------ learned skip gate */

/*
 * The gate is an extension beyond the paper: a 3-layer perceptron
 * (in -> H -> H -> 1, ReLU) that maps screening features to an estimate of
 * cos(q_res, d_res), used in place of Algorithm 3's distribution-matching map.
 * Features of one screened edge (in = 2r + 4, all float):
 *   [0, r)      w / |w|, w = P q_res = Pq - alpha_q P c   (0 if |w| = 0)
 *   [r, 2r)     u_d
 *   2r          t_hat = w.u_d / |w|
 *   2r + 1      rho_q / ub        (ub = sqrt of the screening bound)
 *   2r + 2      rho_d / ub
 *   2r + 3      (alpha_q - alpha_d)^2 c.c / ub^2
 * The gated estimate is Eq. 2 with t = f(x) + eps_gate.
 */
#define FINGER_GATE_FEATURES(r) (2 * (r) + 4)

/* Weight layout (float, host): W1 [H][in], b1 [H], W2 [H][H], b2 [H],
 * W3 [H], b3 [1]; 1 <= H <= 64 and in == FINGER_GATE_FEATURES(rank).  The
 * handle keeps a bf16 copy used by the search kernel.  Synchronous.
 * Errors: EINVAL (NULL arguments, rank-0 or FINGER_IP handle, in_dim or H
 * out of range), EDEVICE (allocation or copy failed). */
FINGER_API int finger_gate_attach(finger_tables* t, const float* weights /* host */,
                       int32_t in_dim, int32_t hidden, double eps_gate);

/*
 * finger_gate_targets - training targets from a feature log written by
 * finger_search: for row i, t_i = cos(q_res, d_res) recovered from the logged
 * exact squared distance through Eq. 2,
 *   q_res.d_res = (|q_proj - d_proj|^2 + |q_res|^2 + |d_res|^2 - d2) / 2,
 * with |q_res|, |d_res| and |q_proj - d_proj|^2 taken from features 2r+1..2r+3
 * scaled back by the logged bound ub2.  Rows with a zero residual get 0.
 *   log_features [rows][2r+4], log_targets [rows][2] (d2, ub2), out [rows].
 * Async.  Errors: EINVAL (NULL pointers, rows < 0, rank < 1).
 */
FINGER_API int finger_gate_targets(const float* log_features, const float* log_targets,
                                   int64_t rows, int32_t rank, float* out, void* stream);

/* Number of floats in the weight layout above. */
FINGER_API int64_t finger_gate_param_count(int32_t in_dim, int32_t hidden);

/*
 * Training kernels (bf16 operands, float32 accumulation).  Weights, grads and
 * Adam moments are float [P] in the layout above (device).
 *   finger_mlp_forward:  x [B][in] float -> y [B] float.
 *   finger_mlp_backward: loss = mean over the batch of (y - target)^2;
 *                        writes grad [P] (overwritten) and *loss (device
 *                        float, may be NULL).  Per-block partial gradients go
 *                        to the caller's workspace of at least
 *                        finger_mlp_backward_workspace_size bytes (256-byte
 *                        aligned); the call allocates nothing.
 *   finger_adam_step:    Adam (Kingma & Ba) with bias correction at step t >= 1.
 * 1 <= in_dim <= 512, 1 <= hidden <= 64.  Async.  Errors: EINVAL (sizes,
 * NULL pointers, workspace too small), EDEVICE.
 */
FINGER_API int finger_mlp_forward(const float* weights, int32_t in_dim, int32_t hidden,
                       const float* x, int64_t batch, float* y, void* stream);
FINGER_API int finger_mlp_backward_workspace_size(int32_t in_dim, int32_t hidden, int64_t batch,
                                                  size_t* bytes /* host */);
FINGER_API int finger_mlp_backward(const float* weights, int32_t in_dim, int32_t hidden,
                        const float* x, const float* target, int64_t batch,
                        float* grad, float* loss, void* workspace, size_t workspace_bytes,
                        void* stream);

/*
 * finger_gate_calibrate - the gate's correction term, the analogue of
 * Algorithm 2's eps for the learned map: eps_gate = mean over the rows of
 * |target - f(x)|, with f evaluated by the forward kernel and the mean
 * accumulated in float64 in a fixed order (deterministic).  Typically the
 * rows are a held-out part of a finger_search feature log and the targets
 * come from finger_gate_targets.  Synchronous; allocates its scratch
 * (rows floats plus a few KB) and frees it before returning.
 * Errors: EINVAL (NULL pointers, rows < 1, sizes as above), ENOMEM, EDEVICE.
 */
FINGER_API int finger_gate_calibrate(const float* weights, int32_t in_dim, int32_t hidden,
                                     const float* x, const float* target, int64_t rows,
                                     double* eps_gate /* host */, void* stream);
FINGER_API int finger_adam_step(float* weights, const float* grad, float* m1, float* m2,
                     int64_t count, float lr, float beta1, float beta2, float eps,
                     int32_t step, void* stream);

/* ----------------------------------------------------------- checkpoint */

/*
 * The build costs minutes on the paper's CPU (Table 1, Supplementary F) and
 * seconds here; a tables image lets a process skip it.
 *
 * finger_tables_export - write the handle's tables into one host image:
 * a header (magic "FINGERTB", format version 1, n, m, r, max_degree, code
 * type, metric, sigma mode, pivot count, build seed, the five
 * distribution-matching constants, corr(X, Y), eps_gate, and checksums of
 * the graph rows and of the points the tables were built over), a section
 * table, then every table (basis in float64 and float32, eigenvalues, node
 * table, edge table, codes and scales, pivot operands, build samples and
 * cosines, packed gate weights) at 256-byte aligned offsets, and last the
 * finger_checksum64 of all preceding bytes.  Upper layers attached with
 * finger_hierarchy_attach are not part of the image (attach them again).
 *   buf   host, or NULL to query the size into *bytes.
 *   bytes in: capacity of buf; out: the image size.
 * Synchronous.  Errors: EINVAL, EOVERFLOW (buffer too small), EDEVICE.
 */
FINGER_API int finger_tables_export(const finger_tables* t, void* buf /* host */,
                                    size_t* bytes /* host */);

/*
 * finger_tables_import - a handle from an image written by
 * finger_tables_export, over the caller's data and graph (borrowed as in
 * finger_build_tables).  The image is checked on the host first (magic,
 * version, checksum, header ranges, section table: ECORRUPT; n, m,
 * max_degree against the arguments: EINVAL), before any device call; then
 * the checksums of the graph rows and of the points (after normalization
 * for FINGER_ANGULAR) must equal the image's (EINVAL otherwise).  Searches
 * on the imported handle return exactly what they return on the exported
 * one.  Synchronous.  Errors: EINVAL, ECORRUPT, ENODEV, ENOMEM, EDEVICE.
 */
FINGER_API int finger_tables_import(const void* buf /* host */, size_t bytes, const float* data,
                                    int64_t n, int32_t m, const int32_t* graph, int32_t max_degree,
                                    finger_tables** out /* host */, void* stream);

/*
 * finger_checksum64 - the image checksum: the bytes are read as
 * little-endian 64-bit words w_0, w_1, ... (the last one zero padded); four
 * lanes start at h_0..h_3 = 0x243F6A8885A308D3, 0x13198A2E03707344,
 * 0xA4093822299F31D0, 0x082EFA98EC4E6C89 and word i updates lane j = i mod 4
 * as h_j = rotl64((h_j xor w_i) * 0x9E3779B97F4A7C15, 31); then x = byte
 * count and for j = 0..3: x = (x xor h_j) * 0xBF58476D1CE4E5B9, x ^= x >> 29;
 * the result is x xor (x >> 32).  Host only; p may be NULL when bytes = 0.
 */
FINGER_API uint64_t finger_checksum64(const void* p /* host */, size_t bytes);

/* Message for the last failed call on this thread ("" if none). */
FINGER_API const char* finger_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FINGER_H */
