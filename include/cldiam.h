/*
 * cldiam.h - C ABI of libcldiam.so, the MI355X (gfx950) implementation of the
 * CL-DIAM diameter approximation of Ceccarello, Pietracaprina, Pucci, Upfal,
 * "A practical parallel algorithm for diameter approximation of massive
 * weighted graphs" (arXiv:1506.03265).
 *
 * Conventions shared by every entry point
 *   - Graphs are undirected, with positive integer edge weights (Section 2).
 *     They are passed as a symmetric CSR: every edge {u,v} appears as the two
 *     arcs u->v and v->u with the same weight; each row is sorted by strictly
 *     increasing column; there are no self loops.
 *   - Every pointer named d_* is DEVICE memory on the current HIP device and is
 *     owned by the caller.  Every pointer named h_* is HOST memory.  The library
 *     allocates no device memory: scratch comes from a caller workspace `ws` of
 *     at least the size returned by the matching *_workspace_size query, aligned
 *     to 256 bytes.  The workspace may be reused between calls but not shared
 *     by calls that run at the same time.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every entry point
 *     enqueues its work on that stream and returns after it has completed
 *     (the decomposition steers itself from values it reads back), so outputs
 *     are ready when the call returns.
 *   - Return value: CLDIAM_OK (0) or a negative status below.  On error the
 *     outputs are unspecified; cldiam_last_error() gives a message for the
 *     calling thread.  No exception or signal crosses the ABI.
 *   - All arithmetic is integer; results are deterministic and bit-identical
 *     to a sequential execution of the method.
 *   - Entry points may be called from several host threads at once on
 *     different streams and workspaces.
 */
#ifndef CLDIAM_H
#define CLDIAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLDIAM_OK 0
#define CLDIAM_EINVAL (-1)     /* bad argument or malformed CSR */
#define CLDIAM_ENOMEM (-2)     /* workspace too small */
#define CLDIAM_EOVERFLOW (-3)  /* Delta would exceed 2^31, or a u32 distance would overflow */
#define CLDIAM_EHIP (-4)       /* HIP runtime error */
#define CLDIAM_ESTAGES (-5)    /* more than CLDIAM_MAX_STAGES stages */
#define CLDIAM_ETIMEOUT (-6)   /* a device-side wait exceeded its time limit */

#define CLDIAM_MAX_STAGES 4096
#define CLDIAM_STAGE_LOG 64

/* Human-readable name of a status code (static string). */
const char *cldiam_strerror(int status);
/* Detail of the last error on the calling thread (static per thread). */
const char *cldiam_last_error(void);
/* Library version string. */
const char *cldiam_version(void);
/* Pinned host memory held by the library (bytes): small readback buffers that
 * calls take from a pool and give back when they return, so it grows only with
 * the number of calls in flight at the same time. */
int64_t cldiam_pinned_host_bytes(void);

/* Device CSR of one graph (all DEVICE pointers, caller-owned).
 * n >= 1 nodes (n < 2^31), m arcs (m = 2 x edges, m < 2^40; row offsets are 64-bit). */
typedef struct {
  int32_t n;
  int32_t pad;
  int64_t m;
  const int64_t *d_row_ptr; /* n+1 offsets, d_row_ptr[0] = 0, d_row_ptr[n] = m (m < 2^40) */
  const int32_t *d_col;     /* m column ids in [0, n) */
  const uint32_t *d_w;      /* m weights >= 1 */
} cldiam_csr;

/* ------------------------------------------------------------- ingest ---
 * Validates a CSR (symmetric with equal weights, columns in range and
 * strictly increasing per row, no self loops, weights >= 1) and packs its arcs
 * as d_arcs[a] = (uint64_t)w << 32 | col with every row re-sorted by
 * (weight, column).  Light arcs (w <= Delta, Section 3) of a row are then a
 * prefix of that row.  The packed arcs are the graph operand of every other
 * entry point.  Also returns the sum of all arc weights (for the default
 * initial Delta).  Returns CLDIAM_EINVAL if validation fails. */
size_t cldiam_load_csr_workspace_size(int32_t n, int64_t m);
int cldiam_load_csr(const cldiam_csr *g, uint64_t *d_arcs, uint64_t *h_weight_sum, void *ws, size_t ws_bytes,
                    void *stream);

/* ------------------------------------------------------ decomposition ---
 * CLUSTER(G, tau) of Algorithm 1 (Section 3): stages that draw random new
 * centers among uncovered nodes, grow all clusters by Delta-growing steps
 * (light-edge relaxation bounded by Delta) until at least half of the
 * uncovered nodes are covered, doubling Delta when needed, and finally make
 * the few remaining nodes singleton clusters.
 *
 * Precise behaviour (the readings of the paper this library implements):
 *   - log is log2, gamma = 4 ln 2; stages run while the uncovered count U is
 *     at least ceil(8 tau log2 n) (and n > 1, U > 0);
 *   - in stage s (from 0) node v is a new center iff word 0 of
 *     Philox4x32-10(counter = (v, s, 0, 0), key = (seed lo, seed hi)) is below
 *     T = floor(p 2^32), p = ((gamma tau) log2 n) / U in IEEE double
 *     (T = 2^32 when p >= 1);
 *   - growth runs every Delta to its fixpoint; a node keeps the lexicographic
 *     minimum (distance, center id) over all offers; nodes assigned in earlier
 *     stages act as sources at distance 0 with their cluster's label, which is
 *     Procedure Contract's effect;
 *   - Delta starts at delta0 (0 = floor(sum of arc weights / m), at least 1),
 *     persists across stages, and doubles while fewer than half of U is
 *     covered and some uncovered node is still reachable; Delta above 2^31 is
 *     CLDIAM_EOVERFLOW;
 *   - a node assigned in stage s with growth distance d to cluster c gets
 *     D = d + R(c), R(c) being the largest D in c after stage s-1; so D is an
 *     upper bound on the distance from the center, and max D is the
 *     clustering radius bound used by the estimate.
 * Outputs: d_cluster[v] = center node id of v's cluster (a center has
 * d_cluster[c] = c); d_D[v] as above. */
typedef struct {
  uint32_t tau;      /* >= 1 */
  uint32_t delta0;   /* initial Delta; 0 = floor(sum of arc weights / m) */
  uint64_t seed;     /* Philox key */
  uint32_t variant;  /* CLDIAM_VARIANT_* */
  uint32_t step_cap; /* CLDIAM_VARIANT_STEPS: most Delta-growing steps per PartialGrowth call; 0 = no cap */
} cldiam_params;

/* CLDIAM_VARIANT_FIXPOINT (0): the behaviour described above (every Delta
 * grown to its fixpoint, schedule-independent results).
 * CLDIAM_VARIANT_STEPS (1): Procedure PartialGrowth of Algorithm 1 taken
 * literally.  Growth runs in synchronous Delta-growing steps: all offers of a
 * step are computed from the state before the step; a node accepts an offer
 * only if its distance is strictly smaller than the node's own (among the
 * offers of one step the smallest distance, then the smallest center, wins).
 * A PartialGrowth call stops after a step that updates no state, or once at
 * least half of the stage's uncovered nodes are covered, or after step_cap
 * steps; Delta doubles one step at a time while fewer than half are covered
 * (a stage whose growth has stopped with no uncovered node reachable keeps
 * what it covered); if the new centers alone cover half, the stage performs
 * no step.  The statistics then carry the paper's round and work counters:
 * rounds (steps), messages (offers sent: every node updated by the previous
 * step, or a source at a stage's or a Delta's first step, offers over each
 * arc with d_u + w <= Delta) and updates (node states changed). */
#define CLDIAM_VARIANT_FIXPOINT 0u
#define CLDIAM_VARIANT_STEPS 1u
/* CLDIAM_VARIANT_CLUSTER2 (2): CLUSTER2(G, tau) of Algorithm 2 (Section 4).
 * First CLUSTER(G, tau) as above gives R_CL = max D; then iterations
 * i = 1 .. ceil(log2 n): each uncovered node becomes a new center iff word 0
 * of Philox4x32-10(counter = (v, i, 0, 1), key = seed) is below
 * floor(min(1, 2^i / n) 2^32) (2^32 when 2^i >= n), and all clusters grow to
 * the fixpoint with Delta2 = 2 R_CL.  Procedure Contract2 is implicit: a node
 * assigned in the previous iteration at growth distance d_u offers its label
 * at d_u + w - Delta2 over each edge with w <= Delta2 to an unassigned
 * neighbour.  A node reached in iteration i by a cluster whose center was
 * drawn in iteration j gets D = d + Delta2 (i - j), the length of a path from
 * the center.  Statistics: stages = levels = iterations, delta_end = Delta2,
 * radius = max D, radius1 = R_CL; Delta2 above 2^31 is CLDIAM_EOVERFLOW. */
#define CLDIAM_VARIANT_CLUSTER2 2u

typedef struct {
  int32_t stages;       /* executed stages */
  int32_t levels;       /* Delta values tried (growth to fixpoint per value) */
  uint32_t delta0;      /* initial Delta used */
  uint32_t delta_end;   /* Delta at the end */
  int32_t stop;         /* ceil(8 tau log2 n) */
  int32_t num_clusters; /* centers drawn + singletons */
  int32_t singletons;
  int32_t sweeps;       /* device relaxation sweeps (schedule dependent) */
  uint64_t radius;      /* max over nodes of D */
  uint64_t arcs_scanned;/* arcs read by relaxation (schedule dependent) */
  int32_t status;       /* per-graph status (CLDIAM_OK or an error) */
  int32_t grid_blocks;  /* workgroups of the persistent launch (0 = host-driven) */
  float kernel_ms;      /* device time of the job's control loop (HIP events) */
  int32_t iterations;   /* control steps of the whole job */
  uint64_t rounds;      /* CLDIAM_VARIANT_STEPS: Delta-growing steps executed */
  uint64_t messages;    /* CLDIAM_VARIANT_STEPS: offers sent */
  uint64_t updates;     /* CLDIAM_VARIANT_STEPS: node states changed */
  uint64_t radius1;     /* CLDIAM_VARIANT_CLUSTER2: radius R_CL of the preliminary CLUSTER run */
  /* per stage s < min(stages, CLDIAM_STAGE_LOG) */
  int32_t stage_uncovered[CLDIAM_STAGE_LOG];
  int32_t stage_centers[CLDIAM_STAGE_LOG];
  int32_t stage_covered[CLDIAM_STAGE_LOG];
  uint32_t stage_delta[CLDIAM_STAGE_LOG];
} cldiam_stats;

/* Driver of the device-side control loop. */
#define CLDIAM_DRIVER_AUTO 0       /* the faster driver on this device (host-driven on MI355X) */
#define CLDIAM_DRIVER_HOST 1       /* one launch per sweep, host polls */
#define CLDIAM_DRIVER_PERSISTENT 2 /* one cooperative launch for the whole job */

/* Schedule knobs of a decomposition job.  They change only how the work is
 * scheduled on the device, never the results. */
typedef struct {
  int32_t local_rounds; /* workgroup-local relaxation rounds per sweep (at least 16 while a frontier has
                           at most 32768 nodes); < 0 = default: 16 on graphs with at most 16 arcs per
                           node, on denser ones 2 above 2^21 nodes and 0 below */
  int32_t grid_blocks;  /* workgroups per sweep; 0 = one per compute unit */
  float bucket_width;   /* distance bucket of a relaxation sweep, in mean arc weights: a sweep relaxes
                           only frontier nodes whose tentative distance is below (smallest distance on
                           the frontier) + width, and keeps the others for later sweeps of the same
                           growth; 0 = default (CLDIAM_BUCKET_DEFAULT), < 0 = no bucket */
  int32_t row_bucket_shift; /* nodes whose rows hold more than 32 arcs are relaxed only once their
                           tentative distance is below (smallest distance on the frontier) +
                           Delta / 2^shift, so that long rows are rarely scanned twice in one growth;
                           0 = default: floor(log2 m) / 2 - 6 clamped to [5, 8] (wider buckets, fewer
                           sweeps, on small graphs); < 0 = no such bucket; values above 31 act as 31.
                           Synchronous steps use none. */
  int32_t chunk_factor; /* chunks of a growth sweep per workgroup: the first goes to each workgroup, the
                           rest to whichever workgroup is free next; 0 = default (3 on graphs of more
                           than 2^21 nodes with more than 16 arcs per node, else 1), at most 64 */
  int32_t wave_row_min; /* threads per row: rows of more arcs than this are relaxed by one wave (64
                           threads) instead of one thread, and take the long-row bucket above;
                           0 = default (32; 128 on graphs with more than 16 arcs per node), at most
                           2^20 */
  int32_t group_row_min;/* rows of more arcs than this are relaxed by the whole workgroup (1024 threads);
                           0 = default (8192), at least wave_row_min */
  int32_t local_queue;  /* queue tile of the local rounds: slots of a workgroup's queue of improved nodes
                           (64 .. 4096); 0 = default (4096) */
  int32_t local_cutoff; /* a workgroup ends its local rounds once this percentage of the sweep's
                           workgroups have finished the sweep (their work then waits for the next sweep,
                           which spreads it over the whole grid); 1 .. 100 (100: never), 0 = default
                           (75) */
  int32_t pull_mode;    /* CLDIAM_PULL_*: offers over arcs that became light when Delta grew, and from the
                           sources of a new stage, can only reach unreached nodes.  In pull mode those
                           nodes take their best offer from their neighbours, reading keys written
                           earlier in the same pass (and NEXT is computed from their side), instead of
                           the blocked nodes pushing to them.  Results are the same in every mode.
                           CLUSTER2 and the literal steps never pull. */
} cldiam_tuning;
#define CLDIAM_BUCKET_DEFAULT 8.0f
#define CLDIAM_PULL_AUTO 0    /* pull from the first stage on when rows of more than 8x the average degree
                                 hold more than 1/8 of the arcs; else switch to pull mode once the heavy
                                 arcs of the blocked rows exceed 8 per unreached node */
#define CLDIAM_PULL_NEVER 1
#define CLDIAM_PULL_ALWAYS 2  /* pull from the first stage on */

/* One graph description of a batch (graph operand in DEVICE memory). */
typedef struct {
  int32_t n;
  int32_t pad;
  int64_t m;
  const int64_t *d_row_ptr; /* n+1 arc offsets, as passed to cldiam_load_csr */
  const uint64_t *d_arcs;   /* m packed arcs from cldiam_load_csr */
  uint64_t weight_sum;      /* sum of arc weights (cldiam_load_csr) */
  cldiam_params params;
  int32_t *d_cluster;       /* out, n */
  uint64_t *d_D;            /* out, n */
} cldiam_graph;

/* Workspace for a batch whose node counts sum to total_n (over num_graphs). */
size_t cldiam_decompose_workspace_size(int64_t total_n, int32_t num_graphs);

/* Decomposes num_graphs independent graphs in one device job; per-graph
 * results equal those of separate single-graph calls.  h_stats (host,
 * num_graphs entries, may be NULL) receives per-graph statistics.
 * driver: one of CLDIAM_DRIVER_*; tuning may be NULL (defaults).  A failure of one graph is reported in its
 * stats status and as the return value (the first failing graph's status). */
int cldiam_decompose_batch(int32_t num_graphs, const cldiam_graph *h_graphs, cldiam_stats *h_stats, int driver,
                           const cldiam_tuning *tuning, void *ws, size_t ws_bytes, void *stream);

/* Single-graph convenience form of cldiam_decompose_batch. */
int cldiam_decompose(const cldiam_graph *h_graph, cldiam_stats *h_stats, int driver, const cldiam_tuning *tuning,
                     void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------- continuous-batching server ---
 * A long-lived decomposition job for request streams.  Requests (one graph
 * each, same description as a batch entry) are queued by
 * cldiam_server_submit at any time; every cldiam_server_step admits queued
 * requests in arrival order while a slot and a free node range of the
 * workspace are available, advances every admitted graph together by up to
 * max_sweeps sweeps, and moves the graphs that finished to the completion
 * list read by cldiam_server_poll.  A finished graph's d_cluster / d_D hold
 * its results, identical to a cldiam_decompose call on the same graph; its
 * slot and node range are reused at once.  The server owns no device memory
 * beyond the caller's workspace (cldiam_server_workspace_size of the node
 * capacity and slot count); host state is released by cldiam_server_destroy.
 * A server is used from one host thread at a time. */
typedef struct cldiam_server cldiam_server;
size_t cldiam_server_workspace_size(int64_t node_capacity, int32_t max_graphs);
int cldiam_server_create(cldiam_server **out, int64_t node_capacity, int32_t max_graphs, const cldiam_tuning *tuning,
                         void *ws, size_t ws_bytes, void *stream);
void cldiam_server_destroy(cldiam_server *server);
/* Queues one request; CLDIAM_ENOMEM when the graph can never fit. */
int cldiam_server_submit(cldiam_server *server, const cldiam_graph *h_graph, uint64_t tag);
/* Admits, runs up to max_sweeps sweeps, collects finished requests; returns the
 * numbers of admitted (running) and still queued requests. */
int cldiam_server_step(cldiam_server *server, int32_t max_sweeps, int32_t *h_active, int32_t *h_queued);
/* Up to max_done finished requests (tags and statistics, oldest first). */
int cldiam_server_poll(cldiam_server *server, uint64_t *h_tags, cldiam_stats *h_stats, int32_t max_done,
                       int32_t *h_ndone);

/* ---------------------------------------------------- quotient graph ---
 * Weighted quotient graph G_C of Section 4: one node per cluster, numbered by
 * ascending center id; for every edge {u,v} of G with c_u != c_v an edge
 * between their clusters of weight w(u,v) + D_u + D_v; of parallel edges only
 * the lightest is kept.  Outputs (DEVICE, caller-sized for the worst case):
 *   d_qcenter[k]      center node id of quotient node i (ascending)
 *   d_qrow_ptr[k+1]   symmetric CSR offsets (int64), rows sorted by column
 *   d_qcol[<= m]      quotient neighbours
 *   d_qw[<= m]        quotient weights (u64)
 * and on the host *h_k = k and *h_qm = number of quotient arcs (2 x edges).
 * Arrays sized n+1 (row_ptr), n (center) and m (col, w) always suffice.
 * d_cluster must label every node with a center (a node c with
 * d_cluster[c] = c), as cldiam_decompose does; any other labelling returns
 * CLDIAM_EINVAL before a label is used as an index.  More than 2^32 - 1
 * distinct cluster pairs after the per-workgroup aggregation return
 * CLDIAM_EOVERFLOW. */
size_t cldiam_quotient_workspace_size(int32_t n, int64_t m);
int cldiam_build_quotient(int32_t n, int64_t m, const int64_t *d_row_ptr, const uint64_t *d_arcs,
                          const int32_t *d_cluster, const uint64_t *d_D, int32_t *d_qcenter, int64_t *d_qrow_ptr,
                          int32_t *d_qcol, uint64_t *d_qw, int32_t *h_k, int64_t *h_qm, void *ws, size_t ws_bytes,
                          void *stream);

/* ---------------------------------------------------------- estimate ---
 * Phi(G_C) = exact largest finite shortest-path distance between two nodes of
 * the quotient graph (k nodes, symmetric CSR from cldiam_build_quotient), and
 * Phi_approx = Phi(G_C) + 2 radius, the conservative estimate of Section 4
 * (radius = max D of the decomposition).  Results on the host.  Row offsets
 * that do not run from 0 to qm without decreasing, or a column outside
 * [0, k), return CLDIAM_EINVAL before the CSR is traversed. */
size_t cldiam_estimate_workspace_size(int32_t k, int64_t qm);
int cldiam_estimate_diameter(int32_t k, int64_t qm, const int64_t *d_qrow_ptr, const int32_t *d_qcol,
                             const uint64_t *d_qw, uint64_t radius, uint64_t *h_phi_gc, uint64_t *h_phi_approx,
                             void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same estimate
 * with no workspace argument.  Its scratch (control words and, above 3072
 * quotient nodes, per-workgroup distance and queue slices) is a static 32 MiB
 * device array of the library; each GPU holds its own copy from the first
 * call on that device until the process ends.  The call allocates nothing
 * (no device or pinned memory; results are read back into host stack memory).
 * k above CLDIAM_NOALLOC_MAX_K returns CLDIAM_EINVAL before any device work.
 * Every call on one GPU uses that GPU's array: calls that overlap in time on
 * the same GPU (from several threads or streams) race and must not be made.
 * Results are identical to cldiam_estimate_diameter's. */
#define CLDIAM_NOALLOC_MAX_K 32768
int cldiam_estimate_diameter_noalloc(int32_t k, int64_t qm, const int64_t *d_qrow_ptr, const int32_t *d_qcol,
                                     const uint64_t *d_qw, uint64_t radius, uint64_t *h_phi_gc,
                                     uint64_t *h_phi_approx, void *stream);

/* ------------------------------------------------ SSSP (the competitor) ---
 * Delta-stepping single-source shortest paths (Meyer and Sanders), the
 * baseline of Section 5: twice the largest finite distance from one source is
 * a 2-approximation of the diameter.  d_dist[v] receives the exact distance
 * (0xFFFFFFFF = unreachable); *h_max_dist the largest finite one.
 * bucket_delta = 0 picks the default width: 16 x floor(sum of arc weights /
 * m), at least 1 and at most 2^31 (1 on a graph without arcs), computed on
 * the device from d_arcs.  A finite distance >= 0xFFFFFFFF returns
 * CLDIAM_EOVERFLOW. */
size_t cldiam_sssp_workspace_size(int32_t n, int64_t m);
int cldiam_sssp_delta_stepping(int32_t n, int64_t m, const int64_t *d_row_ptr, const uint64_t *d_arcs,
                               int32_t source, uint32_t bucket_delta, uint32_t *d_dist, uint64_t *h_max_dist,
                               void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CLDIAM_H */
