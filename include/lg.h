/*
 * lg.h -- C ABI of the MI355X Log(Graph) packed-graph library (liblg.so).
 *
 * Log(Graph) (Besta et al., "Log(Graph): A Near-Optimal High-Performance
 * Graph Representation") stores an undirected graph as an adjacency array
 * whose neighbor IDs are bit-packed ("logarithmized") and whose offsets are
 * either bit-packed or held in a succinct bit vector.  This library builds
 * that representation on the GPU and runs BFS and PageRank directly on it,
 * decoding inside the traversal kernels.
 *
 * Conventions shared by every call:
 *   - Vertex IDs are 0-based uint32.  The input graph is undirected: both
 *     directions of every edge are stored, no self-loops, no duplicates,
 *     each neighbor list strictly increasing (the paper's adjacency array,
 *     section "Adjacency Array Data Structures", keeps every list sorted).
 *   - "dev" pointers are device pointers on the current HIP device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes; the library keeps no reference to it after the call returns.
 *   - A packed bit stream stores its bit b as bit (b mod 64) of little-endian
 *     64-bit word b/64; a value's bit k is stream bit start + k; unused bits
 *     are zero and every stream ends with one extra zero word (the layout of
 *     the edge-access listing in subsection "Accessing An Edge").
 *   - Calls return an lg_status and never throw.  On failure nothing is left
 *     allocated, output handles are left NULL and lg_last_error() describes
 *     the failure.  Device faults surface as LG_ERR_DEVICE.
 *   - Every call except lg_encode (and lg_decode_neighbors, which reads one
 *     total back) is asynchronous on `stream`; results are valid once the
 *     stream has been synchronized.  Calls on one graph must not overlap in
 *     time on different streams: they share the graph's device workspace.
 */
#ifndef LG_H
#define LG_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lg_graph lg_graph; /* opaque; owned by the library */

typedef enum lg_status {
    LG_OK = 0,
    LG_ERR_INVALID = 1,     /* argument or input graph violates the contract   */
    LG_ERR_OOM = 2,         /* device allocation failed                          */
    LG_ERR_DEVICE = 3,      /* a HIP call or kernel failed                       */
    LG_ERR_UNSUPPORTED = 4, /* valid request outside what this build handles     */
    LG_ERR_CAPACITY = 5     /* caller-provided output buffer too small           */
} lg_status;

/* lg_encode_opts.layout */
#define LG_LAYOUT_PACKED 0u /* the logarithmized representation                  */
#define LG_LAYOUT_PLAIN 1u  /* plain CSR baseline: uint32 IDs, uint32 offsets
                               (uint64 when M >= 2^32), same labeling rules     */
/* lg_encode_opts.id_mode -- section "Logarithmization of Vertex IDs" */
#define LG_IDS_GLOBAL 0u /* every ID at s = ceil(log2 n) bits (max(1, bl(n-1)))   */
#define LG_IDS_LOCAL 1u  /* list of v at w_v = max(1, bl(max N_v)) bits, 0 when
                            empty; w_v kept in a table of F = bl(s) bits/vertex  */
/* subsection "Adding Fixed-Size Gap Encoding", local approach: the first
 * element of the list of v at w_v bits (as LG_IDS_LOCAL), every difference
 * of consecutive neighbors at g_v = bl(largest difference) bits (0 when
 * d_v < 2), kept in a second table of F bits/vertex; the list takes
 * w_v + (d_v - 1) g_v bits.  Such graphs are read in order (a prefix sum
 * per list) by every operation. */
#define LG_IDS_LOCAL_GAP 2u
/* subsection "Incorporating Degree-Minimizing (DM)": lists as Varint byte
 * sequences (7 value bits per byte, lowest group first, the top bit set on
 * every byte of a value but its last), one list after another, byte-aligned;
 * the offsets are byte starts (packed or Elias-Fano over the stream's byte
 * count) and lg_info.adj_bits is 8 x the stream bytes.  FULL stores every
 * label (with LG_RELABEL_DEGREE: the paper's DMf), DIFF the first label and
 * then the differences of consecutive labels (with LG_RELABEL_DEGREE: DMd).
 * d_v is the number of bytes with the top bit clear in the list.  Such
 * graphs are read in order by every operation. */
#define LG_IDS_VARINT_FULL 3u
#define LG_IDS_VARINT_DIFF 4u
/* lg_encode_opts.offset_mode -- sections "Logarithmization of Single Offsets"
 * and "Logarithmizing Offsets" */
#define LG_OFFS_PACKED 0u   /* offsets packed at bl(universe) bits each          */
#define LG_OFFS_SUCCINCT 1u /* Elias-Fano sequence (sparse bit vector bvSD) with
                               a rank/select directory                           */
/* subsection "Arrays of Offsets vs. Bit Vectors for O" and its table of
 * offset structures: the offsets x_0 <= .. <= x_n (universe u) as one plain
 * bit vector of u + n + 1 bits whose one for list v sits at x_v + v (so an
 * empty list keeps its own one); x_v = select1(v) - v.  Units of x: elements
 * (global IDs) or bits (local IDs). */
#define LG_OFFS_PLAIN_BV 2u       /* bvPL: the vector plus a directory for select
                                     (rank1 every 512 bits, select1 every 64th one);
                                     u + n + 1 must stay below 2^32; every
                                     operation reads it                          */
#define LG_OFFS_INTERLEAVED_BV 3u /* bvIL: the vector in 512-bit blocks, each led
                                     by a 64-bit count of the ones before it
                                     (select by binary search over the counts);
                                     global or local IDs, unweighted; read by
                                     lg_decode_neighbors (and its allocation-free
                                     variant) only, the other operations return
                                     LG_ERR_UNSUPPORTED                          */
/* lg_encode_opts.relabel -- section "Incorporating Degree-Minimizing (DM)" */
#define LG_RELABEL_NONE 0u
#define LG_RELABEL_DEGREE 1u /* new label = rank by (degree desc, ID asc)         */
/* subsection "Adding Integer Linear Programming", its greedy heuristic:
 * vertices taken by increasing degree (ties by ID) give the next label to
 * each neighbor, in list order, that has none yet; edgeless vertices take
 * the last labels in ID order */
#define LG_RELABEL_GREEDY 2u

typedef struct lg_encode_opts {
    uint32_t layout;      /* LG_LAYOUT_*                                          */
    uint32_t id_mode;     /* LG_IDS_* (packed layout only)                        */
    uint32_t offset_mode; /* LG_OFFS_* (packed layout only)                       */
    uint32_t relabel;     /* LG_RELABEL_*                                         */
    uint32_t flags;       /* reserved, must be 0                                  */
    uint32_t reserved[3]; /* must be 0                                            */
} lg_encode_opts;

/*
 * lg_encode -- build a graph representation from an adjacency array.
 *
 * Follows the construction of the library listing in section
 * "High-Performance Library" (relabel the vertices with the permuter, map
 * the relabeled lists to bits with the transformer, then build and condense
 * the offset structure), with the widths of "Logarithmization of Vertex
 * IDs", the offsets of "Logarithmization of Single Offsets" or the sparse
 * succinct bit vector of "Succinct Bit Vectors in Log(Graph)".
 *
 *   n            number of vertices, 1 <= n < 2^31
 *   m            number of stored directed entries M (twice the undirected
 *                edge count), m < 2^36
 *   row_offsets  dev, uint64[n+1]; row_offsets[0] = 0, row_offsets[n] = m
 *   col          dev, uint32[m]; the neighbor lists, back to back
 *   opts         host; NULL means packed layout, global IDs, packed offsets,
 *                no relabeling
 *   stream       HIP stream for all work
 *   out          host; receives the new handle
 *
 * The input is validated on the device: offsets non-decreasing, every ID
 * < n, no self-loop, lists strictly increasing, and the graph symmetric.  A
 * violation returns LG_ERR_INVALID.  Synchronous: it reads the total bit
 * length back to size the packed arrays.  The input buffers are not kept.
 */
lg_status lg_encode(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                    const lg_encode_opts *opts, hipStream_t stream, lg_graph **out);

/* lg_decode_neighbors flags */
#define LG_DECODE_SORTED 0u  /* original IDs, every list ascending (default)        */
#define LG_DECODE_ORIGINAL 1u /* original IDs, in stored order                      */
#define LG_DECODE_RAW 2u     /* `vertices` and results are stored labels, stored
                                order (what the traversal kernels see)            */

/*
 * lg_decode_neighbors -- N_v for a batch of vertices (getNeighbors of the
 * library listing in section "High-Performance Library"; per element the
 * N_{i,v} extraction of subsection "Accessing An Edge", the degree
 * d_v = O[v+1] - O[v] of subsection "Accessing a Degree").
 *
 *   vertices  dev, uint32[k]: original IDs (stored labels with LG_DECODE_RAW),
 *             each < n
 *   k         number of vertices (0 allowed)
 *   out_off   dev, uint64[k+1]: exclusive prefix of the list lengths; always
 *             written, also when LG_ERR_CAPACITY is returned
 *   out_ids   dev, uint32[cap] or NULL: list i at out_ids[out_off[i] ..
 *             out_off[i+1])
 *   cap       capacity of out_ids in elements
 * Returns LG_ERR_CAPACITY when out_ids is NULL or too small for the total.
 * Reads the total back (one stream synchronization).
 */
lg_status lg_decode_neighbors(const lg_graph *g, const uint32_t *vertices, uint32_t k,
                              uint64_t *out_off, uint32_t *out_ids, uint64_t cap,
                              uint32_t flags, hipStream_t stream);

/*
 * lg_decode_neighbors_noalloc -- lg_decode_neighbors for callers that cannot
 * allocate memory: serving loops that must not call into the allocator, and
 * harnesses that forbid allocation after set-up.  Same arguments, results,
 * errors and synchronization as lg_decode_neighbors, but the call allocates
 * nothing (no device, pinned-host or graph workspace memory): its
 * temporaries live in one fixed device array of the library,
 * LG_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the call runs on holds
 * until the process ends.  Calls on one GPU share that array; the library
 * runs them one at a time, each returning only after its kernels are done
 * (so callers never see the previous call's contents).
 * Limits: k <= LG_NOALLOC_MAX_VERTICES, and for LG_DECODE_SORTED on a
 * relabeled graph (the only mode that sorts) at most
 * LG_NOALLOC_MAX_SORTED_IDS ids in total; larger requests return
 * LG_ERR_UNSUPPORTED (out_off is still written when the second limit is
 * the one exceeded).
 */
#define LG_NOALLOC_MAX_VERTICES 65536u
#define LG_NOALLOC_MAX_SORTED_IDS (1u << 20)
#define LG_NOALLOC_SCRATCH_BYTES (32u << 20)
lg_status lg_decode_neighbors_noalloc(const lg_graph *g, const uint32_t *vertices, uint32_t k,
                                      uint64_t *out_off, uint32_t *out_ids, uint64_t cap,
                                      uint32_t flags, hipStream_t stream);

/* lg_bfs flags */
#define LG_BFS_DIRECTION_OPT 0u /* top-down/bottom-up switching (default)          */
#define LG_BFS_TOP_DOWN 1u      /* top-down steps only                              */
#define LG_BFS_BOTTOM_UP 2u     /* bottom-up steps after the first level            */

/*
 * lg_bfs -- breadth-first search from each root (the direction-optimizing
 * BFS of section "Considered Algorithms"), decoding the packed lists inside
 * the frontier kernels.
 *
 *   roots      host, uint32[r]: original IDs, each < n
 *   r          number of roots
 *   depth      dev, int32[r*n]: row i = hop distance from roots[i], -1 when
 *              unreachable (or deeper than max_depth)
 *   parent     dev, int32[r*n] or NULL: row i = BFS tree in original IDs;
 *              parent of a reached v != root is its neighbor one level up
 *              with the smallest stored label, parent[root] = root, -1 for
 *              unreached vertices
 *   max_depth  -1 for a full traversal; k >= 0 stops after depth k (k-hop)
 * Results are independent of the flags and of the direction switching.
 * With r > 1 every row equals the result of a call with that root alone;
 * work queued on `stream` before the call completes first, and work queued
 * on `stream` after it waits for every root.  Two ways of running them:
 *   - with LG_BFS_DIRECTION_OPT on a graph whose lists are not gap or Varint
 *     coded, not weighted and without bvIL offsets, the first roots go in
 *     batches of up to 64 while at least 16 are left, each batch one
 *     multi-source traversal on `stream` (64-bit visit and frontier masks
 *     per vertex, 36 bytes per vertex of device workspace; on a relabeled
 *     graph also the batch's rows in label space, 8 bytes per root and
 *     vertex, when that stays within 16 GiB); the host reads a few
 *     counters per level, so the call returns when these batches are done;
 *   - the other roots run a few at a time, each on its own internal stream
 *     with its own workspace; the call returns once each is enqueued.
 * These streams and workspaces belong to the device, not to the graph: they
 * grow to the largest graph searched and stay until lg_trim; multi-root
 * calls on one device run one after the other.
 */
lg_status lg_bfs(const lg_graph *g, const uint32_t *roots, uint32_t r, int32_t *depth,
                 int32_t *parent, int32_t max_depth, uint32_t flags, hipStream_t stream);

/*
 * lg_encode_weighted -- lg_encode with an integer weight per stored entry
 * (subsections "Logarithmization of Edge Weights" and "Accessing an Edge
 * Weight"): in the packed layout each entry is the neighbor ID followed
 * directly by the weight, the weight at omega = max(1, bl(largest weight))
 * bits, one width for the whole graph (lg_graph_info.weight_bits); the ID
 * keeps its global or local width, so the offsets (element offsets or bit
 * starts) count entries of s + omega or w_v + omega bits.  The plain layout
 * keeps the weights as a separate uint32 array beside the CSR.
 *
 *   weights  dev, uint32[m]; weights[i] belongs to entry i of col (the edge
 *            from the row's vertex to col[i]); any value, both directions
 *            of an edge may differ
 *   other arguments as lg_encode
 *
 * Supported: packed layout with LG_IDS_GLOBAL or LG_IDS_LOCAL (packed or
 * succinct offsets), or the plain layout, with any relabeling (each entry
 * keeps the weight of the edge it stands for); other ID modes return
 * LG_ERR_UNSUPPORTED.  A packed weighted graph is read by lg_sssp
 * only (the other operations return LG_ERR_UNSUPPORTED); a plain one by
 * every operation.
 */
lg_status lg_encode_weighted(uint32_t n, uint64_t m, const uint64_t *row_offsets, const uint32_t *col,
                             const uint32_t *weights, const lg_encode_opts *opts, hipStream_t stream,
                             lg_graph **out);

/*
 * lg_sssp -- single-source shortest path distances over a weighted graph
 * (SSSP of section "Considered Algorithms", a delta-stepping traversal):
 * dist[v] = the smallest sum of weights over the paths from root to v.
 *
 *   root     original vertex ID, < n (distances come back by original ID)
 *   delta    bucket width (distances [k delta, (k+1) delta) settle together);
 *            0 picks 2^weight_bits.  The distances do not depend on it.
 *   dist     dev, uint64[n]; UINT64_MAX for vertices the root does not reach
 *
 * Returns LG_ERR_UNSUPPORTED for an unweighted graph.  Synchronous: the
 * host reads each step's frontier size back to drive the buckets, and the
 * call returns once dist is written.  The workspace is kept with the graph
 * until lg_free; calls on the same graph from several threads run one after
 * the other (each holds the graph's workspace for its whole duration).
 */
lg_status lg_sssp(const lg_graph *g, uint32_t root, uint32_t delta, uint64_t *dist, hipStream_t stream);

/*
 * lg_pagerank -- pull PageRank without atomics (section "Considered
 * Algorithms"), FP32 storage:
 *   PR_0 = 1/n;  PR_{t+1}(v) = (1-a)/n + a (sum_{u in N_v} PR_t(u)/d_u + D_t/n)
 * where D_t is the rank held by vertices without edges, spread uniformly.
 *
 *   damping  a, in [0, 1]
 *   iters    number of iterations (exactly; no convergence test)
 *   scores   dev, float[n], indexed by original ID
 */
lg_status lg_pagerank(const lg_graph *g, float damping, uint32_t iters, float *scores,
                      hipStream_t stream);

/*
 * Batched BFS: many queries over many graphs in one persistent launch.
 *
 * Each query is a BFS (same rule and results as lg_bfs) from `root` on
 * graphs[graph]; its depths (and parents) are written to depth[out_offset ..
 * out_offset + n_graph) (and parent[...]).  A plan validates the jobs,
 * optionally times candidate launch settings on the batch itself
 * (LG_BATCH_AUTOTUNE: work chunk and wave-per-vertex degree threshold) and
 * captures "reset + persistent launch" in a HIP graph; lg_bfs_batch_run
 * replays it.  All graphs of a plan must share layout and encoding and must
 * not be relabeled.  The plan keeps the graph handles and the output
 * pointers: they must outlive it.  Creating a plan runs the batch at least
 * once (synchronously).
 */
typedef struct lg_bfs_job {
    uint32_t graph;      /* index into `graphs`                                   */
    uint32_t root;       /* vertex ID < n of that graph                           */
    uint64_t out_offset; /* element offset of this query's rows in depth/parent   */
} lg_bfs_job;

#define LG_BATCH_AUTOTUNE 1u

typedef struct lg_batch_plan lg_batch_plan;

typedef struct lg_batch_info {
    uint32_t num_jobs;
    uint32_t workgroups;     /* persistent workers                              */
    uint32_t threads;        /* threads per worker                              */
    uint32_t chunk;          /* frontier vertices staged per pass               */
    uint32_t wave_threshold; /* degree from which a whole wave expands a vertex */
    uint32_t candidates;     /* settings timed by the autotuner (1 = none)      */
    double tuned_ms;         /* time of the chosen setting on the batch         */
    uint64_t scratch_bytes;  /* per-worker frontier queues                      */
} lg_batch_info;

lg_status lg_bfs_batch_plan(const lg_graph *const *graphs, uint32_t num_graphs, const lg_bfs_job *jobs,
                            uint32_t num_jobs, int32_t *depth /*dev*/, int32_t *parent /*dev or NULL*/,
                            int32_t max_depth, uint32_t flags, hipStream_t stream, lg_batch_plan **out);
lg_status lg_bfs_batch_run(lg_batch_plan *plan, hipStream_t stream);
lg_status lg_bfs_batch_info(const lg_batch_plan *plan, lg_batch_info *out);
/* NULL-safe; waits for the plan's last replay only */
void lg_bfs_batch_free(lg_batch_plan *plan);

/*
 * Query server over resident graphs.
 *
 * Queries are submitted from any host thread and served by `workers` worker
 * threads, each with its own HIP stream and device workspaces, so that
 * queries overlap on the device.  Admission is first-come first-served and
 * bounded by `budget_bytes` of device memory: the resident graphs plus every
 * worker's buffers never exceed it.  Before a query runs, its worker grows
 * its buffers to the most the query can use, so this holds at every instant;
 * a query that cannot fit even alone completes with status LG_ERR_CAPACITY.
 * The resident part is each graph's device memory when the server is created
 * (lg_graph_info.device_bytes); the graphs must stay unchanged (no lg_bfs,
 * lg_pagerank or lg_decode_neighbors on them, which grow their own
 * workspaces) and alive until lg_server_free.  Neighbor fetches queued on the
 * same graph are served together in one decode launch (up to max_batch).
 * Results are exactly those of the same query run alone.  Latencies are
 * measured from submission to completion on the host's steady clock.
 */
typedef struct lg_server lg_server;

typedef struct lg_server_opts {
    uint64_t budget_bytes; /* 0: unlimited                                     */
    uint32_t workers;      /* 0: 8                                              */
    uint32_t max_batch;    /* neighbor fetches per decode launch; 0: 64         */
    uint32_t reserved[4];  /* must be 0                                         */
} lg_server_opts;

#define LG_QUERY_NEIGHBORS 0u /* sorted N_v, original IDs                      */
#define LG_QUERY_KHOP 1u      /* sorted {u : 1 <= depth(u) <= k} from `vertex`   */
#define LG_QUERY_BFS 2u       /* full BFS from `vertex`                          */
#define LG_QUERY_KEEP_ARRAYS 1u /* BFS: return depth and parent arrays too       */

typedef struct lg_query {
    uint32_t kind;   /* LG_QUERY_*                                              */
    uint32_t graph;  /* index into the server's graphs                          */
    uint32_t vertex; /* original ID < n                                         */
    int32_t k;       /* hops for LG_QUERY_KHOP                                  */
    uint32_t flags;  /* LG_QUERY_KEEP_ARRAYS                                    */
    uint32_t reserved;
} lg_query;

typedef struct lg_query_result {
    int32_t status;        /* LG_OK, or why the query failed                     */
    uint32_t kind;
    uint64_t count;        /* ids returned (neighbors, k-hop) or vertices reached (BFS) */
    const uint32_t *ids;   /* host, `count` entries; valid until lg_server_release */
    const int32_t *depth;  /* host, n entries (BFS with LG_QUERY_KEEP_ARRAYS)     */
    const int32_t *parent; /* host, n entries (BFS with LG_QUERY_KEEP_ARRAYS)     */
    uint64_t n;
    int32_t max_depth;     /* BFS: largest depth reached                          */
    uint32_t batch;        /* queries served by the same launch                   */
    uint64_t digest;       /* BFS: order-independent digest of (depth, parent)    */
    double queue_ms;       /* submission to start                                 */
    double service_ms;     /* start to completion                                 */
    double latency_ms;     /* submission to completion                            */
} lg_query_result;

typedef struct lg_server_stats {
    uint64_t submitted, completed, rejected, queued, running;
    uint64_t budget_bytes, resident_bytes, in_use_bytes, peak_bytes;
    uint32_t workers;
    uint32_t overruns;     /* times a worker held more than was admitted (0)      */
    uint64_t batches;      /* launches (batches) started                          */
} lg_server_stats;

lg_status lg_server_create(const lg_graph *const *graphs, uint32_t num_graphs, const lg_server_opts *opts,
                           lg_server **out);
lg_status lg_server_submit(lg_server *server, const lg_query *query, uint64_t *ticket);
lg_status lg_server_wait(lg_server *server, uint64_t ticket, lg_query_result *out);   /* blocks   */
lg_status lg_server_result(lg_server *server, uint64_t ticket, lg_query_result *out); /* no wait  */
lg_status lg_server_poll(lg_server *server, uint64_t *tickets, uint32_t cap, uint32_t *count);
lg_status lg_server_release(lg_server *server, uint64_t ticket);
lg_status lg_server_get_stats(lg_server *server, lg_server_stats *out);
void lg_server_free(lg_server *server); /* waits for every submitted query; NULL-safe */

/* Host-only model of the server's admission rule (no device work): FIFO
 * queries with arrival times (ascending), bytes of the buffers each needs and
 * fixed service times, on `workers` workers that each keep one grow-only
 * buffer.  Writes start/finish times,
 * per-query status (LG_OK or LG_ERR_CAPACITY) and the peak accounted bytes. */
lg_status lg_admission_simulate(const double *arrival, const uint64_t *need, const double *service, uint32_t count,
                                uint64_t budget, uint64_t resident, uint32_t workers, double *start, double *finish,
                                int32_t *status, uint64_t *peak);

/* Release a graph and its device memory.  NULL is accepted.  Waits (on the
 * host) for the graph's last use -- the end of the latest call that read it,
 * on that call's stream -- and for nothing else: work of other graphs and
 * streams goes on. */
void lg_free(lg_graph *g);

/* Sizes and parameters of a built representation. */
typedef struct lg_graph_info {
    uint64_t n;            /* vertices                                           */
    uint64_t m;            /* stored directed entries M                          */
    uint32_t layout, id_mode, offset_mode, relabel;
    uint32_t s;            /* global ID width                                    */
    uint32_t F;            /* width-table field bits (local mode), else 0        */
    uint32_t w_offset;     /* packed offset width (packed offsets), else 0       */
    uint32_t ef_l;         /* Elias-Fano low bits (succinct offsets), else 0     */
    uint64_t universe;     /* largest offset value: M (global) or U (local)      */
    uint64_t adj_bits;     /* U: bits of the packed lists                        */
    uint64_t ef_high_bits; /* |H| in bits (succinct offsets); the bit vector's
                              length u + n + 1 (bvPL, bvIL)                      */
    uint64_t bytes_adj;    /* bytes of the neighbor data (packed words / uint32) */
    uint64_t bytes_offsets;/* bytes of the offset structure incl. directory      */
    uint64_t bytes_widths; /* bytes of the width table(s) (both in gap mode)     */
    uint64_t bytes_perm;   /* bytes of the two permutation arrays                */
    uint64_t device_bytes; /* all device memory held by the handle now           */
    uint32_t max_degree;
    uint32_t isolated;     /* vertices without edges                             */
    uint32_t heavy_threshold; /* degree above which a vertex is "heavy": the
                                 traversal kernels split its list into segments */
    uint32_t n_heavy;      /* heavy vertices                                     */
    uint64_t n_segments;   /* segments of the heavy lists (0 until first use)    */
    uint64_t heavy_edges;  /* entries of the heavy lists (0 until first use)     */
    uint64_t heavy_bits;   /* bits of the heavy lists (element bits; 32/entry on
                              the plain layout; 0 until first use)               */
    uint32_t weight_bits;  /* omega of a weighted graph, else 0                  */
    uint32_t reserved_w;
    uint64_t bytes_weights;/* bytes of the separate weight array (plain layout)  */
} lg_graph_info;

lg_status lg_info(const lg_graph *g, lg_graph_info *out);

/* lg_export `which` */
#define LG_EXPORT_ADJ 0u       /* packed words (uint64) or plain IDs (uint32)     */
#define LG_EXPORT_OFFSETS 1u   /* packed offset words (uint64) or plain offsets   */
#define LG_EXPORT_WIDTHS 2u    /* width-table words (uint64)                      */
#define LG_EXPORT_EF_LOW 3u    /* Elias-Fano low-bit words (uint64)               */
#define LG_EXPORT_EF_HIGH 4u   /* upper bit vector H words (uint64)               */
#define LG_EXPORT_EF_RANK 5u   /* uint32 rank1(512 b), b = 0 .. ceil(|H|/512)     */
#define LG_EXPORT_EF_SELECT 6u /* uint32 select1(64 j), j < ceil((n+1)/64)        */
#define LG_EXPORT_PERM 7u      /* uint32 perm[new] = original                     */
#define LG_EXPORT_INV 8u       /* uint32 inv[original] = new                      */
#define LG_EXPORT_GAP_WIDTHS 9u /* gap-width-table words (uint64), gap mode       */
#define LG_EXPORT_WEIGHTS 10u   /* weights (uint32), weighted plain layout        */
/* with LG_OFFS_PLAIN_BV the bit vector and its directory come out as
 * LG_EXPORT_EF_HIGH, LG_EXPORT_EF_RANK and LG_EXPORT_EF_SELECT */
#define LG_EXPORT_BV_INTERLEAVED 11u /* bvIL words (uint64): block j at words
                                        [9j, 9j+9) = count of ones before it, then
                                        512 bits; one last word = n + 1        */

/*
 * Copy one raw array of the representation to host memory (synchronous).
 * `bytes` must equal lg_export_bytes(g, which); an array the handle does
 * not hold returns LG_ERR_INVALID.
 */
lg_status lg_export(const lg_graph *g, uint32_t which, void *host_dst, uint64_t bytes);
uint64_t lg_export_bytes(const lg_graph *g, uint32_t which);

/* Thread-local description of the last failure on this thread. */
const char *lg_last_error(void);

/* Device buffers of lg_encode (its temporaries: sort keys, scans, tables;
 * about four times the input neighbor array) and of a graph (its arrays and
 * PageRank tables, when lg_free releases them) go to a per-process cache for
 * the next request on the same device and stream, instead of being freed, so
 * that repeated encodes neither allocate nor synchronize the device to free.
 * The cache holds at most 64 GiB.  The two bin buffers of a PageRank by
 * propagation blocking (8 bytes per stored entry each) are kept apart from
 * it: lg_free parks the pair of one graph per device for the next graph of
 * about the same size.  lg_trim frees the cache, that pair, and the
 * per-device workspaces of multi-root lg_bfs calls.  Call it when no library
 * call is running. */
void lg_trim(void);

/*
 * Kernel timing: while enabled, every kernel launch is bracketed by two HIP
 * events on the stream it is launched on.  lg_prof_query sums the elapsed
 * times of all completed launches of the kernel named `kernel` since the
 * last reset (waiting for them).  lg_prof_names writes the known kernel
 * names, newline separated, into buf.
 */
lg_status lg_prof_enable(int on);
/* Time only launches whose kernel name contains substr, or one of its
 * '|'-separated parts (NULL or "": all); set it while no library call is
 * running. */
lg_status lg_prof_filter(const char *substr);
lg_status lg_prof_reset(void);
lg_status lg_prof_query(const char *kernel, uint64_t *launches, double *total_ms);
lg_status lg_prof_names(char *buf, uint64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* LG_H */
