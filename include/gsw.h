/*
 * gsw.h -- graph-property-switched breadth-first search on MI355X (gfx950).
 *
 * C ABI of libgsw.so.  Plain pointers and sizes only; no C++ types cross it
 * and no C++ exception escapes it.  Every call returns a gsw_status; on a
 * non-OK status gsw_last_error() holds a message for the calling thread and
 * the contents of output buffers are unspecified.  GSW_EHIP reports a failed
 * HIP runtime call; HIP errors can be sticky, so a process that sees it
 * should not keep using the device.
 *
 * The method (Verstraaten, Varbanescu, de Laat, "Using Graph Properties to
 * Speed-up GPU-based Graph Traversal: A Model-driven Approach", 2017):
 * level-synchronous BFS whose frontier expansion at each level is done by one
 * of several interchangeable kernels (Section III-A), the kernel being chosen
 * per level by a binary decision tree over graph and frontier properties
 * (Section IV-A), with the paper's rule for undecided leaves.
 *
 * Graph convention: CSR with int64 row offsets and int32 column ids,
 * 1 <= n < 2^31 vertices.  Row v lists the out-neighbours of v (the arcs
 * v -> u); an undirected graph stores every edge as two arcs.  Self-loops and
 * repeated entries are tolerated and do not change any result.  A graph whose
 * arcs do not all have their reverse is directed: the library then also
 * keeps the transpose (the in-arcs of every vertex), over which the
 * bottom-up and reverse-edge-list kernels run.
 *
 * Ownership: the caller owns every buffer it passes and the library never
 * frees them.  Objects returned through gsw_*_create are owned by the caller
 * and released with the matching gsw_*_destroy.
 *
 * Threading: calls on one gsw_graph are serialised internally (one BFS at a
 * time per graph).  Different graphs may be used from different threads.
 */
#ifndef GSW_H
#define GSW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSW_ABI_VERSION 4

typedef enum {
  GSW_OK = 0,
  GSW_EINVAL = -1,   /* malformed argument or graph */
  GSW_ENOMEM = -2,   /* device or host allocation failed */
  GSW_EHIP = -3,     /* a HIP runtime call failed */
  GSW_ERANGE = -4,   /* a result does not fit its type (int8 levels > 127) */
  GSW_EBUSY = -5,    /* no free slot */
  GSW_ENOTREE = -6,  /* tree policy without a tree */
  GSW_ENOTSYM = -7   /* reserved (bottom-up kernels run on directed graphs over in-arcs) */
} gsw_status;

/*
 * Frontier-expansion kernels (Section III-A).  Each one performs a whole BFS
 * level: given the vertices at depth d it finds every unvisited vertex
 * adjacent to them, gives it depth d+1 and a parent at depth d, and emits the
 * next frontier both as a queue and as a bitmap, so any kernel may follow any
 * other at the next level.
 */
enum {
  GSW_K_PUSH_VERTEX = 0,  /* top-down, one lane per frontier vertex ("vertex push") */
  GSW_K_PUSH_WAVE4 = 1,   /* top-down, W lanes cooperate on each frontier vertex, */
  GSW_K_PUSH_WAVE8 = 2,   /*   W vertices per group ("vertex push warp", virtual */
  GSW_K_PUSH_WAVE16 = 3,  /*   warps of W lanes inside a 64-lane wavefront)       */
  GSW_K_PUSH_WAVE32 = 4,
  GSW_K_PUSH_WAVE64 = 5,
  GSW_K_PUSH_EDGE = 6,    /* top-down, one lane per frontier edge (edge-centric) */
  GSW_K_PULL_BITMAP = 7,  /* bottom-up, one lane per unvisited vertex, early exit
                             on the first neighbour in the frontier bitmap ("vertex pull") */
  GSW_K_VERTEX_SCAN = 8,  /* vertex push over all n vertices, testing depth == d */
  GSW_K_EDGE_SCAN = 9,    /* edge list: one lane per arc over all arcs in source order,
                             testing the depth of the arc's origin (needs the origin array) */
  GSW_K_REV_EDGE_SCAN = 10, /* reverse edge list: one lane per arc over all arcs in
                             destination order (every vertex's in-arcs), testing the depth
                             of the arc's source (needs the in-arcs' origin array) */
  GSW_N_BASE_KERNELS = 11
};

/*
 * Frontier-count variants (Section III-A, "Variants"): how the lanes that
 * discover vertices add them to the next frontier, whose size is the level's
 * count.  WORKGROUP stages a workgroup's discoveries in LDS and reserves
 * their queue places with one global atomic per workgroup; WAVE with one per
 * wavefront (ballot and popcount); THREAD with one per discovering lane.  The
 * global counters are spread over 8 queue segments in every variant.  A
 * kernel id combines a base kernel and a variant; the plain GSW_K_* ids are
 * the WORKGROUP variant.
 */
enum { GSW_COUNT_WORKGROUP = 0, GSW_COUNT_WAVE = 1, GSW_COUNT_THREAD = 2, GSW_N_COUNT_VARIANTS = 3 };
#define GSW_N_KERNELS (GSW_N_BASE_KERNELS * GSW_N_COUNT_VARIANTS)
#define GSW_KERNEL_ID(base, variant) ((base) + GSW_N_BASE_KERNELS * (variant))
#define GSW_KERNEL_BASE(k) ((k) % GSW_N_BASE_KERNELS)
#define GSW_KERNEL_COUNT(k) ((k) / GSW_N_BASE_KERNELS)

/* Kernel used when the tree cannot decide at the first level (Section IV-A:
 * the edge-centric implementation, as the least likely to be very slow). */
#define GSW_DEFAULT_KERNEL GSW_K_PUSH_EDGE

/* Graph creation flags. */
#define GSW_ASSUME_SYMMETRIC 0x1u /* skip the symmetry check; caller vouches that every arc
                                     has its reverse */
#define GSW_WITH_ORIGIN 0x2u      /* build the per-arc origin array now, not on first use */
#define GSW_TRUSTED 0x4u          /* skip validation of offsets and columns */

/*
 * Per-level feature vector fed to the tree (Section IV-A feature list: graph
 * size, the 5-number summary and standard deviation of the out-, in- and
 * absolute degrees, frontier size and discovered count, each absolute and as
 * a fraction of n; the paper's best model uses graph size, fraction
 * discovered, the out-degree distribution and the frontier's vertex count,
 * Section IV-B):
 *    0 n vertices     2.. 7 out-degree {min, Q1, median, Q3, max, std}
 *    1 arcs (CSR      8..13 in-degree  {min, Q1, median, Q3, max, std}
 *      entries)      14..19 absolute degree {min, Q1, median, Q3, max, std}
 *   20 frontier vertices n_f(d)      22 discovered (depths 0..d)
 *   21 n_f(d) / n                    23 discovered / n
 * Quartiles interpolate linearly between order statistics; std is the
 * population one (ddof 0).  The absolute degree of v counts the arcs that
 * enter or leave v, an arc and its reverse once: out(v) + in(v) minus the
 * arcs v -> u whose reverse u -> v exists.  On a symmetric graph the three
 * distributions equal the degree distribution.  Features 0..19 are constant
 * for a graph.
 */
#define GSW_N_FEATURES 24
#define GSW_N_GRAPH_FEATURES 20

typedef struct gsw_graph gsw_graph;
typedef struct gsw_tree gsw_tree;

/* One row per BFS level and source. */
typedef struct {
  int32_t source_idx;   /* index into the sources array */
  int32_t level;        /* d: this row expanded the depth-d vertices */
  int32_t kernel;       /* kernel id (GSW_KERNEL_ID) that ran */
  int32_t flags;        /* bit0: tree leaf undecided, fallback rule applied;
                           bit2: run by a single-workgroup multi-level launch */
  int64_t n_frontier;   /* n_f(d): vertices at depth d */
  int64_t discovered;   /* vertices at depths 0..d */
  int64_t n_next;       /* vertices found at depth d+1 (0 on the last row) */
  int64_t e_frontier;   /* e_f(d): arcs leaving the depth-d vertices (sum of their
                           out-degrees), or -1 unless gsw_bfs_opts.count_arcs */
  float ms;             /* time of this level (device wall clock from its first
                           workgroup's start to its last one's end, both
                           launches of a two-launch push_edge level; see
                           time_levels), or -1 when not timed */
  int32_t launch;       /* index (from 0, per source) of the level-kernel launch that
                           completed this level (a push_edge level on more than 512
                           entries takes two launches; a single-workgroup launch
                           runs several levels; some launches complete none) */
} gsw_level_trace;

enum { GSW_POLICY_TREE = 0, GSW_POLICY_FIXED = 1, GSW_POLICY_SCHEDULE = 2 };

typedef struct {
  int32_t policy;            /* GSW_POLICY_* */
  int32_t fixed_kernel;      /* GSW_POLICY_FIXED: kernel for every level */
  const int32_t *schedule;   /* GSW_POLICY_SCHEDULE: kernel per level (host array); */
  int32_t schedule_len;      /*   levels beyond the end repeat the last entry */
  const gsw_tree *tree;      /* GSW_POLICY_TREE */
  int32_t time_levels;       /* fill gsw_level_trace.ms with each level's time.  1: the
                                level's first workgroup stamps the GPU's constant-rate
                                wall clock when it starts, its last workgroup reads the
                                clock when it ends and posts the difference in the
                                level's record.  2: HIP events recorded on the stream
                                after every launch of the level kernel; a level's time
                                runs from the event before its first launch to the one
                                after its last (what a kernel profiler reports for the
                                launches, with the events' own small cost) */
  int32_t canonical_parents; /* 1: parent[v] = smallest neighbour one level up */
  int32_t device_ptrs;       /* 1: levels/parents are device pointers; 0: host */
  int32_t max_workgroups;    /* > 0: cap on every level-kernel launch's workgroups (levels
                                that ask for more stride over their work; results are
                                the same); 0: the library sizes each launch */
  int32_t count_arcs;        /* 1: fill gsw_level_trace.e_frontier: the lanes that discover
                                a vertex add its out-degree to per-level counters (16
                                more bytes read per discovered vertex) */
  int32_t no_solo;           /* 1: never run levels in single-workgroup launches.  0 (the
                                default): while the frontier is small (at most 512
                                vertices, with bounded arcs) and the policy names a
                                queue-driven top-down kernel (push_vertex, push_wave,
                                push_edge), one workgroup of 1024 threads runs such levels
                                one after another in a single launch, deciding each next
                                kernel itself, instead of one launch of the whole grid per
                                level; results are the same.  Off with time_levels = 2. */
  void *stream;              /* hipStream_t for the work; NULL = library stream */
} gsw_bfs_opts;

/* Fills opts with: tree policy, no tree, host pointers, library stream. */
void gsw_bfs_opts_default(gsw_bfs_opts *opts);

/* ---------------------------------------------------------------- graphs */

/* Host-only check of a CSR graph: 1 <= n < 2^31, nnz >= 0, offs[0] == 0,
 * offs non-decreasing, offs[n] == nnz, every column in [0, n).  When
 * is_symmetric is non-NULL it receives 1 if every arc has its reverse, else 0
 * (cost O(nnz log deg)).  Needs no GPU. */
gsw_status gsw_graph_validate(int64_t n, int64_t nnz, const int64_t *offs, const int32_t *cols,
                              int32_t *is_symmetric);

/* Copies a host CSR into device memory owned by the graph.  flags: GSW_*
 * creation flags.  Degree statistics are computed here (host, untimed). */
gsw_status gsw_graph_create_host(int64_t n, int64_t nnz, const int64_t *offs, const int32_t *cols,
                                 uint32_t flags, gsw_graph **out);

/* Borrows a device CSR (e.g. torch tensors); the caller keeps d_offs/d_cols
 * alive and unchanged until gsw_graph_destroy.  Validation and statistics
 * copy the arrays to the host once (skipped checks with GSW_TRUSTED). */
gsw_status gsw_graph_create_device(int64_t n, int64_t nnz, const int64_t *d_offs,
                                   const int32_t *d_cols, uint32_t flags, void *stream,
                                   gsw_graph **out);

void gsw_graph_destroy(gsw_graph *g);

/* n, nnz, out-degree deg_stats = {min, q1, median, q3, max, std}, device
 * bytes held by the graph (CSR, transpose of a directed graph, origin
 * arrays, BFS workspace).  Any output may be NULL. */
gsw_status gsw_graph_info(const gsw_graph *g, int64_t *n, int64_t *nnz, double deg_stats[6],
                          size_t *dev_bytes);

/* 1 when every arc has its reverse (checked, or vouched for with
 * GSW_ASSUME_SYMMETRIC), else 0. */
int32_t gsw_graph_symmetric(const gsw_graph *g);

/* Device bytes of the single-source BFS workspace of g (allocated by the
 * first gsw_bfs or gsw_bfs_profile call and held until gsw_graph_destroy),
 * whether allocated yet or not: what a server must budget before it runs
 * single-source queries on g. */
size_t gsw_graph_workspace_bytes(const gsw_graph *g);

/* Out-degree statistics of a host CSR, as used in the feature vector:
 * {min, q1, median, q3, max, std}.  Host only; needs no GPU. */
gsw_status gsw_degree_stats(int64_t n, const int64_t *offs, double out[6]);

/* The 20 graph features (see GSW_N_FEATURES: n, arcs, out-, in- and
 * absolute-degree statistics) of a host CSR.  Host only; needs no GPU. */
gsw_status gsw_graph_features_host(int64_t n, int64_t nnz, const int64_t *offs, const int32_t *cols,
                                   double out[GSW_N_GRAPH_FEATURES]);

/* The tree's feature vector (see GSW_N_FEATURES) for a level whose frontier
 * has n_frontier vertices after `discovered` vertices have depths 0..d. */
gsw_status gsw_level_features(const gsw_graph *g, int64_t n_frontier, int64_t discovered,
                              double out[GSW_N_FEATURES]);

/* ----------------------------------------------------------------- trees */

/* Builds a tree from flat node arrays (a fitted CART tree): node 0 is the
 * root; left[i] == -1 marks a leaf; an inner node sends x to left[i] when
 * (double)(float)x[feature[i]] <= threshold[i], else to right[i] (features
 * are compared in float32, as scikit-learn does).  value[i*n_classes + c] is
 * the weight of class c in node i's bucket; class_kernel[c] is the GSW_K_*
 * of class c.  A leaf whose largest weight is shared by two or more classes
 * is undecided (Section IV-A, "unknown prediction"). */
gsw_status gsw_tree_create(int32_t n_nodes, int32_t n_classes, const int32_t *feature,
                           const double *threshold, const int32_t *left, const int32_t *right,
                           const double *value, const int32_t *class_kernel, gsw_tree **out);
void gsw_tree_destroy(gsw_tree *t);

/* Reads a tree from the JSON export of a fitted CART tree: an object with
 * the arrays "feature", "threshold", "left", "right" (one entry per node;
 * -1 children at leaves), "value" (per node, the class weights) and
 * "class_kernel" (the kernel id of each class), as gsw_tree_create takes
 * them.  When the object has "feature_names" it must list this library's
 * GSW_N_FEATURES feature names in order (guards against a tree trained on
 * another feature layout).  Other keys are ignored.  GSW_EINVAL on a
 * malformed file. */
gsw_status gsw_tree_load(const char *json_path, gsw_tree **out);

/* Name of feature i (as in the JSON export), "?" out of range. */
const char *gsw_feature_name(int32_t i);

/* Host-side prediction for one feature vector.  An undecided leaf repeats
 * prev_kernel when level > 0 and gives GSW_DEFAULT_KERNEL at level 0
 * (Section IV-A); *unknown is set to 1 in that case.  Needs no GPU. */
gsw_status gsw_tree_predict(const gsw_tree *t, const double x[GSW_N_FEATURES], int32_t prev_kernel,
                            int32_t level, int32_t *kernel, int32_t *unknown);

/* ------------------------------------------------------------------- BFS */

/*
 * Level-synchronous BFS from each of n_sources sources (Section III-A: all
 * depths start at infinity, the root at 0; every level gives depth d+1 to the
 * unvisited neighbours of depth-d vertices; the search ends when a level
 * finds nothing).
 *   sources  host array of n_sources vertex ids in [0, n).
 *   levels   [n_sources][n] int32: hop distance from the source, -1 if
 *            unreachable.  Device memory when opts->device_ptrs, else host.
 *   parents  [n_sources][n] int32 or NULL: a neighbour one level up
 *            (parent[source] = source, -1 if unreachable).  Not unique
 *            unless opts->canonical_parents.
 *   trace    host array of trace_cap rows or NULL; *trace_len (may be NULL)
 *            receives the number of rows produced, which can exceed
 *            trace_cap (extra rows are dropped).
 * The policy is applied on the device: at the end of each level the last
 * workgroup computes the features of the next level, picks its kernel and
 * posts a record (the trace row) to mapped host memory, so the host queues
 * levels ahead (a push_edge level takes two launches of the level kernel:
 * its prefix sum, then its expansion).  The policy, the
 * unknown rule and the float32 feature comparison are those of
 * gsw_tree_predict.
 */
gsw_status gsw_bfs(const gsw_graph *g, const int32_t *sources, int32_t n_sources, int32_t *levels,
                   int32_t *parents, gsw_level_trace *trace, int32_t trace_cap,
                   int32_t *trace_len, const gsw_bfs_opts *opts);

/*
 * Per-level timing of every listed kernel from the same BFS state (the
 * training data of Section IV-A).  At each level the state is saved, each
 * kernel in kernels[0..n_kernels) runs `reps` times from the saved state and
 * times[level*n_kernels + k] receives the median level time in ms (the
 * level's launches as gsw_bfs queues them: two for push_edge); then the
 * BFS advances one level with advance_kernel (or, when advance_kernel < 0,
 * with the fastest kernel just measured).  frontier[level] receives
 * n_f(level).  Stops at max_levels rows (GSW_ERANGE if the BFS is longer).
 * Kernels that cannot run (none since directed graphs keep their transpose)
 * would get a time of -1.
 */
gsw_status gsw_bfs_profile(const gsw_graph *g, int32_t source, const int32_t *kernels,
                           int32_t n_kernels, int32_t reps, int32_t advance_kernel, float *times,
                           int64_t *frontier, int32_t max_levels, int32_t *n_levels, void *stream);

/*
 * gsw_bfs for callers that cannot allocate memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * kernels and results as gsw_bfs; it calls no hipMalloc, hipFree,
 * hipHostMalloc or other allocating routine and creates no events.  Its
 * kernels' working memory (bitmaps, frontier queues, counters, level
 * control, push_edge scan arrays, the head copy of the in-arcs, the level
 * records, the device copy of the tree or schedule) is one fixed device
 * array of GSW_NOALLOC_SCRATCH_BYTES per GPU, held from the library's first
 * use of that GPU until the process ends.  Limits (GSW_EINVAL beyond them,
 * checked before any GPU work): n <= GSW_NOALLOC_MAX_VERTICES, a tree of at
 * most GSW_NOALLOC_MAX_TREE_NODES nodes, a schedule of at most
 * GSW_NOALLOC_MAX_SCHEDULE entries; opts is required and must have
 * device_ptrs = 1 (levels and parents in device memory; sources stay a host
 * array) and time_levels 0 or 1; a fixed kernel or a schedule naming
 * edge_scan or rev_edge_scan needs the graph's origin arrays to exist
 * already (GSW_WITH_ORIGIN at creation), and a tree leaf naming one runs the
 * default kernel instead when they do not.  Every call shares its GPU's
 * array, which keeps the last call's contents; the call rebuilds or clears
 * what it reads before reading it.  Calls from threads of one process are
 * serialised by a lock and each returns after its work on the stream has
 * finished; work that overlaps a call on the same GPU through any other
 * route into this array (another thread bypassing the library, a captured
 * replay still running) races with it.  The level records are read by
 * copying them from device memory after every eight launches, so a
 * search costs one host wait per eight launches.
 */
#define GSW_NOALLOC_MAX_VERTICES (1 << 19)
#define GSW_NOALLOC_MAX_TREE_NODES 4095
#define GSW_NOALLOC_MAX_SCHEDULE 4096
#define GSW_NOALLOC_SCRATCH_BYTES 50774528 /* 48.4 MiB */
gsw_status gsw_bfs_noalloc(const gsw_graph *g, const int32_t *sources, int32_t n_sources,
                           int32_t *levels, int32_t *parents, gsw_level_trace *trace,
                           int32_t trace_cap, int32_t *trace_len, const gsw_bfs_opts *opts);

/* ----------------------------------------------------------- batched BFS */

#define GSW_MSBFS_MAX_SOURCES 1024
#define GSW_MSBFS_LEVEL_CAP 127 /* int8 levels */

typedef struct {
  float push_to_pull;  /* per source: switch it to bottom-up when its frontier's arcs exceed
                          this fraction of the arcs it has not reached yet ... */
  float pull_to_push;  /* ... and back to top-down when they fall below this fraction of all arcs */
  int32_t device_ptrs; /* 1: levels (and wide_levels) are device memory; 0: host */
  int32_t graph;       /* 1: replay a captured two-level HIP graph; 0: launch each kernel */
  int32_t block_size;  /* threads per workgroup of the level kernels: 128, 256 or 512
                          (0 = 256); an autotuned knob, results do not depend on it */
  int32_t fallback;    /* 1: sources still running after depth GSW_MSBFS_LEVEL_CAP are
                          rerun one by one on the int32 single-source path (below);
                          0: such a batch returns GSW_ERANGE */
  int32_t *wide_levels;  /* fallback: [wide_cap][n] int32, receives the full hop distances
                            of the rerun sources, in increasing source index */
  int32_t *wide_index;   /* fallback: host int32[wide_cap], receives their source indices */
  int32_t wide_cap;      /* fallback: rows wide_levels has room for */
  int32_t *n_wide;       /* fallback, may be NULL: receives the number of rerun sources
                            (GSW_ERANGE when it is above wide_cap) */
  const gsw_tree *tree;  /* fallback: policy of the rerun (NULL: the default kernel at
                            every level) */
  void *stream;        /* hipStream_t; NULL = library stream */
} gsw_msbfs_opts;

/* Fills opts: push_to_pull 0.07, pull_to_push 0.01, graph 1, block size 256, no
 * fallback, host pointers. */
void gsw_msbfs_opts_default(gsw_msbfs_opts *opts);

/*
 * Multi-source BFS of up to GSW_MSBFS_MAX_SOURCES sources in one traversal
 * (not in the paper; a batching of its level-synchronous BFS).  Every vertex
 * carries one bit per source; in each level every source either pushes its
 * frontier bits along the arcs or has them pulled into its unvisited
 * vertices, chosen per source by the thresholds above (bottom-up needs a
 * symmetric graph; otherwise every level is top-down), so one pass over the
 * edges serves the whole batch.
 *   levels    [n_sources][n] int8: hop distance from sources[i], -1 if
 *             unreachable.  Sources may repeat.
 *   n_levels  receives the number of levels run (may be NULL).
 * A source still running after discovering depth GSW_MSBFS_LEVEL_CAP has
 * depths int8 cannot hold.  Without opts->fallback the call then returns
 * GSW_ERANGE (levels unspecified).  With it, the batch stops at the cap and
 * every such source is rerun on the single-source path (gsw_bfs with
 * opts->tree, or the default kernel): its full int32 distances go to the
 * next row of opts->wide_levels and its index to opts->wide_index, and its
 * int8 row holds the distance where it is at most GSW_MSBFS_LEVEL_CAP and
 * INT8_MIN (-128) where it is larger (-1 still means unreachable).  Levels
 * are never truncated silently.
 */
gsw_status gsw_msbfs(const gsw_graph *g, const int32_t *sources, int32_t n_sources, int8_t *levels,
                     int32_t *n_levels, const gsw_msbfs_opts *opts);

/* -------------------------------------------------- connected components */

/*
 * Weakly connected components: a second traversal on the same switching
 * framework (the paper expects its per-iteration choice of interchangeable
 * kernels to carry over to other traversal algorithms, Section VI).  Every
 * arc joins its two ends whatever its direction.
 *   Phase 1 (symmetric graphs with arcs, opts->bfs_first): the component of
 *   a vertex of largest out-degree (the smallest id among ties) is found by
 *   the level-switched BFS of gsw_bfs, with opts->tree choosing each level's
 *   kernel.
 *   Phase 2: minimum-label propagation over the other vertices with arcs,
 *   each starting from its own id, until an iteration changes no label.
 *   Each iteration runs one of two kernels: PUSH (one lane per vertex whose
 *   label fell in the previous iteration lowers its neighbours' labels with
 *   atomicMin) or PULL (one lane per vertex left to phase 2 takes the
 *   smallest label among its neighbours), chosen per iteration by
 *   opts->policy.
 * On a directed graph a vertex's neighbours are its out- and in-neighbours
 * (over the transpose the library keeps) and phase 1 is skipped.
 *   labels        [n] int32: the smallest vertex id of v's component
 *                 (device memory when opts->device_ptrs, else host).
 *   n_components  receives the number of components (isolated vertices
 *                 count one each); may be NULL.
 *   trace         host array of trace_cap rows or NULL; *trace_len (may be
 *                 NULL) receives the rows produced (phase 1 as row 0 when it
 *                 runs), which can exceed trace_cap.
 * The graph's working memory for this call (4 int32 arrays of n and a bitmap)
 * is allocated on first use and held until gsw_graph_destroy.
 */
enum { GSW_CC_SWITCH = 0, GSW_CC_PUSH = 1, GSW_CC_PULL = 2 };   /* gsw_cc_opts.policy */
enum { GSW_CC_K_BFS = 0, GSW_CC_K_PUSH = 1, GSW_CC_K_PULL = 2 }; /* gsw_cc_trace.kernel */

typedef struct {
  int32_t iteration; /* from 0; phase 1, when it runs, is iteration 0 */
  int32_t kernel;    /* GSW_CC_K_* */
  int64_t n_active;  /* vertices whose label fell in the previous iteration (all the
                        vertices left to phase 2 at its first iteration; phase 1: 1, its seed) */
  int64_t e_active;  /* their arcs (out + in on a directed graph); -1 on the phase-1 row */
  int64_t changed;   /* vertices whose label this iteration lowered (phase 1: vertices reached) */
  float ms;          /* HIP events around the iteration's launches (phase 1: the BFS and
                        the labelling of its component) */
  int32_t pad;
} gsw_cc_trace;

typedef struct {
  int32_t policy;        /* GSW_CC_SWITCH: pull when the active vertices' arcs exceed
                            pull_above x the arcs of all vertices left to phase 2, else push;
                            GSW_CC_PUSH / GSW_CC_PULL: that kernel at every iteration */
  int32_t bfs_first;     /* 1: phase 1 on symmetric graphs; 0: propagation only */
  const gsw_tree *tree;  /* policy of the phase-1 BFS (NULL: the default kernel at every level) */
  float pull_above;      /* GSW_CC_SWITCH threshold, >= 0 */
  int32_t device_ptrs;   /* 1: labels is device memory; 0: host */
  void *stream;          /* hipStream_t; NULL = library stream */
} gsw_cc_opts;

/* Fills opts: switch policy, pull_above 0.05, phase 1 on, no tree, host labels,
 * library stream. */
void gsw_cc_opts_default(gsw_cc_opts *opts);

gsw_status gsw_cc(const gsw_graph *g, int32_t *labels, int64_t *n_components, gsw_cc_trace *trace,
                  int32_t trace_cap, int32_t *trace_len, const gsw_cc_opts *opts);

/* -------------------------------------------------------- serving sessions */

/*
 * A session runs many single-source BFS queries on one graph as one
 * continuously batched multi-source traversal: each query owns one of up to
 * GSW_MSBFS_MAX_SOURCES slots (one bit per vertex mask).  A query admitted
 * while others are in flight joins at the next level boundary with its own
 * start level, so queries of different ages share every pass over the edges;
 * a slot finishes when its frontier is empty and is reused after its result
 * has been fetched.  Each slot picks its own direction every level (the rule
 * of gsw_msbfs_opts), so a young query pushes while older ones pull in the
 * same pass.  Results are int32 hop distances (-1 unreachable), equal to a
 * single-source BFS from the same source.  Device memory: 4 masks of
 * n * ceil(slots/64) words plus slots * n int32 levels.  admit, info and
 * set_thresholds may be called from any thread while another thread is in
 * step or fetch (step and fetch are serialised with each other); sessions of
 * different graphs or of the same graph run concurrently on their own
 * streams.
 */
typedef struct gsw_session gsw_session;

/* Device memory a session of max_slots slots on g allocates (what a server
 * must budget for it). */
size_t gsw_session_bytes(const gsw_graph *g, int32_t max_slots);

gsw_status gsw_session_create(const gsw_graph *g, int32_t max_slots, gsw_session **out);
void gsw_session_destroy(gsw_session *ss);

/* Takes a free slot for a query from `source`; GSW_EBUSY when none is free. */
gsw_status gsw_session_admit(gsw_session *ss, int32_t source, int32_t *slot);

/* Runs levels until a slot finishes, max_levels levels have run, or no slot
 * is admitted or running.  Queries admitted before or during the call join
 * at the next level boundary.  finished[0..*n_finished) receives the
 * finished slots (finished_cap should be at least the slot count);
 * *levels_run the number of levels run (0: nothing to run). */
gsw_status gsw_session_step(gsw_session *ss, int32_t max_levels, int32_t *finished,
                            int32_t finished_cap, int32_t *n_finished, int32_t *levels_run);

/* Copies a finished slot's n levels (device or host memory) and frees it. */
gsw_status gsw_session_fetch(gsw_session *ss, int32_t slot, int32_t *levels, int32_t device_ptr);

/* Cancels the query in `slot` (for deadlines and client disconnects): one
 * admitted but not started yet is dropped at once; a running one becomes
 * inert at the next level boundary (it discovers nothing more) and, once
 * its frontier is empty, gsw_session_step clears its partial levels on the
 * device and frees the slot without reporting it.  Other queries are not
 * affected.  GSW_EINVAL when the slot holds no admitted or running query
 * (a finished one must be fetched). */
gsw_status gsw_session_cancel(gsw_session *ss, int32_t slot);

/* Slot count, slots in use, levels run so far, device bytes held. */
gsw_status gsw_session_info(const gsw_session *ss, int32_t *slots, int32_t *busy,
                            int64_t *iteration, size_t *dev_bytes);

/* Sets the session's level counter (the iteration that gsw_session_info
 * reports and new queries record as their start) to `iteration`, in
 * [0, 2^62].  Only while no query is running (GSW_EBUSY otherwise); a level
 * still queued then has nothing to advance and is waited for and dropped.
 * Admitted queries that have not started yet and finished ones that have not
 * been fetched keep their results.  The counter
 * is 64-bit and never wraps in practice; this call lets a long-lived server
 * restart the numbering and lets tests start a session at any count. */
gsw_status gsw_session_rebase(gsw_session *ss, int64_t iteration);

/* Direction thresholds as in gsw_msbfs_opts (defaults 0.07 / 0.01). */
gsw_status gsw_session_set_thresholds(gsw_session *ss, float push_to_pull, float pull_to_push);

/* ------------------------------------------------------------------ misc */

const char *gsw_last_error(void);
const char *gsw_kernel_name(int32_t kernel_id); /* base name, then ".wave" or ".thread" for
                                                   those count variants; "?" for an unknown id */
int32_t gsw_abi_version(void);
/* Build stamp: a digest of the sources the library was compiled from (the
 * Python binding refuses a library whose stamp differs from the sources
 * beside it), or "unstamped". */
const char *gsw_source_digest(void);

#ifdef __cplusplus
}
#endif

#endif /* GSW_H */
