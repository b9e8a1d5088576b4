/*
 * slimsell.h -- C ABI of the MI355X SlimSell BFS library (libslimsell.so).
 *
 * SlimSell BFS (Besta et al., "SlimSell: A Vectorizable Graph Representation
 * for Breadth-First Search", arXiv 2010.09913) computes breadth-first search
 * as one sparse-matrix dense-vector product per level over a Sell-C-sigma
 * layout that keeps only column indices (Section III-B, "Reducing Storage
 * Complexity with SlimSell"), under one of four semirings (Section III-A),
 * optionally skipping finished chunks (SlimWork, Section III-C) and splitting
 * long chunks into dynamically scheduled pieces (SlimChunk, Section III-D).
 *
 * Conventions shared by every entry point
 *   - Return value: 0 (SS_OK) on success, a negative ss_status on failure.
 *     slimsell_last_error() returns a thread-local message for the last
 *     failure on the calling thread.
 *   - Vertex IDs are 0-based int32 in the caller's (original) numbering.
 *   - Pointers documented "host" are ordinary CPU memory; "device" pointers are
 *     HIP device memory (e.g. torch CUDA tensors on ROCm).  The library never
 *     frees memory it did not allocate.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     BFS calls enqueue work on it; argument errors are reported
 *     synchronously, HIP errors at the call that observes them or at
 *     slimsell_sync().
 *   - A graph object is not safe for concurrent use: calls that use one graph
 *     must not overlap (they share its device workspace).
 */
#ifndef SLIMSELL_H
#define SLIMSELL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SS_OK = 0,
  SS_EINVAL = -1, /* bad argument (range, null pointer, unsupported combination) */
  SS_ENOMEM = -2, /* host or device allocation failed */
  SS_EHIP = -3,   /* a HIP runtime call or a kernel failed */
  SS_EUNSUP = -4, /* feature not available (e.g. no device) */
  SS_EITER = -5   /* the level cap was reached before the BFS finished */
} ss_status;

/* The four semirings of Section III-A. */
typedef enum {
  SS_TROPICAL = 0, /* (min, +): frontier = distances, int32 */
  SS_REAL = 1,     /* (+, *): fp32 frontier, binarised by the filter g */
  SS_BOOLEAN = 2,  /* (|, &): uint8 frontier */
  SS_SELMAX = 3    /* (max, *): int32 vertex values; yields parents directly */
} ss_semiring;

/* Chunk height.  One chunk is one 64-lane wavefront of rows. */
#define SS_CHUNK_HEIGHT 64

/* ------------------------------------------------------------------ layout */

/*
 * Host-side SlimSell layout (Section III-B; Sell-C-sigma in Section II-D):
 *   rows are the vertices, sorted by decreasing degree inside windows of sigma
 *   consecutive original IDs (stable on the ID), then relabelled to their
 *   sorted position; chunk i holds rows [64 i, 64 i + 64).
 *   col[cs[i] + 64 j + lane] is the relabelled ID of the j-th neighbour of row
 *   64 i + lane, or -1 where the row is shorter than the chunk (padding); a
 *   row lists its neighbours by decreasing original ID, so a product that
 *   keeps the largest ID (sel-max, and the DP transformation) may stop at the
 *   first qualifying neighbour.
 *   The number of vertices is padded to a multiple of 64 with phantom rows
 *   (degree 0, never reachable).
 */
typedef struct ss_layout ss_layout;

typedef struct {
  int32_t n;            /* vertices */
  int32_t n_pad;        /* n rounded up to a multiple of 64 */
  int32_t C;            /* chunk height, always 64 */
  int32_t sigma;        /* sorting scope used */
  int64_t n_chunks;     /* n_pad / 64 */
  int64_t entries;      /* directed edge cells E (non-marker cells) = 2 x undirected edges */
  int64_t cells;        /* length of col = E + padding P */
  int32_t max_cl;       /* longest chunk, in columns (= max degree) */
  int32_t pad0;
  const int32_t* col;   /* [cells]   column-major per chunk, -1 = padding */
  const int64_t* cs;    /* [n_chunks + 1] offset of chunk i in col; cs[n_chunks] = cells */
  const int32_t* cl;    /* [n_chunks] columns of chunk i */
  const int32_t* v;     /* [n_pad]   original ID + 1 of each row, 0 for phantom rows */
  const int32_t* perm;  /* [n]       row of each original vertex */
  const int32_t* degree;/* [n_pad]   degree of each row */
} ss_layout_view;

/*
 * Build the SlimSell layout on the host from an undirected tuple list.
 *   src, dst : host int32[m], IDs in [0, n).  Self-loops are dropped, both
 *              directions of every tuple are kept once (duplicates dropped).
 *   C        : must be 64.
 *   sigma    : sorting scope; a multiple of 64 in [64, n_pad], or 1 (no sort),
 *              or 0 meaning n_pad (sort all rows).
 * On success *out owns host memory until slimsell_layout_free().
 * Errors: SS_EINVAL (n < 1, m < 0, null pointer, ID out of range, bad C or
 * sigma), SS_ENOMEM.
 */
int slimsell_layout_build(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                          int32_t C, int32_t sigma, ss_layout** out);

/* Fill *view with pointers into the layout (valid until it is freed). */
int slimsell_layout_view(const ss_layout* layout, ss_layout_view* view);

void slimsell_layout_free(ss_layout* layout);

/* ------------------------------------------------------------------- graph */

/* Device-resident SlimSell graph plus its BFS workspace (opaque). */
typedef struct ss_graph ss_graph;

/*
 * slimsell_layout_build followed by an upload to the current HIP device.
 * Same arguments and errors, plus SS_EHIP / SS_EUNSUP when no device is usable.
 */
int slimsell_build(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t C,
                   int32_t sigma, void* stream, ss_graph** out);

/*
 * Several graphs as one device graph: the disjoint union of their SlimSell
 * layouts, each graph's rows padded to whole chunks, so no chunk mixes graphs.
 * Vertex v of graph i has the union ID voff_i + v with voff_i = n_0 + ... +
 * n_{i-1}.  Single-root BFS (slimsell_bfs) treats the union as one graph;
 * slimsell_bfs_batch runs up to 64 roots in every graph at once.
 *   num_graphs     : >= 1.
 *   edge_offsets   : host int64[num_graphs + 1]; graph i's tuples are
 *                    src/dst[edge_offsets[i] .. edge_offsets[i+1]).
 *   src, dst       : host int32, graph-local IDs in [0, n_i).
 *   n_per_graph    : host int32[num_graphs], each >= 1.
 *   C, sigma       : as slimsell_layout_build, applied to every graph
 *                    (sigma 0 = sort all rows of that graph).
 * A union of two or more graphs starts with the launch configuration
 * {split_len 128, waves_per_group 8, unroll 8, max_groups 0, pack_cols 0,
 * lds_kib 0} (one wavefront per work unit, balanced by the dispatcher),
 * not the single-graph default; slimsell_tune_set or slimsell_autotune
 * replace it.
 * Errors: as slimsell_build; the union must have fewer than 2^31 rows.
 */
int slimsell_build_multi(int32_t num_graphs, const int64_t* edge_offsets, const int32_t* src,
                         const int32_t* dst, const int32_t* n_per_graph, int32_t C,
                         int32_t sigma, void* stream, ss_graph** out);

/* Number of graphs in a (possibly multi-graph) device graph and, if not NULL,
 * each graph's vertex count and union-ID offset (host int64[num_graphs]). */
int slimsell_graph_parts(const ss_graph* g, int32_t* num_graphs, int64_t* n_per_graph,
                         int64_t* vertex_offset);

/* Upload an existing host layout to the current device. */
int slimsell_build_from_layout(const ss_layout* layout, void* stream, ss_graph** out);

/* Size figures of a built graph (host outputs, any may be NULL). */
int slimsell_graph_info(const ss_graph* g, int64_t* n, int64_t* entries, int64_t* padding,
                        int64_t* chunks, int64_t* max_cl);

/*
 * Degree of every vertex in the canonical graph (self-loops and duplicates
 * dropped), in original IDs: host int32[n].
 */
int slimsell_graph_degrees(const ss_graph* g, int32_t* degree);

/*
 * Launch configuration of the level kernel for one graph (Section III-D's
 * SlimChunk split plus the MI355X launch shape).  BFS calls use it where
 * ss_bfs_opts leaves a field to the graph (split_len = -1, waves_per_group = 0).
 *   split_len       : SlimChunk piece length in columns; 0 = never split.
 *   waves_per_group : wavefronts per workgroup: 1, 2, 4, 8 or 16.
 *   unroll          : columns per gather block: 4, 8 or 16.
 *   max_groups      : cap on workgroups per level launch; 0 = one wavefront
 *                     per work unit (hardware dispatch does the balancing),
 *                     else units are strided over the capped grid.
 *   pack_cols       : chunks shorter than split_len are packed into runs of
 *                     at most this many columns per work unit; 0 = one chunk
 *                     per unit; -1 = split_len.
 *   lds_kib         : KiB of the gathered vector's prefix (the highest-degree
 *                     rows under a full sort) that each workgroup stages in
 *                     LDS once per level: 0, 16, 32 or 64.  Pays off with a
 *                     capped grid (max_groups), where each workgroup serves
 *                     many work units.
 */
typedef struct {
  int32_t split_len;
  int32_t waves_per_group;
  int32_t unroll;
  int32_t max_groups;
  int32_t pack_cols;
  int32_t lds_kib;
} ss_tune;

/* Set / read the graph's launch configuration.  SS_EINVAL on a bad field. */
int slimsell_tune_set(ss_graph* g, const ss_tune* tune);
int slimsell_tune_get(const ss_graph* g, ss_tune* tune);

/*
 * Autotuner: measures the level kernel's launch configuration on this graph
 * and stores the fastest in it (slimsell_tune_set).  Coordinate descent over
 * split_len {0, 64, ..., 4096}, waves_per_group {1, ..., 16}, unroll
 * {4, 8, 16}, max_groups {0, 1024, 4096}, pack_cols {0, 32, 128} and
 * lds_kib {0, 32, 64}, two passes; each configuration is timed (events, init to finalise) over the
 * given roots, median of `repeats`.  Results are cached per graph class
 * (semiring, batched, log2 n, mean degree, degree skew) for the process.
 * Results of BFS calls do not depend on the configuration.
 *   semiring   : the semiring to tune for (ignored when batched = 1).
 *   batched    : 1 = tune for slimsell_bfs_batch (64-root boolean SpMM).
 *   roots      : host int32[num_roots], roots to time (num_roots >= 1).
 *   repeats    : timed repetitions per configuration (0 = 3).
 *   force      : 1 = ignore the class cache.
 * On return *result holds the chosen configuration and its time, the time of
 * the configuration in force before the call, and the evaluation count.
 */
typedef struct {
  uint32_t size;
  int32_t semiring;
  int32_t batched;
  int32_t num_roots;
  const int32_t* roots;
  int32_t repeats;
  int32_t force;
  void* stream;
} ss_autotune_opts;

typedef struct {
  ss_tune best;
  float best_ms;        /* summed BFS time over the roots, chosen configuration */
  float before_ms;      /* same, configuration in force before the call */
  int32_t evaluated;    /* configurations timed (0 when served from the cache) */
  int32_t from_cache;
} ss_autotune_result;

int slimsell_autotune(ss_graph* g, const ss_autotune_opts* opts, ss_autotune_result* result);

/* Release a graph and its device memory. */
void slimsell_free(ss_graph* g);

/* ---------------------------------------------------------------------- BFS */

/* Per-level record (see ss_bfs_opts.flags). */
typedef struct {
  int64_t discovered;     /* vertices that entered the frontier at this level */
  int64_t frontier_edges; /* sum of their degrees */
  int64_t active_chunks;  /* chunks processed by a pull level (not skipped by SlimWork) */
  int64_t active_cells;   /* col cells read: 64 x columns swept (pull) or cells of the
                             frontier rows (push) */
  int64_t max_active_cl;  /* longest processed chunk, in columns */
  float ms;               /* kernel time of the level (events), 0 if not timed */
  int32_t variant;        /* variant run by a scheduled level, -1 otherwise */
} ss_level_stats;

/* Per-root record (see ss_bfs_opts.flags). */
typedef struct {
  int32_t iterations;    /* SpMV iterations = eccentricity + 1 */
  int32_t launches;      /* level kernels launched, incl. look-ahead ones that exit at once */
  float kernel_ms;       /* summed time of all those level kernels (SS_STATS_TIME) */
  float bfs_ms;          /* init kernel start to finalise end on the stream (SS_STATS_TIME) */
  /* the DP transformation's sweep kernel, when parents are asked of a
   * semiring other than sel-max (0 otherwise): its time (SS_STATS_TIME or
   * SS_STATS_TIME_BFS) and the chunks and col cells it swept
   * (SS_STATS_COUNTERS with level_stats_out) */
  float dp_ms;
  int32_t pad0;
  int64_t dp_chunks;
  int64_t dp_cells;
} ss_run_stats;

#define SS_STATS_TIME 1     /* hipEvents around every level kernel and every BFS */
#define SS_STATS_COUNTERS 2 /* fused per-level counters (a few atomics per wavefront) */
/* hipEvents around every BFS only (bfs_ms; kernel_ms and per-level ms stay 0):
 * no per-level host work, for runs with thousands of levels */
#define SS_STATS_TIME_BFS 16
/* Run all levels of a BFS in one cooperative (persistent) kernel launch with a
 * device-wide barrier between levels, instead of one launch per level: one
 * 1024-thread workgroup per compute unit (capped by the graph's max_groups).
 * With a schedule, every workgroup computes each level's variant from the
 * same counters and the push phases (scatter, long-row segments, post) are
 * separated by device-wide barriers too; results and per-level variants are
 * those of the launch-per-level form.  Per-level times are not available in
 * this mode; a barrier that waits more than 5 s is reported as SS_EHIP. */
#define SS_RUN_PERSISTENT 4
/* Comparator: run the levels on Sell-C-sigma instead of SlimSell (Section
 * II-D, Table "sizes"): a val array (1 = edge, 0 = padding) is streamed beside
 * a col array whose padding cells hold a valid row, so each cell costs 8 bytes
 * instead of 4.  Built on the device at first use (2 x 4 B per cell).  Same
 * results; single-root levels only (no schedule, no persistent launch). */
#define SS_SELL_VAL 8
/* Plain single-root runs record, per level, one bit per chunk that gained
 * frontier rows (a frontier summary, 2 KiB per million vertices, kept where it
 * is at most 32 KiB).  While few chunks hold frontier rows (how few depends
 * on the share of gathers the LDS prefix serves), the next level stages it in
 * LDS and reads a term of the product from memory only when its row's chunk
 * holds frontier rows; every other term is the semiring's
 * identity for each row whose value can still change, so results are
 * unchanged.  A level records its summary only if it used one itself.  The
 * batched SpMM keeps one too (a chunk is flagged when a row gained root
 * bits).  This flag turns the summary off (every term outside the staged
 * prefix is read).  Runs with a schedule never use it. */
#define SS_NO_SUMMARY 32
/* Learned schedule: every workgroup of a level stages the model only once
 * the level's features lie within tau of an anchor of the model's training
 * domain, one memory round trip later, instead of while it reads the
 * counters.  Without this flag a graph's learned runs choose by themselves:
 * up front on the first run and after any run with a level inside the
 * domain, only inside the domain after a run with none.  The decisions are
 * the same either way; only their cost differs. */
#define SS_SCHED_LAZY 64

/*
 * Per-call options.  Zero-initialise, set size = sizeof(ss_bfs_opts).
 *   slimwork        : 0 = every row of every chunk is computed (plain SlimSell);
 *                     1 = skip chunks whose rows are all final (SlimWork,
 *                     Section III-C);
 *                     2 = SlimWork plus row-level masking: inside a processed
 *                     chunk a row that is final issues no loads, the column
 *                     sweep stops at the longest row still live, and under
 *                     tropical, boolean and sel-max a row stops at its first
 *                     frontier neighbour (its value is then final; sel-max
 *                     rows list neighbours by decreasing original ID).
 *                     Results are identical in all three modes.
 *   split_len       : SlimChunk piece length in columns (Section III-D):
 *                     0 = chunks are never split, >0 = split chunks longer than
 *                     this, -1 = the graph's tuned value (see slimsell_autotune),
 *                     falling back to the built-in default.
 *   waves_per_group : wavefronts per workgroup (1, 2, 4, 8 or 16; 0 = default).
 *   schedule        : per-level variant choice among {pull without split,
 *                     pull split 256, pull split 1024, push from the frontier}:
 *                     0 = none (every level pulls with the graph's configuration);
 *                     1 = learned (slimsell_sched_load), falling back to the fixed
 *                         heuristic when no model is loaded or its scores are
 *                         not finite;
 *                     2 = the fixed heuristic: pull (with the graph's split
 *                         length) once the frontier's edges exceed 1/14 of the
 *                         edges not yet discovered, push before (the direction
 *                         rule of Beamer et al., alpha = 14);
 *                     3..6 = force variant 0..3 on every level.
 *                     Scheduling needs slimwork = 2.
 *   max_levels      : cap on SpMV iterations (0 = n + 1).  Reaching it
 *                     returns SS_EITER.
 *   stream          : hipStream_t.
 *   iterations_out  : host int32[num_roots] or NULL: SpMV iterations per root
 *                     (eccentricity + 1; the last one discovers nothing).
 *   flags           : SS_STATS_TIME, SS_STATS_TIME_BFS, SS_STATS_COUNTERS,
 *                     SS_RUN_PERSISTENT, SS_SELL_VAL, SS_NO_SUMMARY,
 *                     SS_SCHED_LAZY.
 *   level_cap       : levels per root recorded in level_stats_out.
 *   level_stats_out : host ss_level_stats[num_roots * level_cap] or NULL;
 *                     entry [r * level_cap + k - 1] describes level k of root r.
 *                     Counter fields need SS_STATS_COUNTERS, ms needs
 *                     SS_STATS_TIME; unused entries are zeroed.
 *   run_stats_out   : host ss_run_stats[num_roots] or NULL.
 * Requesting any statistics makes the call wait for the stream at its end.
 */
typedef struct {
  uint32_t size;
  int32_t slimwork;
  int32_t split_len;
  int32_t waves_per_group;
  int32_t schedule;
  int32_t max_levels;
  void* stream;
  int32_t* iterations_out;
  int32_t flags;
  int32_t level_cap;
  ss_level_stats* level_stats_out;
  ss_run_stats* run_stats_out;
} ss_bfs_opts;

/*
 * BFS from each root in turn, one SpMV per level under semiring s.
 *   roots     : host int32[num_roots], each in [0, n).
 *   dist      : device int32[num_roots * n]; row r receives hop distances from
 *               roots[r] (-1 = unreachable).  Required.
 *   parent    : device int32[num_roots * n] or NULL: the largest-ID
 *               neighbour one level closer; parent[root] = root; -1 =
 *               unreachable.  SS_SELMAX yields it from the product itself;
 *               the other semirings run the DP transformation
 *               (slimsell_dp_parents) after each root's BFS, inside the
 *               timed region (Section II-C; "DP" vs "No-DP").
 *   real_val  : device float[num_roots * n] or NULL; SS_REAL only: the
 *               real-semiring value x_{d(v)}^v at discovery, i.e. the number
 *               of neighbours one level closer (root 1, unreachable 0).
 * Errors: SS_EINVAL (root out of range, real_val with a non-real semiring,
 * bad options), SS_EITER, SS_EHIP.
 */
int slimsell_bfs(ss_graph* g, const int32_t* roots, int32_t num_roots, ss_semiring s,
                 const ss_bfs_opts* opts, int32_t* dist, int32_t* parent, float* real_val);

/*
 * Allocation-free BFS, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the computation, arguments, outputs and errors of slimsell_bfs,
 * with the per-call workspace (frontier vectors, row states, distances,
 * SlimChunk combine buffers, level tags, frontier summaries) in one fixed
 * 64 MiB device array that the library holds on every GPU it runs on until
 * the process ends.  The call makes no hipMalloc, hipFree or other
 * allocating call; outputs are the caller's.
 *   Scratch needed: 8 KiB + 5 B per chunk + the frontier summaries (at most
 *   32 KiB) + per row: tropical 8 B, real 21 B, boolean 11 B, sel-max
 *   13.25 B, and for parents by the DP transformation 4.25 B more (tropical)
 *   or 4 B more (real, boolean); more than 64 MiB is SS_EINVAL (sel-max fits
 *   about 5 million rows).
 *   opts   : slimwork, split_len, waves_per_group, max_levels, stream and
 *            iterations_out as slimsell_bfs; flags 0 or SS_NO_SUMMARY;
 *            schedule 0; level_stats_out and run_stats_out NULL (anything
 *            else is SS_EINVAL).  split_len must name a configuration whose
 *            work units exist: the graph's own (split_len = -1; prepared by
 *            slimsell_build and slimsell_tune_set) or one an earlier
 *            slimsell_bfs call used; otherwise SS_EINVAL.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (a call initialises everything it reads): calls that overlap on
 * one GPU race, whatever their graphs or streams.  The graph's level-report
 * ring is used as in slimsell_bfs, so calls on one graph must not overlap.
 */
int slimsell_bfs_noalloc(ss_graph* g, const int32_t* roots, int32_t num_roots, ss_semiring s,
                         const ss_bfs_opts* opts, int32_t* dist, int32_t* parent,
                         float* real_val);

/*
 * DP transformation (Section II-C): parents from BFS distances.  For every
 * vertex v with dist[v] >= 1, parent[v] = the largest original ID u among
 * v's neighbours with dist[u] = dist[v] - 1 (-1 if there is none); a vertex
 * with dist 0 is its own parent; dist < 0 gives -1.  One sweep of the
 * SlimSell layout per root, by the level kernel with the reached rows live,
 * that gathers dist mod 3 as a 2-bit code (a neighbour is one level closer,
 * at the same level or one further, so the code decides); a row stops at its
 * first qualifying neighbour, the largest.  The input must be BFS distances
 * on this graph (other input gives unspecified parents, never an
 * out-of-bounds access).
 *   dist      : device int32[num_roots * n], original vertex order (as
 *               slimsell_bfs or slimsell_bfs_batch write it).
 *   parent    : device int32[num_roots * n], written.
 *   stream    : hipStream_t.  Uses the graph's workspace: calls on one graph
 *               must be ordered (one stream), as for slimsell_bfs.
 * Errors: SS_EINVAL (NULL graph/pointers, num_roots < 0), SS_EHIP.
 */
int slimsell_dp_parents(ss_graph* g, const int32_t* dist, int32_t num_roots, int32_t* parent,
                        void* stream);

/* ------------------------------------------------------- learned schedule */

/*
 * Scheduler model (not in the paper): an FP32 MLP 6 -> 32 -> 32 -> 4 with ReLU
 * that maps six features of the previous level's frontier to the predicted
 * log-time of each variant; the smallest wins.  Parameter layout (1412
 * floats): W1[32][6], b1[32], W2[32][32], b2[32], W3[4][32], b3[4].
 * Features, in order: log2(1+n_f)/log2 n; log2(1+m_f)/log2(1+2m);
 * log2(1+m_u)/log2(1+2m); clamp(log2((1+m_f)/(1+n_f))/16, 0, 1);
 * clamp(log2((1+m_u)/n)/8, +-1); clamp(log2((1+m_f)/(1+m_u))/16, +-1) --
 * n_f, m_f: vertices and edge ends of the frontier; m_u: edge ends of the
 * vertices not yet discovered; n vertices, m undirected edges.  They measure
 * the push work (m_f) and the pull work (m_u) on log scales relative to the
 * graph, so they carry across graph sizes.
 *
 * A model may also carry its training domain: count = 1412 + 2 + 6K floats,
 * the parameters, then tau > 0, K (1..1024, as a float) and K feature
 * vectors.  A level whose features lie farther than tau (Euclidean) from all
 * K vectors is decided by the fixed heuristic, as are levels with non-finite
 * scores.
 */
#define SS_SCHED_PARAMS 1412
#define SS_SCHED_FEATURES 6
#define SS_SCHED_VARIANTS 4

/* Install the process-wide model: host float[count], count = 1412 (the
 * parameters) or 1412 + 2 + 6K (parameters and training domain, see above);
 * copied.  Non-finite parameters are accepted, and the fixed heuristic then
 * takes over at run time.  Errors: SS_EINVAL for any other count, tau <= 0,
 * K outside 1..1024 or non-finite anchors. */
int slimsell_sched_load(const float* weights, int64_t count);
/* Remove the model (learned scheduling then uses the fixed heuristic). */
int slimsell_sched_clear(void);
/* Per-level record of the last scheduled run on g: host float[cap][12] =
 * 6 features, 4 scores, chosen variant, level.  The scores are 0 without a
 * model and for a level outside the model's training domain (farther than
 * tau from every anchor), which the model does not score.  *levels
 * receives the records written: the last scheduled run's level count (its
 * iterations, at most min(n + 2, 65536)), clamped to cap; 0 before any
 * scheduled run. */
int slimsell_sched_log(const ss_graph* g, float* out, int32_t cap, int32_t* levels);

/*
 * Model training on the GPU.  Loss: mean squared error over the N x 4
 * targets; optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8), full batch.
 *   x       : host float[N][6] features; y: host float[N][4] targets.
 *   init    : host float[1412] starting weights, or NULL for a seeded
 *             He-uniform start (seed).
 * slimsell_sched_grad evaluates the loss and its gradient once;
 * slimsell_sched_forward the scores.  Outputs are host arrays.
 */
int slimsell_sched_grad(const float* weights, const float* x, const float* y, int64_t n,
                        float* grad, float* loss, void* stream);
int slimsell_sched_forward(const float* weights, const float* x, int64_t n, float* scores,
                           void* stream);
int slimsell_sched_train(const float* x, const float* y, int64_t n, int32_t steps, float lr,
                         uint64_t seed, const float* init, float* weights_out, float* loss_out,
                         void* stream);

/*
 * Batched BFS as a boolean SpMM (not in the paper; multi-source BFS): every
 * row carries a 64-bit frontier mask, one bit per root, so one sweep of the
 * SlimSell layout advances up to 64 BFS at once: X = OR over the row's
 * neighbours of F, new = X & ~visited.  In a multi-graph, slot b runs root b
 * of every graph in the same sweep (the graphs are disjoint), so all graphs
 * are solved by one level loop.
 *   roots           : host int32[num_graphs * roots_per_graph]; entry
 *                     [i * roots_per_graph + b] is a graph-local root of graph
 *                     i, or -1 for an unused slot.
 *   roots_per_graph : 1..64.
 *   dist            : device int32; graph i's block starts at
 *                     roots_per_graph * voff_i and is laid out
 *                     [roots_per_graph][n_i] (hop distances, -1 unreachable
 *                     or unused slot).  For one graph this is [b][n].
 * opts as slimsell_bfs (slimwork, split via the graph's configuration,
 * statistics; iterations_out[0] receives the level count of the union).
 * Levels are capped at 65534.  Errors: SS_EINVAL (root out of range,
 * roots_per_graph out of range), SS_EITER, SS_EHIP, SS_ENOMEM.
 */
int slimsell_bfs_batch(ss_graph* g, const int32_t* roots, int32_t roots_per_graph,
                       const ss_bfs_opts* opts, int32_t* dist);

/* Wait for all work on `stream`; returns SS_EHIP if any of it failed. */
int slimsell_sync(void* stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char* slimsell_last_error(void);

/* Library version string. */
const char* slimsell_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SLIMSELL_H */
