// Internal declarations of libslimsell (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/slimsell.h"

namespace ss {

constexpr int kC = SS_CHUNK_HEIGHT;  // rows per chunk = wavefront width on CDNA
constexpr int32_t kInf = 0x7FFFFFFE; // tropical infinity; kInf + 1 does not overflow

int set_error(int code, const std::string& msg);

// SS_EHIP with the launch error, if the last kernel launch failed.
inline int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return SS_OK;
}

// Process-wide scheduler model (slimsell_sched_load); version 0 = none.
bool sched_model(std::vector<float>* out, uint64_t* version);

// Host layout (arrays described in slimsell.h, ss_layout_view).
struct Layout {
  int32_t n = 0, n_pad = 0, sigma = 0;
  int64_t n_chunks = 0, entries = 0, cells = 0;
  int32_t max_cl = 0;
  std::vector<int32_t> col;
  std::vector<int64_t> cs;
  std::vector<int32_t> cl;
  std::vector<int32_t> v;
  std::vector<int32_t> perm;
  std::vector<int32_t> degree;
};

int build_layout(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t C,
                 int32_t sigma, Layout** out);

// One unit of work for one wavefront.  Either a run of whole chunks
// [c0, c1) (c1 > c0 + 1, or a single unsplit chunk), or one piece
// [j0, j1) (columns) of chunk c0 (c1 == c0 + 1).
struct Unit {
  int32_t c0, c1;
  int32_t j0, j1;
};

// Work decomposition of one graph for one SlimChunk split length.
struct UnitList {
  int32_t split_len = 0;  // 0: never split
  int32_t pack_cols = 0;  // small chunks are packed into runs of up to this many columns
  int64_t count = 0;      // number of units
  int64_t split_chunks = 0;
  Unit* d_units = nullptr;      // device [count]
  int32_t* d_pieces = nullptr;  // device [n_chunks] pieces per chunk (1 = unsplit)
  // The pieces of a split chunk arrive in bundles of kBundle consecutive
  // pieces: a piece counts itself in its bundle's counter, the last piece of
  // a bundle counts the bundle in the chunk's counter, and the last bundle
  // post-processes the chunk, so no counter takes more than kBundle, or the
  // chunk's bundle count, atomics per level.
  std::vector<Unit> h_units;    // host copy of d_units (longest first)
  std::vector<int64_t> h_cols;  // columns of each unit
  int32_t* d_bundle = nullptr;  // device [n_chunks] first bundle counter of a split chunk
  int32_t* d_arrive2 = nullptr; // device [bundles] bundle counters (zero between levels)
  int64_t bundles = 0;
  // Per-wavefront assignments of the units for a grid of W wavefronts (by
  // W): the units reordered so that wavefront w's are [off[w], off[w + 1]),
  // chosen longest first onto the least-loaded wavefront.
  struct Assignment {
    Unit* d_units = nullptr;
    int32_t* d_off = nullptr;
  };
  std::map<int64_t, Assignment> assign;
};

// Workgroups of a level launch over n_units work units.
inline int64_t level_groups(int64_t n_units, int waves, int64_t max_groups) {
  int64_t groups = (n_units + waves - 1) / waves;
  if (groups < 1) groups = 1;
  if (max_groups > 0 && groups > max_groups) groups = max_groups;
  return groups;
}
constexpr int32_t kBundle = 16;  // pieces per arrival bundle

// Device workspace reused by every BFS on a graph.
struct Workspace {
  int64_t n_pad = 0;
  void* vec_a = nullptr;      // frontier / x buffer A   (4 B per row)
  void* vec_b = nullptr;      // frontier / x buffer B   (4 B per row)
  int32_t* state = nullptr;   // p (sel-max) or unused   (4 B per row)
  uint8_t* g = nullptr;       // filter g (real/boolean) (1 B per row)
  int32_t* d = nullptr;       // distances (row order)   (4 B per row)
  float* rv = nullptr;        // real value at discovery (4 B per row)
  int32_t* acc = nullptr;     // SlimChunk partial combine buffer (4 B per row)
  int32_t* arrive = nullptr;  // SlimChunk arrival counters (4 B per chunk)
  uint8_t* done = nullptr;    // 1 once every row of the chunk is final (1 B per chunk)
  uint64_t* any = nullptr;    // [kRing] per-level tag (run_id << 32 | level) if it found rows
  unsigned long long* counters = nullptr;  // per-level counters, see LevelArgs::counters
  int64_t counter_words = 0;               // capacity of counters[]
  // frontier queues (rows discovered at a level), learned-schedule state
  int32_t* q[2] = {nullptr, nullptr};  // [n_pad] each, by level parity
  int32_t* qn = nullptr;               // [kRing] queue length per level
  int32_t* variant = nullptr;          // [kRing] chosen variant per level
  uint64_t* decided = nullptr;         // [kRing] tagged decision per level (schedule kernel)
  unsigned long long* ring_ctr = nullptr;  // [kRing * kRingSlots * kCountFields]
  double* sched_sums = nullptr;        // [8] running totals for the features, 2 buffers
  float* sched_log = nullptr;          // [sched_log_cap * 12] features, scores, variant
  int64_t sched_log_cap = 0;
  int64_t sched_log_levels = 0;        // levels the last scheduled run recorded
  float* model = nullptr;              // [kModelCap] device copy of the scheduler model
  uint64_t model_version = 0;          // version of the process model copied there
  int2* segs = nullptr;                 // push segments: capacity seg_cap
  int64_t seg_cap = 0;
  int32_t* seg_n = nullptr;             // [2] segment counts by level parity
  unsigned* bar = nullptr;              // [2] grid barrier of the persistent kernel
  int32_t* pstatus = nullptr;           // [4] persistent run: levels, error, level cap
  // frontier summaries: one bit per chunk, set when a row of the chunk entered
  // the frontier; three buffers of summ_words words (level k writes k mod 3,
  // reads k - 1 mod 3 and clears k + 1 mod 3), then three words saying
  // whether the level wrote its buffer; nullptr when too large
  uint32_t* summ = nullptr;
  int32_t summ_words = 0;
  // host-mapped report ring written by the GPU: (tag << 1) | found
  // [kRing] level reports, then one word the learned schedule sets when its
  // model decides a level of the run (the level lies in its domain)
  volatile uint64_t* h_report = nullptr;
  uint64_t* d_report = nullptr;  // device view of h_report
};

constexpr int kBatchSemiring = 4;  // level-kernel policy id of the batched SpMM
constexpr int kDpSemiring = 5;     // level-kernel policy id of the DP transformation's sweep

// Device workspace of the batched SpMM (allocated on first use).
struct BatchWorkspace {
  int64_t n_pad = 0;
  unsigned long long* vis = nullptr;    // [n_pad] roots that reached the row
  unsigned long long* fa = nullptr;     // [n_pad] frontier masks, buffer A
  unsigned long long* fb = nullptr;     // [n_pad] frontier masks, buffer B
  unsigned long long* acc64 = nullptr;  // [n_pad] SlimChunk partial combine
  uint16_t* lvl = nullptr;              // [n_pad * 64] level of each (row, slot)
  unsigned long long* full = nullptr;   // [n_chunks] slots in use by the chunk's graph
  int32_t* root_rows = nullptr;         // [capacity] root row of each used slot
  int32_t* slots = nullptr;             // [capacity] slot of each used root
  int64_t root_cap = 0;
};

constexpr int kCountSlots = 16;  // statistics counter atomics are spread over this many slots
// The schedule's counters (read on the critical path of every scheduled
// level) are spread wider: one slot per lane of a wavefront, so a level's
// workgroups meet at most a few to an address (atomics on one address from
// all XCDs are serialised by the memory system).
constexpr int kRingSlots = 64;
// counter fields: discovered, active chunks, active cells, max active cl,
// degree sum of the discovered rows (frontier edges of the next level)
constexpr int kCountFields = 5;
constexpr int kVariants = 4;     // learned-schedule variants
constexpr int kPullVariants = 3; // pull with split 0 / 256 / 1024; variant 3 = push
constexpr int kPush = 3;
constexpr int kStop = -2;        // variant tag of a level past the end of the BFS
constexpr int kModelSize = 6 * 32 + 32 + 32 * 32 + 32 + 32 * 4 + 4;  // 1412 parameters
constexpr int kFeatures = 6;
// A model may carry its training domain after the parameters: tau, K, then K
// feature vectors (anchors); a level farther than tau from every anchor falls
// back to the fixed heuristic.  The library appends the anchors' bounding box
// widened by tau (6 lower, then 6 upper bounds): a level outside it is
// farther than tau from every anchor, which settles the test without the
// model or the anchor scan.  Then a coarse map of the box: kCellBins bins per
// feature (6 scales: bins per unit of each feature), and one bit per cell,
// set where the cell meets some anchor's cube of half-width tau (plus the
// box's margin).  A level in a clear cell is farther than tau from every
// anchor too.
constexpr int kMaxAnchors = 1024;
constexpr int kCellBins = 4;
constexpr int kCellWords = 4096 / 32;  // kCellBins^6 bits
constexpr int kModelCap =
    kModelSize + 2 + kMaxAnchors * kFeatures + 2 * kFeatures + kFeatures + kCellWords;
constexpr int kRing = 1024;  // level tags / reports are kept in rings of this size

struct Graph {
  int device = 0;
  int64_t n_cu = 0;  // compute units of the device
  int32_t n = 0, n_pad = 0, sigma = 0;
  int64_t n_chunks = 0, entries = 0, cells = 0;
  int32_t max_cl = 0;
  int32_t* d_col = nullptr;
  int64_t* d_cs = nullptr;
  int32_t* d_cl = nullptr;
  int32_t* d_v = nullptr;
  int32_t* d_perm = nullptr;
  int32_t* d_deg = nullptr;     // degree of each row (row order)
  // Sell-C-sigma comparator (built on first use): col with padding cells
  // holding row 0 and the val array (1 = edge, 0 = padding)
  int32_t* d_scol = nullptr;
  int32_t* d_sval = nullptr;
  std::vector<int32_t> h_perm;  // row of each original vertex
  std::vector<int32_t> h_cl;    // chunk lengths (for unit decomposition)
  std::vector<int32_t> h_degree;  // degree of each original vertex
  // prefix sums over chunks of the row degrees: the cells whose column lies
  // in the first k chunks of rows number h_chunk_deg[k] (the matrix is
  // symmetric), which says how many gathers an LDS prefix of rows serves
  std::vector<int64_t> h_chunk_deg;
  std::vector<void*> ev_pool;     // hipEvent_t pool for SS_STATS_TIME
  std::map<std::pair<int32_t, int32_t>, UnitList> units;  // by (split_len, pack_cols)
  Workspace ws;
  BatchWorkspace bw;
  // multi-graph description (one graph: num_graphs = 1, voff = {0, n})
  int32_t num_graphs = 1;
  std::vector<int64_t> h_voff;    // [num_graphs + 1] union-ID offset of each graph
  std::vector<int64_t> h_roff;    // [num_graphs + 1] row offset of each graph
  int64_t* d_voff = nullptr;
  uint32_t run_id = 0;
  ss_tune tune{128, 16, 4, 512, 0, 64};  // launch configuration (slimsell_tune_set / autotune)
  int32_t lds_cap = 0;                // largest LDS prefix the device allows, bytes
  int32_t lds_dev = 0;                // dynamic LDS the device allows one workgroup, bytes
  std::mutex mu;
};

// Arguments of one level kernel.
struct LevelArgs {
  const int32_t* col;
  const int32_t* val;  // Sell-C-sigma comparator: val beside col (nullptr = SlimSell)
  const int64_t* cs;
  const int32_t* cl;
  const int32_t* v;
  const int32_t* deg;  // degree of each row
  const Unit* units;
  const int32_t* pieces;
  int64_t n_units;
  const int32_t* bundle;   // per chunk: first bundle counter (split chunks)
  int32_t* arrive2;        // bundle counters
  int32_t piece_cols;      // columns per piece (the split length); 0 = no split
  // per-wavefront unit ranges [wave_off[w], wave_off[w + 1]) of `units` for
  // the launch grid's wavefronts (level_groups), or nullptr: round-robin
  const int32_t* wave_off;
  const void* vin;   // frontier read this level (gathered)
  void* vout;        // frontier written this level
  int32_t* state;    // p for sel-max; f for tropical (single buffer)
  uint8_t* g;
  int32_t* d;
  float* rv;
  int32_t* acc;
  int32_t* arrive;
  uint8_t* done;     // per chunk: all rows final (nullptr: not kept)
  uint64_t* any;
  // per-level counters of this root: [(level * kCountSlots + slot) * kCountFields + field]
  unsigned long long* counters;
  uint64_t* report;
  // learned schedule / push variant (variant == nullptr: pull with `units`)
  const int32_t* variant;
  const Unit* vunits[kPullVariants];
  const int32_t* vwave_off[kPullVariants];  // their per-wavefront ranges, or nullptr
  const int32_t* vpieces[kPullVariants];
  int64_t vn_units[kPullVariants];
  const int32_t* vbundle[kPullVariants];
  int32_t* varrive2[kPullVariants];
  int32_t vpiece_cols[kPullVariants];
  const int32_t* q_in;   // frontier rows of the previous level
  int32_t* q_out;        // frontier rows of this level
  int32_t* qn;           // [kRing] queue lengths
  unsigned long long* ring_ctr;  // per-level counters for the schedule (ring)
  int2* segs;            // push: segments (row, first cell) of long frontier rows
  int32_t* seg_n;        // push: segment count of this level (cleared one level ahead)
  // batched SpMM only
  unsigned long long* acc64;
  unsigned long long* vis;
  const unsigned long long* full;
  uint16_t* lvl;
  uint32_t run_id;
  uint32_t n_pad;    // rows (multiple of 64)
  uint32_t lds_bytes;  // prefix of the gathered vector staged in LDS (0 = none)
  uint32_t* summ;      // frontier summaries (Workspace::summ) or nullptr: no gather filter
  int32_t summ_words;
  int32_t filter_limit;  // filter while at most this many chunks hold frontier rows
  int32_t prefix_words;  // summary words that cover the chunks of the LDS prefix's rows
  int32_t level;     // k >= 1
  int32_t slimwork;
  int32_t count_stats;
};

// Dynamic LDS of a level launch: the staged prefix plus the frontier summary.
inline uint32_t level_lds(const LevelArgs& a) {
  return a.lds_bytes + (a.summ ? (uint32_t)a.summ_words * 4u : 0u);
}
constexpr int64_t kSummMaxBytes = 32 * 1024;  // summaries above this size are not kept

// Parameters of the schedule that stay fixed over one run.
struct SchedLaunch {
  uint64_t* any;
  uint64_t* report;
  int32_t* variant;
  int32_t* qn;
  int32_t* seg_n;
  unsigned long long* ring_ctr;
  double* sums;
  const float* model;
  const float* anchors;   // training-domain anchors [n_anchors][6] or nullptr
  const float* box;       // [12] their box widened by tau (lower, upper) or nullptr
  const float* cells;     // [6 + kCellWords] the box's cell map (scales, bits) or nullptr
  uint64_t* decided;      // [kRing] decisions published for later workgroup rounds
  uint64_t* in_box;       // device view of the host word "the model decided a level"
  int32_t eager;          // stage the model up front (the last learned run used it)
  int32_t n_anchors;
  float tau2;             // squared distance beyond which the heuristic decides
  float* log;
  int32_t log_cap;
  int32_t mode;
  int32_t heuristic_pull;
  double n, two_m;
};

// One run in a single cooperative launch: level cap, grid barrier words,
// status words ([0] levels run or -1 at the cap, [1] barrier timed out,
// [2] level-statistics cap), barrier deadline in wall-clock ticks; with
// `sched` set, the scheduled form with frontier queues q0/q1.
struct PersistentRun {
  int32_t cap;
  int64_t max_groups;
  unsigned* bar;
  int32_t* status;
  uint64_t limit;
  const SchedLaunch* sched;
  int32_t* q0;
  int32_t* q1;
};

// Kernel launchers (kernels.hip).
// Rows up to this degree are swept by one lane in a push level; longer rows
// are cut into segments for the segments kernel, which a graph whose degrees
// never exceed it does not need (segments = false).
constexpr int kPushLaneMax = 32;
int launch_push(int semiring, const LevelArgs& a, bool segments, void* stream);
int launch_persistent(int semiring, int unroll, const LevelArgs& a, void* buf_a, void* buf_b,
                      const PersistentRun& r, void* stream);
// One scheduled level: variant choice, then the pull variant or the push
// scatter (launch_push adds the push segments and post kernels).
int launch_sched_level(int semiring, int waves, int unroll, int64_t max_groups,
                       const LevelArgs& a, const SchedLaunch& p, void* stream);
// DP transformation (dp.hip): parents (original IDs) from distances (original
// IDs) of one root, through the workspace's d (4 B per row), g (n_pad / 4
// bytes of codes), acc and state (4 B per row each) and arrive buffers.
// `state` receives each row's best v.  With `counters` (one level's
// counter block, see LevelArgs::counters, written at level index 1) the sweep
// counts its chunks and cells; ev_begin/ev_end (hipEvent_t or NULL) bracket
// the sweep kernel.
// `as` (or NULL: round-robin) is the units' per-wavefront assignment for
// the sweep's grid.  `src` says where the row-order distances come from:
// kDpFromDist gathers the original-order `dist`; right after a BFS on ws,
// kDpFromTropical reads its tropical distance vector (ws.state) and
// kDpFromRowD the distances the real and boolean forms keep in ws.d; with
// those two, `dist_out` (or NULL) receives the run's distances in original
// order, written by the pass that writes the parents.
constexpr int32_t kDpFromDist = 0, kDpFromTropical = 1, kDpFromRowD = 2;
int launch_dp(const Graph& g, const Workspace& ws, const UnitList& ul,
              const UnitList::Assignment* as, int unroll, int waves, int64_t max_groups,
              const int32_t* dist, int32_t src, int32_t* dist_out, int32_t* parent, void* stream,
              unsigned long long* counters = nullptr, void* ev_begin = nullptr,
              void* ev_end = nullptr);
int launch_sched_init(const Graph& g, const Workspace& ws, int32_t root_row, void* stream);
int launch_init(int semiring, const Graph& g, const Workspace& ws, int32_t root_row, bool summary,
                void* stream);
int launch_level(int semiring, int waves, int unroll, int64_t max_groups, const LevelArgs& a,
                 void* stream);
int launch_finalise(int semiring, const Graph& g, const Workspace& ws, int32_t* dist,
                    int32_t* parent, float* real_val, void* stream);
int launch_fill_i32(int32_t* p, int32_t value, int64_t count, void* stream);
// Sell-C-sigma arrays from the SlimSell col (same shape).
int launch_sell_build(const int32_t* col, int64_t cells, int32_t* scol, int32_t* sval,
                      void* stream);
int launch_batch_init(const Graph& g, const BatchWorkspace& b, int32_t count, bool summary,
                      void* stream);
int launch_batch_finalise(const Graph& g, const BatchWorkspace& b, int32_t rpg, int32_t* dist,
                          void* stream);
int launch_fill_u64(unsigned long long* p, unsigned long long value, int64_t count, void* stream);

}  // namespace ss

// The opaque ABI types are the internal structures.
struct ss_layout : public ss::Layout {};
struct ss_graph : public ss::Graph {};
