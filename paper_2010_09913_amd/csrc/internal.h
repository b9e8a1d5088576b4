// Internal declarations of libslimsell (not part of the C ABI).
#pragma once

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
};

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
  uint64_t* any = nullptr;    // [kRing] per-level tag (run_id << 32 | level) if it found rows
  unsigned long long* counters = nullptr;  // per-level counters, see LevelArgs::counters
  int64_t counter_words = 0;               // capacity of counters[]
  // host-mapped report ring written by the GPU: (tag << 1) | found
  volatile uint64_t* h_report = nullptr;
  uint64_t* d_report = nullptr;  // device view of h_report
};

constexpr int kBatchSemiring = 4;  // level-kernel policy id of the batched SpMM

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

constexpr int kCountSlots = 16;  // counter atomics are spread over this many slots
constexpr int kCountFields = 4;  // discovered, active chunks, active columns, max active cl
constexpr int kRing = 1024;  // level tags / reports are kept in rings of this size

struct Graph {
  int device = 0;
  int32_t n = 0, n_pad = 0, sigma = 0;
  int64_t n_chunks = 0, entries = 0, cells = 0;
  int32_t max_cl = 0;
  int32_t* d_col = nullptr;
  int64_t* d_cs = nullptr;
  int32_t* d_cl = nullptr;
  int32_t* d_v = nullptr;
  int32_t* d_perm = nullptr;
  int32_t* d_deg = nullptr;     // degree of each row (row order)
  std::vector<int32_t> h_perm;  // row of each original vertex
  std::vector<int32_t> h_cl;    // chunk lengths (for unit decomposition)
  std::vector<int32_t> h_degree;  // degree of each original vertex
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
  ss_tune tune{256, 1, 8, 0, 0, 0};  // launch configuration (slimsell_tune_set / autotune)
  std::mutex mu;
};

// Arguments of one level kernel.
struct LevelArgs {
  const int32_t* col;
  const int64_t* cs;
  const int32_t* cl;
  const int32_t* v;
  const int32_t* deg;  // degree of each row
  const Unit* units;
  const int32_t* pieces;
  int64_t n_units;
  const void* vin;   // frontier read this level (gathered)
  void* vout;        // frontier written this level
  int32_t* state;    // p for sel-max; f for tropical (single buffer)
  uint8_t* g;
  int32_t* d;
  float* rv;
  int32_t* acc;
  int32_t* arrive;
  uint64_t* any;
  // per-level counters of this root: [(level * kCountSlots + slot) * kCountFields + field]
  unsigned long long* counters;
  uint64_t* report;
  // batched SpMM only
  unsigned long long* acc64;
  unsigned long long* vis;
  const unsigned long long* full;
  uint16_t* lvl;
  uint32_t run_id;
  uint32_t n_pad;    // rows (multiple of 64)
  int32_t level;     // k >= 1
  int32_t slimwork;
  int32_t count_stats;
};

// Kernel launchers (kernels.hip).
int launch_init(int semiring, const Graph& g, const Workspace& ws, int32_t root_row, void* stream);
int launch_level(int semiring, int waves, int unroll, int64_t max_groups, const LevelArgs& a,
                 void* stream);
int launch_finalise(int semiring, const Graph& g, const Workspace& ws, int32_t* dist,
                    int32_t* parent, float* real_val, void* stream);
int launch_fill_i32(int32_t* p, int32_t value, int64_t count, void* stream);
int launch_batch_init(const Graph& g, const BatchWorkspace& b, int32_t count, void* stream);
int launch_batch_finalise(const Graph& g, const BatchWorkspace& b, int32_t rpg, int32_t* dist,
                          void* stream);
int launch_fill_u64(unsigned long long* p, unsigned long long value, int64_t count, void* stream);

}  // namespace ss

// The opaque ABI types are the internal structures.
struct ss_layout : public ss::Layout {};
struct ss_graph : public ss::Graph {};
