// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <mutex>
#include <vector>

#include "../../include/gsw.h"

namespace gsw {

// Records a message for gsw_last_error() and returns the status.
gsw_status fail(gsw_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define GSW_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return ::gsw::fail(GSW_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                         __FILE__, __LINE__);                                                 \
  } while (0)

#define GSW_TRY(expr)                 \
  do {                                \
    gsw_status s_ = (expr);           \
    if (s_ != GSW_OK) return s_;      \
  } while (0)

// Frontier queues are split into kQueueBins segments, one per residue of the
// producing workgroup id, each with room for every vertex; a workgroup stages
// its discoveries in LDS and appends them with one atomic on its segment's
// counter.  Same-address atomics serialise (about 11 ns each on MI355X), so
// spreading the appends over several counters keeps a level's append cost
// small.  Counters sit kCtrStride words apart (separate 128-byte lines).
constexpr int kQueueBins = 8;
constexpr int kCtrStride = 32;
constexpr int kCtrSlot = kQueueBins * kCtrStride;  // words per level in the counter ring

// Device state of one BFS in flight.  Bitmaps are 64-bit words, bit (v & 63)
// of word v >> 6; the last word's bits beyond n are set in `vis` so they are
// never treated as unvisited.
struct Workspace {
  int64_t n = 0, nw = 0;
  unsigned long long* vis = nullptr;     // visited
  unsigned long long* bm[2] = {};        // frontier bitmaps (depth d and d+1)
  int32_t* q[2] = {};                    // frontier queues, kQueueBins segments of n
  uint32_t* ctr = nullptr;               // ring of 4 levels x kCtrSlot words
  int64_t* scan = nullptr;               // push_edge: per-entry exclusive degree scan
  int64_t* ebeg = nullptr;               // push_edge: row start per queue entry
  int64_t* bsum = nullptr;               // push_edge: per-block sums
  unsigned long long* etot = nullptr;    // push_edge: total frontier edges
  int32_t* lvl_tmp = nullptr;            // levels when the caller passes host memory
  int32_t* par_tmp = nullptr;            // parents when the caller passes host memory
  uint32_t* h_ctr = nullptr;             // pinned host copy of one counter slot
  uint32_t* h_flag = nullptr;            // mapped host memory: frontier size per level slot
  uint32_t* d_flag = nullptr;            // the same memory as seen by the device
  hipEvent_t ev[2] = {};
  unsigned long long* tst = nullptr;     // per-workgroup start/end wall-clock stamps of a level
  unsigned long long* lvl_ticks = nullptr;  // per-level kernel duration in wall-clock ticks
  unsigned long long* h_ticks = nullptr;    // pinned host copy of lvl_ticks
  double tick_ms = 0.0;                     // milliseconds per wall-clock tick
  size_t bytes = 0;
};

struct MsWorkspace;  // batched BFS state (gsw_msbfs.hip)

}  // namespace gsw

struct gsw_graph {
  int device = 0;
  int64_t n = 0, nnz = 0;
  const int64_t* offs = nullptr;  // device
  const int32_t* cols = nullptr;  // device
  int32_t* origin = nullptr;      // device, built on demand (edge_scan)
  unsigned long long* iso = nullptr;  // device bitmap of degree-0 vertices (symmetric graphs)
  bool owns_csr = false;
  int symmetric = 0;              // 1 when checked or vouched for
  double deg_stats[6] = {};       // min, q1, median, q3, max, std
  size_t csr_bytes = 0, origin_bytes = 0;
  gsw::Workspace ws;
  gsw::MsWorkspace* ms = nullptr; // batched BFS workspace, sized for the largest batch seen
  // batched BFS: rows longer than the chunked-row limit as (vertex << 32 |
  // chunk index) entries, built on first use; -1 = not built yet
  unsigned long long* heavy = nullptr;
  int64_t n_heavy = -1;
  hipStream_t stream = nullptr;   // library stream for this graph
  std::mutex mu;
};

struct gsw_tree {
  int32_t n_nodes = 0, n_classes = 0;
  std::vector<int32_t> feature, left, right, class_kernel;
  std::vector<double> threshold, value;
};

namespace gsw {

// Kernel launchers (gsw_kernels.hip).
struct LevelLaunch {
  const int64_t* offs;
  const int32_t* cols;
  const int32_t* origin;
  int32_t* level;
  int32_t* parent;          // may be null
  unsigned long long* vis;
  const unsigned long long* fr;  // frontier bitmap of depth d (pull only)
  unsigned long long* nx;        // depth d+1 bitmap, written whole by pull
  const int32_t* qin;       // queue of depth d (kQueueBins segments)
  const uint32_t* cin;      // its segment counts (a counter slot)
  int32_t* qout;            // queue of depth d+1
  uint32_t* cout;           // its segment counters (zero on entry)
  uint32_t* cclr;           // counter slot to zero for the level after next
  unsigned long long* tst;  // wall-clock stamps per workgroup (null: not timed)
  int64_t n, nw, nnz;
  uint32_t n_in;
  int32_t d;
};

gsw_status launch_init(const gsw_graph* g, int32_t* level, int32_t* parent, int32_t source,
                       hipStream_t s);
gsw_status launch_level(const gsw_graph* g, int kernel, const LevelLaunch& a, hipStream_t s);
gsw_status launch_frontier_bitmap(const gsw_graph* g, const int32_t* level, int32_t d,
                                  unsigned long long* bm, hipStream_t s);
gsw_status launch_isolated(const gsw_graph* g, unsigned long long* iso, hipStream_t s);
gsw_status launch_finalize(const uint32_t* cslot, uint32_t* d_flag, unsigned long long* tst,
                           unsigned long long* ticks, hipStream_t s);
gsw_status launch_canonical_parents(const gsw_graph* g, const int32_t* level, int32_t* parent,
                                    hipStream_t s);
gsw_status launch_build_origin(const gsw_graph* g, int32_t* origin, hipStream_t s);

gsw_status ensure_workspace(gsw_graph* g);
gsw_status ensure_origin(gsw_graph* g);
hipStream_t pick_stream(gsw_graph* g, void* user_stream);

bool kernel_is_pull(int k);
void ms_release(gsw_graph* g);

// Marker of a level-size slot in host memory that the device has not written.
constexpr uint32_t kNotReady = 0xffffffffu;
constexpr int kFlagSlots = 4;
// Levels of one BFS whose kernel time time_levels records (later levels get -1).
constexpr int kMaxTimedLevels = 8192;
// Workgroups whose start/end stamps time a level (larger grids stamp from
// their first kStampBlocks workgroups).
constexpr int kStampBlocks = 4096;

}  // namespace gsw
