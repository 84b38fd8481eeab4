// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
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

// Host wait for a record that a kernel posts to mapped host memory: spins on
// posted(), asking the stream for errors now and then so a failed launch
// cannot leave the host spinning.  A stream that reports idle before the
// record is seen is not taken at its word: it is synchronized once, and the
// record then has kRecordGraceMs to appear before *missing is set.  The
// record of a level that really ran is therefore never reported missing
// because the idle report came early; a record that never comes costs the
// grace period.  Returns the stream's error, if any.
constexpr int kRecordGraceMs = 5000;

template <class Posted>
hipError_t await_record(Posted posted, hipStream_t s, bool* missing) {
  *missing = false;
  bool idle = false;
  std::chrono::steady_clock::time_point since{};
  for (uint64_t it = 0;; ++it) {
    if (posted()) return hipSuccess;
    if ((it & 4095u) == 4095u) {
      if (!idle) {
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) {
          idle = true;
          const hipError_t e2 = hipStreamSynchronize(s);
          if (e2 != hipSuccess) return e2;
          since = std::chrono::steady_clock::now();
        } else if (e != hipErrorNotReady) {
          return e;
        }
      } else if (std::chrono::steady_clock::now() - since > std::chrono::milliseconds(kRecordGraceMs)) {
        *missing = !posted();
        return hipSuccess;
      }
    }
    __builtin_ia32_pause();
  }
}

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
struct BfsCtl;

// Bottom-up probes start from a dense copy of kHeadArcs in-arcs of every
// vertex ([n][kHeadArcs], -1 past the row's end): a wave's unvisited
// vertices read theirs as consecutive 16-byte records instead of one
// scattered cache line per row, and only rows still unresolved after them
// are read in the CSR.  On a graph whose out-degrees are skewed
// (head_ranking_pays) the single-source workspace ranks them: the
// kHeadArcs in-neighbours of largest out-degree among the row's first
// kHeadScan arcs (a vertex of larger degree is in a large frontier sooner),
// so most vertices of a large bottom-up level resolve in the head; rows that
// do not are then probed from their start.  Otherwise, and on the
// no-allocation path, which rebuilds the head on every call, the head is the
// row's first kHeadArcs arcs and the rest of the row is probed past them.
constexpr int kHeadArcs = 4;
constexpr int kHeadScan = 256;

// Per-level arc counters (gsw_bfs_opts.count_arcs): a ring of 4 levels of
// kQueueBins 64-bit counters, kArcStride words apart.
constexpr int kArcStride = 16;
constexpr int kArcSlot = kQueueBins * kArcStride;

__host__ __device__ inline int kernel_base(int k) { return k % GSW_N_BASE_KERNELS; }
__host__ __device__ inline int kernel_count(int k) { return k / GSW_N_BASE_KERNELS; }

struct Workspace {
  int64_t n = 0, nw = 0;
  unsigned long long* vis = nullptr;     // visited
  unsigned long long* bm[3] = {};        // frontier bitmaps, depth d in bm[d % 3]
  int32_t* q[2] = {};                    // frontier queues, kQueueBins segments of n
  uint32_t* ctr = nullptr;               // ring of 4 levels x kCtrSlot words
  unsigned long long* actr = nullptr;    // ring of 4 levels x kArcSlot arc counters
  int64_t* scan = nullptr;               // push_edge: per-entry exclusive degree scan
  int64_t* ebeg = nullptr;               // push_edge: row start per queue entry
  int64_t* bsum = nullptr;               // push_edge: per-block sums
  int32_t* head = nullptr;               // pull: first kHeadArcs in-arcs of every vertex
  int32_t* lvl_tmp = nullptr;            // levels when the caller passes host memory
  int32_t* par_tmp = nullptr;            // parents when the caller passes host memory
  uint32_t* h_ctr = nullptr;             // pinned host copy of one counter slot
  BfsCtl* ctl = nullptr;                 // device level control
  unsigned long long* done = nullptr;    // finished-workgroup counters of the running launch
  BfsCtl* h_ctl = nullptr;               // pinned staging for control-block uploads (profiling)
  unsigned long long* ring = nullptr;    // mapped host memory: per-level records
  unsigned long long* d_ring = nullptr;  // the same memory as seen by the device
  unsigned long long* d_tree = nullptr;  // device copy of the tree's nodes (packed) ...
  int32_t* d_thr = nullptr;              // ... and integer thresholds
  int32_t tree_cap = 0;                  // nodes the device copy has room for
  int32_t tree_nodes = 0;                // nodes of the device copy (specialised to this graph)
  uint64_t tree_id = 0;                  // tree currently uploaded (0: none)
  int32_t* d_sched = nullptr;            // device copy of a schedule
  int32_t sched_cap = 0;
  std::vector<int32_t> sched_host;       // the schedule that d_sched holds
  hipEvent_t ev[2] = {};
  static constexpr int kLaunchEvents = 16;  // ring of per-launch events (time_levels = 2)
  hipEvent_t lev[kLaunchEvents] = {};
  double tick_ms = 0.0;                  // milliseconds per wall-clock tick
  size_t bytes = 0;
  bool head_built = false;               // head holds the graph's rows
  bool head_ranked = false;              // head holds ranked in-arcs, not the first ones
  bool ready = false;                    // every buffer allocated and built
  int64_t ring_used = -1;                // ring slots the last search may have written (-1: all)
};

struct MsWorkspace;  // batched BFS state (gsw_msbfs.hip)
struct CcWorkspace;  // connected-components state (gsw_cc.hip)

}  // namespace gsw

struct gsw_graph {
  int device = 0;
  int64_t n = 0, nnz = 0;
  const int64_t* offs = nullptr;  // device
  const int32_t* cols = nullptr;  // device
  int32_t* origin = nullptr;      // device, built on demand (edge_scan): row of every arc
  // in-arcs (the transpose): the same arrays as offs/cols on a symmetric
  // graph, a library-owned copy on a directed one
  const int64_t* roffs = nullptr;
  const int32_t* rcols = nullptr;
  int32_t* rorigin = nullptr;     // device, built on demand (rev_edge_scan): row of every in-arc
  unsigned long long* iso = nullptr;  // device bitmap of vertices without in-arcs
  bool owns_csr = false;
  int symmetric = 0;              // 1 when checked or vouched for
  double deg_stats[6] = {};       // out-degree: min, q1, median, q3, max, std
  double gfeat[GSW_N_GRAPH_FEATURES] = {};  // graph features of the tree
  size_t csr_bytes = 0, origin_bytes = 0, rcsr_bytes = 0;
  gsw::Workspace ws;
  gsw::MsWorkspace* ms = nullptr; // batched BFS workspace, sized for the largest batch seen
  // batched BFS: rows longer than the chunked-row limit as (vertex << 32 |
  // chunk index) entries, built on first use; -1 = not built yet
  unsigned long long* heavy = nullptr;
  int64_t n_heavy = -1;
  gsw::CcWorkspace* cc = nullptr; // connected components, allocated on first use
  hipStream_t stream = nullptr;   // library stream for this graph
  std::mutex mu;
};

struct gsw_tree {
  int32_t n_nodes = 0, n_classes = 0;
  std::vector<int32_t> feature, left, right, class_kernel;
  std::vector<double> threshold, value;
  std::vector<int32_t> leaf_kernel;  // per node: the leaf's kernel, -1 when undecided (tie)
  uint64_t id = 0;                   // unique per created tree (device copies are keyed by it)
};

namespace gsw {

// Single-source level control in device memory: set by the init kernel and,
// for every next level, by the last workgroup of the current level's kernel.
struct BfsCtl {
  int32_t d;        // level to run next
  int32_t kernel;   // its kernel (kCtlDone once a level found nothing)
  int32_t prev;     // kernel of level d-1
  int32_t flags;    // trace flags of that choice (bit0 undecided leaf, bit1 pull replaced)
  long long nf;     // frontier size of level d
  long long disc;   // vertices discovered through depth d
  unsigned long long done;   // running launch: finished groups << 40 | queue entries they appended
  int32_t phase;             // push_edge: 0 = prefix launch, 1 = expansion launch, 2 = both in one
  int32_t grid;              // workgroups that run this launch of level d (the rest exit)
  unsigned long long t_begin;  // wall clock at the start of the running level (timed levels)
  long long etot;              // push_edge: arcs of the frontier (set by the prefix launch)
  long long ef;                // arcs of the depth-d frontier (count_arcs), else -1
  int32_t clean;               // 1: the bitmap of depth d-1 (bm[(d + 2) % 3]) is already all zero
  int32_t pad;
};
// Workgroups count themselves finished, together with the queue entries they
// appended, in kDoneGroups 64-bit counters (by index modulo kDoneGroups,
// kCtrStride words apart); the last of each group then adds its group's sums
// to BfsCtl::done, so the launch's last workgroup learns the next frontier's
// size from its own atomic.  Same-address atomics serialise, so a full
// launch on one counter would cost about 15 us per level.
constexpr int kDoneGroups = 16;
constexpr int32_t kCtlDone = -1;

// push_edge with at most kEdgeFuse frontier entries runs in one launch
// (every workgroup scans the whole queue in LDS); a larger one takes two.
constexpr int64_t kEdgeFuse = 512;
__host__ __device__ inline int32_t level_first_phase(int kernel, int64_t nf) {
  return kernel >= 0 && kernel_base(kernel) == GSW_K_PUSH_EDGE ? (nf <= kEdgeFuse ? 2 : 0) : 0;
}
__host__ __device__ inline int level_launches(int kernel, int64_t nf) {
  return kernel >= 0 && kernel_base(kernel) == GSW_K_PUSH_EDGE && nf > kEdgeFuse ? 2 : 1;
}

// How the device picks the next level's kernel (a kernel argument): the same
// policies and rules as the host's choice for level 0.
struct BfsPolicy {
  int32_t policy, fixed, sched_len, symmetric;
  int32_t has_origin;        // edge_scan can run (its origin array exists)
  int32_t has_rorigin;       // rev_edge_scan can run (the in-arcs' origin array exists)
  const int32_t* sched;      // device copy of the schedule
  const unsigned long long* t_node;  // tree nodes, packed (see tree_node_pack)
  const int32_t* t_thr;      // per node: the split holds when its count is <= t_thr
  int32_t t_nodes;           // nodes of the tree
  int32_t pad2;
};

// Buffers of one single-source BFS (a kernel argument of the level kernels).
struct BfsBase {
  const int64_t* offs;
  const int32_t* cols;
  const int32_t* origin;
  const int64_t* roffs;            // in-arcs (== offs/cols on a symmetric graph)
  const int32_t* rcols;
  const int32_t* rorigin;
  const int32_t* head;             // first kHeadArcs in-arcs of every vertex, -1 padded
  int32_t* level;
  int32_t* parent;                 // may be null
  unsigned long long* vis;
  unsigned long long* bm[3];
  int32_t* q[2];
  uint32_t* ctr;
  unsigned long long* actr;        // arc counters (count_arcs)
  unsigned long long* done;        // kDoneGroups workgroup counters, kCtrStride words apart
  int64_t* scan;                   // push_edge: block-local exclusive arc offsets per queue entry
  int64_t* ebeg;                   // push_edge: row start per queue entry
  int64_t* bsum;                   // push_edge: arcs per scan block, then their exclusive prefix
  unsigned long long* ring;        // device address of the host record ring
  BfsCtl* ctl;                     // two slots: launch j reads j % 2, writes the other
  int64_t n, nw, nnz;
  int32_t timed;                   // record each level's duration
  int32_t grid_max;                // workgroups of a level-kernel launch
  int32_t count_arcs;              // accumulate the next frontier's out-degrees
  int32_t solo;                    // levels one single-workgroup launch may run (0: such launches off)
  int32_t deg_max;                 // largest out-degree (clamped to 2^31 - 1)
  int32_t head_ranked;             // head holds ranked in-arcs (bottom-up rows are then probed from their start)
};

// Single-workgroup multi-level launches (k_level_solo): while the frontier
// is small, one workgroup of kSoloBlock threads runs consecutive top-down
// levels from the queue, applies the policy between them and posts every
// level's record, instead of one launch of the whole grid per level.  A
// level qualifies when its kernel is a queue-driven top-down one
// (push_vertex, push_wave, push_edge), its frontier has at most kSoloMax
// vertices and its arcs are bounded: by the graph's largest degree, or, in
// the shrinking tail of a search that has reached 1% of the graph, by a
// check of the actual arc count (at most kSoloMaxArcs) before the level
// starts.  A launch runs at most kSoloMaxLevels levels.
// One compute unit's memory pipeline bounds such a workgroup: measured on
// MI355X (2048 x 2048 grid), a level costs it about 3.5 us up to 64
// frontier vertices, 4.3 us up to 256 and 6.4 us up to 512, then grows with
// the frontier (12 us up to 1024, 22 us up to 2048), while a level kernel
// launch costs about 6 us on the device plus about 3 us between launches at
// any of these sizes; hence kSoloMax = 512.
constexpr int kSoloBlock = 1024;
constexpr int kSoloSlots = 2;  // frontier entries per thread at most
constexpr int64_t kSoloMax = 512;
static_assert(kSoloMax <= (int64_t)kSoloBlock * kSoloSlots, "every frontier entry has a thread slot");
constexpr int64_t kSoloMaxArcs = 65536;
constexpr int kSoloMaxLevels = 32;
constexpr int32_t kSoloTree = 1024;  // tree nodes the workgroup holds in LDS
__host__ __device__ inline bool solo_eligible(int k, long long nn, long long nf, long long disc_next, long long n,
                                              int32_t deg_max) {
  if (k < 0 || kernel_base(k) > GSW_K_PUSH_EDGE) return false;
  if (nn < 1 || nn > kSoloMax) return false;
  if ((long long)deg_max * nn <= kSoloMaxArcs) return true;
  return nn <= nf && disc_next * 100 >= n;
}

// A tree node in 8 bytes for the device walk: left and right child (int16,
// -1 at a leaf), the count the split tests (0: next frontier size,
// 1: vertices discovered through the next depth), leaf kernel + 1 (0 when
// the leaf's classes tie; kernel ids fit the byte).  Trees of up to 32767
// nodes.
inline unsigned long long tree_node_pack(int32_t left, int32_t right, int32_t count, int32_t leaf_kernel) {
  return (unsigned long long)(uint16_t)(int16_t)left | ((unsigned long long)(uint16_t)(int16_t)right << 16) |
         ((unsigned long long)(uint8_t)count << 32) | ((unsigned long long)(uint8_t)(leaf_kernel + 1) << 40);
}
constexpr int32_t kMaxTreeNodes = 32767;

// Host ring of per-level records: record of level d at (d % kBfsRing) * kBfsRec.
// Every word carries the level's tag (rec_tag) in its top 16 bits and a
// value below 2^48 in the rest, so the host takes a record once all its
// words bear the tag, whatever order their stores arrive in, and the device
// never waits for them.
constexpr int kBfsRing = 256;
constexpr int kBfsRec = 16;
enum : int {
  kRecKernel = 0,   // kernel that ran level d
  kRecFlags = 1,    // its trace flags
  kRecNf = 2,       // frontier size of level d
  kRecDisc = 3,     // discovered through depth d
  kRecNext = 4,     // size of the depth-(d+1) frontier
  kRecTicks = 5,    // wall-clock ticks of the level (timed levels)
  kRecNextKernel = 6,  // kernel chosen for level d+1, plus one (0: none)
  kRecEf = 7,          // arcs of the depth-d frontier plus one (0: not counted)
  kRecLaunch = 8,      // index of the level-kernel launch that completed level d
  kBfsRecWords = 9
};
// Trace flag of a level run by a single-workgroup multi-level launch.
constexpr int32_t kFlagSolo = 4;
constexpr unsigned long long kRecValueMask = (1ull << 48) - 1ull;
// Never zero (the cleared ring) and different for the 8 levels sharing a slot.
__host__ __device__ inline unsigned long long rec_tag(long long d) {
  return (unsigned long long)(((d + 1) & 0x7fff) | 0x8000) << 48;
}

// Kernel launchers (gsw_kernels.hip).
// iso: bitmap of the vertices without in-arcs (they start visited), or null.
gsw_status launch_init(const gsw_graph* g, const BfsBase& b, const unsigned long long* iso, int32_t source,
                       int32_t k0, int32_t flags0, hipStream_t s);
// Launch j (counted from 0 after launch_init) of the level kernel: runs what
// control slot j % 2 names -- a level, or the scan or the expansion of a
// push_edge level -- or nothing once the search has ended.  `workgroups`
// (clamped to [1, b.grid_max]) is the launch size; a level that asks for
// more workgroups than the launch has runs on the launch's, striding.
gsw_status launch_level_auto(const gsw_graph* g, const BfsBase& b, const BfsPolicy& p, int32_t j,
                             int32_t workgroups, hipStream_t s);
// Launch j as a single-workgroup multi-level launch: runs the levels that
// qualify from the one control slot j % 2 names (none when it does not
// qualify; the slot then passes to launch j + 1 unchanged).
gsw_status launch_level_solo(const gsw_graph* g, const BfsBase& b, const BfsPolicy& p, int32_t j, hipStream_t s);
// Workgroups of a level-kernel launch on a graph of n vertices (nw bitmap words).
int32_t level_kernel_grid(int64_t n, int64_t nw);
// Workgroups of that launch that run a level of `kernel` with n_in frontier entries.
int32_t level_participants(int kernel, int64_t n_in, const BfsBase& b);
gsw_status launch_isolated(const gsw_graph* g, unsigned long long* iso, hipStream_t s);
gsw_status launch_canonical_parents(const gsw_graph* g, const int32_t* level, int32_t* parent,
                                    hipStream_t s);
gsw_status launch_build_origin(const int64_t* offs, int64_t n, int32_t* origin, hipStream_t s);
// Whether the single-source workspace ranks the head (out-degree standard deviation above the mean).
bool head_ranking_pays(const gsw_graph* g);
// ranked: the kHeadArcs in-neighbours of largest out-degree (see kHeadArcs), else the first ones.
gsw_status launch_build_head(const gsw_graph* g, int32_t* head, bool ranked, hipStream_t s);

// ----- pieces of the single-source level loop (gsw_bfs.cpp)
// A level's record, decoded.
struct Record {
  int kernel;
  int32_t flags;
  int64_t nf, disc, next;
  unsigned long long ticks;
  int next_kernel;  // kCtlDone when the search ended
  int64_t ef;       // arcs of the level's frontier, -1 when not counted
  int64_t launch;   // launch that completed the level
};
// Level d's record from a ring (host memory), if all its words bear d's tag.
bool take_record(const volatile unsigned long long* ring, int64_t d, Record* rec);
void trace_row(gsw_level_trace* t, int32_t src_idx, int64_t d, const Record& r, bool timed, double tick_ms);
// Workgroups for the launches queued after a record (quiet phases get few).
int32_t launch_size(int next_kernel, int64_t nn, int64_t nf, int64_t nf_prev, int64_t disc, int64_t d, int64_t n,
                    int32_t cap);
// Level 0's kernel on the host (the device applies the same rules later).
int first_kernel(const gsw_graph* g, const gsw_bfs_opts* o, bool has_origin, bool has_rorigin, int32_t* flags);
// Buffers for specialise_tree, each with room for the tree's n_nodes
// (stack: n_nodes + 1); nodes/thr receive the specialised tree.
struct TreeBuf {
  int32_t *order, *newid, *stack;
  unsigned long long* nodes;
  int32_t* thr;
};
// The tree specialised to the graph (splits on graph features decided, level
// splits as integer count thresholds); returns its node count.
int32_t specialise_tree(const gsw_graph* g, const gsw_tree* t, const TreeBuf& buf);
BfsPolicy device_policy(const gsw_graph* g, const Workspace& w, const gsw_bfs_opts* o, bool has_origin,
                        bool has_rorigin);
BfsBase make_base(const gsw_graph* g, const Workspace& w, int32_t* lv, int32_t* pa, bool timed, bool count_arcs);

gsw_status ensure_workspace(gsw_graph* g);
size_t workspace_bytes(const gsw_graph* g);  // what ensure_workspace allocates in all
gsw_status ensure_origin(gsw_graph* g);
gsw_status ensure_rorigin(gsw_graph* g);
// Single-source BFS rows [count][n] int32 into device memory, with the graph's
// lock already held (the batched path's fallback); policy from tree (NULL:
// the default kernel at every level).
gsw_status bfs_rows_locked(gsw_graph* g, const int32_t* sources, int32_t count, int32_t* d_levels,
                           const gsw_tree* tree, hipStream_t s);
hipStream_t pick_stream(gsw_graph* g, void* user_stream);

bool kernel_is_pull(int k);
// The kernel of base `base` and the count variant of k.
inline int kernel_with_base(int k, int base) { return base + GSW_N_BASE_KERNELS * kernel_count(k); }
void ms_release(gsw_graph* g);
void cc_release(gsw_graph* g);
size_t cc_workspace_bytes(const gsw_graph* g);


}  // namespace gsw
