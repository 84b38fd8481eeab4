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

// Per-level counters written by the expansion kernels (16 bytes).
struct LevelCtr {
  uint32_t n_next;   // vertices discovered at depth d+1
  uint32_t pad;
  unsigned long long e_next;
};

// Device state of one BFS in flight.  Bitmaps are 64-bit words, bit (v & 63)
// of word v >> 6; the last word's bits beyond n are set in `vis` so they are
// never treated as unvisited.
struct Workspace {
  int64_t n = 0, nw = 0;
  unsigned long long* vis = nullptr;     // visited
  unsigned long long* bm[3] = {};        // rotating frontier bitmaps
  int32_t* q[2] = {};                    // frontier queues
  LevelCtr* ctr = nullptr;               // ring of 4 counters
  int64_t* scan = nullptr;               // push_edge: per-entry exclusive degree scan
  int64_t* ebeg = nullptr;               // push_edge: row start per queue entry
  int64_t* bsum = nullptr;               // push_edge: per-block sums
  unsigned long long* etot = nullptr;    // push_edge: total frontier edges
  int32_t* lvl_tmp = nullptr;            // levels when the caller passes host memory
  int32_t* par_tmp = nullptr;            // parents when the caller passes host memory
  LevelCtr* h_ctr = nullptr;             // pinned host copy of one counter
  hipEvent_t ev[2] = {};
  size_t bytes = 0;
};

}  // namespace gsw

struct gsw_graph {
  int device = 0;
  int64_t n = 0, nnz = 0;
  const int64_t* offs = nullptr;  // device
  const int32_t* cols = nullptr;  // device
  int32_t* origin = nullptr;      // device, built on demand (edge_scan)
  bool owns_csr = false;
  int symmetric = 0;              // 1 when checked or vouched for
  double deg_stats[6] = {};       // min, q1, median, q3, max, std
  size_t csr_bytes = 0, origin_bytes = 0;
  gsw::Workspace ws;
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
  int32_t* parent;  // may be null
  unsigned long long* vis;
  const unsigned long long* fr;
  unsigned long long* nx;
  unsigned long long* clr;
  const int32_t* qin;
  int32_t* qout;
  LevelCtr* ctr;
  LevelCtr* ctr_clr;
  int64_t n, nw, nnz;
  uint32_t n_in;
  int32_t d;
};

gsw_status launch_init(const gsw_graph* g, int32_t* level, int32_t* parent, int32_t source,
                       hipStream_t s);
gsw_status launch_level(const gsw_graph* g, int kernel, const LevelLaunch& a, hipStream_t s);
gsw_status launch_canonical_parents(const gsw_graph* g, const int32_t* level, int32_t* parent,
                                    hipStream_t s);
gsw_status launch_build_origin(const gsw_graph* g, int32_t* origin, hipStream_t s);

gsw_status ensure_workspace(gsw_graph* g);
gsw_status ensure_origin(gsw_graph* g);
hipStream_t pick_stream(gsw_graph* g, void* user_stream);

bool kernel_is_pull(int k);

}  // namespace gsw
