// Frontier-expansion kernels for gfx950 (CDNA4, 64-lane wavefronts).
//
// Every kernel performs one whole BFS level d (Section III-A): it finds the
// unvisited vertices adjacent to depth-d vertices, gives each depth d+1 and a
// parent at depth d, and appends it to the depth-(d+1) queue.  The frontier
// bitmaps rotate over three buffers (depth d in bm[d % 3]): the bottom-up
// kernel writes the depth-(d+1) bitmap in full, the top-down kernels set the
// bits of the vertices they discover, and every level zeroes the buffer of
// the level after next.  Any kernel can therefore
// run the next level; only the queue's order and the parent choice depend on
// the kernel, never the levels.
//
// The choice of the next level's kernel is made on the device: the last
// workgroup of a level to finish sums the next frontier's size, forms the
// feature vector, applies the policy (the decision tree walked with the same
// float32-against-float64 rule as the host, a fixed kernel or a schedule),
// stores it in the level control block and posts the level's record to a
// ring in mapped host memory.  One kernel, k_level_auto, runs whichever
// variant the control block names, so the host can queue levels ahead
// without waiting for their results.  push_edge, whose prefix sum needs a
// grid-wide step, takes two of those launches: a scan whose last workgroup
// scans the block sums, then the expansion.
//
// Ownership of a new vertex v is decided by atomicOr on its 64-bit visited
// word: exactly one lane sees the bit clear and becomes the writer of v's
// level, parent and queue slot.  A plain load of the word first filters out
// vertices already visited (a stale read only costs an atomic, because bits
// are only ever set).
//
// Appends to the next frontier come in the paper's three count variants
// (Section III-A, "Variants"), part of the kernel id: WORKGROUP stages a
// workgroup's appends in LDS (one LDS atomic per wavefront and round) and
// flushes them with one global atomic per workgroup into the queue segment
// of its bin (a workgroup whose stage fills up appends further rounds
// directly, one atomic per wavefront); WAVE reserves places with one global
// atomic per wavefront and round; THREAD with one per discovering lane.
// Same-address atomics serialise, so every variant spreads its counters over
// kQueueBins segments.  Producer grids are persistent (at most kMaxGrid
// workgroups, grid-stride loops) so that few workgroups flush.
#include <hip/hip_runtime.h>

#include "gsw_device.h"
#include "gsw_internal.h"

namespace gsw {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxGrid = 1536;                   // persistent producer grids (6 per CU; measured best)
constexpr int kStage = 2048;                     // LDS-staged queue entries per workgroup
constexpr int kScanItems = 4;                    // push_edge: entries per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;   // entries per scan block
constexpr int kEdgeChunk = 1024;                 // push_edge: arcs per chunk (4 per lane)
constexpr int kEdgeWin = 512;                    // push_edge: queue entries a chunk stages in LDS
constexpr int kPullEager = 8;                    // pull: neighbours probed per lane up front
constexpr int kPullChunk = 8;                    // pull: visited words (512 vertices) per wave step
constexpr int kTreeLaneNodes = 4;                // level end: tree nodes per lane of one wave (256)

typedef unsigned long long u64;

// One level's view of the buffers.
struct Args {
  const int64_t* __restrict__ offs;
  const int32_t* __restrict__ cols;
  const int32_t* __restrict__ origin;
  const int64_t* __restrict__ roffs;   // in-arcs (the same arrays as offs/cols when symmetric)
  const int32_t* __restrict__ rcols;
  const int32_t* __restrict__ rorigin;
  const int32_t* __restrict__ head;  // kHeadArcs in-arcs of every vertex, -1 padded
  int32_t head_ranked;               // 1: ranked, not the row's first arcs
  int32_t* __restrict__ level;
  int32_t* __restrict__ parent;
  u64* vis;
  const u64* __restrict__ fr;  // depth-d frontier bitmap
  u64* nx;                     // depth-(d+1) bitmap
  u64* bclr;                   // bitmap of the level after next, zeroed here
  const int32_t* __restrict__ qin;
  const uint32_t* cin;
  int32_t* __restrict__ qout;
  uint32_t* cout;
  uint32_t* cclr;
  u64* aout;         // arc counters of the next frontier (count_arcs)
  u64* aclr;         // those of the level after next, zeroed here
  BfsCtl* ctl;       // this launch's control slot
  BfsCtl* ctl_next;  // the next launch's
  u64* done;
  int64_t n, nw, nnz;
  uint32_t n_in;
  int32_t d;
  int32_t set_nx;  // top-down kernels set the discovered vertices' bits in nx
  int32_t timed;
  int32_t grid;    // workgroups taking part in the level (grid-stride loops use it)
  int32_t cv;      // count variant (GSW_COUNT_*)
  int32_t count_arcs;
  int32_t j;       // index of this launch (posted in the level's record)
  uint32_t per;    // push_vertex, push_wave: frontier entries per workgroup
};

__host__ __device__ inline Args make_args(const BfsBase& b, int32_t j, int32_t d, uint32_t n_in, int32_t set_nx,
                                          int32_t grid) {
  Args a;
  a.offs = b.offs;
  a.cols = b.cols;
  a.origin = b.origin;
  a.roffs = b.roffs;
  a.rcols = b.rcols;
  a.rorigin = b.rorigin;
  a.head = b.head;
  a.head_ranked = b.head_ranked;
  a.level = b.level;
  a.parent = b.parent;
  a.vis = b.vis;
  a.fr = b.bm[d % 3];
  a.nx = b.bm[(d + 1) % 3];
  a.bclr = b.bm[(d + 2) % 3];
  a.qin = b.q[d & 1];
  a.cin = b.ctr + (size_t)(d & 3) * kCtrSlot;
  a.qout = b.q[(d + 1) & 1];
  a.cout = b.ctr + (size_t)((d + 1) & 3) * kCtrSlot;
  a.cclr = b.ctr + (size_t)((d + 2) & 3) * kCtrSlot;
  a.aout = b.actr + (size_t)((d + 1) & 3) * kArcSlot;
  a.aclr = b.actr + (size_t)((d + 2) & 3) * kArcSlot;
  a.ctl = b.ctl + (j & 1);
  a.ctl_next = b.ctl + ((j + 1) & 1);
  a.done = b.done;
  a.n = b.n;
  a.nw = b.nw;
  a.nnz = b.nnz;
  a.n_in = n_in;
  a.d = d;
  a.set_nx = set_nx;
  a.timed = b.timed;
  a.grid = grid;
  a.cv = 0;
  a.count_arcs = b.count_arcs;
  a.j = j;
  a.per = kBlock;
  return a;
}

__host__ __device__ inline int64_t div_up(int64_t x, int64_t y) { return (x + y - 1) / y; }

// Frontier entries per workgroup of the lane-per-vertex push kernels
// (push_vertex, push_wave): the entries spread over the launch's
// participating workgroups, at least kPushMinPer and at most kBlock per
// workgroup, so a small frontier holding hubs has them walked by many
// workgroups at once instead of by the few that a full 256 entries each
// would give it.
constexpr int64_t kPushMinPer = 16;
__host__ __device__ inline uint32_t push_per(int64_t n_in, int32_t grid_max) {
  const int64_t per = div_up(n_in, grid_max);
  return (uint32_t)(per < kPushMinPer ? kPushMinPer : (per > kBlock ? kBlock : per));
}

// Workgroups that run a level of kernel k with n_in frontier entries: a lane
// per entry for the queue-driven top-down kernels, a lane per vertex or arc
// for the all-vertex and all-arc ones, the whole launch for pull.
__host__ __device__ inline int32_t level_grid(int k, int64_t n_in, const BfsBase& b) {
  int64_t need;
  switch (kernel_base(k)) {
    case GSW_K_PULL_BITMAP: need = b.grid_max; break;
    case GSW_K_VERTEX_SCAN: need = div_up(b.n, kBlock); break;
    case GSW_K_EDGE_SCAN:
    case GSW_K_REV_EDGE_SCAN: need = div_up(b.nnz, kBlock); break;
    case GSW_K_PUSH_EDGE:  // its prefix launch, or every workgroup when fused
      need = level_first_phase(k, n_in) == 2 ? (int64_t)b.grid_max : div_up(n_in, kScanTile);
      break;
    default: need = div_up(n_in, push_per(n_in, b.grid_max)); break;
  }
  if (need < 1) need = 1;
  return (int32_t)(need < b.grid_max ? need : b.grid_max);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ u64 lanes_below(int lane) { return (1ull << lane) - 1ull; }

__device__ __forceinline__ int my_bin() { return (int)(blockIdx.x % kQueueBins); }

// Level timing: workgroup 0 of the level's first kernel stamps the
// constant-rate wall clock; the level's last workgroup to finish reads it at
// the end.  (Workgroups are dispatched in index order.)
__device__ __forceinline__ void level_begin(const Args& a) {
  if (a.timed && blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(&a.ctl->t_begin, (u64)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Zero the counter slots that the level after next appends to.
__device__ __forceinline__ void clear_ahead(const Args& a) {
  if (blockIdx.x == 0 && threadIdx.x < kQueueBins) {
    a.cclr[threadIdx.x * kCtrStride] = 0u;
    a.aclr[threadIdx.x * kArcStride] = 0ull;
  }
}

// Zero the frontier bitmap of the level after next, spread over every
// workgroup of the launch (also those that take no part in the level: the
// buffer is next written two launches later).
__device__ __forceinline__ void clear_bitmap(u64* bclr, int64_t nw) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nw; i += stride) bclr[i] = 0ull;
}

// ----------------------------------------------------------- queue input
// The input queue is the concatenation of its kQueueBins segments.
struct QueueIn {
  uint32_t pre[kQueueBins + 1];
};

// Counters of all four slots, one per lane of wave 0 (lane = slot * 8 + bin),
// loaded at the start of a launch beside the control slot, before the level
// (and so the slot it reads) is known.
__device__ __forceinline__ uint32_t counters_prefetch(const uint32_t* ctr) {
  const int t = threadIdx.x;
  return t < 4 * kQueueBins ? ctr[(size_t)(t / kQueueBins) * kCtrSlot + (t % kQueueBins) * kCtrStride] : 0u;
}

// Segment offsets of the input queue from counter slot `slot`.  Every thread
// calls it.
__device__ __forceinline__ void queue_in_load(uint32_t cpre, int slot, QueueIn& q) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int bin = lane % kQueueBins;
    const uint32_t v = (uint32_t)__shfl((int)cpre, slot * kQueueBins + bin);
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < kQueueBins; off <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)inc, off);
      if (bin >= off) inc += y;
    }
    if (lane < kQueueBins) q.pre[lane] = inc - v;
    if (lane == kQueueBins - 1) q.pre[kQueueBins] = inc;
  }
  __syncthreads();
}

__device__ __forceinline__ int32_t queue_at(const Args& a, const QueueIn& q, uint32_t i) {
  int b = 0;
#pragma unroll
  for (int k = 1; k < kQueueBins; ++k) b += i >= q.pre[k] ? 1 : 0;
  return a.qin[(int64_t)b * a.n + (i - q.pre[b])];
}

// ---------------------------------------------------------- queue output
struct alignas(16) Stage {
  int32_t buf[kStage];  // also the last workgroup's copy of the tree (16-byte nodes first)
  u64 arcs;        // out-degrees of the workgroup's discoveries (count_arcs)
  uint32_t n;      // entries reserved (may exceed kStage once it overflowed)
  uint32_t valid;  // reservations at or past this position went to global memory
  uint32_t base;
};

__device__ __forceinline__ void stage_init(Stage& s) {
  if (threadIdx.x == 0) {
    s.n = 0u;
    s.valid = kStage;
    s.arcs = 0ull;
  }
  __syncthreads();
}

// Appends the winning lanes' vertices to the next frontier in the level's
// count variant.  Called by every active lane of the wave with the same
// control flow; no workgroup barrier inside.
__device__ __forceinline__ void stage_push(Stage& s, const Args& a, bool win, int32_t v) {
  if (a.count_arcs && win) atomicAdd(&s.arcs, (u64)(a.offs[v + 1] - a.offs[v]));
  const u64 m = __ballot(win);
  if (m == 0ull) return;
  const int lane = lane_id();
  uint32_t* ctr = a.cout + my_bin() * kCtrStride;
  int32_t* seg = a.qout + (int64_t)my_bin() * a.n;
  if (a.cv == GSW_COUNT_THREAD) {  // one global atomic per discovering lane
    if (win) seg[atomicAdd(ctr, 1u)] = v;
    return;
  }
  const int leader = __ffsll((long long)m) - 1;
  const uint32_t k = (uint32_t)__popcll(m);
  const uint32_t r = (uint32_t)__popcll(m & lanes_below(lane));
  if (a.cv == GSW_COUNT_WAVE) {  // one global atomic per wavefront
    uint32_t pos = 0;
    if (lane == leader) pos = atomicAdd(ctr, k);
    pos = (uint32_t)__shfl((int)pos, leader);
    if (win) seg[pos + r] = v;
    return;
  }
  uint32_t pos = 0;
  if (lane == leader) {
    pos = atomicAdd(&s.n, k);
    if (pos + k > (uint32_t)kStage) {
      atomicMin(&s.valid, pos);
      pos = (uint32_t)kStage + atomicAdd(a.cout + my_bin() * kCtrStride, k);
    }
  }
  pos = (uint32_t)__shfl((int)pos, leader);
  if (win) {
    if (pos < (uint32_t)kStage)
      s.buf[pos + r] = v;
    else
      seg[(pos - (uint32_t)kStage) + r] = v;
  }
}

// The launch's "finished" count: each workgroup adds (1 << 40 | entries it
// appended) to its group's counter, the group's last adds the group's sums to
// the launch counter (see BfsCtl::done).
constexpr u64 kDoneOne = 1ull << 40;  // one finished workgroup (or group)
constexpr u64 kDoneMask = kDoneOne - 1ull;

// Thread 0's part of the finish count: adds (one workgroup, `appended`
// entries) and returns whether this workgroup is the launch's last; *total
// then holds every participating workgroup's appends.
__device__ __forceinline__ bool count_finished(const Args& a, uint32_t appended, u64* total) {
  const uint32_t grid = (uint32_t)a.grid;
  const u64 mine = kDoneOne | (u64)appended;
  *total = (u64)appended;
  if (grid > (unsigned)kDoneGroups) {
    const uint32_t gidx = blockIdx.x % (unsigned)kDoneGroups;
    const uint32_t in_group = grid / kDoneGroups + (gidx < grid % kDoneGroups ? 1u : 0u);
    const u64 g_old = atomicAdd(a.done + gidx * kCtrStride, mine);
    if ((g_old >> 40) != in_group - 1u) return false;
    const u64 group = (g_old + mine) & kDoneMask;
    const u64 old = atomicAdd(&a.ctl->done, kDoneOne | group);
    *total = (old & kDoneMask) + group;
    return (old >> 40) == (unsigned)kDoneGroups - 1u;
  }
  if (grid > 1u) {
    const u64 old = atomicAdd(&a.ctl->done, mine);
    *total = (old & kDoneMask) + (u64)appended;
    return (old >> 40) == grid - 1u;
  }
  return true;  // a launch of one workgroup needs no count
}

// The last workgroup resets the finish counters for the next launch.
__device__ __forceinline__ void reset_finished(const Args& a) {
  if (threadIdx.x < kDoneGroups) a.done[threadIdx.x * kCtrStride] = 0ull;
  if (threadIdx.x == 0) a.ctl->done = 0ull;
}

// Sum over the queue bins (or arc bins) of a level's 32-bit (64-bit)
// counters, read at the device's coherence point by the launch's last
// workgroup once every other one has counted itself finished.
__device__ __forceinline__ u64 sum_bins32(uint32_t* c) {
  u64 t = 0ull;
#pragma unroll
  for (int b = 0; b < kQueueBins; ++b) t += (u64)atomicAdd(c + b * kCtrStride, 0u);
  return t;
}
__device__ __forceinline__ u64 sum_bins64(u64* c) {
  u64 t = 0ull;
#pragma unroll
  for (int b = 0; b < kQueueBins; ++b) t += atomicAdd(c + b * kArcStride, 0ull);
  return t;
}

// The staged entries' flush and the finish count in one step: thread 0 issues the queue
// reservation and the count together (the level's end needs only the
// count; the entries are read by the next launch).  In the WAVE and THREAD
// variants the workgroup's appends went to the bin counters already (their
// atomics returned before the barrier), so the count carries none and the
// last workgroup sums the bin counters instead.  With count_arcs the
// workgroup's arc sum goes to its bin's arc counter, acknowledged before
// the finish count.  Every thread calls it; returns (in every thread)
// whether this is the launch's last workgroup, and *total holds the next
// frontier's size there.
__device__ __forceinline__ bool stage_flush_finish(Stage& s, const Args& a, u64* total) {
  __shared__ u64 s_total;
  __shared__ uint32_t s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t cnt = s.n < s.valid ? s.n : s.valid;
    s.valid = cnt;
    const uint32_t base = cnt ? atomicAdd(a.cout + my_bin() * kCtrStride, cnt) : 0u;
    if (a.count_arcs && s.arcs) {
      atomicAdd(a.aout + my_bin() * kArcStride, s.arcs);
      __builtin_amdgcn_s_waitcnt(0);  // performed before this workgroup counts itself finished
    }
    u64 tot = 0ull;
    const bool last = count_finished(a, s.n, &tot);
    if (last && a.cv != GSW_COUNT_WORKGROUP) tot = sum_bins32(a.cout);
    s_last = last ? 1u : 0u;
    s_total = tot;
    s.base = base;
  }
  __syncthreads();
  const uint32_t cnt = s.valid;
  int32_t* dst = a.qout + (int64_t)my_bin() * a.n + s.base;
  for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) dst[i] = s.buf[i];
  *total = s_total;
  const bool last = s_last != 0u;
  if (last) reset_finished(a);
  return last;
}

// True for the one lane (device-wide) that first sets v's visited bit.
__device__ __forceinline__ bool claim(u64* vis, int32_t v) {
  const u64 bit = 1ull << (v & 63);
  u64* w = vis + (v >> 6);
  if (*w & bit) return false;
  return (atomicOr(w, bit) & bit) == 0ull;
}

__device__ __forceinline__ void settle(const Args& a, int32_t v, int32_t u) {
  a.level[v] = a.d + 1;
  if (a.parent) a.parent[v] = u;
  if (a.set_nx) atomicOr(a.nx + (v >> 6), 1ull << (v & 63));
}

// Arcs a lane keeps in flight: the column loads, visited-word loads and
// claiming atomics of kBatch arcs are issued before any result is used, so a
// lane walking a short row pays the memory latency once per batch instead of
// once per arc.
constexpr int kBatch = 4;

// Visits the pairs (v[q], u[q]) with v[q] >= 0.  Every active lane of the
// wave calls it with the same control flow.
__device__ __forceinline__ void visit_batch(Stage& s, const Args& a, const int32_t (&v)[kBatch],
                                            const int32_t (&u)[kBatch]) {
  u64 w[kBatch], old[kBatch];
#pragma unroll
  for (int q = 0; q < kBatch; ++q) w[q] = v[q] >= 0 ? a.vis[v[q] >> 6] : ~0ull;
#pragma unroll
  for (int q = 0; q < kBatch; ++q) {
    const u64 bit = 1ull << (v[q] & 63);
    old[q] = (w[q] & bit) ? bit : atomicOr(a.vis + (v[q] >> 6), bit);
  }
#pragma unroll
  for (int q = 0; q < kBatch; ++q) {
    const bool win = v[q] >= 0 && !(old[q] & (1ull << (v[q] & 63)));
    if (win) settle(a, v[q], u[q]);
    stage_push(s, a, win, v[q]);
  }
}

// Arcs e0, e0 + step, ... below e1 of row u.
__device__ __forceinline__ void visit_row(Stage& s, const Args& a, int64_t e0, int64_t e1, int64_t step,
                                          int32_t u) {
  const int32_t us[kBatch] = {u, u, u, u};
  for (int64_t e = e0; e < e1; e += kBatch * step) {
    int32_t v[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) v[q] = e + q * step < e1 ? a.cols[e + q * step] : -1;
    visit_batch(s, a, v, us);
  }
}

// ------------------------------------------------- next-kernel choice
// Child of tree node nd (packed as tree_node_pack) for a level whose next
// frontier has nf vertices and which has discovered disc vertices through
// the next depth, or, for a leaf, -(leaf kernel + 2) (-1: undecided leaf).
// The device copy of the tree is specialised to the graph on upload: its
// splits compare one of those two counts with an integer threshold that
// decides exactly as the host's float comparison of the feature does.
__device__ __forceinline__ int32_t tree_step(u64 nd, int32_t thr, int32_t nf, int32_t disc) {
  const int left = (int)(int16_t)(uint16_t)(nd & 0xffffull);
  if (left == -1) return -((int32_t)((nd >> 40) & 0xffull) - 1) - 2;
  const int right = (int)(int16_t)(uint16_t)((nd >> 16) & 0xffffull);
  const int32_t c = ((nd >> 32) & 1ull) ? disc : nf;
  return c <= thr ? left : right;
}

// Kernel for a tree leaf (-1: undecided, repeat prev, the previous level's
// kernel) or any other policy's pick, after the fixup every choice gets:
// the edge lists need their origin arrays.
__device__ __forceinline__ int choose_leaf(const BfsPolicy& p, int k, int prev, int32_t* flags) {
  *flags = 0;
  if (k < 0) {
    k = prev;
    *flags |= 1;
  }
  if (kernel_base(k) == GSW_K_EDGE_SCAN && !p.has_origin) k = GSW_DEFAULT_KERNEL;
  if (kernel_base(k) == GSW_K_REV_EDGE_SCAN && !p.has_rorigin) k = GSW_DEFAULT_KERNEL;
  return k;
}

// Kernel for level d (d >= 1) with frontier nf and nf + earlier discoveries
// = disc; prev = kernel of level d-1.  The same rules as the host's choice;
// a tree is walked here from global memory one node at a time (the level's
// end evaluates trees that fit its LDS table in parallel instead).
__device__ __forceinline__ int choose_next(const BfsPolicy& p, int32_t d, long long nf, long long disc, int prev,
                                           int32_t* flags) {
  int k = GSW_DEFAULT_KERNEL;
  if (p.policy == GSW_POLICY_FIXED) {
    k = p.fixed;
  } else if (p.policy == GSW_POLICY_SCHEDULE) {
    k = p.sched[d < p.sched_len ? d : p.sched_len - 1];
  } else {
    int32_t x = 0;
    do {
      x = tree_step(p.t_node[x], p.t_thr[x], (int32_t)nf, (int32_t)disc);
    } while (x >= 0);
    k = x == -1 ? -1 : -x - 2;
  }
  return choose_leaf(p, k, prev, flags);
}

// True (in every thread) in the last workgroup of the launch to get here,
// for a launch that appends nothing (push_edge's prefix launch).  Called by
// every thread of every participating workgroup.
__device__ __forceinline__ bool launch_last(const Args& a) {
  __shared__ uint32_t s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 none = 0ull;
    s_last = count_finished(a, 0u, &none) ? 1u : 0u;
  }
  __syncthreads();
  const bool last = s_last != 0u;
  if (last) reset_finished(a);
  return last;
}

// Tree nodes of a specialised tree of up to 64 * kTreeLaneNodes nodes, in
// wave 0's registers (node i on lane i % 64, slot i / 64), loaded by every
// workgroup before it counts itself finished so that the last one has them.
struct TreeLanes {
  u64 nd[kTreeLaneNodes];
  int32_t thr[kTreeLaneNodes];
};

__device__ __forceinline__ TreeLanes tree_prefetch(const BfsPolicy& p) {
  TreeLanes t;
  const int tid = threadIdx.x;
  const bool wave = p.policy == GSW_POLICY_TREE && p.t_nodes <= 64 * kTreeLaneNodes;
#pragma unroll
  for (int q = 0; q < kTreeLaneNodes; ++q) {
    const int i = tid + 64 * q;
    t.nd[q] = 0ull;
    t.thr[q] = 0;
    if (wave && tid < 64 && i < p.t_nodes) {
      t.nd[q] = p.t_node[i];
      t.thr[q] = p.t_thr[i];
    }
  }
  return t;
}

// End of a level, called by every thread of every workgroup of the level's
// last launch after stage_flush_finish: the last workgroup to finish, which
// has the next frontier's size from the finish count, picks the next
// kernel, posts the level's record to the host ring and writes the next
// launch's control slot.  The device copy of a tree
// is specialised to the graph (only splits on the level features remain):
// when it has at most 64 * kTreeLaneNodes nodes, wave 0 of every workgroup
// loads them (node i on lane i % 64) before the count, and the last one
// evaluates every node's split at once and follows the children with lane
// shuffles.  A larger tree is
// evaluated the same way by the whole last workgroup into a child table in
// `lds` (lds_bytes of LDS free by now, the flushed append stage; 4 bytes per
// node); one beyond that is walked from global memory.
__device__ __forceinline__ void level_end(const Args& a, const BfsBase* base, const BfsPolicy& p, u64* ring,
                                          int k_run, void* lds, int lds_bytes, const TreeLanes& tl, bool last,
                                          u64 total) {
  const int tid = threadIdx.x;
  const bool tree = p.policy == GSW_POLICY_TREE;
  const bool tree_wave = tree && p.t_nodes <= 64 * kTreeLaneNodes;
  const bool tree_par = tree && !tree_wave && (long long)p.t_nodes * 4 <= (long long)lds_bytes;
  if (!last) return;
  BfsCtl* c = a.ctl;
  int32_t* l_next = reinterpret_cast<int32_t*>(lds);
  u64 nd0 = 0ull, nd1 = 0ull;
  int32_t th0 = 0, th1 = 0;
  if (tree_par) {
    if (tid < p.t_nodes) {
      nd0 = p.t_node[tid];
      th0 = p.t_thr[tid];
    }
    if (tid + kBlock < p.t_nodes) {
      nd1 = p.t_node[tid + kBlock];
      th1 = p.t_thr[tid + kBlock];
    }
  } else if (tid >= 64) {
    return;  // wave 0 finishes the level
  }
  const long long disc0 = c->disc;
  const uint32_t nn = (uint32_t)total;  // the next frontier: every workgroup's appends
  if (tree_par) {
    const long long nd = disc0 + (long long)nn;
    if (nn > 0) {
      const int32_t cf = (int32_t)nn, cd = (int32_t)nd;
      if (tid < p.t_nodes) l_next[tid] = tree_step(nd0, th0, cf, cd);
      if (tid + kBlock < p.t_nodes) l_next[tid + kBlock] = tree_step(nd1, th1, cf, cd);
      for (int i = tid + 2 * kBlock; i < p.t_nodes; i += kBlock) l_next[i] = tree_step(p.t_node[i], p.t_thr[i], cf, cd);
    }
    __syncthreads();
    if (tid >= 64) return;
  }
  const long long ndisc = disc0 + (long long)nn;
  int32_t nflags = 0;
  int32_t next = kCtlDone;
  if (nn > 0) {
    if (tree_wave) {
      const int slots = (p.t_nodes + 63) >> 6;
      int32_t ch[kTreeLaneNodes];
#pragma unroll
      for (int q = 0; q < kTreeLaneNodes; ++q)
        ch[q] = q < slots ? tree_step(tl.nd[q], tl.thr[q], (int32_t)nn, (int32_t)ndisc) : 0;
      // follow the children from the root: the node index is uniform, so each
      // step is a register read across lanes
      int32_t x = __builtin_amdgcn_readlane(ch[0], 0);
      while (x >= 0) {
        const int slot = x >> 6;
        int32_t c = ch[0];
#pragma unroll
        for (int q = 1; q < kTreeLaneNodes; ++q) c = slot == q ? ch[q] : c;
        x = __builtin_amdgcn_readlane(c, x & 63);
      }
      next = choose_leaf(p, x == -1 ? -1 : -x - 2, k_run, &nflags);
    } else if (tree_par) {
      int32_t x = l_next[0];
      while (x >= 0) x = l_next[x];
      next = choose_leaf(p, x == -1 ? -1 : -x - 2, k_run, &nflags);
    } else {
      next = choose_next(p, a.d + 1, (long long)nn, ndisc, k_run, &nflags);
    }
  }
  if (tid != 0) return;
  u64 ticks = 0ull;
  if (a.timed) {
    const u64 t0 = __hip_atomic_load(&c->t_begin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 t1 = (u64)wall_clock64();
    ticks = t1 > t0 ? t1 - t0 : 0ull;
  }
  const int32_t d = a.d;
  const long long nf = c->nf, disc = disc0;
  const long long ef_next = a.count_arcs ? (long long)sum_bins64(a.aout) : -1;
  u64* r = ring + (size_t)(d % kBfsRing) * kBfsRec;
  const u64 tag = rec_tag(d);
  const u64 rec[kBfsRecWords] = {(u64)k_run, (u64)c->flags, (u64)nf, (u64)disc, (u64)nn, ticks & kRecValueMask,
                              (u64)(next + 1), (u64)(c->ef + 1) & kRecValueMask, (u64)a.j};
#pragma unroll
  for (int i = 0; i < kBfsRecWords; ++i)
    __hip_atomic_store(r + i, tag | rec[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  BfsCtl* cn = a.ctl_next;
  cn->d = d + 1;
  cn->kernel = next;
  cn->prev = k_run;
  cn->flags = nflags;
  cn->nf = (long long)nn;
  cn->disc = ndisc;
  cn->done = 0ull;
  cn->phase = level_first_phase(next, (int64_t)nn);
  cn->t_begin = 0ull;
  cn->grid = next >= 0 ? level_grid(next, (int64_t)nn, *base) : 1;
  cn->etot = 0;
  cn->ef = ef_next;
  cn->clean = 0;
}

// ---------------------------------------------------------------- init
// Levels and parents, visited (source, padding and -- on a symmetric graph --
// degree-0 vertices, which can never be reached), the three frontier
// bitmaps (depth 0 = the source), the depth-0 queue, the counter ring and
// the control block for level 0.
__global__ void __launch_bounds__(kBlock) k_init(BfsBase b, const u64* __restrict__ iso, int32_t s,
                                                 int32_t k0, int32_t flags0) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // 16-byte stores where both arrays allow them; every element is written by
  // exactly one thread, the source's with its own values
  const bool vec = ((uintptr_t)b.level & 15u) == 0u && ((uintptr_t)b.parent & 15u) == 0u;
  const int64_t n4 = vec ? b.n >> 2 : 0;
  int4* l4 = reinterpret_cast<int4*>(b.level);
  int4* p4 = reinterpret_cast<int4*>(b.parent);
  for (int64_t i = gid; i < n4; i += stride) {
    int4 lv = make_int4(-1, -1, -1, -1), pv = lv;
    if (i == (int64_t)(s >> 2)) {
      const int k = s & 3;
      lv.x = k == 0 ? 0 : lv.x; lv.y = k == 1 ? 0 : lv.y; lv.z = k == 2 ? 0 : lv.z; lv.w = k == 3 ? 0 : lv.w;
      pv.x = k == 0 ? s : pv.x; pv.y = k == 1 ? s : pv.y; pv.z = k == 2 ? s : pv.z; pv.w = k == 3 ? s : pv.w;
    }
    l4[i] = lv;
    if (b.parent) p4[i] = pv;
  }
  for (int64_t i = 4 * n4 + gid; i < b.n; i += stride) {
    b.level[i] = i == s ? 0 : -1;
    if (b.parent) b.parent[i] = i == s ? s : -1;
  }
  const int64_t sw = s >> 6;
  const u64 sbit = 1ull << (s & 63);
  const int tail = (int)(b.n & 63);
  for (int64_t w = gid; w < b.nw; w += stride) {
    u64 pad = 0ull;
    if (w == b.nw - 1 && tail) pad = ~0ull << tail;  // bits beyond n count as visited
    const u64 here = w == sw ? sbit : 0ull;
    b.vis[w] = here | pad | (iso ? iso[w] : 0ull);
    b.bm[0][w] = here;
    b.bm[1][w] = 0ull;
    b.bm[2][w] = 0ull;
  }
  if (gid == 0) {
    b.q[0][0] = s;  // segment 0 of the depth-0 queue
    BfsCtl* c = b.ctl;
    c->d = 0;
    c->kernel = k0;
    c->prev = GSW_DEFAULT_KERNEL;
    c->flags = flags0;
    c->nf = 1;
    c->disc = 1;
    c->done = 0ull;
    c->phase = level_first_phase(k0, 1);
    c->t_begin = 0ull;
    c->grid = level_grid(k0, 1, b);
    c->etot = 0;
    c->ef = b.count_arcs ? (long long)(b.offs[s + 1] - b.offs[s]) : -1;
    c->clean = 1;
  }
  if (gid < 4 * kCtrSlot) b.ctr[gid] = gid == 0 ? 1u : 0u;
  if (gid < 4 * kArcSlot) b.actr[gid] = 0ull;
  if (gid < kDoneGroups) b.done[gid * kCtrStride] = 0ull;
}

// ------------------------------------------------------------ long rows
// The queue- and vertex-driven variants give a frontier row to one lane (or
// to W lanes).  A row that would take that walk more than kLongTrips trips is
// set aside instead and, at the end of the round, walked by the whole
// workgroup: its kBlock lanes spread over the arcs of every set-aside row
// (an LDS prefix sum over their lengths, then a binary search per arc).  A
// hub in the frontier then costs a workgroup's pass over its arcs rather
// than one lane's serial walk; rows within the limit are walked as the
// variant defines.
constexpr int kLongTrips = 32;

struct LongRows {
  int64_t beg[kBlock];
  int64_t pre[kBlock + 1];  // row lengths, then their exclusive prefix sum
  int64_t wsum[kWaves];
  int32_t u[kBlock];
  uint32_t n[3];  // set-aside count of round r in n[r % 3]
};

// Every thread of the workgroup calls it once before the first round.
__device__ __forceinline__ void long_init(LongRows& L) {
  if (threadIdx.x < 3) L.n[threadIdx.x] = 0u;
  __syncthreads();
}

// Round r's counter is n[r % 3]; thread 0 zeroes n[(r + 1) % 3] at the start
// of round r.  Its last readers (round r - 2) passed round r - 1's barrier
// before thread 0 did, and its next writers (round r + 1) come after round
// r's barrier, so no other barrier is needed when nothing was set aside.
__device__ __forceinline__ void long_round_begin(LongRows& L, uint32_t r) {
  if (threadIdx.x == 0) L.n[(r + 1) % 3] = 0u;
}

// Sets row [beg, end) of u aside when it is longer than limit arcs; each
// thread sets aside at most one row per round.
__device__ __forceinline__ bool long_defer(LongRows& L, uint32_t r, int32_t u, int64_t beg, int64_t end,
                                           int64_t limit) {
  if (end - beg <= limit) return false;
  const uint32_t k = atomicAdd(&L.n[r % 3], 1u);
  L.u[k] = u;
  L.beg[k] = beg;
  L.pre[k] = end - beg;
  return true;
}

// Walks round r's set-aside rows with the whole workgroup.  Every thread
// calls it (uniform control flow).
__device__ __forceinline__ void long_walk(LongRows& L, uint32_t r, Stage& st, const Args& a) {
  __syncthreads();
  const uint32_t n = L.n[r % 3];
  if (n == 0u) return;
  const int t = threadIdx.x;
  const int lane = lane_id();
  const int wave = t >> 6;
  const int64_t len = (uint32_t)t < n ? L.pre[t] : 0;
  int64_t inc = len;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) L.wsum[wave] = inc;
  __syncthreads();  // every length is read before the prefix sums overwrite them
  int64_t below = 0, total = 0;
  for (int w = 0; w < kWaves; ++w) {
    below += w < wave ? L.wsum[w] : 0;
    total += L.wsum[w];
  }
  if ((uint32_t)t < n) L.pre[t + 1] = below + inc;
  if (t == 0) L.pre[0] = 0;
  __syncthreads();
  for (int64_t e0 = t; e0 < total; e0 += kBatch * kBlock) {
    int32_t v[kBatch], u[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int64_t e = e0 + (int64_t)q * kBlock;
      v[q] = -1;
      u[q] = 0;
      if (e < total) {
        uint32_t lo = 0, hi = n;  // last row whose prefix is <= e
        while (hi - lo > 1u) {
          const uint32_t mid = (lo + hi) >> 1;
          if (L.pre[mid] <= e) lo = mid; else hi = mid;
        }
        v[q] = a.cols[L.beg[lo] + (e - L.pre[lo])];
        u[q] = L.u[lo];
      }
    }
    visit_batch(st, a, v, u);
  }
  __syncthreads();  // the rows are read before the next round sets new ones aside
}

// ------------------------------------------------- push_vertex (lane / vertex)
__device__ __forceinline__ void body_push_vertex(const Args& a, Stage& st, const QueueIn& qi, LongRows& L) {
  const uint32_t stride = (uint32_t)a.grid * a.per;
  long_init(L);
  uint32_t r = 0;
  for (uint32_t base = blockIdx.x * a.per; base < a.n_in; base += stride, ++r) {
    long_round_begin(L, r);
    const uint32_t i = base + threadIdx.x;
    int32_t u = 0;
    int64_t beg = 0, end = 0;
    if (threadIdx.x < a.per && i < a.n_in) {
      u = queue_at(a, qi, i);
      beg = a.offs[u];
      end = a.offs[u + 1];
      if (long_defer(L, r, u, beg, end, kLongTrips)) end = beg;
    }
    visit_row(st, a, beg, end, 1, u);
    long_walk(L, r, st, a);
  }
}

// ------------------------------------- push_wave<W> (W lanes / vertex, W vertices / group)
// The paper's virtual warps (Section III-A, vertex push warp): a group of W
// lanes takes W frontier vertices and walks their rows one after another,
// the W lanes striding over each row together.
template <int W>
__device__ __forceinline__ void body_push_wave(const Args& a, Stage& st, const QueueIn& qi, LongRows& L) {
  const int lane = lane_id();
  const int sub = lane & (W - 1);
  const int first = lane & ~(W - 1);
  const uint32_t stride = (uint32_t)a.grid * a.per;
  long_init(L);
  uint32_t r = 0;
  for (uint32_t base = blockIdx.x * a.per; base < a.n_in; base += stride, ++r) {
    long_round_begin(L, r);
    const uint32_t i = base + threadIdx.x;  // this lane's own entry
    int32_t u = 0;
    int64_t beg = 0, end = 0;
    if (threadIdx.x < a.per && i < a.n_in) {
      u = queue_at(a, qi, i);
      beg = a.offs[u];
      end = a.offs[u + 1];
      if (long_defer(L, r, u, beg, end, (int64_t)kLongTrips * W)) end = beg;
    }
    for (int j = 0; j < W; ++j) {
      const int src = first + j;
      const int32_t uj = __shfl(u, src);
      const int64_t bj = __shfl(beg, src);
      const int64_t ej = __shfl(end, src);
      visit_row(st, a, bj + sub, ej, W, uj);
    }
    long_walk(L, r, st, a);
  }
}

// ------------------------------------------------ push_edge (lane / frontier arc)
// Section III-A, edge push: every arc leaving the frontier gets a lane.  The
// frontier's arcs are numbered by an exclusive prefix sum of the queue
// entries' degrees, computed by the level's first launch (block-local scans
// of kScanTile entries; the launch's last workgroup scans the block sums).
// The second launch splits the arc range evenly over its workgroups; each
// finds the entry holding its first arc with a cooperative search, then
// walks its range in chunks of kEdgeChunk arcs, staging the entries a chunk
// spans in LDS so that each lane finds its arc's entry there.
struct EdgeScan {
  const int64_t* scan;
  const int64_t* ebeg;
  const int64_t* bsum;
};

// Arc offset of queue entry i.
__device__ __forceinline__ int64_t gscan(const EdgeScan& es, int64_t i) {
  return es.scan[i] + es.bsum[i / kScanTile];
}

// Last entry i in [lo, hi] with gscan(i) <= t, given gscan(lo) <= t; one lane.
__device__ __forceinline__ int64_t find_entry(const EdgeScan& es, int64_t lo, int64_t hi, int64_t t) {
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (gscan(es, mid) <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct EdgeLds {
  int64_t start[kEdgeWin];  // arc offset of each staged entry
  int64_t beg[kEdgeWin];    // its row start
  int32_t u[kEdgeWin];      // its vertex
  int64_t wsum[kWaves];
  int32_t cnt[kWaves];
};
static_assert(kEdgeFuse <= kEdgeWin && kEdgeFuse <= 2 * kBlock, "fused push_edge stages every entry");

// Number of workgroup lanes with pred set (every thread calls it).
__device__ __forceinline__ int block_count(bool pred, int32_t* cnt) {
  const u64 m = __ballot(pred);
  if (lane_id() == 0) cnt[threadIdx.x >> 6] = __popcll(m);
  __syncthreads();
  int c = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) c += cnt[w];
  __syncthreads();  // cnt is rewritten by the next call
  return c;
}

// The same search by the whole workgroup: each round probes kBlock evenly
// spaced entries at once and keeps the interval between the last probe at
// or below t and the next one (two rounds up to 65536 entries).
__device__ __forceinline__ int64_t find_entry_block(const EdgeScan& es, int64_t lo, int64_t hi, int64_t t,
                                                    int32_t* cnt) {
  while (hi > lo) {
    const int64_t step = (hi - lo + kBlock) / kBlock;  // ceil((hi - lo + 1) / kBlock)
    const int64_t q = lo + (int64_t)threadIdx.x * step;
    const int c = block_count(q <= hi && gscan(es, q) <= t, cnt);  // probes true form a prefix, c >= 1
    lo += (int64_t)(c - 1) * step;
    hi = lo + step - 1 < hi ? lo + step - 1 : hi;
  }
  return lo;
}

// First launch: degree and row start per entry, block-local exclusive scan,
// block sums.  Scan blocks are spread over the launch's workgroups.
__device__ __forceinline__ void body_edge_prefix(const Args& a, const QueueIn& qi, const BfsBase& b,
                                                 int64_t* wsum) {
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t nb = div_up((int64_t)a.n_in, kScanTile);
  for (int64_t blk = blockIdx.x; blk < nb; blk += a.grid) {
    const int64_t base = blk * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t deg[kScanItems];
    int64_t tot = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t i = base + k;
      deg[k] = 0;
      if (i < a.n_in) {
        const int32_t u = queue_at(a, qi, (uint32_t)i);
        const int64_t rb = a.offs[u];
        b.ebeg[i] = rb;
        deg[k] = a.offs[u + 1] - rb;
      }
      tot += deg[k];
    }
    int64_t inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int64_t run = inc - tot;
    for (int k = 0; k < wid; ++k) run += wsum[k];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t i = base + k;
      if (i < a.n_in) b.scan[i] = run;
      run += deg[k];
    }
    if (threadIdx.x == kBlock - 1) {
      // read by this launch's last workgroup, maybe on another XCD: a
      // device-coherent store, complete before this workgroup counts itself
      __hip_atomic_store(b.bsum + blk, run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();  // wsum is rewritten by the next block
  }
}

// End of the first launch: its last workgroup turns the block sums into
// their exclusive prefix, stores the arc total and names the second launch.
__device__ __forceinline__ void edge_prefix_end(const Args& a, const BfsBase& b, int64_t* wsum) {
  if (!launch_last(a)) return;
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t nb = div_up((int64_t)a.n_in, kScanTile);
  const int64_t per = div_up(nb, kBlock);
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  int64_t tot = 0;
  for (int64_t i = lo; i < hi; ++i)
    tot += __hip_atomic_load(b.bsum + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int64_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t run = inc - tot;
  for (int k = 0; k < wid; ++k) run += wsum[k];
  for (int64_t i = lo; i < hi; ++i) {
    const int64_t x = __hip_atomic_load(b.bsum + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b.bsum[i] = run;
    run += x;
  }
  if (threadIdx.x == kBlock - 1) {
    const BfsCtl* c = a.ctl;
    BfsCtl* cn = a.ctl_next;
    const int64_t chunks = div_up(run, kEdgeChunk);
    cn->d = c->d;
    cn->kernel = c->kernel;
    cn->prev = c->prev;
    cn->flags = c->flags;
    cn->nf = c->nf;
    cn->disc = c->disc;
    cn->done = 0ull;
    cn->phase = 1;
    cn->t_begin = __hip_atomic_load(&c->t_begin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cn->grid = (int32_t)(chunks < 1 ? 1 : (chunks < b.grid_max ? chunks : b.grid_max));
    cn->etot = run;
    cn->ef = c->ef;
    cn->clean = c->clean;
  }
}

// Second launch: workgroup w takes arcs [etot*w/G, etot*(w+1)/G).
__device__ __forceinline__ void body_edge_expand(const Args& a, Stage& st, const QueueIn& qi, const EdgeScan& es,
                                                 EdgeLds& L, int64_t total) {
  const int64_t G = a.grid;
  const int64_t e_lo = total * (int64_t)blockIdx.x / G;
  const int64_t e_hi = total * ((int64_t)blockIdx.x + 1) / G;
  if (e_lo >= e_hi) return;
  const int64_t last = (int64_t)a.n_in - 1;
  const int tid = threadIdx.x;
  int64_t i0 = find_entry_block(es, 0, last, e_lo, L.cnt);
  for (int64_t c0 = e_lo; c0 < e_hi; c0 += kEdgeChunk) {
    const int64_t c1 = (c0 + kEdgeChunk < e_hi ? c0 + kEdgeChunk : e_hi) - 1;
    // entries from i0 whose arcs start by c1: m of them (a prefix), staged
    // when they fit the window
    int m = 0;
    for (int g = 0; g < kEdgeWin; g += kBlock) {
      const int64_t i = i0 + g + tid;
      const int64_t sv = i <= last ? gscan(es, i) : INT64_MAX;
      L.start[g + tid] = sv;
      const int c = block_count(sv <= c1, L.cnt);
      m += c;
      if (c < kBlock) break;
    }
    const bool staged = m < kEdgeWin;
    if (staged) {
      for (int k = tid; k < m; k += kBlock) {
        L.beg[k] = es.ebeg[i0 + k];
        L.u[k] = queue_at(a, qi, (uint32_t)(i0 + k));
      }
    }
    __syncthreads();
    int32_t v[kBatch], u[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int64_t t = c0 + (int64_t)j * kBlock + tid;
      v[j] = -1;
      u[j] = 0;
      if (t <= c1) {
        if (staged) {
          int lo = 0, hi = m - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.start[mid] <= t) lo = mid; else hi = mid - 1;
          }
          v[j] = a.cols[L.beg[lo] + (t - L.start[lo])];
          u[j] = L.u[lo];
        } else {
          const int64_t k = find_entry(es, i0, last, t);
          v[j] = a.cols[es.ebeg[k] + (t - gscan(es, k))];
          u[j] = queue_at(a, qi, (uint32_t)k);
        }
      }
    }
    visit_batch(st, a, v, u);
    __syncthreads();  // the window is rewritten by the next chunk
    if (c1 + 1 < e_hi) {
      // the entry holding arc c1 + 1 is at or after the one holding c1
      i0 = staged ? i0 + m - 1 : find_entry_block(es, i0, last, c1 + 1, L.cnt);
    }
  }
}

// Both launches in one, for at most kEdgeFuse entries: every workgroup of
// the launch reads the whole queue and scans its degrees in LDS, so each
// knows the arc total and needs no search; workgroups beyond the number
// the total calls for leave (returns false) and a.grid becomes that number.
__device__ __forceinline__ bool body_edge_fused(Args& a, Stage& st, const QueueIn& qi, EdgeLds& L) {
  int64_t* wsum = L.wsum;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  const int n_in = (int)(a.n_in < (uint32_t)kEdgeFuse ? a.n_in : (uint32_t)kEdgeFuse);  // == a.n_in
  int64_t deg[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int i = 2 * tid + q;
    deg[q] = 0;
    if (i < n_in) {
      const int32_t u = queue_at(a, qi, (uint32_t)i);
      const int64_t rb = a.offs[u];
      deg[q] = a.offs[u + 1] - rb;
      L.u[i] = u;
      L.beg[i] = rb;
    }
  }
  const int64_t tot = deg[0] + deg[1];
  int64_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t run = inc - tot, total = 0;
  for (int w = 0; w < kWaves; ++w) {
    run += w < wid ? wsum[w] : 0;
    total += wsum[w];
  }
  if (2 * tid < n_in) L.start[2 * tid] = run;
  if (2 * tid + 1 < n_in) L.start[2 * tid + 1] = run + deg[0];
  __syncthreads();
  const int64_t chunks = div_up(total, kEdgeChunk);
  const int64_t G = chunks < 1 ? 1 : (chunks < a.grid ? chunks : a.grid);
  if ((int64_t)blockIdx.x >= G) return false;
  a.grid = (int32_t)G;
  const int64_t e_lo = total * (int64_t)blockIdx.x / G;
  const int64_t e_hi = total * ((int64_t)blockIdx.x + 1) / G;
  for (int64_t c0 = e_lo; c0 < e_hi; c0 += kEdgeChunk) {
    int32_t v[kBatch], u[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int64_t t = c0 + (int64_t)j * kBlock + tid;
      v[j] = -1;
      u[j] = 0;
      if (t < e_hi) {
        int lo = 0, hi = n_in - 1;  // last entry whose arcs start at or before t
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (L.start[mid] <= t) lo = mid; else hi = mid - 1;
        }
        v[j] = a.cols[L.beg[lo] + (t - L.start[lo])];
        u[j] = L.u[lo];
      }
    }
    visit_batch(st, a, v, u);
  }
  return true;
}

// ------------------------------------------ pull_bitmap (wave / 512 vertices)
// A wave takes kPullChunk visited words (512 vertices) at a time and puts
// their unvisited vertices on its lanes, 64 per round, in vertex order: a
// level with few unvisited vertices costs one short round per 512 vertices
// instead of one dependent load chain per 64.  Each lane looks for an
// in-neighbour of its vertex (a u with an arc u -> v; on a symmetric graph
// any neighbour) in the frontier bitmap, in row order, and stops at the
// first one (Section III-A, vertex pull).  Phase 1: every lane probes the
// first kHeadArcs neighbours of its row from the dense head copy (the lanes'
// records are consecutive, so most vertices, which find a frontier
// neighbour among their first few, never touch their CSR row), then, if
// still unresolved, the next kPullEager with independent loads (many misses
// in flight instead of one dependent chain).  Phase 2: rows that are longer
// and still unresolved are scanned by the whole wavefront, 64 neighbours per
// step, one row at a time -- a high-degree row does not stall its wave for
// deg(v) dependent steps.  Discoveries are ORed into the wave's own LDS copy
// of its words' next-frontier bits; every word of the depth-(d+1) bitmap is
// written.
__device__ __forceinline__ u64 readlane64(u64 x, int i) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), i);
  return ((u64)hi << 32) | lo;
}


// The chunk's k-th unvisited vertex (k in compacted order) and its word and
// bit within the chunk.
struct PullV {
  int32_t v;
  int kw, bit;
  bool mine;
};

__device__ __forceinline__ PullV pull_vertex(int k, int total, int64_t w0, const u64 (&todo)[kPullChunk],
                                             const int (&first)[kPullChunk]) {
  PullV p;
  p.mine = k < total;
  int kw = 0;
#pragma unroll
  for (int i = 1; i < kPullChunk; ++i) kw += k >= first[i] ? 1 : 0;
  u64 t = 0ull;
  int f0 = 0;
#pragma unroll
  for (int i = 0; i < kPullChunk; ++i)
    if (i == kw) {
      t = todo[i];
      f0 = first[i];
    }
  p.kw = kw;
  p.bit = p.mine ? nth_set_bit(t, k - f0) : 0;
  p.v = (int32_t)((w0 + kw) * 64 + p.bit);
  return p;
}

// First in-neighbour of p.v among its head arcs that is in the frontier
// (-1: none); *more: the row goes on past them.
__device__ __forceinline__ int32_t pull_head_hit(const Args& a, const PullV& p, const int4 (&h)[kHeadArcs / 4],
                                                 bool* more) {
  int32_t hu[kHeadArcs];
#pragma unroll
  for (int r = 0; r < kHeadArcs / 4; ++r) {
    hu[4 * r] = h[r].x;
    hu[4 * r + 1] = h[r].y;
    hu[4 * r + 2] = h[r].z;
    hu[4 * r + 3] = h[r].w;
  }
  u64 hw[kHeadArcs];
#pragma unroll
  for (int q = 0; q < kHeadArcs; ++q) hw[q] = hu[q] >= 0 ? a.fr[hu[q] >> 6] : 0ull;
  int32_t par = -1;
#pragma unroll
  for (int q = kHeadArcs - 1; q >= 0; --q)
    if (hu[q] >= 0 && ((hw[q] >> (hu[q] & 63)) & 1ull)) par = hu[q];
  *more = p.mine && hu[kHeadArcs - 1] >= 0;
  return par;
}

// The rest of an unresolved row [beg, end) past its head arcs: its own lane
// goes on kPullEager arcs at a time with independent loads up to kPullLane
// arcs into the row (the lanes of a wavefront in step, each on its own
// row), then rows longer still are scanned by the whole wavefront 64 arcs
// at a time, one row after another.  Every lane calls it (uniform control
// flow); returns the lane's parent, the first in-neighbour in row order in
// the frontier.
constexpr int64_t kPullLane = 64;
__device__ __forceinline__ int32_t pull_row_rest(const Args& a, bool mine, int32_t par, int64_t beg, int64_t end) {
  const int lane = lane_id();
  const int64_t lim = end - beg < kPullLane ? end - beg : kPullLane;
  for (int64_t off = a.head_ranked ? 0 : kHeadArcs; __any(mine && par < 0 && off < lim); off += kPullEager) {
    if (mine && par < 0 && off < lim) {
      int32_t u[kPullEager];
      u64 fw[kPullEager];
#pragma unroll
      for (int q = 0; q < kPullEager; ++q) u[q] = off + q < lim ? a.rcols[beg + off + q] : -1;
#pragma unroll
      for (int q = 0; q < kPullEager; ++q) fw[q] = u[q] >= 0 ? a.fr[u[q] >> 6] : 0ull;
#pragma unroll
      for (int q = kPullEager - 1; q >= 0; --q)
        if (u[q] >= 0 && ((fw[q] >> (u[q] & 63)) & 1ull)) par = u[q];
    }
  }
  constexpr int64_t kProbed = kPullLane;
  u64 rest = __ballot(mine && par < 0 && end - beg > kProbed);
  while (rest != 0ull) {
    const int owner = __ffsll((long long)rest) - 1;
    rest &= rest - 1ull;
    const int64_t lo = __shfl(beg, owner) + kProbed;
    const int64_t hi = __shfl(end, owner);
    int32_t hit = -1;
    for (int64_t cc = lo; cc < hi; cc += 64) {
      const int64_t e = cc + lane;
      int32_t x = -1;
      bool h = false;
      if (e < hi) {
        x = a.rcols[e];
        h = (a.fr[x >> 6] >> (x & 63)) & 1ull;
      }
      const u64 hm = __ballot(h);
      if (hm != 0ull) {
        hit = __shfl(x, __ffsll((long long)hm) - 1);
        break;
      }
    }
    if (lane == owner) par = hit;
  }
  return par;
}

__device__ __forceinline__ void pull_settle(const Args& a, Stage& st, u64* found_w, const PullV& p, int32_t par) {
  const bool found = p.mine && par >= 0;
  if (found) {
    a.level[p.v] = a.d + 1;
    if (a.parent) a.parent[p.v] = par;
    atomicOr(&found_w[p.kw], 1ull << p.bit);
  }
  stage_push(st, a, found, p.v);
}

__device__ __forceinline__ void body_pull(const Args& a, Stage& st, u64 (*s_found)[kPullChunk]) {
  const int lane = lane_id();
  u64* found_w = s_found[threadIdx.x >> 6];
  const int64_t nwaves = (int64_t)a.grid * kWaves;
  const int64_t nchunks = (a.nw + kPullChunk - 1) / kPullChunk;
  for (int64_t c = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; c < nchunks; c += nwaves) {
    const int64_t w0 = c * kPullChunk;
    const bool word_lane = lane < kPullChunk && w0 + lane < a.nw;
    const u64 seen = word_lane ? a.vis[w0 + lane] : ~0ull;
    // inclusive prefix of the unvisited counts of the chunk's words (lanes 0..7)
    int inc = __popcll(~seen);
#pragma unroll
    for (int off = 1; off < kPullChunk; off <<= 1) {
      const int y = __shfl_up(inc, off);
      if (lane >= off) inc += y;
    }
    const int total = __builtin_amdgcn_readlane(inc, kPullChunk - 1);
    if (word_lane) found_w[lane] = 0ull;
    if (total == 0) {
      if (word_lane) a.nx[w0 + lane] = 0ull;
      continue;
    }
    u64 todo[kPullChunk];
    int first[kPullChunk];  // compacted index of each word's first unvisited vertex
#pragma unroll
    for (int i = 0; i < kPullChunk; ++i) {
      todo[i] = ~readlane64(seen, i);
      first[i] = __builtin_amdgcn_readlane(inc, i) - __popcll(todo[i]);
    }
    // two of the chunk's unvisited vertices per lane and step (compacted
    // positions r0 + lane and r0 + 64 + lane): their head records and
    // frontier-word probes are in flight together
    for (int r0 = 0; r0 < total; r0 += 128) {
      const PullV A = pull_vertex(r0 + lane, total, w0, todo, first);
      const PullV B = pull_vertex(r0 + 64 + lane, total, w0, todo, first);
      int4 hA[kHeadArcs / 4], hB[kHeadArcs / 4];
#pragma unroll
      for (int r = 0; r < kHeadArcs / 4; ++r) {
        hA[r] = make_int4(-1, -1, -1, -1);
        hB[r] = hA[r];
      }
#pragma unroll
      for (int r = 0; r < kHeadArcs / 4; ++r) {
        if (A.mine) hA[r] = reinterpret_cast<const int4*>(a.head)[(int64_t)A.v * (kHeadArcs / 4) + r];
        if (B.mine) hB[r] = reinterpret_cast<const int4*>(a.head)[(int64_t)B.v * (kHeadArcs / 4) + r];
      }
      bool moreA = false, moreB = false;
      int32_t parA = pull_head_hit(a, A, hA, &moreA);
      int32_t parB = pull_head_hit(a, B, hB, &moreB);
      // the row's bounds only when it may go on past the head and that found nothing
      int64_t begA = 0, endA = 0, begB = 0, endB = 0;
      if (moreA && parA < 0) {
        begA = a.roffs[A.v];
        endA = a.roffs[A.v + 1];
      }
      if (moreB && parB < 0) {
        begB = a.roffs[B.v];
        endB = a.roffs[B.v + 1];
      }
      parA = pull_row_rest(a, A.mine, parA, begA, endA);
      parB = pull_row_rest(a, B.mine, parB, begB, endB);
      pull_settle(a, st, found_w, A, parA);
      pull_settle(a, st, found_w, B, parB);
    }
    // the LDS words are this wave's alone and its LDS operations complete in
    // order; the barrier only keeps the compiler from moving the reads up
    __builtin_amdgcn_wave_barrier();
    if (word_lane) {
      const u64 fm = found_w[lane];
      a.nx[w0 + lane] = fm;
      if (fm) a.vis[w0 + lane] = seen | fm;  // this wave is the word's only writer in a pull level
    }
  }
}

// ------------------------------------------ vertex_scan (lane / vertex, all n)
__device__ __forceinline__ void body_vertex_scan(const Args& a, Stage& st, LongRows& L) {
  const int64_t stride = (int64_t)a.grid * kBlock;
  long_init(L);
  uint32_t r = 0;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < a.n; base += stride, ++r) {
    long_round_begin(L, r);
    const int64_t v = base + threadIdx.x;
    int64_t beg = 0, end = 0;
    if (v < a.n && a.level[v] == a.d) {
      beg = a.offs[v];
      end = a.offs[v + 1];
      if (long_defer(L, r, (int32_t)v, beg, end, kLongTrips)) end = beg;
    }
    visit_row(st, a, beg, end, 1, (int32_t)v);
    long_walk(L, r, st, a);
  }
}

// -------------------------------------------- edge_scan (lane / arc, all arcs)
__device__ __forceinline__ void body_edge_scan(const Args& a, Stage& st) {
  const int64_t stride = (int64_t)a.grid * kBlock;
  // uniform trip count so every lane of a wave reaches the ballots together
  const int64_t rounds = (a.nnz + stride - 1) / stride;
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t r = 0; r < rounds; ++r, e += stride) {
    bool win = false;
    int32_t v = 0;
    if (e < a.nnz) {
      const int32_t u = a.origin[e];
      if (a.level[u] == a.d) {
        v = a.cols[e];
        win = claim(a.vis, v);
        if (win) settle(a, v, u);
      }
    }
    stage_push(st, a, win, v);
  }
}

// ------------------------------- rev_edge_scan (lane / arc, destination order)
// The reverse edge list (Section III-A): a lane per arc of the in-arc lists,
// whose rows are the arcs' destinations.  A lane whose destination v is
// still unvisited (the visited word of consecutive lanes is mostly the same)
// tests the depth of the arc's source u and, when it is d, claims v.
__device__ __forceinline__ void body_rev_edge_scan(const Args& a, Stage& st) {
  const int64_t stride = (int64_t)a.grid * kBlock;
  const int64_t rounds = (a.nnz + stride - 1) / stride;
  int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t r = 0; r < rounds; ++r, e += stride) {
    bool win = false;
    int32_t v = 0;
    if (e < a.nnz) {
      v = a.rorigin[e];
      if (!((a.vis[v >> 6] >> (v & 63)) & 1ull)) {
        const int32_t u = a.rcols[e];
        if (a.level[u] == a.d) {
          win = claim(a.vis, v);
          if (win) settle(a, v, u);
        }
      }
    }
    stage_push(st, a, win, v);
  }
}

// ------------------------------------------------ one level, any variant
// Launch j of a search runs what control slot j % 2 names: level ctl->d with
// kernel ctl->kernel (push_edge: its scan or, in the next launch, its
// expansion), and writes slot (j + 1) % 2 for the next launch.  Late
// workgroups of a launch therefore never see the next launch's state.  Once
// the search has ended a launch does nothing but pass that on.
union LevelLds {
  LongRows lr;
  u64 found[kWaves][kPullChunk];
  EdgeLds edge;
  int64_t wsum[kWaves];
};

__global__ void __launch_bounds__(kBlock) k_level_auto(BfsBase b, BfsPolicy p, int32_t j) {
  __shared__ Stage st;
  __shared__ QueueIn qi;
  __shared__ LevelLds lds;
  const uint32_t cpre = counters_prefetch(b.ctr);
  const BfsCtl* c = b.ctl + (j & 1);
  const int k_id = c->kernel;  // the kernel id the level runs (base kernel and count variant)
  if (k_id < 0 || k_id >= GSW_N_KERNELS) {
    if (blockIdx.x == 0 && threadIdx.x == 0) b.ctl[(j + 1) & 1].kernel = kCtlDone;
    return;
  }
  const int k = kernel_base(k_id);
  const int32_t d = c->d;
  // the launch may be smaller than the level asks for: its workgroups then
  // stride over the work
  const int32_t grid = c->grid < (int32_t)gridDim.x ? c->grid : (int32_t)gridDim.x;
  const int32_t phase = k == GSW_K_PUSH_EDGE ? c->phase : 0;
  if (phase != 1 && d > 0) clear_bitmap(b.bm[(d + 2) % 3], b.nw);  // k_init zeroed it for level 0
  if ((int32_t)blockIdx.x >= grid) return;  // not needed for this launch (grid <= the launch)
  Args a = make_args(b, j, d, 0u, 1, grid);
  a.cv = kernel_count(k_id);
  if (phase != 1) {
    level_begin(a);
    clear_ahead(a);
  }
  stage_init(st);
  if (k != GSW_K_PULL_BITMAP && k != GSW_K_VERTEX_SCAN && k != GSW_K_EDGE_SCAN && k != GSW_K_REV_EDGE_SCAN) {
    queue_in_load(cpre, d & 3, qi);
    a.n_in = qi.pre[kQueueBins];
    a.per = push_per(a.n_in, a.grid);  // spread over the workgroups that take part
  }
  if (k == GSW_K_PUSH_EDGE && phase == 0) {
    body_edge_prefix(a, qi, b, lds.wsum);
    edge_prefix_end(a, b, lds.wsum);
    return;
  }
  if (k == GSW_K_PUSH_EDGE && phase == 2) {
    if (!body_edge_fused(a, st, qi, lds.edge)) return;
    const TreeLanes tl = tree_prefetch(p);
    u64 total = 0ull;
    const bool last = stage_flush_finish(st, a, &total);
    level_end(a, &b, p, b.ring, k_id, st.buf, (int)sizeof(st.buf), tl, last, total);
    return;
  }
  switch (k) {
    case GSW_K_PUSH_VERTEX: body_push_vertex(a, st, qi, lds.lr); break;
    case GSW_K_PUSH_WAVE4: body_push_wave<4>(a, st, qi, lds.lr); break;
    case GSW_K_PUSH_WAVE8: body_push_wave<8>(a, st, qi, lds.lr); break;
    case GSW_K_PUSH_WAVE16: body_push_wave<16>(a, st, qi, lds.lr); break;
    case GSW_K_PUSH_WAVE32: body_push_wave<32>(a, st, qi, lds.lr); break;
    case GSW_K_PUSH_WAVE64: body_push_wave<64>(a, st, qi, lds.lr); break;
    case GSW_K_PUSH_EDGE: {
      const EdgeScan es{b.scan, b.ebeg, b.bsum};
      body_edge_expand(a, st, qi, es, lds.edge, c->etot);
      break;
    }
    case GSW_K_PULL_BITMAP: body_pull(a, st, lds.found); break;
    case GSW_K_VERTEX_SCAN: body_vertex_scan(a, st, lds.lr); break;
    case GSW_K_REV_EDGE_SCAN: body_rev_edge_scan(a, st); break;
    default: body_edge_scan(a, st); break;
  }
  const TreeLanes tl = tree_prefetch(p);
  u64 total = 0ull;
  const bool last = stage_flush_finish(st, a, &total);
  level_end(a, &b, p, b.ring, k_id, st.buf, (int)sizeof(st.buf), tl, last, total);
}

// ------------------------------------ single-workgroup multi-level launches
// While the frontier is small (kSoloMax vertices, arcs bounded), one
// workgroup of kSoloBlock threads runs level after level of the queue-driven
// top-down expansion, applying the policy between levels and posting every
// level's record, so a long run of small levels (a high-diameter graph, the
// tail of a scale-free search) costs one launch instead of one launch of the
// whole grid per level.  Each level: every thread takes up to kSoloSlots
// frontier vertices (entry i = thread + kSoloBlock * slot) and walks rows of
// up to kSoloShort arcs itself, all its arcs in flight together; longer rows
// are set aside and their arcs spread over the whole workgroup through a
// prefix of their lengths (so one row never holds one thread).  Discoveries
// go to the queue segment 0 of the next depth with one LDS reservation per
// wavefront; the frontier bitmaps are not kept while the workgroup runs
// (all three are zero then) and the one of the depth the workgroup hands
// back is rebuilt from the queue when it stops.
constexpr int kSoloShort = 8;
constexpr int kSoloLong = kSoloBlock;  // long rows set aside per level at most
constexpr int kSoloWaves = kSoloBlock / 64;

struct SoloLds {
  u64 t_node[kSoloTree];
  int32_t t_thr[kSoloTree];
  int32_t t_next[kSoloTree];
  int64_t lbeg[kSoloLong];      // long rows: first arc
  int32_t lu[kSoloLong];        // long rows: vertex
  int32_t lpre[kSoloLong + 1];  // long rows: arc counts, then their exclusive prefix
  int32_t wsum[kSoloWaves];
  u64 esum;                     // arcs of the level's frontier
  uint32_t cnt;                 // next-frontier entries reserved
  uint32_t nlong;               // long rows set aside
  uint32_t nn;                  // the next frontier's size, for every thread
  int32_t go, next, nflags, pad;
};

// Claims the targets v[q] >= 0 (visited-word load, then the atomic where the
// bit is clear) for sources u[q / PER]; winners get depth d + 1, their
// parent, and a place in qout reserved by one LDS atomic per wavefront.
// Every lane of the wavefront calls it.
template <int N, int PER>
__device__ __forceinline__ void solo_visit(const BfsBase& b, int32_t d, int32_t* qout, uint32_t* cnt,
                                           const int32_t (&v)[N], const int32_t (&u)[N / PER]) {
  u64 w[N];
#pragma unroll
  for (int q = 0; q < N; ++q) w[q] = v[q] >= 0 ? b.vis[v[q] >> 6] : ~0ull;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const u64 bit = 1ull << (v[q] & 63);
    if (!(w[q] & bit)) w[q] = atomicOr(b.vis + (v[q] >> 6), bit);  // the word before this lane's bit
  }
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    const bool win = v[q] >= 0 && !(w[q] & (1ull << (v[q] & 63)));
    if (win) {
      b.level[v[q]] = d + 1;
      if (b.parent) b.parent[v[q]] = u[q / PER];
      ++mine;
    }
  }
  const int lane = lane_id();
  uint32_t inc = mine;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)inc, off);
    if (lane >= off) inc += y;
  }
  const uint32_t total = (uint32_t)__shfl((int)inc, 63);
  if (total == 0u) return;
  uint32_t base = 0u;
  if (lane == 63) base = atomicAdd(cnt, total);
  base = (uint32_t)__shfl((int)base, 63) + inc - mine;
#pragma unroll
  for (int q = 0; q < N; ++q)
    if (v[q] >= 0 && !(w[q] & (1ull << (v[q] & 63)))) qout[base++] = v[q];
}

// Entry i of the depth-d queue as a level kernel wrote it (kQueueBins segments).
__device__ __forceinline__ int32_t solo_queue_binned(const BfsBase& b, int32_t d, const QueueIn& qi, uint32_t i) {
  int bin = 0;
#pragma unroll
  for (int k = 1; k < kQueueBins; ++k) bin += i >= qi.pre[k] ? 1 : 0;
  return b.q[d & 1][(int64_t)bin * b.n + (i - qi.pre[bin])];
}

// Hands depth L back to the level kernel: its frontier (f entries, segment 0
// of the depth-L queue) becomes the queue's only segment and the depth-L
// bitmap, the counters the level will append to are zeroed, and control
// slot cn describes level L.  Every thread calls it.
__device__ __forceinline__ void solo_publish(const BfsBase& b, BfsCtl* cn, int32_t L, int32_t kernel, int32_t prev,
                                             int32_t flags, long long f, long long disc, long long ef) {
  const int tid = threadIdx.x;
  const int32_t* q = b.q[L & 1];
  u64* bm = b.bm[L % 3];
  for (long long i = tid; i < f; i += kSoloBlock) {
    const int32_t v = q[i];
    atomicOr(bm + (v >> 6), 1ull << (v & 63));
  }
  if (tid < kQueueBins) {
    b.ctr[(size_t)(L & 3) * kCtrSlot + tid * kCtrStride] = tid == 0 ? (uint32_t)f : 0u;
    b.ctr[(size_t)((L + 1) & 3) * kCtrSlot + tid * kCtrStride] = 0u;
    b.actr[(size_t)((L + 1) & 3) * kArcSlot + tid * kArcStride] = 0ull;
  }
  if (tid == 0) {
    cn->d = L;
    cn->kernel = kernel;
    cn->prev = prev;
    cn->flags = flags;
    cn->nf = f;
    cn->disc = disc;
    cn->done = 0ull;
    cn->phase = level_first_phase(kernel, f);
    cn->t_begin = 0ull;
    cn->grid = level_grid(kernel, f, b);
    cn->etot = 0;
    cn->ef = ef;
    cn->clean = 1;
  }
}

__global__ void __launch_bounds__(kSoloBlock) k_level_solo(BfsBase b, BfsPolicy p, int32_t j) {
  __shared__ SoloLds L;
  __shared__ QueueIn qi;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wid = tid >> 6;
  const uint32_t cpre = counters_prefetch(b.ctr);
  const BfsCtl* c = b.ctl + (j & 1);
  BfsCtl* cn = b.ctl + ((j + 1) & 1);
  int32_t k_id = c->kernel;
  int32_t d = c->d;
  long long nf = c->nf, disc = c->disc;
  int32_t prev = c->prev, flags = c->flags;
  const bool tree = p.policy == GSW_POLICY_TREE;
  const bool ok = b.solo > 0 && k_id >= 0 && k_id < GSW_N_KERNELS && kernel_base(k_id) <= GSW_K_PUSH_EDGE &&
                  nf >= 1 && nf <= kSoloMax && (!tree || p.t_nodes <= kSoloTree);
  if (!ok) {  // not a level for this launch: the slot passes on unchanged
    if (tid == 0) *cn = *c;
    return;
  }
  if (tid == 0) {
    L.esum = 0ull;
    L.cnt = 0u;
    L.nlong = 0u;
  }
  if (tree)
    for (int i = tid; i < p.t_nodes; i += kSoloBlock) {
      L.t_node[i] = p.t_node[i];
      L.t_thr[i] = p.t_thr[i];
    }
  queue_in_load(cpre, d & 3, qi);  // ends with a barrier
  if ((long long)qi.pre[kQueueBins] < nf) nf = (long long)qi.pre[kQueueBins];  // never past the queue's entries
  const bool check_arcs = (long long)b.deg_max * kSoloMax > kSoloMaxArcs;
  for (int lv = 0;; ++lv) {
    u64 t0 = 0ull;
    if (b.timed && tid == 0) t0 = (u64)wall_clock64();
    // the level's frontier: binned as the level kernel left it on the first
    // level, segment 0 afterwards
    int32_t u[kSoloSlots];
    int64_t beg[kSoloSlots], end[kSoloSlots];
    bool lng[kSoloSlots];
#pragma unroll
    for (int q = 0; q < kSoloSlots; ++q) {
      const long long i = tid + (long long)q * kSoloBlock;
      u[q] = -1;
      if (i < nf) u[q] = lv == 0 ? solo_queue_binned(b, d, qi, (uint32_t)i) : b.q[d & 1][i];
    }
    u64 arcs = 0ull;
#pragma unroll
    for (int q = 0; q < kSoloSlots; ++q) {
      beg[q] = end[q] = 0;
      if (u[q] >= 0) {
        beg[q] = b.offs[u[q]];
        end[q] = b.offs[u[q] + 1];
      }
      const int64_t deg = end[q] - beg[q];
      arcs += (u64)deg;
      lng[q] = false;
      if (deg > kSoloShort) {  // set aside while there is room, else walked by this thread
        const uint32_t at = atomicAdd(&L.nlong, 1u);
        if (at < (uint32_t)kSoloLong) {
          L.lu[at] = u[q];
          L.lbeg[at] = beg[q];
          L.lpre[at] = (int32_t)(deg < kSoloMaxArcs ? deg : kSoloMaxArcs + 1);
          lng[q] = true;
        }
      }
    }
    if (check_arcs || b.count_arcs) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) arcs += __shfl_xor(arcs, off);
      if (lane == 0 && arcs) atomicAdd(&L.esum, arcs);
    }
    __syncthreads();
    const u64 esum = L.esum;
    const uint32_t nlong = L.nlong < (uint32_t)kSoloLong ? L.nlong : (uint32_t)kSoloLong;
    if (esum > (u64)kSoloMaxArcs) {
      // too many arcs for one workgroup: the level goes back to the level
      // kernel untouched (on the first level nothing has changed at all)
      if (lv == 0) {
        if (tid == 0) *cn = *c;
      } else {
        solo_publish(b, cn, d, k_id, prev, flags, nf, disc, b.count_arcs ? (long long)esum : -1);
      }
      return;
    }
    if (lv == 0) {
      // the bitmaps are not kept here: clear the depth-d frontier's words and,
      // unless known clean, the depth-(d-1) bitmap
#pragma unroll
      for (int q = 0; q < kSoloSlots; ++q)
        if (u[q] >= 0) b.bm[d % 3][u[q] >> 6] = 0ull;
      if (!c->clean)
        for (int64_t i = tid; i < b.nw; i += kSoloBlock) b.bm[(d + 2) % 3][i] = 0ull;
    }
    int32_t* qout = b.q[(d + 1) & 1];
    // rows not set aside: a pair of slots' next four arcs each in flight together
    for (int r0 = 0;; r0 += 4) {
      bool any_more = false;
#pragma unroll
      for (int h = 0; h < kSoloSlots; h += 2) {
        const bool more = (!lng[h] && beg[h] + r0 < end[h]) || (!lng[h + 1] && beg[h + 1] + r0 < end[h + 1]);
        if (!__any(more)) continue;
        any_more = true;
        int32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int q = h + (k >> 2);
          const int64_t e = beg[q] + r0 + (k & 3);
          v[k] = !lng[q] && e < end[q] ? b.cols[e] : -1;
        }
        const int32_t us[2] = {u[h], u[h + 1]};
        solo_visit<8, 4>(b, d, qout, &L.cnt, v, us);
      }
      if (!any_more) break;
    }
    // long rows: their arcs over the whole workgroup
    if (nlong > 0u) {
      const int32_t x = tid < (int)nlong ? L.lpre[tid] : 0;
      int32_t inc = x;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
      }
      if (lane == 63) L.wsum[wid] = inc;
      __syncthreads();
      int32_t before = 0;
      for (int w = 0; w < wid; ++w) before += L.wsum[w];
      if (tid < (int)nlong) L.lpre[tid] = before + inc - x;
      if (tid == (int)nlong - 1) L.lpre[nlong] = before + inc;
      __syncthreads();
      const int32_t total = L.lpre[nlong];
      const int32_t rounds = (total + 4 * kSoloBlock - 1) / (4 * kSoloBlock);  // the same in every thread
      for (int32_t r = 0; r < rounds; ++r) {
        int32_t v[4], us[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int32_t a = tid + (4 * r + k) * kSoloBlock;
          v[k] = -1;
          us[k] = 0;
          if (a < total) {
            int lo = 0, hi = (int)nlong - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (L.lpre[mid] <= a) lo = mid; else hi = mid - 1;
            }
            v[k] = b.cols[L.lbeg[lo] + (a - L.lpre[lo])];
            us[k] = L.lu[lo];
          }
        }
        solo_visit<4, 1>(b, d, qout, &L.cnt, v, us);
      }
    }
    __syncthreads();
    // level end: the policy picks the next kernel; the level's record
    const uint32_t nn = L.cnt;
    const long long ndisc = disc + (long long)nn;
    if (tree && nn > 0u) {
      if (tid < p.t_nodes) L.t_next[tid] = tree_step(L.t_node[tid], L.t_thr[tid], (int32_t)nn, (int32_t)ndisc);
      __syncthreads();
    }
    if (tid == 0) {
      int32_t next = kCtlDone, nflags = 0;
      if (nn > 0u) {
        if (tree) {
          int32_t x = L.t_next[0];
          while (x >= 0) x = L.t_next[x];
          next = choose_leaf(p, x == -1 ? -1 : -x - 2, k_id, &nflags);
        } else {
          next = choose_next(p, d + 1, (long long)nn, ndisc, k_id, &nflags);
        }
      }
      u64 ticks = 0ull;
      if (b.timed) {
        const u64 t1 = (u64)wall_clock64();
        ticks = t1 > t0 ? t1 - t0 : 0ull;
      }
      u64* r = b.ring + (size_t)(d % kBfsRing) * kBfsRec;
      const u64 tag = rec_tag(d);
      const long long ef = b.count_arcs ? (long long)esum : -1;
      const u64 rec[kBfsRecWords] = {(u64)k_id, (u64)(flags | kFlagSolo), (u64)nf, (u64)disc, (u64)nn,
                                  ticks & kRecValueMask, (u64)(next + 1), (u64)(ef + 1) & kRecValueMask,
                                  (u64)j};
#pragma unroll
      for (int i = 0; i < kBfsRecWords; ++i)
        __hip_atomic_store(r + i, tag | rec[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      L.go = lv + 1 < b.solo && solo_eligible(next, (long long)nn, nf, ndisc, b.n, b.deg_max) ? 1 : 0;
      L.next = next;
      L.nflags = nflags;
      L.nn = nn;
      L.cnt = 0u;
      L.nlong = 0u;
      L.esum = 0ull;
    }
    __syncthreads();
    const int32_t next = L.next, nflags = L.nflags;
    const long long nnx = (long long)L.nn;
    if (!L.go) {
      if (nnx == 0) {
        if (tid == 0) {
          cn->d = d + 1;
          cn->kernel = kCtlDone;
          cn->prev = k_id;
          cn->flags = 0;
          cn->nf = 0;
          cn->disc = ndisc;
          cn->done = 0ull;
          cn->phase = 0;
          cn->t_begin = 0ull;
          cn->grid = 1;
          cn->etot = 0;
          cn->ef = -1;
          cn->clean = 1;
        }
        return;
      }
      long long ef_next = -1;
      if (b.count_arcs) {  // the next frontier's arcs, for its record
        u64 a = 0ull;
        const int32_t* q = b.q[(d + 1) & 1];
        for (long long i = tid; i < nnx; i += kSoloBlock) {
          const int32_t v = q[i];
          a += (u64)(b.offs[v + 1] - b.offs[v]);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        if (lane == 0 && a) atomicAdd(&L.esum, a);
        __syncthreads();
        ef_next = (long long)L.esum;
      }
      solo_publish(b, cn, d + 1, next, k_id, nflags, nnx, ndisc, ef_next);
      return;
    }
    prev = k_id;
    k_id = next;
    flags = nflags;
    nf = nnx;
    disc = ndisc;
    ++d;
  }
}

// ------------------------------------------------------------ helpers
// Bit v set when v has no in-arcs (only a source can reach depth 0 there).
__global__ void __launch_bounds__(kBlock) k_isolated(const int64_t* __restrict__ offs,
                                                     u64* __restrict__ iso, int64_t n, int64_t nw) {
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; w < nw; w += nwaves) {
    const int64_t v = w * 64 + lane;
    const u64 m = __ballot(v < n && offs[v + 1] == offs[v]);
    if (lane == 0) iso[w] = m;
  }
}

__global__ void __launch_bounds__(kBlock) k_build_head(const int64_t* __restrict__ offs,
                                                       const int32_t* __restrict__ cols,
                                                       int4* __restrict__ head, int64_t n) {
  static_assert(kHeadArcs % 4 == 0, "whole int4 records per row");
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const int64_t beg = offs[v], deg = offs[v + 1] - beg;
#pragma unroll
    for (int r = 0; r < kHeadArcs / 4; ++r) {
      int4 h;
      h.x = deg > 4 * r ? cols[beg + 4 * r] : -1;
      h.y = deg > 4 * r + 1 ? cols[beg + 4 * r + 1] : -1;
      h.z = deg > 4 * r + 2 ? cols[beg + 4 * r + 2] : -1;
      h.w = deg > 4 * r + 3 ? cols[beg + 4 * r + 3] : -1;
      head[v * (kHeadArcs / 4) + r] = h;
    }
  }
}

// The ranked head: per vertex (rows of in-arcs), the four in-neighbours of
// largest out-degree among the row's first kHeadScan arcs, in decreasing
// degree (an earlier arc first among equal degrees), -1 padded.
__global__ void __launch_bounds__(kBlock) k_build_head_ranked(const int64_t* __restrict__ roffs,
                                                              const int32_t* __restrict__ rcols,
                                                              const int64_t* __restrict__ offs,
                                                              int4* __restrict__ head, int64_t n) {
  static_assert(kHeadArcs == 4, "one int4 record per row");
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlock) {
    const int64_t beg = roffs[v], deg = roffs[v + 1] - beg;
    const int64_t lim = deg < kHeadScan ? deg : kHeadScan;
    int32_t id[4] = {-1, -1, -1, -1};
    int64_t dg[4] = {-1, -1, -1, -1};
    for (int64_t e = 0; e < lim; ++e) {
      const int32_t u = rcols[beg + e];
      const int64_t du = offs[u + 1] - offs[u];
      if (du > dg[3]) {  // insertion into the four largest so far
        int k = 3;
        while (k > 0 && du > dg[k - 1]) {
          dg[k] = dg[k - 1];
          id[k] = id[k - 1];
          --k;
        }
        dg[k] = du;
        id[k] = u;
      }
    }
    head[v] = make_int4(id[0], id[1], id[2], id[3]);
  }
}

// parent[v] = the smallest u with an arc u -> v one level up (rows of the
// in-arcs, any order).
__global__ void __launch_bounds__(kBlock) k_canonical_parents(const int64_t* __restrict__ offs,
                                                              const int32_t* __restrict__ cols,
                                                              const int32_t* __restrict__ level,
                                                              int32_t* __restrict__ parent,
                                                              int64_t n) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int32_t lv = level[v];
  if (lv <= 0) return;
  int32_t best = 0x7fffffff;
  for (int64_t e = offs[v]; e < offs[v + 1]; ++e) {
    const int32_t u = cols[e];
    if (u < best && level[u] == lv - 1) best = u;
  }
  parent[v] = best;
}

__global__ void __launch_bounds__(kBlock) k_build_origin(const int64_t* __restrict__ offs,
                                                         int32_t* __restrict__ origin, int64_t n) {
  // one wave per row: lanes stride over the row
  const int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (v >= n) return;
  const int lane = lane_id();
  for (int64_t e = offs[v] + lane; e < offs[v + 1]; e += 64) origin[e] = (int32_t)v;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline unsigned persistent_grid(int64_t work_blocks) {
  if (work_blocks < 1) return 1u;
  return (unsigned)(work_blocks < kMaxGrid ? work_blocks : kMaxGrid);
}

}  // namespace

int32_t level_participants(int kernel, int64_t n_in, const BfsBase& b) { return level_grid(kernel, n_in, b); }

// Grid of the any-variant level kernel: enough workgroups for a pull over all
// bitmap words and for a lane per vertex, at most kMaxGrid.
int32_t level_kernel_grid(int64_t n, int64_t nw) {
  const int64_t pull_blocks = cdiv(cdiv(nw, kPullChunk), kWaves);
  const int64_t vert_blocks = cdiv(n, kBlock);
  return (int32_t)persistent_grid(pull_blocks > vert_blocks ? pull_blocks : vert_blocks);
}

bool kernel_is_pull(int k) { return k >= 0 && kernel_base(k) == GSW_K_PULL_BITMAP; }

gsw_status launch_init(const gsw_graph* g, const BfsBase& b, const unsigned long long* iso, int32_t source,
                       int32_t k0, int32_t flags0, hipStream_t s) {
  int64_t blocks = cdiv(g->n, kBlock * 4);
  if (blocks < cdiv(4 * kCtrSlot, kBlock)) blocks = cdiv(4 * kCtrSlot, kBlock);
  const unsigned grid = (unsigned)(blocks > kMaxGrid ? kMaxGrid : blocks);
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, b, (const u64*)iso, source, k0, flags0);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_level_solo(const gsw_graph* g, const BfsBase& b, const BfsPolicy& p, int32_t j, hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_level_solo, dim3(1), dim3(kSoloBlock), 0, s, b, p, j);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_level_auto(const gsw_graph* g, const BfsBase& b, const BfsPolicy& p, int32_t j,
                             int32_t workgroups, hipStream_t s) {
  (void)g;
  const int32_t wg = workgroups < 1 ? 1 : (workgroups < b.grid_max ? workgroups : b.grid_max);
  hipLaunchKernelGGL(k_level_auto, dim3((unsigned)wg), dim3(kBlock), 0, s, b, p, j);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_build_head(const gsw_graph* g, int32_t* head, bool ranked, hipStream_t s) {
  if (ranked)
    hipLaunchKernelGGL(k_build_head_ranked, dim3(persistent_grid(cdiv(g->n, kBlock))), dim3(kBlock), 0, s,
                       g->roffs, g->rcols, g->offs, reinterpret_cast<int4*>(head), g->n);
  else
    hipLaunchKernelGGL(k_build_head, dim3(persistent_grid(cdiv(g->n, kBlock))), dim3(kBlock), 0, s, g->roffs,
                       g->rcols, reinterpret_cast<int4*>(head), g->n);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_isolated(const gsw_graph* g, unsigned long long* iso, hipStream_t s) {
  const int64_t nw = (g->n + 63) / 64;
  hipLaunchKernelGGL(k_isolated, dim3(persistent_grid(cdiv(nw, kWaves))), dim3(kBlock), 0, s,
                     g->roffs, iso, g->n, nw);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_canonical_parents(const gsw_graph* g, const int32_t* level, int32_t* parent,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_canonical_parents, dim3((unsigned)cdiv(g->n, kBlock)), dim3(kBlock), 0, s,
                     g->roffs, g->rcols, level, parent, g->n);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_build_origin(const int64_t* offs, int64_t n, int32_t* origin, hipStream_t s) {
  hipLaunchKernelGGL(k_build_origin, dim3((unsigned)cdiv(n * 64, kBlock)), dim3(kBlock), 0, s, offs, origin, n);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

}  // namespace gsw
