// Frontier-expansion kernels for gfx950 (CDNA4, 64-lane wavefronts).
//
// Every kernel performs one whole BFS level d (Section III-A): it finds the
// unvisited vertices adjacent to depth-d vertices, gives each depth d+1 and a
// parent at depth d, and appends it to the depth-(d+1) queue.  The frontier
// bitmaps rotate over three buffers (depth d in bm[d % 3]): the bottom-up
// kernel writes the depth-(d+1) bitmap in full, the top-down kernels set the
// bits of the vertices they discover (push_edge leaves it to a rebuild from
// the level array, run only when the next level is bottom-up), and every
// level zeroes the buffer of the level after next.  Any kernel can therefore
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
// without waiting for their results; push_edge, whose prefix sum needs a
// grid-wide step, is launched by the host as three kernels when the device
// names it.
//
// Ownership of a new vertex v is decided by atomicOr on its 64-bit visited
// word: exactly one lane sees the bit clear and becomes the writer of v's
// level, parent and queue slot.  A plain load of the word first filters out
// vertices already visited (a stale read only costs an atomic, because bits
// are only ever set).
//
// Appends are staged per workgroup in LDS (one LDS atomic per wavefront and
// round) and flushed with one global atomic per workgroup into the queue
// segment of its bin; a workgroup whose stage fills up appends further rounds
// directly, one atomic per wavefront.  (The paper compared a global atomic
// per thread with warp- and block-level reductions, Section III-A
// "Variants"; here the aggregation is per workgroup because same-address
// atomics serialise.)  Producer grids are persistent (at most kMaxGrid
// workgroups, grid-stride loops) so that few workgroups flush.
#include <hip/hip_runtime.h>

#include "gsw_internal.h"

namespace gsw {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxGrid = 2048;                   // persistent producer grids (8 per CU)
constexpr int kStage = 2048;                     // LDS-staged queue entries per workgroup
constexpr int kScanItems = 4;                    // push_edge: entries per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;   // entries per scan block
constexpr int kEdgeTile = 1024;                  // push_edge: edges per tile
constexpr int kEdgeWin = kEdgeTile;              // push_edge: queue entries staged per tile
constexpr int kPullEager = 8;                    // pull: neighbours probed per lane up front
constexpr int kPullChunk = 8;                    // pull: visited words (512 vertices) per wave step

typedef unsigned long long u64;

// One level's view of the buffers.
struct Args {
  const int64_t* __restrict__ offs;
  const int32_t* __restrict__ cols;
  const int32_t* __restrict__ origin;
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
  BfsCtl* ctl;
  uint32_t* done;
  int64_t n, nw, nnz;
  uint32_t n_in;
  int32_t d;
  int32_t set_nx;  // top-down kernels set the discovered vertices' bits in nx
  int32_t timed;
  int32_t grid;    // workgroups taking part in the level (grid-stride loops use it)
};

__host__ __device__ inline Args make_args(const BfsBase& b, int32_t d, uint32_t n_in, int32_t set_nx,
                                          int32_t grid) {
  Args a;
  a.offs = b.offs;
  a.cols = b.cols;
  a.origin = b.origin;
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
  a.ctl = b.ctl;
  a.done = b.done;
  a.n = b.n;
  a.nw = b.nw;
  a.nnz = b.nnz;
  a.n_in = n_in;
  a.d = d;
  a.set_nx = set_nx;
  a.timed = b.timed;
  a.grid = grid;
  return a;
}

__host__ __device__ inline int64_t div_up(int64_t x, int64_t y) { return (x + y - 1) / y; }

// Workgroups that run a level of kernel k with n_in frontier entries: a lane
// per entry for the queue-driven top-down kernels, a lane per vertex or arc
// for the all-vertex and all-arc ones, the whole launch for pull.
__host__ __device__ inline int32_t level_grid(int k, int64_t n_in, const BfsBase& b) {
  int64_t need;
  switch (k) {
    case GSW_K_PULL_BITMAP: need = b.grid_max; break;
    case GSW_K_VERTEX_SCAN: need = div_up(b.n, kBlock); break;
    case GSW_K_EDGE_SCAN: need = div_up(b.nnz, kBlock); break;
    default: need = div_up(n_in, kBlock); break;
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

// Zero the counter slot that the level after next appends to.
__device__ __forceinline__ void clear_ahead(const Args& a) {
  if (blockIdx.x == 0 && threadIdx.x < kQueueBins) a.cclr[threadIdx.x * kCtrStride] = 0u;
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

__device__ __forceinline__ void queue_in_load(const Args& a, QueueIn& q) {
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = 0; b < kQueueBins; ++b) {
      q.pre[b] = acc;
      acc += a.cin[b * kCtrStride];
    }
    q.pre[kQueueBins] = acc;
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
  uint32_t n;      // entries reserved (may exceed kStage once it overflowed)
  uint32_t valid;  // reservations at or past this position went to global memory
  uint32_t base;
};

__device__ __forceinline__ void stage_init(Stage& s) {
  if (threadIdx.x == 0) {
    s.n = 0u;
    s.valid = kStage;
  }
  __syncthreads();
}

// Appends the winning lanes' vertices.  Called by every active lane of the
// wave with the same control flow; no workgroup barrier inside.
__device__ __forceinline__ void stage_push(Stage& s, const Args& a, bool win, int32_t v) {
  const u64 m = __ballot(win);
  if (m == 0ull) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)m) - 1;
  const uint32_t k = (uint32_t)__popcll(m);
  uint32_t pos = 0;
  if (lane == leader) {
    pos = atomicAdd(&s.n, k);
    if (pos + k > (uint32_t)kStage) {
      atomicMin(&s.valid, pos);
      pos = (uint32_t)kStage + atomicAdd(a.cout + my_bin() * kCtrStride, k);
    }
  }
  pos = (uint32_t)__shfl((int)pos, leader);
  const uint32_t r = (uint32_t)__popcll(m & lanes_below(lane));
  if (win) {
    if (pos < (uint32_t)kStage)
      s.buf[pos + r] = v;
    else
      a.qout[(int64_t)my_bin() * a.n + (pos - (uint32_t)kStage) + r] = v;
  }
}

// Copies the staged entries to the workgroup's queue segment.  Every thread
// of the workgroup must call it.
__device__ __forceinline__ void stage_flush(Stage& s, const Args& a) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t cnt = s.n < s.valid ? s.n : s.valid;
    s.valid = cnt;
    s.base = cnt ? atomicAdd(a.cout + my_bin() * kCtrStride, cnt) : 0u;
  }
  __syncthreads();
  const uint32_t cnt = s.valid;
  int32_t* dst = a.qout + (int64_t)my_bin() * a.n + s.base;
  for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) dst[i] = s.buf[i];
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
// Feature i of level d+1's vector (Section IV-A list; the order of
// gsw_level_features).
__device__ __forceinline__ double feature(const BfsPolicy& p, int i, double nf, double disc) {
  switch (i) {
    case 8: return nf;
    case 9: return nf / p.feat[0];
    case 10: return disc;
    case 11: return disc / p.feat[0];
    default: return p.feat[i < 8 ? i : 0];
  }
}

// Kernel for level d (d >= 1) with frontier nf and nf + earlier discoveries
// = disc; prev = kernel of level d-1.  The same rules as the host's choice.
__device__ __forceinline__ int choose_next(const BfsPolicy& p, const u64* t_node, const double* t_thr, int32_t d,
                           long long nf, long long disc, int prev, int32_t* flags) {
  *flags = 0;
  int k = GSW_DEFAULT_KERNEL;
  if (p.policy == GSW_POLICY_FIXED) {
    k = p.fixed;
  } else if (p.policy == GSW_POLICY_SCHEDULE) {
    k = p.sched[d < p.sched_len ? d : p.sched_len - 1];
  } else {
    int node = 0;
    u64 nd = t_node[0];
    for (;;) {
      const int left = (int)(int16_t)(uint16_t)(nd & 0xffffull);
      if (left == -1) break;
      const int right = (int)(int16_t)(uint16_t)((nd >> 16) & 0xffffull);
      const double xv = (double)(float)feature(p, (int)((nd >> 32) & 0xffull), (double)nf, (double)disc);
      node = xv <= t_thr[node] ? left : right;
      nd = t_node[node];
    }
    const int leaf = (int)((nd >> 40) & 0xffull) - 1;
    if (leaf >= 0) {
      k = leaf;
    } else {
      k = prev;  // undecided leaf: repeat the previous level's kernel (d >= 1)
      *flags |= 1;
    }
  }
  if (k == GSW_K_PULL_BITMAP && !p.symmetric) {
    k = GSW_DEFAULT_KERNEL;
    *flags |= 2;
  }
  if (k == GSW_K_EDGE_SCAN && !p.has_origin) k = GSW_DEFAULT_KERNEL;
  return k;
}

// End of a level, called by every thread of every workgroup of the level's
// last kernel: the last workgroup to finish sums the next frontier's
// segments, picks the next kernel, posts the level's record to the host
// ring (its first word last) and rewrites the control block.  Each
// workgroup's queue-segment atomics have returned before it counts itself
// finished, so the last one sees every segment's final size.  That
// workgroup first copies the tree into `lds` (lds_bytes of LDS free by now,
// the flushed append stage) with all its threads, so the walk does not pay
// a global-memory round trip per node (8 bytes and a threshold per node:
// 512 nodes fit the 8 KiB stage).
__device__ __forceinline__ void level_end(const Args& a, const BfsBase* base, const BfsPolicy& p, u64* ring, int k_run,
                          void* lds, int lds_bytes) {
  __shared__ uint32_t s_last;
  __shared__ uint32_t s_nn;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_s_waitcnt(0);
    const uint32_t grid = (uint32_t)a.grid;
    uint32_t last = 1u;  // a level of one workgroup needs no count
    if (grid > (unsigned)kDoneGroups) {
      const uint32_t gidx = blockIdx.x % (unsigned)kDoneGroups;
      const uint32_t in_group = grid / kDoneGroups + (gidx < grid % kDoneGroups ? 1u : 0u);
      last = 0u;
      if (atomicAdd(a.done + gidx * kCtrStride, 1u) == in_group - 1u)
        last = atomicAdd(&a.ctl->done_blocks, 1u) == (unsigned)kDoneGroups - 1u ? 1u : 0u;
    } else if (grid > 1u) {
      last = atomicAdd(&a.ctl->done_blocks, 1u) == grid - 1u ? 1u : 0u;
    }
    s_last = last;
  }
  __syncthreads();
  if (!s_last) return;
  const int tid = threadIdx.x;
  const bool tree_lds = p.policy == GSW_POLICY_TREE && p.t_nodes * 16 <= lds_bytes;
  u64* l_node = reinterpret_cast<u64*>(lds);
  double* l_thr = reinterpret_cast<double*>(l_node + (tree_lds ? p.t_nodes : 0));
  if (tree_lds) {
    for (int i = tid; i < p.t_nodes; i += kBlock) {
      l_node[i] = p.t_node[i];
      l_thr[i] = p.t_thr[i];
    }
  }
  if (tid < 64) {  // wave 0: the next frontier's segments
    uint32_t x = tid < kQueueBins
                     ? __hip_atomic_load(a.cout + tid * kCtrStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : 0u;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off);
    if (tid == 0) s_nn = x;
  }
  if (tid < kDoneGroups) a.done[tid * kCtrStride] = 0u;
  __syncthreads();
  if (tid != 0) return;
  BfsCtl* c = a.ctl;
  const uint32_t nn = s_nn;
  u64 ticks = 0ull;
  if (a.timed) {
    const u64 t0 = __hip_atomic_load(&c->t_begin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 t1 = (u64)wall_clock64();
    ticks = t1 > t0 ? t1 - t0 : 0ull;
  }
  const int32_t d = a.d;
  const long long nf = c->nf, disc = c->disc, ndisc = disc + (long long)nn;
  int32_t nflags = 0;
  const int32_t next = nn > 0 ? choose_next(p, tree_lds ? l_node : p.t_node, tree_lds ? l_thr : p.t_thr, d + 1,
                                             (long long)nn, ndisc, k_run, &nflags)
                               : kCtlDone;
  u64* r = ring + (size_t)(d % kBfsRing) * kBfsRec;
  __hip_atomic_store(r + kRecKernel, (u64)k_run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(r + kRecFlags, (u64)c->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(r + kRecNf, (u64)nf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(r + kRecDisc, (u64)disc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(r + kRecNext, (u64)nn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(r + kRecTicks, ticks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(r + kRecNextKernel, (u64)(long long)next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  c->d = d + 1;
  c->kernel = next;
  c->grid = next >= 0 ? level_grid(next, (int64_t)nn, *base) : 1;
  c->prev = k_run;
  c->flags = nflags;
  c->nf = (long long)nn;
  c->disc = ndisc;
  c->done_blocks = 0u;
  // the host reads only the record: its other words are stored (system
  // scope, to host memory) before the first word, no cache writeback needed
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(r + kRecSeq, (u64)d + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
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
  for (int64_t i = gid; i < b.n; i += stride) {
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
    c->done_blocks = 0u;
    c->t_begin = 0ull;
    c->grid = level_grid(k0, 1, b);
  }
  if (gid < 4 * kCtrSlot) b.ctr[gid] = gid == 0 ? 1u : 0u;
  if (gid < kDoneGroups) b.done[gid * kCtrStride] = 0u;
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
  const uint32_t stride = (uint32_t)a.grid * kBlock;
  long_init(L);
  uint32_t r = 0;
  for (uint32_t base = blockIdx.x * kBlock; base < a.n_in; base += stride, ++r) {
    long_round_begin(L, r);
    const uint32_t i = base + threadIdx.x;
    int32_t u = 0;
    int64_t beg = 0, end = 0;
    if (i < a.n_in) {
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
  const uint32_t stride = (uint32_t)a.grid * kBlock;
  long_init(L);
  uint32_t r = 0;
  for (uint32_t base = blockIdx.x * kBlock; base < a.n_in; base += stride, ++r) {
    long_round_begin(L, r);
    const uint32_t i = base + threadIdx.x;  // this lane's own entry
    int32_t u = 0;
    int64_t beg = 0, end = 0;
    if (i < a.n_in) {
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

// ------------------------------------------------ push_edge (lane / frontier edge)
// Phase 1: per-entry degree and row start, block-local exclusive scan.
__global__ void __launch_bounds__(kBlock) k_edge_scan_local(Args a, int64_t* __restrict__ scan,
                                                            int64_t* __restrict__ ebeg,
                                                            int64_t* __restrict__ bsum) {
  level_begin(a);
  __shared__ int64_t wsum[kWaves];
  __shared__ QueueIn qi;
  clear_ahead(a);
  queue_in_load(a, qi);
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t deg[kScanItems];
  int64_t tot = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    deg[k] = 0;
    if (i < a.n_in) {
      const int32_t u = queue_at(a, qi, (uint32_t)i);
      const int64_t b = a.offs[u];
      ebeg[i] = b;
      deg[k] = a.offs[u + 1] - b;
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
    if (i < a.n_in) scan[i] = run;
    run += deg[k];
  }
  if (threadIdx.x == kBlock - 1 && (int64_t)blockIdx.x * kScanTile < (int64_t)a.n_in)
    bsum[blockIdx.x] = run;
}

// Phase 2: exclusive scan of the block sums (one workgroup), total -> etot.
__global__ void __launch_bounds__(1024) k_edge_scan_blocks(int64_t* __restrict__ bsum, int64_t nb,
                                                           u64* __restrict__ etot) {
  __shared__ int64_t wsum[1024 / 64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  int64_t tot = 0;
  for (int64_t i = lo; i < hi; ++i) tot += bsum[i];
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
    const int64_t x = bsum[i];
    bsum[i] = run;
    run += x;
  }
  if (threadIdx.x == 1023) *etot = (u64)run;
}

__device__ __forceinline__ int64_t gscan(const int64_t* scan, const int64_t* bsum, int64_t i) {
  return scan[i] + bsum[i / kScanTile];
}

// Largest entry index i in [lo, hi] with gscan(i) <= t (gscan(lo) <= t holds).
__device__ __forceinline__ int64_t find_entry(const int64_t* scan, const int64_t* bsum, int64_t lo,
                                              int64_t hi, int64_t t) {
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (gscan(scan, bsum, mid) <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Phase 3: tiles of kEdgeTile consecutive frontier edges; the queue entries a
// tile spans are staged in LDS and each lane locates its edge's entry by
// binary search there.
__global__ void __launch_bounds__(kBlock) k_edge_expand(Args a, const int64_t* __restrict__ scan,
                                                        const int64_t* __restrict__ ebeg,
                                                        const int64_t* __restrict__ bsum,
                                                        const u64* __restrict__ etot, BfsPolicy p,
                                                        BfsBase b) {
  __shared__ int64_t s_start[kEdgeWin + 1];
  __shared__ int64_t s_beg[kEdgeWin];
  __shared__ int32_t s_u[kEdgeWin];
  __shared__ int64_t s_range[2];
  __shared__ Stage st;
  __shared__ QueueIn qi;
  clear_bitmap(a.bclr, a.nw);
  stage_init(st);
  queue_in_load(a, qi);
  const int64_t total = (int64_t)*etot;
  const int64_t ntiles = (total + kEdgeTile - 1) / kEdgeTile;
  const int64_t last = (int64_t)a.n_in - 1;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t t0 = tile * kEdgeTile;
    const int64_t t1 = (t0 + kEdgeTile < total ? t0 + kEdgeTile : total) - 1;
    if (threadIdx.x < 2) s_range[threadIdx.x] = find_entry(scan, bsum, 0, last, threadIdx.x ? t1 : t0);
    __syncthreads();
    const int64_t i0 = s_range[0], i1 = s_range[1];
    const int64_t span = i1 - i0 + 1;
    const bool staged = span <= kEdgeWin;
    if (staged) {
      for (int64_t k = threadIdx.x; k < span; k += kBlock) {
        s_start[k] = gscan(scan, bsum, i0 + k);
        s_beg[k] = ebeg[i0 + k];
        s_u[k] = queue_at(a, qi, (uint32_t)(i0 + k));
      }
    }
    __syncthreads();
    for (int r = 0; r < kEdgeTile / kBlock; ++r) {
      const int64_t t = t0 + r * kBlock + threadIdx.x;
      const bool live = t <= t1;
      int32_t v = 0, u = 0;
      if (live) {
        int64_t st0, eb;
        if (staged) {
          int64_t lo = 0, hi = span - 1;
          while (lo < hi) {
            const int64_t mid = lo + (hi - lo + 1) / 2;
            if (s_start[mid] <= t) lo = mid; else hi = mid - 1;
          }
          st0 = s_start[lo];
          eb = s_beg[lo];
          u = s_u[lo];
        } else {
          const int64_t j = find_entry(scan, bsum, i0, i1, t);
          st0 = gscan(scan, bsum, j);
          eb = ebeg[j];
          u = queue_at(a, qi, (uint32_t)j);
        }
        v = a.cols[eb + (t - st0)];
      }
      bool win = false;
      if (live) {
        win = claim(a.vis, v);
        if (win) settle(a, v, u);
      }
      stage_push(st, a, win, v);
    }
    __syncthreads();
  }
  stage_flush(st, a);
  level_end(a, &b, p, b.ring, GSW_K_PUSH_EDGE, st.buf, (int)sizeof(st.buf));
}

// ------------------------------------------ pull_bitmap (wave / 512 vertices)
// A wave takes kPullChunk visited words (512 vertices) at a time and puts
// their unvisited vertices on its lanes, 64 per round, in vertex order: a
// level with few unvisited vertices costs one short round per 512 vertices
// instead of one dependent load chain per 64.  Each lane looks for a
// neighbour of its vertex in the frontier bitmap, in row order, and stops at
// the first one (Section III-A, vertex pull).  Phase 1: every lane probes the
// first kPullEager neighbours of its row with independent loads (many misses
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

// Position of the k-th (from 0) set bit of m; k < popcount(m).
__device__ __forceinline__ int nth_set_bit(u64 m, int k) {
  int pos = 0;
  int c = __popc((unsigned)m);
  if (k >= c) { k -= c; m >>= 32; pos += 32; }
  c = __popc((unsigned)(m & 0xffffull));
  if (k >= c) { k -= c; m >>= 16; pos += 16; }
  c = __popc((unsigned)(m & 0xffull));
  if (k >= c) { k -= c; m >>= 8; pos += 8; }
  c = __popc((unsigned)(m & 0xfull));
  if (k >= c) { k -= c; m >>= 4; pos += 4; }
  c = __popc((unsigned)(m & 0x3ull));
  if (k >= c) { k -= c; m >>= 2; pos += 2; }
  if (k >= (int)(m & 1ull)) pos += 1;
  return pos;
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
    for (int r0 = 0; r0 < total; r0 += 64) {
      const int k = r0 + lane;
      const bool mine = k < total;
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
      const int bit = mine ? nth_set_bit(t, k - f0) : 0;
      const int32_t v = (int32_t)((w0 + kw) * 64 + bit);
      int64_t beg = 0, end = 0;
      if (mine) {
        beg = a.offs[v];
        end = a.offs[v + 1];
      }
      int32_t u[kPullEager];
      u64 fw[kPullEager];
#pragma unroll
      for (int q = 0; q < kPullEager; ++q) u[q] = beg + q < end ? a.cols[beg + q] : -1;
#pragma unroll
      for (int q = 0; q < kPullEager; ++q) fw[q] = u[q] >= 0 ? a.fr[u[q] >> 6] : 0ull;
      int32_t par = -1;
#pragma unroll
      for (int q = kPullEager - 1; q >= 0; --q)
        if (u[q] >= 0 && ((fw[q] >> (u[q] & 63)) & 1ull)) par = u[q];
      u64 rest = __ballot(mine && par < 0 && end - beg > kPullEager);
      while (rest != 0ull) {
        const int owner = __ffsll((long long)rest) - 1;
        rest &= rest - 1ull;
        const int64_t lo = __shfl(beg, owner) + kPullEager;
        const int64_t hi = __shfl(end, owner);
        int32_t hit = -1;
        for (int64_t cc = lo; cc < hi; cc += 64) {
          const int64_t e = cc + lane;
          int32_t x = -1;
          bool h = false;
          if (e < hi) {
            x = a.cols[e];
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
      const bool found = par >= 0;
      if (found) {
        a.level[v] = a.d + 1;
        if (a.parent) a.parent[v] = par;
        atomicOr(&found_w[kw], 1ull << bit);
      }
      stage_push(st, a, found, v);
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

// ------------------------------------------------ one level, any variant
// Runs level ctl->d with the kernel ctl->kernel names; does nothing when that
// is push_edge (launched by the host) or when the search has ended.
__global__ void __launch_bounds__(kBlock) k_level_auto(BfsBase b, BfsPolicy p) {
  __shared__ Stage st;
  __shared__ QueueIn qi;
  __shared__ u64 s_found[kWaves][kPullChunk];
  __shared__ LongRows lr;
  const int k = b.ctl->kernel;
  if (k < 0 || k >= GSW_N_KERNELS || k == GSW_K_PUSH_EDGE) return;
  const int32_t d = b.ctl->d;
  const int32_t grid = b.ctl->grid;
  clear_bitmap(b.bm[(d + 2) % 3], b.nw);
  if ((int32_t)blockIdx.x >= grid) return;  // not needed for this level (grid <= the launch)
  Args a = make_args(b, d, 0u, 1, grid);
  level_begin(a);
  clear_ahead(a);
  stage_init(st);
  if (k != GSW_K_PULL_BITMAP && k != GSW_K_VERTEX_SCAN && k != GSW_K_EDGE_SCAN) {
    queue_in_load(a, qi);
    a.n_in = qi.pre[kQueueBins];
  }
  switch (k) {
    case GSW_K_PUSH_VERTEX: body_push_vertex(a, st, qi, lr); break;
    case GSW_K_PUSH_WAVE4: body_push_wave<4>(a, st, qi, lr); break;
    case GSW_K_PUSH_WAVE8: body_push_wave<8>(a, st, qi, lr); break;
    case GSW_K_PUSH_WAVE16: body_push_wave<16>(a, st, qi, lr); break;
    case GSW_K_PUSH_WAVE32: body_push_wave<32>(a, st, qi, lr); break;
    case GSW_K_PUSH_WAVE64: body_push_wave<64>(a, st, qi, lr); break;
    case GSW_K_PULL_BITMAP: body_pull(a, st, s_found); break;
    case GSW_K_VERTEX_SCAN: body_vertex_scan(a, st, lr); break;
    default: body_edge_scan(a, st); break;
  }
  stage_flush(st, a);
  level_end(a, &b, p, b.ring, k, st.buf, (int)sizeof(st.buf));
}

// Frontier bitmap of depth ctl->d from the level array, after a push_edge
// level when the next level is bottom-up (or always with force).
__global__ void __launch_bounds__(kBlock) k_rebuild_bitmap(BfsBase b, int32_t force) {
  const BfsCtl* c = b.ctl;
  if (!force && c->kernel != GSW_K_PULL_BITMAP) return;
  const int32_t d = c->d;
  u64* bm = b.bm[d % 3];
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t w = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; w < b.nw; w += nwaves) {
    const int64_t v = w * 64 + lane;
    const u64 m = __ballot(v < b.n && b.level[v] == d);
    if (lane == 0) bm[w] = m;
  }
}

// ------------------------------------------------------------ helpers
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

bool kernel_is_pull(int k) { return k == GSW_K_PULL_BITMAP; }

gsw_status launch_init(const gsw_graph* g, const BfsBase& b, int32_t source, int32_t k0, int32_t flags0,
                       hipStream_t s) {
  int64_t blocks = cdiv(g->n, kBlock * 4);
  if (blocks < cdiv(4 * kCtrSlot, kBlock)) blocks = cdiv(4 * kCtrSlot, kBlock);
  const unsigned grid = (unsigned)(blocks > 65536 ? 65536 : blocks);
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, b, (const u64*)g->iso, source, k0, flags0);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_level_auto(const gsw_graph* g, const BfsBase& b, const BfsPolicy& p, hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_level_auto, dim3((unsigned)b.grid_max), dim3(kBlock), 0, s, b, p);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_level_edge(const gsw_graph* g, const BfsBase& b, const BfsPolicy& p, int32_t d,
                             uint32_t n_in, bool force_bitmap, hipStream_t s) {
  const Workspace& w = g->ws;
  Args a = make_args(b, d, n_in, 0, kMaxGrid);
  const int64_t nb = cdiv(n_in, kScanTile) > 0 ? cdiv(n_in, kScanTile) : 1;
  hipLaunchKernelGGL(k_edge_scan_local, dim3((unsigned)nb), dim3(kBlock), 0, s, a, w.scan, w.ebeg, w.bsum);
  hipLaunchKernelGGL(k_edge_scan_blocks, dim3(1), dim3(1024), 0, s, w.bsum, nb, w.etot);
  hipLaunchKernelGGL(k_edge_expand, dim3(kMaxGrid), dim3(kBlock), 0, s, a, (const int64_t*)w.scan,
                     (const int64_t*)w.ebeg, (const int64_t*)w.bsum, (const u64*)w.etot, p, b);
  hipLaunchKernelGGL(k_rebuild_bitmap, dim3(persistent_grid(cdiv(b.nw, kWaves))), dim3(kBlock), 0, s, b,
                     force_bitmap ? 1 : 0);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_rebuild_bitmap(const gsw_graph* g, const BfsBase& b, hipStream_t s) {
  (void)g;
  hipLaunchKernelGGL(k_rebuild_bitmap, dim3(persistent_grid(cdiv(b.nw, kWaves))), dim3(kBlock), 0, s, b, 1);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_isolated(const gsw_graph* g, unsigned long long* iso, hipStream_t s) {
  const int64_t nw = (g->n + 63) / 64;
  hipLaunchKernelGGL(k_isolated, dim3(persistent_grid(cdiv(nw, kWaves))), dim3(kBlock), 0, s,
                     g->offs, iso, g->n, nw);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_canonical_parents(const gsw_graph* g, const int32_t* level, int32_t* parent,
                                    hipStream_t s) {
  hipLaunchKernelGGL(k_canonical_parents, dim3((unsigned)cdiv(g->n, kBlock)), dim3(kBlock), 0, s,
                     g->offs, g->cols, level, parent, g->n);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_build_origin(const gsw_graph* g, int32_t* origin, hipStream_t s) {
  hipLaunchKernelGGL(k_build_origin, dim3((unsigned)cdiv(g->n * 64, kBlock)), dim3(kBlock), 0, s,
                     g->offs, origin, g->n);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

}  // namespace gsw
