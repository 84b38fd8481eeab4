// Frontier-expansion kernels for gfx950 (CDNA4, 64-lane wavefronts).
//
// Every kernel performs one whole BFS level d (Section III-A): it finds the
// unvisited vertices adjacent to depth-d vertices, gives each depth d+1 and a
// parent at depth d, and emits the depth-(d+1) frontier twice -- as a queue
// (for the top-down kernels) and as a bitmap (for the bottom-up kernel) -- so
// that any kernel can run the next level.  Only the queue's order and the
// parent choice depend on the kernel; levels do not.
//
// Ownership of a new vertex v is decided by atomicOr on its 64-bit visited
// word: exactly one lane sees the bit clear and becomes the writer of v's
// level, parent, next-bitmap bit and queue slot.  A plain load of the word
// first filters out vertices already visited (a stale read only costs an
// atomic, because bits are only ever set).
//
// The next queue is appended wave-aggregated: one atomicAdd per wavefront
// per round of discoveries, lanes placed by their rank among the winners.
// (The paper tried one global atomic per thread and warp/block reductions,
// Section III-A "Variants"; on this hardware the per-wave form is used.)
//
// Each launch also zeroes the bitmap and counter that the level after next
// will use, so a level costs one launch.
#include <hip/hip_runtime.h>

#include "gsw_internal.h"

namespace gsw {
namespace {

constexpr int kBlock = 256;
constexpr int kClearPerThread = 8;
constexpr int kScanItems = 4;                     // push_edge: entries per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;    // entries per scan block
constexpr int kEdgeTile = 1024;                   // push_edge: edges per tile
constexpr int kEdgeWin = kEdgeTile;               // push_edge: queue entries staged per tile

typedef unsigned long long u64;

struct Args {
  const int64_t* __restrict__ offs;
  const int32_t* __restrict__ cols;
  const int32_t* __restrict__ origin;
  int32_t* __restrict__ level;
  int32_t* __restrict__ parent;
  u64* vis;
  const u64* __restrict__ fr;
  u64* nx;
  u64* clr;
  const int32_t* __restrict__ qin;
  int32_t* __restrict__ qout;
  LevelCtr* ctr;
  LevelCtr* ctr_clr;
  int64_t n, nw, nnz;
  uint32_t n_in;
  int32_t d;
};

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ u64 lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Zero this launch's share of the bitmap (and counter) the level after next uses.
__device__ __forceinline__ void clear_ahead(const Args& a) {
  if (a.clr) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nw; i += stride)
      a.clr[i] = 0ull;
  }
  if (a.ctr_clr && blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctr_clr->n_next = 0u;
    a.ctr_clr->e_next = 0ull;
  }
}

// True for the one lane (device-wide) that first sets v's visited bit.
__device__ __forceinline__ bool claim(u64* vis, int32_t v) {
  const u64 bit = 1ull << (v & 63);
  u64* w = vis + (v >> 6);
  if (*w & bit) return false;
  return (atomicOr(w, bit) & bit) == 0ull;
}

// Appends the winning lanes' vertices to the next queue: one atomic per wave.
// Called by every active lane of the wave with the same control flow.
__device__ __forceinline__ void wave_append(bool win, int32_t v, int32_t* qout, uint32_t* count) {
  const u64 m = __ballot(win);
  if (m == 0ull) return;
  const int lane = lane_id();
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, leader);
  if (win) qout[base + (uint32_t)__popcll(m & lanes_below(lane))] = v;
}

// Level/parent/next-bit writes of a newly owned vertex.
__device__ __forceinline__ void settle(const Args& a, int32_t v, int32_t u) {
  a.level[v] = a.d + 1;
  if (a.parent) a.parent[v] = u;
  atomicOr(a.nx + (v >> 6), 1ull << (v & 63));
}

__device__ __forceinline__ void visit(const Args& a, int32_t v, int32_t u) {
  const bool win = claim(a.vis, v);
  if (win) settle(a, v, u);
  wave_append(win, v, a.qout, &a.ctr->n_next);
}

// ---------------------------------------------------------------- init
__global__ void __launch_bounds__(kBlock) k_init(int32_t* __restrict__ level,
                                                 int32_t* __restrict__ parent, u64* vis, u64* b0,
                                                 u64* b1, u64* b2, int32_t* q0, LevelCtr* ctr,
                                                 int64_t n, int64_t nw, int32_t s) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = gid; i < n; i += stride) {
    level[i] = i == s ? 0 : -1;
    if (parent) parent[i] = i == s ? s : -1;
  }
  const int64_t sw = s >> 6;
  const u64 sbit = 1ull << (s & 63);
  const int tail = (int)(n & 63);
  for (int64_t w = gid; w < nw; w += stride) {
    u64 pad = 0ull;
    if (w == nw - 1 && tail) pad = ~0ull << tail;  // bits beyond n count as visited
    const u64 here = w == sw ? sbit : 0ull;
    vis[w] = here | pad;
    b0[w] = here;
    b1[w] = 0ull;
    b2[w] = 0ull;
  }
  if (gid == 0) q0[0] = s;
  if (gid < 4) {
    ctr[gid].n_next = 0u;
    ctr[gid].pad = 0u;
    ctr[gid].e_next = 0ull;
  }
}

// ------------------------------------------------- push_vertex (lane / vertex)
__global__ void __launch_bounds__(kBlock) k_push_vertex(Args a) {
  clear_ahead(a);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t u = 0;
  int64_t beg = 0, end = 0;
  if (i < a.n_in) {
    u = a.qin[i];
    beg = a.offs[u];
    end = a.offs[u + 1];
  }
  for (int64_t e = beg; e < end; ++e) visit(a, a.cols[e], u);
}

// ------------------------------------- push_wave<W> (W lanes / vertex, W vertices / group)
template <int W>
__global__ void __launch_bounds__(kBlock) k_push_wave(Args a) {
  clear_ahead(a);
  const int lane = lane_id();
  const int sub = lane & (W - 1);
  const int first = lane & ~(W - 1);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;  // this lane's own entry
  int32_t u = 0;
  int64_t beg = 0, end = 0;
  if (i < a.n_in) {
    u = a.qin[i];
    beg = a.offs[u];
    end = a.offs[u + 1];
  }
  for (int j = 0; j < W; ++j) {
    const int src = first + j;
    const int32_t uj = __shfl(u, src);
    const int64_t bj = __shfl(beg, src);
    const int64_t ej = __shfl(end, src);
    for (int64_t e = bj + sub; e < ej; e += W) visit(a, a.cols[e], uj);
  }
}

// ------------------------------------------------ push_edge (lane / frontier edge)
// Phase 1: per-entry degree, block-local exclusive scan.
__global__ void __launch_bounds__(kBlock) k_edge_scan_local(Args a, int64_t* __restrict__ scan,
                                                            int64_t* __restrict__ ebeg,
                                                            int64_t* __restrict__ bsum) {
  clear_ahead(a);
  __shared__ int64_t wsum[kBlock / 64];
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
      const int32_t u = a.qin[i];
      const int64_t b = a.offs[u];
      ebeg[i] = b;
      deg[k] = a.offs[u + 1] - b;
    }
    tot += deg[k];
  }
  // inclusive scan of per-thread totals within the wave
  int64_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(inc, off);
    if (lane >= off) inc += y;
  }
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t wpre = 0;
  for (int k = 0; k < wid; ++k) wpre += wsum[k];
  int64_t run = wpre + inc - tot;  // exclusive prefix of this thread within the block
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
                                                        const u64* __restrict__ etot) {
  __shared__ int64_t s_start[kEdgeWin + 1];
  __shared__ int64_t s_beg[kEdgeWin];
  __shared__ int32_t s_u[kEdgeWin];
  __shared__ int64_t s_range[2];
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
      for (int64_t k = threadIdx.x; k < span; k += blockDim.x) {
        s_start[k] = gscan(scan, bsum, i0 + k);
        s_beg[k] = ebeg[i0 + k];
        s_u[k] = a.qin[i0 + k];
      }
    }
    __syncthreads();
    for (int r = 0; r < kEdgeTile / kBlock; ++r) {
      const int64_t t = t0 + r * kBlock + threadIdx.x;
      const bool live = t <= t1;
      int32_t v = 0, u = 0;
      if (live) {
        int64_t j, st, eb;
        if (staged) {
          int64_t lo = 0, hi = span - 1;
          while (lo < hi) {
            const int64_t mid = lo + (hi - lo + 1) / 2;
            if (s_start[mid] <= t) lo = mid; else hi = mid - 1;
          }
          st = s_start[lo];
          eb = s_beg[lo];
          u = s_u[lo];
          j = lo;
        } else {
          j = find_entry(scan, bsum, i0, i1, t);
          st = gscan(scan, bsum, j);
          eb = ebeg[j];
          u = a.qin[j];
        }
        (void)j;
        v = a.cols[eb + (t - st)];
      }
      bool win = false;
      if (live) {
        win = claim(a.vis, v);
        if (win) settle(a, v, u);
      }
      wave_append(win, v, a.qout, &a.ctr->n_next);
    }
    __syncthreads();
  }
}

// ------------------------------------------- pull_bitmap (wave / 64-vertex word)
__global__ void __launch_bounds__(kBlock) k_pull(Args a) {
  clear_ahead(a);
  const int lane = lane_id();
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (w >= a.nw) return;  // whole wave
  const u64 seen = a.vis[w];
  const u64 todo = ~seen;
  if (todo == 0ull) return;  // whole wave
  const int32_t v = (int32_t)(w * 64 + lane);
  bool found = false;
  int32_t par = -1;
  if ((todo >> lane) & 1ull) {
    const int64_t end = a.offs[v + 1];
    for (int64_t e = a.offs[v]; e < end; ++e) {
      const int32_t u = a.cols[e];
      if ((a.fr[u >> 6] >> (u & 63)) & 1ull) {
        found = true;
        par = u;
        break;
      }
    }
  }
  const u64 fm = __ballot(found);
  if (fm == 0ull) return;
  if (found) {
    a.level[v] = a.d + 1;
    if (a.parent) a.parent[v] = par;
  }
  uint32_t base = 0;
  if (lane == 0) {
    a.vis[w] = seen | fm;  // this wave is the word's only writer in a pull level
    a.nx[w] = fm;
    base = atomicAdd(&a.ctr->n_next, (uint32_t)__popcll(fm));
  }
  base = (uint32_t)__shfl((int)base, 0);
  if (found) a.qout[base + (uint32_t)__popcll(fm & lanes_below(lane))] = v;
}

// ------------------------------------------ vertex_scan (lane / vertex, all n)
__global__ void __launch_bounds__(kBlock) k_vertex_scan(Args a) {
  clear_ahead(a);
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t beg = 0, end = 0;
  if (v < a.n && a.level[v] == a.d) {
    beg = a.offs[v];
    end = a.offs[v + 1];
  }
  for (int64_t e = beg; e < end; ++e) visit(a, a.cols[e], (int32_t)v);
}

// -------------------------------------------- edge_scan (lane / arc, all arcs)
__global__ void __launch_bounds__(kBlock) k_edge_scan(Args a) {
  clear_ahead(a);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // uniform trip count so every lane of a wave reaches the ballots together
  const int64_t rounds = (a.nnz + stride - 1) / stride;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    wave_append(win, v, a.qout, &a.ctr->n_next);
  }
}

// ------------------------------------------------------------ helpers
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

Args to_args(const LevelLaunch& l) {
  Args a;
  a.offs = l.offs;
  a.cols = l.cols;
  a.origin = l.origin;
  a.level = l.level;
  a.parent = l.parent;
  a.vis = l.vis;
  a.fr = l.fr;
  a.nx = l.nx;
  a.clr = l.clr;
  a.qin = l.qin;
  a.qout = l.qout;
  a.ctr = l.ctr;
  a.ctr_clr = l.ctr_clr;
  a.n = l.n;
  a.nw = l.nw;
  a.nnz = l.nnz;
  a.n_in = l.n_in;
  a.d = l.d;
  return a;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Blocks needed so that clear_ahead touches each word at most kClearPerThread times.
inline int64_t clear_blocks(int64_t nw) { return cdiv(nw, (int64_t)kBlock * kClearPerThread); }

inline unsigned grid_of(int64_t work_blocks, int64_t nw) {
  int64_t g = work_blocks > clear_blocks(nw) ? work_blocks : clear_blocks(nw);
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <int W>
void push_wave_launch(const Args& a, hipStream_t s) {
  hipLaunchKernelGGL(k_push_wave<W>, dim3(grid_of(cdiv(a.n_in, kBlock), a.nw)), dim3(kBlock), 0, s,
                     a);
}

}  // namespace

bool kernel_is_pull(int k) { return k == GSW_K_PULL_BITMAP; }

gsw_status launch_init(const gsw_graph* g, int32_t* level, int32_t* parent, int32_t source,
                       hipStream_t s) {
  const Workspace& w = g->ws;
  const int64_t blocks = cdiv(g->n, kBlock * 4);
  const unsigned grid = (unsigned)(blocks < 1 ? 1 : (blocks > 65536 ? 65536 : blocks));
  hipLaunchKernelGGL(k_init, dim3(grid), dim3(kBlock), 0, s, level, parent, w.vis, w.bm[0], w.bm[1],
                     w.bm[2], w.q[0], w.ctr, g->n, w.nw, source);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

gsw_status launch_level(const gsw_graph* g, int kernel, const LevelLaunch& l, hipStream_t s) {
  const Args a = to_args(l);
  switch (kernel) {
    case GSW_K_PUSH_VERTEX:
      hipLaunchKernelGGL(k_push_vertex, dim3(grid_of(cdiv(a.n_in, kBlock), a.nw)), dim3(kBlock), 0,
                         s, a);
      break;
    case GSW_K_PUSH_WAVE4: push_wave_launch<4>(a, s); break;
    case GSW_K_PUSH_WAVE8: push_wave_launch<8>(a, s); break;
    case GSW_K_PUSH_WAVE16: push_wave_launch<16>(a, s); break;
    case GSW_K_PUSH_WAVE32: push_wave_launch<32>(a, s); break;
    case GSW_K_PUSH_WAVE64: push_wave_launch<64>(a, s); break;
    case GSW_K_PUSH_EDGE: {
      const Workspace& w = g->ws;
      const int64_t nb = cdiv(a.n_in, kScanTile);
      hipLaunchKernelGGL(k_edge_scan_local, dim3(grid_of(nb, a.nw)), dim3(kBlock), 0, s, a, w.scan,
                         w.ebeg, w.bsum);
      hipLaunchKernelGGL(k_edge_scan_blocks, dim3(1), dim3(1024), 0, s, w.bsum, nb, w.etot);
      // enough tiles in flight to fill the chip; tiles are grid-strided
      hipLaunchKernelGGL(k_edge_expand, dim3(2048), dim3(kBlock), 0, s, a, w.scan, w.ebeg, w.bsum,
                         w.etot);
      break;
    }
    case GSW_K_PULL_BITMAP:
      hipLaunchKernelGGL(k_pull, dim3(grid_of(cdiv(a.nw * 64, kBlock), a.nw)), dim3(kBlock), 0, s,
                         a);
      break;
    case GSW_K_VERTEX_SCAN:
      hipLaunchKernelGGL(k_vertex_scan, dim3(grid_of(cdiv(a.n, kBlock), a.nw)), dim3(kBlock), 0, s,
                         a);
      break;
    case GSW_K_EDGE_SCAN: {
      int64_t blocks = cdiv(a.nnz, kBlock * 8);
      if (blocks > 8192) blocks = 8192;
      hipLaunchKernelGGL(k_edge_scan, dim3(grid_of(blocks, a.nw)), dim3(kBlock), 0, s, a);
      break;
    }
    default:
      return fail(GSW_EINVAL, "unknown kernel id %d", kernel);
  }
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

int64_t edge_scan_blocks_needed(int64_t n) { return cdiv(n, kScanTile); }

}  // namespace gsw
