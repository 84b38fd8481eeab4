// Weakly connected components on the level-switching framework.
//
// The paper expects its per-iteration choice among interchangeable kernels
// to carry over to other traversal algorithms (Section VI).  Components are
// computed here in two phases:
//
//  1. On a symmetric graph, the component of a vertex of largest degree is
//     found by the level-switched BFS itself (the tree picks each level's
//     kernel, Sections III-A and IV-A): its reached vertices take the
//     smallest id among them as their label.  On scale-free and mesh-like
//     graphs this one component holds almost every arc.
//  2. Every other vertex with arcs starts with its own id as label, and
//     minimum-label propagation runs until no label changes.  Each
//     iteration runs one of two interchangeable kernels, chosen per
//     iteration from the active set (the vertices whose label fell in the
//     previous iteration), as BFS levels are chosen from the frontier:
//       push  one lane per active vertex lowers its neighbours' labels with
//             atomicMin; a lowered vertex joins the next active list once
//             (a bitmap claim);
//       pull  one lane per remaining vertex takes the minimum over all its
//             neighbours' labels (no atomics; every arc of the remaining
//             vertices is read).
//     The switching rule pulls once the active vertices' arcs exceed a
//     fraction of the remaining vertices' arcs (the frontier-arc criterion
//     of direction-optimising traversal), else pushes.
//
// Arcs join their ends whatever their direction: on a directed graph both
// the out-arcs and the in-arcs (the transpose the library keeps) of a vertex
// are its neighbours, and phase 1 is skipped (a BFS over out-arcs does not
// reach a weak component).  Labels fall monotonically, so a stale read of a
// label (higher than its current value) only delays a change to a later
// iteration; an iteration that changes nothing read every label as the
// previous iteration left it, which is the fixed point: every arc's ends carry
// the same label, the smallest id of the component.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "gsw_internal.h"

namespace gsw {

using u64 = unsigned long long;

struct CcWorkspace {
  int64_t n = 0;
  int32_t* tmp = nullptr;   // labels when the caller passes host memory
  int32_t* rest = nullptr;  // vertices left to phase 2 (with arcs, not reached in phase 1)
  int32_t* q[2] = {};       // active lists
  u64* mark = nullptr;      // bit per vertex: already on the next active list (push)
  u64* ctr = nullptr;       // device counters (kCcCtr words)
  u64* h_ctr = nullptr;     // pinned copy
  hipEvent_t ev[2] = {};
  int32_t seed = -1;        // a vertex of largest out-degree (computed once per graph)
  size_t bytes = 0;
};

namespace {

constexpr int kCcBlock = 256;
constexpr int64_t kCcLane = 32;  // rows of at most this many arcs are walked by their own lane
constexpr int kCcBatch = 8;      // arcs a lane keeps in flight (column loads, then label loads)
constexpr int kCcGridMax = 2048;
// counters, 16 words apart
enum : int { kCtrCount = 0, kCtrArcs = 16, kCtrKey = 32, kCtrReached = 48, kCtrRoots = 64, kCcCtr = 80 };

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned cc_grid(int64_t items) {
  const int64_t b = cdiv(items < 1 ? 1 : items, kCcBlock);
  return (unsigned)(b < kCcGridMax ? b : kCcGridMax);
}

__device__ __forceinline__ int cc_lane() { return (int)__lane_id(); }

__device__ __forceinline__ u64 wave_sum(u64 x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

__device__ __forceinline__ int32_t wave_min(int32_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = min(x, __shfl_xor(x, off));
  return x;
}

// Combines one value per thread over the workgroup (op: max, min or sum);
// the result is valid in thread 0.  Reductions over all n vertices end with
// one global atomic per workgroup: one per wave (8192 on one counter for a
// launch of 2048 workgroups) serialise into tens of microseconds.
template <class Op>
__device__ __forceinline__ u64 cc_block_reduce(u64 x, Op op) {
  __shared__ u64 part[kCcBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = op(x, __shfl_xor(x, off));
  if (cc_lane() == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < kCcBlock / 64; ++w) x = op(x, part[w]);
  return x;
}
struct CcMax {
  __device__ u64 operator()(u64 a, u64 b) const { return a > b ? a : b; }
};
struct CcMin {
  __device__ u64 operator()(u64 a, u64 b) const { return a < b ? a : b; }
};
struct CcSum {
  __device__ u64 operator()(u64 a, u64 b) const { return a + b; }
};

// Appends the lanes with `take` set to list (one atomic per wave); every
// active lane of the wave calls it with the same control flow.
__device__ __forceinline__ void cc_append(bool take, int32_t v, int32_t* list, u64* count) {
  const u64 m = __ballot(take);
  if (m == 0ull) return;
  const int lane = cc_lane();
  const int leader = __ffsll((long long)m) - 1;
  u64 pos = 0;
  if (lane == leader) pos = atomicAdd(count, (u64)__popcll(m));
  pos = __shfl(pos, leader);
  if (take) list[pos + (u64)__popcll(m & ((1ull << lane) - 1ull))] = v;
}

// Workgroup staging of list appends for loops whose trip count is uniform
// over the workgroup: entries gather in LDS and go out with one global
// atomic per kCcStage of them (appends to one counter serialise, about 11 ns
// each, so one atomic per wave would cost more than the kernel's reads when
// millions of vertices change).  Every thread calls cc_stage_add and
// cc_stage_flush at the same points.
constexpr int kCcStage = 2048;
struct CcStage {
  int32_t buf[kCcStage];
  uint32_t n;
  unsigned long long base;
};

__device__ __forceinline__ void cc_stage_init(CcStage& S) {
  if (threadIdx.x == 0) S.n = 0u;
  __syncthreads();
}

__device__ __forceinline__ void cc_stage_flush(CcStage& S, int32_t* list, u64* count) {
  __syncthreads();
  const uint32_t m = S.n;
  if (m == 0u) return;  // uniform: every thread read the same S.n after the barrier
  if (threadIdx.x == 0) S.base = atomicAdd(count, (u64)m);
  __syncthreads();
  const u64 b = S.base;
  for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) list[b + i] = S.buf[i];
  __syncthreads();
  if (threadIdx.x == 0) S.n = 0u;
  __syncthreads();
}

// Adds the threads with `take` set (at most one entry per thread per call);
// flushes first when the buffer could overflow.
__device__ __forceinline__ void cc_stage_add(CcStage& S, bool take, int32_t v, int32_t* list, u64* count) {
  __syncthreads();
  if (S.n + blockDim.x > (uint32_t)kCcStage) cc_stage_flush(S, list, count);
  const u64 m = __ballot(take);
  if (m == 0ull) return;
  const int lane = cc_lane();
  const int leader = __ffsll((long long)m) - 1;
  uint32_t pos = 0;
  if (lane == leader) pos = atomicAdd(&S.n, (uint32_t)__popcll(m));
  pos = (uint32_t)__shfl((int)pos, leader);
  if (take) S.buf[pos + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = v;
}

__device__ __forceinline__ int64_t cc_degree(const int64_t* offs, const int64_t* roffs, int32_t v) {
  int64_t d = offs[v + 1] - offs[v];
  if (roffs) d += roffs[v + 1] - roffs[v];
  return d;
}

// A vertex of largest out-degree, the smallest id among ties: the maximum of
// (degree << 32 | (2^31 - 1 - v)).
__global__ void __launch_bounds__(kCcBlock) k_cc_argmax(const int64_t* __restrict__ offs, int64_t n, u64* key) {
  u64 best = 0ull;
  for (int64_t v = (int64_t)blockIdx.x * kCcBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kCcBlock) {
    int64_t d = offs[v + 1] - offs[v];
    if (d > 0x7fffffff) d = 0x7fffffff;
    const u64 k = ((u64)d << 32) | (u64)(0x7fffffffu - (uint32_t)v);
    best = k > best ? k : best;
  }
  best = cc_block_reduce(best, CcMax());
  if (threadIdx.x == 0) atomicMax(key, best);
}

// Phase 1 result: the smallest reached id and the number of reached vertices.
__global__ void __launch_bounds__(kCcBlock) k_cc_reached(const int32_t* __restrict__ level, int64_t n, u64* first,
                                                         u64* reached) {
  u64 lo = (u64)n, cnt = 0ull;
  for (int64_t v = (int64_t)blockIdx.x * kCcBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kCcBlock)
    if (level[v] >= 0) {
      lo = (u64)v < lo ? (u64)v : lo;
      ++cnt;
    }
  lo = cc_block_reduce(lo, CcMin());
  __syncthreads();  // the partials are reused by the second reduction
  cnt = cc_block_reduce(cnt, CcSum());
  if (threadIdx.x == 0) {
    if (lo < (u64)n) atomicMin(first, lo);
    if (cnt) atomicAdd(reached, cnt);
  }
}

// Initial labels: phase 1's component takes *first (level, when given, is
// the BFS row and may be the label array itself), every other vertex its own
// id; the vertices with arcs outside phase 1's component form the list
// `rest` (count and arcs in the counters).
__global__ void __launch_bounds__(kCcBlock) k_cc_seed(const int32_t* level, const u64* first,
                                                      const int64_t* __restrict__ offs,
                                                      const int64_t* __restrict__ roffs, int64_t n, int32_t* label,
                                                      int32_t* rest, u64* ctr) {
  __shared__ CcStage S;
  cc_stage_init(S);
  const int32_t gmin = level ? (int32_t)*first : 0;
  u64 arcs = 0ull;
  for (int64_t base = (int64_t)blockIdx.x * kCcBlock; base < n; base += (int64_t)gridDim.x * kCcBlock) {
    const int64_t v = base + threadIdx.x;
    bool take = false;
    if (v < n) {
      const bool reached = level && level[v] >= 0;
      label[v] = reached ? gmin : (int32_t)v;
      if (!reached) {
        const int64_t d = cc_degree(offs, roffs, (int32_t)v);
        take = d > 0;
        arcs += (u64)d;
      }
    }
    cc_stage_add(S, take, (int32_t)v, rest, ctr + kCtrCount);
  }
  cc_stage_flush(S, rest, ctr + kCtrCount);
  arcs = cc_block_reduce(arcs, CcSum());
  if (threadIdx.x == 0 && arcs) atomicAdd(ctr + kCtrArcs, arcs);
}

// Lowers v's label to lu; true when it fell and v was not yet on the next
// active list (the caller appends it).  A stale plain read of label[v] is
// never below its current value, so the test only skips arcs atomicMin
// would not change.
__device__ __forceinline__ bool cc_lower(int32_t* label, u64* mark, int32_t v, int32_t lu) {
  if (lu >= label[v]) return false;
  if (lu >= atomicMin(label + v, lu)) return false;
  const u64 bit = 1ull << (v & 63);
  return (atomicOr(mark + (v >> 6), bit) & bit) == 0ull;
}

// Push: every active vertex lowers the labels of its neighbours (out-arcs,
// and in-arcs on a directed graph).  Rows of at most kCcLane arcs are walked
// by their own lane, one arc per step; longer ones by the whole wavefront,
// 64 arcs per step, one row after another.
__global__ void __launch_bounds__(kCcBlock) k_cc_push(const int32_t* __restrict__ qin, int64_t nin, int32_t* label,
                                                      const int64_t* __restrict__ offs,
                                                      const int32_t* __restrict__ cols,
                                                      const int64_t* __restrict__ roffs,
                                                      const int32_t* __restrict__ rcols, u64* mark, int32_t* qout,
                                                      u64* ctr) {
  const int lane = cc_lane();
  u64 arcs = 0ull;
  const int nrows = roffs ? 2 : 1;
  for (int64_t base = (int64_t)blockIdx.x * kCcBlock; base < nin; base += (int64_t)gridDim.x * kCcBlock) {
    const int64_t i = base + threadIdx.x;
    const bool mine = i < nin;
    const int32_t u = mine ? qin[i] : 0;
    const int32_t lu = mine ? label[u] : 0;
    for (int r = 0; r < nrows; ++r) {
      const int64_t* ro = r == 0 ? offs : roffs;
      const int32_t* co = r == 0 ? cols : rcols;
      int64_t beg = 0, end = 0;
      if (mine) {
        beg = ro[u];
        end = ro[u + 1];
      }
      const bool own = end - beg <= kCcLane;
      for (int64_t k = 0; __any(own && beg + k < end); k += kCcBatch) {
        int32_t v[kCcBatch], lw[kCcBatch];
#pragma unroll
        for (int q = 0; q < kCcBatch; ++q) v[q] = own && beg + k + q < end ? co[beg + k + q] : -1;
#pragma unroll
        for (int q = 0; q < kCcBatch; ++q) lw[q] = v[q] >= 0 ? label[v[q]] : 0x7fffffff;
#pragma unroll
        for (int q = 0; q < kCcBatch; ++q) {
          // the plain read filters: only arcs that would lower a label reach the atomics
          const bool take = v[q] >= 0 && lu < lw[q] && cc_lower(label, mark, v[q], lu);
          if (take) arcs += (u64)cc_degree(offs, roffs, v[q]);
          cc_append(take, v[q], qout, ctr + kCtrCount);
        }
      }
      u64 longs = __ballot(!own);
      while (longs != 0ull) {
        const int owner = __ffsll((long long)longs) - 1;
        longs &= longs - 1ull;
        const int64_t lo = __shfl(beg, owner), hi = __shfl(end, owner);
        const int32_t lw = __shfl(lu, owner);
        for (int64_t c = lo; c < hi; c += 64) {
          const int64_t e = c + lane;
          bool take = false;
          int32_t v = 0;
          if (e < hi) {
            v = co[e];
            take = cc_lower(label, mark, v, lw);
            if (take) arcs += (u64)cc_degree(offs, roffs, v);
          }
          cc_append(take, v, qout, ctr + kCtrCount);
        }
      }
    }
  }
  arcs = cc_block_reduce(arcs, CcSum());
  if (threadIdx.x == 0 && arcs) atomicAdd(ctr + kCtrArcs, arcs);
}

// Pull: every remaining vertex takes the smallest label among itself and its
// neighbours; the ones whose label fell form the next active list.  Only a
// vertex's own lane writes its label in a pull iteration.
__global__ void __launch_bounds__(kCcBlock) k_cc_pull(const int32_t* __restrict__ rest, int64_t nrest,
                                                      int32_t* label, const int64_t* __restrict__ offs,
                                                      const int32_t* __restrict__ cols,
                                                      const int64_t* __restrict__ roffs,
                                                      const int32_t* __restrict__ rcols, int32_t* qout, u64* ctr) {
  __shared__ CcStage S;
  cc_stage_init(S);
  const int lane = cc_lane();
  u64 arcs = 0ull;
  const int nrows = roffs ? 2 : 1;
  for (int64_t base = (int64_t)blockIdx.x * kCcBlock; base < nrest; base += (int64_t)gridDim.x * kCcBlock) {
    const int64_t i = base + threadIdx.x;
    const bool mine = i < nrest;
    const int32_t v = mine ? rest[i] : 0;
    const int32_t lv = mine ? label[v] : 0;
    int32_t m = lv;
    for (int r = 0; r < nrows; ++r) {
      const int64_t* ro = r == 0 ? offs : roffs;
      const int32_t* co = r == 0 ? cols : rcols;
      int64_t beg = 0, end = 0;
      if (mine) {
        beg = ro[v];
        end = ro[v + 1];
      }
      const bool own = end - beg <= kCcLane;
      for (int64_t k = 0; __any(own && beg + k < end); k += kCcBatch) {
        if (own && beg + k < end) {
          int32_t u[kCcBatch];
#pragma unroll
          for (int q = 0; q < kCcBatch; ++q) u[q] = beg + k + q < end ? co[beg + k + q] : -1;
#pragma unroll
          for (int q = 0; q < kCcBatch; ++q)
            if (u[q] >= 0) m = min(m, label[u[q]]);
        }
      }
      u64 longs = __ballot(!own);
      while (longs != 0ull) {
        const int owner = __ffsll((long long)longs) - 1;
        longs &= longs - 1ull;
        const int64_t lo = __shfl(beg, owner), hi = __shfl(end, owner);
        int32_t w = 0x7fffffff;
        for (int64_t c = lo + lane; c < hi; c += 64 * 4) {
          int32_t u[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) u[q] = c + 64 * q < hi ? co[c + 64 * q] : -1;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (u[q] >= 0) w = min(w, label[u[q]]);
        }
        w = wave_min(w);
        if (lane == owner) m = min(m, w);
      }
    }
    const bool take = mine && m < lv;
    if (take) {
      label[v] = m;
      arcs += (u64)cc_degree(offs, roffs, v);
    }
    cc_stage_add(S, take, v, qout, ctr + kCtrCount);
  }
  cc_stage_flush(S, qout, ctr + kCtrCount);
  arcs = cc_block_reduce(arcs, CcSum());
  if (threadIdx.x == 0 && arcs) atomicAdd(ctr + kCtrArcs, arcs);
}

// Clears the list's bits of the mark bitmap (the only bits set after a push).
__global__ void __launch_bounds__(kCcBlock) k_cc_unmark(const int32_t* __restrict__ list, const u64* count,
                                                        u64* mark) {
  const int64_t cnt = (int64_t)*count;
  for (int64_t i = (int64_t)blockIdx.x * kCcBlock + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * kCcBlock)
    mark[list[i] >> 6] = 0ull;
}

// Components = vertices that are their own label.
__global__ void __launch_bounds__(kCcBlock) k_cc_roots(const int32_t* __restrict__ label, int64_t n, u64* roots) {
  u64 c = 0ull;
  for (int64_t v = (int64_t)blockIdx.x * kCcBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kCcBlock)
    c += label[v] == (int32_t)v ? 1ull : 0ull;
  c = cc_block_reduce(c, CcSum());
  if (threadIdx.x == 0 && c) atomicAdd(roots, c);
}

__global__ void k_cc_zero(u64* ctr, int words) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) ctr[i] = 0ull;
}

void cc_free(CcWorkspace* w) {
  if (!w) return;
  void* p[] = {w->tmp, w->rest, w->q[0], w->q[1], w->mark, w->ctr};
  for (void* x : p)
    if (x) (void)hipFree(x);
  if (w->h_ctr) (void)hipHostFree(w->h_ctr);
  for (hipEvent_t e : w->ev)
    if (e) (void)hipEventDestroy(e);
  delete w;
}

size_t cc_bytes_for(int64_t n) {
  const size_t nw = (size_t)cdiv(n, 64);
  return 4 * (size_t)n * sizeof(int32_t) + nw * sizeof(u64) + kCcCtr * sizeof(u64);
}

gsw_status ensure_cc(gsw_graph* g) {
  if (g->cc) return GSW_OK;
  CcWorkspace* w = new (std::nothrow) CcWorkspace();
  if (!w) return fail(GSW_ENOMEM, "host allocation failed");
  w->n = g->n;
  const size_t nb = (size_t)g->n * sizeof(int32_t);
  struct Item {
    void** p;
    size_t bytes;
  } items[] = {{(void**)&w->tmp, nb},
               {(void**)&w->rest, nb},
               {(void**)&w->q[0], nb},
               {(void**)&w->q[1], nb},
               {(void**)&w->mark, (size_t)cdiv(g->n, 64) * sizeof(u64)},
               {(void**)&w->ctr, kCcCtr * sizeof(u64)}};
  for (auto& it : items) {
    if (hipMalloc(it.p, it.bytes) != hipSuccess) {
      (void)hipGetLastError();
      cc_free(w);
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for connected components failed", it.bytes);
    }
    w->bytes += it.bytes;
  }
  // (the mark bitmap is cleared by every call, on its stream)
  if (hipHostMalloc((void**)&w->h_ctr, kCcCtr * sizeof(u64), hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&w->ev[0]) != hipSuccess || hipEventCreate(&w->ev[1]) != hipSuccess) {
    (void)hipGetLastError();
    cc_free(w);
    return fail(GSW_EHIP, "connected-components staging memory or events");
  }
  g->cc = w;
  return GSW_OK;
}

// Reads the counters back (waits for the stream).
gsw_status cc_read(CcWorkspace& w, hipStream_t s) {
  GSW_HIP(hipMemcpyAsync(w.h_ctr, w.ctr, kCcCtr * sizeof(u64), hipMemcpyDeviceToHost, s));
  GSW_HIP(hipStreamSynchronize(s));
  return GSW_OK;
}

void cc_row(gsw_cc_trace* t, int32_t it, int32_t kernel, int64_t n_active, int64_t e_active, int64_t changed,
            float ms) {
  t->iteration = it;
  t->kernel = kernel;
  t->n_active = n_active;
  t->e_active = e_active;
  t->changed = changed;
  t->ms = ms;
}

}  // namespace

void cc_release(gsw_graph* g) {
  cc_free(g->cc);
  g->cc = nullptr;
}

size_t cc_workspace_bytes(const gsw_graph* g) { return g->cc ? g->cc->bytes : 0; }

}  // namespace gsw

using namespace gsw;

extern "C" {

void gsw_cc_opts_default(gsw_cc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->policy = GSW_CC_SWITCH;
  o->bfs_first = 1;
  o->pull_above = 0.05f;
}

gsw_status gsw_cc(const gsw_graph* cg, int32_t* labels, int64_t* n_components, gsw_cc_trace* trace,
                  int32_t trace_cap, int32_t* trace_len, const gsw_cc_opts* opts) {
  clear_error();
  if (trace_len) *trace_len = 0;
  if (n_components) *n_components = 0;
  if (!cg || !labels) return fail(GSW_EINVAL, "null graph or labels");
  if (trace_cap < 0 || (trace_cap > 0 && !trace)) return fail(GSW_EINVAL, "trace_cap > 0 without a trace");
  gsw_cc_opts def;
  gsw_cc_opts_default(&def);
  const gsw_cc_opts* o = opts ? opts : &def;
  if (o->policy != GSW_CC_SWITCH && o->policy != GSW_CC_PUSH && o->policy != GSW_CC_PULL)
    return fail(GSW_EINVAL, "unknown components policy %d", o->policy);
  if (!(o->pull_above >= 0.0f)) return fail(GSW_EINVAL, "pull_above must be >= 0");
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  std::lock_guard<std::mutex> lock(g->mu);
  GSW_HIP(hipSetDevice(g->device));
  GSW_TRY(ensure_cc(g));
  CcWorkspace& w = *g->cc;
  const hipStream_t s = pick_stream(g, o->stream);
  const int64_t n = g->n;
  const int64_t* roffs = g->symmetric ? nullptr : g->roffs;
  const int32_t* rcols = g->symmetric ? nullptr : g->rcols;
  int32_t* lab = o->device_ptrs ? labels : w.tmp;
  int32_t rows = 0;
  auto add_row = [&](int32_t it, int32_t k, int64_t na, int64_t ea, int64_t ch, float ms) {
    if (trace && rows < trace_cap) cc_row(&trace[rows], it, k, na, ea, ch, ms);
    ++rows;
  };
  auto zero = [&]() { hipLaunchKernelGGL(k_cc_zero, dim3(1), dim3(128), 0, s, w.ctr, (int)kCcCtr); };
  auto elapsed = [&]() -> float {
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, w.ev[0], w.ev[1]);
    return ms;
  };

  // fresh memory, or a call that failed half-way, may hold marks
  GSW_HIP(hipMemsetAsync(w.mark, 0, (size_t)cdiv(n, 64) * sizeof(u64), s));
  zero();
  const bool bfs = o->bfs_first && g->symmetric && g->nnz > 0;
  if (bfs) {
    if (w.seed < 0) {
      hipLaunchKernelGGL(k_cc_argmax, dim3(cc_grid(n)), dim3(kCcBlock), 0, s, g->offs, n, w.ctr + kCtrKey);
      GSW_HIP(hipGetLastError());
      GSW_TRY(cc_read(w, s));
      w.seed = (int32_t)(0x7fffffffu - (uint32_t)(w.h_ctr[kCtrKey] & 0xffffffffull));
      zero();
    }
    const int32_t seed = w.seed;
    GSW_HIP(hipEventRecord(w.ev[0], s));
    GSW_TRY(bfs_rows_locked(g, &seed, 1, lab, o->tree, s));
    // the smallest reached id (starts at n) and the reached count
    w.h_ctr[0] = (u64)n;
    GSW_HIP(hipMemcpyAsync(w.ctr + kCtrKey, w.h_ctr, sizeof(u64), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_cc_reached, dim3(cc_grid(n)), dim3(kCcBlock), 0, s, (const int32_t*)lab, n,
                       w.ctr + kCtrKey, w.ctr + kCtrReached);
    GSW_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_cc_seed, dim3(cc_grid(n)), dim3(kCcBlock), 0, s, bfs ? (const int32_t*)lab : nullptr,
                     (const u64*)(w.ctr + kCtrKey), g->offs, roffs, n, lab, w.rest, w.ctr);
  GSW_HIP(hipGetLastError());
  if (bfs) GSW_HIP(hipEventRecord(w.ev[1], s));
  GSW_TRY(cc_read(w, s));
  const int64_t n_rest = (int64_t)w.h_ctr[kCtrCount];
  const int64_t e_rest = (int64_t)w.h_ctr[kCtrArcs];
  if (bfs) add_row(0, GSW_CC_K_BFS, 1, -1, (int64_t)w.h_ctr[kCtrReached], elapsed());

  const int32_t* act = w.rest;
  int64_t n_act = n_rest, e_act = e_rest;
  int cur = 0;
  for (int32_t it = bfs ? 1 : 0; n_act > 0; ++it) {
    int k;
    if (o->policy == GSW_CC_PUSH) k = GSW_CC_K_PUSH;
    else if (o->policy == GSW_CC_PULL) k = GSW_CC_K_PULL;
    else k = (double)e_act > (double)o->pull_above * (double)e_rest ? GSW_CC_K_PULL : GSW_CC_K_PUSH;
    int32_t* out = w.q[cur];
    zero();
    GSW_HIP(hipEventRecord(w.ev[0], s));
    if (k == GSW_CC_K_PUSH) {
      hipLaunchKernelGGL(k_cc_push, dim3(cc_grid(n_act)), dim3(kCcBlock), 0, s, act, n_act, lab, g->offs, g->cols,
                         roffs, rcols, w.mark, out, w.ctr);
      GSW_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_cc_unmark, dim3(cc_grid(n_act)), dim3(kCcBlock), 0, s, (const int32_t*)out,
                         (const u64*)(w.ctr + kCtrCount), w.mark);
    } else {
      hipLaunchKernelGGL(k_cc_pull, dim3(cc_grid(n_rest)), dim3(kCcBlock), 0, s, (const int32_t*)w.rest, n_rest,
                         lab, g->offs, g->cols, roffs, rcols, out, w.ctr);
    }
    GSW_HIP(hipGetLastError());
    GSW_HIP(hipEventRecord(w.ev[1], s));
    GSW_TRY(cc_read(w, s));
    const int64_t changed = (int64_t)w.h_ctr[kCtrCount];
    add_row(it, k, n_act, e_act, changed, elapsed());
    act = out;
    n_act = changed;
    e_act = (int64_t)w.h_ctr[kCtrArcs];
    cur ^= 1;
  }
  zero();
  hipLaunchKernelGGL(k_cc_roots, dim3(cc_grid(n)), dim3(kCcBlock), 0, s, (const int32_t*)lab, n, w.ctr + kCtrRoots);
  GSW_HIP(hipGetLastError());
  if (!o->device_ptrs)
    GSW_HIP(hipMemcpyAsync(labels, lab, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GSW_TRY(cc_read(w, s));
  if (n_components) *n_components = (int64_t)w.h_ctr[kCtrRoots];
  if (trace_len) *trace_len = rows;
  return GSW_OK;
}

}  // extern "C"
