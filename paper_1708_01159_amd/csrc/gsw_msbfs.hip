// Batched multi-source BFS: up to 1024 sources traverse one graph together.
//
// Every vertex carries W = ceil(B/64) 64-bit masks, one bit per source:
// visited, frontier (depth d) and next frontier (depth d+1).  A level is
// either top-down (each frontier vertex ORs its frontier mask, minus what a
// neighbour has already seen, into the neighbour's next mask) or bottom-up
// (each vertex with unvisited sources ORs its neighbours' frontier masks and
// stops once every unvisited source is covered).  One pass over the edges
// thus advances every source whose frontier touches them: the edge stream is
// shared by the whole batch.  The per-source result is the same hop distance
// as a single-source BFS (Section III-A); levels are stored as int8 (-1 =
// unreachable) and a depth above 127 is reported as a range error.
//
// Layout: masks are vertex-major ([n][W] words, one 128-byte line per vertex
// at B = 1024), worked on by groups of W lanes (lane j owns word j) so a
// vertex's masks are read and written coalesced.  Levels are kept
// vertex-major ([n][B] bytes, each lane writing its own 64-byte run) and
// transposed to [B][n] at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "gsw_internal.h"

namespace gsw {
namespace {

typedef unsigned long long u64;

constexpr int kMsBlock = 256;
constexpr int kMsMaxGrid = 2048;
constexpr int kMsStats = 8;        // stat counters, spread like the queue bins
constexpr int kMsStatStride = 32;  // u64 words between counters

struct MsArgs {
  const int64_t* __restrict__ offs;
  const int32_t* __restrict__ cols;
  u64* vis;
  const u64* __restrict__ fr;  // depth-d masks
  u64* frn;                    // depth-(d+1) masks (written for every vertex)
  u64* nx;                     // top-down scratch: ORed masks, zero between levels
  int8_t* lev;                 // [n][B] levels, vertex-major
  u64* stats;                  // [kMsStats][2]: vertices with new bits, their degree sum
  int64_t n;
  int32_t W, B;                // words per vertex, sources
  int32_t d;
  // serving sessions: int32 levels per slot ([slots][n]), level = d + 1 -
  // start[slot] where d is the session's iteration; OR of the new frontier
  // masks per word (which slots are still running), spread over kMsStats rows
  int32_t* dist;
  const int32_t* start;
  u64* active;
};

constexpr int kMaxWords = GSW_MSBFS_MAX_SOURCES / 64;  // mask words per vertex at most

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Sources with bit positions >= B in the last word do not exist: treat them
// as visited so they never look unreached.
__device__ __forceinline__ u64 valid_bits(int j, int W, int B) {
  if (j < W - 1 || (B & 63) == 0) return ~0ull;
  return (1ull << (B & 63)) - 1ull;
}

// Levels d+1 for the sources in `m` at vertex v, word j.
__device__ __forceinline__ void write_levels(const MsArgs& a, int64_t v, int j, u64 m) {
  if (a.dist) {
    while (m) {
      const int b = __ffsll((long long)m) - 1;
      m &= m - 1ull;
      const int slot = j * 64 + b;
      a.dist[(int64_t)slot * a.n + v] = a.d + 1 - a.start[slot];
    }
    return;
  }
  int8_t* row = a.lev + v * (int64_t)a.B + (int64_t)j * 64;
  const int8_t val = (int8_t)(a.d + 1 > 127 ? 127 : a.d + 1);
  while (m) {
    const int b = __ffsll((long long)m) - 1;
    m &= m - 1ull;
    row[b] = val;
  }
}

// Block-wide sums of (vertices with new sources, their degree), one atomic
// per block into one of kMsStats spread counters.
__device__ __forceinline__ void add_stats(const MsArgs& a, u64 nv, u64 ne) {
  __shared__ u64 s_v, s_e;
  if (threadIdx.x == 0) {
    s_v = 0ull;
    s_e = 0ull;
  }
  __syncthreads();
  // wave reduction, then one LDS atomic per wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nv += __shfl_xor(nv, off);
    ne += __shfl_xor(ne, off);
  }
  if (lane_id() == 0 && (nv | ne)) {
    atomicAdd(&s_v, nv);
    atomicAdd(&s_e, ne);
  }
  __syncthreads();
  if (threadIdx.x == 0 && (s_v | s_e)) {
    u64* c = a.stats + (size_t)(blockIdx.x % kMsStats) * kMsStatStride;
    atomicAdd(c, s_v);
    atomicAdd(c + 1, s_e);
  }
}

// Sessions: OR of this lane's new-frontier words into the active masks
// (LDS per block, then one atomic per word into the block's spread row).
__device__ __forceinline__ void add_active(const MsArgs& a, int j, u64 act) {
  if (!a.active) return;
  __shared__ u64 s_act[kMaxWords];
  if (threadIdx.x < kMaxWords) s_act[threadIdx.x] = 0ull;
  __syncthreads();
  if (act) atomicOr(&s_act[j], act);
  __syncthreads();
  if (threadIdx.x < (unsigned)a.W && s_act[threadIdx.x])
    atomicOr(a.active + (size_t)(blockIdx.x % kMsStats) * kMaxWords + threadIdx.x, s_act[threadIdx.x]);
}

// Group geometry: groups of G = W (rounded to a power of two, at most 64)
// lanes, one vertex per group.
struct Group {
  int G, sub, first;  // lanes per group, lane within group, first lane of group in the wave
  int64_t gid, ngroups;
};

__device__ __forceinline__ Group group_of(int G) {
  Group g;
  g.G = G;
  const int lane = lane_id();
  g.sub = lane & (G - 1);
  g.first = lane & ~(G - 1);
  const int64_t tid = (int64_t)blockIdx.x * kMsBlock + threadIdx.x;
  g.gid = tid / G;
  g.ngroups = (int64_t)gridDim.x * kMsBlock / G;
  return g;
}

// OR of a per-lane flag over the lanes of this lane's group.
__device__ __forceinline__ bool group_any(bool x, const Group& g) {
  const u64 m = __ballot(x);
  const u64 gm = g.G == 64 ? ~0ull : (((1ull << g.G) - 1ull) << g.first);
  return (m & gm) != 0ull;
}

__device__ __forceinline__ bool group_all(bool x, const Group& g) {
  const u64 m = __ballot(x);
  const u64 gm = g.G == 64 ? ~0ull : (((1ull << g.G) - 1ull) << g.first);
  return (m & gm) == gm;
}

// ------------------------------------------------------------------ init
// Masks of n vertices (bits of sources >= nsrc start visited) and levels
// [n][brow] set to -1 (brow = 64 W, so rows are whole 8-byte words).
__global__ void __launch_bounds__(kMsBlock) k_ms_init(u64* vis, u64* fr, u64* nx, int8_t* lev,
                                                      int64_t n, int W, int nsrc, int brow) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  const int64_t gid = (int64_t)blockIdx.x * kMsBlock + threadIdx.x;
  const int64_t words = n * W;
  for (int64_t i = gid; i < words; i += stride) {
    const int j = (int)(i % W);
    vis[i] = ~valid_bits(j, W, nsrc);
    fr[i] = 0ull;
    nx[i] = 0ull;
  }
  const int64_t lw = n * (int64_t)brow / 8;
  u64* l8 = reinterpret_cast<u64*>(lev);
  for (int64_t i = gid; i < lw; i += stride) l8[i] = ~0ull;
}

// Sources are set after init (a separate launch, so no ordering issue).
__global__ void k_ms_sources(u64* vis, u64* fr, int8_t* lev, int W, int B,
                             const int32_t* __restrict__ src, int nsrc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsrc) return;
  const int64_t s = src[i];
  const u64 bit = 1ull << (i & 63);
  atomicOr(vis + s * W + (i >> 6), bit);
  atomicOr(fr + s * W + (i >> 6), bit);
  lev[s * (int64_t)B + i] = 0;
}

// --------------------------------------------------------------- top-down
// Group per frontier vertex u (grid-stride); for each neighbour v, lane j
// ORs fr[u][j] & ~vis[v][j] into nx[v][j].
__global__ void __launch_bounds__(kMsBlock) k_ms_push(MsArgs a, int G) {
  const Group g = group_of(G);
  const int j = g.sub;
  const bool lane_live = j < a.W;
  for (int64_t u = g.gid; u < a.n; u += g.ngroups) {
    const u64 f = lane_live ? a.fr[u * a.W + j] : 0ull;
    if (!group_any(f != 0ull, g)) continue;  // u is in no source's frontier
    const int64_t end = a.offs[u + 1];
    for (int64_t e = a.offs[u]; e < end; ++e) {
      const int64_t v = a.cols[e];
      if (f) {
        const u64 m = f & ~a.vis[v * a.W + j];
        if (m) atomicOr(a.nx + v * a.W + j, m);
      }
    }
  }
}

// After a top-down level: new = nx & ~vis, then vis |= new, frn = new,
// nx = 0, levels for the new bits, and the level's statistics.
__global__ void __launch_bounds__(kMsBlock) k_ms_update(MsArgs a, int G) {
  const Group g = group_of(G);
  const int j = g.sub;
  const bool lane_live = j < a.W;
  u64 nv = 0, ne = 0, act = 0;
  for (int64_t v = g.gid; v < a.n; v += g.ngroups) {
    u64 nw = 0ull;
    if (lane_live) {
      const int64_t i = v * a.W + j;
      const u64 x = a.nx[i];
      const u64 s = a.vis[i];
      nw = x & ~s;
      if (x) a.nx[i] = 0ull;
      if (nw) {
        a.vis[i] = s | nw;
        write_levels(a, v, j, nw);
      }
      a.frn[i] = nw;
      act |= nw;
    }
    if (group_any(nw != 0ull, g) && g.sub == 0) {
      nv += 1;
      ne += (u64)(a.offs[v + 1] - a.offs[v]);
    }
  }
  add_stats(a, nv, ne);
  add_active(a, j, act);
}

// -------------------------------------------------------------- bottom-up
// Group per vertex v with unvisited sources: OR the neighbours' frontier
// masks restricted to what v still needs, stop when every needed source is
// covered; v's own masks are updated in place (v's group is their only
// writer), frn is written for every vertex.
__global__ void __launch_bounds__(kMsBlock) k_ms_pull(MsArgs a, int G) {
  const Group g = group_of(G);
  const int j = g.sub;
  const bool lane_live = j < a.W;
  u64 nv = 0, ne = 0, act = 0;
  for (int64_t v = g.gid; v < a.n; v += g.ngroups) {
    const int64_t i = v * a.W + j;
    const u64 s = lane_live ? a.vis[i] : ~0ull;
    const u64 need = ~s;
    u64 acc = 0ull;
    if (group_any(need != 0ull, g)) {
      const int64_t end = a.offs[v + 1];
      for (int64_t e = a.offs[v]; e < end; ++e) {
        const int64_t u = a.cols[e];
        if (lane_live && need) acc |= a.fr[u * a.W + j] & need;
        if (group_all(acc == need, g)) break;
      }
    }
    if (lane_live) {
      if (acc) {
        a.vis[i] = s | acc;
        write_levels(a, v, j, acc);
      }
      a.frn[i] = acc;
      act |= acc;
    }
    if (group_any(acc != 0ull, g) && g.sub == 0) {
      nv += 1;
      ne += (u64)(a.offs[v + 1] - a.offs[v]);
    }
  }
  add_stats(a, nv, ne);
  add_active(a, j, act);
}

// Sum of the spread statistics counters to mapped host memory, then zero.
__global__ void k_ms_finalize(u64* stats, u64* host) {
  const int lane = lane_id();
  u64 v = 0, e = 0;
  if (lane < kMsStats) {
    v = stats[lane * kMsStatStride];
    e = stats[lane * kMsStatStride + 1];
    stats[lane * kMsStatStride] = 0ull;
    stats[lane * kMsStatStride + 1] = 0ull;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_xor(v, off);
    e += __shfl_xor(e, off);
  }
  if (lane == 0) {
    __hip_atomic_store(host + 1, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(host, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// [n][B] -> [nsrc][n] levels through 64x64-byte LDS tiles.
__global__ void __launch_bounds__(256) k_ms_transpose(const int8_t* __restrict__ in,
                                                      int8_t* __restrict__ out, int64_t n, int B,
                                                      int nsrc) {
  __shared__ int8_t tile[64][65];
  const int64_t v0 = (int64_t)blockIdx.x * 64;
  const int s0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int r = ty; r < 64; r += 4) {
    const int64_t v = v0 + r;
    const int s = s0 + tx;
    tile[r][tx] = (v < n && s < B) ? in[v * B + s] : (int8_t)-1;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int s = s0 + r;
    const int64_t v = v0 + tx;
    if (s < nsrc && v < n) out[(int64_t)s * n + v] = tile[tx][r];
  }
}

// ------------------------------------------------------------- sessions
// vis = (vis & ~clr) | set on every vertex: slots being admitted start
// unvisited everywhere, freed slots become inert (visited everywhere).
__global__ void __launch_bounds__(kMsBlock) k_ss_masks(u64* vis, int64_t n, int W,
                                                       const u64* __restrict__ clr,
                                                       const u64* __restrict__ set) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  for (int64_t i = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; i < n * W; i += stride) {
    const int j = (int)(i % W);
    vis[i] = (vis[i] & ~clr[j]) | set[j];
  }
}

// Admitted slots: the source's bit in vis and in the current frontier, level 0.
__global__ void k_ss_seed(u64* vis, u64* fr, int32_t* dist, int64_t n, int W,
                          const int32_t* __restrict__ src, const int32_t* __restrict__ slot,
                          int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t s = src[i];
  const int k = slot[i];
  const u64 bit = 1ull << (k & 63);
  atomicOr(vis + s * W + (k >> 6), bit);
  atomicOr(fr + s * W + (k >> 6), bit);
  dist[(int64_t)k * n + s] = 0;
}

__global__ void __launch_bounds__(kMsBlock) k_ss_fill(int32_t* p, int64_t count, int32_t val) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  for (int64_t i = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; i < count; i += stride) p[i] = val;
}

// Level statistics and the OR of the active rows to mapped host memory
// ([0] vertices with new bits, [1] their degree sum, [2 + j] active word j),
// then zero.  [0] is stored last.
__global__ void k_ss_finalize(u64* stats, u64* active, int W, u64* host) {
  const int lane = lane_id();
  u64 v = 0, e = 0;
  if (lane < kMsStats) {
    v = stats[lane * kMsStatStride];
    e = stats[lane * kMsStatStride + 1];
    stats[lane * kMsStatStride] = 0ull;
    stats[lane * kMsStatStride + 1] = 0ull;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_xor(v, off);
    e += __shfl_xor(e, off);
  }
  if (lane < W) {
    u64 x = 0ull;
    for (int b = 0; b < kMsStats; ++b) {
      x |= active[b * kMaxWords + lane];
      active[b * kMaxWords + lane] = 0ull;
    }
    __hip_atomic_store(host + 2 + lane, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __syncthreads();
  if (lane == 0) {
    __hip_atomic_store(host + 1, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(host, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int group_lanes(int W) {
  int G = 1;
  while (G < W) G <<= 1;
  return G;  // W <= 16 -> G <= 16
}

inline unsigned ms_grid(int64_t groups, int G) {
  const int64_t blocks = cdiv(groups * G, kMsBlock);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, kMsMaxGrid));
}

}  // namespace

struct MsWorkspace {
  int64_t n = 0;
  int W = 0, B = 0;
  u64 *vis = nullptr, *fr = nullptr, *frn = nullptr, *nx = nullptr, *stats = nullptr;
  int8_t* lev = nullptr;
  int32_t* src = nullptr;
  u64* h_stats = nullptr;  // mapped host memory
  u64* d_hstats = nullptr;
  size_t bytes = 0;
};

namespace {
void ms_free(MsWorkspace* m) {
  if (!m) return;
  void* p[] = {m->vis, m->fr, m->frn, m->nx, m->stats, m->lev, m->src};
  for (void* x : p)
    if (x) (void)hipFree(x);
  if (m->h_stats) (void)hipHostFree(m->h_stats);
  delete m;
}

gsw_status ms_ensure(gsw_graph* g, int W, int B) {
  MsWorkspace*& m = g->ms;
  if (m && m->W >= W && m->B >= B) return GSW_OK;
  ms_free(m);
  m = new (std::nothrow) MsWorkspace();
  if (!m) return fail(GSW_ENOMEM, "host allocation failed");
  m->n = g->n;
  m->W = W;
  m->B = W * 64;
  const size_t mb = (size_t)g->n * W * sizeof(u64);
  struct Item {
    void** p;
    size_t bytes;
  } items[] = {{(void**)&m->vis, mb},
               {(void**)&m->fr, mb},
               {(void**)&m->frn, mb},
               {(void**)&m->nx, mb},
               {(void**)&m->stats, (size_t)kMsStats * kMsStatStride * sizeof(u64)},
               {(void**)&m->lev, (size_t)g->n * m->B},
               {(void**)&m->src, (size_t)m->B * sizeof(int32_t)}};
  for (auto& it : items) {
    hipError_t e = hipMalloc(it.p, it.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ms_free(m);
      m = nullptr;
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for the batched BFS failed", it.bytes);
    }
    m->bytes += it.bytes;
  }
  GSW_HIP(hipMemset(m->stats, 0, (size_t)kMsStats * kMsStatStride * sizeof(u64)));
  GSW_HIP(hipHostMalloc((void**)&m->h_stats, 64 * sizeof(u64),
                        hipHostMallocMapped | hipHostMallocCoherent));
  GSW_HIP(hipHostGetDevicePointer((void**)&m->d_hstats, m->h_stats, 0));
  return GSW_OK;
}

gsw_status ms_wait(MsWorkspace* m, hipStream_t s, u64* nv, u64* ne) {
  volatile u64* f = m->h_stats;
  for (uint64_t it = 0;; ++it) {
    const u64 v = f[0];
    if (v != ~0ull) {
      *nv = v;
      *ne = f[1];
      return GSW_OK;
    }
    if ((it & 4095u) == 4095u) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (f[0] != ~0ull) continue;
        return fail(GSW_EHIP, "batched level finished without reporting its statistics");
      }
      if (e != hipErrorNotReady) return fail(GSW_EHIP, "batched BFS: %s", hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
}
}  // namespace

void ms_release(gsw_graph* g) {
  ms_free(g->ms);
  g->ms = nullptr;
}

}  // namespace gsw

using namespace gsw;

extern "C" {

void gsw_msbfs_opts_default(gsw_msbfs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->push_to_pull = 0.05f;
  o->pull_to_push = 0.01f;
}

gsw_status gsw_msbfs(const gsw_graph* cg, const int32_t* sources, int32_t n_sources, int8_t* levels,
                     int32_t* n_levels, const gsw_msbfs_opts* opts) {
  clear_error();
  if (n_levels) *n_levels = 0;
  if (!cg || !sources || !levels) return fail(GSW_EINVAL, "null graph, sources or levels");
  if (n_sources < 1 || n_sources > GSW_MSBFS_MAX_SOURCES)
    return fail(GSW_EINVAL, "n_sources=%d out of [1, %d]", n_sources, GSW_MSBFS_MAX_SOURCES);
  gsw_msbfs_opts def;
  gsw_msbfs_opts_default(&def);
  const gsw_msbfs_opts* o = opts ? opts : &def;
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= g->n)
      return fail(GSW_EINVAL, "source %d (index %d) out of [0, %lld)", sources[i], i, (long long)g->n);
  std::lock_guard<std::mutex> lock(g->mu);
  GSW_HIP(hipSetDevice(g->device));
  const bool pull_ok = g->symmetric != 0;
  const int W = (n_sources + 63) / 64;
  GSW_TRY(ms_ensure(g, W, W * 64));
  MsWorkspace* m = g->ms;
  const hipStream_t s = pick_stream(g, o->stream);
  const int B = W * 64;  // level rows per vertex in the workspace
  const int G = group_lanes(W);
  GSW_HIP(hipMemcpyAsync(m->src, sources, (size_t)n_sources * sizeof(int32_t), hipMemcpyHostToDevice, s));
  {
    const int64_t work = std::max<int64_t>(g->n * W, g->n * (int64_t)B / 8);
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(work, kMsBlock), 65536);
    hipLaunchKernelGGL(k_ms_init, dim3(grid), dim3(kMsBlock), 0, s, m->vis, m->fr, m->nx, m->lev,
                       g->n, W, n_sources, B);
    hipLaunchKernelGGL(k_ms_sources, dim3((unsigned)cdiv(n_sources, 256)), dim3(256), 0, s, m->vis,
                       m->fr, m->lev, W, B, (const int32_t*)m->src, n_sources);
    GSW_HIP(hipGetLastError());
  }
  MsArgs a;
  a.offs = g->offs;
  a.cols = g->cols;
  a.vis = m->vis;
  a.lev = m->lev;
  a.stats = m->stats;
  a.dist = nullptr;
  a.start = nullptr;
  a.active = nullptr;
  a.n = g->n;
  a.W = W;
  a.B = B;
  u64* cur = m->fr;
  u64* nxt = m->frn;
  // frontier statistics of depth 0 (for the direction choice)
  u64 nf = 0, ef = 0;
  {
    std::vector<int32_t> uniq(sources, sources + n_sources);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    nf = uniq.size();
  }
  bool pull = false;
  const double nnz = (double)std::max<int64_t>(g->nnz, 1);
  int32_t d = 0;
  for (;; ++d) {
    // direction: pull once the frontier's edges are a large share of all
    // arcs, back to push when the frontier is small again
    if (pull_ok) {
      if (!pull && ef > (u64)(o->push_to_pull * nnz)) pull = true;
      else if (pull && ef < (u64)(o->pull_to_push * nnz)) pull = false;
    }
    a.fr = cur;
    a.frn = nxt;
    a.nx = m->nx;
    a.d = d;
    m->h_stats[0] = ~0ull;
    if (pull) {
      hipLaunchKernelGGL(k_ms_pull, dim3(ms_grid(g->n, G)), dim3(kMsBlock), 0, s, a, G);
    } else {
      hipLaunchKernelGGL(k_ms_push, dim3(ms_grid(g->n, G)), dim3(kMsBlock), 0, s, a, G);
      hipLaunchKernelGGL(k_ms_update, dim3(ms_grid(g->n, G)), dim3(kMsBlock), 0, s, a, G);
    }
    hipLaunchKernelGGL(k_ms_finalize, dim3(1), dim3(64), 0, s, m->stats, m->d_hstats);
    GSW_HIP(hipGetLastError());
    u64 nv = 0, ne = 0;
    GSW_TRY(ms_wait(m, s, &nv, &ne));
    if (nv == 0) break;
    if (d + 1 > GSW_MSBFS_LEVEL_CAP)
      return fail(GSW_ERANGE, "a source reaches depth %d > %d (int8 levels)", d + 1, GSW_MSBFS_LEVEL_CAP);
    nf = nv;
    ef = ne;
    std::swap(cur, nxt);
  }
  if (n_levels) *n_levels = d + 1;
  // [n][B] -> [n_sources][n]
  int8_t* out = levels;
  int8_t* tmp = nullptr;
  if (!o->device_ptrs) {
    GSW_HIP(hipMalloc((void**)&tmp, (size_t)n_sources * g->n));
    out = tmp;
  }
  hipLaunchKernelGGL(k_ms_transpose, dim3((unsigned)cdiv(g->n, 64), (unsigned)cdiv(n_sources, 64)),
                     dim3(256), 0, s, (const int8_t*)m->lev, out, g->n, B, n_sources);
  gsw_status st = GSW_OK;
  if (hipGetLastError() != hipSuccess) st = fail(GSW_EHIP, "transpose launch failed");
  if (st == GSW_OK && tmp) {
    if (hipMemcpyAsync(levels, tmp, (size_t)n_sources * g->n, hipMemcpyDeviceToHost, s) != hipSuccess)
      st = fail(GSW_EHIP, "copying levels to the host failed");
  }
  if (hipStreamSynchronize(s) != hipSuccess && st == GSW_OK) st = fail(GSW_EHIP, "stream synchronize failed");
  if (tmp) (void)hipFree(tmp);
  (void)nf;
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------ sessions
struct gsw_session {
  gsw_graph* g = nullptr;
  int W = 0, slots = 0;
  u64 *vis = nullptr, *fr = nullptr, *frn = nullptr, *nx = nullptr;
  u64 *stats = nullptr, *active = nullptr, *masks = nullptr;  // masks: clr[W] then set[W]
  int32_t *dist = nullptr, *start_d = nullptr, *seed = nullptr;  // seed: src[slots] then slot[slots]
  u64 *h_stats = nullptr, *d_hstats = nullptr;
  std::vector<int32_t> start_h, source;
  std::vector<int8_t> state;  // 0 free, 1 admitted (seeded at the next step), 2 running, 3 finished
  std::vector<u64> freed;     // slots freed since the last step (made inert then)
  int64_t it = 0;             // levels run by this session
  u64 ef = 0;
  bool pull = false;
  float push_to_pull = 0.05f, pull_to_push = 0.01f;
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  std::mutex mu;
};

namespace {

void ss_free(gsw_session* ss) {
  if (!ss) return;
  void* p[] = {ss->vis, ss->fr, ss->frn, ss->nx, ss->stats, ss->active, ss->masks, ss->dist,
               ss->start_d, ss->seed};
  for (void* x : p)
    if (x) (void)hipFree(x);
  if (ss->h_stats) (void)hipHostFree(ss->h_stats);
  if (ss->stream) (void)hipStreamDestroy(ss->stream);
  delete ss;
}

gsw_status ss_wait(gsw_session* ss, u64* nv, u64* ne) {
  volatile u64* f = ss->h_stats;
  for (uint64_t k = 0;; ++k) {
    if (f[0] != ~0ull) {
      *nv = f[0];
      *ne = f[1];
      return GSW_OK;
    }
    if ((k & 4095u) == 4095u) {
      const hipError_t e = hipStreamQuery(ss->stream);
      if (e == hipSuccess) {
        if (f[0] != ~0ull) continue;
        return fail(GSW_EHIP, "session level finished without reporting its statistics");
      }
      if (e != hipErrorNotReady) return fail(GSW_EHIP, "session: %s", hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
}

}  // namespace

extern "C" {

gsw_status gsw_session_create(const gsw_graph* cg, int32_t max_slots, gsw_session** out) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  *out = nullptr;
  if (!cg) return fail(GSW_EINVAL, "graph is null");
  if (max_slots < 1 || max_slots > GSW_MSBFS_MAX_SOURCES)
    return fail(GSW_EINVAL, "max_slots=%d out of [1, %d]", max_slots, GSW_MSBFS_MAX_SOURCES);
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  GSW_HIP(hipSetDevice(g->device));
  gsw_session* ss = new (std::nothrow) gsw_session();
  if (!ss) return fail(GSW_ENOMEM, "host allocation failed");
  ss->g = g;
  ss->W = (max_slots + 63) / 64;
  ss->slots = max_slots;
  const int64_t n = g->n;
  const size_t mb = (size_t)n * ss->W * sizeof(u64);
  struct Item {
    void** p;
    size_t bytes;
  } items[] = {{(void**)&ss->vis, mb},
               {(void**)&ss->fr, mb},
               {(void**)&ss->frn, mb},
               {(void**)&ss->nx, mb},
               {(void**)&ss->stats, (size_t)kMsStats * kMsStatStride * sizeof(u64)},
               {(void**)&ss->active, (size_t)kMsStats * kMaxWords * sizeof(u64)},
               {(void**)&ss->masks, 2 * (size_t)kMaxWords * sizeof(u64)},
               {(void**)&ss->dist, (size_t)max_slots * n * sizeof(int32_t)},
               {(void**)&ss->start_d, (size_t)max_slots * sizeof(int32_t)},
               {(void**)&ss->seed, 2 * (size_t)max_slots * sizeof(int32_t)}};
  for (auto& it : items) {
    hipError_t e = hipMalloc(it.p, it.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ss_free(ss);
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for a session failed", it.bytes);
    }
    ss->bytes += it.bytes;
  }
  gsw_status st = GSW_OK;
  if (hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&ss->h_stats, 64 * sizeof(u64), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&ss->d_hstats, ss->h_stats, 0) != hipSuccess)
    st = fail(GSW_EHIP, "session stream or mapped memory");
  if (st == GSW_OK) {
    const hipStream_t s = ss->stream;
    // every slot starts inert: visited everywhere, in no frontier, levels -1
    if (hipMemsetAsync(ss->vis, 0xff, mb, s) != hipSuccess || hipMemsetAsync(ss->fr, 0, mb, s) != hipSuccess ||
        hipMemsetAsync(ss->frn, 0, mb, s) != hipSuccess || hipMemsetAsync(ss->nx, 0, mb, s) != hipSuccess ||
        hipMemsetAsync(ss->stats, 0, (size_t)kMsStats * kMsStatStride * sizeof(u64), s) != hipSuccess ||
        hipMemsetAsync(ss->active, 0, (size_t)kMsStats * kMaxWords * sizeof(u64), s) != hipSuccess ||
        hipMemsetAsync(ss->dist, 0xff, (size_t)max_slots * n * sizeof(int32_t), s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(GSW_EHIP, "session initialisation failed");
  }
  if (st != GSW_OK) {
    ss_free(ss);
    return st;
  }
  ss->start_h.assign((size_t)max_slots, 0);
  ss->source.assign((size_t)max_slots, -1);
  ss->state.assign((size_t)max_slots, 0);
  ss->freed.assign((size_t)ss->W, 0ull);
  *out = ss;
  return GSW_OK;
}

void gsw_session_destroy(gsw_session* ss) { ss_free(ss); }

gsw_status gsw_session_admit(gsw_session* ss, int32_t source, int32_t* slot) {
  clear_error();
  if (!ss || !slot) return fail(GSW_EINVAL, "null argument");
  if (source < 0 || source >= ss->g->n) return fail(GSW_EINVAL, "source %d out of range", source);
  std::lock_guard<std::mutex> lock(ss->mu);
  for (int k = 0; k < ss->slots; ++k) {
    if (ss->state[(size_t)k] == 0) {
      ss->state[(size_t)k] = 1;
      ss->source[(size_t)k] = source;
      ss->start_h[(size_t)k] = (int32_t)ss->it;
      *slot = k;
      return GSW_OK;
    }
  }
  return fail(GSW_EBUSY, "all %d slots are in use", ss->slots);
}

gsw_status gsw_session_step(gsw_session* ss, int32_t max_levels, int32_t* finished, int32_t finished_cap,
                            int32_t* n_finished, int32_t* levels_run) {
  clear_error();
  if (n_finished) *n_finished = 0;
  if (levels_run) *levels_run = 0;
  if (!ss || max_levels < 1 || (finished_cap > 0 && !finished)) return fail(GSW_EINVAL, "bad step arguments");
  std::lock_guard<std::mutex> lock(ss->mu);
  gsw_graph* g = ss->g;
  GSW_HIP(hipSetDevice(g->device));
  const hipStream_t s = ss->stream;
  const int W = ss->W;
  const int64_t n = g->n;
  // admit: clear the admitted slots' bits, make freed slots inert, seed sources
  std::vector<u64> msk(2 * (size_t)kMaxWords, 0ull);
  std::vector<int32_t> seed_src, seed_slot;
  for (int k = 0; k < ss->slots; ++k)
    if (ss->state[(size_t)k] == 1) {
      msk[(size_t)(k >> 6)] |= 1ull << (k & 63);
      seed_src.push_back(ss->source[(size_t)k]);
      seed_slot.push_back(k);
    }
  bool any_mask = !seed_src.empty();
  for (int j = 0; j < W; ++j) {
    msk[(size_t)kMaxWords + j] = ss->freed[(size_t)j] & ~msk[(size_t)j];
    any_mask = any_mask || msk[(size_t)kMaxWords + j];
    ss->freed[(size_t)j] = 0ull;
  }
  const int G = group_lanes(W);
  if (any_mask) {
    GSW_HIP(hipMemcpyAsync(ss->masks, msk.data(), msk.size() * sizeof(u64), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ss_masks, dim3((unsigned)std::min<int64_t>(cdiv(n * W, kMsBlock), 65536)),
                       dim3(kMsBlock), 0, s, ss->vis, n, W, (const u64*)ss->masks,
                       (const u64*)(ss->masks + kMaxWords));
  }
  if (!seed_src.empty()) {
    const int c = (int)seed_src.size();
    GSW_HIP(hipMemcpyAsync(ss->seed, seed_src.data(), c * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GSW_HIP(hipMemcpyAsync(ss->seed + ss->slots, seed_slot.data(), c * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GSW_HIP(hipMemcpyAsync(ss->start_d, ss->start_h.data(), ss->slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ss_seed, dim3((unsigned)cdiv(c, 256)), dim3(256), 0, s, ss->vis, ss->fr, ss->dist, n,
                       W, (const int32_t*)ss->seed, (const int32_t*)(ss->seed + ss->slots), c);
    for (int32_t k : seed_slot) ss->state[(size_t)k] = 2;
  }
  GSW_HIP(hipGetLastError());
  MsArgs a;
  a.offs = g->offs;
  a.cols = g->cols;
  a.vis = ss->vis;
  a.nx = ss->nx;
  a.lev = nullptr;
  a.stats = ss->stats;
  a.n = n;
  a.W = W;
  a.B = W * 64;
  a.dist = ss->dist;
  a.start = ss->start_d;
  a.active = ss->active;
  const bool pull_ok = g->symmetric != 0;
  const double nnz = (double)std::max<int64_t>(g->nnz, 1);
  int32_t nfin = 0, run = 0;
  for (; run < max_levels; ++run) {
    bool running = false;
    for (int k = 0; k < ss->slots && !running; ++k) running = ss->state[(size_t)k] == 2;
    if (!running) break;
    if (pull_ok) {
      if (!ss->pull && ss->ef > (u64)(ss->push_to_pull * nnz)) ss->pull = true;
      else if (ss->pull && ss->ef < (u64)(ss->pull_to_push * nnz)) ss->pull = false;
    } else {
      ss->pull = false;
    }
    a.fr = ss->fr;
    a.frn = ss->frn;
    a.d = (int32_t)ss->it;
    ss->h_stats[0] = ~0ull;
    if (ss->pull) {
      hipLaunchKernelGGL(k_ms_pull, dim3(ms_grid(n, G)), dim3(kMsBlock), 0, s, a, G);
    } else {
      hipLaunchKernelGGL(k_ms_push, dim3(ms_grid(n, G)), dim3(kMsBlock), 0, s, a, G);
      hipLaunchKernelGGL(k_ms_update, dim3(ms_grid(n, G)), dim3(kMsBlock), 0, s, a, G);
    }
    hipLaunchKernelGGL(k_ss_finalize, dim3(1), dim3(64), 0, s, ss->stats, ss->active, W, ss->d_hstats);
    GSW_HIP(hipGetLastError());
    u64 nv = 0, ne = 0;
    GSW_TRY(ss_wait(ss, &nv, &ne));
    ss->it += 1;
    ss->ef = ne;
    std::swap(ss->fr, ss->frn);
    volatile u64* act = ss->h_stats + 2;
    for (int k = 0; k < ss->slots; ++k) {
      if (ss->state[(size_t)k] != 2) continue;
      if (((act[k >> 6] >> (k & 63)) & 1ull) == 0ull) {
        ss->state[(size_t)k] = 3;
        if (nfin < finished_cap) finished[nfin] = k;
        ++nfin;
      }
    }
    if (nfin > 0) {
      ++run;
      break;
    }
  }
  if (n_finished) *n_finished = nfin;
  if (levels_run) *levels_run = run;
  return GSW_OK;
}

gsw_status gsw_session_fetch(gsw_session* ss, int32_t slot, int32_t* levels, int32_t device_ptr) {
  clear_error();
  if (!ss || !levels) return fail(GSW_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(ss->mu);
  if (slot < 0 || slot >= ss->slots || ss->state[(size_t)slot] != 3)
    return fail(GSW_EINVAL, "slot %d has no finished result", slot);
  GSW_HIP(hipSetDevice(ss->g->device));
  const hipStream_t s = ss->stream;
  const int64_t n = ss->g->n;
  int32_t* row = ss->dist + (int64_t)slot * n;
  GSW_HIP(hipMemcpyAsync(levels, row, (size_t)n * sizeof(int32_t),
                         device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  hipLaunchKernelGGL(k_ss_fill, dim3((unsigned)std::min<int64_t>(cdiv(n, kMsBlock), 65536)), dim3(kMsBlock), 0,
                     s, row, n, -1);
  GSW_HIP(hipGetLastError());
  GSW_HIP(hipStreamSynchronize(s));
  ss->state[(size_t)slot] = 0;
  ss->source[(size_t)slot] = -1;
  ss->freed[(size_t)(slot >> 6)] |= 1ull << (slot & 63);
  return GSW_OK;
}

gsw_status gsw_session_info(const gsw_session* ss, int32_t* slots, int32_t* busy, int64_t* iteration,
                            size_t* dev_bytes) {
  clear_error();
  if (!ss) return fail(GSW_EINVAL, "session is null");
  if (slots) *slots = ss->slots;
  if (busy) {
    int32_t b = 0;
    for (int8_t x : ss->state) b += x != 0;
    *busy = b;
  }
  if (iteration) *iteration = ss->it;
  if (dev_bytes) *dev_bytes = ss->bytes;
  return GSW_OK;
}

gsw_status gsw_session_set_thresholds(gsw_session* ss, float push_to_pull, float pull_to_push) {
  clear_error();
  if (!ss) return fail(GSW_EINVAL, "session is null");
  ss->push_to_pull = push_to_pull;
  ss->pull_to_push = pull_to_push;
  return GSW_OK;
}

}  // extern "C"
