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
};

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Sources with bit positions >= B in the last word do not exist: treat them
// as visited so they never look unreached.
__device__ __forceinline__ u64 valid_bits(int j, int W, int B) {
  if (j < W - 1 || (B & 63) == 0) return ~0ull;
  return (1ull << (B & 63)) - 1ull;
}

// Levels d+1 for the sources in `m` at vertex v, word j.
__device__ __forceinline__ void write_levels(const MsArgs& a, int64_t v, int j, u64 m) {
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
  u64 nv = 0, ne = 0;
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
    }
    if (group_any(nw != 0ull, g) && g.sub == 0) {
      nv += 1;
      ne += (u64)(a.offs[v + 1] - a.offs[v]);
    }
  }
  add_stats(a, nv, ne);
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
  u64 nv = 0, ne = 0;
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
    }
    if (group_any(acc != 0ull, g) && g.sub == 0) {
      nv += 1;
      ne += (u64)(a.offs[v + 1] - a.offs[v]);
    }
  }
  add_stats(a, nv, ne);
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
