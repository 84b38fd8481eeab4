// Batched multi-source BFS: up to 1024 sources traverse one graph together.
//
// Every vertex carries W = ceil(B/64) 64-bit masks, one bit per source:
// visited, frontier (depth d) and next frontier (depth d+1).  Each source
// picks its own direction every level with the rule the single-source search
// uses (its frontier's edges against a fraction of all arcs), so one level
// runs both halves for disjoint sets of sources:
//   top-down   each frontier vertex ORs its frontier mask (restricted to the
//              top-down sources), minus what a neighbour has already seen,
//              into the neighbour's accumulator;
//   bottom-up  each vertex with unvisited bottom-up sources ORs its
//              neighbours' frontier masks and stops once all of them are
//              covered.
// One pass over the edges advances every source whose frontier touches
// them.  The per-source result is the same hop distance as a single-source
// BFS (Section III-A); levels are stored as int8 (-1 = unreachable) and a
// depth above 127 is reported as a range error.
//
// Layout: masks are vertex-major ([n][W] words, one 128-byte line per vertex
// at B = 1024), worked on by groups of G = W (rounded up to a power of two)
// lanes, lane j of a group owning word j, so a vertex's masks are read and
// written coalesced.  Beside the masks, three 1-bit-per-vertex bitmaps (512
// KiB at 4M vertices, held in L2): the frontier of depth d and of depth d+1
// (any source) and the vertices whose accumulator the top-down pass touched.
// A wave works on one 64-vertex bitmap word at a time and only on the
// vertices whose bits say there is work, so a level with a small frontier
// costs little more than the bitmaps; bottom-up probes test the frontier bit
// (L2) before loading a neighbour's mask.  Rows are walked by the vertex's
// group up to kMsLong arcs, by the whole wave up to kMsHeavy arcs, and
// beyond that in kMsChunk-arc chunks spread over the grid (top-down; a
// bottom-up walk stops early and stays with one wave).  Levels are kept
// vertex-major ([n][B] bytes, each lane updating its own 64-byte run word by
// word) and transposed to [B][n] at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "gsw_device.h"
#include "gsw_internal.h"

namespace gsw {
namespace {

typedef unsigned long long u64;

constexpr int kMsBlock = 256;     // workgroup size of the helper kernels, default of the level kernels
constexpr int kMsMaxBlock = 512;  // level kernels: 128, 256 or 512 threads (gsw_msbfs_opts.block_size)
constexpr int kMsMaxWaves = 8192; // level kernels: wavefronts per launch at most
constexpr int kMsStats = 8;        // stat counters, spread like the queue bins
constexpr int kMsStatStride = 32;  // u64 words between counters
constexpr int kMsLong = 32;        // rows longer than this are walked by the whole wave
constexpr int kMsHeavy = 1024;     // top-down: rows longer than this go through the chunk list
constexpr int kMsChunk = 256;      // arcs per chunk of a heavy row
constexpr int kMaxWords = GSW_MSBFS_MAX_SOURCES / 64;  // mask words per vertex at most
constexpr int kMaxSlots = GSW_MSBFS_MAX_SOURCES;

// Per-level records in mapped host memory, a ring of kRing: the record of
// level d sits at (d % kRing) * kRecWords: [0] d + 1 (stored last), [1]
// vertices with new bits, [2] their degree sum, [kRecActive + j] OR of the
// new frontier's word j (which sources are still running).
constexpr int kRing = 8;
constexpr int kRecWords = 32;
constexpr int kRecActive = 3;

// Level control in device memory.  The finalize kernel of level d writes it
// for level d+1 (and a session's seeding kernel adds new sources); the
// level's kernels read it.  So the host need not see a level's result before
// it queues the next level.
struct MsCtl {
  u64 pmask[kMaxWords];  // sources expanded top-down this level
  u64 qmask[kMaxWords];  // sources expanded bottom-up this level
  double to_pull;        // bottom-up once frontier arcs > to_pull x the source's unexplored arcs
  double to_push;        // top-down again once frontier arcs < to_push x all arcs
  u64 arcs;              // arcs of the graph
  int32_t any_push, any_pull;
  long long d;           // this level's index (a session counts levels for as long as it lives)
  int32_t pull_ok;       // bottom-up allowed (symmetric graph)
  int32_t nslots, W;
  uint8_t pull[kMaxSlots];    // per source: expanded bottom-up at its last level
  u64 explored[kMaxSlots];    // per source: arcs of the vertices it has reached
};

struct MsArgs {
  const int64_t* __restrict__ offs;
  const int32_t* __restrict__ cols;
  u64* vis;
  const u64* __restrict__ fr;   // depth-d masks
  u64* frn;                     // depth-(d+1) masks; holds depth d-1's until rewritten
  u64* nx;                      // top-down accumulator, zero between levels
  const u64* __restrict__ fbm;  // bit v: v is in some source's depth-d frontier
  u64* fbm_n;                   // the same for depth d+1 (holds depth d-1's until rewritten)
  u64* tbm;                     // bit v: the top-down pass touched nx[v] (zero between levels)
  const u64* __restrict__ heavy;  // chunk list of rows longer than kMsHeavy
  int64_t n_heavy;
  int8_t* lev;                  // [n][B] levels, vertex-major
  u64* stats;                   // [kMsStats] rows: vertices with new bits, their degree sum
  u64* slot_ef;                 // [kMsStats][kMaxSlots]: per source, degree sum of its new frontier
  u64* active;                  // [kMsStats][kMaxWords]: OR of the new frontier masks
  // serving sessions: int32 levels + 1 per slot ([slots][n], 0 = not
  // reached), level = d + 1 - start[slot] where d is the session's iteration
  // (null for the batch)
  int32_t* dist;
  const long long* start;
  MsCtl* ctl;
  int64_t n;
  int32_t W, B;  // words per vertex, level bytes per vertex
};

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Sources with bit positions >= B in the last word do not exist: treat them
// as visited so they never look unreached.
__device__ __forceinline__ u64 valid_bits(int j, int W, int B) {
  if (j < W - 1 || (B & 63) == 0) return ~0ull;
  return (1ull << (B & 63)) - 1ull;
}


// 8 bits -> 8 bytes holding 0x01 where the bit is set.
__device__ __forceinline__ u64 bits_to_bytes(u64 c) {
  c = (c | (c << 28)) & 0x0000000F0000000Full;
  c = (c | (c << 14)) & 0x0003000300030003ull;
  c = (c | (c << 7)) & 0x0101010101010101ull;
  return c;
}

// Levels d+1 for the sources in `m` (word j) at vertex v.  Only v's group
// writes v's levels, so the batch's 8-byte read-modify-writes need no atomics.
__device__ __forceinline__ void write_levels(const MsArgs& a, long long d, int64_t v, int j, u64 m) {
  if (a.dist) {
    while (m) {
      const int b = __ffsll((long long)m) - 1;
      m &= m - 1ull;
      const int slot = j * 64 + b;
      a.dist[(int64_t)slot * a.n + v] = (int32_t)(d + 2 - a.start[slot]);
    }
    return;
  }
  u64* row = reinterpret_cast<u64*>(a.lev + v * (int64_t)a.B + (int64_t)j * 64);
  const u64 val = (u64)(uint8_t)(d + 1 > 127 ? 127 : d + 1) * 0x0101010101010101ull;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const u64 c = (m >> (8 * k)) & 0xffull;
    if (!c) continue;
    const u64 bm = bits_to_bytes(c) * 0xffull;
    row[k] = (row[k] & ~bm) | (val & bm);
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

// OR of this lane's new-frontier words into the active masks (LDS per
// block, then one atomic per word into the block's spread row).
__device__ __forceinline__ void add_active(const MsArgs& a, int j, u64 act) {
  __shared__ u64 s_act[kMaxWords];
  if (threadIdx.x < kMaxWords) s_act[threadIdx.x] = 0ull;
  __syncthreads();
  if (act) atomicOr(&s_act[j], act);
  __syncthreads();
  if (threadIdx.x < (unsigned)a.W && s_act[threadIdx.x])
    atomicOr(a.active + (size_t)(blockIdx.x % kMsStats) * kMaxWords + threadIdx.x, s_act[threadIdx.x]);
}

// Wave geometry: groups of G lanes (a power of two <= 16), one vertex per
// group; the waves of the grid take 64-vertex bitmap words in turn.
struct Wave {
  int G, j, gi, gpw, lane;
  u64 gmask;  // this lane's group within the wave
  int64_t wave, nwaves;
};

__device__ __forceinline__ Wave wave_of(int G) {
  Wave w;
  w.lane = lane_id();
  w.G = G;
  w.j = w.lane & (G - 1);
  w.gi = w.lane / G;
  w.gpw = 64 / G;
  w.gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << (w.gi * G));
  w.wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  w.nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  return w;
}

// ------------------------------------------------------------------ init
// Masks of n vertices (bits of sources >= nsrc start visited), the bitmaps
// and levels [n][brow] set to -1 (brow = 64 W, so rows are whole 8-byte
// words).  Both frontier mask buffers start at zero: later levels rewrite a
// vertex's next-frontier masks only where they are or were nonzero.
__global__ void __launch_bounds__(kMsBlock) k_ms_init(u64* vis, u64* fr, u64* frn, u64* nx, u64* bms,
                                                      int8_t* lev, int64_t n, int W, int nsrc, int brow) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  const int64_t gid = (int64_t)blockIdx.x * kMsBlock + threadIdx.x;
  const int64_t words = n * W;
  for (int64_t i = gid; i < words; i += stride) {
    const int j = (int)(i % W);
    vis[i] = ~valid_bits(j, W, nsrc);
    fr[i] = 0ull;
    frn[i] = 0ull;
    nx[i] = 0ull;
  }
  const int64_t nb = 3 * ((n + 63) / 64);
  for (int64_t i = gid; i < nb; i += stride) bms[i] = 0ull;
  const int64_t lw = n * (int64_t)brow / 8;
  u64* l8 = reinterpret_cast<u64*>(lev);
  for (int64_t i = gid; i < lw; i += stride) l8[i] = ~0ull;
}

// Sources are set after init (a separate launch, so no ordering issue).
__global__ void k_ms_sources(u64* vis, u64* fr, u64* fbm, int8_t* lev, int W, int B,
                             const int32_t* __restrict__ src, int nsrc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nsrc) return;
  const int64_t s = src[i];
  const u64 bit = 1ull << (i & 63);
  atomicOr(vis + s * W + (i >> 6), bit);
  atomicOr(fr + s * W + (i >> 6), bit);
  atomicOr(fbm + (s >> 6), 1ull << (s & 63));
  lev[s * (int64_t)B + i] = 0;
}

// Chunk list of the rows longer than kMsHeavy: entry (v << 32 | c) stands
// for arcs [offs[v] + c kMsChunk, min(offs[v+1], offs[v] + (c+1) kMsChunk)).
// With list == null only the total is added to *cursor.
__global__ void __launch_bounds__(kMsBlock) k_heavy_build(const int64_t* __restrict__ offs, int64_t n,
                                                          u64* list, u64* cursor) {
  const Wave w = wave_of(1);
  for (int64_t base = w.wave * 64; base < n; base += w.nwaves * 64) {
    const int64_t v = base + w.lane;
    long long nch = 0;
    if (v < n) {
      const int64_t d = offs[v + 1] - offs[v];
      if (d > kMsHeavy) nch = (d + kMsChunk - 1) / kMsChunk;
    }
    long long inc = nch;  // inclusive scan over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long y = __shfl_up(inc, off);
      if (w.lane >= off) inc += y;
    }
    const long long tot = __shfl(inc, 63);
    if (tot == 0) continue;
    u64 b0 = 0ull;
    if (w.lane == 0) b0 = atomicAdd(cursor, (u64)tot);
    b0 = __shfl(b0, 0);
    if (list)
      for (long long c = 0; c < nch; ++c) list[b0 + (u64)(inc - nch + c)] = ((u64)v << 32) | (u64)c;
  }
}

// --------------------------------------------------------------- top-down
// ORs f & ~vis[v][j] into nx[v][j] for the arcs beg, beg + step, ... < end;
// the first writer of an accumulator word marks v in the touched bitmap.
// Four arcs at a time: their column loads, visited-word loads and atomics
// are each issued before any result is used.
constexpr int kMsBatch = 4;

__device__ __forceinline__ void push_arcs(const MsArgs& a, u64 f, int j, int64_t beg, int64_t end,
                                          int step) {
  for (int64_t e = beg; e < end; e += kMsBatch * step) {
    int64_t v[kMsBatch];
    u64 m[kMsBatch], old[kMsBatch];
#pragma unroll
    for (int q = 0; q < kMsBatch; ++q) v[q] = e + q * step < end ? (int64_t)a.cols[e + q * step] : -1;
#pragma unroll
    for (int q = 0; q < kMsBatch; ++q) m[q] = v[q] >= 0 ? f & ~a.vis[v[q] * a.W + j] : 0ull;
#pragma unroll
    for (int q = 0; q < kMsBatch; ++q) old[q] = m[q] ? atomicOr(a.nx + v[q] * a.W + j, m[q]) : ~0ull;
#pragma unroll
    for (int q = 0; q < kMsBatch; ++q)
      if (!old[q]) atomicOr(a.tbm + (v[q] >> 6), 1ull << (v[q] & 63));
  }
}

// Every frontier vertex u of a top-down source: lane j pushes
// fr[u][j] & pmask[j] along u's arcs.
__global__ void __launch_bounds__(kMsMaxBlock) k_ms_push(MsArgs a, int G) {
  if (!a.ctl->any_push) return;
  const Wave w = wave_of(G);
  const int j = w.j;
  const u64 pm = j < a.W ? a.ctl->pmask[j] : 0ull;
  const int64_t nwords = (a.n + 63) / 64;
  for (int64_t wd = w.wave; wd < nwords; wd += w.nwaves) {
    const u64 word = a.fbm[wd];
    if (!word) continue;
    const int cnt = __popcll(word);
    for (int r0 = 0; r0 < cnt; r0 += w.gpw) {
      const int k = r0 + w.gi;
      const bool has = k < cnt;
      const int64_t u = wd * 64 + (has ? nth_set_bit(word, k) : 0);
      const u64 f = (has && pm) ? (a.fr[u * a.W + j] & pm) : 0ull;
      const bool act = (__ballot(f != 0ull) & w.gmask) != 0ull;
      int64_t beg = 0, end = 0;
      if (act) {
        beg = a.offs[u];
        end = a.offs[u + 1];
      }
      const int64_t deg = end - beg;
      if (f && deg <= kMsLong) push_arcs(a, f, j, beg, end, 1);
      // medium rows: the whole wave, group gi taking arcs gi, gi + 64/G, ...
      u64 lm = __ballot(deg > kMsLong && deg <= kMsHeavy && j == 0);
      while (lm) {
        const int src = __ffsll((long long)lm) - 1;
        lm &= lm - 1ull;
        const int64_t b = __shfl((long long)beg, src);
        const int64_t en = __shfl((long long)end, src);
        const u64 fw = __shfl(f, src + j);
        if (fw) push_arcs(a, fw, j, b + w.gi, en, w.gpw);
      }
    }
  }
  // heavy rows: the chunk list dealt out one entry per wave, so that the
  // consecutive chunks of one hub's row go to different waves
  for (int64_t c = w.wave; c < a.n_heavy; c += w.nwaves) {
    const u64 ent = a.heavy[c];
    const int64_t u = (int64_t)(ent >> 32);
    if (!((a.fbm[u >> 6] >> (u & 63)) & 1ull)) continue;
    const int64_t ci = (int64_t)(ent & 0xffffffffull);
    const u64 fw = pm ? (a.fr[u * a.W + j] & pm) : 0ull;
    if (__ballot(fw != 0ull) == 0ull) continue;
    const int64_t b = a.offs[u] + ci * kMsChunk;
    const int64_t en = std::min<int64_t>(a.offs[u + 1], b + kMsChunk);
    if (fw) push_arcs(a, fw, j, b + w.gi, en, w.gpw);
  }
}

// ------------------------------------------------------ bottom-up + update
// Each 64-vertex word: the vertices with possible work are all of them when
// some source pulls, else those the top-down pass touched or whose stale
// next-frontier masks must be cleared.  For such a vertex v: the bottom-up
// sources it still needs (~vis & qmask) are looked up in the neighbours'
// frontier masks (frontier bit first), stopping once all are covered; what
// the top-down pass left in nx (minus vis) joins them.  v's group is the only
// writer of v's masks and levels; the wave writes the word of the next
// frontier bitmap whole.  Also accumulates the level's statistics: vertices
// with new bits and their degrees, per source the degree sum of its new
// frontier (each source's direction is steered by it), and the OR of the new
// frontier masks.
__global__ void __launch_bounds__(kMsMaxBlock) k_ms_level(MsArgs a, int G) {
  __shared__ u64 s_ef[kMaxSlots];
  const Wave w = wave_of(G);
  const int j = w.j;
  const bool lane_live = j < a.W;
  const MsCtl* ctl = a.ctl;
  const long long d = ctl->d;
  const bool any_push = ctl->any_push != 0, any_pull = ctl->any_pull != 0;
  const u64 qm = lane_live ? ctl->qmask[j] : 0ull;
  const int nslots = a.W * 64;
  for (int k = threadIdx.x; k < nslots; k += blockDim.x) s_ef[k] = 0ull;
  __syncthreads();
  u64 nv = 0, ne = 0, act = 0;
  const int64_t nwords = (a.n + 63) / 64;
  for (int64_t wd = w.wave; wd < nwords; wd += w.nwaves) {
    const int64_t base = wd * 64;
    const u64 valid = base + 64 <= a.n ? ~0ull : ((1ull << (a.n - base)) - 1ull);
    const u64 stale = a.fbm_n[wd];
    const u64 touched = any_push ? a.tbm[wd] : 0ull;
    const u64 work = (any_pull ? ~0ull : (touched | stale)) & valid;
    u64 nbits = 0ull;
    const int cnt = __popcll(work);
    for (int r0 = 0; r0 < cnt; r0 += w.gpw) {
      const int k = r0 + w.gi;
      const bool has = k < cnt;
      const int bit = has ? nth_set_bit(work, k) : 0;
      const int64_t v = base + bit;
      const bool in = has && lane_live;
      const int64_t i = v * a.W + j;
      const u64 x = (in && ((touched >> bit) & 1ull)) ? a.nx[i] : 0ull;
      const u64 s = (in && (x || qm)) ? a.vis[i] : ~0ull;
      const u64 need = ~s & qm;
      const bool want = (__ballot(need != 0ull) & w.gmask) != 0ull;
      int64_t beg = 0, end = 0;
      if (want) {
        beg = a.offs[v];
        end = a.offs[v + 1];
      }
      const bool lng = end - beg > kMsLong;
      u64 acc = 0ull;
      if (want && !lng) {
        for (int64_t e = beg; e < end; ++e) {
          const int64_t u = a.cols[e];
          if (need && ((a.fbm[u >> 6] >> (u & 63)) & 1ull)) acc |= a.fr[u * a.W + j] & need;
          if ((__ballot(acc == need) & w.gmask) == w.gmask) break;
        }
      }
      u64 lm = __ballot(lng && j == 0);
      while (lm) {
        const int src = __ffsll((long long)lm) - 1;
        lm &= lm - 1ull;
        const int64_t b = __shfl((long long)beg, src);
        const int64_t en = __shfl((long long)end, src);
        const u64 nw = __shfl(need, src + j);
        u64 c = 0ull;
        for (int64_t e0 = b; e0 < en; e0 += w.gpw) {  // same trip count on every lane
          const int64_t e = e0 + w.gi;
          if (e < en && nw) {
            const int64_t u = a.cols[e];
            if ((a.fbm[u >> 6] >> (u & 63)) & 1ull) c |= a.fr[u * a.W + j] & nw;
          }
          for (int off = G; off < 64; off <<= 1) c |= __shfl_xor(c, off);
          if (__all(c == nw)) break;
        }
        if (w.gi * G == src) acc = c;
      }
      const u64 nb = (x & ~s) | acc;  // acc is within ~s
      const bool grp_new = (__ballot(nb != 0ull) & w.gmask) != 0ull;
      if (grp_new && !want) {
        beg = a.offs[v];
        end = a.offs[v + 1];
      }
      const u64 deg = (u64)(end - beg);
      if (in) {
        if (x) a.nx[i] = 0ull;
        if (nb) {
          a.vis[i] = s | nb;
          write_levels(a, d, v, j, nb);
          u64 m = nb;
          while (m) {
            const int bt = __ffsll((long long)m) - 1;
            m &= m - 1ull;
            atomicAdd(&s_ef[j * 64 + bt], deg);
          }
        }
        if (nb || ((stale >> bit) & 1ull)) a.frn[i] = nb;
        act |= nb;
      }
      if (grp_new && j == 0) {
        nv += 1;
        ne += deg;
        nbits |= 1ull << bit;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nbits |= __shfl_xor(nbits, off);
    if (w.lane == 0) {
      a.fbm_n[wd] = nbits;
      if (touched) a.tbm[wd] = 0ull;
    }
  }
  add_stats(a, nv, ne);
  add_active(a, j, act);
  __syncthreads();
  u64* row = a.slot_ef + (size_t)(blockIdx.x % kMsStats) * kMaxSlots;
  for (int k = threadIdx.x; k < nslots; k += blockDim.x)
    if (s_ef[k]) atomicAdd(row + k, s_ef[k]);
}

// End of level d: sums the spread counters, sets each running source's
// direction for level d+1 and the masks, advances ctl->d, and publishes the
// level's record to the host ring (its first word last).  The counters are
// zeroed for the next level.  Direction, per source as in direction-
// optimising BFS: bottom-up once the new frontier's arcs exceed to_pull of
// the arcs the source has not reached yet (a bottom-up pass is shared by all
// pulling sources, and one with a small frontier would make every vertex
// scan its whole row), top-down again once they fall below to_push of all
// arcs.
__global__ void __launch_bounds__(256) k_ms_finalize(MsCtl* ctl, u64* stats, u64* active, u64* slot_ef,
                                                     u64* ring) {
  __shared__ u64 s_act[kMaxWords], s_p[kMaxWords], s_q[kMaxWords];
  __shared__ u64 s_v, s_e;
  const int t = threadIdx.x;
  const int W = ctl->W, nslots = ctl->nslots;
  const long long d = ctl->d;
  if (t < kMaxWords) {
    u64 x = 0ull;
    if (t < W)
      for (int r = 0; r < kMsStats; ++r) {
        x |= active[r * kMaxWords + t];
        active[r * kMaxWords + t] = 0ull;
      }
    s_act[t] = x;
    s_p[t] = 0ull;
    s_q[t] = 0ull;
  }
  if (t < 64) {  // wave 0
    u64 v = 0, e = 0;
    if (t < kMsStats) {
      v = stats[t * kMsStatStride];
      e = stats[t * kMsStatStride + 1];
      stats[t * kMsStatStride] = 0ull;
      stats[t * kMsStatStride + 1] = 0ull;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v += __shfl_xor(v, off);
      e += __shfl_xor(e, off);
    }
    if (t == 0) {
      s_v = v;
      s_e = e;
    }
  }
  __syncthreads();
  const double to_pull = ctl->to_pull, to_push = ctl->to_push;
  const u64 arcs = ctl->arcs;
  const bool pull_ok = ctl->pull_ok != 0;
  for (int k = t; k < nslots; k += 256) {
    u64 ef = 0ull;
    for (int r = 0; r < kMsStats; ++r) {
      ef += slot_ef[r * kMaxSlots + k];
      slot_ef[r * kMaxSlots + k] = 0ull;
    }
    if ((s_act[k >> 6] >> (k & 63)) & 1ull) {
      const u64 ex = ctl->explored[k] + ef;
      ctl->explored[k] = ex;
      const double unexplored = ex < arcs ? (double)(arcs - ex) : 0.0;
      uint8_t p = ctl->pull[k];
      if (!pull_ok) p = 0;
      else if (!p && (double)ef > to_pull * unexplored) p = 1;
      else if (p && (double)ef < to_push * (double)arcs) p = 0;
      ctl->pull[k] = p;
      atomicOr(p ? &s_q[k >> 6] : &s_p[k >> 6], 1ull << (k & 63));
    }
  }
  __syncthreads();
  u64* rec = ring + (size_t)(d % kRing) * kRecWords;
  if (t < kMaxWords) {
    ctl->pmask[t] = s_p[t];
    ctl->qmask[t] = s_q[t];
    if (t < W) __hip_atomic_store(rec + kRecActive + t, s_act[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (t == 0) {
    u64 p = 0ull, q = 0ull;
    for (int j = 0; j < kMaxWords; ++j) {
      p |= s_p[j];
      q |= s_q[j];
    }
    ctl->any_push = p != 0ull;
    ctl->any_pull = q != 0ull;
    ctl->d = d + 1;
    __hip_atomic_store(rec + 1, s_v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(rec + 2, s_e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __threadfence_system();
  __syncthreads();
  if (t == 0) __hip_atomic_store(rec, (u64)d + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// [n][B] -> [nsrc][n] levels through 64x64-byte LDS tiles.
// A 128-vertex x 128-source tile moved as 4-byte words, so both the reads
// (128 source bytes of a vertex) and the writes (128 vertex bytes of a
// source) cover whole 128-byte lines.  B is a multiple of 64, so every input
// word is whole and aligned; with B = 64 the upper half of the tile is empty.
constexpr int kTr = 128;
__global__ void __launch_bounds__(256) k_ms_transpose(const int8_t* __restrict__ in,
                                                      int8_t* __restrict__ out, int64_t n, int B,
                                                      int nsrc) {
  constexpr int kW = kTr / 4;  // words per tile row
  __shared__ uint32_t tile[kTr][kW + 1];  // [vertex][word of 4 sources], padded
  const int64_t v0 = (int64_t)blockIdx.x * kTr;
  const int s0 = blockIdx.y * kTr;
  for (int i = threadIdx.x; i < kTr * kW; i += 256) {
    const int r = i / kW, wd = i % kW;
    const int64_t v = v0 + r;
    const int s = s0 + 4 * wd;
    tile[r][wd] = v < n && s < B ? *reinterpret_cast<const uint32_t*>(in + v * B + s) : 0xffffffffu;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kTr * kW; i += 256) {
    const int sr = i / kW, wd = i % kW;  // source s0 + sr, vertices v0 + 4 wd .. + 3
    const int s = s0 + sr;
    if (s >= nsrc) continue;
    const int sh = 8 * (sr & 3);
    uint32_t x = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) x |= ((tile[4 * wd + k][sr >> 2] >> sh) & 0xffu) << (8 * k);
    const int64_t v = v0 + 4 * wd;
    int8_t* dst = out + (int64_t)s * n + v;
    if (v + 3 < n && (reinterpret_cast<uintptr_t>(dst) & 3u) == 0u) {
      *reinterpret_cast<uint32_t*>(dst) = x;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (v + k < n) dst[k] = (int8_t)((x >> (8 * k)) & 0xffu);
    }
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

// Admitted slots: the source's bit in vis, in the current frontier and its
// bitmap, level 0 (stored as 1), and the slot joins the next level top-down.
__global__ void k_ss_seed(u64* vis, u64* fr, u64* fbm, int32_t* dist, MsCtl* ctl, int64_t n, int W,
                          const int32_t* __restrict__ src, const int32_t* __restrict__ slot, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t s = src[i];
  const int k = slot[i];
  const u64 bit = 1ull << (k & 63);
  atomicOr(vis + s * W + (k >> 6), bit);
  atomicOr(fr + s * W + (k >> 6), bit);
  atomicOr(fbm + (s >> 6), 1ull << (s & 63));
  dist[(int64_t)k * n + s] = 1;
  ctl->pull[k] = 0;
  ctl->explored[k] = 0ull;
  atomicOr(&ctl->pmask[k >> 6], bit);
  atomicAnd(&ctl->qmask[k >> 6], ~bit);
  ctl->any_push = 1;
}

// Sets a session's level counter (in stream order with its levels).
__global__ void k_ss_set_level(MsCtl* ctl, long long d) {
  if (threadIdx.x == 0) ctl->d = d;
}

// Direction thresholds of a session, in stream order with its levels.
__global__ void k_ss_thresholds(MsCtl* ctl, double to_pull, double to_push) {
  if (threadIdx.x == 0) {
    ctl->to_pull = to_pull;
    ctl->to_push = to_push;
  }
}

// A finished slot's levels: out[v] = row[v] - 1 (-1 = not reached), and the
// row is cleared for the slot's next query.
__global__ void __launch_bounds__(kMsBlock) k_ss_take(int32_t* row, int32_t* __restrict__ out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  for (int64_t i = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; i < n; i += stride) {
    out[i] = row[i] - 1;
    row[i] = 0;
  }
}

// A cancelled slot's row, cleared for its next query.
__global__ void __launch_bounds__(kMsBlock) k_ss_clear(int32_t* row, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  for (int64_t i = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; i < n; i += stride) row[i] = 0;
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int group_lanes(int W) {
  int G = 1;
  while (G < W) G <<= 1;
  return G;  // W <= 16 -> G <= 16
}

// One wave per 64-vertex word for one pass, at most kMsMaxWaves waves, in
// workgroups of bs threads.
inline unsigned ms_grid(int64_t n, int bs = kMsBlock) {
  const int64_t blocks = cdiv(cdiv(n, 64), bs / 64);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, (int64_t)kMsMaxWaves * 64 / bs));
}

// Spread statistics counters, the level control block and the host ring of
// one traversal.
struct LevelStats {
  u64 *stats = nullptr, *active = nullptr, *slot_ef = nullptr;
  MsCtl* ctl = nullptr;    // device
  MsCtl* h_ctl = nullptr;  // pinned staging for uploads of the control block
  u64 *ring = nullptr, *d_ring = nullptr;  // mapped host memory (kRing records)
  size_t bytes = 0;
};

// Device bytes of a traversal's statistics counters and control block.
size_t stats_bytes() {
  return (size_t)kMsStats * kMsStatStride * sizeof(u64) + (size_t)kMsStats * kMaxWords * sizeof(u64) +
         (size_t)kMsStats * kMaxSlots * sizeof(u64) + sizeof(MsCtl);
}

// The counters are cleared on `s`, the stream that will use them, and the
// call waits for it: a clear on the null stream is asynchronous to the host
// and unordered with a non-blocking stream, so under load it could land
// after the traversal has started and zero its control block.
gsw_status stats_alloc(LevelStats* st, hipStream_t s) {
  const size_t sb = (size_t)kMsStats * kMsStatStride * sizeof(u64);
  const size_t ab = (size_t)kMsStats * kMaxWords * sizeof(u64);
  const size_t eb = (size_t)kMsStats * kMaxSlots * sizeof(u64);
  const size_t cb = sizeof(MsCtl);
  void** ps[] = {(void**)&st->stats, (void**)&st->active, (void**)&st->slot_ef, (void**)&st->ctl};
  const size_t bs[] = {sb, ab, eb, cb};
  for (int k = 0; k < 4; ++k) {
    if (hipMalloc(ps[k], bs[k]) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for level statistics failed", bs[k]);
    }
    st->bytes += bs[k];
    GSW_HIP(hipMemsetAsync(*ps[k], 0, bs[k], s));
  }
  GSW_HIP(hipStreamSynchronize(s));
  GSW_HIP(hipHostMalloc((void**)&st->h_ctl, sizeof(MsCtl), hipHostMallocDefault));
  std::memset(st->h_ctl, 0, sizeof(MsCtl));
  GSW_HIP(hipHostMalloc((void**)&st->ring, (size_t)kRing * kRecWords * sizeof(u64),
                        hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(st->ring, 0, (size_t)kRing * kRecWords * sizeof(u64));
  GSW_HIP(hipHostGetDevicePointer((void**)&st->d_ring, st->ring, 0));
  return GSW_OK;
}

void stats_free(LevelStats* st) {
  void* p[] = {st->stats, st->active, st->slot_ef, st->ctl};
  for (void* x : p)
    if (x) (void)hipFree(x);
  if (st->h_ctl) (void)hipHostFree(st->h_ctl);
  if (st->ring) (void)hipHostFree(st->ring);
  *st = LevelStats();
}

// Waits until level d's record is in the ring; returns its words through
// *rec.  A record that never comes is reported with what the ring slot and
// the device's level counter hold.
gsw_status wait_record(const LevelStats& st, int64_t d, hipStream_t s, const char* who,
                       const volatile u64** rec) {
  const volatile u64* r = st.ring + (size_t)(d % kRing) * kRecWords;
  bool missing = false;
  const hipError_t e = await_record([&]() -> bool { return r[0] == (u64)d + 1ull; }, s, &missing);
  if (e != hipSuccess) return fail(GSW_EHIP, "%s: %s", who, hipGetErrorString(e));
  if (missing) {
    long long dev = -1;
    (void)hipMemcpy(&dev, &st.ctl->d, sizeof dev, hipMemcpyDeviceToHost);
    return fail(GSW_EHIP, "%s: level %lld finished without reporting (its ring slot holds %llu, the device "
                "level counter %lld)", who, (long long)d, (unsigned long long)r[0], dev);
  }
  *rec = r;
  return GSW_OK;
}

// Fills the staging control block for a traversal whose first level expands
// the sources in `first` top-down.
void ctl_reset(MsCtl* c, const u64* first, int W, int nslots, bool pull_ok, int64_t arcs, double to_pull,
               double to_push) {
  std::memset(c, 0, sizeof *c);
  for (int j = 0; j < W; ++j) c->pmask[j] = first ? first[j] : 0ull;
  for (int j = 0; j < W; ++j) c->any_push |= c->pmask[j] != 0ull;
  c->to_pull = to_pull;
  c->to_push = to_push;
  c->arcs = (u64)arcs;
  c->pull_ok = pull_ok ? 1 : 0;
  c->nslots = nslots;
  c->W = W;
}

// Builds the graph's chunk list of rows longer than kMsHeavy once (count,
// allocate, fill); the caller holds the graph's lock.
gsw_status ensure_heavy(gsw_graph* g) {
  if (g->n_heavy >= 0) return GSW_OK;
  u64* cur = nullptr;
  GSW_HIP(hipMalloc((void**)&cur, sizeof(u64)));
  gsw_status st = GSW_OK;
  u64 total = 0;
  const unsigned grid = ms_grid(g->n);
  if (hipMemset(cur, 0, sizeof(u64)) != hipSuccess) st = fail(GSW_EHIP, "heavy-row count");
  if (st == GSW_OK) {
    hipLaunchKernelGGL(k_heavy_build, dim3(grid), dim3(kMsBlock), 0, 0, g->offs, g->n, (u64*)nullptr, cur);
    if (hipGetLastError() != hipSuccess || hipMemcpy(&total, cur, sizeof(u64), hipMemcpyDeviceToHost) != hipSuccess)
      st = fail(GSW_EHIP, "heavy-row count");
  }
  u64* list = nullptr;
  if (st == GSW_OK && total > 0) {
    if (hipMalloc((void**)&list, total * sizeof(u64)) != hipSuccess) {
      (void)hipGetLastError();
      st = fail(GSW_ENOMEM, "hipMalloc(%llu) for the heavy-row chunk list failed",
                (unsigned long long)(total * sizeof(u64)));
    } else if (hipMemset(cur, 0, sizeof(u64)) != hipSuccess) {
      st = fail(GSW_EHIP, "heavy-row list");
    } else {
      hipLaunchKernelGGL(k_heavy_build, dim3(grid), dim3(kMsBlock), 0, 0, g->offs, g->n, list, cur);
      if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        st = fail(GSW_EHIP, "heavy-row list");
    }
  }
  (void)hipFree(cur);
  if (st != GSW_OK) {
    if (list) (void)hipFree(list);
    return st;
  }
  g->heavy = list;
  g->n_heavy = (int64_t)total;
  return GSW_OK;
}

// Queues one level: the top-down pass (it returns at once when no source
// pushes), the bottom-up + update pass and the finalize kernel.  The
// statistics pointers of the arguments are taken from `st`.
gsw_status launch_ms_level(MsArgs a, const LevelStats& st, int G, int bs, hipStream_t s) {
  a.stats = st.stats;
  a.active = st.active;
  a.slot_ef = st.slot_ef;
  a.ctl = st.ctl;
  // every buffer the kernels touch must be there: a missing one would be a
  // device fault, so it is an error here
  const void* need[] = {a.offs, a.cols, a.vis, a.fr, a.frn, a.nx, a.fbm, a.fbm_n, a.tbm,
                        a.stats, a.active, a.slot_ef, a.ctl, st.d_ring};
  for (const void* p : need)
    if (!p) return fail(GSW_EINVAL, "batched level launched with a missing buffer");
  if ((!a.dist && !a.lev) || (a.dist && !a.start) || (a.n_heavy > 0 && !a.heavy) || a.W < 1 ||
      a.W > kMaxWords || a.B != 64 * a.W || G < a.W || G > 16 || (G & (G - 1)) != 0 ||
      (bs != 128 && bs != 256 && bs != 512))
    return fail(GSW_EINVAL, "batched level launched with inconsistent arguments");
  const unsigned grid = ms_grid(a.n, bs);
  hipLaunchKernelGGL(k_ms_push, dim3(grid), dim3(bs), 0, s, a, G);
  hipLaunchKernelGGL(k_ms_level, dim3(grid), dim3(bs), 0, s, a, G);
  hipLaunchKernelGGL(k_ms_finalize, dim3(1), dim3(256), 0, s, st.ctl, st.stats, st.active, st.slot_ef,
                     st.d_ring);
  return GSW_OK;
}

}  // namespace

struct MsWorkspace {
  int64_t n = 0;
  int W = 0, B = 0;
  int bs = 0;  // block size the captured graph was made with
  u64 *vis = nullptr, *fr = nullptr, *frn = nullptr, *nx = nullptr;
  u64* bms = nullptr;  // 3 bitmaps of ceil(n/64) words: frontier (two) and touched
  int8_t* lev = nullptr;
  int32_t* src = nullptr;
  LevelStats st;
  // two levels (even, odd: the mask and bitmap buffers swap roles) captured
  // once as a graph and replayed
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t bytes = 0;
};

namespace {
void ms_free(MsWorkspace* m) {
  if (!m) return;
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  if (m->cap) (void)hipStreamDestroy(m->cap);
  void* p[] = {m->vis, m->fr, m->frn, m->nx, m->bms, m->lev, m->src};
  for (void* x : p)
    if (x) (void)hipFree(x);
  stats_free(&m->st);
  delete m;
}

gsw_status ms_ensure(gsw_graph* g, int W, hipStream_t s) {
  GSW_TRY(ensure_heavy(g));
  MsWorkspace*& m = g->ms;
  if (m && m->W == W) return GSW_OK;
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
               {(void**)&m->bms, 3 * (size_t)cdiv(g->n, 64) * sizeof(u64)},
               {(void**)&m->lev, (size_t)g->n * m->B},
               {(void**)&m->src, (size_t)m->B * sizeof(int32_t)}};
  gsw_status st = GSW_OK;
  for (auto& it : items) {
    if (hipMalloc(it.p, it.bytes) != hipSuccess) {
      (void)hipGetLastError();
      st = fail(GSW_ENOMEM, "hipMalloc(%zu) for the batched BFS failed", it.bytes);
      break;
    }
    m->bytes += it.bytes;
  }
  if (st == GSW_OK) st = stats_alloc(&m->st, s);
  if (st != GSW_OK) {
    ms_free(m);
    m = nullptr;
    return st;
  }
  m->bytes += m->st.bytes;
  return GSW_OK;
}

// Level arguments of the batch; `odd` swaps the frontier buffers.
MsArgs ms_args(const gsw_graph* g, const MsWorkspace* m, bool odd) {
  MsArgs a;
  std::memset(&a, 0, sizeof a);
  const int64_t nw = cdiv(g->n, 64);
  a.offs = g->offs;
  a.cols = g->cols;
  a.vis = m->vis;
  a.fr = odd ? m->frn : m->fr;
  a.frn = odd ? m->fr : m->frn;
  a.nx = m->nx;
  a.fbm = m->bms + (odd ? nw : 0);
  a.fbm_n = m->bms + (odd ? 0 : nw);
  a.tbm = m->bms + 2 * nw;
  a.heavy = g->heavy;
  a.n_heavy = g->n_heavy;
  a.lev = m->lev;
  a.ctl = m->st.ctl;
  a.n = g->n;
  a.W = m->W;
  a.B = m->B;
  return a;
}

// Captures the even and the odd level as one graph (once per workspace and
// block size).
gsw_status ms_capture(gsw_graph* g, MsWorkspace* m, int G, int bs) {
  if (m->exec && m->bs == bs) return GSW_OK;
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->exec = nullptr;
  m->graph = nullptr;
  if (!m->cap) GSW_HIP(hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking));
  GSW_HIP(hipStreamBeginCapture(m->cap, hipStreamCaptureModeRelaxed));
  gsw_status ls = launch_ms_level(ms_args(g, m, false), m->st, G, bs, m->cap);
  if (ls == GSW_OK) ls = launch_ms_level(ms_args(g, m, true), m->st, G, bs, m->cap);
  const hipError_t e1 = hipGetLastError();
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(m->cap, &graph);
  if (ls != GSW_OK || e1 != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    if (ls != GSW_OK) return ls;
    return fail(GSW_EHIP, "capturing the batched level graph failed: %s",
                hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(GSW_EHIP, "instantiating the batched level graph failed");
  }
  m->graph = graph;
  m->exec = exec;
  m->bs = bs;
  return GSW_OK;
}

// int32 distances -> int8 row: the distance where it fits, INT8_MIN where it
// is above the int8 cap, -1 where unreachable.
__global__ void __launch_bounds__(kMsBlock) k_ms_narrow(const int32_t* __restrict__ wide, int8_t* __restrict__ row,
                                                         int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kMsBlock;
  for (int64_t i = (int64_t)blockIdx.x * kMsBlock + threadIdx.x; i < n; i += stride) {
    const int32_t x = wide[i];
    row[i] = (int8_t)(x > GSW_MSBFS_LEVEL_CAP ? -128 : x);
  }
}
}  // namespace

void ms_release(gsw_graph* g) {
  ms_free(g->ms);
  g->ms = nullptr;
  if (g->heavy) (void)hipFree(g->heavy);
  g->heavy = nullptr;
  g->n_heavy = -1;
}

}  // namespace gsw

using namespace gsw;

extern "C" {

void gsw_msbfs_opts_default(gsw_msbfs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->push_to_pull = 0.07f;
  o->pull_to_push = 0.01f;
  o->graph = 1;
  o->block_size = kMsBlock;
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
  const int bs = o->block_size == 0 ? kMsBlock : o->block_size;
  if (bs != 128 && bs != 256 && bs != 512) return fail(GSW_EINVAL, "block_size %d: 128, 256 or 512", o->block_size);
  if (o->fallback && o->n_wide) *o->n_wide = 0;
  if (o->fallback && o->wide_cap < 0) return fail(GSW_EINVAL, "wide_cap %d is negative", o->wide_cap);
  if (o->fallback && o->wide_cap > 0 && (!o->wide_levels || !o->wide_index))
    return fail(GSW_EINVAL, "fallback with room for %d rows needs wide_levels and wide_index", o->wide_cap);
  std::lock_guard<std::mutex> lock(g->mu);
  GSW_HIP(hipSetDevice(g->device));
  const int W = (n_sources + 63) / 64;
  const hipStream_t s = pick_stream(g, o->stream);
  GSW_TRY(ms_ensure(g, W, s));
  MsWorkspace* m = g->ms;
  const int B = W * 64;  // level bytes per vertex in the workspace
  const int G = group_lanes(W);
  const int64_t nw = cdiv(g->n, 64);
  if (o->graph) GSW_TRY(ms_capture(g, m, G, bs));
  // the ring must not hold records of an earlier call with the same level numbers
  std::memset(m->st.ring, 0, (size_t)kRing * kRecWords * sizeof(u64));
  std::vector<u64> first((size_t)W, 0ull);
  for (int32_t i = 0; i < n_sources; ++i) first[(size_t)(i >> 6)] |= 1ull << (i & 63);
  ctl_reset(m->st.h_ctl, first.data(), W, n_sources, g->symmetric != 0, g->nnz, o->push_to_pull,
            o->pull_to_push);
  GSW_HIP(hipMemcpyAsync(m->st.ctl, m->st.h_ctl, sizeof(MsCtl), hipMemcpyHostToDevice, s));
  GSW_HIP(hipMemcpyAsync(m->src, sources, (size_t)n_sources * sizeof(int32_t), hipMemcpyHostToDevice, s));
  {
    const int64_t work = std::max<int64_t>(g->n * W, g->n * (int64_t)B / 8);
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(work, kMsBlock), 65536);
    hipLaunchKernelGGL(k_ms_init, dim3(grid), dim3(kMsBlock), 0, s, m->vis, m->fr, m->frn, m->nx, m->bms,
                       m->lev, g->n, W, n_sources, B);
    hipLaunchKernelGGL(k_ms_sources, dim3((unsigned)cdiv(n_sources, 256)), dim3(256), 0, s, m->vis,
                       m->fr, m->bms, m->lev, W, B, (const int32_t*)m->src, n_sources);
    GSW_HIP(hipGetLastError());
  }
  (void)nw;
  // Levels are queued up to kAhead beyond the last one whose record the host
  // has read; levels after the last productive one find nothing and change
  // nothing.  The captured graph queues two levels per launch.
  constexpr int64_t kAhead = 2;
  int64_t queued = 0, d = 0;
  gsw_status st = GSW_OK;
  std::vector<int32_t> wide;  // fallback: indices of the sources past the cap
  for (;;) {
    while (queued - d < kAhead) {
      if (o->graph) {
        if (hipGraphLaunch(m->exec, s) != hipSuccess) {
          st = fail(GSW_EHIP, "launching the batched level graph failed");
          break;
        }
        queued += 2;
      } else {
        st = launch_ms_level(ms_args(g, m, (queued & 1) != 0), m->st, G, bs, s);
        if (st != GSW_OK) break;
        queued += 1;
      }
    }
    if (st == GSW_OK && hipGetLastError() != hipSuccess) st = fail(GSW_EHIP, "batched level launch failed");
    if (st != GSW_OK) break;
    const volatile u64* rec = nullptr;
    st = wait_record(m->st, d, s, "batched BFS", &rec);
    if (st != GSW_OK) break;
    if (rec[1] == 0) break;  // level d found nothing: d + 1 levels ran
    if (d + 1 > GSW_MSBFS_LEVEL_CAP) {
      if (!o->fallback) {
        st = fail(GSW_ERANGE, "a source reaches depth %lld > %d (int8 levels)", (long long)d + 1,
                  GSW_MSBFS_LEVEL_CAP);
        break;
      }
      // the sources that found vertices at depth cap + 1 are rerun in int32
      for (int32_t i = 0; i < n_sources; ++i)
        if ((rec[kRecActive + (i >> 6)] >> (i & 63)) & 1ull) wide.push_back(i);
      break;
    }
    ++d;
  }
  if (st == GSW_OK && !wide.empty()) {
    if (o->n_wide) *o->n_wide = (int32_t)wide.size();
    if ((int32_t)wide.size() > o->wide_cap)
      st = fail(GSW_ERANGE, "%zu sources reach depths above %d, wide_levels has room for %d", wide.size(),
                GSW_MSBFS_LEVEL_CAP, o->wide_cap);
  }
  if (st != GSW_OK) {
    (void)hipStreamSynchronize(s);
    return st;
  }
  if (n_levels) *n_levels = (int32_t)(d + 1);
  // [n][B] -> [n_sources][n]
  int8_t* out = levels;
  int8_t* tmp = nullptr;
  if (!o->device_ptrs) {
    if (hipMalloc((void**)&tmp, (size_t)n_sources * g->n) != hipSuccess) {
      (void)hipStreamSynchronize(s);
      return fail(GSW_ENOMEM, "hipMalloc for the level copy-back failed");
    }
    out = tmp;
  }
  hipLaunchKernelGGL(k_ms_transpose, dim3((unsigned)cdiv(g->n, kTr), (unsigned)cdiv(n_sources, kTr)),
                     dim3(256), 0, s, (const int8_t*)m->lev, out, g->n, B, n_sources);
  if (hipGetLastError() != hipSuccess) st = fail(GSW_EHIP, "transpose launch failed");
  if (st == GSW_OK && !wide.empty()) {
    // the rerun, into the caller's rows (device) or a staging buffer (host)
    const size_t wb = wide.size() * (size_t)g->n * sizeof(int32_t);
    int32_t* dw = o->wide_levels;
    int32_t* wtmp = nullptr;
    if (!o->device_ptrs) {
      if (hipMalloc((void**)&wtmp, wb) != hipSuccess) {
        (void)hipGetLastError();
        st = fail(GSW_ENOMEM, "hipMalloc(%zu) for the int32 rerun failed", wb);
      }
      dw = wtmp;
    }
    std::vector<int32_t> wsrc(wide.size());
    for (size_t k = 0; k < wide.size(); ++k) wsrc[k] = sources[wide[k]];
    if (st == GSW_OK) st = bfs_rows_locked(g, wsrc.data(), (int32_t)wide.size(), dw, o->tree, s);
    for (size_t k = 0; st == GSW_OK && k < wide.size(); ++k) {
      hipLaunchKernelGGL(k_ms_narrow, dim3((unsigned)std::min<int64_t>(cdiv(g->n, kMsBlock), 4096)), dim3(kMsBlock),
                         0, s, (const int32_t*)(dw + k * g->n), out + (size_t)wide[k] * g->n, g->n);
      if (hipGetLastError() != hipSuccess) st = fail(GSW_EHIP, "narrowing launch failed");
      o->wide_index[k] = wide[k];
    }
    if (st == GSW_OK && wtmp &&
        hipMemcpyAsync(o->wide_levels, wtmp, wb, hipMemcpyDeviceToHost, s) != hipSuccess)
      st = fail(GSW_EHIP, "copying the int32 rerun to the host failed");
    if (wtmp) {
      (void)hipStreamSynchronize(s);
      (void)hipFree(wtmp);
    }
  }
  if (st == GSW_OK && tmp) {
    if (hipMemcpyAsync(levels, tmp, (size_t)n_sources * g->n, hipMemcpyDeviceToHost, s) != hipSuccess)
      st = fail(GSW_EHIP, "copying levels to the host failed");
  }
  if (hipStreamSynchronize(s) != hipSuccess && st == GSW_OK) st = fail(GSW_EHIP, "stream synchronize failed");
  if (tmp) (void)hipFree(tmp);
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------ sessions
struct gsw_session {
  gsw_graph* g = nullptr;
  int W = 0, slots = 0;
  u64 *vis = nullptr, *fr = nullptr, *frn = nullptr, *nx = nullptr;
  u64* bms = nullptr;     // frontier bitmaps (depth d, d+1) and the touched bitmap
  u64* fbm[2] = {};       // fbm[0] pairs with fr, fbm[1] with frn (swapped together)
  u64* masks = nullptr;   // clr[kMaxWords] then set[kMaxWords]
  int32_t *dist = nullptr, *seed = nullptr;  // seed: src[slots] then slot[slots]
  long long* start_d = nullptr;             // start level of every slot (device)
  int32_t* take = nullptr;  // device staging for fetches into host memory
  LevelStats st;
  // pinned staging for the per-boundary uploads (masks; seed src/slot; start
  // of every slot), kStage sets used in turn: an async copy reads its set
  // when it runs on the stream, and with up to two levels queued beyond the
  // one the host waits for, a set is rewritten only after the level it fed
  // has finished
  static constexpr int kStage = 4;
  u64* h_masks = nullptr;    // [kStage][2 kMaxWords]
  int32_t* h_seed = nullptr;   // [kStage][2 slots]
  long long* h_start = nullptr;  // [kStage][slots]
  std::vector<long long> start_up;  // start level of every slot, as uploaded
  std::vector<int32_t> source;
  std::vector<int64_t> start;  // level at which a running slot was seeded
  std::vector<int8_t> state;   // 0 free, 1 admitted (seeded at the next level boundary), 2 running, 3 finished,
                               // 4 cancelled while running (inert from the next boundary; freed once its frontier is empty)
  std::vector<u64> freed;      // slots freed since the last boundary (made inert then)
  int64_t queued = 0;          // levels queued on the stream
  int64_t done = 0;            // levels whose record has been read
  float push_to_pull = 0.07f, pull_to_push = 0.01f;
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  std::mutex mu;       // host state shared with admit / fetch / info
  std::mutex step_mu;  // one step or fetch at a time
};

namespace {

void ss_free(gsw_session* ss) {
  if (!ss) return;
  if (ss->stream) (void)hipStreamSynchronize(ss->stream);  // a level may still be queued
  void* p[] = {ss->vis, ss->fr, ss->frn, ss->nx, ss->bms, ss->masks, ss->dist, ss->start_d, ss->seed, ss->take};
  for (void* x : p)
    if (x) (void)hipFree(x);
  stats_free(&ss->st);
  void* hp[] = {ss->h_masks, ss->h_seed, ss->h_start};
  for (void* x : hp)
    if (x) (void)hipHostFree(x);
  if (ss->stream) (void)hipStreamDestroy(ss->stream);
  delete ss;
}

}  // namespace

extern "C" {

size_t gsw_session_bytes(const gsw_graph* g, int32_t max_slots) {
  if (!g || max_slots < 1 || max_slots > GSW_MSBFS_MAX_SOURCES) return 0;
  const int64_t n = g->n;
  const size_t W = (size_t)(max_slots + 63) / 64;
  const size_t words = (size_t)cdiv(n, 64);
  return 4 * (size_t)n * W * sizeof(u64) + 3 * words * sizeof(u64) + 2 * (size_t)kMaxWords * sizeof(u64) +
         (size_t)max_slots * n * sizeof(int32_t) + (size_t)max_slots * sizeof(long long) +
         2 * (size_t)max_slots * sizeof(int32_t) + (size_t)n * sizeof(int32_t) + stats_bytes();
}

gsw_status gsw_session_create(const gsw_graph* cg, int32_t max_slots, gsw_session** out) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  *out = nullptr;
  if (!cg) return fail(GSW_EINVAL, "graph is null");
  if (max_slots < 1 || max_slots > GSW_MSBFS_MAX_SOURCES)
    return fail(GSW_EINVAL, "max_slots=%d out of [1, %d]", max_slots, GSW_MSBFS_MAX_SOURCES);
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  GSW_HIP(hipSetDevice(g->device));
  {
    std::lock_guard<std::mutex> lock(g->mu);
    GSW_TRY(ensure_heavy(g));
  }
  gsw_session* ss = new (std::nothrow) gsw_session();
  if (!ss) return fail(GSW_ENOMEM, "host allocation failed");
  ss->g = g;
  ss->W = (max_slots + 63) / 64;
  ss->slots = max_slots;
  const int64_t n = g->n;
  const int64_t nw = cdiv(n, 64);
  const size_t mb = (size_t)n * ss->W * sizeof(u64);
  const size_t bb = 3 * (size_t)nw * sizeof(u64);
  struct Item {
    void** p;
    size_t bytes;
  } items[] = {{(void**)&ss->vis, mb},
               {(void**)&ss->fr, mb},
               {(void**)&ss->frn, mb},
               {(void**)&ss->nx, mb},
               {(void**)&ss->bms, bb},
               {(void**)&ss->masks, 2 * (size_t)kMaxWords * sizeof(u64)},
               {(void**)&ss->dist, (size_t)max_slots * n * sizeof(int32_t)},
               {(void**)&ss->start_d, (size_t)max_slots * sizeof(long long)},
               {(void**)&ss->seed, 2 * (size_t)max_slots * sizeof(int32_t)},
               {(void**)&ss->take, (size_t)n * sizeof(int32_t)}};
  for (auto& it : items) {
    hipError_t e = hipMalloc(it.p, it.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ss_free(ss);
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for a session failed", it.bytes);
    }
    ss->bytes += it.bytes;
  }
  ss->fbm[0] = ss->bms;
  ss->fbm[1] = ss->bms + nw;
  gsw_status st = GSW_OK;
  if (hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking) != hipSuccess) {
    ss->stream = nullptr;
    st = fail(GSW_EHIP, "session stream");
  }
  if (st == GSW_OK) st = stats_alloc(&ss->st, ss->stream);
  if (st == GSW_OK) {
    ss->bytes += ss->st.bytes;
    if (hipHostMalloc((void**)&ss->h_masks, gsw_session::kStage * 2 * (size_t)kMaxWords * sizeof(u64),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ss->h_seed, gsw_session::kStage * 2 * (size_t)max_slots * sizeof(int32_t),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ss->h_start, gsw_session::kStage * (size_t)max_slots * sizeof(long long),
                      hipHostMallocDefault) != hipSuccess)
      st = fail(GSW_EHIP, "session pinned staging memory");
  }
  if (st == GSW_OK) {
    const hipStream_t s = ss->stream;
    ctl_reset(ss->st.h_ctl, nullptr, ss->W, max_slots, g->symmetric != 0, g->nnz, ss->push_to_pull,
              ss->pull_to_push);
    // every slot starts inert: visited everywhere, in no frontier, not reached
    if (hipMemsetAsync(ss->vis, 0xff, mb, s) != hipSuccess || hipMemsetAsync(ss->fr, 0, mb, s) != hipSuccess ||
        hipMemsetAsync(ss->frn, 0, mb, s) != hipSuccess || hipMemsetAsync(ss->nx, 0, mb, s) != hipSuccess ||
        hipMemsetAsync(ss->bms, 0, bb, s) != hipSuccess ||
        hipMemsetAsync(ss->dist, 0, (size_t)max_slots * n * sizeof(int32_t), s) != hipSuccess ||
        hipMemcpyAsync(ss->st.ctl, ss->st.h_ctl, sizeof(MsCtl), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(GSW_EHIP, "session initialisation failed");
  }
  if (st != GSW_OK) {
    ss_free(ss);
    return st;
  }
  ss->start_up.assign((size_t)max_slots, 0);
  ss->source.assign((size_t)max_slots, -1);
  ss->start.assign((size_t)max_slots, 0);
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
      *slot = k;
      return GSW_OK;
    }
  }
  return fail(GSW_EBUSY, "all %d slots are in use", ss->slots);
}

namespace {

// Level boundary of a session: seeds the queries admitted since the last
// one (they join level ss->queued), makes freed slots inert and queues the
// level.  Returns false through *queued when no slot is running or waiting.
gsw_status ss_queue_level(gsw_session* ss, bool* queued_one) {
  *queued_one = false;
  gsw_graph* g = ss->g;
  const hipStream_t s = ss->stream;
  const int W = ss->W;
  const int64_t n = g->n;
  int c = 0;
  bool any_mask = false, running = false;
  const int si = (int)(ss->queued % gsw_session::kStage);
  u64* h_masks = ss->h_masks + (size_t)si * 2 * kMaxWords;
  int32_t* h_seed = ss->h_seed + (size_t)si * 2 * ss->slots;
  long long* h_start = ss->h_start + (size_t)si * ss->slots;
  {
    std::lock_guard<std::mutex> lock(ss->mu);
    u64* clr = h_masks;
    u64* set = h_masks + kMaxWords;
    for (int j = 0; j < kMaxWords; ++j) clr[j] = set[j] = 0ull;
    for (int k = 0; k < ss->slots; ++k) {
      if (ss->state[(size_t)k] == 1) {
        clr[k >> 6] |= 1ull << (k & 63);
        h_seed[c] = ss->source[(size_t)k];
        h_seed[ss->slots + c] = k;
        ss->start_up[(size_t)k] = (long long)ss->queued;
        ss->start[(size_t)k] = ss->queued;
        ss->state[(size_t)k] = 2;
        ++c;
      }
      running = running || ss->state[(size_t)k] == 2 || ss->state[(size_t)k] == 4;
    }
    for (int j = 0; j < W; ++j) {
      set[j] = ss->freed[(size_t)j] & ~clr[j];
      any_mask = any_mask || clr[j] || set[j];
      ss->freed[(size_t)j] = 0ull;
    }
  }
  if (any_mask) {
    GSW_HIP(hipMemcpyAsync(ss->masks, h_masks, 2 * (size_t)kMaxWords * sizeof(u64), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ss_masks, dim3((unsigned)std::min<int64_t>(cdiv(n * W, kMsBlock), 65536)),
                       dim3(kMsBlock), 0, s, ss->vis, n, W, (const u64*)ss->masks,
                       (const u64*)(ss->masks + kMaxWords));
  }
  if (c > 0) {
    std::memcpy(h_start, ss->start_up.data(), (size_t)ss->slots * sizeof(long long));
    GSW_HIP(hipMemcpyAsync(ss->seed, h_seed, 2 * (size_t)ss->slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
    GSW_HIP(hipMemcpyAsync(ss->start_d, h_start, ss->slots * sizeof(long long), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ss_seed, dim3((unsigned)cdiv(c, 256)), dim3(256), 0, s, ss->vis, ss->fr, ss->fbm[0],
                       ss->dist, ss->st.ctl, n, W, (const int32_t*)ss->seed, (const int32_t*)(ss->seed + ss->slots),
                       c);
  }
  GSW_HIP(hipGetLastError());
  if (!running) {
    // nothing to run: no level will be queued after these copies, so wait
    // for them before the staging set can come round again
    if (any_mask) GSW_HIP(hipStreamSynchronize(s));
    return GSW_OK;
  }
  MsArgs a;
  std::memset(&a, 0, sizeof a);
  a.offs = g->offs;
  a.cols = g->cols;
  a.vis = ss->vis;
  a.fr = ss->fr;
  a.frn = ss->frn;
  a.nx = ss->nx;
  a.fbm = ss->fbm[0];
  a.fbm_n = ss->fbm[1];
  a.tbm = ss->bms + 2 * cdiv(n, 64);
  a.heavy = g->heavy;
  a.n_heavy = g->n_heavy;
  a.dist = ss->dist;
  a.start = ss->start_d;
  a.ctl = ss->st.ctl;
  a.n = n;
  a.W = W;
  a.B = W * 64;
  GSW_TRY(launch_ms_level(a, ss->st, group_lanes(W), kMsBlock, s));
  GSW_HIP(hipGetLastError());
  std::swap(ss->fr, ss->frn);
  std::swap(ss->fbm[0], ss->fbm[1]);
  ss->queued += 1;
  *queued_one = true;
  return GSW_OK;
}

}  // namespace

gsw_status gsw_session_step(gsw_session* ss, int32_t max_levels, int32_t* finished, int32_t finished_cap,
                            int32_t* n_finished, int32_t* levels_run) {
  clear_error();
  if (n_finished) *n_finished = 0;
  if (levels_run) *levels_run = 0;
  if (!ss || max_levels < 1 || (finished_cap > 0 && !finished)) return fail(GSW_EINVAL, "bad step arguments");
  std::lock_guard<std::mutex> step_lock(ss->step_mu);
  GSW_HIP(hipSetDevice(ss->g->device));
  // One level is kept queued beyond the one being waited for, so the device
  // goes from level to level without waiting for the host; queries admitted
  // meanwhile join at the next boundary the host reaches.
  int32_t nfin = 0, run = 0;
  while (run < max_levels) {
    while (ss->queued - ss->done < 2) {
      bool q = false;
      GSW_TRY(ss_queue_level(ss, &q));
      if (!q) break;
    }
    if (ss->queued == ss->done) break;  // nothing queued, nothing running
    const volatile u64* rec = nullptr;
    GSW_TRY(wait_record(ss->st, ss->done, ss->stream, "session", &rec));
    const int64_t d = ss->done;
    ss->done += 1;
    ++run;
    std::lock_guard<std::mutex> lock(ss->mu);
    for (int k = 0; k < ss->slots; ++k) {
      const int8_t stk = ss->state[(size_t)k];
      if ((stk != 2 && stk != 4) || ss->start[(size_t)k] > d) continue;
      if (((rec[kRecActive + (k >> 6)] >> (k & 63)) & 1ull) != 0ull) continue;
      if (stk == 2) {
        ss->state[(size_t)k] = 3;
        if (nfin < finished_cap) finished[nfin] = k;
        ++nfin;
      } else {
        // a cancelled query whose frontier is empty: its partial levels are
        // cleared (in stream order, after every level queued so far, none of
        // which can write the row any more) and the slot is free again
        hipLaunchKernelGGL(k_ss_clear, dim3((unsigned)std::min<int64_t>(cdiv(ss->g->n, kMsBlock), 65536)),
                           dim3(kMsBlock), 0, ss->stream, ss->dist + (int64_t)k * ss->g->n, ss->g->n);
        if (hipGetLastError() != hipSuccess) return fail(GSW_EHIP, "clearing a cancelled slot failed");
        ss->state[(size_t)k] = 0;
        ss->source[(size_t)k] = -1;
      }
    }
    if (nfin > 0) break;
  }
  if (n_finished) *n_finished = nfin;
  if (levels_run) *levels_run = run;
  return GSW_OK;
}

gsw_status gsw_session_fetch(gsw_session* ss, int32_t slot, int32_t* levels, int32_t device_ptr) {
  clear_error();
  if (!ss || !levels) return fail(GSW_EINVAL, "null argument");
  std::lock_guard<std::mutex> step_lock(ss->step_mu);
  {
    std::lock_guard<std::mutex> lock(ss->mu);
    if (slot < 0 || slot >= ss->slots || ss->state[(size_t)slot] != 3)
      return fail(GSW_EINVAL, "slot %d has no finished result", slot);
  }
  GSW_HIP(hipSetDevice(ss->g->device));
  const hipStream_t s = ss->stream;
  const int64_t n = ss->g->n;
  int32_t* row = ss->dist + (int64_t)slot * n;
  int32_t* dst = device_ptr ? levels : ss->take;
  hipLaunchKernelGGL(k_ss_take, dim3((unsigned)std::min<int64_t>(cdiv(n, kMsBlock), 65536)), dim3(kMsBlock), 0, s,
                     row, dst, n);
  GSW_HIP(hipGetLastError());
  if (!device_ptr)
    GSW_HIP(hipMemcpyAsync(levels, ss->take, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GSW_HIP(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lock(ss->mu);
  ss->state[(size_t)slot] = 0;
  ss->source[(size_t)slot] = -1;
  ss->freed[(size_t)(slot >> 6)] |= 1ull << (slot & 63);
  return GSW_OK;
}

gsw_status gsw_session_cancel(gsw_session* ss, int32_t slot) {
  clear_error();
  if (!ss) return fail(GSW_EINVAL, "session is null");
  std::lock_guard<std::mutex> lock(ss->mu);
  if (slot < 0 || slot >= ss->slots) return fail(GSW_EINVAL, "slot %d out of [0, %d)", slot, ss->slots);
  switch (ss->state[(size_t)slot]) {
    case 1:  // not seeded yet: its bits are still inert
      ss->state[(size_t)slot] = 0;
      ss->source[(size_t)slot] = -1;
      return GSW_OK;
    case 2:  // inert from the next boundary; gsw_session_step frees it once its frontier is empty
      ss->state[(size_t)slot] = 4;
      ss->freed[(size_t)(slot >> 6)] |= 1ull << (slot & 63);
      return GSW_OK;
    default:
      return fail(GSW_EINVAL, "slot %d holds no admitted or running query (state %d)", slot,
                  (int)ss->state[(size_t)slot]);
  }
}

gsw_status gsw_session_info(const gsw_session* css, int32_t* slots, int32_t* busy, int64_t* iteration,
                            size_t* dev_bytes) {
  clear_error();
  if (!css) return fail(GSW_EINVAL, "session is null");
  gsw_session* ss = const_cast<gsw_session*>(css);
  std::lock_guard<std::mutex> lock(ss->mu);
  if (slots) *slots = ss->slots;
  if (busy) {
    int32_t b = 0;
    for (int8_t x : ss->state) b += x != 0;
    *busy = b;
  }
  if (iteration) *iteration = ss->done;
  if (dev_bytes) *dev_bytes = ss->bytes;
  return GSW_OK;
}

gsw_status gsw_session_rebase(gsw_session* ss, int64_t iteration) {
  clear_error();
  if (!ss) return fail(GSW_EINVAL, "session is null");
  if (iteration < 0 || iteration > ((int64_t)1 << 62))
    return fail(GSW_EINVAL, "iteration %lld out of [0, 2^62]", (long long)iteration);
  std::lock_guard<std::mutex> step_lock(ss->step_mu);
  std::lock_guard<std::mutex> lock(ss->mu);
  for (int k = 0; k < ss->slots; ++k)
    if (ss->state[(size_t)k] == 2 || ss->state[(size_t)k] == 4) return fail(GSW_EBUSY, "slot %d is running", k);
  // levels still queued have no running query to advance: waiting for them
  // here and dropping their records changes no slot's state
  GSW_HIP(hipSetDevice(ss->g->device));
  GSW_HIP(hipStreamSynchronize(ss->stream));
  // records of earlier levels must not be mistaken for those of the new numbering
  std::memset(ss->st.ring, 0, (size_t)kRing * kRecWords * sizeof(u64));
  hipLaunchKernelGGL(k_ss_set_level, dim3(1), dim3(64), 0, ss->stream, ss->st.ctl, (long long)iteration);
  GSW_HIP(hipGetLastError());
  GSW_HIP(hipStreamSynchronize(ss->stream));
  ss->queued = iteration;
  ss->done = iteration;
  return GSW_OK;
}

gsw_status gsw_session_set_thresholds(gsw_session* ss, float push_to_pull, float pull_to_push) {
  clear_error();
  if (!ss) return fail(GSW_EINVAL, "session is null");
  std::lock_guard<std::mutex> lock(ss->step_mu);
  ss->push_to_pull = push_to_pull;
  ss->pull_to_push = pull_to_push;
  GSW_HIP(hipSetDevice(ss->g->device));
  hipLaunchKernelGGL(k_ss_thresholds, dim3(1), dim3(64), 0, ss->stream, ss->st.ctl, (double)push_to_pull,
                     (double)pull_to_push);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

}  // extern "C"
