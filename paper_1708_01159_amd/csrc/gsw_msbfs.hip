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

#include "gsw_internal.h"

namespace gsw {
namespace {

typedef unsigned long long u64;

constexpr int kMsBlock = 256;
constexpr int kMsMaxGrid = 2048;
constexpr int kMsStats = 8;        // stat counters, spread like the queue bins
constexpr int kMsStatStride = 32;  // u64 words between counters
constexpr int kMsLong = 32;        // rows longer than this are walked by the whole wave
constexpr int kMsHeavy = 1024;     // top-down: rows longer than this go through the chunk list
constexpr int kMsChunk = 256;      // arcs per chunk of a heavy row
constexpr int kMaxWords = GSW_MSBFS_MAX_SOURCES / 64;  // mask words per vertex at most
constexpr int kMaxSlots = GSW_MSBFS_MAX_SOURCES;

// Mapped host words written by the finalize kernel: [0] vertices with new
// bits (stored last, ~0 while the level runs), [1] their degree sum,
// [kHostActive + j] OR of the new frontier's word j, [kHostEf + k] source k's
// new frontier edges.
constexpr int kHostActive = 2;
constexpr int kHostEf = 32;
constexpr int kHostWords = kHostEf + kMaxSlots;

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
  const int32_t* start;
  int64_t n;
  int32_t W, B;  // words per vertex, level bytes per vertex
  int32_t d;
  int32_t any_push;       // the top-down pass ran this level (nx and tbm hold its bits)
  int32_t any_pull;       // some source expands bottom-up this level
  u64 pmask[kMaxWords];   // sources expanded top-down this level
  u64 qmask[kMaxWords];   // sources expanded bottom-up this level
};

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Sources with bit positions >= B in the last word do not exist: treat them
// as visited so they never look unreached.
__device__ __forceinline__ u64 valid_bits(int j, int W, int B) {
  if (j < W - 1 || (B & 63) == 0) return ~0ull;
  return (1ull << (B & 63)) - 1ull;
}

// Word j of a per-source mask held in the kernel arguments (uniform loads,
// then a per-lane select).
__device__ __forceinline__ u64 mask_word(const u64 (&m)[kMaxWords], int j) {
  u64 r = 0ull;
#pragma unroll
  for (int w = 0; w < kMaxWords; ++w)
    if (w == j) r = m[w];
  return r;
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

// 8 bits -> 8 bytes holding 0x01 where the bit is set.
__device__ __forceinline__ u64 bits_to_bytes(u64 c) {
  c = (c | (c << 28)) & 0x0000000F0000000Full;
  c = (c | (c << 14)) & 0x0003000300030003ull;
  c = (c | (c << 7)) & 0x0101010101010101ull;
  return c;
}

// Levels d+1 for the sources in `m` (word j) at vertex v.  Only v's group
// writes v's levels, so the batch's 8-byte read-modify-writes need no atomics.
__device__ __forceinline__ void write_levels(const MsArgs& a, int64_t v, int j, u64 m) {
  if (a.dist) {
    while (m) {
      const int b = __ffsll((long long)m) - 1;
      m &= m - 1ull;
      const int slot = j * 64 + b;
      a.dist[(int64_t)slot * a.n + v] = a.d + 2 - a.start[slot];
    }
    return;
  }
  u64* row = reinterpret_cast<u64*>(a.lev + v * (int64_t)a.B + (int64_t)j * 64);
  const u64 val = (u64)(uint8_t)(a.d + 1 > 127 ? 127 : a.d + 1) * 0x0101010101010101ull;
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
  w.wave = ((int64_t)blockIdx.x * kMsBlock + threadIdx.x) >> 6;
  w.nwaves = ((int64_t)gridDim.x * kMsBlock) >> 6;
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
__device__ __forceinline__ void push_arcs(const MsArgs& a, u64 f, int j, int64_t beg, int64_t end,
                                          int step) {
  for (int64_t e = beg; e < end; e += step) {
    const int64_t v = a.cols[e];
    const u64 m = f & ~a.vis[v * a.W + j];
    if (m) {
      const u64 old = atomicOr(a.nx + v * a.W + j, m);
      if (!old) atomicOr(a.tbm + (v >> 6), 1ull << (v & 63));
    }
  }
}

// Every frontier vertex u of a top-down source: lane j pushes
// fr[u][j] & pmask[j] along u's arcs.
__global__ void __launch_bounds__(kMsBlock) k_ms_push(MsArgs a, int G) {
  const Wave w = wave_of(G);
  const int j = w.j;
  const u64 pm = j < a.W ? mask_word(a.pmask, j) : 0ull;
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
  // heavy rows: one chunk per wave step, for the chunks whose vertex is in
  // the frontier
  for (int64_t c0 = w.wave * 64; c0 < a.n_heavy; c0 += w.nwaves * 64) {
    const int64_t c = c0 + w.lane;
    u64 ent = 0ull;
    bool live = false;
    if (c < a.n_heavy) {
      ent = a.heavy[c];
      const int64_t u = (int64_t)(ent >> 32);
      live = ((a.fbm[u >> 6] >> (u & 63)) & 1ull) != 0ull;
    }
    u64 lm = __ballot(live);
    while (lm) {
      const int src = __ffsll((long long)lm) - 1;
      lm &= lm - 1ull;
      const u64 e_ = __shfl(ent, src);
      const int64_t u = (int64_t)(e_ >> 32);
      const int64_t ci = (int64_t)(e_ & 0xffffffffull);
      const u64 fw = pm ? (a.fr[u * a.W + j] & pm) : 0ull;
      if (__ballot(fw != 0ull) == 0ull) continue;
      const int64_t b = a.offs[u] + ci * kMsChunk;
      const int64_t en = std::min<int64_t>(a.offs[u + 1], b + kMsChunk);
      if (fw) push_arcs(a, fw, j, b + w.gi, en, w.gpw);
    }
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
__global__ void __launch_bounds__(kMsBlock) k_ms_level(MsArgs a, int G) {
  __shared__ u64 s_ef[kMaxSlots];
  const Wave w = wave_of(G);
  const int j = w.j;
  const bool lane_live = j < a.W;
  const u64 qm = lane_live ? mask_word(a.qmask, j) : 0ull;
  const int nslots = a.W * 64;
  for (int k = threadIdx.x; k < nslots; k += kMsBlock) s_ef[k] = 0ull;
  __syncthreads();
  u64 nv = 0, ne = 0, act = 0;
  const int64_t nwords = (a.n + 63) / 64;
  for (int64_t wd = w.wave; wd < nwords; wd += w.nwaves) {
    const int64_t base = wd * 64;
    const u64 valid = base + 64 <= a.n ? ~0ull : ((1ull << (a.n - base)) - 1ull);
    const u64 stale = a.fbm_n[wd];
    const u64 touched = a.any_push ? a.tbm[wd] : 0ull;
    const u64 work = (a.any_pull ? ~0ull : (touched | stale)) & valid;
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
          write_levels(a, v, j, nb);
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
  for (int k = threadIdx.x; k < nslots; k += kMsBlock)
    if (s_ef[k]) atomicAdd(row + k, s_ef[k]);
}

// Sums the spread counters into mapped host memory (layout at kHostEf), then
// zeroes them.  Word 0 is stored last, after every other word is visible.
__global__ void __launch_bounds__(256) k_ms_finalize(u64* stats, u64* active, u64* slot_ef, int W,
                                                     int nslots, u64* host) {
  const int t = threadIdx.x;
  for (int k = t; k < nslots; k += 256) {
    u64 x = 0ull;
    for (int r = 0; r < kMsStats; ++r) {
      x += slot_ef[r * kMaxSlots + k];
      slot_ef[r * kMaxSlots + k] = 0ull;
    }
    __hip_atomic_store(host + kHostEf + k, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (t < W) {
    u64 x = 0ull;
    for (int r = 0; r < kMsStats; ++r) {
      x |= active[r * kMaxWords + t];
      active[r * kMaxWords + t] = 0ull;
    }
    __hip_atomic_store(host + kHostActive + t, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  u64 v = 0, e = 0;
  if (t < 64) {  // wave 0
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
  }
  __threadfence_system();
  __syncthreads();
  if (t == 0) {
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

// Admitted slots: the source's bit in vis, in the current frontier and its
// bitmap, level 0 (stored as 1).
__global__ void k_ss_seed(u64* vis, u64* fr, u64* fbm, int32_t* dist, int64_t n, int W,
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

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int group_lanes(int W) {
  int G = 1;
  while (G < W) G <<= 1;
  return G;  // W <= 16 -> G <= 16
}

// One wave per 64-vertex word for one pass, at most kMsMaxGrid blocks.
inline unsigned ms_grid(int64_t n) {
  const int64_t blocks = cdiv(cdiv(n, 64), kMsBlock / 64);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, kMsMaxGrid));
}

// Spread statistics counters and the mapped host words of one traversal.
struct LevelStats {
  u64 *stats = nullptr, *active = nullptr, *slot_ef = nullptr;
  u64 *h = nullptr, *d_h = nullptr;  // mapped host memory (kHostWords)
  size_t bytes = 0;
};

gsw_status stats_alloc(LevelStats* st) {
  const size_t sb = (size_t)kMsStats * kMsStatStride * sizeof(u64);
  const size_t ab = (size_t)kMsStats * kMaxWords * sizeof(u64);
  const size_t eb = (size_t)kMsStats * kMaxSlots * sizeof(u64);
  void** ps[] = {(void**)&st->stats, (void**)&st->active, (void**)&st->slot_ef};
  const size_t bs[] = {sb, ab, eb};
  for (int k = 0; k < 3; ++k) {
    if (hipMalloc(ps[k], bs[k]) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for level statistics failed", bs[k]);
    }
    st->bytes += bs[k];
    GSW_HIP(hipMemset(*ps[k], 0, bs[k]));
  }
  GSW_HIP(hipHostMalloc((void**)&st->h, kHostWords * sizeof(u64), hipHostMallocMapped | hipHostMallocCoherent));
  GSW_HIP(hipHostGetDevicePointer((void**)&st->d_h, st->h, 0));
  return GSW_OK;
}

void stats_free(LevelStats* st) {
  void* p[] = {st->stats, st->active, st->slot_ef};
  for (void* x : p)
    if (x) (void)hipFree(x);
  if (st->h) (void)hipHostFree(st->h);
  *st = LevelStats();
}

// Spins until the level's finalize kernel has published word 0, polling the
// stream for errors now and then.
gsw_status stats_wait(const LevelStats& st, hipStream_t s, const char* who) {
  volatile u64* f = st.h;
  for (uint64_t it = 0;; ++it) {
    if (f[0] != ~0ull) return GSW_OK;
    if ((it & 4095u) == 4095u) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (f[0] != ~0ull) continue;
        return fail(GSW_EHIP, "%s: level finished without reporting its statistics", who);
      }
      if (e != hipErrorNotReady) return fail(GSW_EHIP, "%s: %s", who, hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
}

// Per-source direction, the single-source rule applied to each source:
// bottom-up once its frontier's edges exceed push_to_pull of all arcs, back
// to top-down below pull_to_push.  Sources not running are in neither mask.
struct Direction {
  std::vector<uint8_t> pull;
  std::vector<u64> ef;
  void reset(int slots) {
    pull.assign((size_t)slots, 0);
    ef.assign((size_t)slots, 0ull);
  }
  void start(int k) {
    pull[(size_t)k] = 0;
    ef[(size_t)k] = 0ull;
  }
  // running: W words; fills pm/qm (kMaxWords words each)
  void choose(const u64* running, int W, bool pull_ok, double a_arcs, double b_arcs, u64* pm,
              u64* qm) {
    for (int j = 0; j < kMaxWords; ++j) pm[j] = qm[j] = 0ull;
    for (int j = 0; j < W; ++j) {
      u64 r = running[j];
      while (r) {
        const int b = __builtin_ctzll(r);
        r &= r - 1ull;
        const size_t k = (size_t)j * 64 + b;
        if (pull_ok) {
          if (!pull[k] && (double)ef[k] > a_arcs) pull[k] = 1;
          else if (pull[k] && (double)ef[k] < b_arcs) pull[k] = 0;
        } else {
          pull[k] = 0;
        }
        (pull[k] ? qm : pm)[j] |= 1ull << b;
      }
    }
  }
};

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

// Launches one level: the top-down pass when some source pushes, then the
// bottom-up + update pass and the finalize kernel.  a.pmask / a.qmask and
// the mask and bitmap pointers are set by the caller.
gsw_status launch_ms_level(MsArgs& a, const LevelStats& st, int G, int nslots, hipStream_t s) {
  a.stats = st.stats;
  a.active = st.active;
  a.slot_ef = st.slot_ef;
  a.any_push = 0;
  a.any_pull = 0;
  for (int j = 0; j < kMaxWords; ++j) {
    a.any_push |= a.pmask[j] != 0ull;
    a.any_pull |= a.qmask[j] != 0ull;
  }
  const unsigned grid = ms_grid(a.n);
  if (a.any_push) hipLaunchKernelGGL(k_ms_push, dim3(grid), dim3(kMsBlock), 0, s, a, G);
  hipLaunchKernelGGL(k_ms_level, dim3(grid), dim3(kMsBlock), 0, s, a, G);
  hipLaunchKernelGGL(k_ms_finalize, dim3(1), dim3(256), 0, s, st.stats, st.active, st.slot_ef, a.W, nslots,
                     st.d_h);
  GSW_HIP(hipGetLastError());
  return GSW_OK;
}

}  // namespace

struct MsWorkspace {
  int64_t n = 0;
  int W = 0, B = 0;
  u64 *vis = nullptr, *fr = nullptr, *frn = nullptr, *nx = nullptr;
  u64* bms = nullptr;  // 3 bitmaps of ceil(n/64) words: frontier d, frontier d+1, touched
  int8_t* lev = nullptr;
  int32_t* src = nullptr;
  LevelStats st;
  size_t bytes = 0;
};

namespace {
void ms_free(MsWorkspace* m) {
  if (!m) return;
  void* p[] = {m->vis, m->fr, m->frn, m->nx, m->bms, m->lev, m->src};
  for (void* x : p)
    if (x) (void)hipFree(x);
  stats_free(&m->st);
  delete m;
}

gsw_status ms_ensure(gsw_graph* g, int W) {
  GSW_TRY(ensure_heavy(g));
  MsWorkspace*& m = g->ms;
  if (m && m->W >= W) return GSW_OK;
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
  if (st == GSW_OK) st = stats_alloc(&m->st);
  if (st != GSW_OK) {
    ms_free(m);
    m = nullptr;
    return st;
  }
  m->bytes += m->st.bytes;
  return GSW_OK;
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
  o->push_to_pull = 0.002f;
  o->pull_to_push = 0.0005f;
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
  GSW_TRY(ms_ensure(g, W));
  MsWorkspace* m = g->ms;
  const hipStream_t s = pick_stream(g, o->stream);
  const int B = W * 64;  // level bytes per vertex in the workspace
  const int G = group_lanes(W);
  const int64_t nw = cdiv(g->n, 64);
  u64* fbm[2] = {m->bms, m->bms + nw};
  GSW_HIP(hipMemcpyAsync(m->src, sources, (size_t)n_sources * sizeof(int32_t), hipMemcpyHostToDevice, s));
  {
    const int64_t work = std::max<int64_t>(g->n * W, g->n * (int64_t)B / 8);
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(work, kMsBlock), 65536);
    hipLaunchKernelGGL(k_ms_init, dim3(grid), dim3(kMsBlock), 0, s, m->vis, m->fr, m->frn, m->nx, m->bms,
                       m->lev, g->n, W, n_sources, B);
    hipLaunchKernelGGL(k_ms_sources, dim3((unsigned)cdiv(n_sources, 256)), dim3(256), 0, s, m->vis,
                       m->fr, fbm[0], m->lev, W, B, (const int32_t*)m->src, n_sources);
    GSW_HIP(hipGetLastError());
  }
  MsArgs a;
  std::memset(&a, 0, sizeof a);
  a.offs = g->offs;
  a.cols = g->cols;
  a.vis = m->vis;
  a.nx = m->nx;
  a.tbm = m->bms + 2 * nw;
  a.heavy = g->heavy;
  a.n_heavy = g->n_heavy;
  a.lev = m->lev;
  a.n = g->n;
  a.W = W;
  a.B = B;
  u64* cur = m->fr;
  u64* nxt = m->frn;
  std::vector<u64> running((size_t)W, 0ull);
  for (int32_t i = 0; i < n_sources; ++i) running[(size_t)(i >> 6)] |= 1ull << (i & 63);
  Direction dir;
  dir.reset(B);
  const double nnz = (double)std::max<int64_t>(g->nnz, 1);
  int32_t d = 0;
  for (;; ++d) {
    dir.choose(running.data(), W, pull_ok, o->push_to_pull * nnz, o->pull_to_push * nnz, a.pmask, a.qmask);
    a.fr = cur;
    a.frn = nxt;
    a.fbm = fbm[d & 1];
    a.fbm_n = fbm[(d + 1) & 1];
    a.d = d;
    m->st.h[0] = ~0ull;
    GSW_TRY(launch_ms_level(a, m->st, G, n_sources, s));
    GSW_TRY(stats_wait(m->st, s, "batched BFS"));
    const volatile u64* h = m->st.h;
    if (h[0] == 0) break;
    if (d + 1 > GSW_MSBFS_LEVEL_CAP) {
      (void)hipStreamSynchronize(s);
      return fail(GSW_ERANGE, "a source reaches depth %d > %d (int8 levels)", d + 1, GSW_MSBFS_LEVEL_CAP);
    }
    for (int j = 0; j < W; ++j) running[(size_t)j] = h[kHostActive + j];
    for (int32_t k = 0; k < n_sources; ++k) dir.ef[(size_t)k] = h[kHostEf + k];
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
  int32_t *dist = nullptr, *start_d = nullptr, *seed = nullptr;  // seed: src[slots] then slot[slots]
  int32_t* take = nullptr;  // device staging for fetches into host memory
  LevelStats st;
  // pinned staging for the per-level uploads: masks, then seed src/slot, then start
  u64* h_masks = nullptr;
  int32_t* h_seed = nullptr;
  int32_t* h_start = nullptr;
  std::vector<int32_t> source;
  std::vector<int8_t> state;  // 0 free, 1 admitted (seeded at the next level boundary), 2 running, 3 finished
  std::vector<u64> freed;     // slots freed since the last level (made inert then)
  Direction dir;
  int64_t it = 0;  // levels run by this session
  float push_to_pull = 0.002f, pull_to_push = 0.0005f;
  hipStream_t stream = nullptr;
  size_t bytes = 0;
  std::mutex mu;       // host state shared with admit / fetch / info
  std::mutex step_mu;  // one step or fetch at a time
};

namespace {

void ss_free(gsw_session* ss) {
  if (!ss) return;
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
               {(void**)&ss->start_d, (size_t)max_slots * sizeof(int32_t)},
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
  gsw_status st = stats_alloc(&ss->st);
  if (st == GSW_OK) {
    ss->bytes += ss->st.bytes;
    if (hipStreamCreateWithFlags(&ss->stream, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&ss->h_masks, 2 * (size_t)kMaxWords * sizeof(u64), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ss->h_seed, 2 * (size_t)max_slots * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ss->h_start, (size_t)max_slots * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      st = fail(GSW_EHIP, "session stream or pinned staging memory");
  }
  if (st == GSW_OK) {
    const hipStream_t s = ss->stream;
    // every slot starts inert: visited everywhere, in no frontier, not reached
    if (hipMemsetAsync(ss->vis, 0xff, mb, s) != hipSuccess || hipMemsetAsync(ss->fr, 0, mb, s) != hipSuccess ||
        hipMemsetAsync(ss->frn, 0, mb, s) != hipSuccess || hipMemsetAsync(ss->nx, 0, mb, s) != hipSuccess ||
        hipMemsetAsync(ss->bms, 0, bb, s) != hipSuccess ||
        hipMemsetAsync(ss->dist, 0, (size_t)max_slots * n * sizeof(int32_t), s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(GSW_EHIP, "session initialisation failed");
  }
  if (st != GSW_OK) {
    ss_free(ss);
    return st;
  }
  std::memset(ss->h_start, 0, (size_t)max_slots * sizeof(int32_t));
  ss->source.assign((size_t)max_slots, -1);
  ss->state.assign((size_t)max_slots, 0);
  ss->freed.assign((size_t)ss->W, 0ull);
  ss->dir.reset(max_slots);
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

gsw_status gsw_session_step(gsw_session* ss, int32_t max_levels, int32_t* finished, int32_t finished_cap,
                            int32_t* n_finished, int32_t* levels_run) {
  clear_error();
  if (n_finished) *n_finished = 0;
  if (levels_run) *levels_run = 0;
  if (!ss || max_levels < 1 || (finished_cap > 0 && !finished)) return fail(GSW_EINVAL, "bad step arguments");
  std::lock_guard<std::mutex> step_lock(ss->step_mu);
  gsw_graph* g = ss->g;
  GSW_HIP(hipSetDevice(g->device));
  const hipStream_t s = ss->stream;
  const int W = ss->W;
  const int64_t n = g->n;
  const int G = group_lanes(W);
  const bool pull_ok = g->symmetric != 0;
  const double nnz = (double)std::max<int64_t>(g->nnz, 1);
  MsArgs a;
  std::memset(&a, 0, sizeof a);
  a.offs = g->offs;
  a.cols = g->cols;
  a.vis = ss->vis;
  a.nx = ss->nx;
  a.tbm = ss->bms + 2 * cdiv(n, 64);
  a.heavy = g->heavy;
  a.n_heavy = g->n_heavy;
  a.n = n;
  a.W = W;
  a.B = W * 64;
  a.dist = ss->dist;
  a.start = ss->start_d;
  int32_t nfin = 0, run = 0;
  std::vector<u64> running((size_t)W);
  for (; run < max_levels; ++run) {
    // level boundary: take the queries admitted since the last level, make
    // freed slots inert, pick each running slot's direction
    int c = 0;
    bool any_mask = false;
    {
      std::lock_guard<std::mutex> lock(ss->mu);
      u64* clr = ss->h_masks;
      u64* set = ss->h_masks + kMaxWords;
      for (int j = 0; j < kMaxWords; ++j) clr[j] = set[j] = 0ull;
      for (int k = 0; k < ss->slots; ++k)
        if (ss->state[(size_t)k] == 1) {
          clr[k >> 6] |= 1ull << (k & 63);
          ss->h_seed[c] = ss->source[(size_t)k];
          ss->h_seed[ss->slots + c] = k;
          ss->h_start[k] = (int32_t)ss->it;
          ss->state[(size_t)k] = 2;
          ss->dir.start(k);
          ++c;
        }
      for (int j = 0; j < W; ++j) {
        set[j] = ss->freed[(size_t)j] & ~clr[j];
        any_mask = any_mask || clr[j] || set[j];
        ss->freed[(size_t)j] = 0ull;
      }
      std::fill(running.begin(), running.end(), 0ull);
      for (int k = 0; k < ss->slots; ++k)
        if (ss->state[(size_t)k] == 2) running[(size_t)(k >> 6)] |= 1ull << (k & 63);
    }
    bool any_running = false;
    for (u64 r : running) any_running = any_running || r;
    if (any_mask) {
      GSW_HIP(hipMemcpyAsync(ss->masks, ss->h_masks, 2 * (size_t)kMaxWords * sizeof(u64), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_ss_masks, dim3((unsigned)std::min<int64_t>(cdiv(n * W, kMsBlock), 65536)),
                         dim3(kMsBlock), 0, s, ss->vis, n, W, (const u64*)ss->masks,
                         (const u64*)(ss->masks + kMaxWords));
    }
    if (c > 0) {
      GSW_HIP(hipMemcpyAsync(ss->seed, ss->h_seed, 2 * (size_t)ss->slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
      GSW_HIP(hipMemcpyAsync(ss->start_d, ss->h_start, ss->slots * sizeof(int32_t), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_ss_seed, dim3((unsigned)cdiv(c, 256)), dim3(256), 0, s, ss->vis, ss->fr, ss->fbm[0],
                         ss->dist, n, W, (const int32_t*)ss->seed, (const int32_t*)(ss->seed + ss->slots), c);
    }
    GSW_HIP(hipGetLastError());
    if (!any_running) {
      if (any_mask) GSW_HIP(hipStreamSynchronize(s));
      break;
    }
    ss->dir.choose(running.data(), W, pull_ok, ss->push_to_pull * nnz, ss->pull_to_push * nnz, a.pmask, a.qmask);
    a.fr = ss->fr;
    a.frn = ss->frn;
    a.fbm = ss->fbm[0];
    a.fbm_n = ss->fbm[1];
    a.d = (int32_t)ss->it;
    ss->st.h[0] = ~0ull;
    GSW_TRY(launch_ms_level(a, ss->st, G, ss->slots, s));
    GSW_TRY(stats_wait(ss->st, s, "session"));
    ss->it += 1;
    std::swap(ss->fr, ss->frn);
    std::swap(ss->fbm[0], ss->fbm[1]);
    const volatile u64* h = ss->st.h;
    std::lock_guard<std::mutex> lock(ss->mu);
    for (int k = 0; k < ss->slots; ++k) {
      if (ss->state[(size_t)k] != 2) continue;
      ss->dir.ef[(size_t)k] = h[kHostEf + k];
      if (((h[kHostActive + (k >> 6)] >> (k & 63)) & 1ull) == 0ull) {
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
  if (iteration) *iteration = ss->it;
  if (dev_bytes) *dev_bytes = ss->bytes;
  return GSW_OK;
}

gsw_status gsw_session_set_thresholds(gsw_session* ss, float push_to_pull, float pull_to_push) {
  clear_error();
  if (!ss) return fail(GSW_EINVAL, "session is null");
  std::lock_guard<std::mutex> lock(ss->step_mu);
  ss->push_to_pull = push_to_pull;
  ss->pull_to_push = pull_to_push;
  return GSW_OK;
}

}  // extern "C"
