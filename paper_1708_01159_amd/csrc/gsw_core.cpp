// Host side of libgsw: errors, graph validation and residency (with the
// transpose of a directed graph), degree statistics, the per-level feature
// vector, the decision tree and its JSON reader.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gsw_internal.h"

namespace gsw {

namespace {
thread_local char g_err[1024] = "";
}

gsw_status fail(gsw_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = '\0'; }

namespace {

// Linear interpolation between order statistics at fraction p of the sorted
// array (the definition numpy.percentile uses by default).
double quantile_sorted(const std::vector<int64_t>& s, double p) {
  const double pos = (double)(s.size() - 1) * p;
  const size_t lo = (size_t)std::floor(pos);
  const size_t hi = std::min(lo + 1, s.size() - 1);
  const double t = pos - (double)lo;
  const double a = (double)s[lo], b = (double)s[hi];
  return t >= 0.5 ? b - (b - a) * (1.0 - t) : a + (b - a) * t;
}

// {min, q1, median, q3, max, std} of a degree sequence (taken by value: sorted here).
void sequence_stats(std::vector<int64_t> deg, double out[6]) {
  const int64_t n = (int64_t)deg.size();
  long double sum = 0.0L;
  for (int64_t v = 0; v < n; ++v) sum += (long double)deg[(size_t)v];
  const long double mean = sum / (long double)n;
  long double ss = 0.0L;
  for (int64_t v = 0; v < n; ++v) {
    const long double x = (long double)deg[(size_t)v] - mean;
    ss += x * x;
  }
  std::sort(deg.begin(), deg.end());
  out[0] = (double)deg.front();
  out[1] = quantile_sorted(deg, 0.25);
  out[2] = quantile_sorted(deg, 0.50);
  out[3] = quantile_sorted(deg, 0.75);
  out[4] = (double)deg.back();
  out[5] = (double)std::sqrt(ss / (long double)n);
}

void degree_stats(int64_t n, const int64_t* offs, double out[6]) {
  std::vector<int64_t> deg((size_t)n);
  for (int64_t v = 0; v < n; ++v) deg[(size_t)v] = offs[v + 1] - offs[v];
  sequence_stats(std::move(deg), out);
}

// Transpose of a CSR: row v of (toffs, tcols) lists the u with an arc u -> v,
// ascending (u is visited in increasing order), repeats kept.
void transpose_csr(int64_t n, const int64_t* offs, const int32_t* cols, std::vector<int64_t>& toffs,
                   std::vector<int32_t>& tcols) {
  const int64_t nnz = offs[n];
  toffs.assign((size_t)n + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) ++toffs[(size_t)cols[e] + 1];
  for (int64_t v = 0; v < n; ++v) toffs[(size_t)v + 1] += toffs[(size_t)v];
  tcols.resize((size_t)nnz);
  std::vector<int64_t> fill(toffs.begin(), toffs.end() - 1);
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = offs[u]; e < offs[u + 1]; ++e) tcols[(size_t)fill[(size_t)cols[e]]++] = (int32_t)u;
}

// The graph features 0..19 (n, arcs, out-, in-, absolute-degree statistics).
// in_offs/in_cols: the transpose (rows ascending), or null on a symmetric
// graph, whose three distributions are the degree distribution.
void graph_features(int64_t n, int64_t nnz, const int64_t* offs, const int32_t* cols, const int64_t* in_offs,
                    const int32_t* in_cols, double out[GSW_N_GRAPH_FEATURES]) {
  out[0] = (double)n;
  out[1] = (double)nnz;
  degree_stats(n, offs, out + 2);
  if (!in_offs) {
    for (int i = 0; i < 6; ++i) out[8 + i] = out[14 + i] = out[2 + i];
    return;
  }
  degree_stats(n, in_offs, out + 8);
  // absolute degree: out(v) + in(v) - (arcs v -> u whose reverse u -> v exists)
  std::vector<int64_t> ad((size_t)n);
  for (int64_t v = 0; v < n; ++v) {
    const int32_t* ib = in_cols + in_offs[v];
    const int32_t* ie = in_cols + in_offs[v + 1];
    int64_t both = 0;
    for (int64_t e = offs[v]; e < offs[v + 1]; ++e)
      if (std::binary_search(ib, ie, cols[e])) ++both;
    ad[(size_t)v] = (offs[v + 1] - offs[v]) + (in_offs[v + 1] - in_offs[v]) - both;
  }
  sequence_stats(std::move(ad), out + 14);
}

gsw_status validate_csr(int64_t n, int64_t nnz, const int64_t* offs, const int32_t* cols) {
  if (n < 1 || n >= ((int64_t)1 << 31)) return fail(GSW_EINVAL, "n=%lld out of [1, 2^31)", (long long)n);
  if (nnz < 0) return fail(GSW_EINVAL, "nnz=%lld is negative", (long long)nnz);
  if (!offs || (nnz > 0 && !cols)) return fail(GSW_EINVAL, "null CSR array");
  if (offs[0] != 0) return fail(GSW_EINVAL, "offs[0]=%lld, expected 0", (long long)offs[0]);
  for (int64_t v = 0; v < n; ++v)
    if (offs[v + 1] < offs[v])
      return fail(GSW_EINVAL, "offs decreases at row %lld", (long long)v);
  if (offs[n] != nnz)
    return fail(GSW_EINVAL, "offs[n]=%lld differs from nnz=%lld", (long long)offs[n], (long long)nnz);
  for (int64_t e = 0; e < nnz; ++e)
    if (cols[e] < 0 || cols[e] >= n)
      return fail(GSW_EINVAL, "cols[%lld]=%d out of [0, %lld)", (long long)e, cols[e], (long long)n);
  return GSW_OK;
}

bool rows_sorted(int64_t n, const int64_t* offs, const int32_t* cols) {
  for (int64_t v = 0; v < n; ++v)
    for (int64_t e = offs[v] + 1; e < offs[v + 1]; ++e)
      if (cols[e - 1] > cols[e]) return false;
  return true;
}

// Every arc (u, v) has its reverse (v, u).
bool check_symmetric(int64_t n, const int64_t* offs, const int32_t* cols) {
  if (rows_sorted(n, offs, cols)) {
    for (int64_t u = 0; u < n; ++u)
      for (int64_t e = offs[u]; e < offs[u + 1]; ++e) {
        const int32_t v = cols[e];
        if (!std::binary_search(cols + offs[v], cols + offs[v + 1], (int32_t)u)) return false;
      }
    return true;
  }
  std::vector<uint64_t> fw, bw;
  fw.reserve((size_t)offs[n]);
  bw.reserve((size_t)offs[n]);
  for (int64_t u = 0; u < n; ++u)
    for (int64_t e = offs[u]; e < offs[u + 1]; ++e) {
      fw.push_back(((uint64_t)u << 32) | (uint32_t)cols[e]);
      bw.push_back(((uint64_t)(uint32_t)cols[e] << 32) | (uint64_t)u);
    }
  std::sort(fw.begin(), fw.end());
  std::sort(bw.begin(), bw.end());
  fw.erase(std::unique(fw.begin(), fw.end()), fw.end());
  bw.erase(std::unique(bw.begin(), bw.end()), bw.end());
  return fw == bw;
}

hipStream_t library_stream(gsw_graph* g) { return g->stream; }

// Host checks and statistics of a new graph; on a directed graph also the
// transpose (returned for upload).
gsw_status make_graph(int64_t n, int64_t nnz, const int64_t* h_offs, const int32_t* h_cols,
                      uint32_t flags, gsw_graph* g, std::vector<int64_t>& t_offs, std::vector<int32_t>& t_cols) {
  g->n = n;
  g->nnz = nnz;
  if (!(flags & GSW_TRUSTED)) GSW_TRY(validate_csr(n, nnz, h_offs, h_cols));
  if (flags & GSW_ASSUME_SYMMETRIC)
    g->symmetric = 1;
  else
    g->symmetric = check_symmetric(n, h_offs, h_cols) ? 1 : 0;
  degree_stats(n, h_offs, g->deg_stats);
  if (!g->symmetric) {
    transpose_csr(n, h_offs, h_cols, t_offs, t_cols);
    graph_features(n, nnz, h_offs, h_cols, t_offs.data(), t_cols.data(), g->gfeat);
  } else {
    graph_features(n, nnz, h_offs, h_cols, nullptr, nullptr, g->gfeat);
  }
  GSW_HIP(hipGetDevice(&g->device));
  GSW_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
  return GSW_OK;
}

// In-arcs on the device: the graph's own arrays when symmetric, else an
// uploaded copy of the transpose.
gsw_status set_in_arcs(gsw_graph* g, const std::vector<int64_t>& t_offs, const std::vector<int32_t>& t_cols) {
  if (g->symmetric) {
    g->roffs = g->offs;
    g->rcols = g->cols;
    return GSW_OK;
  }
  const size_t ob = t_offs.size() * sizeof(int64_t), cb = (t_cols.empty() ? 1 : t_cols.size()) * sizeof(int32_t);
  int64_t* ro = nullptr;
  int32_t* rc = nullptr;
  if (hipMalloc((void**)&ro, ob) != hipSuccess || hipMalloc((void**)&rc, cb) != hipSuccess) {
    (void)hipGetLastError();
    if (ro) (void)hipFree(ro);
    return fail(GSW_ENOMEM, "hipMalloc for the transpose (%zu + %zu bytes) failed", ob, cb);
  }
  g->roffs = ro;
  g->rcols = rc;
  g->rcsr_bytes = ob + cb;
  GSW_HIP(hipMemcpy(ro, t_offs.data(), ob, hipMemcpyHostToDevice));
  if (!t_cols.empty()) GSW_HIP(hipMemcpy(rc, t_cols.data(), t_cols.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  return GSW_OK;
}

}  // namespace

// Ranking the head pays on a skewed out-degree law (standard deviation above
// the mean: R-MAT, Chung-Lu, power laws), where a few in-neighbours of large
// degree enter the frontier long before the rest.  On a narrow law (a
// Poisson or a mesh) the ranks are near ties, so the ranked head resolves
// about as many rows as the first arcs do, and the rows it misses would
// probe their head arcs a second time.
bool head_ranking_pays(const gsw_graph* g) {
  if (g->n <= 0 || g->nnz <= 0) return false;
  const double mean = (double)g->nnz / (double)g->n;
  return g->deg_stats[5] > mean;
}

hipStream_t pick_stream(gsw_graph* g, void* user_stream) {
  return user_stream ? (hipStream_t)user_stream : library_stream(g);
}

namespace {
struct WsItem {
  void** p;
  size_t bytes;
};
constexpr int kWsItems = 16;

// The single-source workspace's device buffers (pointers into w) and sizes.
void workspace_items(int64_t n, Workspace& w, WsItem (&items)[kWsItems]) {
  const int64_t nw = (n + 63) / 64;
  const size_t bmb = (size_t)nw * sizeof(unsigned long long);
  const int64_t nb = (n + 1023) / 1024 + 1;
  const WsItem it[kWsItems] = {
      {(void**)&w.vis, bmb},
      {(void**)&w.bm[0], bmb},
      {(void**)&w.bm[1], bmb},
      {(void**)&w.bm[2], bmb},
      {(void**)&w.ctl, 2 * sizeof(BfsCtl)},
      {(void**)&w.done, (size_t)kDoneGroups * kCtrStride * sizeof(unsigned long long)},
      {(void**)&w.q[0], (size_t)kQueueBins * n * sizeof(int32_t)},
      {(void**)&w.q[1], (size_t)kQueueBins * n * sizeof(int32_t)},
      {(void**)&w.ctr, 4 * kCtrSlot * sizeof(uint32_t)},
      {(void**)&w.actr, 4 * kArcSlot * sizeof(unsigned long long)},
      {(void**)&w.scan, (size_t)n * sizeof(int64_t)},
      {(void**)&w.ebeg, (size_t)n * sizeof(int64_t)},
      {(void**)&w.bsum, (size_t)nb * sizeof(int64_t)},
      {(void**)&w.lvl_tmp, (size_t)n * sizeof(int32_t)},
      {(void**)&w.par_tmp, (size_t)n * sizeof(int32_t)},
      {(void**)&w.head, (size_t)n * kHeadArcs * sizeof(int32_t)},
  };
  for (int i = 0; i < kWsItems; ++i) items[i] = it[i];
}
}  // namespace

size_t workspace_bytes(const gsw_graph* g) {
  Workspace tmp;
  WsItem items[kWsItems];
  workspace_items(g->n, tmp, items);
  size_t b = (size_t)((g->n + 63) / 64) * sizeof(unsigned long long);  // the no-in-arc bitmap
  for (const WsItem& it : items) b += it.bytes;
  return b;
}

gsw_status ensure_workspace(gsw_graph* g) {
  Workspace& w = g->ws;
  if (w.ready) return GSW_OK;
  // every step below is skipped once done, so a call after a failed one
  // resumes where that one stopped instead of using half-built buffers
  const int64_t n = g->n;
  w.n = n;
  w.nw = (n + 63) / 64;
  WsItem items[kWsItems];
  workspace_items(n, w, items);
  for (auto& it : items) {
    if (*it.p) continue;
    hipError_t e = hipMalloc(it.p, it.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for the BFS workspace failed: %s", it.bytes,
                  hipGetErrorString(e));
    }
    w.bytes += it.bytes;
  }
  if (!w.h_ctr) GSW_HIP(hipHostMalloc((void**)&w.h_ctr, kCtrSlot * sizeof(uint32_t), hipHostMallocDefault));
  if (!w.h_ctl) GSW_HIP(hipHostMalloc((void**)&w.h_ctl, sizeof(BfsCtl), hipHostMallocDefault));
  if (!w.ring) {
    GSW_HIP(hipHostMalloc((void**)&w.ring, (size_t)kBfsRing * kBfsRec * sizeof(unsigned long long),
                          hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(w.ring, 0, (size_t)kBfsRing * kBfsRec * sizeof(unsigned long long));
  }
  if (!w.d_ring) GSW_HIP(hipHostGetDevicePointer((void**)&w.d_ring, w.ring, 0));
  if (!w.head_built) {
    const bool ranked = head_ranking_pays(g);
    if (n > 0) {
      GSW_TRY(launch_build_head(g, w.head, ranked, g->stream));
      GSW_HIP(hipStreamSynchronize(g->stream));
    }
    w.head_built = true;
    w.head_ranked = ranked;
  }
  if (!g->iso) {
    const size_t ib = (size_t)w.nw * sizeof(unsigned long long);
    hipError_t e = hipMalloc((void**)&g->iso, ib);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      g->iso = nullptr;
      return fail(GSW_ENOMEM, "hipMalloc(%zu) for the isolated-vertex bitmap failed", ib);
    }
    w.bytes += ib;
    gsw_status st = launch_isolated(g, g->iso, g->stream);
    if (st == GSW_OK && hipStreamSynchronize(g->stream) != hipSuccess)
      st = fail(GSW_EHIP, "building the isolated-vertex bitmap failed");
    if (st != GSW_OK) {  // rebuilt by the next call
      (void)hipFree(g->iso);
      g->iso = nullptr;
      w.bytes -= ib;
      return st;
    }
  }
  if (!w.ev[0]) GSW_HIP(hipEventCreate(&w.ev[0]));
  if (!w.ev[1]) GSW_HIP(hipEventCreate(&w.ev[1]));
  {
    int khz = 0;
    GSW_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g->device));
    w.tick_ms = khz > 0 ? 1.0 / (double)khz : 0.0;
  }
  w.ready = true;
  return GSW_OK;
}

namespace {
// The row of every arc of (offs, n) into *origin, allocated here; on any
// failure *origin stays null, so a later call builds it again.
gsw_status build_origin(gsw_graph* g, const int64_t* offs, int32_t** origin) {
  const size_t bytes = (size_t)g->nnz * sizeof(int32_t);
  int32_t* o = nullptr;
  if (hipMalloc((void**)&o, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(GSW_ENOMEM, "hipMalloc(%zu) for an origin array failed", bytes);
  }
  gsw_status st = launch_build_origin(offs, g->n, o, g->stream);
  if (st == GSW_OK && hipStreamSynchronize(g->stream) != hipSuccess)
    st = fail(GSW_EHIP, "building an origin array failed");
  if (st != GSW_OK) {
    (void)hipFree(o);
    return st;
  }
  *origin = o;
  g->origin_bytes += bytes;
  return GSW_OK;
}
}  // namespace

gsw_status ensure_origin(gsw_graph* g) {
  if (g->origin || g->nnz == 0) return GSW_OK;
  return build_origin(g, g->offs, &g->origin);
}

gsw_status ensure_rorigin(gsw_graph* g) {
  if (g->rorigin || g->nnz == 0) return GSW_OK;
  if (g->symmetric) {  // the in-arcs are the arcs
    GSW_TRY(ensure_origin(g));
    g->rorigin = g->origin;
    return GSW_OK;
  }
  return build_origin(g, g->roffs, &g->rorigin);
}

}  // namespace gsw

using namespace gsw;

namespace {

void free_graph(gsw_graph* g) {
  if (!g) return;
  Workspace& w = g->ws;
  void* dev[] = {w.vis, w.bm[0], w.bm[1], w.bm[2], w.ctl, w.done, w.q[0], w.q[1], w.ctr, w.actr, w.scan,
                 w.ebeg, w.bsum, w.lvl_tmp, w.par_tmp, w.head, w.d_tree, w.d_thr, w.d_sched, g->origin};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (g->rorigin && g->rorigin != g->origin) (void)hipFree(g->rorigin);
  if (g->roffs && g->roffs != g->offs) (void)hipFree((void*)g->roffs);
  if (g->rcols && g->rcols != g->cols) (void)hipFree((void*)g->rcols);
  if (w.h_ctr) (void)hipHostFree(w.h_ctr);
  if (w.h_ctl) (void)hipHostFree(w.h_ctl);
  if (w.ring) (void)hipHostFree(w.ring);
  if (g->iso) (void)hipFree(g->iso);
  for (hipEvent_t ev : w.ev)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : w.lev)
    if (ev) (void)hipEventDestroy(ev);
  if (g->owns_csr) {
    if (g->offs) (void)hipFree((void*)g->offs);
    if (g->cols) (void)hipFree((void*)g->cols);
  }
  ms_release(g);
  cc_release(g);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

// Kernel names: the base kernel, then the count variant unless WORKGROUP.
const char* const kNames[GSW_N_KERNELS] = {
    "push_vertex", "push_wave4", "push_wave8", "push_wave16", "push_wave32", "push_wave64", "push_edge",
    "pull_bitmap", "vertex_scan", "edge_scan", "rev_edge_scan",
    "push_vertex.wave", "push_wave4.wave", "push_wave8.wave", "push_wave16.wave", "push_wave32.wave",
    "push_wave64.wave", "push_edge.wave", "pull_bitmap.wave", "vertex_scan.wave", "edge_scan.wave",
    "rev_edge_scan.wave",
    "push_vertex.thread", "push_wave4.thread", "push_wave8.thread", "push_wave16.thread", "push_wave32.thread",
    "push_wave64.thread", "push_edge.thread", "pull_bitmap.thread", "vertex_scan.thread", "edge_scan.thread",
    "rev_edge_scan.thread"};

const char* const kFeatureNames[GSW_N_FEATURES] = {
    "n_vertices",     "n_edges",        "out_deg_min", "out_deg_q1",      "out_deg_median", "out_deg_q3",
    "out_deg_max",    "out_deg_std",    "in_deg_min",  "in_deg_q1",       "in_deg_median",  "in_deg_q3",
    "in_deg_max",     "in_deg_std",     "abs_deg_min", "abs_deg_q1",      "abs_deg_median", "abs_deg_q3",
    "abs_deg_max",    "abs_deg_std",    "frontier",    "frontier_frac",   "discovered",     "discovered_frac"};

}  // namespace

extern "C" {

const char* gsw_last_error(void) { return g_err; }

const char* gsw_kernel_name(int32_t k) { return (k >= 0 && k < GSW_N_KERNELS) ? kNames[k] : "?"; }

const char* gsw_feature_name(int32_t i) { return (i >= 0 && i < GSW_N_FEATURES) ? kFeatureNames[i] : "?"; }

int32_t gsw_abi_version(void) { return GSW_ABI_VERSION; }

#ifndef GSW_SOURCE_DIGEST
#define GSW_SOURCE_DIGEST "unstamped"
#endif
const char* gsw_source_digest(void) { return GSW_SOURCE_DIGEST; }

void gsw_bfs_opts_default(gsw_bfs_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->policy = GSW_POLICY_TREE;
  o->fixed_kernel = GSW_K_PUSH_VERTEX;
}

gsw_status gsw_graph_validate(int64_t n, int64_t nnz, const int64_t* offs, const int32_t* cols,
                              int32_t* is_symmetric) {
  clear_error();
  GSW_TRY(validate_csr(n, nnz, offs, cols));
  if (is_symmetric) *is_symmetric = check_symmetric(n, offs, cols) ? 1 : 0;
  return GSW_OK;
}

gsw_status gsw_graph_create_host(int64_t n, int64_t nnz, const int64_t* offs, const int32_t* cols,
                                 uint32_t flags, gsw_graph** out) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  *out = nullptr;
  if (!offs || (nnz > 0 && !cols)) return fail(GSW_EINVAL, "null CSR array");
  gsw_graph* g = new (std::nothrow) gsw_graph();
  if (!g) return fail(GSW_ENOMEM, "host allocation failed");
  std::vector<int64_t> t_offs;
  std::vector<int32_t> t_cols;
  gsw_status st = make_graph(n, nnz, offs, cols, flags, g, t_offs, t_cols);
  if (st != GSW_OK) {
    free_graph(g);
    return st;
  }
  g->owns_csr = true;
  const size_t ob = (size_t)(n + 1) * sizeof(int64_t), cb = (size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t);
  hipError_t e1 = hipMalloc((void**)&g->offs, ob);
  hipError_t e2 = e1 == hipSuccess ? hipMalloc((void**)&g->cols, cb) : e1;
  if (e1 != hipSuccess || e2 != hipSuccess) {
    (void)hipGetLastError();
    free_graph(g);
    return fail(GSW_ENOMEM, "hipMalloc for the CSR (%zu + %zu bytes) failed", ob, cb);
  }
  g->csr_bytes = ob + cb;
  st = GSW_OK;
  if (hipMemcpy((void*)g->offs, offs, ob, hipMemcpyHostToDevice) != hipSuccess ||
      (nnz > 0 && hipMemcpy((void*)g->cols, cols, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess))
    st = fail(GSW_EHIP, "copying the CSR to the device failed");
  if (st == GSW_OK) st = set_in_arcs(g, t_offs, t_cols);
  // the uploads ran on the null stream, which the library's non-blocking
  // streams do not wait for: they must have landed before any search reads them
  if (st == GSW_OK && hipStreamSynchronize(nullptr) != hipSuccess) st = fail(GSW_EHIP, "CSR upload");
  if (st == GSW_OK && (flags & GSW_WITH_ORIGIN)) st = ensure_origin(g);
  if (st == GSW_OK && (flags & GSW_WITH_ORIGIN)) st = ensure_rorigin(g);
  if (st != GSW_OK) {
    free_graph(g);
    return st;
  }
  *out = g;
  return GSW_OK;
}

gsw_status gsw_graph_create_device(int64_t n, int64_t nnz, const int64_t* d_offs, const int32_t* d_cols,
                                   uint32_t flags, void* stream, gsw_graph** out) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  *out = nullptr;
  if (!d_offs || (nnz > 0 && !d_cols)) return fail(GSW_EINVAL, "null CSR array");
  if (n < 1 || n >= ((int64_t)1 << 31) || nnz < 0)
    return fail(GSW_EINVAL, "n=%lld or nnz=%lld out of range", (long long)n, (long long)nnz);
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> h_offs((size_t)n + 1);
  std::vector<int32_t> h_cols;
  GSW_HIP(hipMemcpyAsync(h_offs.data(), d_offs, h_offs.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  const bool need_cols = !(flags & GSW_TRUSTED) || !(flags & GSW_ASSUME_SYMMETRIC);
  if (need_cols && nnz > 0) {
    h_cols.resize((size_t)nnz);
    GSW_HIP(hipMemcpyAsync(h_cols.data(), d_cols, (size_t)nnz * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  GSW_HIP(hipStreamSynchronize(s));
  if ((flags & GSW_TRUSTED) && (h_offs[0] != 0 || h_offs[(size_t)n] != nnz))
    return fail(GSW_EINVAL, "offs[0] or offs[n] inconsistent with nnz");
  gsw_graph* g = new (std::nothrow) gsw_graph();
  if (!g) return fail(GSW_ENOMEM, "host allocation failed");
  std::vector<int64_t> t_offs;
  std::vector<int32_t> t_cols;
  gsw_status st = make_graph(n, nnz, h_offs.data(), need_cols ? h_cols.data() : nullptr, flags, g, t_offs, t_cols);
  if (st != GSW_OK) {
    free_graph(g);
    return st;
  }
  g->offs = d_offs;
  g->cols = d_cols;
  g->owns_csr = false;
  st = set_in_arcs(g, t_offs, t_cols);
  if (st == GSW_OK && hipStreamSynchronize(nullptr) != hipSuccess) st = fail(GSW_EHIP, "transpose upload");
  if (st == GSW_OK && (flags & GSW_WITH_ORIGIN)) st = ensure_origin(g);
  if (st == GSW_OK && (flags & GSW_WITH_ORIGIN)) st = ensure_rorigin(g);
  if (st != GSW_OK) {
    free_graph(g);
    return st;
  }
  *out = g;
  return GSW_OK;
}

void gsw_graph_destroy(gsw_graph* g) {
  if (g) (void)hipSetDevice(g->device);
  free_graph(g);
}

gsw_status gsw_graph_info(const gsw_graph* g, int64_t* n, int64_t* nnz, double deg_stats[6],
                          size_t* dev_bytes) {
  clear_error();
  if (!g) return fail(GSW_EINVAL, "graph is null");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (deg_stats) std::memcpy(deg_stats, g->deg_stats, sizeof g->deg_stats);
  if (dev_bytes) *dev_bytes = g->csr_bytes + g->rcsr_bytes + g->origin_bytes + g->ws.bytes + cc_workspace_bytes(g);
  return GSW_OK;
}

int32_t gsw_graph_symmetric(const gsw_graph* g) { return g && g->symmetric ? 1 : 0; }

size_t gsw_graph_workspace_bytes(const gsw_graph* g) { return g ? workspace_bytes(g) : 0; }

gsw_status gsw_graph_features_host(int64_t n, int64_t nnz, const int64_t* offs, const int32_t* cols,
                                   double out[GSW_N_GRAPH_FEATURES]) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  GSW_TRY(validate_csr(n, nnz, offs, cols));
  if (check_symmetric(n, offs, cols)) {
    graph_features(n, nnz, offs, cols, nullptr, nullptr, out);
  } else {
    std::vector<int64_t> t_offs;
    std::vector<int32_t> t_cols;
    transpose_csr(n, offs, cols, t_offs, t_cols);
    graph_features(n, nnz, offs, cols, t_offs.data(), t_cols.data(), out);
  }
  return GSW_OK;
}

gsw_status gsw_degree_stats(int64_t n, const int64_t* offs, double out[6]) {
  clear_error();
  if (n < 1 || !offs || !out) return fail(GSW_EINVAL, "bad arguments");
  degree_stats(n, offs, out);
  return GSW_OK;
}

gsw_status gsw_level_features(const gsw_graph* g, int64_t n_frontier, int64_t discovered,
                              double out[GSW_N_FEATURES]) {
  clear_error();
  if (!g || !out) return fail(GSW_EINVAL, "null argument");
  const double n = (double)g->n;
  for (int i = 0; i < GSW_N_GRAPH_FEATURES; ++i) out[i] = g->gfeat[i];
  out[20] = (double)n_frontier;
  out[21] = (double)n_frontier / n;
  out[22] = (double)discovered;
  out[23] = (double)discovered / n;
  return GSW_OK;
}

gsw_status gsw_tree_create(int32_t n_nodes, int32_t n_classes, const int32_t* feature,
                           const double* threshold, const int32_t* left, const int32_t* right,
                           const double* value, const int32_t* class_kernel, gsw_tree** out) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  *out = nullptr;
  if (n_nodes < 1 || n_classes < 1 || !feature || !threshold || !left || !right || !value || !class_kernel)
    return fail(GSW_EINVAL, "bad tree arrays");
  for (int32_t c = 0; c < n_classes; ++c)
    if (class_kernel[c] < 0 || class_kernel[c] >= GSW_N_KERNELS)
      return fail(GSW_EINVAL, "class %d maps to unknown kernel %d", c, class_kernel[c]);
  for (int32_t i = 0; i < n_nodes; ++i) {
    const bool leaf = left[i] == -1;
    if (leaf) {
      if (right[i] != -1) return fail(GSW_EINVAL, "node %d: one child missing", i);
      continue;
    }
    // children must point forward so every walk ends
    if (left[i] <= i || left[i] >= n_nodes || right[i] <= i || right[i] >= n_nodes)
      return fail(GSW_EINVAL, "node %d: bad children %d/%d", i, left[i], right[i]);
    if (feature[i] < 0 || feature[i] >= GSW_N_FEATURES)
      return fail(GSW_EINVAL, "node %d: feature %d out of range", i, feature[i]);
  }
  gsw_tree* t = new (std::nothrow) gsw_tree();
  if (!t) return fail(GSW_ENOMEM, "host allocation failed");
  t->n_nodes = n_nodes;
  t->n_classes = n_classes;
  t->feature.assign(feature, feature + n_nodes);
  t->threshold.assign(threshold, threshold + n_nodes);
  t->left.assign(left, left + n_nodes);
  t->right.assign(right, right + n_nodes);
  t->value.assign(value, value + (size_t)n_nodes * n_classes);
  t->class_kernel.assign(class_kernel, class_kernel + n_classes);
  // each leaf's decision, with gsw_tree_predict's tie rule (-1: undecided)
  t->leaf_kernel.assign((size_t)n_nodes, -1);
  for (int32_t i = 0; i < n_nodes; ++i) {
    if (left[i] != -1) continue;
    const double* v = value + (size_t)i * n_classes;
    int32_t best = 0, ties = 1;
    for (int32_t c = 1; c < n_classes; ++c) {
      if (v[c] > v[best]) {
        best = c;
        ties = 1;
      } else if (v[c] == v[best]) {
        ++ties;
      }
    }
    t->leaf_kernel[(size_t)i] = ties == 1 ? class_kernel[best] : -1;
  }
  static std::atomic<uint64_t> next_id{1};
  t->id = next_id++;
  *out = t;
  return GSW_OK;
}

void gsw_tree_destroy(gsw_tree* t) { delete t; }

gsw_status gsw_tree_predict(const gsw_tree* t, const double x[GSW_N_FEATURES], int32_t prev_kernel,
                            int32_t level, int32_t* kernel, int32_t* unknown) {
  if (!t || !x || !kernel) return fail(GSW_EINVAL, "null argument");
  int32_t node = 0;
  while (t->left[(size_t)node] != -1) {
    const double xv = (double)(float)x[t->feature[(size_t)node]];
    node = xv <= t->threshold[(size_t)node] ? t->left[(size_t)node] : t->right[(size_t)node];
  }
  const double* v = t->value.data() + (size_t)node * t->n_classes;
  int32_t best = 0, ties = 1;
  for (int32_t c = 1; c < t->n_classes; ++c) {
    if (v[c] > v[best]) {
      best = c;
      ties = 1;
    } else if (v[c] == v[best]) {
      ++ties;
    }
  }
  if (ties == 1) {
    *kernel = t->class_kernel[(size_t)best];
    if (unknown) *unknown = 0;
  } else {
    *kernel = level > 0 ? prev_kernel : GSW_DEFAULT_KERNEL;
    if (unknown) *unknown = 1;
  }
  return GSW_OK;
}

}  // extern "C"

// ------------------------------------------------------------ tree JSON
namespace {

// A small JSON reader for the tree export: values are null, booleans,
// numbers (as double), strings, arrays and objects.  Nesting is limited so a
// hostile file cannot exhaust the stack.
struct JVal {
  enum Kind { kNull, kBool, kNum, kStr, kArr, kObj } kind = kNull;
  double num = 0.0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* key) const {
    for (const auto& kv : obj)
      if (kv.first == key) return &kv.second;
    return nullptr;
  }
};

class JReader {
 public:
  JReader(const char* p, const char* e) : p_(p), e_(e) {}
  bool parse(JVal* out) {
    if (!value(out, 0)) return false;
    ws();
    return p_ == e_;
  }
  size_t offset(const char* base) const { return (size_t)(p_ - base); }

 private:
  const char* p_;
  const char* e_;
  static constexpr int kMaxDepth = 32;

  void ws() {
    while (p_ < e_ && (*p_ == ' ' || *p_ == '\t' || *p_ == '\n' || *p_ == '\r')) ++p_;
  }
  bool lit(const char* w) {
    const size_t k = std::strlen(w);
    if ((size_t)(e_ - p_) < k || std::strncmp(p_, w, k) != 0) return false;
    p_ += k;
    return true;
  }
  bool string(std::string* s) {
    if (p_ >= e_ || *p_ != '"') return false;
    ++p_;
    while (p_ < e_ && *p_ != '"') {
      char c = *p_++;
      if (c == '\\') {
        if (p_ >= e_) return false;
        const char x = *p_++;
        switch (x) {
          case '"': case '\\': case '/': c = x; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'n': c = '\n'; break;
          case 'r': c = '\r'; break;
          case 't': c = '\t'; break;
          case 'u': {  // keep the code unit as '?' unless it is ASCII
            if (e_ - p_ < 4) return false;
            unsigned cp = 0;
            for (int i = 0; i < 4; ++i) {
              const char h = *p_++;
              cp <<= 4;
              if (h >= '0' && h <= '9') cp |= (unsigned)(h - '0');
              else if (h >= 'a' && h <= 'f') cp |= (unsigned)(h - 'a' + 10);
              else if (h >= 'A' && h <= 'F') cp |= (unsigned)(h - 'A' + 10);
              else return false;
            }
            c = cp < 128 ? (char)cp : '?';
            break;
          }
          default: return false;
        }
      } else if ((unsigned char)c < 0x20) {
        return false;
      }
      s->push_back(c);
    }
    if (p_ >= e_) return false;
    ++p_;
    return true;
  }
  bool number(double* x) {
    const char* q = p_;
    if (q < e_ && (*q == '-' || *q == '+')) ++q;
    while (q < e_ && ((*q >= '0' && *q <= '9') || *q == '.' || *q == 'e' || *q == 'E' || *q == '-' || *q == '+')) ++q;
    if (q == p_ || q - p_ > 64) return false;
    char buf[72];
    std::memcpy(buf, p_, (size_t)(q - p_));
    buf[q - p_] = '\0';
    char* end = nullptr;
    *x = std::strtod(buf, &end);
    if (end != buf + (q - p_)) return false;
    p_ = q;
    return true;
  }
  bool value(JVal* v, int depth) {
    if (depth > kMaxDepth) return false;
    ws();
    if (p_ >= e_) return false;
    const char c = *p_;
    if (c == '{') {
      ++p_;
      v->kind = JVal::kObj;
      ws();
      if (p_ < e_ && *p_ == '}') {
        ++p_;
        return true;
      }
      for (;;) {
        ws();
        std::pair<std::string, JVal> kv;
        if (!string(&kv.first)) return false;
        ws();
        if (p_ >= e_ || *p_ != ':') return false;
        ++p_;
        if (!value(&kv.second, depth + 1)) return false;
        v->obj.push_back(std::move(kv));
        ws();
        if (p_ < e_ && *p_ == ',') {
          ++p_;
          continue;
        }
        if (p_ < e_ && *p_ == '}') {
          ++p_;
          return true;
        }
        return false;
      }
    }
    if (c == '[') {
      ++p_;
      v->kind = JVal::kArr;
      ws();
      if (p_ < e_ && *p_ == ']') {
        ++p_;
        return true;
      }
      for (;;) {
        JVal x;
        if (!value(&x, depth + 1)) return false;
        v->arr.push_back(std::move(x));
        ws();
        if (p_ < e_ && *p_ == ',') {
          ++p_;
          continue;
        }
        if (p_ < e_ && *p_ == ']') {
          ++p_;
          return true;
        }
        return false;
      }
    }
    if (c == '"') {
      v->kind = JVal::kStr;
      return string(&v->str);
    }
    if (lit("true")) {
      v->kind = JVal::kBool;
      v->num = 1.0;
      return true;
    }
    if (lit("false")) {
      v->kind = JVal::kBool;
      return true;
    }
    if (lit("null")) {
      v->kind = JVal::kNull;
      return true;
    }
    v->kind = JVal::kNum;
    return number(&v->num);
  }
};

// Numbers of a JSON array into out (integers when `integral`).
gsw_status json_numbers(const JVal* a, const char* key, bool integral, std::vector<double>* out) {
  if (!a || a->kind != JVal::kArr) return fail(GSW_EINVAL, "tree JSON: \"%s\" is missing or not an array", key);
  out->clear();
  for (const JVal& x : a->arr) {
    if (x.kind != JVal::kNum) return fail(GSW_EINVAL, "tree JSON: \"%s\" holds a non-number", key);
    if (integral && (x.num != std::floor(x.num) || std::fabs(x.num) > 2147483647.0))
      return fail(GSW_EINVAL, "tree JSON: \"%s\" holds a non-integer", key);
    out->push_back(x.num);
  }
  return GSW_OK;
}

}  // namespace

extern "C" gsw_status gsw_tree_load(const char* json_path, gsw_tree** out) {
  clear_error();
  if (!out) return fail(GSW_EINVAL, "out is null");
  *out = nullptr;
  if (!json_path) return fail(GSW_EINVAL, "path is null");
  FILE* f = std::fopen(json_path, "rb");
  if (!f) return fail(GSW_EINVAL, "cannot open %s", json_path);
  std::string text;
  char buf[1 << 16];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) {
    text.append(buf, k);
    if (text.size() > ((size_t)1 << 28)) {
      std::fclose(f);
      return fail(GSW_EINVAL, "%s is larger than 256 MiB", json_path);
    }
  }
  std::fclose(f);
  JVal root;
  JReader rd(text.data(), text.data() + text.size());
  if (!rd.parse(&root) || root.kind != JVal::kObj)
    return fail(GSW_EINVAL, "%s: not a JSON object (stopped near byte %zu)", json_path, rd.offset(text.data()));
  if (const JVal* fn = root.get("feature_names")) {
    if (fn->kind != JVal::kArr || fn->arr.size() != (size_t)GSW_N_FEATURES)
      return fail(GSW_EINVAL, "%s: feature_names must list the library's %d features", json_path, GSW_N_FEATURES);
    for (int i = 0; i < GSW_N_FEATURES; ++i)
      if (fn->arr[(size_t)i].kind != JVal::kStr || fn->arr[(size_t)i].str != gsw_feature_name(i))
        return fail(GSW_EINVAL, "%s: feature %d is \"%s\", the library's is \"%s\"", json_path, i,
                    fn->arr[(size_t)i].kind == JVal::kStr ? fn->arr[(size_t)i].str.c_str() : "?", gsw_feature_name(i));
  }
  std::vector<double> feat, thr, left, right, ck;
  GSW_TRY(json_numbers(root.get("feature"), "feature", true, &feat));
  GSW_TRY(json_numbers(root.get("threshold"), "threshold", false, &thr));
  GSW_TRY(json_numbers(root.get("left"), "left", true, &left));
  GSW_TRY(json_numbers(root.get("right"), "right", true, &right));
  GSW_TRY(json_numbers(root.get("class_kernel"), "class_kernel", true, &ck));
  const size_t nn = feat.size();
  if (nn == 0 || thr.size() != nn || left.size() != nn || right.size() != nn || ck.empty())
    return fail(GSW_EINVAL, "%s: node arrays differ in length or are empty", json_path);
  const JVal* val = root.get("value");
  if (!val || val->kind != JVal::kArr || val->arr.size() != nn)
    return fail(GSW_EINVAL, "%s: \"value\" must hold one row per node", json_path);
  const size_t nc = ck.size();
  std::vector<double> value;
  value.reserve(nn * nc);
  for (const JVal& row : val->arr) {
    std::vector<double> r;
    GSW_TRY(json_numbers(&row, "value", false, &r));
    if (r.size() != nc) return fail(GSW_EINVAL, "%s: a value row has %zu classes, expected %zu", json_path, r.size(), nc);
    value.insert(value.end(), r.begin(), r.end());
  }
  std::vector<int32_t> fi(nn), li(nn), ri(nn), ci(nc);
  for (size_t i = 0; i < nn; ++i) {
    li[i] = (int32_t)left[i];
    ri[i] = (int32_t)right[i];
    fi[i] = li[i] == -1 ? 0 : (int32_t)feat[i];  // leaves carry a placeholder feature
  }
  for (size_t c = 0; c < nc; ++c) ci[c] = (int32_t)ck[c];
  return gsw_tree_create((int32_t)nn, (int32_t)nc, fi.data(), thr.data(), li.data(), ri.data(), value.data(),
                         ci.data(), out);
}
