// Host side of libgsw: errors, graph validation and residency, degree
// statistics, the per-level feature vector and the decision tree.
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

void degree_stats(int64_t n, const int64_t* offs, double out[6]) {
  std::vector<int64_t> deg((size_t)n);
  long double sum = 0.0L;
  for (int64_t v = 0; v < n; ++v) {
    deg[(size_t)v] = offs[v + 1] - offs[v];
    sum += (long double)deg[(size_t)v];
  }
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

gsw_status make_graph(int64_t n, int64_t nnz, const int64_t* h_offs, const int32_t* h_cols,
                      uint32_t flags, gsw_graph* g) {
  g->n = n;
  g->nnz = nnz;
  if (!(flags & GSW_TRUSTED)) GSW_TRY(validate_csr(n, nnz, h_offs, h_cols));
  if (flags & GSW_ASSUME_SYMMETRIC)
    g->symmetric = 1;
  else
    g->symmetric = check_symmetric(n, h_offs, h_cols) ? 1 : 0;
  degree_stats(n, h_offs, g->deg_stats);
  GSW_HIP(hipGetDevice(&g->device));
  GSW_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
  return GSW_OK;
}

}  // namespace

hipStream_t pick_stream(gsw_graph* g, void* user_stream) {
  return user_stream ? (hipStream_t)user_stream : library_stream(g);
}

gsw_status ensure_workspace(gsw_graph* g) {
  Workspace& w = g->ws;
  if (w.ready) return GSW_OK;
  // every step below is skipped once done, so a call after a failed one
  // resumes where that one stopped instead of using half-built buffers
  const int64_t n = g->n;
  w.n = n;
  w.nw = (n + 63) / 64;
  const size_t bmb = (size_t)w.nw * sizeof(unsigned long long);
  const int64_t nb = (n + 1023) / 1024 + 1;
  struct Item {
    void** p;
    size_t bytes;
  } items[] = {
      {(void**)&w.vis, bmb},
      {(void**)&w.bm[0], bmb},
      {(void**)&w.bm[1], bmb},
      {(void**)&w.bm[2], bmb},
      {(void**)&w.ctl, 2 * sizeof(BfsCtl)},
      {(void**)&w.done, (size_t)kDoneGroups * kCtrStride * sizeof(unsigned long long)},
      {(void**)&w.q[0], (size_t)kQueueBins * n * sizeof(int32_t)},
      {(void**)&w.q[1], (size_t)kQueueBins * n * sizeof(int32_t)},
      {(void**)&w.ctr, 4 * kCtrSlot * sizeof(uint32_t)},
      {(void**)&w.scan, (size_t)n * sizeof(int64_t)},
      {(void**)&w.ebeg, (size_t)n * sizeof(int64_t)},
      {(void**)&w.bsum, (size_t)nb * sizeof(int64_t)},
      {(void**)&w.lvl_tmp, (size_t)n * sizeof(int32_t)},
      {(void**)&w.par_tmp, (size_t)n * sizeof(int32_t)},
      {(void**)&w.head, (size_t)n * kHeadArcs * sizeof(int32_t)},
  };
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
    if (n > 0) {
      GSW_TRY(launch_build_head(g, w.head, g->stream));
      GSW_HIP(hipStreamSynchronize(g->stream));
    }
    w.head_built = true;
  }
  if (g->symmetric && !g->iso) {
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

gsw_status ensure_origin(gsw_graph* g) {
  if (g->origin || g->nnz == 0) return GSW_OK;
  const size_t bytes = (size_t)g->nnz * sizeof(int32_t);
  hipError_t e = hipMalloc((void**)&g->origin, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    g->origin = nullptr;
    return fail(GSW_ENOMEM, "hipMalloc(%zu) for the origin array failed", bytes);
  }
  g->origin_bytes = bytes;
  GSW_TRY(launch_build_origin(g, g->origin, g->stream));
  GSW_HIP(hipStreamSynchronize(g->stream));
  return GSW_OK;
}

}  // namespace gsw

using namespace gsw;

namespace {

void free_graph(gsw_graph* g) {
  if (!g) return;
  Workspace& w = g->ws;
  void* dev[] = {w.vis, w.bm[0], w.bm[1], w.bm[2], w.ctl, w.done, w.q[0], w.q[1], w.ctr, w.scan, w.ebeg,
                 w.bsum, w.lvl_tmp, w.par_tmp, w.head, w.d_tree, w.d_thr, w.d_sched, g->origin};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (w.h_ctr) (void)hipHostFree(w.h_ctr);
  if (w.h_ctl) (void)hipHostFree(w.h_ctl);
  if (w.ring) (void)hipHostFree(w.ring);
  if (g->iso) (void)hipFree(g->iso);
  for (hipEvent_t ev : w.ev)
    if (ev) (void)hipEventDestroy(ev);
  if (g->owns_csr) {
    if (g->offs) (void)hipFree((void*)g->offs);
    if (g->cols) (void)hipFree((void*)g->cols);
  }
  ms_release(g);
  if (g->stream) (void)hipStreamDestroy(g->stream);
  delete g;
}

const char* const kNames[GSW_N_KERNELS] = {
    "push_vertex", "push_wave4", "push_wave8", "push_wave16", "push_wave32",
    "push_wave64", "push_edge",  "pull_bitmap", "vertex_scan", "edge_scan"};

}  // namespace

extern "C" {

const char* gsw_last_error(void) { return g_err; }

const char* gsw_kernel_name(int32_t k) { return (k >= 0 && k < GSW_N_KERNELS) ? kNames[k] : "?"; }

int32_t gsw_abi_version(void) { return GSW_ABI_VERSION; }

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
  gsw_status st = make_graph(n, nnz, offs, cols, flags, g);
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
  if (st == GSW_OK && (flags & GSW_WITH_ORIGIN)) st = ensure_origin(g);
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
  gsw_status st = make_graph(n, nnz, h_offs.data(), need_cols ? h_cols.data() : nullptr, flags, g);
  if (st != GSW_OK) {
    free_graph(g);
    return st;
  }
  g->offs = d_offs;
  g->cols = d_cols;
  g->owns_csr = false;
  if (flags & GSW_WITH_ORIGIN) st = ensure_origin(g);
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
  if (dev_bytes) *dev_bytes = g->csr_bytes + g->origin_bytes + g->ws.bytes;
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
  out[0] = n;
  out[1] = (double)g->nnz;
  for (int i = 0; i < 6; ++i) out[2 + i] = g->deg_stats[i];
  out[8] = (double)n_frontier;
  out[9] = (double)n_frontier / n;
  out[10] = (double)discovered;
  out[11] = (double)discovered / n;
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
