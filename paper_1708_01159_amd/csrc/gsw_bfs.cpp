// Level loop of the single-source BFS.  The device picks each next level's
// kernel itself (the last workgroup of a level applies the policy and
// writes the next launch's control slot) and posts a record per level to a
// ring in mapped host memory; the host keeps a few launches of the level
// kernel queued and reads the records in order for the trace and the end of
// the search.  A push_edge level on more than kEdgeFuse entries takes two
// launches, any other level one.  Also
// the per-level profiler that measures every kernel from the same saved
// state (the training data of the decision tree).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "gsw_internal.h"

namespace gsw {
namespace {

// Launches of the level kernel queued beyond those that the levels read so
// far have used, plus one more when the next level is push_edge (two
// launches).  Launches queued past the end of the search do nothing.
constexpr int kAhead = 3;
// Single-workgroup launches queued beyond the latest record's: one runs
// many levels, so one more is enough to follow it without a gap.
constexpr int kSoloAhead = 2;

// Launch size for queued levels: the full grid, or kSmallLaunch workgroups
// while the search is in a quiet phase -- the latest frontier the host knows
// of is at most kSmallFrontier and goes to a queue-driven push kernel (the
// all-vertex kernels want the full grid at any frontier size), neither of
// the last two frontiers grew more than twofold, and at least 1% of the
// vertices are discovered -- such as a
// tail or the slowly moving front of a high-diameter graph, whose levels
// need a few workgroups (dispatching the rest of a full launch costs ~1.5 us
// per level).  A scale-free frontier can grow a thousandfold in one level
// early on, which the conditions exclude.  Any size is correct: a level that
// asks for more workgroups than its launch has strides over its work.
constexpr int32_t kSmallLaunch = 16;
constexpr int64_t kSmallFrontier = 4096;

struct Policy {
  const gsw_bfs_opts* o;
  bool has_origin;
  bool has_rorigin;
};

gsw_status check_kernel(const gsw_graph* g, int k) {
  (void)g;
  if (k < 0 || k >= GSW_N_KERNELS) return fail(GSW_EINVAL, "unknown kernel id %d", k);
  return GSW_OK;
}

}  // namespace

int first_kernel(const gsw_graph* g, const gsw_bfs_opts* o, bool has_origin, bool has_rorigin, int32_t* flags) {
  *flags = 0;
  int k = GSW_DEFAULT_KERNEL;
  switch (o->policy) {
    case GSW_POLICY_FIXED:
      k = o->fixed_kernel;
      break;
    case GSW_POLICY_SCHEDULE:
      k = o->schedule[0];
      break;
    default: {
      double x[GSW_N_FEATURES];
      gsw_level_features(g, 1, 1, x);
      int32_t kk = GSW_DEFAULT_KERNEL, unk = 0;
      gsw_tree_predict(o->tree, x, GSW_DEFAULT_KERNEL, 0, &kk, &unk);
      k = kk;
      if (unk) *flags |= 1;
      break;
    }
  }
  if (kernel_base(k) == GSW_K_EDGE_SCAN && !has_origin) k = GSW_DEFAULT_KERNEL;
  if (kernel_base(k) == GSW_K_REV_EDGE_SCAN && !has_rorigin) k = GSW_DEFAULT_KERNEL;
  return k;
}

// The tree specialised to the graph.  A split on one of the graph's own
// features (constant for the graph) is decided here, with the host's float
// rounding, so the copy holds only the nodes reachable through splits on the
// four level features.  Each of those is a non-decreasing function of an
// integer count c in [0, n] -- the next frontier size (features 20, 21 =
// c, c/n) or the vertices discovered through the next depth (22, 23) -- so
// its test, float(feature) <= threshold, holds exactly for c <= T; T is
// found here by bisection with the host's own arithmetic and the device
// compares counts.  The outcome of every walk is unchanged.  Nodes are
// renumbered in preorder, so children still follow their parent.
int32_t specialise_tree(const gsw_graph* g, const gsw_tree* t, const TreeBuf& buf) {
  double gf[GSW_N_FEATURES];
  GSW_TRY(gsw_level_features(g, 0, 0, gf));
  auto resolve = [&](int32_t i) {
    while (t->left[(size_t)i] != -1 && t->feature[(size_t)i] < GSW_N_GRAPH_FEATURES) {
      const double xv = (double)(float)gf[t->feature[(size_t)i]];
      i = xv <= t->threshold[(size_t)i] ? t->left[(size_t)i] : t->right[(size_t)i];
    }
    return i;
  };
  // largest count c in [-1, n] whose feature value passes node i's test
  auto count_threshold = [&](int32_t i) -> int32_t {
    const int f = t->feature[(size_t)i];
    const double thr = t->threshold[(size_t)i];
    auto holds = [&](int64_t c) {
      double x[GSW_N_FEATURES];
      (void)gsw_level_features(g, c, c, x);
      return (double)(float)x[f] <= thr;
    };
    int64_t lo = -1, hi = g->n;  // holds(lo) (or lo = -1), !holds(hi + 1)
    if (holds(hi)) return (int32_t)hi;
    while (hi - lo > 1) {  // holds(lo) or lo == -1, !holds(hi)
      const int64_t mid = lo + (hi - lo) / 2;
      if (holds(mid)) lo = mid; else hi = mid;
    }
    return (int32_t)lo;
  };
  int32_t* order = buf.order;  // kept nodes (old ids) in preorder
  int32_t* newid = buf.newid;
  int32_t* stack = buf.stack;  // a preorder walk keeps at most depth + 1 <= n_nodes entries
  for (int32_t i = 0; i < t->n_nodes; ++i) newid[i] = -1;
  int32_t m = 0, top = 0;
  stack[top++] = resolve(0);
  while (top > 0) {
    const int32_t i = stack[--top];
    newid[(size_t)i] = m;
    order[m++] = i;
    if (t->left[(size_t)i] != -1) {
      stack[top++] = resolve(t->right[(size_t)i]);
      stack[top++] = resolve(t->left[(size_t)i]);
    }
  }
  for (int32_t k = 0; k < m; ++k) {
    const int32_t i = order[(size_t)k];
    const bool leaf = t->left[(size_t)i] == -1;
    const int32_t l = leaf ? -1 : newid[(size_t)resolve(t->left[(size_t)i])];
    const int32_t r = leaf ? -1 : newid[(size_t)resolve(t->right[(size_t)i])];
    const int32_t count = !leaf && t->feature[(size_t)i] >= 22 ? 1 : 0;  // discovered : frontier
    buf.nodes[(size_t)k] = tree_node_pack(l, r, count, t->leaf_kernel[(size_t)i]);
    buf.thr[(size_t)k] = leaf ? 0 : count_threshold(i);
  }
  return m;
}

namespace {

// Device copy of the specialised tree, uploaded once per (workspace, tree).
gsw_status ensure_tree(gsw_graph* g, const gsw_tree* t, hipStream_t s) {
  Workspace& w = g->ws;
  if (w.tree_id == t->id) return GSW_OK;
  if (t->n_nodes > kMaxTreeNodes) return fail(GSW_EINVAL, "tree of %d nodes: at most %d", t->n_nodes, kMaxTreeNodes);
  const size_t nn = (size_t)t->n_nodes;
  std::vector<int32_t> order(nn), newid(nn), stack(nn + 1), thr(nn);
  std::vector<unsigned long long> nodes(nn);
  const TreeBuf buf{order.data(), newid.data(), stack.data(), nodes.data(), thr.data()};
  const int32_t m = specialise_tree(g, t, buf);
  if (w.tree_cap < m) {
    if (w.d_tree) (void)hipFree(w.d_tree);
    if (w.d_thr) (void)hipFree(w.d_thr);
    w.d_tree = nullptr;
    w.d_thr = nullptr;
    w.tree_cap = 0;
    if (hipMalloc((void**)&w.d_tree, (size_t)m * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&w.d_thr, (size_t)m * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSW_ENOMEM, "hipMalloc for the device copy of the tree failed");
    }
    w.tree_cap = m;
  }
  // on the search's stream (ordered before its launches), waited for before
  // the host buffers go
  GSW_HIP(hipMemcpyAsync(w.d_tree, nodes.data(), (size_t)m * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
  GSW_HIP(hipMemcpyAsync(w.d_thr, thr.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, s));
  GSW_HIP(hipStreamSynchronize(s));
  w.tree_nodes = m;
  w.tree_id = t->id;
  return GSW_OK;
}

// Device copy of a schedule; re-uploaded only when its contents change.
gsw_status ensure_schedule(gsw_graph* g, const int32_t* sched, int32_t len, hipStream_t s) {
  Workspace& w = g->ws;
  std::vector<int32_t>* cached = &w.sched_host;
  if (w.d_sched && (int32_t)cached->size() == len && std::equal(cached->begin(), cached->end(), sched))
    return GSW_OK;
  if (w.sched_cap < len) {
    if (w.d_sched) (void)hipFree(w.d_sched);
    w.d_sched = nullptr;
    w.sched_cap = 0;
    if (hipMalloc((void**)&w.d_sched, (size_t)len * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GSW_ENOMEM, "hipMalloc for the device copy of the schedule failed");
    }
    w.sched_cap = len;
  }
  GSW_HIP(hipMemcpyAsync(w.d_sched, sched, (size_t)len * sizeof(int32_t), hipMemcpyHostToDevice, s));
  GSW_HIP(hipStreamSynchronize(s));
  cached->assign(sched, sched + len);
  return GSW_OK;
}

}  // namespace

BfsPolicy device_policy(const gsw_graph* g, const Workspace& w, const gsw_bfs_opts* o, bool has_origin,
                        bool has_rorigin) {
  BfsPolicy p;
  std::memset(&p, 0, sizeof p);
  p.policy = o->policy;
  p.fixed = o->fixed_kernel;
  p.sched_len = o->policy == GSW_POLICY_SCHEDULE ? o->schedule_len : 0;
  p.symmetric = g->symmetric != 0;
  p.has_origin = has_origin ? 1 : 0;
  p.has_rorigin = has_rorigin ? 1 : 0;
  p.sched = w.d_sched;
  p.t_node = w.d_tree;
  p.t_thr = w.d_thr;
  p.t_nodes = o->policy == GSW_POLICY_TREE && o->tree ? w.tree_nodes : 0;
  return p;
}

BfsBase make_base(const gsw_graph* g, const Workspace& w, int32_t* lv, int32_t* pa, bool timed, bool count_arcs) {
  BfsBase b;
  std::memset(&b, 0, sizeof b);
  b.offs = g->offs;
  b.cols = g->cols;
  b.origin = g->origin;
  b.roffs = g->roffs;
  b.rcols = g->rcols;
  b.rorigin = g->rorigin;
  b.head = w.head;
  b.level = lv;
  b.parent = pa;
  b.vis = w.vis;
  for (int i = 0; i < 3; ++i) b.bm[i] = w.bm[i];
  b.q[0] = w.q[0];
  b.q[1] = w.q[1];
  b.ctr = w.ctr;
  b.actr = w.actr;
  b.done = w.done;
  b.scan = w.scan;
  b.ebeg = w.ebeg;
  b.bsum = w.bsum;
  b.ring = w.d_ring;
  b.ctl = w.ctl;
  b.n = g->n;
  b.nw = w.nw;
  b.nnz = g->nnz;
  b.timed = timed ? 1 : 0;
  b.grid_max = level_kernel_grid(g->n, w.nw);
  b.count_arcs = count_arcs ? 1 : 0;
  const double dm = g->deg_stats[4];
  b.deg_max = dm >= 2147483647.0 ? 2147483647 : (int32_t)dm;
  b.head_ranked = w.head_ranked ? 1 : 0;
  b.solo = 0;
  return b;
}

bool take_record(const volatile unsigned long long* ring, int64_t d, Record* rec) {
  const volatile unsigned long long* r = ring + (size_t)(d % kBfsRing) * kBfsRec;
  const unsigned long long tag = rec_tag(d);
  unsigned long long v[kBfsRecWords];
  for (int i = 0; i < kBfsRecWords; ++i) {
    v[i] = r[i];
    if ((v[i] & ~kRecValueMask) != tag) return false;
    v[i] &= kRecValueMask;
  }
  rec->kernel = (int)v[kRecKernel];
  rec->flags = (int32_t)v[kRecFlags];
  rec->nf = (int64_t)v[kRecNf];
  rec->disc = (int64_t)v[kRecDisc];
  rec->next = (int64_t)v[kRecNext];
  rec->ticks = v[kRecTicks];
  rec->next_kernel = (int)v[kRecNextKernel] - 1;
  rec->ef = (int64_t)v[kRecEf] - 1;
  rec->launch = (int64_t)v[kRecLaunch];
  return true;
}

void trace_row(gsw_level_trace* t, int32_t src_idx, int64_t d, const Record& r, bool timed, double tick_ms) {
  t->source_idx = src_idx;
  t->level = (int32_t)d;
  t->kernel = r.kernel;
  t->flags = r.flags;
  t->n_frontier = r.nf;
  t->discovered = r.disc;
  t->n_next = r.next;
  t->e_frontier = r.ef;
  t->ms = timed ? (float)((double)r.ticks * tick_ms) : -1.0f;
  t->launch = (int32_t)r.launch;
}

int32_t launch_size(int next_kernel, int64_t nn, int64_t nf, int64_t nf_prev, int64_t disc, int64_t d, int64_t n,
                    int32_t cap) {
  const int nb = next_kernel >= 0 ? kernel_base(next_kernel) : -1;
  const bool queue_push = nb != GSW_K_PULL_BITMAP && nb != GSW_K_VERTEX_SCAN && nb != GSW_K_EDGE_SCAN &&
                          nb != GSW_K_REV_EDGE_SCAN;
  const bool quiet = queue_push && nn <= kSmallFrontier && nn <= 2 * nf && d > 0 && nf <= 2 * nf_prev &&
                     (disc + nn) * 100 >= n;
  return quiet && kSmallLaunch < cap ? kSmallLaunch : cap;
}

namespace {

// Waits until level d's record is in the ring.
gsw_status wait_record(const gsw_graph* g, int64_t d, hipStream_t s, Record* rec) {
  bool missing = false;
  const hipError_t e = await_record([&]() -> bool { return take_record(g->ws.ring, d, rec); }, s, &missing);
  if (e != hipSuccess) return fail(GSW_EHIP, "level %lld: %s", (long long)d, hipGetErrorString(e));
  if (missing) return fail(GSW_EHIP, "level %lld finished without posting its record", (long long)d);
  return GSW_OK;
}

gsw_status run_levels(gsw_graph* g, const Policy& pol, const BfsPolicy& dp, int32_t src_idx, int32_t src,
                      int32_t* lv, int32_t* pa, gsw_level_trace* trace, int32_t trace_cap, int32_t* rows,
                      hipStream_t s) {
  Workspace& w = g->ws;
  const gsw_bfs_opts* o = pol.o;
  const bool events = o->time_levels == 2;  // per-launch HIP events
  const bool timed = o->time_levels == 1;   // device wall-clock stamps
  // clear the ring slots the last search wrote (its records carry the tags
  // this search's first levels will use)
  const int64_t used = w.ring_used < 0 || w.ring_used > kBfsRing ? kBfsRing : w.ring_used;
  std::memset(w.ring, 0, (size_t)used * kBfsRec * sizeof(unsigned long long));
  w.ring_used = kBfsRing;  // until this search ends normally
  constexpr int kEv = Workspace::kLaunchEvents;
  if (events)
    for (hipEvent_t& e : w.lev)
      if (!e) GSW_HIP(hipEventCreate(&e));
  // event after launch j in slot (j + 1) % kEv; slot 0 follows the init kernel
  auto ev_after = [&](int64_t jj) -> hipEvent_t& { return w.lev[(size_t)((jj + 1) % kEv)]; };
  int32_t flags0 = 0;
  const int k0 = first_kernel(g, o, pol.has_origin, pol.has_rorigin, &flags0);
  BfsBase b = make_base(g, w, lv, pa, timed, o->count_arcs != 0);
  // single-workgroup multi-level launches: not with per-launch events (their
  // levels would share one launch's time), and with a tree its workgroup holds
  b.solo = !o->no_solo && !events && (o->policy != GSW_POLICY_TREE || w.tree_nodes <= kSoloTree) ? kSoloMaxLevels : 0;
  GSW_TRY(launch_init(g, b, g->iso, src, k0, flags0, s));
  if (events) GSW_HIP(hipEventRecord(ev_after(-1), s));
  int64_t launched = 0;  // launches of the level kernels so far
  int64_t consumed = 0;  // of those, launches that completed a level whose record was read
  // A single-workgroup launch may hand its first level back untouched (too
  // many arcs for one workgroup); the launch queued after one is therefore
  // always a full-grid one, which runs whatever level it finds.
  bool solo = b.solo && solo_eligible(k0, 1, 1, 1, g->n, b.deg_max);
  bool last_solo = false;
  int want = solo ? kSoloAhead : kAhead + level_launches(k0, 1) - 1;
  const int32_t cap = o->max_workgroups > 0 && o->max_workgroups < b.grid_max ? o->max_workgroups : b.grid_max;
  int32_t size = cap;
  int64_t nf_prev = 0;  // frontier of the level before the latest record's
  int64_t d = 0;
  for (;; ++d) {
    while (launched - consumed < want) {
      last_solo = solo && !last_solo;
      if (last_solo)
        GSW_TRY(launch_level_solo(g, b, dp, (int32_t)launched, s));
      else
        GSW_TRY(launch_level_auto(g, b, dp, (int32_t)launched, size, s));
      if (events) GSW_HIP(hipEventRecord(ev_after(launched), s));
      ++launched;
    }
    Record r;
    GSW_TRY(wait_record(g, d, s, &r));
    const int64_t nn = r.next;
    const int nk = r.next_kernel;
    const int64_t first_j = consumed;  // launches of this level: first_j .. r.launch
    if (trace && *rows < trace_cap) {
      trace_row(&trace[*rows], src_idx, d, r, timed, w.tick_ms);
      if (events) {
        float ms = 0.0f;
        GSW_HIP(hipEventSynchronize(ev_after(r.launch)));
        GSW_HIP(hipEventElapsedTime(&ms, ev_after(first_j - 1), ev_after(r.launch)));
        trace[*rows].ms = ms;
      }
    }
    if (r.launch + 1 > consumed) consumed = r.launch + 1;
    ++*rows;
    if (nn == 0) break;
    solo = b.solo && solo_eligible(nk, nn, r.nf, r.disc + nn, g->n, b.deg_max);
    want = solo ? kSoloAhead : kAhead + level_launches(nk, nn) - 1;
    size = launch_size(nk, nn, r.nf, nf_prev, r.disc, d, g->n, cap);
    nf_prev = r.nf;
  }
  w.ring_used = d + 1;
  if (o->canonical_parents && pa) GSW_TRY(launch_canonical_parents(g, lv, pa, s));
  return GSW_OK;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

gsw_status dalloc(DevBuf& b, size_t bytes) {
  hipError_t e = hipMalloc(&b.p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(GSW_ENOMEM, "hipMalloc(%zu) failed", bytes);
  }
  return GSW_OK;
}

// Whether the policy can ever name a kernel of base `base` (the edge lists
// need their origin arrays).
bool may_pick(const gsw_bfs_opts* o, int base) {
  switch (o->policy) {
    case GSW_POLICY_FIXED:
      return kernel_base(o->fixed_kernel) == base;
    case GSW_POLICY_SCHEDULE:
      for (int32_t i = 0; i < o->schedule_len; ++i)
        if (kernel_base(o->schedule[i]) == base) return true;
      return false;
    default:
      for (int32_t k : o->tree->class_kernel)
        if (kernel_base(k) == base) return true;
      return false;
  }
}

// The per-source loop of gsw_bfs (the graph's lock held, options checked).
gsw_status bfs_sources(gsw_graph* g, const gsw_bfs_opts* o, const int32_t* sources, int32_t n_sources,
                       int32_t* levels, int32_t* parents, gsw_level_trace* trace, int32_t trace_cap,
                       int32_t* rows) {
  GSW_HIP(hipSetDevice(g->device));
  GSW_TRY(ensure_workspace(g));
  if (may_pick(o, GSW_K_EDGE_SCAN)) GSW_TRY(ensure_origin(g));
  if (may_pick(o, GSW_K_REV_EDGE_SCAN)) GSW_TRY(ensure_rorigin(g));
  const hipStream_t s = pick_stream(g, o->stream);
  if (o->policy == GSW_POLICY_TREE) GSW_TRY(ensure_tree(g, o->tree, s));
  if (o->policy == GSW_POLICY_SCHEDULE) GSW_TRY(ensure_schedule(g, o->schedule, o->schedule_len, s));
  const bool has_origin = g->origin != nullptr || g->nnz == 0;
  const bool has_rorigin = g->rorigin != nullptr || g->nnz == 0;
  const Policy pol{o, has_origin, has_rorigin};
  const BfsPolicy dp = device_policy(g, g->ws, o, has_origin, has_rorigin);
  const int64_t n = g->n;
  for (int32_t i = 0; i < n_sources; ++i) {
    int32_t* lv = o->device_ptrs ? levels + (size_t)i * n : g->ws.lvl_tmp;
    int32_t* pa = parents ? (o->device_ptrs ? parents + (size_t)i * n : g->ws.par_tmp) : nullptr;
    const gsw_status st = run_levels(g, pol, dp, i, sources[i], lv, pa, trace, trace_cap, rows, s);
    if (st != GSW_OK) {
      (void)hipStreamSynchronize(s);
      return st;
    }
    if (!o->device_ptrs) {
      GSW_HIP(hipMemcpyAsync(levels + (size_t)i * n, lv, (size_t)n * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      if (pa)
        GSW_HIP(hipMemcpyAsync(parents + (size_t)i * n, pa, (size_t)n * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
    }
  }
  GSW_HIP(hipStreamSynchronize(s));
  return GSW_OK;
}

}  // namespace

gsw_status bfs_rows_locked(gsw_graph* g, const int32_t* sources, int32_t count, int32_t* d_levels,
                           const gsw_tree* tree, hipStream_t s) {
  gsw_bfs_opts o;
  gsw_bfs_opts_default(&o);
  if (tree) {
    o.policy = GSW_POLICY_TREE;
    o.tree = tree;
  } else {
    o.policy = GSW_POLICY_FIXED;
    o.fixed_kernel = GSW_DEFAULT_KERNEL;
  }
  o.device_ptrs = 1;
  o.stream = s;
  int32_t rows = 0;
  return bfs_sources(g, &o, sources, count, d_levels, nullptr, nullptr, 0, &rows);
}

}  // namespace gsw

using namespace gsw;

extern "C" {

gsw_status gsw_bfs(const gsw_graph* cg, const int32_t* sources, int32_t n_sources, int32_t* levels,
                   int32_t* parents, gsw_level_trace* trace, int32_t trace_cap, int32_t* trace_len,
                   const gsw_bfs_opts* opts) {
  clear_error();
  if (trace_len) *trace_len = 0;
  if (!cg || !sources || n_sources < 0 || (n_sources > 0 && !levels))
    return fail(GSW_EINVAL, "null graph, sources or levels");
  gsw_bfs_opts def;
  gsw_bfs_opts_default(&def);
  const gsw_bfs_opts* o = opts ? opts : &def;
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= g->n)
      return fail(GSW_EINVAL, "source %d (index %d) out of [0, %lld)", sources[i], i, (long long)g->n);
  switch (o->policy) {
    case GSW_POLICY_TREE:
      if (!o->tree) return fail(GSW_ENOTREE, "tree policy without a tree");
      break;
    case GSW_POLICY_FIXED:
      GSW_TRY(check_kernel(g, o->fixed_kernel));
      break;
    case GSW_POLICY_SCHEDULE:
      if (!o->schedule || o->schedule_len < 1) return fail(GSW_EINVAL, "empty schedule");
      for (int32_t i = 0; i < o->schedule_len; ++i) GSW_TRY(check_kernel(g, o->schedule[i]));
      break;
    default:
      return fail(GSW_EINVAL, "unknown policy %d", o->policy);
  }
  std::lock_guard<std::mutex> lock(g->mu);
  int32_t rows = 0;
  GSW_TRY(bfs_sources(g, o, sources, n_sources, levels, parents, trace, trace_cap, &rows));
  if (trace_len) *trace_len = rows;
  return GSW_OK;
}

gsw_status gsw_bfs_profile(const gsw_graph* cg, int32_t source, const int32_t* kernels,
                           int32_t n_kernels, int32_t reps, int32_t advance_kernel, float* times,
                           int64_t* frontier, int32_t max_levels, int32_t* n_levels, void* stream) {
  clear_error();
  if (n_levels) *n_levels = 0;
  if (!cg || !kernels || n_kernels < 1 || reps < 1 || !times || max_levels < 1)
    return fail(GSW_EINVAL, "bad profile arguments");
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  if (source < 0 || source >= g->n) return fail(GSW_EINVAL, "source %d out of range", source);
  for (int32_t i = 0; i < n_kernels; ++i)
    if (kernels[i] < 0 || kernels[i] >= GSW_N_KERNELS) return fail(GSW_EINVAL, "bad kernel id %d", kernels[i]);
  if (advance_kernel >= 0) GSW_TRY(check_kernel(g, advance_kernel));
  std::lock_guard<std::mutex> lock(g->mu);
  GSW_HIP(hipSetDevice(g->device));
  GSW_TRY(ensure_workspace(g));
  for (int32_t i = 0; i < n_kernels; ++i) {
    if (kernel_base(kernels[i]) == GSW_K_EDGE_SCAN) GSW_TRY(ensure_origin(g));
    if (kernel_base(kernels[i]) == GSW_K_REV_EDGE_SCAN) GSW_TRY(ensure_rorigin(g));
  }
  if (advance_kernel >= 0 && kernel_base(advance_kernel) == GSW_K_EDGE_SCAN) GSW_TRY(ensure_origin(g));
  if (advance_kernel >= 0 && kernel_base(advance_kernel) == GSW_K_REV_EDGE_SCAN) GSW_TRY(ensure_rorigin(g));
  Workspace& w = g->ws;
  const hipStream_t s = pick_stream(g, stream);
  const int64_t n = g->n;
  const size_t vb = (size_t)n * sizeof(int32_t), bb = (size_t)w.nw * sizeof(unsigned long long);
  const size_t cb = 4 * kCtrSlot * sizeof(uint32_t);
  DevBuf s_lv, s_pa, s_vis, s_bm, s_q, s_ctr;
  GSW_TRY(dalloc(s_lv, vb));
  GSW_TRY(dalloc(s_pa, vb));
  GSW_TRY(dalloc(s_vis, bb));
  GSW_TRY(dalloc(s_bm, 3 * bb));
  GSW_TRY(dalloc(s_q, (size_t)kQueueBins * vb));
  GSW_TRY(dalloc(s_ctr, cb));
  int32_t* lv = w.lvl_tmp;
  int32_t* pa = w.par_tmp;
  // every level is run with a named kernel: a fixed policy whose choices the
  // profiler overwrites in the control block before each run
  gsw_bfs_opts fo;
  gsw_bfs_opts_default(&fo);
  fo.policy = GSW_POLICY_FIXED;
  fo.fixed_kernel = GSW_DEFAULT_KERNEL;
  const bool has_origin = g->origin != nullptr || g->nnz == 0;
  const bool has_rorigin = g->rorigin != nullptr || g->nnz == 0;
  const BfsPolicy dp = device_policy(g, w, &fo, has_origin, has_rorigin);
  const BfsBase b = make_base(g, w, lv, pa, false, false);
  BfsBase b_solo = b;  // one level per single-workgroup launch
  b_solo.solo = 1;
  std::memset(w.ring, 0, (size_t)kBfsRing * kBfsRec * sizeof(unsigned long long));
  w.ring_used = -1;  // every level reposts its record here: the next search clears the whole ring
  GSW_TRY(launch_init(g, b, g->iso, source, GSW_DEFAULT_KERNEL, 0, s));
  GSW_HIP(hipStreamSynchronize(s));
  int64_t nf = 1;
  int64_t nf1 = 0, nf2 = 0, disc1 = 0;  // frontiers of the two levels before, discovered before this one
  uint32_t bins[kQueueBins] = {1};  // segment sizes of the current queue
  std::vector<float> samples((size_t)reps);
  BfsCtl saved_ctl;
  int cur = 0;  // control slot holding the next level's state
  for (int32_t d = 0;; ++d) {
    if (d >= max_levels) return fail(GSW_ERANGE, "BFS longer than max_levels=%d", max_levels);
    int32_t* qin = w.q[d & 1];
    // copies queue segments of the current frontier only
    auto copy_queue = [&](int32_t* dst, const int32_t* src) -> gsw_status {
      for (int bi = 0; bi < kQueueBins; ++bi)
        if (bins[bi])
          GSW_HIP(hipMemcpyAsync(dst + (size_t)bi * n, src + (size_t)bi * n, bins[bi] * sizeof(int32_t),
                                 hipMemcpyDeviceToDevice, s));
      return GSW_OK;
    };
    auto save = [&]() -> gsw_status {
      GSW_HIP(hipMemcpyAsync(s_lv.p, lv, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(s_pa.p, pa, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(s_vis.p, w.vis, bb, hipMemcpyDeviceToDevice, s));
      for (int i = 0; i < 3; ++i)
        GSW_HIP(hipMemcpyAsync((char*)s_bm.p + i * bb, w.bm[i], bb, hipMemcpyDeviceToDevice, s));
      GSW_TRY(copy_queue((int32_t*)s_q.p, qin));
      GSW_HIP(hipMemcpyAsync(s_ctr.p, w.ctr, cb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(w.h_ctl, w.ctl + cur, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
      GSW_HIP(hipStreamSynchronize(s));
      saved_ctl = *w.h_ctl;
      return GSW_OK;
    };
    // restores the saved state with kernel k named for level d, in slot 0
    // (the next launch is counted as launch 0)
    auto restore = [&](int k) -> gsw_status {
      GSW_HIP(hipMemcpyAsync(lv, s_lv.p, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(pa, s_pa.p, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(w.vis, s_vis.p, bb, hipMemcpyDeviceToDevice, s));
      for (int i = 0; i < 3; ++i)
        GSW_HIP(hipMemcpyAsync(w.bm[i], (char*)s_bm.p + i * bb, bb, hipMemcpyDeviceToDevice, s));
      GSW_TRY(copy_queue(qin, (const int32_t*)s_q.p));
      GSW_HIP(hipMemcpyAsync(w.ctr, s_ctr.p, cb, hipMemcpyDeviceToDevice, s));
      *w.h_ctl = saved_ctl;
      w.h_ctl->kernel = k;
      w.h_ctl->grid = level_participants(k, nf, b);
      w.h_ctl->done = 0ull;
      w.h_ctl->phase = level_first_phase(k, nf);
      GSW_HIP(hipMemcpyAsync(w.ctl, w.h_ctl, sizeof(BfsCtl), hipMemcpyHostToDevice, s));
      GSW_HIP(hipStreamSynchronize(s));  // the staging copy is reused by the next restore
      return GSW_OK;
    };
    // one level with kernel k as the level loop runs it: a single-workgroup
    // launch when the level qualifies for one by the graph's degree bound
    // (never handed back), else the level kernel with the loop's launch size,
    // twice for push_edge on more than kEdgeFuse entries
    auto run = [&](int k, bool timed_bracket) -> gsw_status {
      const bool solo = kernel_base(k) <= GSW_K_PUSH_EDGE && nf <= kSoloMax &&
                        (long long)b.deg_max * nf <= kSoloMaxArcs;
      const int32_t size = launch_size(k, nf, nf1, nf2, disc1, d - 1, n, b.grid_max);
      if (timed_bracket) GSW_HIP(hipEventRecord(w.ev[0], s));
      if (solo) {
        GSW_TRY(launch_level_solo(g, b_solo, dp, 0, s));
      } else {
        GSW_TRY(launch_level_auto(g, b, dp, 0, size, s));
        if (level_launches(k, nf) == 2) GSW_TRY(launch_level_auto(g, b, dp, 1, size, s));
      }
      if (timed_bracket) GSW_HIP(hipEventRecord(w.ev[1], s));
      return GSW_OK;
    };
    GSW_TRY(save());
    for (int32_t ki = 0; ki < n_kernels; ++ki) {
      const int k = kernels[ki];
      for (int32_t r = 0; r < reps; ++r) {
        GSW_TRY(restore(k));
        GSW_TRY(run(k, true));
        GSW_HIP(hipEventSynchronize(w.ev[1]));
        GSW_HIP(hipEventElapsedTime(&samples[(size_t)r], w.ev[0], w.ev[1]));
      }
      std::sort(samples.begin(), samples.end());
      times[(size_t)d * n_kernels + ki] = samples[(size_t)reps / 2];
    }
    // advance with the given kernel, or with this level's fastest one
    int adv = advance_kernel;
    if (adv < 0) {
      float best = 0.0f;
      for (int32_t ki = 0; ki < n_kernels; ++ki) {
        const float t = times[(size_t)d * n_kernels + ki];
        if (t >= 0.0f && (adv < 0 || t < best)) {
          best = t;
          adv = kernels[ki];
        }
      }
    }
    GSW_TRY(restore(adv));
    const bool adv_solo = kernel_base(adv) <= GSW_K_PUSH_EDGE && nf <= kSoloMax &&
                          (long long)b.deg_max * nf <= kSoloMaxArcs;
    GSW_TRY(run(adv, false));
    cur = adv_solo ? 1 : level_launches(adv, nf) & 1;  // slot written by the last launch
    GSW_HIP(hipStreamSynchronize(s));
    Record r;
    GSW_TRY(wait_record(g, d, s, &r));
    const int64_t nn = r.next;
    GSW_HIP(hipMemcpy(w.h_ctr, w.ctr + (size_t)((d + 1) & 3) * kCtrSlot, kCtrSlot * sizeof(uint32_t),
                      hipMemcpyDeviceToHost));
    for (int bi = 0; bi < kQueueBins; ++bi) bins[bi] = w.h_ctr[bi * kCtrStride];
    if (frontier) frontier[d] = nf;
    if (n_levels) *n_levels = d + 1;
    if (nn == 0) break;
    nf2 = nf1;
    nf1 = nf;
    disc1 += nf;
    nf = nn;
  }
  GSW_HIP(hipStreamSynchronize(s));
  return GSW_OK;
}

}  // extern "C"
