// gsw_bfs_noalloc: the single-source BFS of gsw_bfs for callers that cannot
// allocate memory.  Every buffer its kernels need beyond the caller's graph,
// levels and parents -- bitmaps, frontier queues, counters, level control,
// push_edge scan arrays, the head copy of the in-arcs, the vertices without
// in-arcs, the per-level records, the device copies of a tree or schedule --
// lives in one file-scope device array of fixed size, laid out for graphs of
// up to GSW_NOALLOC_MAX_VERTICES vertices.  The level kernels are the same as
// gsw_bfs's; only the buffers and the host's reading of the level records
// differ: the records go to device memory, and the host queues kBatch
// launches at a time (single-workgroup multi-level launches are not used
// here, so each launch completes at most one level), then copies those
// levels' records back and waits.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "gsw_internal.h"

namespace gsw {
namespace {

constexpr int64_t kMaxN = GSW_NOALLOC_MAX_VERTICES;
constexpr int64_t kMaxNw = (kMaxN + 63) / 64;
constexpr int32_t kMaxTree = GSW_NOALLOC_MAX_TREE_NODES;
constexpr int32_t kMaxSched = GSW_NOALLOC_MAX_SCHEDULE;
constexpr int kMaxDevices = 64;

constexpr size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte offsets of the regions inside the array, each 256-byte aligned.
struct Layout {
  size_t vis, bm[3], iso, ctl, done, q[2], ctr, actr, scan, ebeg, bsum, head, ring, tree, thr, sched, total;
};

constexpr Layout make_layout() {
  Layout L{};
  size_t at = 0;
  auto take = [&at](size_t bytes) {
    const size_t p = at;
    at += round256(bytes);
    return p;
  };
  const size_t bmb = (size_t)kMaxNw * sizeof(unsigned long long);
  L.vis = take(bmb);
  L.bm[0] = take(bmb);
  L.bm[1] = take(bmb);
  L.bm[2] = take(bmb);
  L.iso = take(bmb);
  L.ctl = take(2 * sizeof(BfsCtl));
  L.done = take((size_t)kDoneGroups * kCtrStride * sizeof(unsigned long long));
  L.q[0] = take((size_t)kQueueBins * kMaxN * sizeof(int32_t));
  L.q[1] = take((size_t)kQueueBins * kMaxN * sizeof(int32_t));
  L.ctr = take(4 * kCtrSlot * sizeof(uint32_t));
  L.actr = take(4 * kArcSlot * sizeof(unsigned long long));
  L.scan = take((size_t)kMaxN * sizeof(int64_t));
  L.ebeg = take((size_t)kMaxN * sizeof(int64_t));
  L.bsum = take((size_t)((kMaxN + 1023) / 1024 + 1) * sizeof(int64_t));
  L.head = take((size_t)kMaxN * kHeadArcs * sizeof(int32_t));
  L.ring = take((size_t)kBfsRing * kBfsRec * sizeof(unsigned long long));
  L.tree = take((size_t)kMaxTree * sizeof(unsigned long long));
  L.thr = take((size_t)kMaxTree * sizeof(int32_t));
  L.sched = take((size_t)kMaxSched * sizeof(int32_t));
  L.total = at;
  return L;
}

constexpr Layout kLayout = make_layout();
static_assert(kLayout.total == GSW_NOALLOC_SCRATCH_BYTES, "gsw.h states the scratch size");

// The scratch memory.  In host code this name is only a stand-in for the
// array: its device address (one per GPU) comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kLayout.total];

// Per device: the array's device address and the wall-clock period, looked
// up once with that device current.
struct DeviceScratch {
  unsigned char* ptr = nullptr;
  double tick_ms = 0.0;
};
DeviceScratch g_dev[kMaxDevices];

// Serialises every call of the process: the array is one per GPU, and the
// host-side tree buffers below are one per process.
std::mutex g_mu;

// Host buffers for specialising a tree (sized for the largest tree accepted)
// and for the record ring's copy.
int32_t h_order[kMaxTree], h_newid[kMaxTree], h_stack[kMaxTree + 1], h_thr[kMaxTree];
unsigned long long h_nodes[kMaxTree];
unsigned long long h_ring[(size_t)kBfsRing * kBfsRec];

constexpr int kBatch = 8;  // launches queued before each read of the records

gsw_status device_scratch(int device, DeviceScratch** out) {
  if (device < 0 || device >= kMaxDevices) return fail(GSW_EINVAL, "device %d out of range", device);
  DeviceScratch& d = g_dev[device];
  if (!d.ptr) {
    void* p = nullptr;
    GSW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GSW_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
    int khz = 0;
    GSW_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
    d.tick_ms = khz > 0 ? 1.0 / (double)khz : 0.0;
    d.ptr = static_cast<unsigned char*>(p);
  }
  *out = &d;
  return GSW_OK;
}

// A workspace whose device buffers are the regions of the array at `base`
// (only its pointers are used; nothing here is owned or freed).
void scratch_workspace(unsigned char* base, int64_t n, Workspace* w) {
  w->n = n;
  w->nw = (n + 63) / 64;
  w->vis = reinterpret_cast<unsigned long long*>(base + kLayout.vis);
  for (int i = 0; i < 3; ++i) w->bm[i] = reinterpret_cast<unsigned long long*>(base + kLayout.bm[i]);
  w->q[0] = reinterpret_cast<int32_t*>(base + kLayout.q[0]);
  w->q[1] = reinterpret_cast<int32_t*>(base + kLayout.q[1]);
  w->ctr = reinterpret_cast<uint32_t*>(base + kLayout.ctr);
  w->actr = reinterpret_cast<unsigned long long*>(base + kLayout.actr);
  w->scan = reinterpret_cast<int64_t*>(base + kLayout.scan);
  w->ebeg = reinterpret_cast<int64_t*>(base + kLayout.ebeg);
  w->bsum = reinterpret_cast<int64_t*>(base + kLayout.bsum);
  w->head = reinterpret_cast<int32_t*>(base + kLayout.head);
  w->ctl = reinterpret_cast<BfsCtl*>(base + kLayout.ctl);
  w->done = reinterpret_cast<unsigned long long*>(base + kLayout.done);
  w->d_ring = reinterpret_cast<unsigned long long*>(base + kLayout.ring);
  w->d_tree = reinterpret_cast<unsigned long long*>(base + kLayout.tree);
  w->d_thr = reinterpret_cast<int32_t*>(base + kLayout.thr);
  w->d_sched = reinterpret_cast<int32_t*>(base + kLayout.sched);
}

bool names_base(const gsw_bfs_opts* o, int base) {
  if (o->policy == GSW_POLICY_FIXED) return kernel_base(o->fixed_kernel) == base;
  if (o->policy == GSW_POLICY_SCHEDULE)
    for (int32_t i = 0; i < o->schedule_len; ++i)
      if (kernel_base(o->schedule[i]) == base) return true;
  return false;
}

gsw_status check_options(const gsw_graph* g, const gsw_bfs_opts* o) {
  if (g->n > kMaxN)
    return fail(GSW_EINVAL, "graph of %lld vertices: gsw_bfs_noalloc takes at most %lld", (long long)g->n,
                (long long)kMaxN);
  if (!o->device_ptrs) return fail(GSW_EINVAL, "gsw_bfs_noalloc needs device_ptrs = 1 (device levels/parents)");
  if (o->time_levels != 0 && o->time_levels != 1)
    return fail(GSW_EINVAL, "gsw_bfs_noalloc: time_levels must be 0 or 1 (events are not created here)");
  auto bad_kernel = [](int32_t k) { return k < 0 || k >= GSW_N_KERNELS; };
  switch (o->policy) {
    case GSW_POLICY_TREE:
      if (!o->tree) return fail(GSW_ENOTREE, "tree policy without a tree");
      if (o->tree->n_nodes > kMaxTree)
        return fail(GSW_EINVAL, "tree of %d nodes: gsw_bfs_noalloc takes at most %d", o->tree->n_nodes, kMaxTree);
      break;
    case GSW_POLICY_FIXED:
      if (bad_kernel(o->fixed_kernel)) return fail(GSW_EINVAL, "unknown kernel %d", o->fixed_kernel);
      break;
    case GSW_POLICY_SCHEDULE:
      if (!o->schedule || o->schedule_len < 1) return fail(GSW_EINVAL, "empty schedule");
      if (o->schedule_len > kMaxSched)
        return fail(GSW_EINVAL, "schedule of %d levels: gsw_bfs_noalloc takes at most %d", o->schedule_len,
                    kMaxSched);
      for (int32_t i = 0; i < o->schedule_len; ++i)
        if (bad_kernel(o->schedule[i])) return fail(GSW_EINVAL, "unknown kernel %d", o->schedule[i]);
      break;
    default:
      return fail(GSW_EINVAL, "unknown policy %d", o->policy);
  }
  // the edge lists' origin arrays are graph memory, built only by allocating calls
  if (g->nnz > 0 && !g->origin && names_base(o, GSW_K_EDGE_SCAN))
    return fail(GSW_EINVAL, "edge_scan needs the origin array: create the graph with GSW_WITH_ORIGIN");
  if (g->nnz > 0 && !g->rorigin && names_base(o, GSW_K_REV_EDGE_SCAN))
    return fail(GSW_EINVAL, "rev_edge_scan needs the in-arcs' origin array: create the graph with GSW_WITH_ORIGIN");
  return GSW_OK;
}

// Copies the ring slots of levels d .. d + count - 1 into h_ring.
gsw_status copy_records(const Workspace& w, int64_t d, int count, hipStream_t s) {
  const size_t rec = (size_t)kBfsRec * sizeof(unsigned long long);
  const int first = (int)(d % kBfsRing);
  const int a = count < kBfsRing - first ? count : kBfsRing - first;
  GSW_HIP(hipMemcpyAsync(h_ring + (size_t)first * kBfsRec, w.d_ring + (size_t)first * kBfsRec, (size_t)a * rec,
                         hipMemcpyDeviceToHost, s));
  if (count > a) GSW_HIP(hipMemcpyAsync(h_ring, w.d_ring, (size_t)(count - a) * rec, hipMemcpyDeviceToHost, s));
  return GSW_OK;
}

// One source.  The records of the levels run by the launches queued so far
// are all in the ring once the copy that follows them completes: each level
// takes at least one launch, so kBatch launches post at most kBatch records.
gsw_status run_source(gsw_graph* g, const Workspace& w, const gsw_bfs_opts* o, const BfsPolicy& dp,
                      bool has_origin, bool has_rorigin, double tick_ms, int32_t src_idx, int32_t src,
                      int32_t* lv, int32_t* pa, const unsigned long long* iso, gsw_level_trace* trace,
                      int32_t trace_cap, int32_t* rows, hipStream_t s) {
  const bool timed = o->time_levels == 1;
  GSW_HIP(hipMemsetAsync(w.d_ring, 0, (size_t)kBfsRing * kBfsRec * sizeof(unsigned long long), s));
  int32_t flags0 = 0;
  const int k0 = first_kernel(g, o, has_origin, has_rorigin, &flags0);
  const BfsBase b = make_base(g, w, lv, pa, timed, o->count_arcs != 0);  // solo launches off
  GSW_TRY(launch_init(g, b, iso, src, k0, flags0, s));
  const int32_t cap = o->max_workgroups > 0 && o->max_workgroups < b.grid_max ? o->max_workgroups : b.grid_max;
  int32_t j = 0;
  for (int64_t d = 0;;) {
    for (int i = 0; i < kBatch; ++i) GSW_TRY(launch_level_auto(g, b, dp, j++, cap, s));
    GSW_TRY(copy_records(w, d, kBatch, s));
    GSW_HIP(hipStreamSynchronize(s));
    const int64_t d0 = d;
    Record r;
    bool ended = false;
    while (!ended && d - d0 < kBatch && take_record(h_ring, d, &r)) {
      if (trace && *rows < trace_cap) trace_row(&trace[*rows], src_idx, d, r, timed, tick_ms);
      ++*rows;
      ++d;
      ended = r.next == 0;
    }
    if (ended) break;
    if (d == d0) return fail(GSW_EHIP, "level %lld posted no record in %d launches", (long long)d, kBatch);
  }
  if (o->canonical_parents && pa) GSW_TRY(launch_canonical_parents(g, lv, pa, s));
  return GSW_OK;
}

}  // namespace
}  // namespace gsw

using namespace gsw;

extern "C" gsw_status gsw_bfs_noalloc(const gsw_graph* cg, const int32_t* sources, int32_t n_sources,
                                      int32_t* levels, int32_t* parents, gsw_level_trace* trace,
                                      int32_t trace_cap, int32_t* trace_len, const gsw_bfs_opts* opts) {
  clear_error();
  if (trace_len) *trace_len = 0;
  if (!cg || !sources || !opts || n_sources < 0 || (n_sources > 0 && !levels))
    return fail(GSW_EINVAL, "null graph, sources, options or levels");
  gsw_graph* g = const_cast<gsw_graph*>(cg);
  GSW_TRY(check_options(g, opts));
  for (int32_t i = 0; i < n_sources; ++i)
    if (sources[i] < 0 || sources[i] >= g->n)
      return fail(GSW_EINVAL, "source %d (index %d) out of [0, %lld)", sources[i], i, (long long)g->n);
  std::lock_guard<std::mutex> lock(g_mu);
  GSW_HIP(hipSetDevice(g->device));
  DeviceScratch* ds = nullptr;
  GSW_TRY(device_scratch(g->device, &ds));
  const hipStream_t s = pick_stream(g, opts->stream);
  Workspace w;
  scratch_workspace(ds->ptr, g->n, &w);
  unsigned long long* iso = reinterpret_cast<unsigned long long*>(ds->ptr + kLayout.iso);
  // graph-derived buffers, rebuilt every call (the array is shared by every graph)
  GSW_TRY(launch_build_head(g, w.head, false, s));
  GSW_TRY(launch_isolated(g, iso, s));
  if (opts->policy == GSW_POLICY_TREE) {
    const TreeBuf buf{h_order, h_newid, h_stack, h_nodes, h_thr};
    const int32_t m = specialise_tree(g, opts->tree, buf);
    if (m < 1) return fail(GSW_EINVAL, "tree could not be specialised to the graph");
    w.tree_nodes = m;
    GSW_HIP(hipMemcpyAsync(w.d_tree, h_nodes, (size_t)m * sizeof(unsigned long long), hipMemcpyHostToDevice, s));
    GSW_HIP(hipMemcpyAsync(w.d_thr, h_thr, (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, s));
  } else if (opts->policy == GSW_POLICY_SCHEDULE) {
    GSW_HIP(hipMemcpyAsync(w.d_sched, opts->schedule, (size_t)opts->schedule_len * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
  }
  const bool has_origin = g->origin != nullptr || g->nnz == 0;
  const bool has_rorigin = g->rorigin != nullptr || g->nnz == 0;
  const BfsPolicy dp = device_policy(g, w, opts, has_origin, has_rorigin);
  int32_t rows = 0;
  for (int32_t i = 0; i < n_sources; ++i) {
    const gsw_status st = run_source(g, w, opts, dp, has_origin, has_rorigin, ds->tick_ms, i, sources[i],
                                     levels + (size_t)i * g->n, parents ? parents + (size_t)i * g->n : nullptr,
                                     iso, trace, trace_cap, &rows, s);
    if (st != GSW_OK) {
      (void)hipStreamSynchronize(s);
      return st;
    }
  }
  // the host buffers above are reused by the next call
  GSW_HIP(hipStreamSynchronize(s));
  if (trace_len) *trace_len = rows;
  return GSW_OK;
}
