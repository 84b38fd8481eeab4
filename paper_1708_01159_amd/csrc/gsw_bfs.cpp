// Host-driven level loop: per level, read the new frontier size, build the
// feature vector, pick the next kernel (tree, fixed or scheduled policy) and
// launch it.  Also the per-level profiler that measures every kernel from the
// same saved state (the training data of the decision tree).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "gsw_internal.h"

namespace gsw {
namespace {

struct Policy {
  const gsw_bfs_opts* o;
  bool symmetric;
  // Kernel for level d; *flags gets bit0 when the tree leaf was undecided,
  // bit1 when a pull choice was replaced on a non-symmetric graph.
  int choose(const gsw_graph* g, int32_t d, int64_t nf, int64_t disc, int prev, int32_t* flags) const {
    *flags = 0;
    int k = GSW_DEFAULT_KERNEL;
    switch (o->policy) {
      case GSW_POLICY_FIXED:
        k = o->fixed_kernel;
        break;
      case GSW_POLICY_SCHEDULE:
        k = o->schedule[d < o->schedule_len ? d : o->schedule_len - 1];
        break;
      default: {
        double x[GSW_N_FEATURES];
        gsw_level_features(g, nf, disc, x);
        int32_t kk = GSW_DEFAULT_KERNEL, unk = 0;
        gsw_tree_predict(o->tree, x, prev, d, &kk, &unk);
        k = kk;
        if (unk) *flags |= 1;
        break;
      }
    }
    if (kernel_is_pull(k) && !symmetric) {
      k = GSW_DEFAULT_KERNEL;
      *flags |= 2;
    }
    return k;
  }
};

// Buffers of level d: queue q[d&1] with counter slot d&3 in, q[(d+1)&1] and
// slot (d+1)&3 out, slot (d+2)&3 zeroed for the level after next; frontier
// bitmap bm[d&1] in (pull), bm[(d+1)&1] out (pull).
LevelLaunch level_args(const gsw_graph* g, int32_t* lv, int32_t* pa, int32_t d, uint32_t nf) {
  const Workspace& w = g->ws;
  LevelLaunch l;
  l.offs = g->offs;
  l.cols = g->cols;
  l.origin = g->origin;
  l.level = lv;
  l.parent = pa;
  l.vis = w.vis;
  l.fr = w.bm[d & 1];
  l.nx = w.bm[(d + 1) & 1];
  l.qin = w.q[d & 1];
  l.cin = w.ctr + (size_t)(d & 3) * kCtrSlot;
  l.qout = w.q[(d + 1) & 1];
  l.cout = w.ctr + (size_t)((d + 1) & 3) * kCtrSlot;
  l.cclr = w.ctr + (size_t)((d + 2) & 3) * kCtrSlot;
  l.tst = nullptr;
  l.n = g->n;
  l.nw = w.nw;
  l.nnz = g->nnz;
  l.n_in = nf;
  l.d = d;
  return l;
}

// Size of the depth-(d+1) queue (sum over its segments); bins[] receives the
// per-segment counts when non-null.
gsw_status read_next(const gsw_graph* g, int32_t d, hipStream_t s, int64_t* nn, uint32_t* bins) {
  const Workspace& w = g->ws;
  GSW_HIP(hipMemcpyAsync(w.h_ctr, w.ctr + (size_t)((d + 1) & 3) * kCtrSlot,
                         kCtrSlot * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  GSW_HIP(hipStreamSynchronize(s));
  int64_t t = 0;
  for (int b = 0; b < kQueueBins; ++b) {
    t += w.h_ctr[b * kCtrStride];
    if (bins) bins[b] = w.h_ctr[b * kCtrStride];
  }
  *nn = t;
  return GSW_OK;
}

// Waits until the device has stored level d's next-frontier size in host
// memory (k_finalize).  Polls the stream for errors now and then so a failed
// launch cannot leave the host spinning.
gsw_status wait_next(const gsw_graph* g, int32_t d, hipStream_t s, int64_t* nn) {
  volatile uint32_t* f = g->ws.h_flag + (size_t)(d % kFlagSlots) * 64;
  for (uint64_t it = 0;; ++it) {
    const uint32_t v = *f;
    if (v != kNotReady) {
      *nn = (int64_t)v;
      return GSW_OK;
    }
    if ((it & 4095u) == 4095u) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        const uint32_t v2 = *f;
        if (v2 != kNotReady) {
          *nn = (int64_t)v2;
          return GSW_OK;
        }
        return fail(GSW_EHIP, "level %d finished without reporting its frontier size", d);
      }
      if (e != hipErrorNotReady) return fail(GSW_EHIP, "level %d: %s", d, hipGetErrorString(e));
    }
    __builtin_ia32_pause();
  }
}

// One level: the frontier bitmap is rebuilt first when pull follows a
// top-down level (its input bitmap is otherwise stale).
gsw_status run_level(const gsw_graph* g, int k, const LevelLaunch& l, bool fr_valid, hipStream_t s) {
  if (kernel_is_pull(k) && !fr_valid)
    GSW_TRY(launch_frontier_bitmap(g, l.level, l.d, const_cast<unsigned long long*>(l.fr), s));
  return launch_level(g, k, l, s);
}

gsw_status check_kernel(const gsw_graph* g, int k) {
  if (k < 0 || k >= GSW_N_KERNELS) return fail(GSW_EINVAL, "unknown kernel id %d", k);
  if (kernel_is_pull(k) && !g->symmetric)
    return fail(GSW_ENOTSYM, "kernel %s needs a symmetric graph", gsw_kernel_name(k));
  return GSW_OK;
}

gsw_status run_one(gsw_graph* g, const Policy& pol, int32_t src_idx, int32_t src, int32_t* lv,
                   int32_t* pa, gsw_level_trace* trace, int32_t trace_cap, int32_t* rows,
                   hipStream_t s) {
  Workspace& w = g->ws;
  const gsw_bfs_opts* o = pol.o;
  GSW_TRY(launch_init(g, lv, pa, src, s));
  int64_t nf = 1, disc = 1;
  int prev = GSW_DEFAULT_KERNEL;
  bool fr_valid = true;  // init wrote the depth-0 bitmap
  const int32_t row0 = *rows;
  int32_t timed = 0;  // levels bracketed by events (read after the last level)
  for (int32_t d = 0;; ++d) {
    int32_t flags = 0;
    const int k = pol.choose(g, d, nf, disc, prev, &flags);
    if (k == GSW_K_EDGE_SCAN) GSW_TRY(ensure_origin(g));
    const LevelLaunch l = level_args(g, lv, pa, d, (uint32_t)nf);
    const size_t slot = (size_t)(d % kFlagSlots) * 64;
    w.h_flag[slot] = kNotReady;
    const bool timing = o->time_levels && d < kMaxTimedLevels && *rows < trace_cap;
    // the bitmap rebuild before a pull that follows a top-down level stays
    // outside the timed bracket: trace ms is the expansion kernel(s) only
    if (kernel_is_pull(k) && !fr_valid)
      GSW_TRY(launch_frontier_bitmap(g, l.level, l.d, const_cast<unsigned long long*>(l.fr), s));
    LevelLaunch lt = l;
    if (timing) {
      lt.tst = w.tst;
      timed = d + 1;
    }
    GSW_TRY(launch_level(g, k, lt, s));
    GSW_TRY(launch_finalize(l.cout, w.d_flag + slot, timing ? w.tst : nullptr,
                            timing ? w.lvl_ticks + d : nullptr, s));
    fr_valid = kernel_is_pull(k);
    int64_t nn = 0;
    GSW_TRY(wait_next(g, d, s, &nn));
    if (trace && *rows < trace_cap) {
      gsw_level_trace& t = trace[*rows];
      t.source_idx = src_idx;
      t.level = d;
      t.kernel = k;
      t.flags = flags;
      t.n_frontier = nf;
      t.discovered = disc;
      t.n_next = nn;
      t.ms = -1.0f;
      t.reserved = 0;
    }
    ++*rows;
    if (nn == 0) break;
    nf = nn;
    disc += nn;
    prev = k;
  }
  if (o->canonical_parents && pa) GSW_TRY(launch_canonical_parents(g, lv, pa, s));
  GSW_HIP(hipStreamSynchronize(s));
  if (timed > 0 && trace) {
    GSW_HIP(hipMemcpyAsync(w.h_ticks, w.lvl_ticks, (size_t)timed * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    GSW_HIP(hipStreamSynchronize(s));
    for (int32_t d = 0; d < timed && row0 + d < trace_cap; ++d)
      trace[row0 + d].ms = (float)((double)w.h_ticks[d] * w.tick_ms);
  }
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

}  // namespace
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
  GSW_HIP(hipSetDevice(g->device));
  GSW_TRY(ensure_workspace(g));
  const hipStream_t s = pick_stream(g, o->stream);
  const Policy pol{o, g->symmetric != 0};
  const int64_t n = g->n;
  int32_t rows = 0;
  for (int32_t i = 0; i < n_sources; ++i) {
    int32_t* lv = o->device_ptrs ? levels + (size_t)i * n : g->ws.lvl_tmp;
    int32_t* pa = parents ? (o->device_ptrs ? parents + (size_t)i * n : g->ws.par_tmp) : nullptr;
    GSW_TRY(run_one(g, pol, i, sources[i], lv, pa, trace, trace_cap, &rows, s));
    if (!o->device_ptrs) {
      GSW_HIP(hipMemcpyAsync(levels + (size_t)i * n, lv, (size_t)n * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      if (pa)
        GSW_HIP(hipMemcpyAsync(parents + (size_t)i * n, pa, (size_t)n * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
      GSW_HIP(hipStreamSynchronize(s));
    }
  }
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
  for (int32_t i = 0; i < n_kernels; ++i)
    if (kernels[i] == GSW_K_EDGE_SCAN) GSW_TRY(ensure_origin(g));
  if (advance_kernel == GSW_K_EDGE_SCAN) GSW_TRY(ensure_origin(g));
  Workspace& w = g->ws;
  const hipStream_t s = pick_stream(g, stream);
  const int64_t n = g->n;
  const size_t vb = (size_t)n * sizeof(int32_t), bb = (size_t)w.nw * sizeof(unsigned long long);
  const size_t cb = 4 * kCtrSlot * sizeof(uint32_t);
  DevBuf s_lv, s_pa, s_vis, s_bm, s_q, s_ctr;
  GSW_TRY(dalloc(s_lv, vb));
  GSW_TRY(dalloc(s_pa, vb));
  GSW_TRY(dalloc(s_vis, bb));
  GSW_TRY(dalloc(s_bm, 2 * bb));
  GSW_TRY(dalloc(s_q, (size_t)kQueueBins * vb));
  GSW_TRY(dalloc(s_ctr, cb));
  int32_t* lv = w.lvl_tmp;
  int32_t* pa = w.par_tmp;
  GSW_TRY(launch_init(g, lv, pa, source, s));
  int64_t nf = 1;
  uint32_t bins[kQueueBins] = {1};  // segment sizes of the current queue
  bool fr_valid = true;
  std::vector<float> samples((size_t)reps);
  for (int32_t d = 0;; ++d) {
    if (d >= max_levels) return fail(GSW_ERANGE, "BFS longer than max_levels=%d", max_levels);
    int32_t* qin = w.q[d & 1];
    // copies queue segments of the current frontier only
    auto copy_queue = [&](int32_t* dst, const int32_t* src) -> gsw_status {
      for (int b = 0; b < kQueueBins; ++b)
        if (bins[b])
          GSW_HIP(hipMemcpyAsync(dst + (size_t)b * n, src + (size_t)b * n, bins[b] * sizeof(int32_t),
                                 hipMemcpyDeviceToDevice, s));
      return GSW_OK;
    };
    auto save = [&]() -> gsw_status {
      GSW_HIP(hipMemcpyAsync(s_lv.p, lv, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(s_pa.p, pa, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(s_vis.p, w.vis, bb, hipMemcpyDeviceToDevice, s));
      for (int b = 0; b < 2; ++b)
        GSW_HIP(hipMemcpyAsync((char*)s_bm.p + b * bb, w.bm[b], bb, hipMemcpyDeviceToDevice, s));
      GSW_TRY(copy_queue((int32_t*)s_q.p, qin));
      GSW_HIP(hipMemcpyAsync(s_ctr.p, w.ctr, cb, hipMemcpyDeviceToDevice, s));
      return GSW_OK;
    };
    auto restore = [&]() -> gsw_status {
      GSW_HIP(hipMemcpyAsync(lv, s_lv.p, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(pa, s_pa.p, vb, hipMemcpyDeviceToDevice, s));
      GSW_HIP(hipMemcpyAsync(w.vis, s_vis.p, bb, hipMemcpyDeviceToDevice, s));
      for (int b = 0; b < 2; ++b)
        GSW_HIP(hipMemcpyAsync(w.bm[b], (char*)s_bm.p + b * bb, bb, hipMemcpyDeviceToDevice, s));
      GSW_TRY(copy_queue(qin, (const int32_t*)s_q.p));
      GSW_HIP(hipMemcpyAsync(w.ctr, s_ctr.p, cb, hipMemcpyDeviceToDevice, s));
      return GSW_OK;
    };
    GSW_TRY(save());
    const LevelLaunch l = level_args(g, lv, pa, d, (uint32_t)nf);
    for (int32_t ki = 0; ki < n_kernels; ++ki) {
      const int k = kernels[ki];
      if (kernel_is_pull(k) && !g->symmetric) {
        times[(size_t)d * n_kernels + ki] = -1.0f;
        continue;
      }
      for (int32_t r = 0; r < reps; ++r) {
        GSW_TRY(restore());
        GSW_HIP(hipEventRecord(w.ev[0], s));
        GSW_TRY(run_level(g, k, l, fr_valid, s));
        GSW_HIP(hipEventRecord(w.ev[1], s));
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
    GSW_TRY(restore());
    GSW_TRY(run_level(g, adv, l, fr_valid, s));
    fr_valid = kernel_is_pull(adv);
    int64_t nn = 0;
    GSW_TRY(read_next(g, d, s, &nn, bins));
    if (frontier) frontier[d] = nf;
    if (n_levels) *n_levels = d + 1;
    if (nn == 0) break;
    nf = nn;
  }
  GSW_HIP(hipStreamSynchronize(s));
  return GSW_OK;
}

}  // extern "C"
