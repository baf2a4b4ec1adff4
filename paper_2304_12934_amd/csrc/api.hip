// C ABI of libnufftradon (declared in include/nufftradon.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "nufftradon.h"
#include "plan.hpp"
#include "prior_kernels.hpp"
#include "radon_kernels.hpp"

// Opt-in stage timing: a pair of events recorded around every stage launch
// on the caller's stream, read back (and synchronised) on request.
enum {
  kStageFwdRows = 0, kStageFwdCols, kStageFwdInterp, kStageAdjRadial, kStageSpread, kStageAdjCols,
  kStageAdjRows, kStageResidual, kStagePrior, kStageUpdate, kStageSpreadClear, kStageCount
};

struct StageEvents {
  int stage;
  hipEvent_t start, stop;
};

struct nr_plan {
  nr::Plan p;
  bool profiling = false;
  std::vector<StageEvents> recorded;
  std::vector<hipEvent_t> pool;
  std::vector<SliceDesc> host_descs;
  // concurrent lanes: streams (default priority, non-blocking) plus the
  // events that fork them from and join them back to the caller's stream
  int lane_device = -1;
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_done;
  std::vector<hipEvent_t> lane_skew;
  hipEvent_t fork = nullptr;
  // host streaming: copy-in and copy-out streams and the events that order
  // the two chunk buffers between them and the compute stream
  int io_device = -1;
  hipStream_t io_in = nullptr, io_out = nullptr;
  hipEvent_t io_fork = nullptr, io_done = nullptr;
  hipEvent_t h2d_done[2] = {nullptr, nullptr}, comp_done[2] = {nullptr, nullptr}, d2h_done[2] = {nullptr, nullptr};
  void drop_io() {
    for (hipStream_t* st : {&io_in, &io_out})
      if (*st) (void)hipStreamDestroy(*st), *st = nullptr;
    for (hipEvent_t* e : {&io_fork, &io_done, &h2d_done[0], &h2d_done[1], &comp_done[0], &comp_done[1],
                          &d2h_done[0], &d2h_done[1]})
      if (*e) (void)hipEventDestroy(*e), *e = nullptr;
    io_device = -1;
  }
  void drop_lanes() {
    for (hipStream_t l : lanes) (void)hipStreamDestroy(l);
    for (hipEvent_t e : lane_done) (void)hipEventDestroy(e);
    for (hipEvent_t e : lane_skew) (void)hipEventDestroy(e);
    lane_skew.clear();
    if (fork) (void)hipEventDestroy(fork);
    lanes.clear();
    lane_done.clear();
    fork = nullptr;
    lane_device = -1;
  }
  ~nr_plan() {
    for (auto& r : recorded) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    drop_lanes();
    drop_io();
  }
};

struct nr_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~nr_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

thread_local std::string g_err;

nr_status fail(nr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

nr_status hip_fail(hipError_t e, const char* where) {
  return fail(NR_HIP_ERROR, std::string(where) + ": " + hipGetErrorString(e));
}

nrk::KBArgs kb_args(const nr::Plan& p) {
  nrk::KBArgs kb;
  std::memset(&kb, 0, sizeof(kb));
  std::memcpy(kb.c, p.kb.coef.data(), p.kb.coef.size() * sizeof(float));
  return kb;
}

hipEvent_t take_event(nr_plan* plan) {
  if (!plan->pool.empty()) {
    hipEvent_t e = plan->pool.back();
    plan->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs `launch` (which enqueues one stage on `st`), bracketed by events when profiling.
template <class F>
hipError_t timed(nr_plan* plan, int stage, hipStream_t st, F&& launch) {
  if (!plan->profiling) return launch();
  hipEvent_t a = take_event(plan), b = take_event(plan);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, st);
  plan->recorded.push_back({stage, a, b});
  return e;
}

nr_status check_bound(const nr_plan* plan) {
  if (!plan) return fail(NR_INVALID_ARG, "plan is NULL");
  if (!plan->p.d_ws) return fail(NR_INVALID_ARG, "plan has no workspace bound (nr_plan_bind)");
  return NR_OK;
}

nr_status pending_error(const char* where) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, where);
  return NR_OK;
}

nr_status ensure_layout(nr_plan* plan) {
  std::string err;
  const nr_status st = nr::layout_plan(plan->p, err);
  return st == NR_OK ? NR_OK : fail(st, err);
}

int stage_event_id(nr::Stage s) {
  switch (s) {
    case nr::Stage::FwdRows: return kStageFwdRows;
    case nr::Stage::FwdCols: return kStageFwdCols;
    case nr::Stage::FwdInterp:
    case nr::Stage::FwdRadial: return kStageFwdInterp;
    case nr::Stage::AdjRadial: return kStageAdjRadial;
    case nr::Stage::SpreadZero: return kStageSpreadClear;
    case nr::Stage::Spread: return kStageSpread;
    case nr::Stage::AdjCols: return kStageAdjCols;
    case nr::Stage::AdjRows: return kStageAdjRows;
    default: return kStageCount;
  }
}

// The plan's lane streams on the current device (created on first use).
hipError_t ensure_lanes(nr_plan* plan, int n) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (plan->lane_device != dev) plan->drop_lanes();
  plan->lane_device = dev;
  if (!plan->fork && (e = hipEventCreateWithFlags(&plan->fork, hipEventDisableTiming)) != hipSuccess) return e;
  while (int(plan->lanes.size()) < n) {
    hipStream_t l = nullptr;
    hipEvent_t ev = nullptr;
    if ((e = hipStreamCreateWithFlags(&l, hipStreamNonBlocking)) != hipSuccess) return e;
    plan->lanes.push_back(l);
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    plan->lane_done.push_back(ev);
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    plan->lane_skew.push_back(ev);
  }
  return hipSuccess;
}

// Enqueue, for every batch, the forward chain (vol_in -> sino_out), then the
// residual sino_out -= b of its slices (b not null), then the adjoint chain
// (sino_in -> vol_out), as asked.  With several lanes the batches run
// round-robin on the lane streams, which first wait for the work already on
// st; st then waits for every lane.  Each batch's adjoint follows its own
// forward on its lane, with no join in between.
nr_status run_batches(nr_plan* plan, bool fwd, const float* b, bool adj, const float* vol_in, float* vol_out,
                      const float* sino_in, float* sino_out, hipStream_t st, const char* where,
                      const nr_fbp* fbp = nullptr) {
  const nr::Plan& p = plan->p;
  // while stages are being timed they run one at a time on st, so that each
  // event pair times its stage alone
  const int nl = plan->profiling ? 1 : p.n_lanes;
  if (nl > 1) {
    hipError_t e = ensure_lanes(plan, nl);
    if (e == hipSuccess) e = hipEventRecord(plan->fork, st);
    for (int l = 0; l < nl && e == hipSuccess; ++l) e = hipStreamWaitEvent(plan->lanes[size_t(l)], plan->fork, 0);
    if (e != hipSuccess) return hip_fail(e, where);
  }
  auto lane_stream = [&](const nr::Batch& bt) { return nl > 1 ? plan->lanes[size_t(bt.lane)] : st; };
  const nrk::KBArgs kb = kb_args(p);
  const char* base = static_cast<const char*>(p.d_ws);
  nrk::LaunchArgs a{};
  a.descs = reinterpret_cast<const SliceDesc*>(base + p.off_desc);
  a.halo = p.halo;
  a.colpad = p.colpad;
  a.vol_in = vol_in;
  a.vol_out = vol_out;
  a.sino_in = sino_in;
  a.sino_out = sino_out;
  a.fbp_filter = fbp ? fbp->filter : -1;
  a.fbp_order = fbp ? fbp->order : 0;
  a.fbp_inv_cutoff = fbp && fbp->filter == NR_FBP_BUTTERWORTH ? float(1.0 / fbp->cutoff) : 0.f;
  for (size_t bi = 0; bi < p.batches.size(); ++bi) {
    const nr::Batch& bt = p.batches[bi];
    hipStream_t bs = lane_stream(bt);
    std::vector<const nr::StageLaunch*> seq;
    if (fwd)
      for (const nr::StageLaunch& sl : bt.fwd) seq.push_back(&sl);
    if (fwd && b) seq.push_back(nullptr);   // the residual of the batch's slices
    if (adj)
      for (const nr::StageLaunch& sl : bt.adj) seq.push_back(&sl);
    // Lanes start skewed: lane l's first batch waits until lane l-1's first
    // batch has issued 1/nl of its stages, so concurrent lanes run different
    // kinds of stage (transforms, gathers, scatters) rather than the same one.
    const bool first = int(bi) < nl;
    const size_t skew_at = nl > 1 ? std::max<size_t>(1, seq.size() / size_t(nl)) : 0;
    if (nl > 1 && first && bt.lane > 0) {
      const hipError_t e = hipStreamWaitEvent(bs, plan->lane_skew[size_t(bt.lane - 1)], 0);
      if (e != hipSuccess) return hip_fail(e, where);
    }
    for (size_t si = 0; si < seq.size(); ++si) {
      if (nl > 1 && first && si == skew_at && bt.lane + 1 < nl) {
        const hipError_t e = hipEventRecord(plan->lane_skew[size_t(bt.lane)], bs);
        if (e != hipSuccess) return hip_fail(e, where);
      }
      const nr::StageLaunch* slp = seq[si];
      if (!slp) {
        hipError_t e = hipSuccess;
        for (int s : bt.slices) {
          const nr_slice& sl = p.slices[size_t(s)];
          const size_t off = size_t(sl.sino_off), cnt = size_t(sl.n_angles) * sl.n_det;
          e = timed(plan, kStageResidual, bs, [&] { return nrk::launch_residual(sino_out + off, b + off, cnt, bs); });
          if (e != hipSuccess) return hip_fail(e, where);
        }
        continue;
      }
      const nr::StageLaunch& sl = *slp;
      const bool spread = sl.stage == nr::Stage::Spread || sl.stage == nr::Stage::SpreadZero;
      hipError_t e = hipSuccess;
      if (spread && p.tune.spread_mode == 1) {
        // reference spreading, one slice at a time
        if (sl.stage == nr::Stage::SpreadZero) continue;
        for (int s : bt.slices) {
          e = timed(plan, kStageSpread, bs, [&] {
            return nrk::launch_spread_reference(a.descs, s, plan->host_descs[size_t(s)], p.halo, p.colpad, kb,
                                                p.kb.W, bs);
          });
          if (e != hipSuccess) break;
        }
      } else {
        nrk::LaunchArgs la = a;
        la.work = reinterpret_cast<const WorkItem*>(base + p.off_work + sl.work_off);
        la.n_work = sl.n_work;
        e = timed(plan, stage_event_id(sl.stage), bs, [&] {
          return nrk::launch_stage(static_cast<nrk::StageKind>(int(sl.stage)), sl.L, la, kb, p.kb.W,
                                   p.tune.tile_w, p.tune.tile_h, bs);
        });
      }
      if (e != hipSuccess) return hip_fail(e, where);
    }
  }
  if (nl > 1) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < nl && e == hipSuccess; ++l) {
      e = hipEventRecord(plan->lane_done[size_t(l)], plan->lanes[size_t(l)]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, plan->lane_done[size_t(l)], 0);
    }
    if (e != hipSuccess) return hip_fail(e, where);
  }
  return NR_OK;
}

hipError_t ensure_io(nr_plan* plan) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (plan->io_device == dev && plan->io_in) return hipSuccess;
  plan->drop_io();
  plan->io_device = dev;
  for (hipStream_t* st : {&plan->io_in, &plan->io_out})
    if ((e = hipStreamCreateWithFlags(st, hipStreamNonBlocking)) != hipSuccess) return e;
  for (hipEvent_t* ev : {&plan->io_fork, &plan->io_done, &plan->h2d_done[0], &plan->h2d_done[1],
                         &plan->comp_done[0], &plan->comp_done[1], &plan->d2h_done[0], &plan->d2h_done[1]})
    if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return e;
  return hipSuccess;
}

size_t vol_extent(const nr::Plan& p) {
  size_t n = 0;
  for (const nr_slice& sl : p.slices) n = std::max(n, size_t(sl.vol_off) + size_t(sl.n) * sl.n);
  return n;
}

size_t sino_extent(const nr::Plan& p) {
  size_t n = 0;
  for (const nr_slice& sl : p.slices) n = std::max(n, size_t(sl.sino_off) + size_t(sl.n_angles) * sl.n_det);
  return n;
}

nr_status check_prior(const nr_prior* prior) {
  if (!prior) return fail(NR_INVALID_ARG, "prior is NULL");
  if (!(prior->p >= 1.0f && prior->p <= 2.0f) || !(prior->sigma > 0.0f) || !(prior->c > 0.0f) ||
      !(prior->lambda >= 0.0f))
    return fail(NR_INVALID_ARG, "prior needs 1 <= p <= 2, sigma > 0, c > 0, lambda >= 0");
  return NR_OK;
}

nrk::PriorArgs prior_args(const nr_prior* p) {
  return nrk::PriorArgs{p->p, p->sigma, p->c, p->lambda, p->w_face, p->w_edge, p->w_corner};
}

// Runs `enqueue(stream)` under stream capture and instantiates the graph.
template <class F>
nr_status capture(nr_plan* plan, nr_graph** out, F&& enqueue) {
  if (!out) return fail(NR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (nr_status st = pending_error("before graph capture")) return st;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "graph capture stream");
  const bool prof = plan->profiling;
  plan->profiling = false;
  nr_graph* g = new (std::nothrow) nr_graph;
  nr_status status = g ? NR_OK : fail(NR_INTERNAL, "out of host memory");
  if (status == NR_OK) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      status = hip_fail(e, "hipStreamBeginCapture");
    } else {
      status = enqueue(static_cast<nr_stream>(cs));
      hipGraph_t graph = nullptr;
      const hipError_t e2 = hipStreamEndCapture(cs, &graph);
      g->graph = graph;
      if (status == NR_OK && e2 != hipSuccess) status = hip_fail(e2, "hipStreamEndCapture");
      if (status == NR_OK) {
        const hipError_t e3 = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e3 != hipSuccess) status = hip_fail(e3, "hipGraphInstantiate");
      }
    }
  }
  plan->profiling = prof;
  (void)hipStreamDestroy(cs);
  if (status != NR_OK) {
    delete g;
    return status;
  }
  *out = g;
  return NR_OK;
}

}  // namespace

extern "C" {

const char* nr_status_str(nr_status s) {
  switch (s) {
    case NR_OK: return "ok";
    case NR_INVALID_ARG: return "invalid argument";
    case NR_UNSUPPORTED_SIZE: return "unsupported size";
    case NR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case NR_HIP_ERROR: return "HIP error";
    case NR_NONFINITE: return "non-finite value";
    case NR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* nr_last_error(void) { return g_err.c_str(); }

const char* nr_version(void) { return "nufftradon 0.2 (gfx950)"; }

nr_status nr_plan_create(const nr_slice* slices, int32_t n_slices, const double* angles_host,
                         const nr_nufft* params, nr_plan** out) {
  if (!out) return fail(NR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nr_plan* p = new (std::nothrow) nr_plan;
  if (!p) return fail(NR_INTERNAL, "out of host memory");
  try {
    std::string err;
    nr_status st = nr::build_plan(slices, n_slices, angles_host, params, p->p, err);
    if (st == NR_OK) st = nr::layout_plan(p->p, err);
    if (st != NR_OK) {
      delete p;
      return fail(st, err);
    }
  } catch (const std::exception& e) {
    delete p;
    return fail(NR_INTERNAL, e.what());
  }
  *out = p;
  return NR_OK;
}

nr_status nr_plan_workspace_bytes(const nr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(NR_INVALID_ARG, "plan/bytes is NULL");
  if (nr_status st = ensure_layout(const_cast<nr_plan*>(plan))) return st;
  *bytes = plan->p.ws_bytes;
  return NR_OK;
}

nr_status nr_plan_bind(nr_plan* plan, void* d_ws, size_t bytes, nr_stream stream) {
  if (!plan || !d_ws) return fail(NR_INVALID_ARG, "plan/workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(NR_INVALID_ARG, "workspace not 256-byte aligned");
  if (nr_status st = ensure_layout(plan)) return st;
  nr::Plan& p = plan->p;
  if (bytes < p.ws_bytes)
    return fail(NR_WORKSPACE_TOO_SMALL, "workspace has " + std::to_string(bytes) + " bytes, plan needs " +
                                            std::to_string(p.ws_bytes));
  if (nr_status st = pending_error("before nr_plan_bind")) return st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(d_ws);
  plan->host_descs = nr::slice_descs(p, base);
  auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  for (auto& kv : p.deapod)
    if ((e = up(p.off_deapod.at(kv.first), kv.second.data(), kv.second.size() * sizeof(float)))) break;
  for (auto& kv : p.twiddle)
    if (!e && (e = up(p.off_twiddle.at(kv.first), kv.second.data(), kv.second.size() * sizeof(nr::f2)))) break;
  for (auto& kv : p.shift)
    if (!e && (e = up(p.off_shift.at(kv.first), kv.second.data(), kv.second.size() * sizeof(nr::f2)))) break;
  for (nr::Geom& g : p.geoms) {
    if (e) break;
    if ((e = up(g.off_gxy, g.gxy.data(), g.gxy.size() * sizeof(double)))) break;
    if ((e = up(g.off_flip, g.flip.data(), g.flip.size() * sizeof(int32_t)))) break;
    if ((e = up(g.off_pts, g.pts.data(), g.pts.size() * sizeof(int32_t)))) break;
    if ((e = up(g.off_items, g.items.data(), g.items.size() * sizeof(SpreadItem)))) break;
    if ((e = up(g.off_zero, g.zero_tiles.data(), g.zero_tiles.size() * sizeof(int32_t)))) break;
    if ((e = up(g.off_ipts, g.ipts.data(), g.ipts.size() * sizeof(int32_t)))) break;
    if ((e = up(g.off_iitems, g.iitems.data(), g.iitems.size() * sizeof(SpreadItem)))) break;
  }
  if (!e) e = up(p.off_desc, plan->host_descs.data(), plan->host_descs.size() * sizeof(SliceDesc));
  if (!e) e = up(p.off_work, p.work.data(), p.work.size() * sizeof(WorkItem));
  // the host tables are read by the copies: wait here so the caller may reuse
  // or destroy the plan freely afterwards
  if (!e) e = hipStreamSynchronize(st);
  if (e) return hip_fail(e, "nr_plan_bind upload");
  p.d_ws = d_ws;
  p.d_ws_bytes = bytes;
  return NR_OK;
}

nr_status nr_plan_destroy(nr_plan* plan) {
  delete plan;
  return NR_OK;
}

nr_status nr_plan_tune(nr_plan* plan, const char* key, int64_t value) {
  if (!plan || !key) return fail(NR_INVALID_ARG, "plan/key is NULL");
  nr::Tuning t = plan->p.tune;
  if (std::strcmp(key, "spread_mode") == 0) {
    if (value != 0 && value != 1) return fail(NR_INVALID_ARG, "spread_mode must be 0 (tiles) or 1 (atomics)");
    plan->p.tune.spread_mode = int(value);
    return NR_OK;   // no layout change
  } else if (std::strcmp(key, "tile_w") == 0) {
    t.tile_w = int(value);
  } else if (std::strcmp(key, "tile_h") == 0) {
    t.tile_h = int(value);
  } else if (std::strcmp(key, "chunk") == 0) {
    t.chunk = int(value);
  } else if (std::strcmp(key, "streams") == 0) {
    if (value < 1 || value > 8) return fail(NR_INVALID_ARG, "streams must be in [1, 8]");
    t.streams = int(value);
  } else if (std::strcmp(key, "interp_mode") == 0) {
    if (value != 0 && value != 1) return fail(NR_INVALID_ARG, "interp_mode must be 0 (tiles) or 1 (direct)");
    t.interp_mode = int(value);
  } else if (std::strcmp(key, "batch") == 0) {
    if (value < 0) return fail(NR_INVALID_ARG, "batch must be >= 0");
    t.batch = int(value);
  } else if (std::strcmp(key, "batch_mb") == 0) {
    if (value < 0 || value > (1 << 20)) return fail(NR_INVALID_ARG, "batch_mb must be in [0, 2^20]");
    t.batch_mb = int(value);
  } else {
    return fail(NR_INVALID_ARG, std::string("unknown tuning key ") + key);
  }
  // a new layout: the workspace must be queried and bound again
  plan->p.tune = t;
  plan->p.laid_out = false;
  plan->p.d_ws = nullptr;
  plan->p.d_ws_bytes = 0;
  return NR_OK;
}

nr_status nr_plan_profile(nr_plan* plan, int32_t enable) {
  if (!plan) return fail(NR_INVALID_ARG, "plan is NULL");
  plan->profiling = enable != 0;
  return NR_OK;
}

nr_status nr_plan_profile_read(nr_plan* plan, double* ms, int64_t* launches, int32_t n_stages) {
  if (!plan || !ms || !launches || n_stages < 0) return fail(NR_INVALID_ARG, "plan/ms/launches is NULL");
  for (int i = 0; i < n_stages; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  hipError_t err = hipSuccess;
  if (!plan->recorded.empty()) err = hipEventSynchronize(plan->recorded.back().stop);
  for (auto& r : plan->recorded) {
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, r.start, r.stop);
    if (r.stage < n_stages) {
      ms[r.stage] += t;
      launches[r.stage] += 1;
    }
    plan->pool.push_back(r.start);
    plan->pool.push_back(r.stop);
  }
  plan->recorded.clear();
  if (err != hipSuccess) return hip_fail(err, "nr_plan_profile_read");
  return NR_OK;
}

nr_status radon_fwd(nr_plan* plan, const float* d_vol, float* d_sino, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_vol || !d_sino) return fail(NR_INVALID_ARG, "d_vol/d_sino is NULL");
  if (nr_status st = pending_error("before radon_fwd")) return st;
  return run_batches(plan, true, nullptr, false, d_vol, nullptr, nullptr, d_sino, static_cast<hipStream_t>(stream),
                     "radon_fwd launch");
}

nr_status radon_adj(nr_plan* plan, const float* d_sino, float* d_vol, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_vol || !d_sino) return fail(NR_INVALID_ARG, "d_vol/d_sino is NULL");
  if (nr_status st = pending_error("before radon_adj")) return st;
  return run_batches(plan, false, nullptr, true, nullptr, d_vol, d_sino, nullptr, static_cast<hipStream_t>(stream),
                     "radon_adj launch");
}

nr_status radon_fbp(nr_plan* plan, const nr_fbp* filter, const float* d_sino, float* d_vol, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!filter || !d_vol || !d_sino) return fail(NR_INVALID_ARG, "radon_fbp: NULL argument");
  if (filter->filter != NR_FBP_RAMP && filter->filter != NR_FBP_BUTTERWORTH)
    return fail(NR_INVALID_ARG, "radon_fbp: filter must be NR_FBP_RAMP or NR_FBP_BUTTERWORTH");
  if (filter->filter == NR_FBP_BUTTERWORTH &&
      (!(filter->cutoff > 0.0 && filter->cutoff < 1e30) || filter->order < 1 || filter->order > 16))
    return fail(NR_INVALID_ARG, "radon_fbp: Butterworth needs a finite cutoff > 0 and 1 <= order <= 16");
  if (nr_status st = pending_error("before radon_fbp")) return st;
  return run_batches(plan, false, nullptr, true, nullptr, d_vol, d_sino, nullptr, static_cast<hipStream_t>(stream),
                     "radon_fbp launch", filter);
}

nr_status radon_stream(nr_plan* plan, int32_t what, const nr_fbp* filter, const float* h_in, float* h_out,
                       int64_t n_chunks, float* const* d_in, float* const* d_out, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (what != NR_STREAM_FWD && what != NR_STREAM_ADJ && what != NR_STREAM_FBP)
    return fail(NR_INVALID_ARG, "radon_stream: what must be NR_STREAM_FWD, NR_STREAM_ADJ or NR_STREAM_FBP");
  if (n_chunks < 0) return fail(NR_INVALID_ARG, "radon_stream: n_chunks < 0");
  if (n_chunks == 0) return NR_OK;
  if (!h_in || !h_out || !d_in || !d_out || !d_in[0] || !d_in[1] || !d_out[0] || !d_out[1])
    return fail(NR_INVALID_ARG, "radon_stream: NULL argument");
  const float* bufs[4] = {d_in[0], d_in[1], d_out[0], d_out[1]};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (bufs[i] == bufs[j]) return fail(NR_INVALID_ARG, "radon_stream: the four device buffers must be distinct");
  if (what == NR_STREAM_FBP) {
    if (!filter) return fail(NR_INVALID_ARG, "radon_stream: NR_STREAM_FBP needs a filter");
    if (filter->filter != NR_FBP_RAMP && filter->filter != NR_FBP_BUTTERWORTH)
      return fail(NR_INVALID_ARG, "radon_stream: filter must be NR_FBP_RAMP or NR_FBP_BUTTERWORTH");
    if (filter->filter == NR_FBP_BUTTERWORTH &&
        (!(filter->cutoff > 0.0 && filter->cutoff < 1e30) || filter->order < 1 || filter->order > 16))
      return fail(NR_INVALID_ARG, "radon_stream: Butterworth needs a finite cutoff > 0 and 1 <= order <= 16");
  }
  if (nr_status st = pending_error("before radon_stream")) return st;
  const nr::Plan& p = plan->p;
  const bool fwd = what == NR_STREAM_FWD;
  const size_t n_in = fwd ? vol_extent(p) : sino_extent(p), n_out = fwd ? sino_extent(p) : vol_extent(p);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = ensure_io(plan);
  // the copy streams start after the work already on the caller's stream
  if (e == hipSuccess) e = hipEventRecord(plan->io_fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(plan->io_in, plan->io_fork, 0);
  if (e == hipSuccess) e = hipStreamWaitEvent(plan->io_out, plan->io_fork, 0);
  if (e != hipSuccess) return hip_fail(e, "radon_stream set-up");
  for (int64_t i = 0; i < n_chunks; ++i) {
    const int b = int(i & 1);
    // copy in: buffer b is free once the computation of chunk i-2 is done
    if (i >= 2) e = hipStreamWaitEvent(plan->io_in, plan->comp_done[b], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d_in[b], h_in + size_t(i) * n_in, n_in * sizeof(float), hipMemcpyHostToDevice,
                         plan->io_in);
    if (e == hipSuccess) e = hipEventRecord(plan->h2d_done[b], plan->io_in);
    // compute: after its input arrived and chunk i-2's output left d_out[b]
    if (e == hipSuccess) e = hipStreamWaitEvent(st, plan->h2d_done[b], 0);
    if (e == hipSuccess && i >= 2) e = hipStreamWaitEvent(st, plan->d2h_done[b], 0);
    if (e != hipSuccess) return hip_fail(e, "radon_stream copy in");
    nr_status s = fwd ? run_batches(plan, true, nullptr, false, d_in[b], nullptr, nullptr, d_out[b], st,
                                    "radon_stream launch")
                      : run_batches(plan, false, nullptr, true, nullptr, d_out[b], d_in[b], nullptr, st,
                                    "radon_stream launch", what == NR_STREAM_FBP ? filter : nullptr);
    if (s != NR_OK) return s;
    e = hipEventRecord(plan->comp_done[b], st);
    // copy out
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->io_out, plan->comp_done[b], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_out + size_t(i) * n_out, d_out[b], n_out * sizeof(float), hipMemcpyDeviceToHost,
                         plan->io_out);
    if (e == hipSuccess) e = hipEventRecord(plan->d2h_done[b], plan->io_out);
    if (e != hipSuccess) return hip_fail(e, "radon_stream copy out");
  }
  // the caller's stream waits for the last copy back (and so for every copy)
  e = hipEventRecord(plan->io_done, plan->io_out);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, plan->io_done, 0);
  if (e != hipSuccess) return hip_fail(e, "radon_stream join");
  return NR_OK;
}

nr_status radon_normal(nr_plan* plan, const float* d_vol, const float* d_b, float* d_sino, float* d_vol_out,
                       nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_vol || !d_sino || !d_vol_out) return fail(NR_INVALID_ARG, "radon_normal: NULL argument");
  if (nr_status st = pending_error("before radon_normal")) return st;
  return run_batches(plan, true, d_b, true, d_vol, d_vol_out, d_sino, d_sino, static_cast<hipStream_t>(stream),
                     "radon_normal launch");
}

nr_status radon_residual(nr_plan* plan, const float* d_vol, const float* d_b, float* d_r, double* d_value,
                         nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_vol || !d_b || !d_r) return fail(NR_INVALID_ARG, "radon_residual: NULL argument");
  const size_t sino_total = sino_extent(plan->p);
  if (nr_status s = radon_fwd(plan, d_vol, d_r, stream)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = timed(plan, kStageResidual, st, [&] {
    return d_value ? nrk::launch_residual_norm(d_r, d_b, sino_total, d_value, st)
                   : nrk::launch_residual(d_r, d_b, sino_total, st);
  });
  if (e != hipSuccess) return hip_fail(e, "radon_residual launch");
  return NR_OK;
}

nr_status qggmrf_grad(const float* d_vol, int32_t nz, int32_t n, const nr_prior* prior, float scale,
                      float* d_grad_accum, double* d_value, nr_stream stream) {
  if (!d_vol || !d_grad_accum) return fail(NR_INVALID_ARG, "d_vol/d_grad_accum is NULL");
  if (nz < 1 || n < 1) return fail(NR_INVALID_ARG, "nz and n must be >= 1");
  if (nr_status st = check_prior(prior)) return st;
  if (nr_status st = pending_error("before qggmrf_grad")) return st;
  const hipError_t e = nrk::launch_qggmrf(d_vol, d_grad_accum, d_value, nz, n, prior_args(prior), scale,
                                          static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "qggmrf_grad launch");
  return NR_OK;
}

nr_status mbir_step(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, const float* d_b, float* d_x,
                    float* d_x_prev, float* d_y, float* d_grad, float* d_scratch, double* d_state,
                    nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!params || !d_b || !d_x || !d_x_prev || !d_y || !d_grad || !d_scratch || !d_state)
    return fail(NR_INVALID_ARG, "mbir_step: NULL argument");
  if (nr_status st = check_prior(prior)) return st;
  if (!(params->inv_L > 0.0f)) return fail(NR_INVALID_ARG, "inv_L must be > 0");
  const nr::Plan& p = plan->p;
  const int n = p.slices[0].n;
  const int nz = int(p.slices.size());
  for (int z = 0; z < nz; ++z) {
    const nr_slice& sl = p.slices[size_t(z)];
    if (sl.n != n || sl.vol_off != int64_t(z) * n * n)
      return fail(NR_INVALID_ARG, "mbir_step: slices must share N and sit at vol_off = z*N*N");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  // R^T (R y - b) into d_grad, batch by batch
  if (nr_status s = radon_normal(plan, d_y, d_b, d_scratch, d_grad, stream)) return s;
  hipError_t e = hipSuccess;
  if (prior->lambda > 0.0f) {
    const nrk::PriorArgs pa = prior_args(prior);
    e = timed(plan, kStagePrior, st, [&] { return nrk::launch_qggmrf(d_y, d_grad, nullptr, nz, n, pa, 1.0f, st); });
    if (e != hipSuccess) return hip_fail(e, "mbir_step prior");
  }
  e = timed(plan, kStageUpdate, st, [&] {
    return nrk::launch_mbir_update(d_x, d_x_prev, d_y, d_grad, size_t(nz) * n * n, params->inv_L, params->nonneg,
                                   d_state, st);
  });
  if (e != hipSuccess) return hip_fail(e, "mbir_step update");
  return NR_OK;
}

nr_status mbir_update(const nr_mbir* params, float* d_x, float* d_x_prev, float* d_y, const float* d_grad,
                      int64_t count, double* d_state, nr_stream stream) {
  if (!params || !d_x || !d_x_prev || !d_y || !d_grad || !d_state)
    return fail(NR_INVALID_ARG, "mbir_update: NULL argument");
  if (count < 1) return fail(NR_INVALID_ARG, "mbir_update: count must be >= 1");
  if (!(params->inv_L > 0.0f)) return fail(NR_INVALID_ARG, "inv_L must be > 0");
  if (nr_status st = pending_error("before mbir_update")) return st;
  const hipError_t e = nrk::launch_mbir_update(d_x, d_x_prev, d_y, d_grad, size_t(count), params->inv_L,
                                               params->nonneg, d_state, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mbir_update launch");
  return NR_OK;
}

nr_status nr_graph_capture_radon(nr_plan* plan, int32_t what, const float* d_vol_in, float* d_sino,
                                 float* d_vol_out, nr_graph** out) {
  if (nr_status st = check_bound(plan)) return st;
  if (what < 1 || what > 3) return fail(NR_INVALID_ARG, "what must be 1 (fwd), 2 (adj) or 3 (fwd then adj)");
  if (!d_sino || ((what & 1) && !d_vol_in) || ((what & 2) && !d_vol_out))
    return fail(NR_INVALID_ARG, "nr_graph_capture_radon: NULL buffer");
  return capture(plan, out, [&](nr_stream s) -> nr_status {
    if (what == 3) return radon_normal(plan, d_vol_in, nullptr, d_sino, d_vol_out, s);
    if (what & 1)
      if (nr_status st = radon_fwd(plan, d_vol_in, d_sino, s)) return st;
    if (what & 2)
      if (nr_status st = radon_adj(plan, d_sino, d_vol_out, s)) return st;
    return NR_OK;
  });
}

nr_status nr_graph_capture_mbir(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, const float* d_b,
                                float* d_x, float* d_x_prev, float* d_y, float* d_grad, float* d_scratch,
                                double* d_state, int32_t iters, nr_graph** out) {
  if (nr_status st = check_bound(plan)) return st;
  if (iters < 1) return fail(NR_INVALID_ARG, "iters must be >= 1");
  return capture(plan, out, [&](nr_stream s) -> nr_status {
    for (int k = 0; k < iters; ++k)
      if (nr_status st = mbir_step(plan, prior, params, d_b, d_x, d_x_prev, d_y, d_grad, d_scratch, d_state, s))
        return st;
    return NR_OK;
  });
}

nr_status nr_graph_launch(nr_graph* graph, nr_stream stream) {
  if (!graph || !graph->exec) return fail(NR_INVALID_ARG, "graph is NULL");
  if (nr_status st = pending_error("before nr_graph_launch")) return st;
  const hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return NR_OK;
}

nr_status nr_graph_destroy(nr_graph* graph) {
  delete graph;
  return NR_OK;
}

nr_status nr_kb_eval(int32_t width, double beta, int32_t count, const double* u, const double* xi,
                     double* phi, double* phihat, double* phi_poly) {
  if (width < 6 || width > 8 || count < 0) return fail(NR_INVALID_ARG, "width must be 6..8, count >= 0");
  nr::KaiserBessel kb;
  kb.init(width, beta);
  for (int i = 0; i < count; ++i) {
    if (u && phi) phi[i] = kb.phi(u[i]);
    if (u && phi_poly) phi_poly[i] = kb.phi_poly(u[i]);
    if (xi && phihat) phihat[i] = kb.phihat(xi[i]);
  }
  return NR_OK;
}

nr_status nr_plan_info(const nr_plan* plan, int32_t index, int64_t* info, int32_t count) {
  if (!plan || !info) return fail(NR_INVALID_ARG, "plan/info is NULL");
  if (nr_status st = ensure_layout(const_cast<nr_plan*>(plan))) return st;
  const nr::Plan& p = plan->p;
  if (index < 0 || index >= int(p.slices.size())) return fail(NR_INVALID_ARG, "slice index out of range");
  const nr::Geom& g = p.geoms[size_t(p.slice_geom[size_t(index)])];
  int64_t launches = 0;
  for (const nr::Batch& bt : p.batches) launches += int64_t(bt.fwd.size() + bt.adj.size());
  const int64_t v[8] = {g.G, int64_t(g.tiles_x) * g.tiles_y, int64_t(g.pts.size()), int64_t(g.items.size()),
                        p.kb.D, p.n_slots, int64_t(p.batches.size()), launches};
  for (int i = 0; i < count && i < 8; ++i) info[i] = v[i];
  return NR_OK;
}

}  // extern "C"
