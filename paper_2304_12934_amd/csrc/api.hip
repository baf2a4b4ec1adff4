// C ABI of libnufftradon (declared in include/nufftradon.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <cstring>
#include <mutex>
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

// Every plan state that kernel arguments depend on (a layout, a bound
// workspace) gets a fresh generation number, unique across plans.
static std::atomic<uint64_t> g_generation{1};
static uint64_t next_generation() { return g_generation.fetch_add(1); }

struct nr_plan {
  nr::Plan p;
  uint64_t gen = next_generation();   // changes on every re-layout and re-bind
  bool profiling = false;
  double tune_best_ms = -1.0;            // last nr_autotune: best pass time
  int tune_trials = 0;
  std::vector<StageEvents> recorded;
  std::vector<hipEvent_t> pool;
  std::vector<SliceDesc> host_descs;
  // concurrent lanes: streams (default priority, non-blocking) plus the
  // events that fork them from and join them back to the caller's stream
  int lane_device = -1;
  int persist_blocks = 0;   // resident workgroups of the persistent kernel (0: not queried yet)
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_done;
  std::vector<hipEvent_t> lane_skew;
  hipEvent_t fork = nullptr;
  // MBIR: the prior gradient runs on its own stream beside the projector
  int side_device = -1;
  hipStream_t side = nullptr;
  hipEvent_t side_fork = nullptr, side_done = nullptr;
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
  void drop_side() {
    if (side) (void)hipStreamDestroy(side), side = nullptr;
    for (hipEvent_t* e : {&side_fork, &side_done})
      if (*e) (void)hipEventDestroy(*e), *e = nullptr;
    side_device = -1;
  }
  ~nr_plan() {
    for (auto& r : recorded) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    drop_lanes();
    drop_io();
    drop_side();
  }
};

struct nr_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const nr_plan* plan = nullptr;   // the captured plan and its generation at capture
  uint64_t gen = 0;
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

// The plan's prior stream on the current device (created on first use).
hipError_t ensure_side(nr_plan* plan) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (plan->side_device == dev && plan->side) return hipSuccess;
  plan->drop_side();
  plan->side_device = dev;
  if ((e = hipStreamCreateWithFlags(&plan->side, hipStreamNonBlocking)) != hipSuccess) return e;
  for (hipEvent_t* ev : {&plan->side_fork, &plan->side_done})
    if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return e;
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
  // a forward + adjoint pass of a plan tuned persistent: each batch is one
  // persistent launch (after a clear of its counters) on its lane
  const bool persist = p.tune.persistent && fwd && adj && !plan->profiling && p.tune.spread_mode == 0;
  if (persist && plan->persist_blocks <= 0) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, where);
    const int per_cu = nrk::persist_blocks_per_cu(p.kb.W);
    // at least one workgroup per XCD queue; a multiple of the queue count
    plan->persist_blocks = std::max(kPersistQueues, per_cu * cus / kPersistQueues * kPersistQueues);
  }
  for (size_t bi = 0; persist && bi < p.batches.size(); ++bi) {
    const nr::Batch& bt = p.batches[bi];
    char* wsb = static_cast<char*>(p.d_ws);
    const int32_t* tab = reinterpret_cast<const int32_t*>(wsb + p.off_ptables) + bt.pt_off;
    int32_t* sync = reinterpret_cast<int32_t*>(wsb + p.off_psync);
    const int n = int(bt.slices.size());
    nrk::PersistArgs pa{};
    pa.entries = reinterpret_cast<const PersistEntry*>(wsb + p.off_pentries) + bt.pe_first;
    pa.qoff = tab;
    pa.need = tab + kPersistQueues + 1;
    pa.dep = pa.need + size_t(n) * kPersistStages;
    pa.tickets = sync + bt.ps_off;
    pa.done = pa.tickets + kPersistQueues;
    pa.error = sync;
    pa.first_slice = bt.slices.front();
    pa.spin_limit = 1 << 18;   // about a second of polling: far beyond any unit's duration
    nrk::LaunchArgs la = a;
    la.sino_sub = b;
    const hipError_t e = nrk::launch_persistent(la, pa, kb, p.kb.W, plan->persist_blocks, pa.tickets,
                                                kPersistQueues + n * kPersistStages, lane_stream(bt));
    if (e != hipSuccess) return hip_fail(e, where);
  }
  for (size_t bi = 0; !persist && bi < p.batches.size(); ++bi) {
    const nr::Batch& bt = p.batches[bi];
    hipStream_t bs = lane_stream(bt);
    std::vector<const nr::StageLaunch*> seq;
    if (fwd)
      for (const nr::StageLaunch& sl : bt.fwd) seq.push_back(&sl);
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
      const nr::StageLaunch& sl = *seq[si];
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
        la.stream_stores = bt.bytes > nr::kLastLevelCacheBytes ? 1 : 0;
        // the stage that writes the sinogram rows subtracts b as it stores them
        if (sl.stage == nr::Stage::FwdRadial || (sl.stage == nr::Stage::FwdInterp && sl.L > 0)) la.sino_sub = b;
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

nr_status check_mbir(const nr_mbir* m) {
  if (!(m->inv_L > 0.0f) || !std::isfinite(m->inv_L)) return fail(NR_INVALID_ARG, "inv_L must be finite and > 0");
  if ((m->restart != 0 && m->restart != 1) || (m->nonneg != 0 && m->nonneg != 1) ||
      (m->monotone != 0 && m->monotone != 1))
    return fail(NR_INVALID_ARG, "restart, nonneg and monotone must be 0 or 1");
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
  g->plan = plan;
  g->gen = plan->gen;
  *out = g;
  return NR_OK;
}

// Copies the plan's tables, the slice descriptors `descs` (pointing into the
// workspace at base) and the work lists into that workspace on st.  The host
// sources must stay alive until the copies have run.
hipError_t upload_tables(const nr::Plan& p, char* base, const std::vector<SliceDesc>& descs, hipStream_t st) {
  auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  for (auto& kv : p.deapod)
    if ((e = up(p.off_deapod.at(kv.first), kv.second.data(), kv.second.size() * sizeof(float)))) return e;
  for (auto& kv : p.twiddle)
    if ((e = up(p.off_twiddle.at(kv.first), kv.second.data(), kv.second.size() * sizeof(nr::f2)))) return e;
  for (auto& kv : p.shift)
    if ((e = up(p.off_shift.at(kv.first), kv.second.data(), kv.second.size() * sizeof(nr::f2)))) return e;
  for (const nr::Geom& g : p.geoms) {
    if ((e = up(g.off_gxy, g.gxy.data(), g.gxy.size() * sizeof(double)))) return e;
    if ((e = up(g.off_flip, g.flip.data(), g.flip.size() * sizeof(int32_t)))) return e;
    if ((e = up(g.off_pts, g.pts.data(), g.pts.size() * sizeof(int32_t)))) return e;
    if ((e = up(g.off_items, g.items.data(), g.items.size() * sizeof(SpreadItem)))) return e;
    if ((e = up(g.off_zero, g.zero_tiles.data(), g.zero_tiles.size() * sizeof(int32_t)))) return e;
    if ((e = up(g.off_ipts, g.ipts.data(), g.ipts.size() * sizeof(int32_t)))) return e;
    if ((e = up(g.off_iitems, g.iitems.data(), g.iitems.size() * sizeof(SpreadItem)))) return e;
  }
  if ((e = up(p.off_desc, descs.data(), descs.size() * sizeof(SliceDesc)))) return e;
  if ((e = up(p.off_pentries, p.pentries.data(), p.pentries.size() * sizeof(PersistEntry)))) return e;
  if ((e = up(p.off_ptables, p.ptables.data(), p.ptables.size() * sizeof(int32_t)))) return e;
  return up(p.off_work, p.work.data(), p.work.size() * sizeof(WorkItem));
}


// ---------------------------------------------------------------------------
// autotuner cache: a JSON object of objects, {"<key>": {"tile_w": 64, ...}}
// ---------------------------------------------------------------------------

using CacheEntry = std::vector<std::pair<std::string, double>>;
using Cache = std::vector<std::pair<std::string, CacheEntry>>;

struct JsonIn {
  const std::string& t;
  size_t i = 0;
  void ws() {
    while (i < t.size() && std::isspace(static_cast<unsigned char>(t[i]))) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    if (!eat('"')) return false;
    out.clear();
    while (i < t.size() && t[i] != '"') {
      if (t[i] == '\\' && i + 1 < t.size()) ++i;
      out.push_back(t[i++]);
    }
    return eat('"');
  }
  bool num(double& v) {
    ws();
    const char* b = t.c_str() + i;
    char* e = nullptr;
    v = std::strtod(b, &e);
    if (e == b) return false;
    i += size_t(e - b);
    return true;
  }
};

// Parses the cache file's text; false (and an empty cache) when it is not of that form.
bool parse_cache(const std::string& text, Cache& out) {
  out.clear();
  JsonIn in{text};
  if (!in.eat('{')) return false;
  if (in.eat('}')) return true;
  do {
    std::string key;
    CacheEntry e;
    if (!in.str(key) || !in.eat(':') || !in.eat('{')) return out.clear(), false;
    if (!in.eat('}')) {
      do {
        std::string name;
        double v = 0.0;
        if (!in.str(name) || !in.eat(':') || !in.num(v)) return out.clear(), false;
        e.emplace_back(name, v);
      } while (in.eat(','));
      if (!in.eat('}')) return out.clear(), false;
    }
    out.emplace_back(key, e);
  } while (in.eat(','));
  return in.eat('}') || (out.clear(), false);
}

std::string format_cache(const Cache& c) {
  std::string s = "{\n";
  for (size_t k = 0; k < c.size(); ++k) {
    s += " \"" + c[k].first + "\": {";
    for (size_t j = 0; j < c[k].second.size(); ++j) {
      char buf[64];
      std::snprintf(buf, sizeof(buf), "%.17g", c[k].second[j].second);
      s += (j ? ", \"" : "\"") + c[k].second[j].first + "\": " + buf;
    }
    s += k + 1 < c.size() ? "},\n" : "}\n";
  }
  return s + "}\n";
}

// FNV-1a over the bytes of the plan's geometry and kernel parameters and the
// device's name: the cache key of a tuning.
std::string geometry_key(const nr::Plan& p, const std::string& device) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* data, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(data);
    for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 1099511628211ull;
  };
  mix(device.data(), device.size());
  mix(&p.kb.W, sizeof(p.kb.W));
  mix(&p.kb.beta, sizeof(p.kb.beta));
  for (const nr_slice& sl : p.slices) {
    const int32_t v[3] = {sl.n, sl.n_det, sl.n_angles};
    mix(v, sizeof(v));
    mix(&sl.center, sizeof(sl.center));
    mix(p.angles.data() + sl.angle_off, size_t(sl.n_angles) * sizeof(double));
  }
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%016llx", static_cast<unsigned long long>(h));
  return buf;
}

const char* const kTuneKeys[] = {"tile_w", "tile_h", "chunk", "batch_mb", "streams"};

int64_t tune_value(const nr::Tuning& t, const std::string& k) {
  if (k == "tile_w") return t.tile_w;
  if (k == "tile_h") return t.tile_h;
  if (k == "chunk") return t.chunk;
  if (k == "batch_mb") return t.batch_mb;
  if (k == "streams") return t.streams;
  if (k == "batch") return t.batch;
  if (k == "interp_mode") return t.interp_mode;
  if (k == "spread_mode") return t.spread_mode;
  if (k == "persistent") return t.persistent;
  return INT64_MIN;
}

void set_tune_value(nr::Tuning& t, const std::string& k, int64_t v) {
  if (k == "tile_w") t.tile_w = int(v);
  else if (k == "tile_h") t.tile_h = int(v);
  else if (k == "chunk") t.chunk = int(v);
  else if (k == "batch_mb") t.batch_mb = int(v);
  else if (k == "streams") t.streams = int(v);
}

// The autotuner's search space: the batch budget, the number of streams,
// the spreading tile and the spreading/interpolation item size.
const int kTuneBudgets[] = {1, 160, 640, 1400, 2048};
const int kTuneStreams[] = {1, 2, 3, 6};
const int kTuneTiles[][2] = {{64, 32}, {32, 32}, {64, 64}, {128, 32}};
const int kTuneChunks[] = {256, 512, 1024};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Buffers of one timed pass in the autotuner's scratch: volume, back-projection, sinogram.
size_t tune_buffer_bytes(const nr::Plan& p) {
  return 2 * align256(vol_extent(p) * sizeof(float)) + align256(sino_extent(p) * sizeof(float));
}

// Workspace bytes of the plan under tuning t (lays the plan out for it).
nr_status layout_bytes(nr_plan* plan, const nr::Tuning& t, size_t& bytes) {
  plan->p.tune = t;
  plan->p.laid_out = false;
  std::string err;
  const nr_status st = nr::layout_plan(plan->p, err);
  if (st != NR_OK) return fail(st, err);
  bytes = plan->p.ws_bytes;
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
  plan->host_descs = nr::slice_descs(p, static_cast<char*>(d_ws));
  hipError_t e = upload_tables(p, static_cast<char*>(d_ws), plan->host_descs, st);
  if (!e) e = nrk::launch_fill_int(reinterpret_cast<int*>(static_cast<char*>(d_ws) + p.off_psync), p.psync_ints, 0, st);
  // the host tables are read by the copies: wait here so the caller may reuse
  // or destroy the plan freely afterwards
  if (!e) e = hipStreamSynchronize(st);
  if (e) return hip_fail(e, "nr_plan_bind upload");
  p.d_ws = d_ws;
  p.d_ws_bytes = bytes;
  plan->gen = next_generation();
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
  } else if (std::strcmp(key, "persistent") == 0) {
    if (value != 0 && value != 1) return fail(NR_INVALID_ARG, "persistent must be 0 or 1");
    t.persistent = int(value);
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
  plan->gen = next_generation();
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
  // copy in chunk i into buffer i & 1, which is free once the computation of
  // chunk i - 2 is done
  auto copy_in = [&](int64_t i) {
    const int b = int(i & 1);
    hipError_t ce = i >= 2 ? hipStreamWaitEvent(plan->io_in, plan->comp_done[b], 0) : hipSuccess;
    if (ce == hipSuccess)
      ce = hipMemcpyAsync(d_in[b], h_in + size_t(i) * n_in, n_in * sizeof(float), hipMemcpyHostToDevice,
                          plan->io_in);
    if (ce == hipSuccess) ce = hipEventRecord(plan->h2d_done[b], plan->io_in);
    return ce;
  };
  e = copy_in(0);
  if (e != hipSuccess) return hip_fail(e, "radon_stream copy in");
  for (int64_t i = 0; i < n_chunks; ++i) {
    const int b = int(i & 1);
    // the next chunk's copy is enqueued before this chunk's computation and
    // copy out: enqueueing a copy that waits on another stream's event can
    // hold the host until that event completes, and the copy in of chunk
    // i + 1 must not be enqueued only after the computation of chunk i
    if (i + 1 < n_chunks) e = copy_in(i + 1);
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
  if (nr_status st = pending_error("before radon_residual")) return st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the forward's radial stage stores R f - b
  if (nr_status s = run_batches(plan, true, d_b, false, d_vol, nullptr, nullptr, d_r, st, "radon_residual launch"))
    return s;
  if (d_value) {
    const size_t sino_total = sino_extent(plan->p);
    const hipError_t e = timed(plan, kStageResidual, st, [&] {
      return nrk::launch_half_sum_squares(d_r, sino_total, d_value, st);
    });
    if (e != hipSuccess) return hip_fail(e, "radon_residual norm");
  }
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
  if (nr_status st = check_mbir(params)) return st;
  const nr::Plan& p = plan->p;
  const int n = p.slices[0].n;
  const int nz = int(p.slices.size());
  for (int z = 0; z < nz; ++z) {
    const nr_slice& sl = p.slices[size_t(z)];
    if (sl.n != n || sl.vol_off != int64_t(z) * n * n)
      return fail(NR_INVALID_ARG, "mbir_step: slices must share N and sit at vol_off = z*N*N");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t count = size_t(nz) * n * n;
  const nrk::PriorArgs pa = prior_args(prior);
  hipError_t e = hipSuccess;
  if (!params->monotone) {
    // The prior gradient (arithmetic-bound) runs beside the projector
    // (memory-bound) on the plan's prior stream, into d_x_prev: the update
    // overwrites d_x_prev without reading it, and adds it to d_grad first.
    // While stages are timed, it runs on st before the projector instead.
    const bool prior_on = prior->lambda > 0.0f;
    const bool side = prior_on && !plan->profiling;
    if (side) {
      e = ensure_side(plan);
      if (e == hipSuccess) e = hipEventRecord(plan->side_fork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(plan->side, plan->side_fork, 0);
      if (e == hipSuccess) e = nrk::launch_qggmrf(d_y, d_x_prev, nullptr, nz, n, pa, 1.0f, plan->side, false);
      if (e == hipSuccess) e = hipEventRecord(plan->side_done, plan->side);
      if (e != hipSuccess) return hip_fail(e, "mbir_step prior");
    } else if (prior_on) {
      e = timed(plan, kStagePrior, st, [&] {
        return nrk::launch_qggmrf(d_y, d_x_prev, nullptr, nz, n, pa, 1.0f, st, false);
      });
      if (e != hipSuccess) return hip_fail(e, "mbir_step prior");
    }
    // R^T (R y - b) into d_grad, batch by batch
    if (nr_status s = radon_normal(plan, d_y, d_b, d_scratch, d_grad, stream)) return s;
    if (side && (e = hipStreamWaitEvent(st, plan->side_done, 0)) != hipSuccess) return hip_fail(e, "mbir_step join");
    e = timed(plan, kStageUpdate, st, [&] {
      return nrk::launch_mbir_update(d_x, d_x_prev, d_y, d_grad, count, params->inv_L, params->nonneg,
                                     params->restart, d_state, st, prior_on);
    });
    if (e != hipSuccess) return hip_fail(e, "mbir_step update");
    return NR_OK;
  }
  // R^T (R y - b) into d_grad, batch by batch
  if (nr_status s = radon_normal(plan, d_y, d_b, d_scratch, d_grad, stream)) return s;
  if (prior->lambda > 0.0f) {
    e = timed(plan, kStagePrior, st, [&] { return nrk::launch_qggmrf(d_y, d_grad, nullptr, nz, n, pa, 1.0f, st); });
    if (e != hipSuccess) return hip_fail(e, "mbir_step prior");
  }
  // monotone: the candidate x' (into d_x_prev) and its objective
  e = timed(plan, kStageUpdate, st, [&] {
    return nrk::launch_mbir_candidate(d_x, d_x_prev, d_y, d_grad, count, params->inv_L, params->nonneg, d_state,
                                      st);
  });
  if (e != hipSuccess) return hip_fail(e, "mbir_step candidate");
  if (nr_status s = radon_residual(plan, d_x_prev, d_b, d_scratch, d_state + nrk::kStPhiData, stream)) return s;
  e = timed(plan, kStagePrior, st, [&] {
    return prior->lambda > 0.0f
               ? nrk::launch_qggmrf(d_x_prev, nullptr, d_state + nrk::kStPhiPrior, nz, n, pa, 1.0f, st)
               : nrk::launch_set_double(d_state + nrk::kStPhiPrior, 0.0, st);
  });
  if (e != hipSuccess) return hip_fail(e, "mbir_step candidate prior");
  e = timed(plan, kStageUpdate, st, [&] {
    return nrk::launch_mbir_finish_monotone(d_x, d_x_prev, d_y, count, params->restart, d_state, st);
  });
  if (e != hipSuccess) return hip_fail(e, "mbir_step monotone update");
  return NR_OK;
}

// ---------------------------------------------------------------------------
// mbir_step without a caller scratch buffer: the residual sinogram lives in a
// file-scope device array, one copy per device, reserved for the life of the
// process.  Its device address comes from hipGetSymbolAddress with the device
// current (the array's name is only a host-side stand-in in host code).
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kNoAllocScratchBytes = NR_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) float scratch[kNoAllocScratchBytes / sizeof(float)];

std::mutex g_scratch_mutex;
std::vector<float*> g_scratch_ptr;   // per device, filled on first use

nr_status scratch_for_current_device(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "mbir_step_noalloc: hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[size_t(dev)]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                 "mbir_step_noalloc: hipGetSymbolAddress(scratch)");
    g_scratch_ptr[size_t(dev)] = static_cast<float*>(ptr);
  }
  *out = g_scratch_ptr[size_t(dev)];
  return NR_OK;
}

}  // namespace

nr_status mbir_step_noalloc(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, const float* d_b,
                            float* d_x, float* d_x_prev, float* d_y, float* d_grad, double* d_state,
                            nr_stream stream) {
  if (!plan) return fail(NR_INVALID_ARG, "plan is NULL");
  const size_t need = sino_extent(plan->p) * sizeof(float);
  if (need > kNoAllocScratchBytes)
    return fail(NR_INVALID_ARG, "mbir_step_noalloc: the plan's sinogram (" + std::to_string(need) +
                                    " bytes) exceeds the library's scratch of " +
                                    std::to_string(kNoAllocScratchBytes) + " bytes; use mbir_step");
  if (nr_status st = check_bound(plan)) return st;
  float* d_scratch = nullptr;
  if (nr_status st = scratch_for_current_device(&d_scratch)) return st;
  // every value of the scratch is written (R y - b) before it is read
  return mbir_step(plan, prior, params, d_b, d_x, d_x_prev, d_y, d_grad, d_scratch, d_state, stream);
}

namespace {

// Device work area of mbir_stream_iterate for a plan of nz uniform slices:
// two input sets (x_k and x_{k-1} with one halo slice each side, and the
// chunk's data), then y and the prior's gradient over the halo-extended
// chunk, the data-term gradient, the residual and two output chunks.
struct StreamMbirLayout {
  size_t ext, vol, sino;                    // float counts
  size_t xk[2], xp[2], b[2], y, gp, g, r, out[2], bytes;   // byte offsets, total
};

nr_status stream_mbir_layout(const nr::Plan& p, StreamMbirLayout& L) {
  if (p.slices.empty()) return fail(NR_INVALID_ARG, "mbir_stream: empty plan");
  const nr_slice& s0 = p.slices[0];
  const int64_t n = s0.n, per_sino = int64_t(s0.n_angles) * s0.n_det;
  for (size_t z = 0; z < p.slices.size(); ++z) {
    const nr_slice& sl = p.slices[z];
    if (sl.n != s0.n || sl.n_angles != s0.n_angles || sl.n_det != s0.n_det || sl.vol_off != int64_t(z) * n * n ||
        sl.sino_off != int64_t(z) * per_sino)
      return fail(NR_INVALID_ARG,
                  "mbir_stream: the plan's slices must share N, angles and bins and sit at vol_off = z*N*N, "
                  "sino_off = z*n_angles*n_det");
  }
  const size_t nz = p.slices.size();
  L.vol = nz * size_t(n) * size_t(n);
  L.ext = (nz + 2) * size_t(n) * size_t(n);
  L.sino = nz * size_t(per_sino);
  size_t off = 0;
  auto take = [&](size_t floats) {
    const size_t o = off;
    off = align256(off + floats * sizeof(float));
    return o;
  };
  for (int k = 0; k < 2; ++k) {
    L.xk[k] = take(L.ext);
    L.xp[k] = take(L.ext);
    L.b[k] = take(L.sino);
  }
  L.y = take(L.ext);
  L.gp = take(L.ext);
  L.g = take(L.vol);
  L.r = take(L.sino);
  L.out[0] = take(L.vol);
  L.out[1] = take(L.vol);
  L.bytes = off;
  return NR_OK;
}

}  // namespace

nr_status mbir_stream_work_bytes(const nr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(NR_INVALID_ARG, "mbir_stream_work_bytes: NULL argument");
  StreamMbirLayout L{};
  if (nr_status st = stream_mbir_layout(plan->p, L)) return st;
  *bytes = L.bytes;
  return NR_OK;
}

nr_status mbir_stream_iterate(nr_plan* plan, const nr_prior* prior, const nr_mbir* params, int64_t n_chunks,
                              const float* h_b, const float* h_x, const float* h_x_prev, float* h_x_next,
                              void* d_work, size_t work_bytes, double* d_state, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!params || !h_b || !h_x || !h_x_prev || !h_x_next || !d_work || !d_state)
    return fail(NR_INVALID_ARG, "mbir_stream_iterate: NULL argument");
  if (n_chunks < 1) return fail(NR_INVALID_ARG, "mbir_stream_iterate: n_chunks < 1");
  if (nr_status st = check_prior(prior)) return st;
  if (nr_status st = check_mbir(params)) return st;
  if (params->monotone) return fail(NR_INVALID_ARG, "mbir_stream_iterate: the monotone step is not supported");
  if (h_x_next == h_x || h_x_next == h_x_prev)
    return fail(NR_INVALID_ARG, "mbir_stream_iterate: h_x_next must not alias h_x or h_x_prev");
  const nr::Plan& p = plan->p;
  StreamMbirLayout L{};
  if (nr_status st = stream_mbir_layout(p, L)) return st;
  if (work_bytes < L.bytes) return fail(NR_WORKSPACE_TOO_SMALL, "mbir_stream_iterate: work area too small");
  if (nr_status st = pending_error("before mbir_stream_iterate")) return st;
  const int n = p.slices[0].n;
  const size_t slice = size_t(n) * size_t(n);
  const int64_t nz = int64_t(p.slices.size()), Z = nz * n_chunks;
  char* w = static_cast<char*>(d_work);
  auto F = [&](size_t off) { return reinterpret_cast<float*>(w + off); };
  hipStream_t st = static_cast<hipStream_t>(stream);
  const nrk::PriorArgs pa = prior_args(prior);
  const bool prior_on = prior->lambda > 0.0f;
  hipError_t e = ensure_io(plan);
  // the step's dot product accumulates over the chunks from zero
  if (e == hipSuccess) e = nrk::launch_set_double(d_state + nrk::kStDot, 0.0, st);
  if (e == hipSuccess) e = hipEventRecord(plan->io_fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(plan->io_in, plan->io_fork, 0);
  if (e == hipSuccess) e = hipStreamWaitEvent(plan->io_out, plan->io_fork, 0);
  if (e != hipSuccess) return hip_fail(e, "mbir_stream_iterate set-up");
  // chunk c holds slices [c nz, (c+1) nz); its input buffers hold slices
  // [c nz - 1, (c+1) nz + 1) clipped to the volume, slice c nz - 1 at index 0
  auto lo = [&](int64_t c) { return std::max<int64_t>(c * nz - 1, 0); };
  auto hi = [&](int64_t c) { return std::min<int64_t>((c + 1) * nz + 1, Z); };
  auto copy_in = [&](int64_t c) {
    const int k = int(c & 1);
    const int64_t z0 = lo(c), z1 = hi(c);
    const size_t first = size_t(z0 - (c * nz - 1)) * slice, count = size_t(z1 - z0) * slice;
    hipError_t ce = c >= 2 ? hipStreamWaitEvent(plan->io_in, plan->comp_done[k], 0) : hipSuccess;
    if (ce == hipSuccess)
      ce = hipMemcpyAsync(F(L.xk[k]) + first, h_x + size_t(z0) * slice, count * sizeof(float),
                          hipMemcpyHostToDevice, plan->io_in);
    if (ce == hipSuccess)
      ce = hipMemcpyAsync(F(L.xp[k]) + first, h_x_prev + size_t(z0) * slice, count * sizeof(float),
                          hipMemcpyHostToDevice, plan->io_in);
    if (ce == hipSuccess)
      ce = hipMemcpyAsync(F(L.b[k]), h_b + size_t(c) * L.sino, L.sino * sizeof(float), hipMemcpyHostToDevice,
                          plan->io_in);
    if (ce == hipSuccess) ce = hipEventRecord(plan->h2d_done[k], plan->io_in);
    return ce;
  };
  e = copy_in(0);
  if (e != hipSuccess) return hip_fail(e, "mbir_stream_iterate copy in");
  for (int64_t c = 0; c < n_chunks; ++c) {
    const int k = int(c & 1);
    // the next chunk's copy in goes ahead of this chunk's work (see radon_stream)
    if (c + 1 < n_chunks) e = copy_in(c + 1);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, plan->h2d_done[k], 0);
    // output buffer k is free once chunk c - 2 has been copied out
    if (e == hipSuccess && c >= 2) e = hipStreamWaitEvent(st, plan->d2h_done[k], 0);
    if (e != hipSuccess) return hip_fail(e, "mbir_stream_iterate copy in");
    const int64_t z0 = lo(c), z1 = hi(c);
    const size_t first = size_t(z0 - (c * nz - 1)) * slice, count = size_t(z1 - z0) * slice;
    // y = x_k + beta (x_k - x_{k-1}) over the chunk and its halo slices
    e = nrk::launch_mbir_extrapolate(F(L.y) + first, F(L.xk[k]) + first, F(L.xp[k]) + first, count, d_state, st);
    // the prior's gradient over the extended chunk (its halo slices' own
    // values are wrong, missing their outer neighbours, and unused)
    if (e == hipSuccess && prior_on)
      e = nrk::launch_qggmrf(F(L.y) + first, F(L.gp) + first, nullptr, int(z1 - z0), n, pa, 1.0f, st, false);
    if (e != hipSuccess) return hip_fail(e, "mbir_stream_iterate prior");
    // R^T (R y - b) over the chunk's own slices
    if (nr_status s = radon_normal(plan, F(L.y) + slice, F(L.b[k]), F(L.r), F(L.g), stream)) return s;
    // x_{k+1} = y - g/L and the restart test's dot product
    e = nrk::launch_mbir_dot_accumulate(F(L.xk[k]) + slice, F(L.y) + slice, F(L.g),
                                        prior_on ? F(L.gp) + slice : nullptr, L.vol, params->inv_L, params->nonneg,
                                        d_state, F(L.out[k]), st);
    if (e == hipSuccess) e = hipEventRecord(plan->comp_done[k], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(plan->io_out, plan->comp_done[k], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_x_next + size_t(c) * L.vol, F(L.out[k]), L.vol * sizeof(float), hipMemcpyDeviceToHost,
                         plan->io_out);
    if (e == hipSuccess) e = hipEventRecord(plan->d2h_done[k], plan->io_out);
    if (e != hipSuccess) return hip_fail(e, "mbir_stream_iterate chunk");
  }
  // restart test and momentum for the next step, then the caller's stream
  // waits for the last copy out
  e = nrk::launch_mbir_finalize(d_state, params->restart, st);
  if (e == hipSuccess) e = hipEventRecord(plan->io_done, plan->io_out);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, plan->io_done, 0);
  if (e != hipSuccess) return hip_fail(e, "mbir_stream_iterate join");
  return NR_OK;
}

nr_status mbir_update(const nr_mbir* params, float* d_x, float* d_x_prev, float* d_y, const float* d_grad,
                      int64_t count, double* d_state, nr_stream stream) {
  if (!params || !d_x || !d_x_prev || !d_y || !d_grad || !d_state)
    return fail(NR_INVALID_ARG, "mbir_update: NULL argument");
  if (count < 1) return fail(NR_INVALID_ARG, "mbir_update: count must be >= 1");
  if (nr_status st = check_mbir(params)) return st;
  if (params->monotone)
    return fail(NR_INVALID_ARG, "mbir_update: the monotone step needs the objective (use mbir_step)");
  if (nr_status st = pending_error("before mbir_update")) return st;
  const hipError_t e = nrk::launch_mbir_update(d_x, d_x_prev, d_y, const_cast<float*>(d_grad), size_t(count),
                                               params->inv_L,
                                               params->nonneg, params->restart, d_state,
                                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mbir_update launch");
  return NR_OK;
}

nr_status mbir_state_init(double* d_state, nr_stream stream) {
  if (!d_state) return fail(NR_INVALID_ARG, "mbir_state_init: NULL state");
  if (nr_status st = pending_error("before mbir_state_init")) return st;
  const hipError_t e = nrk::launch_mbir_state_init(d_state, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mbir_state_init launch");
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
  // the kernels' arguments hold the workspace and layout of the capture
  if (graph->plan && graph->plan->gen != graph->gen)
    return fail(NR_INVALID_ARG, "nr_graph_launch: the plan was re-tuned or re-bound since the capture");
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

// ---------------------------------------------------------------------------
// set-up arithmetic of the MBIR step (Sec. 3)
// ---------------------------------------------------------------------------

nr_status nr_prior_init(nr_prior* out, float p, float sigma, float c, float lambda, int32_t weights) {
  if (!out) return fail(NR_INVALID_ARG, "nr_prior_init: out is NULL");
  double w[4] = {0.0, 0.0, 0.0, 0.0};   // by squared distance 1, 2, 3
  for (int d2 = 1; d2 <= 3; ++d2) {
    if (weights == NR_WEIGHTS_INV_DISTANCE) w[d2] = 1.0 / std::sqrt(double(d2));
    else if (weights == NR_WEIGHTS_GAUSSIAN) w[d2] = std::exp(-0.5 * d2);
    else return fail(NR_INVALID_ARG, "nr_prior_init: weights must be NR_WEIGHTS_INV_DISTANCE or NR_WEIGHTS_GAUSSIAN");
  }
  const double total = 6.0 * w[1] + 12.0 * w[2] + 8.0 * w[3];   // 6 faces, 12 edges, 8 corners
  *out = nr_prior{p, sigma, c, lambda, float(w[1] / total), float(w[2] / total), float(w[3] / total)};
  return check_prior(out);
}

nr_status nr_prior_lipschitz(const nr_prior* prior, double* out) {
  if (!out) return fail(NR_INVALID_ARG, "nr_prior_lipschitz: out is NULL");
  if (nr_status st = check_prior(prior)) return st;
  // Hessian row m of H: diagonal (2 lambda/sigma^2) sum_n w_mn rho''(.), off-diagonal
  // -(2 lambda/sigma^2) w_mn rho''(.), with 0 <= rho'' <= rho''(0) = 2/c (Gershgorin)
  const double wsum = 6.0 * prior->w_face + 12.0 * prior->w_edge + 8.0 * prior->w_corner;
  *out = 8.0 * double(prior->lambda) * wsum / (double(prior->c) * double(prior->sigma) * double(prior->sigma));
  return NR_OK;
}

nr_status nr_mbir_params(double lipschitz_data, const nr_prior* prior, int32_t restart, int32_t nonneg,
                         int32_t monotone, nr_mbir* out) {
  if (!out) return fail(NR_INVALID_ARG, "nr_mbir_params: out is NULL");
  if (!(lipschitz_data >= 0.0) || !std::isfinite(lipschitz_data))
    return fail(NR_INVALID_ARG, "nr_mbir_params: the data term's Lipschitz constant must be finite and >= 0");
  double lh = 0.0;
  if (prior)
    if (nr_status st = nr_prior_lipschitz(prior, &lh)) return st;
  const double L = lipschitz_data + lh;
  if (!(L > 0.0)) return fail(NR_INVALID_ARG, "nr_mbir_params: L = L_R + L_H must be > 0");
  *out = nr_mbir{float(1.0 / L), restart, nonneg, monotone};
  return check_mbir(out);
}

nr_status nr_power_lipschitz(nr_plan* plan, int32_t iters, uint64_t seed, double safety, float* d_v, float* d_w,
                             float* d_sino, double* d_work, double* h_out, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_v || !d_w || !d_sino || !d_work || !h_out) return fail(NR_INVALID_ARG, "nr_power_lipschitz: NULL argument");
  if (d_v == d_w) return fail(NR_INVALID_ARG, "nr_power_lipschitz: d_v and d_w must differ");
  if (iters < 1 || !(safety >= 1.0) || !std::isfinite(safety))
    return fail(NR_INVALID_ARG, "nr_power_lipschitz: iters >= 1 and finite safety >= 1");
  if (nr_status st = pending_error("before nr_power_lipschitz")) return st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const nr::Plan& p = plan->p;
  const size_t ext = vol_extent(p);
  // v: seeded uniform values on every slice, zero between slices; w starts at
  // zero so that cells outside the slices stay zero
  hipError_t e = nrk::launch_fill_value(d_v, ext, 0.f, st);
  if (e == hipSuccess) e = nrk::launch_fill_value(d_w, ext, 0.f, st);
  for (const nr_slice& sl : p.slices)
    if (e == hipSuccess)
      e = nrk::launch_fill_random(d_v + sl.vol_off, size_t(sl.n) * sl.n, seed, uint64_t(sl.vol_off), st);
  if (e == hipSuccess) e = nrk::launch_normalize(d_v, d_v, ext, d_work, st);
  if (e != hipSuccess) return hip_fail(e, "nr_power_lipschitz start");
  for (int k = 0; k < iters; ++k) {
    // w = R^T R v, then v = w / ||w||, ||w||^2 left in d_work
    if (nr_status s = radon_normal(plan, d_v, nullptr, d_sino, d_w, stream)) return s;
    e = nrk::launch_normalize(d_v, d_w, ext, d_work, st);
    if (e != hipSuccess) return hip_fail(e, "nr_power_lipschitz step");
  }
  double ss = 0.0;
  e = hipMemcpyAsync(&ss, d_work, sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "nr_power_lipschitz read-back");
  if (!std::isfinite(ss)) return fail(NR_NONFINITE, "nr_power_lipschitz: non-finite norm");
  *h_out = safety * std::sqrt(ss);
  return NR_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

nr_status nr_plan_get_tune(const nr_plan* plan, const char* key, int64_t* value) {
  if (!plan || !key || !value) return fail(NR_INVALID_ARG, "nr_plan_get_tune: NULL argument");
  const std::string k = key;
  if (k == "autotune_us") {
    *value = plan->tune_best_ms < 0.0 ? -1 : int64_t(std::llround(plan->tune_best_ms * 1e3));
    return NR_OK;
  }
  if (k == "autotune_trials") {
    *value = plan->tune_trials;
    return NR_OK;
  }
  const int64_t v = tune_value(plan->p.tune, k);
  if (v == INT64_MIN) return fail(NR_INVALID_ARG, "nr_plan_get_tune: unknown key " + k);
  *value = v;
  return NR_OK;
}

nr_status nr_autotune_scratch_bytes(nr_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(NR_INVALID_ARG, "nr_autotune_scratch_bytes: NULL argument");
  const nr::Tuning keep = plan->p.tune;
  const bool was_laid_out = plan->p.laid_out;
  size_t most = 0, tables = 0, b = 0;
  nr_status st = NR_OK;
  // the slot areas of every batch budget and stream count at the current tile
  for (int mb : kTuneBudgets)
    for (int ns : kTuneStreams) {
      nr::Tuning t = keep;
      t.batch_mb = mb;
      t.streams = ns;
      if ((st = layout_bytes(plan, t, b)) != NR_OK) break;
      most = std::max(most, b);
    }
  // and the tables of every tile shape at the smallest item size
  for (const auto& tw : kTuneTiles) {
    if (st != NR_OK) break;
    nr::Tuning t = keep;
    t.tile_w = tw[0];
    t.tile_h = tw[1];
    t.chunk = kTuneChunks[0];
    if ((st = layout_bytes(plan, t, b)) != NR_OK) break;
    tables = std::max(tables, plan->p.off_slot);
  }
  plan->p.tune = keep;
  plan->p.laid_out = false;
  std::string err;
  if (was_laid_out || st == NR_OK) (void)nr::layout_plan(plan->p, err);
  if (st != NR_OK) return st;
  *bytes = tune_buffer_bytes(plan->p) + most + tables + (size_t(1) << 20);
  return NR_OK;
}

nr_status nr_autotune(nr_plan* plan, void* d_scratch, size_t bytes, const char* cache_json, nr_stream stream) {
  if (!plan || !d_scratch) return fail(NR_INVALID_ARG, "nr_autotune: plan/scratch is NULL");
  if (reinterpret_cast<uintptr_t>(d_scratch) % 256 != 0) return fail(NR_INVALID_ARG, "nr_autotune: scratch not 256-byte aligned");
  if (nr_status st = pending_error("before nr_autotune")) return st;
  // the plan is unbound from here on (its workspace may already be released)
  plan->p.d_ws = nullptr;
  plan->p.d_ws_bytes = 0;
  plan->gen = next_generation();
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipDeviceProp_t prop;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return hip_fail(e, "nr_autotune device");
  nr::Plan& p = plan->p;
  const std::string key = geometry_key(p, std::string(prop.name) + "/" + prop.gcnArchName);
  // a cached tuning for this geometry and device: apply it, no timing
  Cache cache;
  if (cache_json) {
    std::ifstream f(cache_json);
    if (f) {
      std::stringstream ss;
      ss << f.rdbuf();
      (void)parse_cache(ss.str(), cache);
    }
    for (const auto& kv : cache)
      if (kv.first == key) {
        nr::Tuning t = p.tune;
        double ms = -1.0;
        for (const auto& f2 : kv.second) {
          if (f2.first == "ms") ms = f2.second;
          else set_tune_value(t, f2.first, int64_t(f2.second));
        }
        size_t b = 0;
        if (nr_status s = layout_bytes(plan, t, b)) return s;
        p.d_ws = nullptr;
        p.d_ws_bytes = 0;
        plan->gen = next_generation();
        plan->tune_best_ms = ms;
        plan->tune_trials = 0;
        return NR_OK;
      }
  }
  // buffers of the timed passes, then the candidate's workspace
  const size_t nv = vol_extent(p), ns = sino_extent(p);
  char* base = static_cast<char*>(d_scratch);
  float* vol = reinterpret_cast<float*>(base);
  float* back = reinterpret_cast<float*>(base + align256(nv * sizeof(float)));
  float* sino = reinterpret_cast<float*>(base + 2 * align256(nv * sizeof(float)));
  const size_t used = tune_buffer_bytes(p);
  if (bytes < used + 256) return fail(NR_WORKSPACE_TOO_SMALL, "nr_autotune: scratch smaller than one pass's buffers");
  char* ws = base + used;
  const size_t ws_room = bytes - used;
  e = nrk::launch_fill_random(vol, nv, 0x5eedull, 0, st);
  if (e != hipSuccess) return hip_fail(e, "nr_autotune fill");
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(e, "nr_autotune events");
  }
  const bool prof = plan->profiling;
  plan->profiling = false;
  const int reps = 3;
  int trials = 0;
  // one forward + adjoint pass per repetition under tuning t; +inf when the
  // workspace does not fit the scratch
  auto time_of = [&](const nr::Tuning& t, double& ms) -> nr_status {
    ms = HUGE_VAL;
    size_t need = 0;
    if (nr_status s = layout_bytes(plan, t, need)) return s;
    if (need > ws_room) return NR_OK;
    if (nr_status s = nr_plan_bind(plan, ws, ws_room, stream)) return s;
    if (nr_status s = radon_normal(plan, vol, nullptr, sino, back, stream)) return s;   // warm-up
    hipError_t he = hipEventRecord(t0, st);
    for (int r = 0; r < reps && he == hipSuccess; ++r)
      if (nr_status s = radon_normal(plan, vol, nullptr, sino, back, stream)) return s;
    if (he == hipSuccess) he = hipEventRecord(t1, st);
    if (he == hipSuccess) he = hipEventSynchronize(t1);
    float el = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&el, t0, t1);
    if (he != hipSuccess) return hip_fail(he, "nr_autotune timing");
    ms = double(el) / reps;
    ++trials;
    return NR_OK;
  };
  // coordinate search from the plan's current setting, one parameter at a time
  nr::Tuning best = p.tune;
  double best_ms = HUGE_VAL;
  nr_status status = time_of(best, best_ms);
  auto consider = [&](nr::Tuning t) {
    double ms = HUGE_VAL;
    if (status == NR_OK) status = time_of(t, ms);
    if (status == NR_OK && ms < best_ms) best = t, best_ms = ms;
  };
  for (int mb : kTuneBudgets)
    if (mb != best.batch_mb) { nr::Tuning t = best; t.batch_mb = mb; consider(t); }
  for (int n : kTuneStreams)
    if (n != best.streams) { nr::Tuning t = best; t.streams = n; consider(t); }
  for (const auto& tw : kTuneTiles)
    if (tw[0] != best.tile_w || tw[1] != best.tile_h) { nr::Tuning t = best; t.tile_w = tw[0]; t.tile_h = tw[1]; consider(t); }
  for (int c : kTuneChunks)
    if (c != best.chunk) { nr::Tuning t = best; t.chunk = c; consider(t); }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  plan->profiling = prof;
  // the plan keeps the best setting, unbound (the scratch was the caller's)
  size_t b = 0;
  if (status == NR_OK) status = layout_bytes(plan, best, b);
  p.d_ws = nullptr;
  p.d_ws_bytes = 0;
  plan->gen = next_generation();
  if (status != NR_OK) return status;
  if (!(best_ms < HUGE_VAL)) return fail(NR_WORKSPACE_TOO_SMALL, "nr_autotune: no candidate fits the scratch");
  plan->tune_best_ms = best_ms;
  plan->tune_trials = trials;
  if (cache_json) {
    CacheEntry entry;
    for (const char* k : kTuneKeys) entry.emplace_back(k, double(tune_value(best, k)));
    entry.emplace_back("ms", best_ms);
    bool found = false;
    for (auto& kv : cache)
      if (kv.first == key) kv.second = entry, found = true;
    if (!found) cache.emplace_back(key, entry);
    const std::string tmp = std::string(cache_json) + ".tmp";
    {
      std::ofstream f(tmp, std::ios::trunc);
      if (!f) return fail(NR_INVALID_ARG, std::string("nr_autotune: cannot write ") + tmp);
      f << format_cache(cache);
    }
    if (std::rename(tmp.c_str(), cache_json) != 0)
      return fail(NR_INVALID_ARG, std::string("nr_autotune: cannot replace ") + cache_json);
  }
  return NR_OK;
}

nr_status nr_plan_check(nr_plan* plan, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t flag = 0;
  int32_t* d_flag = reinterpret_cast<int32_t*>(static_cast<char*>(plan->p.d_ws) + plan->p.off_psync);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(&flag, d_flag, sizeof(flag), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "nr_plan_check");
  if (flag != 0) {
    e = nrk::launch_fill_int(d_flag, 1, 0, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "nr_plan_check reset");
    return fail(NR_INTERNAL, "a persistent launch gave up waiting for a stage (its results are invalid)");
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
  for (const nr::Batch& bt : p.batches)
    launches += p.tune.persistent ? 2 : int64_t(bt.fwd.size() + bt.adj.size());   // clear + persistent kernel
  const int64_t v[8] = {g.G, int64_t(g.tiles_x) * g.tiles_y, int64_t(g.pts.size()), int64_t(g.items.size()),
                        p.kb.D, p.n_slots, int64_t(p.batches.size()), launches};
  for (int i = 0; i < count && i < 8; ++i) info[i] = v[i];
  return NR_OK;
}

}  // extern "C"
