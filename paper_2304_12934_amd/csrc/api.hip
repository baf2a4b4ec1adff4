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
enum { kStageResidual = int(nrk::Stage::Count), kStagePrior, kStageUpdate, kStageCount };

struct StageEvents {
  int stage;
  hipEvent_t start, stop;
};

struct nr_plan {
  nr::Plan p;
  int spread_mode = 0;   // 0: LDS tiles, 1: global atomics (reference)
  bool profiling = false;
  std::vector<StageEvents> recorded;
  std::vector<hipEvent_t> pool;
  ~nr_plan() {
    for (auto& r : recorded) {
      hipEventDestroy(r.start);
      hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : pool) hipEventDestroy(e);
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

template <class T>
const T* ws_ptr(const nr::Plan& p, size_t off) {
  return reinterpret_cast<const T*>(static_cast<const char*>(p.d_ws) + off);
}
template <class T>
T* ws_mut(const nr::Plan& p, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(p.d_ws) + off);
}

nrk::KBArgs kb_args(const nr::Plan& p) {
  nrk::KBArgs kb;
  std::memset(&kb, 0, sizeof(kb));
  std::memcpy(kb.c, p.kb.coef.data(), p.kb.coef.size() * sizeof(float));
  return kb;
}

nrk::SliceArgs slice_args(const nr::Plan& p, int s) {
  const nr_slice& sl = p.slices[size_t(s)];
  const nr::Geom& g = p.geoms[size_t(p.slice_geom[size_t(s)])];
  nrk::SliceArgs a;
  std::memset(&a, 0, sizeof(a));
  a.N = sl.n;
  a.Nt = sl.n_det;
  a.na = sl.n_angles;
  a.G = g.G;
  a.H = g.H;
  a.rows = g.rows;
  a.cols = g.cols;
  a.halo = p.halo;
  a.colpad = p.colpad;
  a.deapod = ws_ptr<float>(p, p.off_deapod.at(sl.n));
  a.tw_G = ws_ptr<float2>(p, p.off_twiddle.at(g.G));
  a.tw_Nt = ws_ptr<float2>(p, p.off_twiddle.at(sl.n_det));
  a.gxy = ws_ptr<double>(p, g.off_gxy);
  a.flip = ws_ptr<int>(p, g.off_flip);
  a.T = ws_mut<float2>(p, p.off_slot + p.slot_t);
  a.ext = ws_mut<float2>(p, p.off_slot + p.slot_ext);
  a.yh = ws_mut<float2>(p, p.off_slot + p.slot_yh);
  a.pts = ws_ptr<int>(p, g.off_pts);
  a.items = ws_ptr<SpreadItem>(p, g.off_items);
  a.zero_tiles = ws_ptr<int>(p, g.off_zero);
  a.n_items = int(g.items.size());
  a.n_zero = int(g.zero_tiles.size());
  a.tile_w = g.tile_w;
  a.tile_h = g.tile_h;
  a.tiles_x = g.tiles_x;
  return a;
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

const char* nr_version(void) { return "nufftradon 0.1 (gfx950)"; }

nr_status nr_plan_create(const nr_slice* slices, int32_t n_slices, const double* angles_host,
                         const nr_nufft* params, nr_plan** out) {
  if (!out) return fail(NR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nr_plan* p = new (std::nothrow) nr_plan;
  if (!p) return fail(NR_INTERNAL, "out of host memory");
  try {
    std::string err;
    const nr_status st = nr::build_plan(slices, n_slices, angles_host, params, p->p, err);
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
  *bytes = plan->p.ws_bytes;
  return NR_OK;
}

nr_status nr_plan_bind(nr_plan* plan, void* d_ws, size_t bytes, nr_stream stream) {
  if (!plan || !d_ws) return fail(NR_INVALID_ARG, "plan/workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) return fail(NR_INVALID_ARG, "workspace not 256-byte aligned");
  nr::Plan& p = plan->p;
  if (bytes < p.ws_bytes)
    return fail(NR_WORKSPACE_TOO_SMALL, "workspace has " + std::to_string(bytes) + " bytes, plan needs " +
                                            std::to_string(p.ws_bytes));
  if (nr_status st = pending_error("before nr_plan_bind")) return st;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(d_ws);
  auto up = [&](size_t off, const void* src, size_t n) -> hipError_t {
    if (n == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  for (auto& kv : p.deapod)
    if ((e = up(p.off_deapod.at(kv.first), kv.second.data(), kv.second.size() * sizeof(float)))) break;
  for (auto& kv : p.twiddle)
    if (!e && (e = up(p.off_twiddle.at(kv.first), kv.second.data(), kv.second.size() * sizeof(nr::f2)))) break;
  for (nr::Geom& g : p.geoms) {
    if (e) break;
    if ((e = up(g.off_gxy, g.gxy.data(), g.gxy.size() * sizeof(double)))) break;
    if ((e = up(g.off_flip, g.flip.data(), g.flip.size() * sizeof(int32_t)))) break;
    if ((e = up(g.off_pts, g.pts.data(), g.pts.size() * sizeof(int32_t)))) break;
    if ((e = up(g.off_items, g.items.data(), g.items.size() * sizeof(SpreadItem)))) break;
    if ((e = up(g.off_zero, g.zero_tiles.data(), g.zero_tiles.size() * sizeof(int32_t)))) break;
  }
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
  if (std::strcmp(key, "spread_mode") == 0) {
    if (value != 0 && value != 1) return fail(NR_INVALID_ARG, "spread_mode must be 0 (tiles) or 1 (atomics)");
    plan->spread_mode = int(value);
    return NR_OK;
  }
  return fail(NR_INVALID_ARG, std::string("unknown tuning key ") + key);
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
  const nr::Plan& p = plan->p;
  const nrk::KBArgs kb = kb_args(p);
  for (int s = 0; s < int(p.slices.size()); ++s) {
    nrk::SliceArgs a = slice_args(p, s);
    a.vol_in = d_vol + p.slices[size_t(s)].vol_off;
    a.sino_out = d_sino + p.slices[size_t(s)].sino_off;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    for (nrk::Stage stage : {nrk::Stage::FwdRows, nrk::Stage::FwdCols, nrk::Stage::FwdInterp}) {
      const hipError_t e = timed(plan, int(stage), st, [&] {
        return nrk::launch_stage(stage, a, kb, p.kb.W, plan->spread_mode, st);
      });
      if (e != hipSuccess) return hip_fail(e, "radon_fwd launch");
    }
  }
  return NR_OK;
}

nr_status radon_adj(nr_plan* plan, const float* d_sino, float* d_vol, nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_vol || !d_sino) return fail(NR_INVALID_ARG, "d_vol/d_sino is NULL");
  if (nr_status st = pending_error("before radon_adj")) return st;
  const nr::Plan& p = plan->p;
  const nrk::KBArgs kb = kb_args(p);
  for (int s = 0; s < int(p.slices.size()); ++s) {
    nrk::SliceArgs a = slice_args(p, s);
    a.sino_in = d_sino + p.slices[size_t(s)].sino_off;
    a.vol_out = d_vol + p.slices[size_t(s)].vol_off;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    for (nrk::Stage stage : {nrk::Stage::AdjRadial, nrk::Stage::Spread, nrk::Stage::AdjCols, nrk::Stage::AdjRows}) {
      const hipError_t e = timed(plan, int(stage), st, [&] {
        return nrk::launch_stage(stage, a, kb, p.kb.W, plan->spread_mode, st);
      });
      if (e != hipSuccess) return hip_fail(e, "radon_adj launch");
    }
  }
  return NR_OK;
}

static nr_status check_prior(const nr_prior* prior) {
  if (!prior) return fail(NR_INVALID_ARG, "prior is NULL");
  if (!(prior->p >= 1.0f && prior->p <= 2.0f) || !(prior->sigma > 0.0f) || !(prior->c > 0.0f) ||
      !(prior->lambda >= 0.0f))
    return fail(NR_INVALID_ARG, "prior needs 1 <= p <= 2, sigma > 0, c > 0, lambda >= 0");
  return NR_OK;
}

static nrk::PriorArgs prior_args(const nr_prior* p) {
  return nrk::PriorArgs{p->p, p->sigma, p->c, p->lambda, p->w_face, p->w_edge, p->w_corner};
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
  size_t sino_total = 0;
  for (int z = 0; z < nz; ++z) {
    const nr_slice& sl = p.slices[size_t(z)];
    if (sl.n != n || sl.vol_off != int64_t(z) * n * n)
      return fail(NR_INVALID_ARG, "mbir_step: slices must share N and sit at vol_off = z*N*N");
    sino_total = std::max(sino_total, size_t(sl.sino_off) + size_t(sl.n_angles) * sl.n_det);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (nr_status s = radon_fwd(plan, d_y, d_scratch, stream)) return s;
  hipError_t e = timed(plan, kStageResidual, st, [&] { return nrk::launch_residual(d_scratch, d_b, sino_total, st); });
  if (e != hipSuccess) return hip_fail(e, "mbir_step residual");
  if (nr_status s = radon_adj(plan, d_scratch, d_grad, stream)) return s;
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

nr_status radon_residual(nr_plan* plan, const float* d_vol, const float* d_b, float* d_r, double* d_value,
                         nr_stream stream) {
  if (nr_status st = check_bound(plan)) return st;
  if (!d_vol || !d_b || !d_r) return fail(NR_INVALID_ARG, "radon_residual: NULL argument");
  const nr::Plan& p = plan->p;
  size_t sino_total = 0;
  for (const nr_slice& sl : p.slices)
    sino_total = std::max(sino_total, size_t(sl.sino_off) + size_t(sl.n_angles) * sl.n_det);
  if (nr_status s = radon_fwd(plan, d_vol, d_r, stream)) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const hipError_t e = timed(plan, kStageResidual, st, [&] {
    return d_value ? nrk::launch_residual_norm(d_r, d_b, sino_total, d_value, st)
                   : nrk::launch_residual(d_r, d_b, sino_total, st);
  });
  if (e != hipSuccess) return hip_fail(e, "radon_residual launch");
  return NR_OK;
}

nr_status mbir_update(const nr_mbir* params, float* d_x, float* d_x_prev, float* d_y, const float* d_grad,
                      int64_t count, double* d_state, nr_stream stream) {
  if (!params || !d_x || !d_x_prev || !d_y || !d_grad || !d_state) return fail(NR_INVALID_ARG, "mbir_update: NULL argument");
  if (count < 1) return fail(NR_INVALID_ARG, "mbir_update: count must be >= 1");
  if (!(params->inv_L > 0.0f)) return fail(NR_INVALID_ARG, "inv_L must be > 0");
  if (nr_status st = pending_error("before mbir_update")) return st;
  const hipError_t e = nrk::launch_mbir_update(d_x, d_x_prev, d_y, d_grad, size_t(count), params->inv_L,
                                               params->nonneg, d_state, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mbir_update launch");
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
  const nr::Plan& p = plan->p;
  if (index < 0 || index >= int(p.slices.size())) return fail(NR_INVALID_ARG, "slice index out of range");
  const nr::Geom& g = p.geoms[size_t(p.slice_geom[size_t(index)])];
  const int64_t v[5] = {g.G, int64_t(g.tiles_x) * g.tiles_y, int64_t(g.pts.size()), int64_t(g.items.size()),
                        p.kb.D};
  for (int i = 0; i < count && i < 5; ++i) info[i] = v[i];
  return NR_OK;
}

}  // extern "C"
