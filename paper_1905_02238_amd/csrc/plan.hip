// plan.hip -- fsmi_plan: a beam batch bound once, scheduled once, optionally
// autotuned (wave/tile threshold timed on the caller's own inputs) and captured
// into a HIP graph, then replayed with one launch per evaluation.
#include <stdio.h>

#include <algorithm>
#include <new>
#include <vector>

#include "fsmi_internal.h"

struct fsmi_plan_s {
  fsmi_ctx ctx = nullptr;
  fsmi::EvalConst ec{};
  int prec_idx = 0, variant = 0, bound_idx = 0;
  int64_t n_beams = 0;
  const int64_t* off = nullptr;
  const float* occ = nullptr;
  const double* bound = nullptr;
  const float* sigma = nullptr;
  double* mi = nullptr;
  int32_t* d_sched = nullptr;    // beam order, bin histogram, queue counters
  int wave_max = 0;
  int max_len = 0;
  int64_t n_long = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_tried = 0;
  int tried[16] = {};
  float tried_ms[16] = {};
};

using namespace fsmi;

namespace {

// Sort the beams into bins for threshold `wave_max`; read back how many are
// tile-per-beam.  Synchronous.
hipError_t plan_schedule(fsmi_plan p, int wave_max) {
  hipStream_t st = p->ctx->stream;
  hipError_t e = launch_beam_schedule(st, p->off, p->n_beams, wave_max, p->d_sched);
  if (e != hipSuccess) return e;
  int32_t n_long = 0;
  e = hipMemcpyAsync(&n_long, p->d_sched + beam_sched_n_long_index(p->n_beams), 4,
                     hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  p->wave_max = wave_max;
  p->n_long = n_long;
  return hipSuccess;
}

hipError_t plan_enqueue(fsmi_plan p, hipStream_t st) {
  return launch_beam_kernels(st, p->ctx->num_cu, p->ec, p->n_beams, p->off, p->occ, p->bound,
                             p->sigma, p->mi, p->d_sched, p->ctx->d_status, p->wave_max,
                             p->max_len);
}

// Time each candidate threshold (one warm launch, then the mean of three) and
// keep the fastest.
hipError_t plan_autotune(fsmi_plan p) {
  static const int kCand[] = {32, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 1900};
  std::vector<int> cand;
  const int prec = p->ec.precision;
  for (int t : kCand) {
    if (t >= p->max_len) {   // every beam is wave-per-beam from here on: one candidate
      const int all = std::max(p->max_len, 1);
      if (beam_fits(prec, all, p->max_len)) cand.push_back(all);
      break;
    }
    if (beam_fits(prec, t, p->max_len)) cand.push_back(t);
  }
  if (cand.empty()) cand.push_back(beam_default_wave_max(prec));
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  hipStream_t st = p->ctx->stream;
  int best = cand[0];
  float best_ms = 3.0e38f;
  p->n_tried = 0;
  for (int t : cand) {
    if (p->n_tried == 16) break;
    if ((e = plan_schedule(p, t)) != hipSuccess) break;
    if ((e = plan_enqueue(p, st)) != hipSuccess) break;
    if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = plan_enqueue(p, st);
    if (e != hipSuccess) break;
    if ((e = hipEventRecord(e1, st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    ms /= 3.0f;
    p->tried[p->n_tried] = t;
    p->tried_ms[p->n_tried] = ms;
    ++p->n_tried;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  e = plan_schedule(p, best);
  if (e == hipSuccess) p->ctx->tuned_wave_max[p->prec_idx][p->variant][p->bound_idx] = best;
  return e;
}

hipError_t plan_capture(fsmi_plan p) {
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t el = plan_enqueue(p, cs);
    e = hipStreamEndCapture(cs, &p->graph);
    if (el != hipSuccess) e = el;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  return e;
}

void plan_free(fsmi_plan p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_sched) (void)hipFree(p->d_sched);
  delete p;
}

}  // namespace

extern "C" {

fsmi_status fsmi_plan_eval_beams(fsmi_ctx ctx, const fsmi_params* params, int64_t n_beams,
                                 const int64_t* off, const float* occ, const double* bound,
                                 const float* sigma, double* mi, int32_t wave_max,
                                 uint32_t plan_flags, fsmi_plan* out) {
  if (!ctx || !out) return FSMI_E_INVAL;
  *out = nullptr;
  fsmi_status st;
  if (!check_params(ctx, params, &st)) return st;
  if (n_beams <= 0) return fail(ctx, FSMI_E_INVAL, "a plan needs n_beams > 0");
  if (n_beams >= ((int64_t)1 << 31)) return fail(ctx, FSMI_E_CAPACITY, "n_beams >= 2^31");
  if (!off || !occ || !sigma || !mi) return fail(ctx, FSMI_E_INVAL, "off, occ, sigma, mi are required");
  if (wave_max < 0) return fail(ctx, FSMI_E_INVAL, "wave_max < 0");
  if (params->flags & FSMI_F_LUT)
    return fail(ctx, FSMI_E_UNSUPPORTED, "FSMI_F_LUT is implemented on 2D fsmi_eval_poses");
  if ((params->flags & FSMI_F_SKIP_ZERO) && !bound)
    return fail(ctx, FSMI_E_INVAL, "FSMI_F_SKIP_ZERO needs explicit boundaries");
  if (ext_mode(params) && !bound)
    return fail(ctx, FSMI_E_INVAL, "sigma_slope and FSMI_F_MAX_RANGE need explicit boundaries");
  if (plan_flags & ~(uint32_t)(FSMI_PLAN_AUTOTUNE | FSMI_PLAN_GRAPH))
    return fail(ctx, FSMI_E_INVAL, "unknown plan flags");
  (void)hipSetDevice(ctx->device);
  fsmi_plan p = new (std::nothrow) fsmi_plan_s();
  if (!p) return fail(ctx, FSMI_E_NOMEM, "plan");
  p->ctx = ctx;
  p->ec = to_const(params);
  p->prec_idx = params->precision == FSMI_FP64 ? 1 : 0;
  p->variant = params->variant;
  p->bound_idx = bound ? 1 : 0;
  p->n_beams = n_beams;
  p->off = off;
  p->occ = occ;
  p->bound = bound;
  p->sigma = sigma;
  p->mi = mi;
  hipError_t e = hipMalloc((void**)&p->d_sched, beam_sched_ints(n_beams) * 4);
  if (e != hipSuccess) {
    plan_free(p);
    return from_hip(ctx, e, "plan buffers");
  }
  e = launch_max_len(ctx, off, n_beams, &p->max_len);
  if (e != hipSuccess) {
    plan_free(p);
    return from_hip(ctx, e, "plan max length");
  }
  const int wm = wave_max > 0 ? wave_max : ctx_wave_max(ctx, params, bound != nullptr);
  if (!beam_fits(params->precision, (plan_flags & FSMI_PLAN_AUTOTUNE) ? 32 : wm, p->max_len)) {
    plan_free(p);
    return fail(ctx, FSMI_E_CAPACITY, "a beam is longer than one workgroup's LDS holds");
  }
  e = (plan_flags & FSMI_PLAN_AUTOTUNE) ? plan_autotune(p) : plan_schedule(p, wm);
  if (e == hipSuccess && (plan_flags & FSMI_PLAN_GRAPH)) e = plan_capture(p);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(ctx->stream);
    plan_free(p);
    return from_hip(ctx, e, "plan");
  }
  *out = p;
  return FSMI_OK;
}

fsmi_status fsmi_plan_launch(fsmi_plan p) {
  if (!p) return FSMI_E_INVAL;
  (void)hipSetDevice(p->ctx->device);
  if (p->exec) return from_hip(p->ctx, hipGraphLaunch(p->exec, p->ctx->stream), "plan graph launch");
  return from_hip(p->ctx, plan_enqueue(p, p->ctx->stream), "plan launch");
}

fsmi_status fsmi_plan_get_info(fsmi_plan p, fsmi_plan_info* info) {
  if (!p || !info) return FSMI_E_INVAL;
  *info = fsmi_plan_info{};
  info->wave_max = p->wave_max;
  info->max_len = p->max_len;
  info->n_tile = p->n_long;
  info->n_wave = p->n_beams - p->n_long;
  info->graph = p->exec ? 1 : 0;
  info->n_tried = p->n_tried;
  for (int i = 0; i < p->n_tried; ++i) {
    info->tried_wave_max[i] = p->tried[i];
    info->tried_ms[i] = p->tried_ms[i];
  }
  return FSMI_OK;
}

void fsmi_plan_destroy(fsmi_plan p) {
  if (!p) return;
  (void)hipSetDevice(p->ctx->device);
  (void)hipStreamSynchronize(p->ctx->stream);
  plan_free(p);
}

}  // extern "C"
